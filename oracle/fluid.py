"""Staggered-mesh Navier-Stokes pieces of the fractional step (oracle).

Eqs. (2)-(3) on a staggered Cartesian mesh, second-order centred differences
(Sec. II.B).  Cells i = 0..nx-1, j = 0..ny-1, k = 0..nz-1, spacing h equal in
all directions; arrays are indexed [k, j, i] (x fastest in memory).

  u[k, j, i], i = 0..nx        at (i h, (j+1/2) h, (k+1/2) h)
  v[k, j, i], i = 0..nx        at ((i+1/2) h, j h, (k+1/2) h); i = nx is the
                               outlet ghost (state), i = -1 the inlet ghost
  w[k, j, i]                   like v with y and z exchanged
  p[k, j, i], i = 0..nx-1      at cell centres

Boundary conditions (Sec. II.A): uniform inflow (U, 0, 0) at x = 0, a
non-reflecting convective outflow at x = Lx, periodic in y and z.

Readings where the paper is silent (Sec. II.B names the scheme only):
  * Nonlinear term in divergence form with products of two-point averages;
    diffusion by the 7-point Laplacian; both explicit in the Adams-Bashforth
    right-hand side H (the paper's Crank-Nicolson diffusion is not used).
  * Variable-step AB2 with omega = dt_n / dt_{n-1}, Euler on the first step.
  * Incremental pressure: the predictor carries -G p^n and p^{n+1} = p^n + phi.
  * Inlet ghosts v_{-1} = -v_0, w_{-1} = -w_0 (zero transverse inflow).
  * Convective outflow: first-order upwind with convection speed U for u at
    i = nx and for the v, w ghosts, followed by an additive correction of u at
    i = nx that makes the outflow equal the inflow.
  * Time step from CFL: dt = cfl h / max over cells (|u_c| + |v_c| + |w_c|),
    with u_c the mean of a cell's two faces.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# test hook: v, w zero-gradient ghosts at inlet and outlet (x-invariant flows)
HOOK_VW_NEUMANN_X = 1


@dataclass
class Fields:
    u: np.ndarray   # (nz, ny, nx+1)
    v: np.ndarray   # (nz, ny, nx+1), [..., nx] outlet ghost
    w: np.ndarray   # (nz, ny, nx+1), [..., nx] outlet ghost
    p: np.ndarray   # (nz, ny, nx)


def _ym(a):
    """a at j-1 (periodic)."""
    return np.roll(a, 1, axis=1)


def _yp(a):
    return np.roll(a, -1, axis=1)


def _zm(a):
    return np.roll(a, 1, axis=0)


def _zp(a):
    return np.roll(a, -1, axis=0)


def _with_ghosts(v, nx, hooks):
    """v (nz, ny, nx+1) -> (nz, ny, nx+2) indexed by i+1, with the inlet ghost."""
    nz, ny, _ = v.shape
    g = np.empty((nz, ny, nx + 2))
    g[..., 1:nx + 1] = v[..., :nx]
    if hooks & HOOK_VW_NEUMANN_X:
        g[..., 0] = v[..., 0]
        g[..., nx + 1] = v[..., nx - 1]
    else:
        g[..., 0] = -v[..., 0]
        g[..., nx + 1] = v[..., nx]
    return g


def rhs(f: Fields, h: float, nu: float, hooks: int = 0, advection: bool = True):
    """Explicit right-hand side H = -div(u u) + nu lap(u) of Eq. (2) without pressure.

    Returns (Hu, Hv, Hw) shaped like u, v, w; Hu is filled at i = 1..nx-1,
    Hv and Hw at i = 0..nx-1 (other entries zero).  ``advection=False``
    drops the nonlinear term (used only by the diffusion pins).
    """
    u, v, w = f.u, f.v, f.w
    nz, ny, nxp1 = u.shape
    nx = nxp1 - 1
    vg = _with_ghosts(v, nx, hooks)          # vg[..., i+1] = v_i, i = -1..nx
    wg = _with_ghosts(w, nx, hooks)

    # x-y edge flux Fxy(i, j) at (i h, j h, (k+1/2) h), i = 0..nx:
    #   (u averaged in y) * (v averaged in x)
    uy = 0.5 * (_ym(u) + u)                               # (nz, ny, nx+1)
    vx = 0.5 * (vg[..., 0:nx + 1] + vg[..., 1:nx + 2])    # v at x = i h, i = 0..nx
    Fxy = uy * vx
    # x-z edge flux Fxz(i, k) at (i h, (j+1/2) h, k h)
    uz = 0.5 * (_zm(u) + u)
    wx = 0.5 * (wg[..., 0:nx + 1] + wg[..., 1:nx + 2])
    Fxz = uz * wx
    # y-z edge flux Fyz(j, k) at ((i+1/2) h, j h, k h), i = 0..nx-1
    vz = 0.5 * (_zm(v[..., :nx]) + v[..., :nx])
    wy = 0.5 * (_ym(w[..., :nx]) + w[..., :nx])
    Fyz = vz * wy
    # cell-centre normal fluxes
    uc = 0.5 * (u[..., :nx] + u[..., 1:])
    Fxx = uc * uc
    vc = 0.5 * (v[..., :nx] + _yp(v[..., :nx]))
    Fyy = vc * vc
    wc = 0.5 * (w[..., :nx] + _zp(w[..., :nx]))
    Fzz = wc * wc

    Hu = np.zeros_like(u)
    Hv = np.zeros_like(v)
    Hw = np.zeros_like(w)
    inv_h = 1.0 / h
    c_d = nu / (h * h)

    # u at faces i = 1..nx-1
    ui = u[..., 1:nx]
    lap = ((u[..., 2:nx + 1] + u[..., 0:nx - 1] - 2.0 * ui)
           + (_yp(u)[..., 1:nx] + _ym(u)[..., 1:nx] - 2.0 * ui)
           + (_zp(u)[..., 1:nx] + _zm(u)[..., 1:nx] - 2.0 * ui))
    adv = ((Fxx[..., 1:nx] - Fxx[..., 0:nx - 1])
           + (_yp(Fxy)[..., 1:nx] - Fxy[..., 1:nx])
           + (_zp(Fxz)[..., 1:nx] - Fxz[..., 1:nx])) * inv_h
    Hu[..., 1:nx] = (-adv if advection else 0.0) + c_d * lap

    # v at cells i = 0..nx-1
    vi = v[..., :nx]
    lap = ((vg[..., 2:nx + 2] + vg[..., 0:nx] - 2.0 * vi)
           + (_yp(vi) + _ym(vi) - 2.0 * vi)
           + (_zp(vi) + _zm(vi) - 2.0 * vi))
    adv = ((Fxy[..., 1:nx + 1] - Fxy[..., 0:nx])
           + (Fyy - _ym(Fyy))
           + (_zp(Fyz) - Fyz)) * inv_h
    Hv[..., :nx] = (-adv if advection else 0.0) + c_d * lap

    # w at cells i = 0..nx-1
    wi = w[..., :nx]
    lap = ((wg[..., 2:nx + 2] + wg[..., 0:nx] - 2.0 * wi)
           + (_yp(wi) + _ym(wi) - 2.0 * wi)
           + (_zp(wi) + _zm(wi) - 2.0 * wi))
    adv = ((Fxz[..., 1:nx + 1] - Fxz[..., 0:nx])
           + (_yp(Fyz) - Fyz)
           + (Fzz - _zm(Fzz))) * inv_h
    Hw[..., :nx] = (-adv if advection else 0.0) + c_d * lap
    return Hu, Hv, Hw


def predictor(f: Fields, H, H_old, dt: float, omega: float, h: float):
    """Provisional velocity u~ = u^n + dt[(1 + w/2) H^n - (w/2) H^{n-1} - G p^n].

    Variable-step AB2 (Sec. II.B names AB2).  Returns (ut, vt, wt) shaped like
    u, v, w; boundary entries (u at i = 0 and nx, v/w ghosts at nx) are copied
    from the current state and set by ``outlet``.
    """
    u, v, w, p = f.u, f.v, f.w, f.p
    nx = u.shape[2] - 1
    c1 = 1.0 + 0.5 * omega
    c2 = 0.5 * omega
    inv_h = 1.0 / h
    ut = u.copy()
    vt = v.copy()
    wt = w.copy()
    gpx = (p[..., 1:nx] - p[..., 0:nx - 1]) * inv_h
    ut[..., 1:nx] = u[..., 1:nx] + dt * (c1 * H[0][..., 1:nx] - c2 * H_old[0][..., 1:nx] - gpx)
    gpy = (p - _ym(p)) * inv_h
    vt[..., :nx] = v[..., :nx] + dt * (c1 * H[1][..., :nx] - c2 * H_old[1][..., :nx] - gpy)
    gpz = (p - _zm(p)) * inv_h
    wt[..., :nx] = w[..., :nx] + dt * (c1 * H[2][..., :nx] - c2 * H_old[2][..., :nx] - gpz)
    return ut, vt, wt


def outlet(f: Fields, ut, vt, wt, dt: float, h: float, u_conv: float, hooks: int = 0):
    """Convective outflow du/dt + U du/dx = 0, first-order upwind, on u at i = nx
    and on the v, w ghosts at i = nx (in place on the provisional arrays).
    Under the zero-gradient test hook the ghosts are never read and are left
    unchanged."""
    u, v, w = f.u, f.v, f.w
    nx = u.shape[2] - 1
    c = dt * u_conv / h
    ut[..., nx] = u[..., nx] - c * (u[..., nx] - u[..., nx - 1])
    if not hooks & HOOK_VW_NEUMANN_X:
        vt[..., nx] = v[..., nx] - c * (v[..., nx] - v[..., nx - 1])
        wt[..., nx] = w[..., nx] - c * (w[..., nx] - w[..., nx - 1])


def flux_correct(ut):
    """Add (Q_in - Q_out)/(Ly Lz) to u~ at the outlet face so that the outflow
    equals the inflow; in cell units this is (sum u_0 - sum u_nx)/(ny nz).
    Returns the correction."""
    nz, ny, nxp1 = ut.shape
    nx = nxp1 - 1
    corr = (np.sum(ut[..., 0]) - np.sum(ut[..., nx])) / (ny * nz)
    ut[..., nx] += corr
    return corr


def divergence(ut, vt, wt, h: float):
    """Discrete divergence D u at the cell centres, (nz, ny, nx)."""
    nx = ut.shape[2] - 1
    return ((ut[..., 1:] - ut[..., :nx])
            + (_yp(vt[..., :nx]) - vt[..., :nx])
            + (_zp(wt[..., :nx]) - wt[..., :nx])) / h


def project(f: Fields, ut, vt, wt, phi, dt: float, h: float):
    """u^{n+1} = u~ - dt G phi on the evolved faces, p^{n+1} = p^n + phi (in place on f).

    Boundary faces (u at i = 0 and nx) and the v, w outlet ghosts keep their
    provisional values."""
    nx = ut.shape[2] - 1
    inv_h = 1.0 / h
    u = ut.copy()
    u[..., 1:nx] = ut[..., 1:nx] - dt * (phi[..., 1:] - phi[..., :nx - 1]) * inv_h
    v = vt.copy()
    v[..., :nx] = vt[..., :nx] - dt * (phi - _ym(phi)) * inv_h
    w = wt.copy()
    w[..., :nx] = wt[..., :nx] - dt * (phi - _zm(phi)) * inv_h
    f.u, f.v, f.w = u, v, w
    f.p = f.p + phi


def cfl_dt(f: Fields, h: float, cfl: float):
    """dt = cfl h / max over cells (|u_c| + |v_c| + |w_c|)."""
    u, v, w = f.u, f.v, f.w
    nx = u.shape[2] - 1
    uc = np.abs(0.5 * (u[..., :nx] + u[..., 1:]))
    vc = np.abs(0.5 * (v[..., :nx] + _yp(v[..., :nx])))
    wc = np.abs(0.5 * (w[..., :nx] + _zp(w[..., :nx])))
    smax = float(np.max(uc + vc + wc))
    return cfl * h / smax


# ---------------------------------------------------------------------------
# Crank-Nicolson diffusion with approximate factorisation (Sec. II.B names
# Crank-Nicolson for the diffusive terms and an approximate factorisation for
# the provisional velocity).  Reading, delta form:
#   RHS = dt [(1 + w/2) Hc^n - (w/2) Hc^{n-1} - G p^n + nu L u^n],
#   Hc = -div(u u) (the convective part only),
#   (1 - b Dx)(1 - b Dy)(1 - b Dz) du = RHS,  b = nu dt / 2,  Dd = d^2/dd^2 (3-point),
#   u~ = u^n + du on the evolved nodes,
# solved as du = X^{-1} Y^{-1} Z^{-1} RHS: the periodic y and z factors first,
# then the x factor, whose boundary rows take the increments of the boundary
# values: u: du_0 = 0 (inlet), du_nx = u~_nx - u^n_nx (the convective outflow
# value); v, w: the inlet ghost du_{-1} = -du_0 and the outlet ghost
# increment u~_nx - u^n_nx; under the zero-gradient test hook, du_{-1} = du_0
# and du_nx = du_{nx-1}.
# ---------------------------------------------------------------------------

def _periodic_solve(b, beta, h, axis):
    """(1 - beta D) x = b along a periodic axis: the circulant operator is
    diagonal in the discrete Fourier basis with eigenvalues
    1 + (4 beta / h^2) sin^2(pi m / n)."""
    n = b.shape[axis]
    m = np.arange(n)
    mu = 1.0 + (4.0 * beta / (h * h)) * np.sin(np.pi * m / n) ** 2
    shape = [1] * b.ndim
    shape[axis] = n
    return np.real(np.fft.ifft(np.fft.fft(b, axis=axis) / mu.reshape(shape), axis=axis))


def _x_solve(rhs, r, first_diag, last_diag, last_add):
    """Tridiagonal (-r, diag, -r) along the last axis (lines of length n) with
    the first and last diagonal entries given and last_add added to the last
    row's right-hand side; banded LAPACK solve, every line at once."""
    from scipy.linalg import solve_banded
    n = rhs.shape[-1]
    ab = np.zeros((3, n))
    ab[0, 1:] = -r
    ab[1, :] = 1.0 + 2.0 * r
    ab[1, 0] = first_diag
    ab[1, -1] = last_diag
    ab[2, :-1] = -r
    b = rhs.copy()
    b[..., -1] += last_add
    flat = b.reshape(-1, n).T
    return solve_banded((1, 1), ab, flat).T.reshape(b.shape)


def predictor_cn(f: Fields, Hc, Hc_old, D, ut, vt, wt, dt: float, omega: float, h: float, nu: float,
                 hooks: int = 0):
    """Provisional velocity with Crank-Nicolson diffusion in approximately
    factorised delta form (the reading above), in place on ut, vt, wt, whose
    outlet entries must already hold the convective outflow values.  Hc, Hc_old:
    convective right-hand sides; D = nu L u^n."""
    u, v, w, p = f.u, f.v, f.w, f.p
    nx = u.shape[2] - 1
    c1 = 1.0 + 0.5 * omega
    c2 = 0.5 * omega
    inv_h = 1.0 / h
    beta = 0.5 * nu * dt
    r = beta / (h * h)
    gp = ((p[..., 1:nx] - p[..., 0:nx - 1]) * inv_h, (p - _ym(p)) * inv_h, (p - _zm(p)) * inv_h)
    sl = (slice(1, nx), slice(0, nx), slice(0, nx))
    neumann = bool(hooks & HOOK_VW_NEUMANN_X)
    for c, (st, tl) in enumerate(((u, ut), (v, vt), (w, wt))):
        s = sl[c]
        rhs = dt * (c1 * Hc[c][..., s] - c2 * Hc_old[c][..., s] - gp[c] + D[c][..., s])
        rhs = _periodic_solve(rhs, beta, h, axis=0)      # z
        rhs = _periodic_solve(rhs, beta, h, axis=1)      # y
        if c == 0:
            d_out = tl[..., nx] - st[..., nx]
            du = _x_solve(rhs, r, 1.0 + 2.0 * r, 1.0 + 2.0 * r, r * d_out)
        elif neumann:
            du = _x_solve(rhs, r, 1.0 + r, 1.0 + r, 0.0)
        else:
            d_out = tl[..., nx] - st[..., nx]
            du = _x_solve(rhs, r, 1.0 + 3.0 * r, 1.0 + 2.0 * r, r * d_out)
        tl[..., s] = st[..., s] + du
