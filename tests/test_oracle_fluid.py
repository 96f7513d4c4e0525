"""Pins of the staggered Navier-Stokes pieces (oracle/fluid.py, oracle/solver.py).

* The divergence-form convective term of a discretely divergence-free field
  conserves kinetic energy exactly (skew-symmetry of the staggered second-order
  scheme, Morinishi et al. 1998); the field is built as the discrete curl of a
  vector potential, compactly supported away from the x ends.
* The 7-point diffusion term satisfies summation by parts.
* Manufactured solution: H converges to -div(u u) + nu lap(u), evaluated
  symbolically, at second order in h.
* Uniform free stream, outflow mass balance, post-projection divergence.
* y-z Taylor-Green: with the convective term off, every Fourier mode follows
  the AB2 linear recurrence with the discrete eigenvalue; with it on, the
  solution converges to the closed form exp(-2 nu k^2 t) at second order.
"""
import math
from types import SimpleNamespace

import numpy as np
import pytest
import sympy as sy

from oracle import fluid, poisson
from oracle.solver import Solver, set_state

RNG = np.random.default_rng(5)


def _params(nx, ny, nz, h, re=100.0, u_in=1.0, dt=1e-3, cfl=0.5):
    return SimpleNamespace(nx=nx, ny=ny, nz=nz, lx=nx * h, ly=ny * h, lz=nz * h, re=re,
                           u_in=u_in, dt=dt, cfl=cfl, noise_amp=0.0)


def _curl_field(nx, ny, nz, h, lo, hi):
    """Discrete curl of a random edge vector potential supported on x-index [lo, hi]."""
    Ax = np.zeros((nz, ny, nx + 1))
    Ay = np.zeros((nz, ny, nx + 1))
    Az = np.zeros((nz, ny, nx + 1))
    for A in (Ax, Ay, Az):
        A[..., lo:hi + 1] = RNG.standard_normal((nz, ny, hi + 1 - lo))
    yp = lambda a: np.roll(a, -1, 1)
    zp = lambda a: np.roll(a, -1, 0)
    u = np.zeros((nz, ny, nx + 1))
    u[..., :] = ((yp(Az) - Az) - (zp(Ay) - Ay)) / h                 # faces i = 0..nx
    v = ((zp(Ax) - Ax)[..., :nx] - (Az[..., 1:] - Az[..., :nx])) / h  # cells i = 0..nx-1
    w = ((Ay[..., 1:] - Ay[..., :nx]) - (yp(Ax) - Ax)[..., :nx]) / h
    return u, v, w


def test_curl_field_is_divergence_free():
    u, v, w = _curl_field(12, 8, 6, 0.3, 3, 8)
    vv = np.concatenate([v, v[..., -1:]], axis=2)
    ww = np.concatenate([w, w[..., -1:]], axis=2)
    assert np.max(np.abs(fluid.divergence(u, vv, ww, 0.3))) < 1e-12


def test_convective_energy_conservation():
    nx, ny, nz, h = 16, 10, 8, 0.25
    u, v, w = _curl_field(nx, ny, nz, h, 4, 10)
    assert np.all(u[..., :3] == 0) and np.all(u[..., -3:] == 0)
    vg = np.concatenate([v, np.zeros((nz, ny, 1))], axis=2)
    wg = np.concatenate([w, np.zeros((nz, ny, 1))], axis=2)
    f = fluid.Fields(u=u, v=vg, w=wg, p=np.zeros((nz, ny, nx)))
    Hu, Hv, Hw = fluid.rhs(f, h, nu=0.0)
    dE = np.sum(u * Hu) + np.sum(vg * Hv) + np.sum(wg * Hw)
    scale = np.sum(np.abs(u * Hu)) + np.sum(np.abs(vg * Hv)) + np.sum(np.abs(wg * Hw))
    assert scale > 1.0
    assert abs(dE) < 1e-13 * scale


def test_diffusion_summation_by_parts():
    nx, ny, nz, h = 16, 10, 8, 0.25
    u, v, w = _curl_field(nx, ny, nz, h, 4, 10)
    vg = np.concatenate([v, np.zeros((nz, ny, 1))], axis=2)
    wg = np.concatenate([w, np.zeros((nz, ny, 1))], axis=2)
    f = fluid.Fields(u=u, v=vg, w=wg, p=np.zeros((nz, ny, nx)))
    Hu, Hv, Hw = fluid.rhs(f, h, nu=1.0, advection=False)

    def grad2(a):  # sum of squared differences in x (within the array), y, z (periodic)
        return (np.sum(np.diff(a, axis=2) ** 2) + np.sum((np.roll(a, -1, 1) - a) ** 2)
                + np.sum((np.roll(a, -1, 0) - a) ** 2)) / h ** 2

    lhs = np.sum(u * Hu) + np.sum(vg * Hv) + np.sum(wg * Hw)
    rhs = -(grad2(u) + grad2(v) + grad2(w))
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


def _manufactured(n):
    """Smooth field; returns discrete H and the continuum value at interior faces."""
    Lx, Ly, Lz = 4.0, 2.0, 2.0
    h = Ly / n
    nx, ny, nz = int(round(Lx / h)), n, n
    nu = 0.05
    x, y, z = sy.symbols("x y z")
    g = sy.exp(-((x - 2.0) / 0.6) ** 2)
    U = 0.7 + 0.4 * g * sy.sin(sy.pi * y) * sy.cos(sy.pi * z)
    V = 0.3 * g * sy.cos(sy.pi * y) + 0.2 * sy.sin(sy.pi * z)
    W = -0.25 * g * sy.sin(sy.pi * (y + z))
    vel = (U, V, W)
    coords = (x, y, z)
    H = []
    for a in range(3):
        conv = sum(sy.diff(vel[a] * vel[b], coords[b]) for b in range(3))
        lap = sum(sy.diff(vel[a], c, 2) for c in coords)
        H.append(sy.lambdify(coords, -conv + nu * lap, "numpy"))
    fU, fV, fW = (sy.lambdify(coords, q, "numpy") for q in vel)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx + 1), indexing="ij")
    u = fU(i * h, (j + 0.5) * h, (k + 0.5) * h)
    v = fV((i + 0.5) * h, j * h, (k + 0.5) * h)
    w = fW((i + 0.5) * h, (j + 0.5) * h, k * h)
    f = fluid.Fields(u=u, v=v, w=w, p=np.zeros((nz, ny, nx)))
    Hu, Hv, Hw = fluid.rhs(f, h, nu)
    sl = slice(nx // 4, 3 * nx // 4)
    eu = np.max(np.abs(Hu - H[0](i * h, (j + 0.5) * h, (k + 0.5) * h))[..., sl])
    ev = np.max(np.abs(Hv - H[1]((i + 0.5) * h, j * h, (k + 0.5) * h))[..., sl])
    ew = np.max(np.abs(Hw - H[2]((i + 0.5) * h, (j + 0.5) * h, k * h))[..., sl])
    return np.array([eu, ev, ew])


def test_manufactured_rhs_second_order():
    e1 = _manufactured(16)
    e2 = _manufactured(32)
    ratio = e1 / e2
    assert np.all(ratio > 3.5) and np.all(ratio < 4.6), ratio


def test_free_stream_preserved():
    P = _params(16, 8, 8, 0.125, dt=2e-3)
    S = Solver(P)
    S.step(100)
    u, v, w, p = S.fields()
    assert np.max(np.abs(u - 1.0)) < 1e-14
    assert np.max(np.abs(v)) < 1e-14 and np.max(np.abs(w)) < 1e-14


def test_mass_balance_and_projection():
    P = _params(24, 12, 12, 1.0 / 6, re=50.0, dt=0.0, cfl=0.4)
    P.noise_amp = 0.1
    z = (RNG.standard_normal((12, 12, 25)), RNG.standard_normal((12, 12, 24)),
         RNG.standard_normal((12, 12, 24)))
    S = Solver(P, noise=z)
    for _ in range(5):
        ut, vt, wt, H = S.stage_predict()
        assert abs(np.sum(ut[..., -1]) - np.sum(ut[..., 0])) < 1e-13 * ut[..., 0].size
        d0 = np.max(np.abs(fluid.divergence(ut, vt, wt, S.h)))
        S.stage_project(ut, vt, wt)
        d1 = np.max(np.abs(fluid.divergence(S.f.u, S.f.v, S.f.w, S.h)))
        assert d1 < 1e-12 * d0
        S.H_old = H
        S.dt_prev, S.dt = S.dt, S._next_dt()


def _tg_fields(nx, n, h, amp):
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(nx + 1), indexing="ij")
    kap = 2 * np.pi / (n * h)
    u = np.ones((n, n, nx + 1))
    v = amp * np.sin(kap * j * h) * np.cos(kap * (k + 0.5) * h)
    w = -amp * np.cos(kap * (j + 0.5) * h) * np.sin(kap * k * h)
    return u, v[..., :nx], w[..., :nx], kap


def test_taylor_green_diffusion_ab2_recurrence():
    nx, n, h = 6, 16, 2 * np.pi / 16
    nu = 0.05
    P = _params(nx, n, n, h, re=1 / nu, dt=0.01)
    S = Solver(P, hooks=fluid.HOOK_VW_NEUMANN_X, advection=False)
    u, v, w, kap = _tg_fields(nx, n, h, 0.8)
    set_state(S, u, v, w)
    lam = -nu * (8 / h ** 2) * np.sin(np.pi * h / (n * h)) ** 2
    dt = 0.01
    a_prev, a = 1.0, 1.0
    for step in range(40):
        S.step()
        if step == 0:
            a_new = a * (1 + dt * lam)
        else:
            a_new = a + dt * lam * (1.5 * a - 0.5 * a_prev)
        a_prev, a = a, a_new
        _, vs, ws, _ = S.fields()
        assert np.max(np.abs(vs - a * v)) < 1e-12
        assert np.max(np.abs(ws - a * w)) < 1e-12


def _tg_error(n):
    L = 2 * np.pi
    h = L / n
    nu = 0.1
    dt = 0.2 * h * h
    T = 0.5
    steps = int(round(T / dt))
    dt = T / steps
    P = _params(4, n, n, h, re=1 / nu, dt=dt)
    S = Solver(P, hooks=fluid.HOOK_VW_NEUMANN_X)
    u, v, w, kap = _tg_fields(4, n, h, 1.0)
    set_state(S, u, v, w)
    S.step(steps)
    _, vs, ws, _ = S.fields()
    F = math.exp(-2 * nu * kap ** 2 * T)
    return max(np.max(np.abs(vs - F * v)), np.max(np.abs(ws - F * w)))


def test_taylor_green_closed_form_second_order():
    e1, e2 = _tg_error(16), _tg_error(32)
    assert e1 < 2e-2
    assert 3.5 < e1 / e2 < 4.5, (e1, e2)


def test_inlet_zero_transverse_velocity_eigenmode():
    """v = sin(kappa (i+1/2) h), uniform in y and z, vanishes at the inlet plane:
    with u = 0 it is an exact eigenfunction of the discrete x-Laplacian,
    H = nu * (-(4/h^2) sin^2(kappa h/2)) v, at every cell including i = 0."""
    nx, ny, nz, h, nu = 12, 4, 4, 0.2, 0.3
    kap = 0.37 * np.pi / (nx * h)
    i = np.arange(nx + 1)
    mode = np.sin(kap * (i + 0.5) * h)                       # i = nx: outlet ghost
    v = np.broadcast_to(mode, (nz, ny, nx + 1)).copy()
    f = fluid.Fields(u=np.zeros((nz, ny, nx + 1)), v=v, w=v.copy(), p=np.zeros((nz, ny, nx)))
    Hu, Hv, Hw = fluid.rhs(f, h, nu)
    lam = -(4 / h ** 2) * np.sin(kap * h / 2) ** 2
    assert np.max(np.abs(Hv[..., :nx] - nu * lam * v[..., :nx])) < 1e-12
    assert np.max(np.abs(Hw[..., :nx] - nu * lam * v[..., :nx])) < 1e-12
    assert np.max(np.abs(Hu)) < 1e-12


def test_outlet_transports_linear_profile_exactly():
    """The convective outflow solves v_t + U v_x = 0; for data linear in x the
    upwind update equals the exact solution v(x - U dt)."""
    nx, ny, nz, h, U, dt = 10, 4, 4, 0.3, 1.3, 0.05
    xs_u = np.arange(nx + 1) * h
    xs_c = (np.arange(nx + 1) + 0.5) * h
    a, b = 0.4, -0.9
    u = np.broadcast_to(a + b * xs_u, (nz, ny, nx + 1)).copy()
    v = np.broadcast_to(a + b * xs_c, (nz, ny, nx + 1)).copy()
    f = fluid.Fields(u=u, v=v, w=2 * v, p=np.zeros((nz, ny, nx)))
    ut, vt, wt = u.copy(), v.copy(), 2 * v
    fluid.outlet(f, ut, vt, wt, dt, h, U)
    assert np.max(np.abs(ut[..., nx] - (a + b * (xs_u[nx] - U * dt)))) < 1e-14
    assert np.max(np.abs(vt[..., nx] - (a + b * (xs_c[nx] - U * dt)))) < 1e-14
    assert np.max(np.abs(wt[..., nx] - 2 * (a + b * (xs_c[nx] - U * dt)))) < 1e-14
