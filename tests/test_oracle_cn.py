"""Pins of the Crank-Nicolson / approximate-factorisation predictor
(oracle/fluid.py predictor_cn, Sec. II.B).

* The periodic factor solve equals a dense circulant solve, and the x factor
  a dense tridiagonal solve with the stated boundary rows (brute force).
* y-z Taylor-Green with the convective term off: each step multiplies the
  mode by 1 + dt nu (ly + lz) / ((1 - b ly)(1 - b lz)), b = nu dt / 2, with
  the discrete eigenvalues ly, lz (closed form of the factorised scheme).
* With the convective term on, the solution converges at second order to
  the closed form exp(-2 nu k^2 t) with dt proportional to h (a step that the
  explicit diffusion could not take).
"""
import math
from types import SimpleNamespace

import numpy as np

from oracle import fluid
from oracle.solver import Solver, set_state

RNG = np.random.default_rng(17)


def _params(nx, ny, nz, h, re, dt, u_in=1.0):
    return SimpleNamespace(nx=nx, ny=ny, nz=nz, lx=nx * h, ly=ny * h, lz=nz * h, re=re,
                           u_in=u_in, dt=dt, cfl=0.5, noise_amp=0.0)


def test_periodic_factor_is_a_circulant_solve():
    n, h, beta = 7, 0.3, 0.02
    b = RNG.standard_normal((3, n, 4))
    A = np.eye(n) * (1 + 2 * beta / h ** 2)
    for i in range(n):
        A[i, (i - 1) % n] -= beta / h ** 2
        A[i, (i + 1) % n] -= beta / h ** 2
    x = fluid._periodic_solve(b, beta, h, axis=1)
    want = np.einsum("ij,ajk->aik", np.linalg.inv(A), b)
    assert np.max(np.abs(x - want)) < 1e-13


def test_x_factor_is_a_tridiagonal_solve():
    n, r = 6, 0.37
    b = RNG.standard_normal((2, 3, n))
    add = RNG.standard_normal((2, 3))
    for first in (1 + 2 * r, 1 + 3 * r, 1 + r):
        A = (np.diag(np.full(n, 1 + 2 * r)) + np.diag(np.full(n - 1, -r), 1)
             + np.diag(np.full(n - 1, -r), -1))
        A[0, 0] = first
        x = fluid._x_solve(b, r, first, 1 + 2 * r, add)
        bb = b.copy()
        bb[..., -1] += add
        want = np.einsum("ij,abj->abi", np.linalg.inv(A), bb)
        assert np.max(np.abs(x - want)) < 1e-13


def _tg_fields(nx, n, h, amp):
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(nx + 1), indexing="ij")
    kap = 2 * np.pi / (n * h)
    u = np.ones((n, n, nx + 1))
    v = amp * np.sin(kap * j * h) * np.cos(kap * (k + 0.5) * h)
    w = -amp * np.cos(kap * (j + 0.5) * h) * np.sin(kap * k * h)
    return u, v[..., :nx], w[..., :nx], kap


def test_taylor_green_cn_recurrence():
    nx, n, h = 6, 16, 2 * np.pi / 16
    nu, dt = 0.05, 0.4          # nu dt / h^2 = 0.13, beyond the explicit limit 1/12
    P = _params(nx, n, n, h, re=1 / nu, dt=dt)
    S = Solver(P, hooks=fluid.HOOK_VW_NEUMANN_X, advection=False, diffusion="cn")
    u, v, w, kap = _tg_fields(nx, n, h, 0.8)
    set_state(S, u, v, w)
    lam = -(4 / h ** 2) * np.sin(kap * h / 2) ** 2          # per direction
    b = 0.5 * nu * dt
    g = 1 + dt * nu * (2 * lam) / ((1 - b * lam) * (1 - b * lam))
    a = 1.0
    for step in range(25):
        S.step()
        a *= g
        _, vs, ws, _ = S.fields()
        assert np.max(np.abs(vs - a * v)) < 1e-12
        assert np.max(np.abs(ws - a * w)) < 1e-12


def _tg_error(n):
    L = 2 * np.pi
    h = L / n
    nu = 0.1
    T = 0.5
    steps = int(round(T / (0.1 * h)))      # dt = 0.1 h: nu dt / h^2 = 0.01 / h grows as h shrinks
    dt = T / steps
    P = _params(4, n, n, h, re=1 / nu, dt=dt)
    S = Solver(P, hooks=fluid.HOOK_VW_NEUMANN_X, diffusion="cn")
    u, v, w, kap = _tg_fields(4, n, h, 1.0)
    set_state(S, u, v, w)
    S.step(steps)
    _, vs, ws, _ = S.fields()
    F = math.exp(-2 * nu * kap ** 2 * T)
    return max(np.max(np.abs(vs - F * v)), np.max(np.abs(ws - F * w)))


def test_taylor_green_cn_second_order():
    e1, e2 = _tg_error(16), _tg_error(32)
    assert e1 < 2e-2
    assert 3.5 < e1 / e2 < 4.5, (e1, e2)


def test_factorised_operator_applied_to_the_increment():
    """Apply the dense 1-D factors to du (x with the stated boundary rows) and
    recover the right-hand side of a full predictor_cn call (no hook)."""
    nx, ny, nz, h, nu, dt = 6, 4, 5, 0.3, 0.7, 0.05
    f = fluid.Fields(u=1 + 0.1 * RNG.standard_normal((nz, ny, nx + 1)),
                     v=0.1 * RNG.standard_normal((nz, ny, nx + 1)),
                     w=0.1 * RNG.standard_normal((nz, ny, nx + 1)),
                     p=RNG.standard_normal((nz, ny, nx)))
    Hc = fluid.rhs(f, h, 0.0)
    D = fluid.rhs(f, h, nu, advection=False)
    ut, vt, wt = f.u.copy(), f.v.copy(), f.w.copy()
    fluid.outlet(f, ut, vt, wt, dt, h, 1.0)
    fluid.predictor_cn(f, Hc, Hc, D, ut, vt, wt, dt, 1.0, h, nu)
    beta, r = 0.5 * nu * dt, 0.5 * nu * dt / h ** 2

    def periodic(n):
        A = np.eye(n) * (1 + 2 * r)
        for i in range(n):
            A[i, (i - 1) % n] -= r
            A[i, (i + 1) % n] -= r
        return A
    Z, Y = periodic(nz), periodic(ny)
    for c, (st, tl) in enumerate(((f.u, ut), (f.v, vt), (f.w, wt))):
        s = slice(1, nx) if c == 0 else slice(0, nx)
        du = tl[..., s] - st[..., s]
        n = du.shape[-1]
        X = (np.diag(np.full(n, 1 + 2 * r)) + np.diag(np.full(n - 1, -r), 1)
             + np.diag(np.full(n - 1, -r), -1))
        if c > 0:
            X[0, 0] = 1 + 3 * r
        a = np.einsum("ij,abj->abi", X, du)
        a[..., -1] -= r * (tl[..., nx] - st[..., nx])
        a = np.einsum("ij,ajk->aik", Y, a)
        a = np.einsum("ij,jbk->ibk", Z, a)
        gp = ((f.p[..., 1:nx] - f.p[..., 0:nx - 1]) / h if c == 0 else
              (f.p - np.roll(f.p, 1, axis=1)) / h if c == 1 else (f.p - np.roll(f.p, 1, axis=0)) / h)
        rhs = dt * (1.5 * Hc[c][..., s] - 0.5 * Hc[c][..., s] - gp + D[c][..., s])
        assert np.max(np.abs(a - rhs)) < 1e-12


def test_cn_stable_beyond_the_explicit_limit():
    """nu dt / h^2 = 0.32, about four times the explicit limit 1/12: the explicit
    step amplifies the grid-scale noise without bound, CN keeps it bounded."""
    import synth
    h = 0.125
    w = synth.Workload(name="viscous", nx=48, ny=16, nz=16, lx=48 * h, ly=16 * h, lz=16 * h, re=2.0,
                       dt=0.01, cfl=0.4, steps=10)
    cn = Solver(w, synth.ic_noise(w), None, None, diffusion="cn")
    ex = Solver(w, synth.ic_noise(w), None, None)
    cn.step(10)
    ex.step(10)
    assert max(np.max(np.abs(a)) for a in cn.fields()[1:3]) < 0.1
    assert max(np.max(np.abs(a)) for a in ex.fields()[1:3]) > 1e3
