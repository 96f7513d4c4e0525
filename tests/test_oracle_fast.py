"""Pins of the plain C oracle of the fluid step (oracle/c/ref_step.c, oracle/fast.py).

* Every stage equals the numpy oracle's stage (an independent implementation
  whose own pins tie it to closed forms) on random fields, boxes with
  odd-sized and radix-3 y, z lengths, with and without the zero-gradient
  test hook, to round-off (1e-14 relative).
* The Poisson solve reproduces the discrete eigenvectors
  cos(pi m (i + 1/2)/nx) e^{2 pi i (j n/ny + k l/nz)} with their closed-form
  eigenvalues, and a uniform stream is a fixed point of the whole step.
* Ten coupled steps (passive-grid points and a flag) equal the numpy
  solver's to 1e-13.
"""
import math
from types import SimpleNamespace

import numpy as np
import pytest

import synth
from oracle import delta, fast, fluid, geometry, poisson
from oracle.solver import Solver
from tests.gpu_cases import oracle_flag_args, rel_l2

RNG = np.random.default_rng(11)


def _fields(nx, ny, nz):
    u = 1.0 + 0.4 * RNG.standard_normal((nz, ny, nx + 1))
    v = 0.4 * RNG.standard_normal((nz, ny, nx + 1))
    w = 0.4 * RNG.standard_normal((nz, ny, nx + 1))
    p = RNG.standard_normal((nz, ny, nx))
    return u, v, w, p


def _close(a, b, tol=1e-14):
    a, b = np.asarray(a), np.asarray(b)
    return np.max(np.abs(a - b)) <= tol * max(1.0, np.max(np.abs(b)))


@pytest.mark.parametrize("dims", [(12, 8, 6), (17, 9, 12), (10, 6, 18)])
@pytest.mark.parametrize("hooks", [0, fluid.HOOK_VW_NEUMANN_X])
def test_stages_equal_numpy(dims, hooks):
    nx, ny, nz = dims
    h, nu, dt, omega = 0.07, 0.013, 3e-3, 0.8
    u, v, w, p = _fields(nx, ny, nz)
    f = fluid.Fields(u=u, v=v, w=w, p=p)
    H = fluid.rhs(f, h, nu, hooks)
    Hc = fast.rhs(u, v, w, h, nu, hooks)
    for a, b in zip(Hc, H):
        assert _close(a, b)
    H_old = [x + 0.1 * RNG.standard_normal(x.shape) for x in H]
    ut, vt, wt = fluid.predictor(f, H, H_old, dt, omega, h)
    utc, vtc, wtc = fast.predictor(u, v, w, p, H, H_old, dt, omega, h)
    for a, b in ((utc, ut), (vtc, vt), (wtc, wt)):
        assert _close(a, b)
    fluid.outlet(f, ut, vt, wt, dt, h, 1.0, hooks)
    fast.outlet(u, v, w, utc, vtc, wtc, dt, h, 1.0, hooks)
    assert _close(utc, ut) and _close(vtc, vt) and _close(wtc, wt)
    assert abs(fast.flux_correct(utc) - fluid.flux_correct(ut)) < 1e-14
    assert _close(utc, ut)
    r = fluid.divergence(ut, vt, wt, h)
    assert _close(fast.divergence(utc, vtc, wtc, h), r, 1e-13)
    phi = poisson.solve_poisson(r, h)
    phic = fast.poisson(r, h)
    assert _close(phic - phic.mean(), phi - phi.mean(), 1e-12)
    g = fluid.Fields(u=u.copy(), v=v.copy(), w=w.copy(), p=p.copy())
    fluid.project(g, ut, vt, wt, phi, dt, h)
    uc, vc, wc, pc = u.copy(), v.copy(), w.copy(), p.copy()
    fast.project(ut, vt, wt, phi, dt, h, uc, vc, wc, pc)
    for a, b in ((uc, g.u), (vc, g.v), (wc, g.w), (pc, g.p)):
        assert _close(a, b)
    smax = fast.max_speed(uc, vc, wc)
    assert abs(0.5 * h / smax - fluid.cfl_dt(g, h, 0.5)) <= 1e-15 * (0.5 * h / smax)


def test_ibm_equals_numpy():
    nx, ny, nz, h, dt = 24, 12, 10, 0.1, 2e-3
    u, v, w, _ = _fields(nx, ny, nz)
    K = 57
    X = np.column_stack([RNG.uniform(0.35, nx * h - 0.35, K), RNG.uniform(-0.05, ny * h, K),
                         RNG.uniform(0.0, nz * h + 0.05, K)])
    X[3] = (1.0, 0.55, 0.15)      # on a half-integer of the v and w lattices in y / z
    Ud = RNG.standard_normal((K, 3))
    dV = RNG.uniform(0.5, 2.0, K) * h ** 3
    a = [x.copy() for x in (u, v, w)]
    b = [x.copy() for x in (u, v, w)]
    F = delta.ibm_force(a[0], a[1], a[2], X, Ud, dV, h, dt, nx)
    Fc = fast.ibm(b[0], b[1], b[2], X, Ud, dV, h, dt)
    assert _close(Fc, F, 1e-13)
    for x, y in zip(b, a):
        assert _close(x, y)
    with pytest.raises(ValueError):          # support leaving the evolved x range
        fast.ibm(b[0], b[1], b[2], np.array([[0.05, 0.5, 0.5]]), None, np.ones(1), h, dt)


def test_poisson_eigenvectors():
    nx, ny, nz, h = 20, 12, 18, 0.3
    i = np.arange(nx)[None, None, :]
    j = np.arange(ny)[None, :, None]
    k = np.arange(nz)[:, None, None]
    for (m, n, l) in ((3, 2, 5), (1, 0, 0), (7, 6, 9), (0, 4, 1)):
        e = (np.cos(np.pi * m * (i + 0.5) / nx) * np.cos(2 * np.pi * (j * n / ny + k * l / nz)))
        lam = -(4.0 / h ** 2) * (math.sin(math.pi * m / (2 * nx)) ** 2 + math.sin(math.pi * n / ny) ** 2
                                 + math.sin(math.pi * l / nz) ** 2)
        phi = fast.poisson(lam * e, h)
        assert np.max(np.abs(phi - e)) < 1e-12


def test_uniform_stream_is_steady():
    P = SimpleNamespace(nx=16, ny=8, nz=6, lx=1.6, ly=0.8, lz=0.6, re=100.0, u_in=1.3, dt=0.0, cfl=0.5,
                        noise_amp=0.0)
    S = fast.FastSolver(P)
    assert abs(S.dt - 0.5 * 0.1 / 1.3) <= 1e-15 * S.dt
    S.step(20)
    assert np.max(np.abs(S.u - 1.3)) < 1e-13 and np.max(np.abs(S.v)) < 1e-13 and np.max(np.abs(S.w)) < 1e-13


def _small_grid_flag():
    return synth.Workload(name="grid_flag_small", nx=48, ny=24, nz=24, lx=6.0, ly=3.0, lz=3.0, re=300.0,
                          dt=0.0, cfl=0.4, grid=synth.Grid(x_plane=0.75, mesh=1.5, bar=0.3),
                          flag=synth.Flag(ns=8, length=1.0, x_le=2.0, y_c=1.5, z_c=1.5, bending=0.01))


def test_ten_steps_equal_numpy_solver():
    w = _small_grid_flag()
    noise = synth.ic_noise(w)
    bars = geometry.grid_points_of(w)
    X0 = geometry.flag_lattice(w.flag)
    S = Solver(w, noise, bars, oracle_flag_args(w, X0))
    C = fast.FastSolver(w, noise, bars, oracle_flag_args(w, X0))
    assert abs(C.dt - S.dt) <= 1e-14 * S.dt
    S.step(10)
    C.step(10)
    assert rel_l2(C.fields()[:3], S.fields()[:3]) < 1e-13
    assert rel_l2([C.X], [S.X]) < 1e-13 and C.nsub == S.nsub
    assert abs(C.t - S.t) <= 1e-13 * S.t
