"""Pins of the MLS transfer and the adaptive Lagrangian tiling
(oracle/mls.py, Sec. II.B (ii) and the tiling paragraph of Sec. II.B).

* The weight is the cubic B-spline (four-fold convolution of the unit box,
  from scipy's B-spline basis) at 2q.
* MLS shape functions equal the weighted least-squares fit solved by lstsq
  (an independent formulation), and reproduce linear fields exactly on every
  staggered component, so sum phi = 1 and the first moments vanish.
* Spreading conserves the total force and is the adjoint of interpolation.
* Tiling: closed-form tile counts, areas that add up to the sheet, the four
  barycentres of one quadratic split, the refinement levels of the workloads,
  and a node load whose total force and first moment equal the markers'.
* In the solver, markers moving with a uniform stream feel no force; a sheet
  at rest gives the fluid exactly dt sum F dV and drives the velocity at its
  markers towards the target.
"""
from types import SimpleNamespace

import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import mls
from oracle.delta import ORIGINS

RNG = np.random.default_rng(2103)


def test_weight_is_the_cubic_b_spline():
    b3 = BSpline.basis_element([-2.0, -1.0, 0.0, 1.0, 2.0], extrapolate=False)
    q = np.linspace(0.0, 1.2, 241)
    want = np.nan_to_num(b3(2.0 * q))
    assert np.max(np.abs(mls.spline(q) - want)) < 1e-14


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_shape_functions_are_the_weighted_least_squares_fit(comp):
    h = 0.1
    X = RNG.uniform(1.0, 2.0, (20, 3))
    idx, phi = mls.mls_stencil(X, comp, h, (40, 40, 41))
    o = np.array(ORIGINS[comp]) * h
    for m in range(X.shape[0]):
        nodes = np.stack([idx[m, :, 0], idx[m, :, 1], idx[m, :, 2]], axis=1) * h + o   # no wrap here
        xi = (nodes - X[m]) / h
        W = np.prod(mls.spline(np.abs(xi) / 1.5), axis=1)
        P = np.hstack([np.ones((27, 1)), xi])
        sw = np.sqrt(W)[:, None]
        # the fitted value at X of data e_q is coefficient 0 of the weighted fit
        coef, *_ = np.linalg.lstsq(sw * P, sw * np.eye(27), rcond=None)
        assert np.max(np.abs(coef[0] - phi[m])) < 1e-13


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_linear_fields_reproduced(comp):
    h, nx, ny, nz = 0.125, 24, 16, 16
    X = RNG.uniform([0.6, 0.5, 0.5], [2.2, 1.4, 1.4], (50, 3))   # away from the periodic seam
    shape = (nz, ny, nx + 1)
    o = np.array(ORIGINS[comp]) * h
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx + 1), indexing="ij")
    a0, g = 0.7, np.array([1.3, -0.4, 2.1])
    field = a0 + g[0] * (i * h + o[0]) + g[1] * (j * h + o[1]) + g[2] * (k * h + o[2])
    idx, phi = mls.mls_stencil(X, comp, h, shape)
    U = mls.interpolate(field, idx, phi)
    assert np.max(np.abs(U - (a0 + X @ g))) < 1e-12
    # constants across the periodic seam
    Xs = X.copy()
    Xs[:, 1] = ny * h - 0.01
    Xs[:, 2] = 0.02
    idx, phi = mls.mls_stencil(Xs, comp, h, shape)
    assert np.max(np.abs(mls.interpolate(np.full(shape, 3.0), idx, phi) - 3.0)) < 1e-13


def test_spreading_conserves_force_and_is_adjoint():
    h, nx, ny, nz = 0.125, 24, 16, 16
    shape = (nz, ny, nx + 1)
    X = RNG.uniform([0.6, 0.0, 0.0], [2.2, 2.0, 2.0], (40, 3))
    F = RNG.standard_normal((40, 3))
    dV = RNG.uniform(0.5, 1.5, 40) * h ** 3
    dt = 0.01
    for c in range(3):
        idx, phi = mls.mls_stencil(X, c, h, shape)
        f = np.zeros(shape)
        mls.spread(f, idx, phi, dt * F[:, c] * dV / h ** 3)
        assert abs(np.sum(f) * h ** 3 - dt * np.sum(F[:, c] * dV)) < 1e-14
        u = RNG.standard_normal(shape)
        lhs = np.sum(mls.interpolate(u, idx, phi) * F[:, c] * dV)
        g = np.zeros(shape)
        mls.spread(g, idx, phi, F[:, c] * dV / h ** 3)
        assert abs(lhs - np.sum(u * g) * h ** 3) < 1e-12 * max(1.0, abs(lhs))


def _sheet(ns, length, x0=1.0):
    a, b = np.meshgrid(np.arange(ns), np.arange(ns), indexing="xy")     # [b, a]
    ds = length / (ns - 1)
    X0 = np.zeros((ns, ns, 3))
    X0[..., 0] = x0 + a * ds * np.cos(0.3)
    X0[..., 1] = 0.4 + a * ds * np.sin(0.3)
    X0[..., 2] = 0.2 + b * ds
    return X0


@pytest.mark.parametrize("ns,length,h,L", [(9, 1.0, 0.2, 0), (9, 1.0, 0.1, 1), (5, 1.0, 0.1, 2)])
def test_tiling_counts_areas_levels(ns, length, h, L):
    X0 = _sheet(ns, length)
    tri, beta, dV, lev = mls.build_markers(X0, h)
    ds = length / (ns - 1)
    assert np.all(lev == L) and L == int(np.ceil(np.log2(max(1.0, ds * np.sqrt(2) / h)) - 1e-12))
    assert tri.shape[0] == 2 * (ns - 1) ** 2 * 4 ** L
    assert abs(np.sum(dV) / h - length ** 2) < 1e-13
    assert np.allclose(beta.sum(axis=1), 1.0, atol=1e-15, rtol=0)
    # the sheet's centroid is the volume-weighted mean of the markers
    Xm, _ = mls.marker_state(tri, beta, X0.reshape(-1, 3), np.zeros((ns * ns, 3)))
    cen = np.sum(Xm * dV[:, None], axis=0) / np.sum(dV)
    assert np.max(np.abs(cen - X0.reshape(-1, 3).mean(axis=0))) < 1e-13


def test_one_quadratic_split_barycentres():
    X0 = _sheet(2, 1.0)
    tri, beta, dV, lev = mls.build_markers(X0, 0.8)      # diagonal sqrt(2) > 0.8 >= sqrt(2)/2
    assert np.all(lev == 1) and tri.shape[0] == 8
    want = np.array([[4, 1, 1], [1, 4, 1], [1, 1, 4], [2, 2, 2]]) / 6.0
    assert np.max(np.abs(beta[:4] - want)) < 1e-15
    assert np.array_equal(tri[0], [0, 1, 3]) and np.array_equal(tri[4], [0, 3, 2])


def test_workload_levels():
    # 96 x 96 flag, L = 1, h = 1/64: the cell diagonal 0.0149 fits; 16 x 16, h = 1/16: one split
    assert mls.refine_level(np.sqrt(2) / 95, 1 / 64) == 0
    assert mls.refine_level(np.sqrt(2) / 15, 1 / 16) == 1


def test_node_load_force_and_moment():
    ns = 6
    X0 = _sheet(ns, 1.0)
    tri, beta, dV, _ = mls.build_markers(X0, 0.1)
    X = X0.reshape(-1, 3)
    Xm, _ = mls.marker_state(tri, beta, X, np.zeros_like(X))
    F = RNG.standard_normal((tri.shape[0], 3))
    f = mls.node_load(tri, beta, F, dV, ns * ns)
    assert np.max(np.abs(f.sum(axis=0) + (F * dV[:, None]).sum(axis=0))) < 1e-14
    mom_nodes = np.einsum("vc,vd->cd", f, X)
    mom_markers = -np.einsum("mc,md->cd", F * dV[:, None], Xm)
    assert np.max(np.abs(mom_nodes - mom_markers)) < 1e-13


def test_solver_markers_in_a_uniform_stream_feel_no_force():
    from oracle.solver import Solver
    h, nx, ny, nz = 0.125, 48, 16, 16
    P = SimpleNamespace(nx=nx, ny=ny, nz=nz, lx=nx * h, ly=ny * h, lz=nz * h, re=300.0, u_in=1.0,
                        dt=1e-3, cfl=0.5, noise_amp=0.0)
    X0 = _sheet(7, 1.0, x0=2.0)
    S = Solver(P, flag=dict(X0=X0, length=1.0, rho=1.0, beta=0.01, ks=1e4, coupling="mls"))
    S.V[:] = (1.0, 0.0, 0.0)
    ut, vt, wt, _ = S.stage_predict()
    before = [a.copy() for a in (ut, vt, wt)]
    F = S.stage_ibm(ut, vt, wt)
    assert F.shape[0] == S.mls["tri"].shape[0] > 2 * 36
    assert np.max(np.abs(F)) < 1e-9
    assert max(np.max(np.abs(a - b)) for a, b in zip((ut, vt, wt), before)) < 1e-15


def test_solver_forcing_scale_and_direction():
    """A sheet at rest in a uniform stream: the forcing step gives the fluid
    exactly dt sum F dV of momentum per component (through the solver's own
    interpolation and spreading), and moves the velocity at the markers
    towards their target."""
    from oracle.solver import Solver
    h, nx, ny, nz = 0.125, 48, 16, 16
    P = SimpleNamespace(nx=nx, ny=ny, nz=nz, lx=nx * h, ly=ny * h, lz=nz * h, re=300.0, u_in=1.0,
                        dt=1e-2, cfl=0.5, noise_amp=0.0)
    S = Solver(P, flag=dict(X0=_sheet(7, 1.0, x0=2.0), length=1.0, rho=1.0, beta=0.01, ks=1e4,
                            coupling="mls"))
    ut, vt, wt, _ = S.stage_predict()
    before = [a.copy() for a in (ut, vt, wt)]
    M = S.mls
    Xm, Vm = mls.marker_state(M["tri"], M["beta"], S.X, S.V)
    F = S.stage_ibm(ut, vt, wt)
    for c, (a, b) in enumerate(zip((ut, vt, wt), before)):
        gain = np.sum(a - b) * h ** 3
        want = S.dt * np.sum(F[:, c] * M["dV"])
        assert abs(gain - want) <= 1e-12 * abs(want) + 1e-15, c
    idx, phi = mls.mls_stencil(Xm, 0, h, ut.shape)
    U0 = mls.interpolate(before[0], idx, phi)
    U1 = mls.interpolate(ut, idx, phi)
    assert np.mean(U0) > 0.9 and np.mean(np.abs(U1 - Vm[:, 0])) < 0.8 * np.mean(np.abs(U0 - Vm[:, 0]))
