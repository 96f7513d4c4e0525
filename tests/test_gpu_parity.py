"""GPU-versus-oracle parity of the HIP time step, through the C ABI.

Tolerances: the oracle and the library evaluate the same FP64 formulas with
different summation orders, FMA contraction and FFT/tridiagonal algorithms,
so single stages agree to a few ulp of the largest term (<= 1e-13 relative)
and the full step after 10 steps to <= 1e-12 relative L2 of the velocity
(the target stated for the plain FP64 path).  Index maps are compared bit for
bit.  Pressure is compared after removing its mean (gauge).
"""
import numpy as np
import pytest

import synth
from tests.gpu_cases import build_pair, demean, rel_l2

pytestmark = pytest.mark.gpu

ib = pytest.importorskip("paper_2103_08246_amd")


def small_grid_flag(nx=48, steps=10):
    return synth.Workload(name="grid_flag_small", nx=nx, ny=nx // 2, nz=nx // 2, lx=6.0,
                          ly=3.0, lz=3.0, re=300.0, dt=0.0, cfl=0.4, steps=steps,
                          grid=synth.Grid(x_plane=0.75, mesh=1.5, bar=0.3),
                          flag=synth.Flag(ns=8, length=1.0, x_le=2.0, y_c=1.5, z_c=1.5,
                                          bending=0.01))


def _fields_close(run, S, tol):
    u, v, w, p, t, _ = run.fields()
    uo, vo, wo, po = S.fields()
    assert rel_l2([u, v, w], [uo, vo, wo]) < tol
    return u, v, w, p, t


def test_initial_projection_matches():
    w = synth.flag_64_re200()
    run, S = build_pair(w)
    try:
        _fields_close(run, S, 1e-14)
        sc = ib.get_scalars(run.ctx)
        assert sc["dt"] == S.dt
    finally:
        run.close()


@pytest.mark.parametrize("make", [synth.flag_64_re200, small_grid_flag])
def test_predict_stage(make):
    w = make()
    run, S = build_pair(w)
    try:
        ib.run_stage(run.ctx, ib.STAGE_PREDICT)
        ib.run_stage(run.ctx, ib.STAGE_FLUX)
        ut, vt, wt, H = S.stage_predict()
        nx = w.nx
        g = {k: ib.get_array(run.ctx, a, s) for k, a, s in (
            ("ut", ib.ARR_UT, ut.shape), ("vt", ib.ARR_VT, vt[..., :nx].shape),
            ("wt", ib.ARR_WT, wt[..., :nx].shape), ("hu", ib.ARR_HU, ut.shape),
            ("hv", ib.ARR_HV, vt[..., :nx].shape))}
        assert rel_l2([g["ut"], g["vt"], g["wt"]], [ut, vt[..., :nx], wt[..., :nx]]) < 1e-14
        assert rel_l2([g["hu"], g["hv"]], [H[0], H[1][..., :nx]]) < 1e-13
        vg = ib.get_array(run.ctx, ib.ARR_V_GHOST, (w.nz, w.ny))
        assert np.max(np.abs(vg - S.f.v[..., nx])) == 0.0   # ghost untouched until projection
    finally:
        run.close()


# x lines of every solver shape: two lines per wavefront (32 lanes) with chunks
# of 2-6 rows per lane for nx <= 192, one line per wavefront (64 lanes) with
# chunks of 4, 5, 8 beyond (6 and 12 at 384 and 768 in the timed-instance tests)
@pytest.mark.parametrize("dims", [(33, 16, 16), (64, 32, 32), (96, 48, 24), (128, 64, 96), (150, 16, 16),
                                  (170, 48, 16), (200, 24, 48), (300, 24, 16), (500, 16, 16)])
def test_projection_stage_random(dims):
    nx, ny, nz = dims
    h = 0.05
    w = synth.Workload(name="proj", nx=nx, ny=ny, nz=nz, lx=nx * h, ly=ny * h, lz=nz * h,
                       re=100.0, dt=1e-3, noise_amp=0.0)
    run, S = build_pair(w, with_noise=False)
    try:
        rng = np.random.default_rng(nx + ny + nz)
        ut = 1.0 + 0.3 * rng.standard_normal((nz, ny, nx + 1))
        vt = 0.3 * rng.standard_normal((nz, ny, nx + 1))
        wt = 0.3 * rng.standard_normal((nz, ny, nx + 1))
        ut[..., 0] = 1.0          # the inlet face of u~ is always U (state u at i = 0)
        from oracle import fluid
        fluid.flux_correct(ut)
        for arr, a in ((ib.ARR_UT, ut), (ib.ARR_VT, vt[..., :nx]), (ib.ARR_WT, wt[..., :nx])):
            ib.set_array(run.ctx, arr, a)
        ib.run_stage(run.ctx, ib.STAGE_PROJECT)
        phi_o = S.stage_project(ut.copy(), vt.copy(), wt.copy())
        u, v, ww, p, _, _ = run.fields()
        uo, vo, wo, po = S.fields()
        assert rel_l2([u, v, ww], [uo, vo, wo]) < 1e-13
        phi = ib.get_array(run.ctx, ib.ARR_PHI, (nz, ny, nx))
        assert rel_l2([demean(phi)], [demean(phi_o)]) < 1e-11
        div = fluid.divergence(u, np.concatenate([v, v[..., -1:]], 2),
                               np.concatenate([ww, ww[..., -1:]], 2), S.h)
        d0 = np.max(np.abs(fluid.divergence(ut, vt, wt, S.h)))
        assert np.max(np.abs(div)) < 1e-12 * d0
    finally:
        run.close()


def test_ibm_stage_and_maps():
    w = small_grid_flag()
    run, S = build_pair(w)
    try:
        nb = S.bar_X.shape[0]
        n_total = nb + w.flag.ns ** 2
        X, Ud, dV = S.markers()
        from oracle import delta
        for comp in range(3):
            maps = ib.get_maps(run.ctx, comp, n_total)
            o = np.array(delta.ORIGINS[comp]) * S.h
            ref = np.floor((X - o) / S.h + 0.5).astype(np.int64)
            assert np.array_equal(maps.astype(np.int64), ref)
        for st in (ib.STAGE_PREDICT, ib.STAGE_FLUX, ib.STAGE_IBM):
            ib.run_stage(run.ctx, st)
        ut, vt, wt, H = S.stage_predict()
        F = S.stage_ibm(ut, vt, wt)
        nx = w.nx
        g_ut = ib.get_array(run.ctx, ib.ARR_UT, ut.shape)
        g_vt = ib.get_array(run.ctx, ib.ARR_VT, vt[..., :nx].shape)
        g_wt = ib.get_array(run.ctx, ib.ARR_WT, wt[..., :nx].shape)
        assert rel_l2([g_ut, g_vt, g_wt], [ut, vt[..., :nx], wt[..., :nx]]) < 1e-13
        Fb = ib.get_array(run.ctx, ib.ARR_POINT_F, (nb, 3))
        assert rel_l2([Fb], [F[:nb]]) < 1e-12
        _, _, Ff = run.flag()
        assert rel_l2([Ff.reshape(-1, 3)], [F[nb:]]) < 1e-12
    finally:
        run.close()


@pytest.mark.parametrize("make,steps", [(synth.flag_64_re200, 10), (small_grid_flag, 10)])
def test_full_steps(make, steps):
    w = make()
    run, S = build_pair(w)
    try:
        errs = []
        for n in range(steps):
            run.step(1)
            S.step(1)
            u, v, ww, p, t, k = run.fields()
            uo, vo, wo, po = S.fields()
            errs.append(rel_l2([u, v, ww], [uo, vo, wo]))
        assert k == steps and abs(t - S.t) < 1e-14 * max(1.0, S.t)
        assert max(errs) < 1e-12, errs
        assert rel_l2([demean(p)], [demean(po)]) < 1e-10
        X, V, F = run.flag()
        assert rel_l2([X], [S.X.reshape(X.shape)]) < 1e-13
        # the in-plane springs are stiff (fastest mode omega dts ~ 1.8): a round-off
        # difference d in X drives velocity differences ~ omega d ~ 1e-11 relative
        assert rel_l2([V], [S.V.reshape(V.shape)]) < 1e-10
        sc = ib.get_scalars(run.ctx)
        assert sc["nsub"] == S.nsub
        assert abs(sc["dt"] - S.dt) <= 1e-12 * S.dt
    finally:
        run.close()


def test_ragged_sizes_full_step():
    """nx not a multiple of 64 (padded tridiagonal chunks), y/z lengths with radix 3."""
    w = synth.Workload(name="ragged", nx=96, ny=48, nz=24, lx=6.0, ly=3.0, lz=1.5, re=250.0,
                       dt=0.0, cfl=0.45,
                       flag=synth.Flag(ns=6, length=0.9, x_le=1.5, y_c=1.4, z_c=0.75,
                                       bending=0.02))
    run, S = build_pair(w)
    try:
        for _ in range(5):
            run.step(1)
            S.step(1)
        u, v, ww, p, t, k = run.fields()
        uo, vo, wo, po = S.fields()
        assert rel_l2([u, v, ww], [uo, vo, wo]) < 1e-12
    finally:
        run.close()


def test_unstable_is_reported():
    """A fixed dt far above the CFL limit makes the device raise EUNSTABLE."""
    w = synth.Workload(name="cfl", nx=64, ny=32, nz=32, lx=4.0, ly=2.0, lz=2.0, re=200.0,
                       dt=0.5, noise_amp=0.05)
    run, _ = build_pair(w)
    try:
        run.step(3)
        with pytest.raises(ib.IbdnsError) as e:
            run.fields()
        assert e.value.code == ib.EUNSTABLE
    finally:
        run.close()
