"""Element-wise oracle parity of the exact kernel instances the bench times.

* The predictor (RHS + AB2 step) in every tile shape the autotuner may pick,
  FP64 and mixed precision, on boxes whose extents leave ragged last tiles
  wherever the supported lengths allow it, after one full step so that the
  Adams-Bashforth history H^{n-1} differs from H^n.
* The projection stage (divergence + y FFT, z FFT, x tridiagonal solve,
  inverse FFTs, projection) with the transform lengths and x-line lengths of
  the 768 x 384 x 384 workload: y and z FFTs of 384 and 192 (radix 8 8 6
  and 8 8 3) and x lines of 768, 384 and 192, in FP64 and with the FP32
  provisional velocity of the mixed form.

Tolerances: FP64 stages are the same formulas up to summation order and FMA
contraction (a few ulp: 1e-14 for the predictor, 1e-13 for the projection);
the mixed predictor computes in FP32 (unit round-off 6e-8: 1e-6 relative L2).
"""
import numpy as np
import pytest

import synth
from oracle import fluid
from tests.gpu_cases import build_pair, demean, rel_l2

pytestmark = pytest.mark.gpu
ib = pytest.importorskip("paper_2103_08246_amd")

# y and z lengths are FFT lengths, multiples of 8 (16, 24, 32, 48, ... 768), so
# tiles of 4 or 8 rows and 8 planes always divide them; every other tile
# extent leaves a ragged last tile in one of the boxes: x 200 and 136 against
# 32, 64, 128, 256; y 24 against 16; z 32 against 24 and 48, z 24 against 16,
# 32 and 48.
BOXES = [(200, 24, 32), (136, 48, 24)]


def _box(nx, ny, nz, dt=0.0):
    h = 0.05
    return synth.Workload(name="tile_box", nx=nx, ny=ny, nz=nz, lx=nx * h, ly=ny * h, lz=nz * h,
                          re=150.0, dt=dt, cfl=0.4, noise_amp=0.2)


@pytest.mark.parametrize("box", BOXES, ids=["200x24x32", "136x48x24"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("variant", range(14))
def test_predictor_every_tile(variant, precision, box):
    w = _box(*box)
    prec = ib.FP64 if precision == "fp64" else ib.MIXED
    run, S = build_pair(w, precision=prec)
    try:
        ib.set_tile(run.ctx, variant)
        run.step(1)
        S.step(1)
        if prec == ib.MIXED:
            # restart the oracle from the GPU's FP64 state so that only this
            # predictor's FP32 arithmetic is compared
            from oracle.solver import set_state
            u, v, ww, p, _, _ = run.fields()
            Hold = [ib.get_array(run.ctx, a, s) for a, s in ((ib.ARR_HU, u.shape), (ib.ARR_HV, v.shape),
                                                              (ib.ARR_HW, ww.shape))]
            sc = ib.get_scalars(run.ctx)
            vg = ib.get_array(run.ctx, ib.ARR_V_GHOST, (w.nz, w.ny))
            wg = ib.get_array(run.ctx, ib.ARR_W_GHOST, (w.nz, w.ny))
            set_state(S, u, np.concatenate([v, vg[..., None]], 2), np.concatenate([ww, wg[..., None]], 2), p)
            S.dt, S.dt_prev = sc["dt"], sc["dt_prev"]
            nx = w.nx
            S.H_old = [Hold[0], np.concatenate([Hold[1], np.zeros((w.nz, w.ny, 1))], 2),
                       np.concatenate([Hold[2], np.zeros((w.nz, w.ny, 1))], 2)]
        ib.run_stage(run.ctx, ib.STAGE_PREDICT)
        ib.run_stage(run.ctx, ib.STAGE_FLUX)
        ut, vt, wt, H = S.stage_predict()
        nx = w.nx
        g_ut = ib.get_array(run.ctx, ib.ARR_UT, ut.shape)
        g_vt = ib.get_array(run.ctx, ib.ARR_VT, vt[..., :nx].shape)
        g_wt = ib.get_array(run.ctx, ib.ARR_WT, wt[..., :nx].shape)
        g_hu = ib.get_array(run.ctx, ib.ARR_HU, ut.shape)
        g_hw = ib.get_array(run.ctx, ib.ARR_HW, wt[..., :nx].shape)
        tol_u, tol_h = (1e-14, 1e-13) if prec == ib.FP64 else (1e-6, 1e-5)
        assert rel_l2([g_ut, g_vt, g_wt], [ut, vt[..., :nx], wt[..., :nx]]) < tol_u
        assert rel_l2([g_hu[..., 1:nx], g_hw], [H[0][..., 1:nx], H[2][..., :nx]]) < tol_h
    finally:
        run.close()


@pytest.mark.parametrize("dims", [(16, 384, 384), (768, 24, 24), (384, 192, 24), (192, 24, 192)],
                         ids=["fft384", "tri768", "tri384_ffty192", "tri192_fftz192"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_projection_workload_lengths(dims, precision):
    nx, ny, nz = dims
    h = 0.05
    w = synth.Workload(name="proj", nx=nx, ny=ny, nz=nz, lx=nx * h, ly=ny * h, lz=nz * h,
                       re=100.0, dt=1e-3, noise_amp=0.0)
    prec = ib.FP64 if precision == "fp64" else ib.MIXED
    run, S = build_pair(w, with_noise=False, precision=prec)
    try:
        rng = np.random.default_rng(nx + 3 * ny + 7 * nz)
        ut = 1.0 + 0.3 * rng.standard_normal((nz, ny, nx + 1))
        vt = 0.3 * rng.standard_normal((nz, ny, nx + 1))
        wt = 0.3 * rng.standard_normal((nz, ny, nx + 1))
        ut[..., 0] = 1.0          # the inlet face of u~ is always U (state u at i = 0)
        if prec == ib.MIXED:      # the provisional interior is stored in FP32
            ut[..., 1:nx] = ut[..., 1:nx].astype(np.float32)
            vt[..., :nx] = vt[..., :nx].astype(np.float32)
            wt[..., :nx] = wt[..., :nx].astype(np.float32)
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


def test_tile_index_is_checked():
    w = _box(64, 32, 32, dt=1e-3)
    run = ib.create(ib.domain_from(w), None)
    try:
        for bad in (-1, ib.NUM_TILES):
            with pytest.raises(ib.IbdnsError) as e:
                ib.set_tile(run.ctx, bad)
            assert e.value.code == ib.EINVAL
    finally:
        run.close()
