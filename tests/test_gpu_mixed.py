"""Mixed precision (FP32 RHS/predictor and immersed-boundary transfer, FP64
state, Poisson solve, projection and flag) against the FP64 oracle.

The stated accuracy target for this form: velocity relative L2 <= 1e-5 and
divergence <= 1e-10 after 100 steps.  The divergence bound holds because the
projection runs in FP64 on the exact FP32 values of the provisional velocity,
with FP64 boundary faces.  The same check at the full 768 x 384 x 384 size is
in tests/test_gpu_acceptance.py.
"""
import numpy as np
import pytest

import synth
from oracle import geometry
from oracle import fluid
from tests.gpu_cases import build_pair, rel_l2
from tests.test_gpu_parity import small_grid_flag

pytestmark = pytest.mark.gpu
ib = pytest.importorskip("paper_2103_08246_amd")


def _div_max(run, w, u, v, ww):
    vg = ib.get_array(run.ctx, ib.ARR_V_GHOST, (w.nz, w.ny))
    wg = ib.get_array(run.ctx, ib.ARR_W_GHOST, (w.nz, w.ny))
    d = fluid.divergence(u, np.concatenate([v, vg[..., None]], 2),
                         np.concatenate([ww, wg[..., None]], 2), w.h)
    return float(np.max(np.abs(d)))


@pytest.mark.parametrize("make", [synth.flag_64_re200, small_grid_flag])
def test_mixed_100_steps_vs_fp64_oracle(make):
    w = make()
    import paper_2103_08246_amd as ibm
    from oracle.solver import Solver
    from tests.gpu_cases import oracle_flag_args
    noise = synth.ic_noise(w)
    bars = geometry.grid_points_of(w) if w.grid is not None else None
    X0 = geometry.flag_lattice(w.flag)
    run = ibm.create(ibm.domain_from(w, precision=ibm.MIXED), noise, grid=w.grid if bars is not None else None,
                     flag=ibm.flag_from(w.flag))
    S = Solver(w, noise, bars, oracle_flag_args(w, X0))
    try:
        run.step(100)
        S.step(100)
        u, v, ww, p, t, k = run.fields()
        uo, vo, wo, po = S.fields()
        err = rel_l2([u, v, ww], [uo, vo, wo])
        assert err < 1e-5, err
        assert err > 1e-12        # really ran in FP32
        assert _div_max(run, w, u, v, ww) < 1e-10
        X, V, F = run.flag()
        assert rel_l2([X], [S.X.reshape(X.shape)]) < 1e-6
    finally:
        run.close()
