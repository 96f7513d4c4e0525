"""Acceptance runs on the 768 x 384 x 384 workload (113M cells, Re 1000,
passive grid of 300,672 solid points, 96 x 96 flag, dt from CFL 0.5), in the
launch configuration the bench times (autotuned predictor tile), against the
oracle (the C fluid stages of oracle/fast.py, pinned stage by stage to the
numpy oracle, with the numpy flag model):

* plain FP64, 10 steps: velocity relative L2 <= 1e-12, the target stated for
  the plain path; flag positions <= 1e-13; the same flag sub-step counts,
  time step and time; pressure (mean removed) <= 1e-9: every Poisson solve
  carries a round-off of about cond(L) eps = (12 nx^2 / pi^2) eps ~ 1e-10 at
  nx = 768 for its low x modes, and p sums ten of them;
* mixed precision (FP32 RHS/predictor and immersed-boundary transfer, FP64
  state, Poisson solve, projection and flag), 100 steps from the same inputs
  and seed: velocity relative L2 <= 1e-5 and max |div u| <= 1e-10 against the
  oracle's 100 steps, the form's stated target; the FP64 path after the same
  100 steps stays within 1e-10 of the oracle.

Progress lines go to the terminal while the oracle steps (about 2 s per step
on 16 host threads).
"""
import time

import numpy as np
import pytest

import synth
from oracle import fast, fluid, geometry
from tests.gpu_cases import demean, oracle_flag_args, rel_l2

pytestmark = pytest.mark.gpu
ib = pytest.importorskip("paper_2103_08246_amd")


def _say(capsys, msg):
    with capsys.disabled():
        print(f"  [{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def _max_div(run, w, u, v, ww):
    vg = ib.get_array(run.ctx, ib.ARR_V_GHOST, (w.nz, w.ny))
    wg = ib.get_array(run.ctx, ib.ARR_W_GHOST, (w.nz, w.ny))
    d = fluid.divergence(u, np.concatenate([v, vg[..., None]], 2), np.concatenate([ww, wg[..., None]], 2), w.h)
    return float(np.max(np.abs(d)))


def _oracle(w, noise, capsys):
    bars = geometry.grid_points_of(w)
    X0 = geometry.flag_lattice(w.flag)
    t0 = time.time()
    C = fast.FastSolver(w, noise, bars, oracle_flag_args(w, X0))
    _say(capsys, f"oracle ready ({fast.threads()} threads, {time.time() - t0:.0f} s)")
    return C


def _step_oracle(C, n, capsys):
    for s in range(n):
        t0 = time.time()
        C.step(1)
        _say(capsys, f"oracle step {C.step_count} ({time.time() - t0:.1f} s, dt {C.dt:.6f})")


def test_fp64_ten_steps_vs_oracle(capsys):
    w = synth.grid_flag_768_re1000()
    noise = synth.ic_noise(w)
    run = ib.create(ib.domain_from(w), noise, grid=w.grid, flag=w.flag)
    try:
        variant = ib.autotune(run.ctx)
        _say(capsys, f"GPU run ready, tile {variant}")
        C = _oracle(w, noise, capsys)
        del noise
        assert ib.get_scalars(run.ctx)["dt"] == pytest.approx(C.dt, rel=1e-13)
        run.step(10)
        ib.sync(run.ctx)
        _step_oracle(C, 10, capsys)
        u, v, ww, p, t, k = run.fields()
        uo, vo, wo, po = C.fields()
        err = rel_l2([u, v, ww], [uo, vo, wo])
        _say(capsys, f"velocity rel L2 after 10 steps: {err:.3e}")
        assert k == 10 and abs(t - C.t) <= 1e-12 * C.t
        assert err <= 1e-12, err
        assert rel_l2([demean(p)], [demean(po)]) <= 1e-9
        X, V, F = run.flag()
        assert rel_l2([X], [C.X.reshape(X.shape)]) <= 1e-13
        sc = ib.get_scalars(run.ctx)
        assert sc["nsub"] == C.nsub
        assert abs(sc["dt"] - C.dt) <= 1e-12 * C.dt
    finally:
        run.close()


def test_mixed_hundred_steps_vs_oracle(capsys):
    w = synth.grid_flag_768_re1000()
    noise = synth.ic_noise(w)
    runs = {}
    try:
        for prec in (ib.FP64, ib.MIXED):
            runs[prec] = ib.create(ib.domain_from(w, precision=prec), noise, grid=w.grid, flag=w.flag)
            ib.autotune(runs[prec].ctx)
            runs[prec].step(100)
            ib.sync(runs[prec].ctx)
        _say(capsys, "GPU runs (FP64, mixed) stepped 100 times")
        C = _oracle(w, noise, capsys)
        del noise
        _step_oracle(C, 100, capsys)
        oref = C.fields()
        res = {}
        for prec, name in ((ib.FP64, "fp64"), (ib.MIXED, "mixed")):
            f = runs[prec].fields()
            assert f[5] == 100
            res[name] = (rel_l2(f[:3], oref[:3]), _max_div(runs[prec], w, *f[:3]),
                         rel_l2([runs[prec].flag()[0]], [C.X.reshape(w.flag.ns, w.flag.ns, 3)]))
            _say(capsys, f"{name} after 100 steps vs oracle: velocity rel L2 {res[name][0]:.3e}, "
                         f"max|div| {res[name][1]:.3e}, flag X rel L2 {res[name][2]:.3e}")
        assert 1e-12 < res["mixed"][0] <= 1e-5, res
        assert res["mixed"][1] <= 1e-10, res
        assert res["fp64"][0] <= 1e-10 and res["fp64"][1] <= 1e-10, res
    finally:
        for r in runs.values():
            r.close()
