"""Parity at the full paper-like size (768 x 384 x 384, 113M cells, grid bars
and a 96 x 96 flag) in the launch configuration bench.py times.

The oracle cannot step this size in test time, so: index maps of every
immersed point bit for bit; the provisional velocity on x-slabs around the
bars and the flag against the oracle's RHS/predictor evaluated on the same
slab; after whole steps, properties that hold at any size (divergence at
machine level, outflow = inflow, finite fields, inextensible flag).
"""
import numpy as np
import pytest

import synth
from oracle import geometry
from tests.gpu_cases import rel_l2

pytestmark = pytest.mark.gpu
ib = pytest.importorskip("paper_2103_08246_amd")


@pytest.fixture(scope="module")
def full():
    w = synth.grid_flag_768_re1000()
    noise = synth.ic_noise(w)
    bars = geometry.grid_points_of(w)
    X0 = geometry.flag_lattice(w.flag)
    run = ib.create(ib.domain_from(w), noise, grid=w.grid if bars is not None else None, flag=ib.flag_from(w.flag))
    yield w, run, bars, X0
    run.close()


def test_maps_bit_exact(full):
    w, run, bars, X0 = full
    X = np.concatenate([bars[0], X0.reshape(-1, 3)])
    h = w.h
    for comp in range(3):
        maps = ib.get_maps(run.ctx, comp, X.shape[0]).astype(np.int64)
        o = np.array([0.0 if d == comp else 0.5 * h for d in range(3)])
        ref = np.floor((X - o) / h + 0.5).astype(np.int64)
        assert np.array_equal(maps, ref)


def test_predictor_slabs_match_oracle(full):
    from oracle import fluid
    w, run, bars, X0 = full
    nx, ny, nz = w.nx, w.ny, w.nz
    u, v, ww, p, _, _ = run.fields()
    vg = ib.get_array(run.ctx, ib.ARR_V_GHOST, (nz, ny))
    wg = ib.get_array(run.ctx, ib.ARR_W_GHOST, (nz, ny))
    sc = ib.get_scalars(run.ctx)
    ib.run_stage(run.ctx, ib.STAGE_PREDICT)
    ut = ib.get_array(run.ctx, ib.ARR_UT, (nz, ny, nx + 1))
    vt = ib.get_array(run.ctx, ib.ARR_VT, (nz, ny, nx))
    wt = ib.get_array(run.ctx, ib.ARR_WT, (nz, ny, nx))
    h, nu = w.h, 1.0 / w.re
    for i0, n in ((4, 28), (200, 24), (740, 28)):     # bars, flag, outlet
        hi = min(i0 + n, nx)
        # oracle slab: faces i0..hi, cells i0..hi-1 (+ ghost column)
        us = u[..., i0:hi + 1]
        vs = np.concatenate([v[..., i0:hi], (vg if hi == nx else v[..., hi])[..., None]], 2)
        ws = np.concatenate([ww[..., i0:hi], (wg if hi == nx else ww[..., hi])[..., None]], 2)
        F = fluid.Fields(u=us, v=vs, w=ws, p=p[..., i0:hi])
        H = fluid.rhs(F, h, nu)
        uto, vto, wto = fluid.predictor(F, H, H, sc["dt"], 1.0, h)
        # compare away from the slab's own x ends (the oracle treats them as boundaries)
        a = 1 if i0 > 0 else 0
        b = (hi - i0) - (0 if hi == nx else 1)
        assert rel_l2([ut[..., i0 + a + 1:i0 + b]], [uto[..., a + 1:b]]) < 1e-14
        assert rel_l2([vt[..., i0 + a:i0 + b], wt[..., i0 + a:i0 + b]],
                      [vto[..., a:b], wto[..., a:b]]) < 1e-14


def test_steps_properties(full):
    from oracle import fluid
    w, run, bars, X0 = full
    run.step(3)
    u, v, ww, p, t, k = run.fields()
    assert np.all(np.isfinite(u)) and np.all(np.isfinite(v)) and np.all(np.isfinite(ww))
    vg = ib.get_array(run.ctx, ib.ARR_V_GHOST, (w.nz, w.ny))
    wg = ib.get_array(run.ctx, ib.ARR_W_GHOST, (w.nz, w.ny))
    div = fluid.divergence(u, np.concatenate([v, vg[..., None]], 2),
                           np.concatenate([ww, wg[..., None]], 2), w.h)
    assert np.max(np.abs(div)) < 1e-10
    assert abs(np.sum(u[..., -1]) - np.sum(u[..., 0])) < 1e-12 * u[..., 0].size
    X, V, F = run.flag()
    assert np.all(np.isfinite(X)) and np.array_equal(X[:, 0], X0[:, 0])
    d = X[:, 1:] - X[:, :-1]
    strain = np.abs(np.sqrt(np.sum(d * d, -1)) / (w.flag.length / (w.flag.ns - 1)) - 1)
    assert np.max(strain) < 5e-3
