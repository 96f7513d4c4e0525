"""Batched ensembles: uneven-size independent runs advanced together through
ibdns_batch_* (one launch per stage over all runs, per-size launches for the
FFT and tridiagonal stages, optional hipGraph replay) give exactly the
results of the same runs stepped one by one (the batched kernels run the
same bodies), which are themselves parity-tested against the oracle."""
import numpy as np
import pytest

import synth
from oracle import geometry
from tests.test_gpu_parity import small_grid_flag

pytestmark = pytest.mark.gpu
ib = pytest.importorskip("paper_2103_08246_amd")


def members():
    return [synth.grid_flag_batch_member(96, 0, 2.0),        # 96x48x48, bars, 24x24 flag
            small_grid_flag(),                               # 48x24x24
            synth.flag_64_re200()]                           # 64x32x32, flag only


def make(w, precision=ib.FP64):
    noise = synth.ic_noise(w)
    bars = geometry.grid_points_of(w) if w.grid is not None else None
    X0 = geometry.flag_lattice(w.flag) if w.flag is not None else None
    return ib.create(ib.domain_from(w, precision=precision), noise, grid=w.grid if bars is not None else None,
                     flag=ib.flag_from(w.flag) if w.flag is not None else None)


@pytest.mark.parametrize("graph,tune,precision", [(False, False, ib.FP64), (True, False, ib.FP64),
                                                   (True, True, ib.FP64), (True, False, ib.MIXED)])
def test_batch_equals_single_runs(graph, tune, precision):
    ws = members()
    single = [make(w, precision) for w in ws]
    batched = [make(w, precision) for w in ws]
    b = ib.Batch(batched)
    try:
        if tune:
            v = b.autotune()
            assert 0 <= v < 14   # fourteen predictor tile shapes
        if graph:
            b.use_graph(True)
        b.step(6)
        for r in single:
            r.step(6)
        for rs, rb in zip(single, batched):
            a = rs.fields()
            c = rb.fields()
            for x, y in zip(a[:4], c[:4]):
                assert np.array_equal(x, y)
            assert a[4] == c[4] and a[5] == c[5] == 6
            fa, fc = rs.flag(), rb.flag()
            for x, y in zip(fa, fc):
                assert np.array_equal(x, y)
    finally:
        b.close()
        for r in single + batched:
            r.close()


def test_batch_rejects_mixed_precisions():
    ws = members()[:2]
    runs = [make(ws[0], ib.FP64), make(ws[1], ib.MIXED)]
    try:
        with pytest.raises(ib.IbdnsError) as e:
            ib.Batch(runs)
        assert e.value.code == ib.EINVAL
    finally:
        for r in runs:
            r.close()


def test_single_run_autotune_keeps_parity():
    from tests.gpu_cases import build_pair, rel_l2
    w = small_grid_flag()
    run, S = build_pair(w)
    try:
        v = ib.autotune(run.ctx)
        assert 0 <= v < 14   # fourteen predictor tile shapes
        run.step(5)
        S.step(5)
        u, vv, ww, p, t, k = run.fields()
        uo, vo, wo, po = S.fields()
        assert rel_l2([u, vv, ww], [uo, vo, wo]) < 1e-12
    finally:
        run.close()
