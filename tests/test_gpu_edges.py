"""Edge cases of the GPU time step, through the C ABI.

- The time step runs the flag's sub-steps on a second stream, concurrent with
  the spreading and the pressure solve (plain launch); the stage-by-stage path
  runs them in order on one stream (cooperative launch).  Both must give the
  same bits.
- A flag of the largest supported size (128 x 128 nodes, 16 bands) keeps
  oracle parity.
- A flag whose support reaches the inlet (outside the evolved x range) is
  refused, not silently clipped.
"""
import numpy as np
import pytest

import synth
from oracle import geometry
from tests.gpu_cases import build_pair, rel_l2

pytestmark = pytest.mark.gpu
ib = pytest.importorskip("paper_2103_08246_amd")


def _make(w):
    noise = synth.ic_noise(w)
    bars = geometry.grid_points_of(w) if w.grid is not None else None
    X0 = geometry.flag_lattice(w.flag) if w.flag is not None else None
    return ib.create(ib.domain_from(w), noise, grid=w.grid if bars is not None else None,
                     flag=ib.flag_from(w.flag) if w.flag is not None else None)


def _grid_flag():
    return synth.Workload(name="edge_grid_flag", nx=64, ny=32, nz=32, lx=4.0, ly=2.0, lz=2.0,
                          re=300.0, dt=0.0, cfl=0.4,
                          grid=synth.Grid(x_plane=0.5, mesh=1.0, bar=0.2),
                          flag=synth.Flag(ns=12, length=0.8, x_le=1.6, y_c=1.0, z_c=1.0,
                                          bending=0.01))


def test_overlapped_step_equals_stage_sequence():
    w = _grid_flag()
    a = _make(w)
    b = _make(w)
    try:
        a.step(4)
        for _ in range(4):
            for st in (ib.STAGE_PREDICT, ib.STAGE_FLUX, ib.STAGE_IBM, ib.STAGE_PROJECT,
                       ib.STAGE_FLAG, ib.STAGE_ADVANCE):
                ib.run_stage(b.ctx, st)
        fa, fb = a.fields(), b.fields()
        for x, y in zip(fa[:4], fb[:4]):
            assert np.array_equal(x, y)
        assert fa[4] == fb[4] and fa[5] == fb[5]
        for x, y in zip(a.flag(), b.flag()):
            assert np.array_equal(x, y)
    finally:
        a.close()
        b.close()


def test_largest_flag_parity():
    """128 x 128 nodes: 16 bands of 8 rows, one node per thread."""
    w = synth.Workload(name="big_flag", nx=64, ny=32, nz=32, lx=4.0, ly=2.0, lz=2.0, re=200.0,
                       dt=1e-3, flag=synth.Flag(ns=128, length=1.0, x_le=1.0, y_c=1.0, z_c=1.0,
                                                bending=0.01))
    run, S = build_pair(w)
    try:
        for _ in range(3):
            run.step(1)
            S.step(1)
        u, v, ww, p, t, k = run.fields()
        uo, vo, wo, po = S.fields()
        assert rel_l2([u, v, ww], [uo, vo, wo]) < 1e-12
        X, V, F = run.flag()
        assert rel_l2([X], [S.X.reshape(X.shape)]) < 1e-13
        assert ib.get_scalars(run.ctx)["nsub"] == S.nsub
    finally:
        run.close()


@pytest.mark.parametrize("path", ["step", "stages"])
def test_flag_band_wait_timeout_is_reported(path):
    """A 48 x 48 flag runs in three bands that exchange edge rows every
    sub-step.  With the test hook the bands wait for a count their neighbours
    never reach, under a spin limit of 64 polls: every band gives up, every
    kernel ends, and the step reports ETIMEOUT, which stays set.  Both the
    time step (flag on the second stream, plain launch) and the stage path
    (cooperative launch)."""
    w = synth.Workload(name="wait_flag", nx=64, ny=32, nz=32, lx=4.0, ly=2.0, lz=2.0, re=200.0,
                       dt=1e-3, flag=synth.Flag(ns=48, length=1.0, x_le=1.0, y_c=1.0, z_c=1.0,
                                                bending=0.01))
    run = ib.create(ib.domain_from(w, flags=ib.TEST_FLAG_WAIT_TIMEOUT), synth.ic_noise(w), flag=w.flag)
    try:
        if path == "step":
            run.step(1)
        else:
            for st in (ib.STAGE_PREDICT, ib.STAGE_FLUX, ib.STAGE_IBM, ib.STAGE_PROJECT, ib.STAGE_FLAG,
                       ib.STAGE_ADVANCE):
                ib.run_stage(run.ctx, st)
        with pytest.raises(ib.IbdnsError) as e:
            ib.sync(run.ctx)
        assert e.value.code == ib.ETIMEOUT
        with pytest.raises(ib.IbdnsError) as e:
            run.fields()
        assert e.value.code == ib.ETIMEOUT
    finally:
        run.close()


@pytest.mark.parametrize("ns", [32, 33, 48, 121])
def test_flag_band_shapes_parity(ns):
    """Bands of min(ns, 1024 // ns) rows: 32 is one band of 1024 nodes, 33 two
    bands (31 + 2 rows), 48 three (21 + 21 + 6), 121 sixteen with a last band
    of one row."""
    w = synth.Workload(name=f"flag_bands_{ns}", nx=64, ny=32, nz=32, lx=4.0, ly=2.0, lz=2.0,
                       re=200.0, dt=1e-3, flag=synth.Flag(ns=ns, length=1.0, x_le=1.0, y_c=1.0,
                                                          z_c=1.0, bending=0.01))
    run, S = build_pair(w)
    try:
        for _ in range(2):
            run.step(1)
            S.step(1)
        u, v, ww, p, t, k = run.fields()
        uo, vo, wo, po = S.fields()
        assert rel_l2([u, v, ww], [uo, vo, wo]) < 1e-12
        X, V, F = run.flag()
        assert rel_l2([X], [S.X.reshape(X.shape)]) < 1e-13
        assert rel_l2([V], [S.V.reshape(V.shape)]) < 1e-9
        assert ib.get_scalars(run.ctx)["nsub"] == S.nsub
    finally:
        run.close()


def test_flag_support_outside_x_range_is_rejected():
    """Leading edge half a cell behind the inlet: its support leaves the evolved
    x range, and set_geometry refuses it (a flag that drifts out later is
    reported by the step's status word instead)."""
    w = synth.Workload(name="flag_at_inlet", nx=64, ny=32, nz=32, lx=4.0, ly=2.0, lz=2.0,
                       re=200.0, dt=1e-3, flag=synth.Flag(ns=8, length=0.5, x_le=0.03, y_c=1.0,
                                                          z_c=1.0, bending=0.01))
    with pytest.raises(ib.IbdnsError) as e:
        _make(w)
    assert e.value.code == ib.EINVAL
