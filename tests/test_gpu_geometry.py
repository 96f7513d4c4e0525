"""The bodies the library builds from the problem statement (Sec. II.A) against
the oracle's own construction (oracle/geometry.py): the passive grid's solid
points and volumes, and the flag's reference lattice, bit for bit, on the
workloads' meshes (nc = 1, 2, 3, 6 points per rod side)."""
import numpy as np
import pytest

import synth
from oracle import geometry
from tests.test_gpu_parity import small_grid_flag

pytestmark = pytest.mark.gpu
ib = pytest.importorskip("paper_2103_08246_amd")


@pytest.mark.parametrize("make", [
    small_grid_flag,
    lambda: synth.grid_flag_batch_member(96, 0, 2.0),
    lambda: synth.grid_flag_batch_member(192, 16, 10.0),
    lambda: synth.grid_flag_batch_member(384, 0, 3.0, ns=64, re=1000.0),
    synth.grid_flag_768_re1000,
], ids=["small", "96", "192", "384", "768"])
def test_bodies_bit_exact(make):
    w = make()
    run = ib.create(ib.domain_from(w), None, grid=w.grid, flag=w.flag)
    try:
        X, dV = ib.get_grid_points(run.ctx)
        Xo, dVo = geometry.grid_points_of(w)
        assert X.shape == Xo.shape and X.shape[0] > 0
        assert np.array_equal(X, Xo)
        assert np.array_equal(dV, dVo)
        Xf, Vf, _ = run.flag()
        assert np.array_equal(Xf, geometry.flag_lattice(w.flag))
        assert np.all(Vf == 0.0)
    finally:
        run.close()


def test_no_grid_no_points():
    w = synth.flag_64_re200()
    run = ib.create(ib.domain_from(w), None, flag=w.flag)
    try:
        X, dV = ib.get_grid_points(run.ctx)
        assert X.shape == (0, 3) and dV.shape == (0,)
    finally:
        run.close()
