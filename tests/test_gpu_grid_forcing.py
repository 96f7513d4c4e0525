"""Eulerian forcing of the passive grid (Sec. II.B (i)) on the GPU against the
oracle: the forcing lists node by node, then full coupled steps (grid forced
at its nodes, flag by delta markers); plus the argument and state checks."""
import numpy as np
import pytest

import synth
from oracle import geometry
from tests.gpu_cases import oracle_flag_args, rel_l2
from tests.test_gpu_parity import small_grid_flag

pytestmark = pytest.mark.gpu
ib = pytest.importorskip("paper_2103_08246_amd")


def _oracle_lists(w):
    from oracle import grid_forcing as gf
    g = w.grid
    geom = gf.GridGeometry(g.x_plane, g.mesh, g.bar, w.ly, w.lz)
    out = []
    for comp in range(3):
        NX = w.nx + 1 if comp == 0 else w.nx
        lst = gf.forcing_list(geom, comp, w.nx, w.ny, w.nz, w.lx / w.nx)
        node = np.array([i + NX * (j + w.ny * k) for (k, j, i, kq, jq, iq, wt) in lst], dtype=np.int64)
        src = np.array([-1 if iq < 0 else iq + NX * (jq + w.ny * kq)
                        for (k, j, i, kq, jq, iq, wt) in lst], dtype=np.int64)
        wgt = np.array([wt for (*_, wt) in lst])
        out.append((node, src, wgt))
    return out


def _make(w, flag=True):
    X0 = geometry.flag_lattice(w.flag) if flag else None
    return ib.create(ib.domain_from(w), synth.ic_noise(w), flag=ib.flag_from(w.flag) if flag else None, grid_forcing=w.grid)


def test_lists_match_oracle():
    w = small_grid_flag()
    run = _make(w, flag=False)
    try:
        for comp, (node, src, wgt) in enumerate(_oracle_lists(w)):
            gn, gs, gw = run.grid_forcing(comp)
            assert np.array_equal(gn, node), comp
            assert np.array_equal(gs, src), comp
            assert np.max(np.abs(gw - wgt)) <= 1e-15, comp
            assert np.sum(gs < 0) > 0 and np.sum(gs >= 0) > 0
    finally:
        run.close()


def test_steps_match_oracle():
    from oracle.solver import Solver
    w = small_grid_flag()
    X0 = geometry.flag_lattice(w.flag)
    g = w.grid
    S = Solver(w, synth.ic_noise(w), None, oracle_flag_args(w, X0),
               grid_forcing=dict(x_plane=g.x_plane, mesh=g.mesh, bar=g.bar))
    run = _make(w)
    try:
        for _ in range(10):
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


def test_grid_forcing_state_rules():
    w = small_grid_flag()
    run = ib.create(ib.domain_from(w), synth.ic_noise(w), grid_forcing=w.grid)
    try:
        with pytest.raises(ib.IbdnsError) as e:      # points and node forcing exclude each other
            ib.set_geometry(run.ctx, ib.grid_from(w.grid))
        assert e.value.code == ib.EINVAL
        with pytest.raises(ib.IbdnsError) as e:      # once
            run.set_grid_forcing(ib.domain_from(w), ib.grid_from(w.grid))
        assert e.value.code == ib.ESTATE
        with pytest.raises(ib.IbdnsError) as e:      # batches take grids as points only
            ib.Batch([run])
        assert e.value.code == ib.EINVAL
    finally:
        run.close()
    plain = ib.create(ib.domain_from(w), synth.ic_noise(w))
    try:
        with pytest.raises(ib.IbdnsError) as e:
            plain.grid_forcing(0)
        assert e.value.code == ib.ESTATE
        with pytest.raises(ib.IbdnsError) as e:      # rods reaching the inlet
            plain.set_grid_forcing(ib.domain_from(w), ib.GridParams(0.1, w.grid.mesh, w.grid.bar))
        assert e.value.code == ib.EINVAL
    finally:
        plain.close()
