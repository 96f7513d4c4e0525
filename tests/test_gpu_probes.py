"""Virtual probes on the GPU (Sec. III) against the oracle's probe statistics:
the same seeded run, probes sampled after every projection, records compared
entry by entry; plus the argument checks of ibdns_set_probes."""
import numpy as np
import pytest

import synth
from oracle import geometry
from tests.gpu_cases import oracle_flag_args
from tests.test_gpu_parity import small_grid_flag

pytestmark = pytest.mark.gpu
ib = pytest.importorskip("paper_2103_08246_amd")


def _rel_max(a, b):
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


@pytest.mark.parametrize("n_lags,steps", [(1, 10), (7, 10), (70, 72)])
def test_probe_records_match_oracle(n_lags, steps):
    """70 lags over 72 steps: lanes take lags l and l + 64, and the ring wraps."""
    from oracle.solver import Solver
    w = small_grid_flag()
    pr = synth.probe_layout(w, n_lags)
    noise = synth.ic_noise(w)
    X0 = geometry.flag_lattice(w.flag)
    S = Solver(w, noise, geometry.grid_points_of(w), oracle_flag_args(w, X0), probes=pr)
    run = ib.create(ib.domain_from(w), noise, grid=w.grid,
                    flag=ib.flag_from(w.flag))
    try:
        run.set_probes(pr["n_x"], pr["x0"], pr["dx"], pr["yc"], pr["zc"], pr["dyz"], n_lags)
        for _ in range(steps):
            run.step(1)
            S.step(1)
        rec = run.probe_stats()
        ref = S.probes.rec
        assert rec.shape == ref.shape == (9 * pr["n_x"], 10 + 2 * n_lags)
        assert np.all(rec[:, 0] == steps)
        # sums of sampled velocities: the fields agree to ~1e-13, so do the sums
        assert _rel_max(rec[:, 1:10], ref[:, 1:10]) < 1e-11
        assert _rel_max(rec[:, 10:], ref[:, 10:]) < 1e-11
    finally:
        run.close()


def test_probe_arguments_are_checked():
    w = small_grid_flag()
    run = ib.create(ib.domain_from(w), synth.ic_noise(w))
    try:
        with pytest.raises(ib.IbdnsError) as e:
            run.probe_stats()
        assert e.value.code == ib.ESTATE
        h = w.lx / w.nx
        # v and w are sampled on cell centres: x below h/2 has no left node
        with pytest.raises(ib.IbdnsError) as e:
            run.set_probes(1, 0.25 * h, 1.0, 1.5, 1.5, 0.5, 4)
        assert e.value.code == ib.EINVAL
        # the last station's stencil must stop at the last cell
        with pytest.raises(ib.IbdnsError) as e:
            run.set_probes(2, w.lx - 0.6 * h, 0.5 * h, 1.5, 1.5, 0.5, 4)
        assert e.value.code == ib.EINVAL
        with pytest.raises(ib.IbdnsError) as e:
            run.set_probes(1, 3.0, 1.0, 1.5, 1.5, 0.5, 0)
        assert e.value.code == ib.EINVAL
        run.set_probes(1, 3.0, 1.0, 1.5, 1.5, 0.5, 4)
        assert np.all(run.probe_stats()[:, 0] == 0)
        run.step(2)
        assert np.all(run.probe_stats()[:, 0] == 2)
    finally:
        run.close()
