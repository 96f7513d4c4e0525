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
        # derived quantities of Sec. III per station, on the device
        from oracle.probes import station_statistics
        got = run.station_stats()
        own = station_statistics(rec, n_lags)            # the oracle's rule on the GPU's records
        ref_st = station_statistics(ref, n_lags)         # and on the oracle's own records
        assert len(got) == len(own) == pr["n_x"]
        for g, o, r in zip(got, own, ref_st):
            for key in ("k", "anisotropy"):
                assert abs(g[key] - o[key]) <= 1e-12 * abs(o[key]), key
                # the records agree to ~1e-11 of their scale; a variance is a
                # difference of O(1) moments, so it keeps ~1e-8 of itself
                assert abs(g[key] - r[key]) <= 1e-7 * abs(r[key]), key
            for key in ("f", "g"):
                assert g[key].shape == (n_lags,)
                # over a short transient the trend dominates the lagged products:
                # compare relative to the coefficients' size
                scale = max(1.0, float(np.max(np.abs(o[key]))))
                assert np.max(np.abs(g[key] - o[key])) <= 1e-11 * scale, key
                assert np.max(np.abs(g[key] - r[key])) <= 1e-6 * scale, key
            assert g["f"][0] == pytest.approx(1.0, abs=1e-12) and g["g"][0] == pytest.approx(1.0, abs=1e-12)
    finally:
        run.close()


def test_station_stats_unpaired_lags_and_rules():
    """Lags longer than the record have no pair: NaN; a short or misaligned
    staging buffer and a run without probes are refused."""
    import ctypes
    w = small_grid_flag()
    run = ib.create(ib.domain_from(w), synth.ic_noise(w), grid=w.grid, flag=w.flag)
    try:
        with pytest.raises(ib.IbdnsError) as e:
            run.station_stats()
        assert e.value.code == ib.ESTATE
        pr = synth.probe_layout(w, 7)
        run.set_probes(pr["n_x"], pr["x0"], pr["dx"], pr["yc"], pr["zc"], pr["dyz"], 7)
        run.step(5)
        st = run.station_stats()
        for s in st:
            assert np.all(np.isfinite(s["f"][:5])) and np.all(np.isnan(s["f"][5:]))
            assert np.all(np.isfinite(s["g"][:5])) and np.all(np.isnan(s["g"][5:]))
            assert s["k"] > 0
        import torch
        lib = ib.lib()
        ws = torch.empty(1 << 16, dtype=torch.uint8, device="cuda:0")
        out = np.empty((pr["n_x"], 16))
        D = ctypes.POINTER(ctypes.c_double)
        assert lib.ibdns_get_station_stats(run.ctx, ctypes.c_void_p(ws.data_ptr()), 64,
                                           out.ctypes.data_as(D)) == ib.ENOMEM
        assert lib.ibdns_get_station_stats(run.ctx, ctypes.c_void_p(ws.data_ptr() + 8), ws.numel() - 8,
                                           out.ctypes.data_as(D)) == ib.EINVAL
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
