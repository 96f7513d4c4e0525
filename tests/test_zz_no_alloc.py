"""The station statistics without allocation (ibdns_get_station_stats_noalloc,
staging in the library's static device array) against the workspace form
(ibdns_get_station_stats) through the C ABI: bit for bit, on two calls in a
row, the second with fewer stations and lags; sizes beyond the static array
are refused."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
ib = pytest.importorskip("paper_2103_08246_amd")

D = ctypes.POINTER(ctypes.c_double)


def _small():
    return synth.Workload(name="noalloc_small", nx=48, ny=24, nz=24, lx=6.0, ly=3.0, lz=3.0, re=300.0,
                          dt=0.0, cfl=0.4, grid=synth.Grid(x_plane=0.75, mesh=1.5, bar=0.3),
                          flag=synth.Flag(ns=8, length=1.0, x_le=2.0, y_c=1.5, z_c=1.5, bending=0.01))


def _noalloc(run, n_x, L):
    out = np.full((n_x, 2 + 2 * L), -7.0)
    code = ib.lib().ibdns_get_station_stats_noalloc(run.ctx, out.ctypes.data_as(D))
    return code, out


def _workspace(run, n_x, L):
    import torch
    ws = torch.empty(max(256, n_x * (2 + 2 * L) * 8), dtype=torch.uint8, device="cuda:0")
    out = np.full((n_x, 2 + 2 * L), -9.0)
    code = ib.lib().ibdns_get_station_stats(run.ctx, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                            out.ctypes.data_as(D))
    assert code == ib.OK
    return out


def test_noalloc_equals_workspace_form_twice():
    w = _small()
    run = ib.create(ib.domain_from(w), synth.ic_noise(w), grid=w.grid, flag=w.flag)
    try:
        # first call: 12 stations, 9 lags, 12 samples
        run.set_probes(12, 0.9, 0.35, 1.5, 1.5, 0.5, 9)
        run.step(12)
        code, a = _noalloc(run, 12, 9)
        assert code == ib.OK
        b = _workspace(run, 12, 9)
        assert np.array_equal(a, b) and np.all(np.isfinite(a))
        # second call, smaller: 3 stations, 4 lags, 2 samples (lags 2 and 3 unpaired: NaN)
        run.set_probes(3, 2.4, 0.6, 1.4, 1.6, 0.4, 4)
        run.step(2)
        code, a2 = _noalloc(run, 3, 4)
        assert code == ib.OK
        b2 = _workspace(run, 3, 4)
        assert np.array_equal(a2, b2, equal_nan=True)
        assert np.all(np.isnan(a2[:, 2 + 2:2 + 4])) and np.all(np.isfinite(a2[:, :4]))
        # beyond the static array: 40 stations x (2 + 2 x 4096) doubles > 262,144
        run.set_probes(40, 0.9, 0.1, 1.5, 1.5, 0.5, 4096)
        run.step(1)
        code, _ = _noalloc(run, 40, 4096)
        assert code == ib.ENOMEM
        assert np.all(np.isfinite(_workspace(run, 40, 4096)[:, :3]))
    finally:
        run.close()


def test_noalloc_without_probes():
    w = _small()
    run = ib.create(ib.domain_from(w), None)
    try:
        code, _ = _noalloc(run, 1, 1)
        assert code == ib.ESTATE
    finally:
        run.close()
