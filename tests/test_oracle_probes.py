"""Pins of the virtual-probe statistics (oracle/probes.py, Sec. III).

* Trilinear sampling reproduces multilinear fields a + b x + c y + d z + e x y z
  exactly on each staggered component (checks the staggered origins, the
  index arithmetic and the weights).
* Across the periodic seam the weights land on the wrapped nodes (one-hot
  field, closed-form weight).
* Running sums and lagged products equal the same sums taken over the whole
  stored series at once.
* A sampled cosine gives the variance A^2/2 and the autocorrelation
  cos(omega l) in the derived station statistics.
"""
import numpy as np
import pytest

from oracle import probes
from oracle.solver import Solver

RNG = np.random.default_rng(11)


def _node_coords(comp, nz, ny, nxl, h):
    o = probes._ORIGIN[comp]
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nxl), indexing="ij")
    return (i + o[0]) * h, (j + o[1]) * h, (k + o[2]) * h


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_multilinear_fields_are_reproduced(comp):
    nx, ny, nz, h = 10, 12, 14, 0.3
    nxl = nx + 1 if comp == 0 else nx
    x, y, z = _node_coords(comp, nz, ny, nxl, h)
    a, b, c, d, e = 0.7, -1.3, 0.4, 2.1, 0.25
    field = a + b * x + c * y + d * z + e * x * y * z
    # interior points (no periodic seam crossed)
    X = np.column_stack([RNG.uniform(1.0 * h, (nx - 1.5) * h, 40),
                         RNG.uniform(1.0 * h, (ny - 1.5) * h, 40),
                         RNG.uniform(1.0 * h, (nz - 1.5) * h, 40)])
    got = probes.sample(field, comp, X, h, nxl - 1)
    want = a + b * X[:, 0] + c * X[:, 1] + d * X[:, 2] + e * X[:, 0] * X[:, 1] * X[:, 2]
    assert np.max(np.abs(got - want)) < 1e-12


def test_periodic_seam_weights():
    nx, ny, nz, h = 6, 8, 8, 1.0
    field = np.zeros((nz, ny, nx))
    field[3, ny - 1, 2] = 1.0                      # v node (i=2, j=ny-1, k=3): ((2.5), ny-1, 3.5)
    fy = 0.3                                      # probe between j = ny-1 and the wrapped j = 0
    X = np.array([[2.5 * h, (ny - 1 + fy) * h, 3.5 * h]])
    got = probes.sample(field, 1, X, h, nx - 1)[0]
    assert abs(got - (1.0 - fy)) < 1e-15
    field[3, ny - 1, 2] = 0.0
    field[3, 0, 2] = 1.0
    got = probes.sample(field, 1, X, h, nx - 1)[0]
    assert abs(got - fy) < 1e-15


def test_x_range_is_checked():
    field = np.zeros((4, 4, 6))
    with pytest.raises(ValueError):
        probes.sample(field, 1, np.array([[0.2, 1.0, 1.0]]), 1.0, 5)   # v: x - h/2 < 0


def test_running_sums_equal_whole_series_sums():
    K, T, L = 5, 37, 9
    us, vs, ws = (RNG.standard_normal((T, K)) for _ in range(3))
    st = probes.ProbeStats(np.zeros((K, 3)), L)
    for t in range(T):
        st.add(us[t], vs[t], ws[t])
    r = st.rec
    assert np.all(r[:, 0] == T)
    for col, arr in zip(range(1, 4), (us, vs, ws)):
        assert np.allclose(r[:, col], arr.sum(0), rtol=0, atol=1e-12)
    prods = (us * us, vs * vs, ws * ws, us * vs, us * ws, vs * ws)
    for col, arr in zip(range(4, 10), prods):
        assert np.allclose(r[:, col], arr.sum(0), rtol=0, atol=1e-12)
    for lag in range(L):
        assert np.allclose(r[:, 10 + lag], (us[lag:] * us[:T - lag]).sum(0), rtol=0, atol=1e-12)
        assert np.allclose(r[:, 10 + L + lag], (vs[lag:] * vs[:T - lag]).sum(0), rtol=0, atol=1e-12)


def test_cosine_series_statistics():
    K, T, L = 9, 20000, 12
    om, A, m = 0.21, 0.8, 1.5
    st = probes.ProbeStats(np.zeros((K, 3)), L)
    for t in range(T):
        u = np.full(K, m + A * np.cos(om * t))
        v = np.full(K, A * np.sin(om * t))
        st.add(u, v, np.zeros(K))
    s = probes.station_statistics(st.rec, L)[0]
    assert abs(s["k"] - 0.5 * (A * A / 2 + A * A / 2)) < 2e-3
    assert abs(s["anisotropy"] - 1.0) < 5e-3
    lags = np.arange(L)
    assert np.max(np.abs(s["f"] - np.cos(om * lags))) < 5e-3
    assert np.max(np.abs(s["g"] - np.cos(om * lags))) < 5e-3


def test_positions_and_order():
    P = probes.probe_positions(2, 1.0, 0.5, 3.0, 4.0, 2.0 / 3.0)
    assert P.shape == (18, 3)
    assert np.allclose(P[4], (1.0, 3.0, 4.0))                       # p=0, a=0, b=0
    assert np.allclose(P[9 + 0], (1.5, 3.0 - 2 / 3, 4.0 - 2 / 3))   # p=1, a=-1, b=-1
    assert np.allclose(P[9 + 8], (1.5, 3.0 + 2 / 3, 4.0 + 2 / 3))


def test_solver_samples_after_each_projection():
    """A uniform stream stays uniform: every probe reads (U, 0, 0) each step."""
    from types import SimpleNamespace
    nx, ny, nz, h = 16, 8, 8, 0.25
    P = SimpleNamespace(nx=nx, ny=ny, nz=nz, lx=nx * h, ly=ny * h, lz=nz * h, re=100.0,
                        u_in=1.0, dt=0.01, cfl=0.5, noise_amp=0.0)
    pr = dict(n_x=3, x0=1.0, dx=0.5, yc=1.0, zc=1.0, dyz=0.4, n_lags=4)
    S = Solver(P, probes=pr)
    S.step(5)
    r = S.probes.rec
    assert np.all(r[:, 0] == 5)
    assert np.max(np.abs(r[:, 1] - 5.0)) < 1e-12
    assert np.max(np.abs(r[:, 2:4])) < 1e-12
    assert np.max(np.abs(r[:, 10:14] - np.array([5.0, 4.0, 3.0, 2.0]))) < 1e-12


def test_probe_index_layout():
    """Probe (p, a, b) at (x0 + p dx, yc + a dyz, zc + b dyz) has index
    q = (b+1) + 3 ((a+1) + 3 p): spot values of that stated layout."""
    from oracle.probes import probe_positions
    pos = probe_positions(2, 1.0, 0.5, 3.0, 4.0, 0.25)
    assert np.allclose(pos[0], (1.0, 2.75, 3.75))     # p 0, a -1, b -1
    assert np.allclose(pos[1], (1.0, 2.75, 4.0))      # p 0, a -1, b 0
    assert np.allclose(pos[3], (1.0, 3.0, 3.75))      # p 0, a 0, b -1
    assert np.allclose(pos[17], (1.5, 3.25, 4.25))    # p 1, a 1, b 1


def test_lagged_means_count_only_pairs():
    """Series 1, 2, 3, 4 at every probe of a station: the lag-1 mean product is
    (2*1 + 3*2 + 4*3)/3 = 20/3 (three pairs), mean 2.5, variance 1.25, so
    f(1) = (20/3 - 6.25)/1.25 = 1/3 and f(0) = 1."""
    from oracle.probes import ProbeStats, station_statistics
    S = ProbeStats(np.zeros((9, 3)), 3)
    for x in (1.0, 2.0, 3.0, 4.0):
        S.add(np.full(9, x), np.full(9, x), np.full(9, 0.5 * x))
    st = station_statistics(S.rec, 3)[0]
    assert abs(st["f"][0] - 1.0) < 1e-14 and abs(st["f"][1] - 1.0 / 3.0) < 1e-14
    assert abs(st["f"][2] - ((3 * 1 + 4 * 2) / 2 - 6.25) / 1.25) < 1e-14
