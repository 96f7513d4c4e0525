"""Pins of the regularised-delta transfer (oracle/delta.py).

Checked against facts fixed by the mathematics, not by re-typing the code:
the kernel's moment conditions (Roma, Peskin & Berger 1999: partition of
unity, zero first moment, sum of squares 1/2), brute-force neighbour search
from the staggered layout definition, exact interpolation of linear fields,
and the adjointness of interpolation and spreading.
"""
import numpy as np
import pytest

from oracle import delta

RNG = np.random.default_rng(7)


def test_roma_moments():
    t = RNG.uniform(-50, 50, 100000)
    n = np.floor(t + 0.5)
    taps = [t - (n + d) for d in (-1, 0, 1)]
    w = [delta.roma(r) for r in taps]
    s0 = w[0] + w[1] + w[2]
    s1 = sum(r * ww for r, ww in zip(taps, w))
    s2 = w[0] ** 2 + w[1] ** 2 + w[2] ** 2
    assert np.max(np.abs(s0 - 1.0)) < 1e-15
    assert np.max(np.abs(s1)) < 1e-15
    assert np.max(np.abs(s2 - 0.5)) < 1e-15


def test_roma_support_and_continuity():
    r = np.linspace(-2, 2, 40001)
    w = delta.roma(r)
    assert np.all(w[np.abs(r) >= 1.5] == 0.0)
    assert np.all(w[np.abs(r) < 1.5] > 0.0)
    assert np.max(np.abs(np.diff(w))) < 1e-3          # continuous
    assert np.array_equal(w, delta.roma(-r))            # even


def _node_pos(comp, i, j, k, h):
    """Staggered layout definition: u faces at (i h, (j+1/2) h, (k+1/2) h) etc."""
    x = (i + (0.0 if comp == 0 else 0.5)) * h
    y = (j + (0.0 if comp == 1 else 0.5)) * h
    z = (k + (0.0 if comp == 2 else 0.5)) * h
    return x, y, z


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_index_map_brute_force(comp):
    nx, ny, nz, h = 12, 8, 6, 0.25
    X = np.column_stack([RNG.uniform(3 * h, (nx - 3) * h, 60),
                         RNG.uniform(0, ny * h, 60), RNG.uniform(0, nz * h, 60)])
    idx, wt = delta.stencil(X, comp, h, (nz, ny, nx + 1))
    for kpt in range(X.shape[0]):
        found = {}
        for i in range(-2, nx + 3):
            for j in range(ny):
                for k in range(nz):
                    px, py, pz = _node_pos(comp, i, j, k, h)
                    dx = (X[kpt, 0] - px) / h
                    dy = (X[kpt, 1] - py) / h
                    dy -= ny * np.round(dy / ny)          # periodic distance
                    dz = (X[kpt, 2] - pz) / h
                    dz -= nz * np.round(dz / nz)
                    if abs(dx) < 1.5 and abs(dy) < 1.5 and abs(dz) < 1.5:
                        wv = float(delta.roma(dx) * delta.roma(dy) * delta.roma(dz))
                        if wv > 0:
                            found[(i, j, k)] = wv
        got = {}
        for q in range(27):
            key = tuple(int(v) for v in idx[kpt, q])
            if wt[kpt, q] > 0:
                got[key] = wt[kpt, q]
        assert set(got) == set(found)
        for key in got:
            assert abs(got[key] - found[key]) < 1e-15


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_linear_field_interpolated_exactly(comp):
    nx, ny, nz, h = 16, 12, 10, 0.1
    nxp = nx + 1
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nxp), indexing="ij")
    px, py, pz = _node_pos(comp, i, j, k, h)
    a, b, c, d = 0.3, -1.7, 2.2, 0.9
    field = a + b * px + c * py + d * pz
    X = np.column_stack([RNG.uniform(3 * h, (nx - 3) * h, 200),
                         RNG.uniform(3 * h, (ny - 3) * h, 200),
                         RNG.uniform(3 * h, (nz - 3) * h, 200)])
    idx, wt = delta.stencil(X, comp, h, field.shape)
    U = delta.interpolate(field, idx, wt)
    exact = a + b * X[:, 0] + c * X[:, 1] + d * X[:, 2]
    assert np.max(np.abs(U - exact)) < 1e-13


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_interp_spread_adjoint_and_total(comp):
    nx, ny, nz, h = 14, 10, 8, 0.2
    shape = (nz, ny, nx + 1)
    K = 40
    X = np.column_stack([RNG.uniform(3 * h, (nx - 3) * h, K),
                         RNG.uniform(0, ny * h, K), RNG.uniform(0, nz * h, K)])
    dV = RNG.uniform(0.5, 1.5, K) * h ** 3
    F = RNG.standard_normal(K)
    u = RNG.standard_normal(shape)
    idx, wt = delta.stencil(X, comp, h, shape)
    Iu = delta.interpolate(u, idx, wt)
    S = np.zeros(shape)
    delta.spread(S, idx, wt, F * dV / h ** 3)
    lhs = np.sum(Iu * F * dV)
    rhs = np.sum(u * S) * h ** 3
    assert abs(lhs - rhs) < 1e-14 * max(1.0, abs(lhs)) * 10
    assert abs(np.sum(S) * h ** 3 - np.sum(F * dV)) < 1e-14 * np.sum(np.abs(F * dV)) * 10
