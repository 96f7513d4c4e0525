"""Pins of the Eulerian grid forcing (oracle/grid_forcing.py, Sec. II.B (i)).

* Solid-node counts equal the closed-form count of mesh positions inside each
  rod (integer arithmetic on the rod edges), per staggered component.
* Interface nodes next to a rod face carry the closed-form linear-profile
  weight delta/(delta + h) and the node opposite the face.
* A field that already vanishes linearly at the wall is left unchanged at the
  interface nodes (the linear profile reproduces itself).
* Forcing reads only unforced values (order independence), and the solver
  forces the grid before the flag.
"""
import math
from types import SimpleNamespace

import numpy as np

from oracle import grid_forcing as gf
from oracle.solver import Solver


def _count_in(lo, hi, off, h, n=None):
    """Integers m (0 <= m < n if n) with lo <= (m + off) h <= hi."""
    a = math.ceil(lo / h - off - 1e-12)
    b = math.floor(hi / h - off + 1e-12)
    if n is not None:
        a, b = max(a, 0), min(b, n - 1)
    return max(0, b - a + 1)


def test_solid_counts_closed_form():
    # two rods in each transverse direction (M = L/2: centres at L/4 and 3L/4,
    # away from the periodic seam)
    h, nx, ny, nz = 0.1, 40, 24, 24
    ly = lz = ny * h
    d, xp = 0.75, 1.23
    geom = gf.GridGeometry(xp, ly / 2, d, ly, lz)
    assert np.allclose(sorted(geom.yc), [ly / 4, 3 * ly / 4])
    for comp in range(3):
        o = gf._ORIGIN[comp]
        lst = gf.forcing_list(geom, comp, nx, ny, nz, h)
        solid = sum(1 for e in lst if e[5] < 0)
        cx = _count_in(xp - d / 2, xp + d / 2, o[0], h)
        cy = sum(_count_in(c - d / 2, c + d / 2, o[1], h, ny) for c in geom.yc)
        cz = sum(_count_in(c - d / 2, c + d / 2, o[2], h, nz) for c in geom.zc)
        # y-rods: every y, the z bands; z-rods: every z, the y bands; overlaps once
        want = cx * (ny * cz + nz * cy - cy * cz)
        assert solid == want, (comp, solid, want)


def test_interface_weights_at_a_face():
    h, nx, ny, nz = 1.0, 24, 8, 8
    xp, d = 10.3, 2.0            # faces at x = 9.3 and 11.3
    geom = gf.GridGeometry(xp, 8.0, d, 8.0, 8.0)   # one rod each way: zc = yc = 0.5*8 + 4 - 8 = 0
    lst = {(e[0], e[1], e[2]): e for e in gf.forcing_list(geom, 0, nx, ny, nz, h)}
    # u node at (i, j, k) = (9, 3, 0): z = 0.5 lies inside the y-rod's z band |z - 0| <= 1
    k, j = 0, 3
    e9 = lst[(k, j, 9)]
    assert e9[5] == 8 and abs(e9[6] - 0.3 / 1.3) < 1e-15          # upstream face
    e12 = lst[(k, j, 12)]
    assert e12[5] == 13 and abs(e12[6] - 0.7 / 1.7) < 1e-15        # downstream face
    assert lst[(k, j, 10)][5] == -1 and lst[(k, j, 11)][5] == -1    # solid


def test_linear_wall_profile_is_reproduced():
    h, nx, ny, nz = 1.0, 24, 8, 8
    xp, d = 10.3, 2.0
    geom = gf.GridGeometry(xp, 8.0, d, 8.0, 8.0)
    lists = [gf.forcing_list(geom, c, nx, ny, nz, h) for c in range(3)]
    x_u = np.arange(nx + 1) * h
    wall = xp - d / 2
    ut = np.broadcast_to(2.5 * (x_u - wall), (nz, ny, nx + 1)).copy()  # zero at the upstream face
    vt = np.zeros((nz, ny, nx + 1))
    wt = np.zeros((nz, ny, nx + 1))
    before = ut.copy()
    gf.apply(ut, vt, wt, lists)
    for (k, j, i, kq, jq, iq, w) in lists[0]:
        if iq >= 0 and i < xp and iq == i - 1:
            assert abs(ut[k, j, i] - before[k, j, i]) < 1e-12
        if iq < 0:
            assert ut[k, j, i] == 0.0


def test_forcing_reads_unforced_values():
    h, nx, ny, nz = 0.25, 32, 16, 16
    geom = gf.GridGeometry(2.0, 2.0, 0.6, 4.0, 4.0)
    lists = [gf.forcing_list(geom, c, nx, ny, nz, h) for c in range(3)]
    rng = np.random.default_rng(3)
    a = [rng.standard_normal((nz, ny, nx + 1)) for _ in range(3)]
    b = [x.copy() for x in a]
    gf.apply(*b, lists)
    for c in range(3):
        src = a[c]
        for (k, j, i, kq, jq, iq, w) in reversed(lists[c]):   # any order gives the same
            want = 0.0 if iq < 0 else w * src[kq, jq, iq]
            assert b[c][k, j, i] == want


def test_solver_forces_grid_nodes():
    h, nx, ny, nz = 0.125, 48, 24, 24
    P = SimpleNamespace(nx=nx, ny=ny, nz=nz, lx=nx * h, ly=ny * h, lz=nz * h, re=300.0, u_in=1.0,
                        dt=0.0, cfl=0.4, noise_amp=0.0)
    S = Solver(P, grid_forcing=dict(x_plane=0.75, mesh=1.5, bar=0.3))
    ut, vt, wt, _ = S.stage_predict()
    S.stage_ibm(ut, vt, wt)
    for arr, lst in zip((ut, vt, wt), S.grid_lists):
        solid = [(k, j, i) for (k, j, i, kq, jq, iq, w) in lst if iq < 0]
        assert len(solid) > 0
        assert all(arr[k, j, i] == 0.0 for (k, j, i) in solid)


def test_y_face_source_and_tie_order():
    """h = 1, rods of side 2 at x = 10.3, one rod each way at y = 0 and z = 0.
    u node (i, j, k) = (10, 1, 3): its only solid neighbour is -y (the wall at
    y = 1), so it copies the node opposite, j = 2, with weight 0.5/1.5.  Node
    (10, 1, 1) has solid neighbours at -y and -z at the same distance 0.5: the
    tie goes to -y (the stated order), source (j, k) = (2, 1)."""
    geom = gf.GridGeometry(10.3, 8.0, 2.0, 8.0, 8.0)
    lst = {(e[0], e[1], e[2]): e for e in gf.forcing_list(geom, 0, 24, 8, 8, 1.0)}
    e = lst[(3, 1, 10)]
    assert (e[3], e[4], e[5]) == (3, 2, 10) and abs(e[6] - 0.5 / 1.5) < 1e-15
    e = lst[(1, 1, 10)]
    assert (e[3], e[4], e[5]) == (1, 2, 10) and abs(e[6] - 0.5 / 1.5) < 1e-15


def test_rods_are_closed():
    """A node exactly on a rod face is solid (closed rods): faces at x = 9 and 11."""
    geom = gf.GridGeometry(10.0, 8.0, 2.0, 8.0, 8.0)
    lst = {(e[0], e[1], e[2]): e for e in gf.forcing_list(geom, 0, 24, 8, 8, 1.0)}
    assert lst[(0, 3, 9)][5] == -1 and lst[(0, 3, 11)][5] == -1
    assert lst[(0, 3, 8)][5] == 7          # the fluid node next to the face copies its opposite


def test_grid_solidity_matches_the_paper():
    """tests/golden/grid_solidity.json: at M/d = 4 the paper's grid blocks 44%
    of the cross-section.  The oracle's solid mask, sampled at cell midpoints
    of a fine lattice over the grid plane (400 samples per mesh M), covers
    exactly 1 - (1 - d/M)^2 = 0.4375 of it."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "grid_solidity.json")))
    M = 1.0
    d = M / g["M_over_d"]
    L = 4 * M
    geom = gf.GridGeometry(2.0, M, d, L, L)
    n = 1600
    s = (np.arange(n) + 0.5) * (L / n)
    Y, Z = np.meshgrid(s, s, indexing="ij")
    frac = np.mean(geom.solid(np.full_like(Y, 2.0), Y, Z))
    assert frac == 1.0 - (1.0 - d / M) ** 2
    assert abs(100.0 * frac - g["solidity_percent_printed"]) < 0.5
