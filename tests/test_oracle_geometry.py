"""Pins of the bodies built from the problem statement (oracle/geometry.py, Sec. II.A).

Grid points:
* the point count equals its closed form: per rod running along y, ny
  cross-sections of nc x nc points; per rod running along z, nz minus the
  cross-sections whose axis position lies inside a y-rod, counted from the
  rod edges by integer arithmetic (768 x 384 x 384 box: 300,672 points);
* the summed volume equals d^2 h times the number of cross-sections, the
  volume of the discretised rods;
* no two points coincide or come closer than the lattice spacing (rod
  crossings are counted once);
* every point lies inside a rod, and every rod's points are centred on its
  axis;
* at the paper's M/d = 4, on a mesh where the rod faces fall on cell faces,
  the frontal area of the points blocks exactly 7/16 of the section, the
  solidity the paper prints as 44%.
Flag lattice: hinge line, trailing edge, spacing, pitch angle and centroid.
Time step from the CFL number: a uniform stream and single perturbed faces
against hand-computed maxima of the cell speed.
"""
import json
import math
import os
from types import SimpleNamespace

import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import fluid, geometry
from oracle.solver import Solver

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _box(nx, ny, nz, h):
    return dict(nx=nx, ny=ny, nz=nz, lx=nx * h, ly=ny * h, lz=nz * h)


def _inside_count(axis_pos, d, h, n):
    """Cells m (0 <= m < n, periodic) whose centre (m + 1/2) h is strictly
    within d/2 of axis_pos: integer bounds of the open interval."""
    lo = (axis_pos - 0.5 * d) / h - 0.5
    hi = (axis_pos + 0.5 * d) / h - 0.5
    a = math.floor(lo) + 1
    b = math.ceil(hi) - 1
    return max(0, min(b - a + 1, n))


def _closed_form(grid, box):
    h = box["lx"] / box["nx"]
    nc = max(1, math.floor(grid.bar / h + 0.5))
    n_yrods = round(box["lz"] / grid.mesh)
    n_zrods = round(box["ly"] / grid.mesh)
    axes = [0.5 * box["lz"] + (b + 0.5) * grid.mesh for b in range(n_yrods)]
    covered = sum(_inside_count(a, grid.bar, h, box["nz"]) for a in axes)
    sections = n_yrods * box["ny"] + n_zrods * (box["nz"] - covered)
    return nc, sections


WORKLOADS = [
    # (grid, box): the 768 x 384 x 384 workload (d = 6.4 h, nc = 6), the
    # ensemble meshes (nc = 1, 1, 2, 3) and an odd placement
    (SimpleNamespace(x_plane=0.25, mesh=0.5, bar=0.1), _box(768, 384, 384, 1 / 64)),
    (SimpleNamespace(x_plane=0.25, mesh=0.5, bar=0.1), _box(96, 48, 48, 1 / 8)),
    (SimpleNamespace(x_plane=0.25, mesh=0.5, bar=0.1), _box(128, 64, 64, 3 / 32)),
    (SimpleNamespace(x_plane=0.25, mesh=0.5, bar=0.1), _box(192, 96, 96, 1 / 16)),
    (SimpleNamespace(x_plane=0.25, mesh=0.5, bar=0.1), _box(384, 192, 192, 1 / 32)),
    (SimpleNamespace(x_plane=0.61, mesh=0.7, bar=0.23), _box(64, 40, 40, 0.07)),
]


@pytest.mark.parametrize("grid,box", WORKLOADS)
def test_grid_point_count_and_volume(grid, box):
    X, dV = geometry.grid_points(grid, **box)
    h = box["lx"] / box["nx"]
    nc, sections = _closed_form(grid, box)
    assert X.shape == (sections * nc * nc, 3)
    # the volume of the discretised rods: d^2 per cross-section of length h
    assert abs(dV.sum() - grid.bar ** 2 * h * sections) <= 1e-12 * dV.sum()
    assert np.all(dV > 0)


def test_grid_point_count_of_the_paper_scale_box():
    grid, box = WORKLOADS[0]
    X, _ = geometry.grid_points(grid, **box)
    # 12 rods each way; a rod along z loses the 6 cross-sections that lie in
    # each of the 12 rods along y
    assert X.shape[0] == 12 * 384 * 36 + 12 * (384 - 72) * 36 == 300672


@pytest.mark.parametrize("grid,box", WORKLOADS[::2])
def test_grid_points_distinct_and_inside(grid, box):
    X, _ = geometry.grid_points(grid, **box)
    h = box["lx"] / box["nx"]
    nc = max(1, math.floor(grid.bar / h + 0.5))
    spacing = min(grid.bar / nc, h)
    # periodic in y and z: no pair closer than the lattice spacing
    tree = cKDTree(X, boxsize=[1e9, box["ly"], box["lz"]])
    assert len(tree.query_pairs(0.5 * spacing)) == 0
    assert np.all(X[:, 1] >= 0) and np.all(X[:, 1] < box["ly"])
    assert np.all(X[:, 2] >= 0) and np.all(X[:, 2] < box["lz"])
    assert np.all(np.abs(X[:, 0] - grid.x_plane) < 0.5 * grid.bar)

    def pdist(a, c, L):
        d = np.abs(a - c)
        return np.minimum(d, L - d)
    n_rods = round(box["lz"] / grid.mesh)
    zaxes = [(0.5 * box["lz"] + (b + 0.5) * grid.mesh) % box["lz"] for b in range(n_rods)]
    yaxes = [(0.5 * box["ly"] + (b + 0.5) * grid.mesh) % box["ly"] for b in range(n_rods)]
    in_y = np.min([pdist(X[:, 2], c, box["lz"]) for c in zaxes], axis=0) < 0.5 * grid.bar
    in_z = np.min([pdist(X[:, 1], c, box["ly"]) for c in yaxes], axis=0) < 0.5 * grid.bar
    assert np.all(in_y | in_z)


def test_grid_points_centred_on_the_rod_axes():
    grid, box = WORKLOADS[3]
    X, _ = geometry.grid_points(grid, **box)
    h = box["lx"] / box["nx"]
    nc = max(1, math.floor(grid.bar / h + 0.5))
    per_rod = box["ny"] * nc * nc
    first = X[:per_rod]               # the first rod along y, axis z = Lz/2 + M/2
    assert abs(first[:, 0].mean() - grid.x_plane) < 1e-12
    assert abs(first[:, 2].mean() - (0.5 * box["lz"] + 0.5 * grid.mesh)) < 1e-12
    assert abs(first[:, 1].mean() - 0.5 * box["ly"]) < 1e-12


def test_grid_solidity_printed_by_the_paper():
    with open(os.path.join(GOLDEN, "grid_solidity.json")) as fh:
        g = json.load(fh)
    ratio = g["M_over_d"]
    h = 1.0
    d = 4 * h
    mesh = ratio * d                       # 16 h: rod faces on cell faces
    box = _box(40, 32, 32, h)
    grid = SimpleNamespace(x_plane=12.0, mesh=mesh, bar=d)
    X, dV = geometry.grid_points(grid, **box)
    # every point stands for a box of depth d/nc in x: the frontal area is
    # sum(dV) / d
    solidity = dV.sum() / d / (box["ly"] * box["lz"])
    assert solidity == 1.0 - (1.0 - 1.0 / ratio) ** 2 == 7.0 / 16.0
    assert round(100 * solidity) == g["solidity_percent_printed"]


def test_flag_lattice():
    f = SimpleNamespace(ns=11, length=1.3, x_le=2.1, y_c=1.7, z_c=2.2, pitch=0.1 * math.pi)
    X = geometry.flag_lattice(f)
    ds = f.length / (f.ns - 1)
    # the hinge line (a = 0): x_le, y_c, spanning z_c -+ L/2
    assert np.all(X[:, 0, 0] == f.x_le) and np.all(X[:, 0, 1] == f.y_c)
    assert abs(X[0, 0, 2] - (f.z_c - f.length / 2)) < 1e-15
    assert abs(X[-1, 0, 2] - (f.z_c + f.length / 2)) < 1e-14
    # trailing edge at L (cos theta, sin theta) from the hinge
    assert np.allclose(X[:, -1, 0], f.x_le + f.length * math.cos(f.pitch), atol=1e-14)
    assert np.allclose(X[:, -1, 1], f.y_c + f.length * math.sin(f.pitch), atol=1e-14)
    # spacing ds along a and b, ds sqrt(2) on the cell diagonals
    da = np.linalg.norm(X[:, 1:] - X[:, :-1], axis=2)
    db = np.linalg.norm(X[1:] - X[:-1], axis=2)
    dd = np.linalg.norm(X[1:, 1:] - X[:-1, :-1], axis=2)
    assert np.allclose(da, ds, atol=1e-14) and np.allclose(db, ds, atol=1e-14)
    assert np.allclose(dd, ds * math.sqrt(2), atol=1e-14)
    # pitched by theta about z; centred transversely
    e = X[3, 5] - X[3, 4]
    assert abs(math.atan2(e[1], e[0]) - f.pitch) < 1e-13 and e[2] == 0.0
    c = X.reshape(-1, 3).mean(axis=0)
    want = (f.x_le + 0.5 * f.length * math.cos(f.pitch), f.y_c + 0.5 * f.length * math.sin(f.pitch), f.z_c)
    assert np.allclose(c, want, atol=1e-14)


# ---- time step from the CFL number ----

def _uniform(nx, ny, nz, U):
    return fluid.Fields(u=np.full((nz, ny, nx + 1), U), v=np.zeros((nz, ny, nx + 1)),
                        w=np.zeros((nz, ny, nx + 1)), p=np.zeros((nz, ny, nx)))


def test_cfl_uniform_stream():
    h, cfl, U = 0.05, 0.5, 1.25
    f = _uniform(12, 8, 6, U)
    assert fluid.cfl_dt(f, h, cfl) == cfl * h / U
    # and the solver's first step on a uniform stream
    P = SimpleNamespace(nx=12, ny=8, nz=6, lx=12 * h, ly=8 * h, lz=6 * h, re=100.0, u_in=U,
                        dt=0.0, cfl=cfl, noise_amp=0.0)
    S = Solver(P)
    assert abs(S.dt - cfl * h / U) <= 1e-15 * S.dt


def test_cfl_single_perturbed_faces():
    h, cfl = 0.1, 0.4
    nx, ny, nz = 10, 6, 8
    f = _uniform(nx, ny, nz, 1.0)
    # a v face shared by cells j = 2 and 3 of column (k, i) = (5, 4): their mean
    # |v| is 0.3 / 2, so the cell speed is 1 + 0.15
    f.v[5, 3, 4] = 0.3
    assert abs(fluid.cfl_dt(f, h, cfl) - cfl * h / 1.15) < 1e-15
    # a w face of -0.8 at (k, j, i) = (2, 1, 7): cells k = 1, 2 reach 1 + 0.4
    f.w[2, 1, 7] = -0.8
    assert abs(fluid.cfl_dt(f, h, cfl) - cfl * h / 1.4) < 1e-15
    # a u face of 1.9 at (0, 0, 6): cells i = 5 and 6 of that row reach (1 + 1.9) / 2
    f.u[0, 0, 6] = 1.9
    assert abs(fluid.cfl_dt(f, h, cfl) - cfl * h / 1.45) < 1e-15
    # u and v adding up in one cell: a u face of 2.1 at (5, 3, 5) gives cells
    # i = 4, 5 of row (5, 3) a u mean of 1.55, and cell i = 4 holds the v mean 0.15
    f.u[5, 3, 5] = 2.1
    assert abs(fluid.cfl_dt(f, h, cfl) - cfl * h / 1.7) < 1e-15
