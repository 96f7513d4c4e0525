"""Immersed bodies built from the paper's problem statement (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. II.A places a monoplane passive grid of square rods (side d, mesh M) in
a plane normal to the stream, and downstream of it a square flag of side L,
hinged at its leading edge, centred transversely and pitched by theta = 0.1 pi.
The paper forces the grid at the Eulerian nodes; the delta-point form of the
direct forcing needs the rods as Lagrangian points, and this module states
that reading as plain loops.

Grid points (reading; the paper gives the rods, not a point set):
  * nc = max(1, floor(d/h + 1/2)) points per rod side, at transverse and
    streamwise offsets (q + 1/2) d/nc - d/2, q = 0..nc-1, about the rod axis
    and the plane x = x_plane;
  * one cross-section every h along the rod, at (m + 1/2) h;
  * rods running along y sit at z = Lz/2 + (b + 1/2) M (mod Lz),
    b = 0..round(Lz/M)-1; rods running along z at y = Ly/2 + (b + 1/2) M
    (mod Ly): the box centre faces an opening (the paper centres the
    coordinates on the grid, Sec. II.A);
  * a cross-section of a z-rod whose position z lies strictly within d/2 of a
    y-rod's axis (periodic distance) is left out: that volume is already a
    y-rod's;
  * every point carries the volume (d/nc)^2 h and target velocity 0.
  Order: the y-rods in increasing b, then the z-rods; within a rod the
  position along it, then the streamwise offset, then the transverse offset.

Flag lattice (Sec. II.A): an ns x ns node lattice of spacing ds = L/(ns - 1);
node (a, b), a streamwise from the leading edge, b spanwise, at
  (x_le, y_c, z_c - L/2) + a ds (cos theta, sin theta, 0) + b ds (0, 0, 1).
"""
from __future__ import annotations

import math

import numpy as np


def points_per_side(bar: float, h: float) -> int:
    """nc = max(1, floor(d/h + 1/2))."""
    return max(1, int(math.floor(bar / h + 0.5)))


def rod_axes(length: float, mesh: float) -> list:
    """Axis positions Lc/2 + (b + 1/2) M, wrapped into [0, Lc), b < round(Lc/M)."""
    out = []
    nrods = int(math.floor(length / mesh + 0.5))
    for b in range(nrods):
        c = 0.5 * length + (b + 0.5) * mesh
        if c >= length:
            c = c - length
        out.append(c)
    return out


def _wrap(a: float, length: float) -> float:
    if a < 0.0:
        return a + length
    if a >= length:
        return a - length
    return a


def grid_points(grid, nx: int, ny: int, nz: int, lx: float, ly: float, lz: float):
    """Solid points of the passive grid (the reading above).

    grid: object with x_plane, mesh, bar.  Returns X (K, 3) and dV (K,)."""
    h = lx / nx
    d = grid.bar
    nc = points_per_side(d, h)
    offs = [(q + 0.5) * (d / nc) - 0.5 * d for q in range(nc)]
    z_axes = rod_axes(lz, grid.mesh)     # rods running along y, placed in z
    y_axes = rod_axes(ly, grid.mesh)     # rods running along z, placed in y
    X = []
    for zc in z_axes:
        for m in range(ny):
            y = (m + 0.5) * h
            for ox in offs:
                for ot in offs:
                    X.append((grid.x_plane + ox, y, _wrap(zc + ot, lz)))
    for yc in y_axes:
        for m in range(nz):
            z = (m + 0.5) * h
            covered = False
            for zc in z_axes:
                dz = abs(z - zc)
                if min(dz, lz - dz) < 0.5 * d:
                    covered = True
            if covered:
                continue
            for ox in offs:
                for ot in offs:
                    X.append((grid.x_plane + ox, _wrap(yc + ot, ly), z))
    X = np.array(X, dtype=np.float64).reshape(-1, 3)
    dV = np.full(X.shape[0], (d / nc) * (d / nc) * h)
    return X, dV


def grid_points_of(w):
    """grid_points for a workload object (nx, ny, nz, lx, ly, lz, grid)."""
    if w.grid is None:
        return np.zeros((0, 3)), np.zeros(0)
    return grid_points(w.grid, w.nx, w.ny, w.nz, w.lx, w.ly, w.lz)


def flag_lattice(flag):
    """Reference lattice of the flag, shape (ns, ns, 3) indexed [b, a, component].

    flag: object with ns, length, x_le, y_c, z_c, pitch."""
    ns = flag.ns
    ds = flag.length / (ns - 1)
    ct = math.cos(flag.pitch)
    st = math.sin(flag.pitch)
    z0 = flag.z_c - 0.5 * flag.length
    X = np.empty((ns, ns, 3))
    for b in range(ns):
        for a in range(ns):
            X[b, a, 0] = flag.x_le + (a * ds) * ct
            X[b, a, 1] = flag.y_c + (a * ds) * st
            X[b, a, 2] = z0 + b * ds
    return X
