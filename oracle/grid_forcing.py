"""Eulerian direct forcing of the passive grid (oracle) -- TEST INFRASTRUCTURE ONLY.

Sec. II.B (i): the fixed grid is imposed with the Eulerian direct-forcing
method of Fadlun et al. (2000): the provisional velocity is forced at the
Eulerian velocity nodes themselves, no Lagrangian markers.  The paper names
the method only; this oracle takes the following reading.

Geometry (Sec. II.A, monoplane grid of square rods of side d and mesh M at
x = x_plane): rods along y at z = Lz/2 + (b + 1/2) M (mod Lz), b < round(Lz/M),
and rods along z at y = Ly/2 + (b + 1/2) M (mod Ly), b < round(Ly/M).  A point
is solid when |x - x_plane| <= d/2 and it lies within d/2 (periodic distance)
of a rod's centre line in the transverse coordinate (closed rods).

Forcing, per velocity component, over its evolved nodes (u faces 1..nx-1,
v and w cells 0..nx-1, every j and k):
  * a solid node takes the body velocity, 0;
  * a fluid node with a solid neighbour among its six grid neighbours is an
    interface node: for each such neighbour the wall lies between them, at the
    distance delta = (periodic) distance of the node from the rod's centre
    plane minus d/2 along that axis; the neighbour with the smallest delta
    (ties in the order -x, +x, -y, +y, -z, +z) fixes the axis, and the node
    takes the linear profile between the wall (0) and the node Q opposite to
    that neighbour: u_P = delta / (delta + h) * u_Q, with u_Q the provisional
    value before any forcing (so the result does not depend on the order);
    if Q is not an evolved node the interface node is set to 0.
The grid forcing is applied before the flag's (Lagrangian) forcing.
"""
from __future__ import annotations

import numpy as np

_ORIGIN = ((0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0))


def rod_centres(L, M):
    out = []
    for b in range(int(round(L / M))):
        c = 0.5 * L + (b + 0.5) * M
        if c >= L:
            c -= L
        out.append(c)
    return out


def _pdist(a, c, L):
    d = np.abs(a - c)
    return np.minimum(d, L - d)


class GridGeometry:
    def __init__(self, x_plane, mesh, bar, ly, lz):
        self.xp, self.M, self.d, self.ly, self.lz = x_plane, mesh, bar, ly, lz
        self.zc = rod_centres(lz, mesh)   # rods along y
        self.yc = rod_centres(ly, mesh)   # rods along z

    def solid(self, x, y, z):
        half = 0.5 * self.d
        inx = np.abs(x - self.xp) <= half
        tr = np.zeros(np.broadcast(x, y, z).shape, dtype=bool)
        for c in self.zc:
            tr |= _pdist(z, c, self.lz) <= half
        for c in self.yc:
            tr |= _pdist(y, c, self.ly) <= half
        return inx & tr

    def wall_distance(self, axis, x, y, z):
        """Distance from a fluid point to the rod surface crossed when moving along
        axis towards a solid neighbour: the smallest (over rods) of the centre-plane
        distance minus d/2 among rods whose centre-plane distance exceeds d/2."""
        half = 0.5 * self.d
        if axis == 0:
            return abs(x - self.xp) - half
        cs, coord, L = (self.yc, y, self.ly) if axis == 1 else (self.zc, z, self.lz)
        best = np.inf
        for c in cs:
            dist = _pdist(coord, c, L)
            if dist > half:
                best = min(best, dist - half)
        return best


def forcing_list(geom, comp, nx, ny, nz, h):
    """[(k, j, i, kq, jq, iq or -1, weight)] for one component, in increasing
    (k, j, i) order; solid nodes have iq = -1 and weight 0."""
    o = _ORIGIN[comp]
    i_lo, i_hi = (1, nx - 1) if comp == 0 else (0, nx - 1)
    ii = np.arange(i_lo, i_hi + 1)
    x_all = (np.arange(nx + 1) + o[0]) * h
    y_all = (np.arange(ny) + o[1]) * h
    z_all = (np.arange(nz) + o[2]) * h
    Z, Y, X = np.meshgrid(z_all, y_all, x_all[i_lo:i_hi + 1], indexing="ij")
    S = geom.solid(X, Y, Z)                         # (nz, ny, n_i) over the evolved range
    out = []
    n_i = ii.size
    for k in range(nz):
        for j in range(ny):
            for a in range(n_i):
                i = ii[a]
                if S[k, j, a]:
                    out.append((k, j, i, 0, 0, -1, 0.0))
                    continue
                best = None
                # neighbours in the order -x, +x, -y, +y, -z, +z
                for axis, step in ((0, -1), (0, 1), (1, -1), (1, 1), (2, -1), (2, 1)):
                    if axis == 0:
                        an = a + step
                        if an < 0 or an >= n_i or not S[k, j, an]:
                            continue
                    elif axis == 1:
                        if not S[k, (j + step) % ny, a]:
                            continue
                    else:
                        if not S[(k + step) % nz, j, a]:
                            continue
                    delta = geom.wall_distance(axis, X[k, j, a], Y[k, j, a], Z[k, j, a])
                    if best is None or delta < best[0]:
                        best = (delta, axis, step)
                if best is None:
                    continue
                delta, axis, step = best
                kq, jq, iq = k, j, i
                if axis == 0:
                    iq = i - step
                    if iq < i_lo or iq > i_hi:
                        out.append((k, j, i, 0, 0, -1, 0.0))
                        continue
                elif axis == 1:
                    jq = (j - step) % ny
                else:
                    kq = (k - step) % nz
                out.append((k, j, i, kq, jq, iq, delta / (delta + h)))
    return out


def apply(ut, vt, wt, lists):
    """Force the provisional arrays (indexed [k, j, i]) in place from the lists
    of the three components; every value read is the unforced one."""
    for arr, lst in zip((ut, vt, wt), lists):
        src = arr.copy()
        for (k, j, i, kq, jq, iq, wgt) in lst:
            arr[k, j, i] = 0.0 if iq < 0 else wgt * src[kq, jq, iq]
