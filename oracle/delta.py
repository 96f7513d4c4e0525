"""Direct-forcing immersed boundary with a regularised delta (oracle).

Sec. II.B: the no-slip condition on immersed solids is imposed by a
direct-forcing immersed-boundary method.  The transfer between Lagrangian
points and the staggered Eulerian mesh uses the 3-point regularised delta of
Roma, Peskin and Berger (1999):

    phi(r) = (1 + sqrt(1 - 3 r^2)) / 3                   |r| <= 1/2
    phi(r) = (5 - 3|r| - sqrt(1 - 3 (1 - |r|)^2)) / 6    1/2 <= |r| <= 3/2
    phi(r) = 0                                           otherwise

Reading: single-pass forcing on the provisional velocity u~ (one
interpolation of all points, then one spreading); forcing density
F_k = (U^d_k - U~_k) / dt; spreading u~ += dt sum_k F_k phi phi phi dV_k / h^3,
accumulated per Eulerian point in increasing marker order k.

Each velocity component c lives on its own staggered lattice with origin
o_u = (0, h/2, h/2), o_v = (h/2, 0, h/2), o_w = (h/2, h/2, 0).  For a point X,
t = (X - o_c)/h, the centre node n = floor(t + 1/2) and the taps n-1, n, n+1 in
each direction (wrapped periodically in y and z).
"""
from __future__ import annotations

import numpy as np

ORIGINS = ((0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0))  # in units of h


def roma(r):
    """Roma-Peskin-Berger 3-point kernel, elementwise."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(a)
    m1 = a <= 0.5
    out[m1] = (1.0 + np.sqrt(1.0 - 3.0 * a[m1] * a[m1])) / 3.0
    m2 = (a > 0.5) & (a <= 1.5)
    b = 1.0 - a[m2]
    out[m2] = (5.0 - 3.0 * a[m2] - np.sqrt(np.maximum(1.0 - 3.0 * b * b, 0.0))) / 6.0
    return out


def stencil(X, comp, h, shape):
    """Index map and weights of the 27-tap stencil of component ``comp``.

    X: (K, 3) point positions.  shape: (nz, ny, nxp) of the component's array,
    with nxp the number of x nodes stored.  Returns (idx, wt):
    idx (K, 27, 3) integer (i, j, k) per tap, j and k already wrapped;
    wt (K, 27) products phi(tx - i) phi(ty - j) phi(tz - k).
    Tap order: dk slowest, then dj, then di (each -1, 0, +1).
    """
    X = np.asarray(X, dtype=np.float64)
    nz, ny, _ = shape
    o = np.array(ORIGINS[comp]) * h
    t = (X - o) / h
    n = np.floor(t + 0.5).astype(np.int64)
    K = X.shape[0]
    idx = np.empty((K, 27, 3), dtype=np.int64)
    wt = np.empty((K, 27))
    q = 0
    for dk in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                ii = n[:, 0] + di
                jj = n[:, 1] + dj
                kk = n[:, 2] + dk
                w = roma(t[:, 0] - ii) * roma(t[:, 1] - jj) * roma(t[:, 2] - kk)
                idx[:, q, 0] = ii
                idx[:, q, 1] = np.mod(jj, ny)
                idx[:, q, 2] = np.mod(kk, nz)
                wt[:, q] = w
                q += 1
    return idx, wt


def x_range_ok(idx, comp, nx):
    """True if every tap stays on nodes the step evolves (no boundary faces).

    u is evolved at x faces 1..nx-1; v and w at cells 0..nx-1.
    """
    lo = 1 if comp == 0 else 0
    hi = nx - 1
    return bool(np.all(idx[..., 0] >= lo) and np.all(idx[..., 0] <= hi))


def interpolate(field, idx, wt):
    """U~_k = sum over taps of field * weight (field indexed [k, j, i])."""
    vals = field[idx[..., 2], idx[..., 1], idx[..., 0]]
    return np.sum(vals * wt, axis=1)


def spread(field, idx, wt, amount):
    """field[tap] += amount_k * weight, accumulated in increasing k (in place).

    ``amount`` is per point, already multiplied by dt dV_k / h^3.
    """
    K = idx.shape[0]
    flat_i = idx[..., 0].reshape(-1)
    flat_j = idx[..., 1].reshape(-1)
    flat_k = idx[..., 2].reshape(-1)
    vals = (amount[:, None] * wt).reshape(-1)
    assert vals.shape[0] == 27 * K
    np.add.at(field, (flat_k, flat_j, flat_i), vals)


def ibm_interp(fields, X, Ud, h, dt, nx):
    """Interpolation and force density of every point (fields not modified).
    Returns (F (K, 3), maps [(idx, wt)] per component)."""
    K = X.shape[0]
    F = np.zeros((K, 3))
    maps = []
    for c in range(3):
        idx, wgt = stencil(X, c, h, fields[c].shape)
        if K and not x_range_ok(idx, c, nx):
            raise ValueError("immersed point support leaves the evolved x range")
        U = interpolate(fields[c], idx, wgt) if K else np.zeros(0)
        F[:, c] = (Ud[:, c] - U) / dt
        maps.append((idx, wgt))
    return F, maps


def ibm_spread(fields, maps, F, dV, h, dt):
    """Spreading of every point's forcing, in increasing point order (in place)."""
    h3 = h * h * h
    for c in range(3):
        idx, wgt = maps[c]
        if idx.shape[0]:
            spread(fields[c], idx, wgt, dt * F[:, c] * dV / h3)


def ibm_force(ut, vt, wt_, X, Ud, dV, h, dt, nx):
    """Single-pass direct forcing on the provisional velocity (in place).

    ut, vt, wt_: provisional velocity components (arrays [k, j, i]); X (K, 3),
    Ud (K, 3) target velocities, dV (K,) point volumes.  All points first
    interpolate the unforced u~, then all spread.  Returns F (K, 3), the force
    density applied to the fluid at each point.
    """
    fields = (ut, vt, wt_)
    F, maps = ibm_interp(fields, X, Ud, h, dt, nx)
    ibm_spread(fields, maps, F, dV, h, dt)
    return F
