"""Moving-least-squares transfer and adaptive Lagrangian tiling for the flag
(oracle) -- TEST INFRASTRUCTURE ONLY.

Sec. II.B (ii): the moving flag is coupled by a Lagrangian direct forcing
whose transfer is a moving-least-squares (MLS) interpolation (Vanella and
Balaras 2009; de Tullio and Pascazio 2016); each triangle of the flag's mesh
is tiled down to the local Eulerian resolution by quadratic and barycentric
tiling rules, once at the start or every step.  The paper names the methods
only; this oracle takes the following reading.

MLS (per marker X and velocity component, on that component's staggered
lattice):
  * support: the 3 x 3 x 3 nodes x_k around the centre node n = floor(t + 1/2),
    t = (X - o_c) / h, as for the delta stencil (periodic in y and z);
  * weight W_k = w(|x_k - X|_x / R) w(|.|_y / R) w(|.|_z / R), R = 1.5 h, with
    the cubic spline w(q) = 2/3 - 4 q^2 + 4 q^3 (q <= 1/2),
    4/3 - 4 q + 4 q^2 - 4/3 q^3 (1/2 < q <= 1), 0 beyond;
  * linear basis p(x) = (1, (x - X)/h, (y - Y)/h, (z - Z)/h); moment matrix
    A = sum_k W_k p(x_k) p(x_k)^T; shape functions
    phi_k = p(X)^T A^{-1} W_k p(x_k) = W_k (A^{-1} e_0) . p(x_k);
  * interpolation U(X) = sum_k phi_k u_k; force density F = (U^d - U) / dt;
  * spreading, the transpose scaled by the marker volume:
    u_k += dt F dV phi_k / h^3, accumulated in increasing marker order.
    Sum_k phi_k = 1, so the force on the fluid, sum_k f_k h^3 = sum F dV, is
    exactly that of the markers.

Tiling (reading of the quadratic and barycentric rules, done once on the
reference lattice since the sheet is essentially inextensible):
  * the ns x ns lattice (node id a + ns b) has two triangles per cell
    (a, b): (p00, p10, p11) and (p00, p11, p01), split along the spring
    diagonal p00-p11; cells in increasing id order, the lower triangle first;
  * quadratic rule: a triangle (v0, v1, v2) splits into four at its edge
    midpoints m01, m12, m20, children in the order (v0, m01, m20),
    (m01, v1, m12), (m20, m12, v2), (m01, m12, m20); the rule is applied
    L times, L the smallest level at which every child edge at rest,
    longest parent edge / 2^L, is at most h;
  * barycentric rule: one force marker at the barycentre of every tile, at
    the fixed barycentric coordinates beta (sum of the tile's corner
    coordinates, divided by 3) of its parent triangle: X_m = sum_v beta_v X_v,
    U^d_m = sum_v beta_v V_v; volume dV_m = (area of the parent at rest /
    4^L) h;
  * the load on the structure: node v receives -sum_m beta_mv F_m dV_m
    (increasing m), so the force on the sheet is minus that on the fluid.
"""
from __future__ import annotations

import numpy as np

from .delta import ORIGINS, x_range_ok

R_SUPPORT = 1.5   # MLS weight radius in units of h


def spline(q):
    """Cubic-spline MLS weight w(q), elementwise, q >= 0."""
    q = np.abs(np.asarray(q, dtype=np.float64))
    out = np.zeros_like(q)
    a = q <= 0.5
    out[a] = 2.0 / 3.0 - 4.0 * q[a] ** 2 + 4.0 * q[a] ** 3
    b = (q > 0.5) & (q <= 1.0)
    out[b] = 4.0 / 3.0 - 4.0 * q[b] + 4.0 * q[b] ** 2 - (4.0 / 3.0) * q[b] ** 3
    return out


def mls_stencil(X, comp, h, shape):
    """(idx (K, 27, 3), phi (K, 27)): the support nodes (tap order dk, dj, di
    slowest to fastest, j and k wrapped) and the MLS shape functions."""
    X = np.asarray(X, dtype=np.float64)
    nz, ny, _ = shape
    o = np.array(ORIGINS[comp]) * h
    t = (X - o) / h
    n = np.floor(t + 0.5).astype(np.int64)
    K = X.shape[0]
    idx = np.empty((K, 27, 3), dtype=np.int64)
    P = np.empty((K, 27, 4))
    W = np.empty((K, 27))
    q = 0
    for dk in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                node = n + np.array([di, dj, dk])
                xi = node - t                                  # (x_k - X) / h per axis
                W[:, q] = np.prod(spline(np.abs(xi) / R_SUPPORT), axis=1)
                P[:, q, 0] = 1.0
                P[:, q, 1:] = xi
                idx[:, q, 0] = node[:, 0]
                idx[:, q, 1] = np.mod(node[:, 1], ny)
                idx[:, q, 2] = np.mod(node[:, 2], nz)
                q += 1
    A = np.einsum("kq,kqa,kqb->kab", W, P, P)               # sum_q W p p^T
    e0 = np.zeros((K, 4, 1))
    e0[:, 0, 0] = 1.0
    a = np.linalg.solve(A, e0)[..., 0] if K else np.zeros((0, 4))   # A^{-1} e_0
    phi = W * np.einsum("kqa,ka->kq", P, a)
    return idx, phi


def interpolate(field, idx, phi):
    vals = field[idx[..., 2], idx[..., 1], idx[..., 0]]
    return np.sum(vals * phi, axis=1)


def spread(field, idx, phi, amount):
    """field[tap] += amount_m phi_m,tap in increasing marker order (in place)."""
    vals = (amount[:, None] * phi).reshape(-1)
    np.add.at(field, (idx[..., 2].reshape(-1), idx[..., 1].reshape(-1), idx[..., 0].reshape(-1)), vals)


# ---------------- tiling ----------------

def triangles(ns):
    """Vertex ids (T, 3) of the flag's triangles in marker order."""
    out = []
    for b in range(ns - 1):
        for a in range(ns - 1):
            p00, p10 = a + ns * b, a + 1 + ns * b
            p01, p11 = a + ns * (b + 1), a + 1 + ns * (b + 1)
            out.append((p00, p10, p11))
            out.append((p00, p11, p01))
    return np.array(out, dtype=np.int64)


def refine_level(edge_max, h):
    """Smallest L with edge_max / 2^L <= h."""
    L = 0
    while edge_max / (2 ** L) > h:
        L += 1
    return L


def _tiles(corners, L):
    """Corner barycentric coordinates (3 x 3 rows) of the tiles of a triangle
    after L quadratic splits, in the children order of the rule."""
    if L == 0:
        return [corners]
    c0, c1, c2 = corners
    m01, m12, m20 = (c0 + c1) / 2.0, (c1 + c2) / 2.0, (c2 + c0) / 2.0
    out = []
    for ch in ((c0, m01, m20), (m01, c1, m12), (m20, m12, c2), (m01, m12, m20)):
        out.extend(_tiles(ch, L - 1))
    return out


def build_markers(X0, h):
    """Tiling of the reference lattice X0 (ns, ns, 3): returns
    (tri (M, 3) vertex ids, beta (M, 3), dV (M,), level per triangle (T,))."""
    X0 = np.asarray(X0, dtype=np.float64)
    ns = X0.shape[0]
    Xf = X0.reshape(-1, 3)
    tris = triangles(ns)
    eye = np.eye(3)
    tri_out, beta_out, dv_out, levels = [], [], [], []
    for tri in tris:
        P = Xf[tri]
        edges = [np.linalg.norm(P[1] - P[0]), np.linalg.norm(P[2] - P[1]), np.linalg.norm(P[0] - P[2])]
        L = refine_level(max(edges), h)
        area = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
        levels.append(L)
        for c in _tiles((eye[0], eye[1], eye[2]), L):
            beta_out.append((c[0] + c[1] + c[2]) / 3.0)
            tri_out.append(tri)
            dv_out.append(area / 4 ** L * h)
    return (np.array(tri_out, dtype=np.int64), np.array(beta_out), np.array(dv_out),
            np.array(levels, dtype=np.int64))


def marker_state(tri, beta, X, V):
    """Marker positions and target velocities from the node state (N, 3)."""
    Xm = np.einsum("mv,mvc->mc", beta, X[tri])
    Vm = np.einsum("mv,mvc->mc", beta, V[tri])
    return Xm, Vm


def node_load(tri, beta, F, dV, n_nodes):
    """-sum_m beta_mv F_m dV_m per node, accumulated in increasing m."""
    out = np.zeros((n_nodes, 3))
    contrib = beta[:, :, None] * (F * dV[:, None])[:, None, :]      # (M, 3 vertices, 3 comps)
    np.add.at(out, tri.reshape(-1), contrib.reshape(-1, 3))
    return -out


def mls_interp(fields, X, Ud, h, dt, nx):
    """Interpolation and force density of every marker (fields not modified).
    Returns (F (M, 3), maps [(idx, phi)] per component)."""
    M = X.shape[0]
    F = np.zeros((M, 3))
    maps = []
    for c in range(3):
        idx, phi = mls_stencil(X, c, h, fields[c].shape)
        if M and not x_range_ok(idx, c, nx):
            raise ValueError("marker support leaves the evolved x range")
        U = interpolate(fields[c], idx, phi) if M else np.zeros(0)
        F[:, c] = (Ud[:, c] - U) / dt
        maps.append((idx, phi))
    return F, maps


def mls_spread(fields, maps, F, dV, h, dt):
    h3 = h * h * h
    for c in range(3):
        idx, phi = maps[c]
        if idx.shape[0]:
            spread(fields[c], idx, phi, dt * F[:, c] * dV / h3)
