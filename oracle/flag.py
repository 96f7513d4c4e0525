"""Flag structural model: spring network with bending (oracle).

Sec. II.B models the flag as a thin elastic sheet discretised by a
triangulated Lagrangian mesh, masses on the vertices, springs for in-plane
and out-of-plane deformation, with spring coefficients chosen so that the
sheet is essentially inextensible and the bending stiffness B is the only
elastic parameter; the structural solver has its own, smaller time step.
Sec. II.A: square flag of side L, hinged at its leading edge, mass ratio rho,
bending coefficient beta = B/(rho_f U^2 L^3), no gravity.

Reading used here (the paper gives no formulas):
  * Nodes X[b, a] on an ns x ns lattice, a streamwise (a = 0 the leading
    edge), b spanwise, spacing ds = L/(ns-1), node id a + ns b.  Trapezoid
    weights w = 1/2 on the lattice edges, 1 inside; node area
    dA = ds^2 w_a w_b, node mass m = rho dA.
  * Bending energy (Kirchhoff plate, Poisson ratio 0):
        E_b = beta/2 [ sum ds^2 w_a w_b |k_aa|^2 + sum ds^2 w_a w_b |k_bb|^2
                       + 2 sum_cells ds^2 |k_ab|^2 ]
    k_aa = second difference in a at a = 1..ns-2, k_bb likewise in b, k_ab
    the mixed difference on each lattice cell.  Hinged: no k_aa term at
    a = 0 (free rotation).  Clamped (only for the cantilever pins): a k_aa
    term at a = 0 with the ghost X_{-1} = X_1 - 2 ds t0 and weight w_a = 1/2.
  * In-plane springs on every a-edge, every b-edge and one diagonal
    (a, b)-(a+1, b+1) per cell (the triangulation), energy
    k_s/2 (|X_p - X_q| - l_e)^2 with rest lengths l_e from the reference
    lattice.  k_s (dimensionless, per unit width) large: essentially
    inextensible.
  * Leading-edge nodes a = 0 are fixed.
  * Time integration: velocity Verlet sub-steps of the structure inside one
    fluid step, with the hydrodynamic load of that step held fixed;
    n_sub = ceil(dt / dts_max), dts_max = 1.8 / omega_bound, where
    omega_bound^2 bounds the largest eigenvalue of M^-1 (beta K + spring
    Hessian at rest) by Gershgorin row sums of the mass-scaled matrices.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


class FlagModel:
    HINGED = 0
    CLAMPED = 1

    def __init__(self, X0, length, rho, beta, ks, le_bc=0):
        X0 = np.asarray(X0, dtype=np.float64)
        ns = X0.shape[0]
        assert X0.shape == (ns, ns, 3)
        self.ns = ns
        self.ds = length / (ns - 1)
        self.rho, self.beta, self.ks, self.le_bc = rho, beta, ks, le_bc
        ds = self.ds
        w1 = np.ones(ns)
        w1[0] = w1[-1] = 0.5
        self.wa = w1          # indexed by a
        self.wb = w1.copy()   # indexed by b
        dA = ds * ds * np.outer(self.wb, self.wa)      # [b, a]
        self.dA = dA.reshape(-1)                       # node id a + ns b
        self.mass = rho * self.dA
        self.fixed = np.zeros(ns * ns, dtype=bool)
        self.fixed[[0 + ns * b for b in range(ns)]] = True
        self._build_bending(X0)
        self._build_springs(X0)
        self.dts_max = self._stable_substep()

    # ---------------- bending -----------------
    def nid(self, a, b):
        return a + self.ns * b

    def _build_bending(self, X0):
        ns, ds = self.ns, self.ds
        rows, cols, vals, wts, consts = [], [], [], [], []
        r = 0
        inv = 1.0 / (ds * ds)

        def add_row(entries, weight, const=None):
            nonlocal r
            for (node, coef) in entries:
                rows.append(r)
                cols.append(node)
                vals.append(coef * inv)
            wts.append(weight)
            consts.append(np.zeros(3) if const is None else const)
            r += 1

        for b in range(ns):
            for a in range(1, ns - 1):
                add_row([(self.nid(a - 1, b), 1.0), (self.nid(a, b), -2.0),
                         (self.nid(a + 1, b), 1.0)], ds * ds * self.wa[a] * self.wb[b])
            if self.le_bc == self.CLAMPED:
                t0 = X0[b, 1] - X0[b, 0]
                t0 = t0 / np.linalg.norm(t0)
                # ghost X_{-1} = X_1 - 2 ds t0: k_aa(0) = (2 X_1 - 2 X_0 - 2 ds t0)/ds^2
                add_row([(self.nid(1, b), 2.0), (self.nid(0, b), -2.0)],
                        ds * ds * self.wa[0] * self.wb[b], const=-2.0 * t0 / ds)
        for b in range(1, ns - 1):
            for a in range(ns):
                add_row([(self.nid(a, b - 1), 1.0), (self.nid(a, b), -2.0),
                         (self.nid(a, b + 1), 1.0)], ds * ds * self.wa[a] * self.wb[b])
        for b in range(ns - 1):
            for a in range(ns - 1):
                add_row([(self.nid(a + 1, b + 1), 1.0), (self.nid(a + 1, b), -1.0),
                         (self.nid(a, b + 1), -1.0), (self.nid(a, b), 1.0)], 2.0 * ds * ds)
        n = ns * ns
        D = sp.csr_matrix((vals, (rows, cols)), shape=(r, n))
        W = sp.diags(np.array(wts))
        C = np.array(consts)
        self.D, self.W, self.C = D, W, C
        self.K = (D.T @ W @ D).tocsr()                   # E_b = beta/2 |W^1/2 (D X + C)|^2
        self.b_const = -self.beta * (D.T @ (W @ C))

    def bending_force(self, X):
        """f_b = -dE_b/dX for X (n, 3)."""
        return -self.beta * (self.K @ X) + self.b_const

    def bending_energy(self, X):
        R = self.D @ X + self.C
        return 0.5 * self.beta * float(np.sum(self.W.diagonal()[:, None] * R * R))

    # ---------------- springs -----------------
    def _build_springs(self, X0):
        ns = self.ns
        P, Q = [], []
        for b in range(ns):
            for a in range(ns - 1):
                P.append(self.nid(a, b))
                Q.append(self.nid(a + 1, b))
        for b in range(ns - 1):
            for a in range(ns):
                P.append(self.nid(a, b))
                Q.append(self.nid(a, b + 1))
        for b in range(ns - 1):
            for a in range(ns - 1):
                P.append(self.nid(a, b))
                Q.append(self.nid(a + 1, b + 1))
        self.P = np.array(P)
        self.Q = np.array(Q)
        X = X0.reshape(-1, 3)
        d = X[self.P] - X[self.Q]
        self.rest = np.sqrt(d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2])

    def spring_force(self, X):
        d = X[self.P] - X[self.Q]
        ln = np.sqrt(np.sum(d * d, axis=1))
        coef = self.ks * (ln - self.rest) / ln
        f = np.zeros_like(X)
        np.add.at(f, self.P, -coef[:, None] * d)
        np.add.at(f, self.Q, coef[:, None] * d)
        return f

    def spring_energy(self, X):
        d = X[self.P] - X[self.Q]
        ln = np.sqrt(np.sum(d * d, axis=1))
        return 0.5 * self.ks * float(np.sum((ln - self.rest) ** 2))

    def max_strain(self, X):
        d = X[self.P] - X[self.Q]
        ln = np.sqrt(np.sum(d * d, axis=1))
        return float(np.max(np.abs(ln / self.rest - 1.0)))

    # ---------------- time stepping -----------------
    def _stable_substep(self):
        n = self.ns * self.ns
        m = self.mass
        Kabs = abs(self.K).tocoo()
        rb = np.zeros(n)
        np.add.at(rb, Kabs.row, self.beta * Kabs.data / np.sqrt(m[Kabs.row] * m[Kabs.col]))
        rs = np.zeros(n)
        for (p, q) in ((self.P, self.Q), (self.Q, self.P)):
            np.add.at(rs, p, self.ks * (1.0 / m[p] + 1.0 / np.sqrt(m[p] * m[q])))
        free = ~self.fixed
        om2 = float(np.max((rb + rs)[free]))
        return 1.8 / math.sqrt(om2)

    def forces(self, X, f_ext):
        return self.bending_force(X) + self.spring_force(X) + f_ext

    def advance(self, X, V, f_ext, dt):
        """Advance (X, V) (each (n, 3)) by one fluid step dt under the fixed load
        f_ext (n, 3).  Returns new (X, V) and the number of sub-steps."""
        nsub = int(math.ceil(dt / self.dts_max))
        dts = dt / nsub
        X = X.copy()
        V = V.copy()
        free = ~self.fixed
        inv_m = (1.0 / self.mass)[:, None]
        f = self.forces(X, f_ext)
        for _ in range(nsub):
            V[free] += (0.5 * dts) * (f[free] * inv_m[free])
            X[free] += dts * V[free]
            f = self.forces(X, f_ext)
            V[free] += (0.5 * dts) * (f[free] * inv_m[free])
        return X, V, nsub

