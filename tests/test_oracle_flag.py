"""Pins of the flag structural model (oracle/flag.py).

* Affine placements carry no bending energy (all second differences vanish).
* A rigid rotation about the hinge line is force free.
* Clamped cantilever under uniform load: with the trapezoid weights of the
  model, the discrete tip deflection equals q L^4/(8 beta) (1 + (ds/L)^2)
  exactly; its continuum limit is the Euler-Bernoulli value q L^4/(8 B).
* First bending mode of a clamped plate strip in vacuum:
  omega_1 = 1.8751^2 sqrt(beta/rho)/L^2 (Euler-Bernoulli).
* Forces are minus the gradient of the stored energy (finite differences),
  and the velocity-Verlet sub-steps conserve energy in vacuum.
"""
import math

import numpy as np
import pytest

from oracle.flag import FlagModel

RNG = np.random.default_rng(3)


def flat(ns, L=1.0, pitch=0.0, x_le=0.5, y_c=0.5, z_c=0.5):
    ds = L / (ns - 1)
    X = np.empty((ns, ns, 3))
    for b in range(ns):
        for a in range(ns):
            X[b, a] = (x_le + a * ds * math.cos(pitch), y_c + a * ds * math.sin(pitch),
                       z_c - 0.5 * L + b * ds)
    return X


def test_affine_has_no_bending():
    ns = 9
    F = FlagModel(flat(ns), 1.0, 1.0, 0.3, 100.0, le_bc=0)
    A = RNG.standard_normal((3, 3))
    c = RNG.standard_normal(3)
    X = flat(ns).reshape(-1, 3) @ A.T + c
    assert np.max(np.abs(F.K @ X)) < 1e-9 * np.max(np.abs(F.K.data))
    assert F.bending_energy(X) < 1e-20


def test_rotation_about_hinge_is_force_free():
    ns = 11
    X0 = flat(ns, pitch=0.3)
    F = FlagModel(X0, 1.0, 1.0, 0.05, 1000.0, le_bc=0)
    ang = 0.7
    R = np.array([[math.cos(ang), -math.sin(ang), 0], [math.sin(ang), math.cos(ang), 0], [0, 0, 1]])
    pivot = X0[0, 0].copy()
    X = (X0.reshape(-1, 3) - pivot) @ R.T + pivot
    f = F.forces(X, np.zeros_like(X))
    free = ~F.fixed
    assert np.max(np.abs(f[free])) < 1e-9


@pytest.mark.parametrize("ns", [9, 17, 33, 65])
def test_cantilever_uniform_load(ns):
    import scipy.sparse.linalg as spla
    L, beta, q = 1.0, 0.02, 0.3
    F = FlagModel(flat(ns, L), L, 1.0, beta, 0.0, le_bc=FlagModel.CLAMPED)
    free = np.where(~F.fixed)[0]
    A = (beta * F.K)[free][:, free].tocsc()
    y = spla.spsolve(A, q * F.dA[free])
    tip = y.reshape(ns, ns - 1)[:, -1]        # free nodes are a = 1..ns-1 per b
    ds = L / (ns - 1)
    exact = q * L ** 4 / (8 * beta) * (1 + (ds / L) ** 2)
    # exact up to round-off, which grows with cond(K) ~ ns^4
    tol = max(1e-13, 4e-16 * ns ** 4)
    assert np.max(np.abs(tip - exact)) < tol * exact
    # and the transverse profile is uniform in b (Poisson ratio 0)
    assert np.ptp(tip) < tol * exact


def test_spring_forces_brute_force():
    """Spring force on every node equals the sum over its lattice neighbours
    (a-, b- and (a+1, b+1)-diagonal neighbours) of -k (|d| - l0) d/|d|."""
    ns, ks = 4, 7.0
    X0 = flat(ns)
    F = FlagModel(X0, 1.0, 1.0, 0.0, ks)
    X = X0.reshape(-1, 3) + 0.03 * RNG.standard_normal((ns * ns, 3))
    f = F.spring_force(X)
    ds = 1.0 / (ns - 1)
    for b in range(ns):
        for a in range(ns):
            tot = np.zeros(3)
            for (da, db, l0) in [(1, 0, ds), (-1, 0, ds), (0, 1, ds), (0, -1, ds),
                                 (1, 1, math.sqrt(2) * ds), (-1, -1, math.sqrt(2) * ds)]:
                a2, b2 = a + da, b + db
                if 0 <= a2 < ns and 0 <= b2 < ns:
                    d = X[a + ns * b] - X[a2 + ns * b2]
                    ln = np.linalg.norm(d)
                    tot += -ks * (ln - l0) * d / ln
            assert np.allclose(f[a + ns * b], tot, atol=1e-13, rtol=1e-12)




def test_forces_are_energy_gradient():
    ns = 7
    F = FlagModel(flat(ns, pitch=0.2), 1.0, 1.0, 0.04, 50.0, le_bc=FlagModel.CLAMPED)
    X = flat(ns, pitch=0.2).reshape(-1, 3) + 0.02 * RNG.standard_normal((ns * ns, 3))
    f = F.bending_force(X) + F.spring_force(X)
    E = lambda Y: F.bending_energy(Y) + F.spring_energy(Y)
    eps = 1e-6
    for node in (3, 10, 24, 48):
        for c in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[node, c] += eps
            Xm[node, c] -= eps
            g = (E(Xp) - E(Xm)) / (2 * eps)
            assert abs(-g - f[node, c]) < 1e-6 * max(1.0, abs(g))


def test_energy_conserved_in_vacuum():
    ns = 9
    X0 = flat(ns, pitch=0.3)
    F = FlagModel(X0, 1.0, 1.0, 0.05, 400.0, le_bc=0)
    X = X0.reshape(-1, 3).copy()
    V = np.zeros_like(X)
    V[~F.fixed, 1] = 0.2 * np.linspace(0, 1, ns * ns)[~F.fixed]
    E0 = 0.5 * np.sum(F.mass[:, None] * V ** 2) + F.bending_energy(X) + F.spring_energy(X)
    for _ in range(300):
        X, V, _ = F.advance(X, V, np.zeros_like(X), 0.01)
    E1 = 0.5 * np.sum(F.mass[:, None] * V ** 2) + F.bending_energy(X) + F.spring_energy(X)
    assert abs(E1 - E0) < 5e-3 * E0
    assert F.max_strain(X) < 5e-3


@pytest.mark.parametrize("ns", [17, 33])
def test_first_mode_frequency(ns):
    """Released from the Euler-Bernoulli first-mode shape at small amplitude,
    the clamped strip oscillates at omega_1 = 1.8751^2 sqrt(beta/rho)/L^2 (1%)."""
    L, beta, rho = 1.0, 0.01, 1.0
    X0 = flat(ns, L)
    F = FlagModel(X0, L, rho, beta, 0.0, le_bc=FlagModel.CLAMPED)
    bl = 1.87510407
    sig = (math.sinh(bl) - math.sin(bl)) / (math.cosh(bl) + math.cos(bl))
    s = np.linspace(0, L, ns) * bl / L
    shape = np.cosh(s) - np.cos(s) - sig * (np.sinh(s) - np.sin(s))
    X = X0.reshape(-1, 3).copy()
    X[:, 1] += 1e-3 * L * np.tile(shape / shape[-1], ns)
    V = np.zeros_like(X)
    omega = bl ** 2 * math.sqrt(beta / rho) / L ** 2
    period = 2 * math.pi / omega
    dt = 0.05
    tip = [X[ns - 1, 1]]
    for n in range(int(1.2 * period / dt)):
        X, V, _ = F.advance(X, V, np.zeros_like(X), dt)
        tip.append(X[ns - 1, 1])
    tip = np.array(tip) - X0[0, ns - 1, 1]
    times = dt * np.arange(tip.size)
    imin = np.argmin(tip)
    imax = imin + np.argmax(tip[imin:])

    def refine(i):   # vertex of the parabola through three samples
        y0, y1, y2 = tip[i - 1], tip[i], tip[i + 1]
        return times[i] + 0.5 * dt * (y0 - y2) / (y0 - 2 * y1 + y2)
    T = refine(imax)
    assert abs(T - period) < 0.01 * period, (T, period)


def test_strain_scales_as_one_over_spring_stiffness():
    """Essential inextensibility comes from the in-plane springs alone: under
    a small in-plane pull on the trailing edge (bending off, leading edge
    fixed), the static edge strain of the triangulated network is inversely
    proportional to k_s.  Linear response: the stiffness is the finite-
    difference Jacobian of the spring forces at rest, restricted to the
    in-plane components of the free nodes (a triangulated sheet is rigid in
    its plane)."""
    ns, L = 6, 1.0
    X0 = flat(ns, L=L)                     # in the x-z plane
    x0 = X0.reshape(-1, 3)
    strains = {}
    for ks in (1e3, 1e4, 1e5):
        F = FlagModel(X0, L, 1.0, 0.0, ks, le_bc=0)
        dofs = [(n, c) for n in range(ns * ns) if not F.fixed[n] for c in (0, 2)]
        eta = 1e-7 * F.ds
        J = np.empty((len(dofs), len(dofs)))
        for col, (n, c) in enumerate(dofs):
            xp, xm = x0.copy(), x0.copy()
            xp[n, c] += eta
            xm[n, c] -= eta
            df = (F.spring_force(xp) - F.spring_force(xm)) / (2 * eta)
            J[:, col] = [df[m, cc] for (m, cc) in dofs]
        load = np.array([1e-3 if (m % ns == ns - 1 and cc == 0) else 0.0 for (m, cc) in dofs])
        d = np.linalg.solve(-J, load)
        x = x0.copy()
        for (m, cc), val in zip(dofs, d):
            x[m, cc] += val
        strains[ks] = F.max_strain(x)
    assert strains[1e3] > 1e-6
    assert strains[1e3] / strains[1e4] == pytest.approx(10.0, rel=1e-4)
    assert strains[1e4] / strains[1e5] == pytest.approx(10.0, rel=1e-4)
