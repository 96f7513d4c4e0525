"""The fluid step in plain C (oracle/c/ref_step.c) -- TEST INFRASTRUCTURE ONLY.

The same scheme and readings as ``oracle.solver.Solver`` (Sec. II.B: RHS and
Adams-Bashforth predictor, convective outflow and flux correction, direct
forcing of the grid's points and the flag's nodes with the 3-point delta,
divergence, FFT/tridiagonal Poisson solve, projection, CFL time step; the
flag's spring network by ``oracle.flag.FlagModel``), with the fluid stages as
C loops over the host's cores, so that the 768 x 384 x 384 workload can be
stepped in test time.  Options beyond that path (Crank-Nicolson, Eulerian
grid forcing, MLS markers, probes) exist only in ``Solver``.

The C stages are pinned stage by stage against ``Solver``'s numpy stages
(tests/test_oracle_fast.py), and the whole step against ``Solver`` over ten
steps; the numpy stages carry the closed-form pins.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .flag import FlagModel

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libibdns_ref.so")

_lib = None


def lib():
    """The C oracle, built on first use if it is not there yet."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            from .build_ref import build
            build()
        L = ctypes.CDLL(LIB)
        D = ctypes.POINTER(ctypes.c_double)
        i, d, l_ = ctypes.c_int, ctypes.c_double, ctypes.c_long
        L.ref_rhs.argtypes = [i, i, i, d, d, i, i, D, D, D, D, D, D]
        L.ref_predictor.argtypes = [i, i, i, d, d, d, D, D, D, D, D, D, D, D, D, D, D, D, D]
        L.ref_outlet.argtypes = [i, i, i, d, d, d, i, D, D, D, D, D, D]
        L.ref_flux_correct.argtypes = [i, i, i, D]
        L.ref_flux_correct.restype = d
        L.ref_ibm.argtypes = [i, i, i, d, d, l_, D, D, D, D, D, D, D]
        L.ref_ibm.restype = i
        L.ref_divergence.argtypes = [i, i, i, d, D, D, D, D]
        L.ref_poisson.argtypes = [i, i, i, d, D, D]
        L.ref_project.argtypes = [i, i, i, d, d, D, D, D, D, i, D, D, D, D]
        L.ref_max_speed.argtypes = [i, i, i, D, D, D]
        L.ref_max_speed.restype = d
        L.ref_num_threads.restype = i
        _lib = L
    return _lib


def threads() -> int:
    return lib().ref_num_threads()


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---- the stages, one C call each (arrays in the oracle's [k, j, i] layout) ----

def rhs(u, v, w, h, nu, hooks=0, advection=True, out=None):
    nz, ny, nxp = u.shape
    H = [np.empty_like(u) for _ in range(3)] if out is None else out
    lib().ref_rhs(nxp - 1, ny, nz, h, nu, hooks, 1 if advection else 0, _p(u), _p(v), _p(w),
                  _p(H[0]), _p(H[1]), _p(H[2]))
    return H


def predictor(u, v, w, p, H, H_old, dt, omega, h, out=None):
    nz, ny, nxp = u.shape
    ut, vt, wt = (np.empty_like(u) for _ in range(3)) if out is None else out
    lib().ref_predictor(nxp - 1, ny, nz, h, dt, omega, _p(u), _p(v), _p(w), _p(p), _p(H[0]), _p(H[1]),
                        _p(H[2]), _p(H_old[0]), _p(H_old[1]), _p(H_old[2]), _p(ut), _p(vt), _p(wt))
    return ut, vt, wt


def outlet(u, v, w, ut, vt, wt, dt, h, u_conv, hooks=0):
    nz, ny, nxp = u.shape
    lib().ref_outlet(nxp - 1, ny, nz, h, dt, u_conv, hooks, _p(u), _p(v), _p(w), _p(ut), _p(vt), _p(wt))


def flux_correct(ut):
    nz, ny, nxp = ut.shape
    return lib().ref_flux_correct(nxp - 1, ny, nz, _p(ut))


def ibm(ut, vt, wt, X, Ud, dV, h, dt):
    nz, ny, nxp = ut.shape
    K = X.shape[0]
    F = np.zeros((K, 3))
    X = np.ascontiguousarray(X, dtype=np.float64)
    Ud = None if Ud is None else np.ascontiguousarray(Ud, dtype=np.float64)
    dV = np.ascontiguousarray(dV, dtype=np.float64)
    if lib().ref_ibm(nxp - 1, ny, nz, h, dt, K, _p(X), _p(Ud), _p(dV), _p(ut), _p(vt), _p(wt), _p(F)) != 0:
        raise ValueError("immersed point support leaves the evolved x range")
    return F


def divergence(ut, vt, wt, h, out=None):
    nz, ny, nxp = ut.shape
    r = np.empty((nz, ny, nxp - 1)) if out is None else out
    lib().ref_divergence(nxp - 1, ny, nz, h, _p(ut), _p(vt), _p(wt), _p(r))
    return r


def poisson(r, h, out=None):
    nz, ny, nx = r.shape
    r = np.ascontiguousarray(r)
    phi = np.empty_like(r) if out is None else out
    lib().ref_poisson(nx, ny, nz, h, _p(r), _p(phi))
    return phi


def project(ut, vt, wt, phi, dt, h, u, v, w, p, update_p=True):
    """In place on u, v, w (and p when update_p)."""
    nz, ny, nxp = ut.shape
    lib().ref_project(nxp - 1, ny, nz, h, dt, _p(ut), _p(vt), _p(wt), _p(phi), 1 if update_p else 0,
                      _p(u), _p(v), _p(w), _p(p))


def max_speed(u, v, w):
    nz, ny, nxp = u.shape
    return lib().ref_max_speed(nxp - 1, ny, nz, _p(u), _p(v), _p(w))


class FastSolver:
    """State and time stepper with the C fluid stages (same arguments as
    ``oracle.solver.Solver`` for the delta-coupled path: params, noise, bars
    (X, dV) or None, flag dict (X0, length, rho, beta, ks, le_bc) or None,
    hooks)."""

    def __init__(self, params, noise=None, bars=None, flag=None, hooks: int = 0):
        P = params
        self.nx, self.ny, self.nz = P.nx, P.ny, P.nz
        self.h = P.lx / P.nx
        self.nu = 1.0 / P.re
        self.u_in = P.u_in
        self.dt_fixed = P.dt
        self.cfl = P.cfl
        self.hooks = hooks
        nx, ny, nz = self.nx, self.ny, self.nz
        A = P.noise_amp
        # initial condition (the same reading as Solver)
        self.u = np.full((nz, ny, nx + 1), P.u_in)
        self.v = np.zeros((nz, ny, nx + 1))
        self.w = np.zeros((nz, ny, nx + 1))
        if noise is not None and A != 0.0:
            zu, zv, zw = noise
            self.u[..., 1:] = P.u_in + A * zu[..., 1:]
            self.v[..., :nx] = A * zv
            self.w[..., :nx] = A * zw
        self.v[..., nx] = self.v[..., nx - 1]
        self.w[..., nx] = self.w[..., nx - 1]
        self.p = np.zeros((nz, ny, nx))
        if bars is not None and bars[0].shape[0] > 0:
            self.bar_X = np.ascontiguousarray(bars[0], dtype=np.float64)
            self.bar_dV = np.ascontiguousarray(bars[1], dtype=np.float64)
        else:
            self.bar_X = np.zeros((0, 3))
            self.bar_dV = np.zeros(0)
        self.flag = None
        if flag is not None:
            self.flag = FlagModel(flag["X0"], flag["length"], flag["rho"], flag["beta"], flag["ks"],
                                  flag.get("le_bc", 0))
            self.X = np.asarray(flag["X0"], dtype=np.float64).reshape(-1, 3).copy()
            self.V = np.zeros_like(self.X)
            self.flag_dV = self.flag.dA * self.h
            self.F_flag = np.zeros_like(self.X)
        self.F_bar = np.zeros((self.bar_X.shape[0], 3))
        self.nsub = 0
        # work arrays reused every step (two H buffers: H^n and H^{n-1})
        self._H = [[np.empty_like(self.u) for _ in range(3)] for _ in range(2)]
        self._cur = 0
        self._tilde = [np.empty_like(self.u) for _ in range(3)]
        self._r = np.empty((nz, ny, nx))
        self._phi = np.empty((nz, ny, nx))
        # initial projection with dt = 1, p untouched
        ut, vt, wt = self.u.copy(), self.v.copy(), self.w.copy()
        flux_correct(ut)
        phi = poisson(divergence(ut, vt, wt, self.h), self.h)
        project(ut, vt, wt, phi, 1.0, self.h, self.u, self.v, self.w, self.p, update_p=False)
        self.dt = self._next_dt()
        self.dt_prev = self.dt
        self.H_old = None
        self.t = 0.0
        self.step_count = 0

    def _next_dt(self):
        if self.dt_fixed > 0.0:
            return self.dt_fixed
        return self.cfl * self.h / max_speed(self.u, self.v, self.w)

    def markers(self):
        if self.flag is None:
            return self.bar_X, np.zeros_like(self.bar_X), self.bar_dV
        return (np.concatenate([self.bar_X, self.X]), np.concatenate([np.zeros_like(self.bar_X), self.V]),
                np.concatenate([self.bar_dV, self.flag_dV]))

    def stage_predict(self):
        """S1-S4: (ut, vt, wt, H)."""
        h, dt = self.h, self.dt
        # H^n goes to the buffer that does not hold H^{n-1}
        self._cur = 1 - self._cur if self.H_old is self._H[self._cur] else self._cur
        H = rhs(self.u, self.v, self.w, h, self.nu, self.hooks, out=self._H[self._cur])
        H_old = H if self.H_old is None else self.H_old
        ut, vt, wt = predictor(self.u, self.v, self.w, self.p, H, H_old, dt, dt / self.dt_prev, h,
                               out=self._tilde)
        outlet(self.u, self.v, self.w, ut, vt, wt, dt, h, self.u_in, self.hooks)
        flux_correct(ut)
        return ut, vt, wt, H

    def stage_ibm(self, ut, vt, wt):
        """S5 in place; returns F (K, 3)."""
        X, Ud, dV = self.markers()
        F = ibm(ut, vt, wt, X, Ud, dV, self.h, self.dt)
        nb = self.bar_X.shape[0]
        self.F_bar = F[:nb]
        if self.flag is not None:
            self.F_flag = F[nb:]
        return F

    def stage_project(self, ut, vt, wt):
        """S6-S8; returns phi."""
        r = divergence(ut, vt, wt, self.h, out=self._r)
        r /= self.dt
        phi = poisson(r, self.h, out=self._phi)
        project(ut, vt, wt, phi, self.dt, self.h, self.u, self.v, self.w, self.p)
        return phi

    def stage_flag(self):
        if self.flag is None:
            return
        f_h = -self.F_flag * self.flag_dV[:, None]
        self.X, self.V, self.nsub = self.flag.advance(self.X, self.V, f_h, self.dt)

    def step(self, n: int = 1):
        for _ in range(n):
            ut, vt, wt, H = self.stage_predict()
            self.stage_ibm(ut, vt, wt)
            self.stage_project(ut, vt, wt)
            dt_next = self._next_dt()
            self.stage_flag()
            self.H_old = H
            self.t += self.dt
            self.dt_prev = self.dt
            self.dt = dt_next
            self.step_count += 1

    def fields(self):
        """(u (nz,ny,nx+1), v (nz,ny,nx), w (nz,ny,nx), p (nz,ny,nx)) as in Solver.fields."""
        nx = self.nx
        return (self.u.copy(), self.v[..., :nx].copy(), self.w[..., :nx].copy(), self.p.copy())
