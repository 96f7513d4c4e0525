"""One fractional time step of the immersed-boundary DNS, in the paper's order (oracle).

Sec. II.B: a provisional, non-solenoidal velocity is computed, the
immersed-boundary forcing is applied to it, and it is then projected onto a
divergence-free field by solving a Poisson equation; the structure is
advanced by its own solver.  Steps, per time step n:

  S1  H^n = -div(u u) + nu lap(u)                         (fluid.rhs)
  S2  u~ = u^n + dt[(1+w/2) H^n - (w/2) H^{n-1} - G p^n]  (fluid.predictor)
  S3  convective outflow on u at the outlet and the v, w ghosts  (fluid.outlet)
  S4  outflow flux correction                             (fluid.flux_correct)
  S5  direct forcing on u~: passive-grid points (target 0) then flag nodes
      (target V^n)                                        (delta.ibm_force)
      or, with MLS coupling, the flag's tiling markers    (mls)
  S6  r = D u~ / dt
  S7  L phi = r                                           (poisson.solve_poisson)
  S8  u^{n+1} = u~ - dt G phi,  p^{n+1} = p^n + phi        (fluid.project)
  S9  dt_{n+1}: fixed, or from the CFL number              (fluid.cfl_dt)
  S10 flag: load f_h = -F_k dV_k from S5, spring-network sub-steps (flag)
  S11 H^{n-1} <- H^n, t += dt_n
Optionally (Sec. III) virtual probes sample u^{n+1} after S8 (probes).

Initial condition (reading; the paper starts from a uniform stream):
u = U + A z on every u face i = 1..nx, v = A z and w = A z on every cell,
with z the supplied standard-normal noise; u = U at the inlet face; outlet
ghosts copy the last cell; p = 0; the field is then made divergence-free by
S4 and S6-S8 with dt = 1 (phi discarded), and dt_0 is taken from S9.
"""
from __future__ import annotations

import numpy as np

from . import fluid
from .delta import ibm_force, ibm_interp, ibm_spread
from . import mls
from .flag import FlagModel
from .poisson import solve_poisson
from .probes import ProbeStats, probe_positions
from .grid_forcing import GridGeometry, forcing_list as grid_forcing_list, apply as grid_forcing_apply


class Solver:
    """Oracle state and time stepper.

    params: object with nx, ny, nz, lx, ly, lz, re, u_in, dt, cfl, noise_amp.
    noise: (zu, zv, zw) standard normals, shapes (nz, ny, nx+1), (nz, ny, nx) x2.
    bars: (X (K, 3), dV (K,)) static solid points or None.
    flag: dict(X0=(ns, ns, 3), length, rho, beta, ks, le_bc, coupling) or None;
      coupling "nodes" (default): the flag's nodes are its delta markers;
      "mls": MLS transfer at the markers of the adaptive tiling (oracle.mls).
    """

    def __init__(self, params, noise=None, bars=None, flag=None, hooks: int = 0,
                 advection: bool = True, probes=None, grid_forcing=None, diffusion: str = "explicit"):
        P = params
        self.nx, self.ny, self.nz = P.nx, P.ny, P.nz
        self.h = P.lx / P.nx
        self.nu = 1.0 / P.re
        self.u_in = P.u_in
        self.dt_fixed = P.dt
        self.cfl = P.cfl
        self.hooks = hooks
        self.advection = advection
        if diffusion not in ("explicit", "cn"):
            raise ValueError(diffusion)
        self.diffusion = diffusion
        nx, ny, nz = self.nx, self.ny, self.nz
        A = P.noise_amp
        u = np.full((nz, ny, nx + 1), P.u_in)
        v = np.zeros((nz, ny, nx + 1))
        w = np.zeros((nz, ny, nx + 1))
        if noise is not None and A != 0.0:
            zu, zv, zw = noise
            u[..., 1:] = P.u_in + A * zu[..., 1:]
            v[..., :nx] = A * zv
            w[..., :nx] = A * zw
        v[..., nx] = v[..., nx - 1]
        w[..., nx] = w[..., nx - 1]
        self.f = fluid.Fields(u=u, v=v, w=w, p=np.zeros((nz, ny, nx)))
        # bodies
        if bars is not None and bars[0].shape[0] > 0:
            self.bar_X = np.asarray(bars[0], dtype=np.float64)
            self.bar_dV = np.asarray(bars[1], dtype=np.float64)
        else:
            self.bar_X = np.zeros((0, 3))
            self.bar_dV = np.zeros(0)
        self.flag = None
        if flag is not None:
            self.flag = FlagModel(flag["X0"], flag["length"], flag["rho"], flag["beta"],
                                  flag["ks"], flag.get("le_bc", 0))
            self.X = np.asarray(flag["X0"], dtype=np.float64).reshape(-1, 3).copy()
            self.V = np.zeros_like(self.X)
            self.flag_dV = self.flag.dA * self.h
            self.F_flag = np.zeros_like(self.X)
        self.mls = None
        if flag is not None and flag.get("coupling", "nodes") == "mls":
            tri, beta, dVm, _ = mls.build_markers(flag["X0"], self.h)
            self.mls = dict(tri=tri, beta=beta, dV=dVm)
            self.F_flag = np.zeros((tri.shape[0], 3))
        elif flag is not None and flag.get("coupling", "nodes") != "nodes":
            raise ValueError(flag["coupling"])
        self.F_bar = np.zeros((self.bar_X.shape[0], 3))
        self.nsub = 0
        # Eulerian forcing of the passive grid (dict x_plane, mesh, bar) instead of points
        self.grid_lists = None
        if grid_forcing is not None:
            if self.bar_X.shape[0] > 0:
                raise ValueError("Eulerian grid forcing replaces the static points")
            geom = GridGeometry(grid_forcing["x_plane"], grid_forcing["mesh"], grid_forcing["bar"],
                                P.ly, P.lz)
            self.grid_lists = [grid_forcing_list(geom, c, nx, ny, nz, self.h) for c in range(3)]
        # virtual probes (dict n_x, x0, dx, yc, zc, dyz, n_lags), sampled after each projection
        self.probes = None
        if probes is not None:
            P_ = probes
            self.probes = ProbeStats(probe_positions(P_["n_x"], P_["x0"], P_["dx"], P_["yc"], P_["zc"],
                                                     P_["dyz"]), P_["n_lags"])
        # initial projection with dt = 1 (phi discarded)
        ut, vt, wt = self.f.u.copy(), self.f.v.copy(), self.f.w.copy()
        fluid.flux_correct(ut)
        r = fluid.divergence(ut, vt, wt, self.h)
        phi = solve_poisson(r, self.h)
        p0 = self.f.p.copy()
        fluid.project(self.f, ut, vt, wt, phi, 1.0, self.h)
        self.f.p = p0
        self.dt = self._next_dt()
        self.dt_prev = self.dt
        self.H_old = None
        self.t = 0.0
        self.step_count = 0

    def _next_dt(self):
        if self.dt_fixed > 0.0:
            return self.dt_fixed
        return fluid.cfl_dt(self.f, self.h, self.cfl)

    def markers(self):
        """All immersed points in forcing order: grid points, then flag nodes."""
        if self.flag is None:
            return self.bar_X, np.zeros_like(self.bar_X), self.bar_dV
        X = np.concatenate([self.bar_X, self.X])
        Ud = np.concatenate([np.zeros_like(self.bar_X), self.V])
        dV = np.concatenate([self.bar_dV, self.flag_dV])
        return X, Ud, dV

    # ---- the step, split so that tests can stop after any stage ----
    def stage_predict(self):
        """S1-S4: returns (ut, vt, wt, H).  With Crank-Nicolson diffusion H is
        the convective part only and S2 is fluid.predictor_cn, which needs the
        outflow values of S3 first."""
        f, h, dt = self.f, self.h, self.dt
        omega = dt / self.dt_prev
        if self.diffusion == "cn":
            Hc = fluid.rhs(f, h, 0.0, self.hooks, self.advection)
            D = fluid.rhs(f, h, self.nu, self.hooks, advection=False)
            Hc_old = Hc if self.H_old is None else self.H_old
            ut, vt, wt = f.u.copy(), f.v.copy(), f.w.copy()
            fluid.outlet(f, ut, vt, wt, dt, h, self.u_in, self.hooks)
            fluid.predictor_cn(f, Hc, Hc_old, D, ut, vt, wt, dt, omega, h, self.nu, self.hooks)
            fluid.flux_correct(ut)
            return ut, vt, wt, Hc
        H = fluid.rhs(f, h, self.nu, self.hooks, self.advection)
        H_old = H if self.H_old is None else self.H_old
        ut, vt, wt = fluid.predictor(f, H, H_old, dt, omega, h)
        fluid.outlet(f, ut, vt, wt, dt, h, self.u_in, self.hooks)
        fluid.flux_correct(ut)
        return ut, vt, wt, H

    def stage_ibm(self, ut, vt, wt):
        """S5 on the provisional velocity (in place); returns F (K, 3).  With
        Eulerian grid forcing the grid is forced first, at its nodes."""
        if self.grid_lists is not None:
            grid_forcing_apply(ut, vt, wt, self.grid_lists)
        if self.mls is not None:
            # grid points (delta) and flag markers (MLS) all read the unforced
            # field, then spread in that order
            fields = (ut, vt, wt)
            M = self.mls
            Xm, Vm = mls.marker_state(M["tri"], M["beta"], self.X, self.V)
            Fb, maps_b = ibm_interp(fields, self.bar_X, np.zeros_like(self.bar_X), self.h, self.dt, self.nx)
            Fm, maps_m = mls.mls_interp(fields, Xm, Vm, self.h, self.dt, self.nx)
            ibm_spread(fields, maps_b, Fb, self.bar_dV, self.h, self.dt)
            mls.mls_spread(fields, maps_m, Fm, M["dV"], self.h, self.dt)
            self.F_bar, self.F_flag = Fb, Fm
            return np.concatenate([Fb, Fm])
        X, Ud, dV = self.markers()
        F = ibm_force(ut, vt, wt, X, Ud, dV, self.h, self.dt, self.nx)
        nb = self.bar_X.shape[0]
        self.F_bar = F[:nb]
        if self.flag is not None:
            self.F_flag = F[nb:]
        return F

    def stage_project(self, ut, vt, wt):
        """S6-S8; returns phi."""
        r = fluid.divergence(ut, vt, wt, self.h) / self.dt
        phi = solve_poisson(r, self.h)
        fluid.project(self.f, ut, vt, wt, phi, self.dt, self.h)
        return phi

    def stage_flag(self):
        """S10 with the forcing of this step."""
        if self.flag is None:
            return
        if self.mls is not None:
            M = self.mls
            f_h = mls.node_load(M["tri"], M["beta"], self.F_flag, M["dV"], self.X.shape[0])
        else:
            f_h = -self.F_flag * self.flag_dV[:, None]
        self.X, self.V, self.nsub = self.flag.advance(self.X, self.V, f_h, self.dt)

    def step(self, n: int = 1):
        for _ in range(n):
            ut, vt, wt, H = self.stage_predict()
            self.stage_ibm(ut, vt, wt)
            self.stage_project(ut, vt, wt)
            if self.probes is not None:
                self.probes.sample_fields(self.f, self.h)
            dt_next = self._next_dt()
            self.stage_flag()
            self.H_old = H
            self.t += self.dt
            self.dt_prev = self.dt
            self.dt = dt_next
            self.step_count += 1

    # ---- views in the library's output layout ----
    def fields(self):
        """(u (nz,ny,nx+1), v (nz,ny,nx), w (nz,ny,nx), p (nz,ny,nx))."""
        nx = self.nx
        return (self.f.u.copy(), self.f.v[..., :nx].copy(), self.f.w[..., :nx].copy(),
                self.f.p.copy())


def set_state(S: Solver, u, v, w, p=None):
    """Overwrite the oracle state (tests only); v, w given as (nz, ny, nx) or with ghost."""
    nx = S.nx
    S.f.u = np.array(u, dtype=np.float64, copy=True)
    vv = np.zeros((S.nz, S.ny, nx + 1))
    ww = np.zeros((S.nz, S.ny, nx + 1))
    vv[..., :v.shape[2]] = v
    ww[..., :w.shape[2]] = w
    if v.shape[2] == nx:
        vv[..., nx] = v[..., nx - 1]
        ww[..., nx] = w[..., nx - 1]
    S.f.v, S.f.w = vv, ww
    S.f.p = np.zeros((S.nz, S.ny, nx)) if p is None else np.array(p, dtype=np.float64)
    S.dt = S._next_dt()
    S.dt_prev = S.dt
    S.H_old = None
