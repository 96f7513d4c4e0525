"""Whole-step properties of the oracle (oracle/solver.py).

* Shifting the initial condition and every immersed body by whole cells in
  y or z shifts the solution (periodic directions; the paper's box is
  periodic in y and z, Sec. II.A).
* On the small flag workload: the projected field is divergence free to
  machine level, the outflow equals the inflow, the flag stays essentially
  inextensible and its leading edge does not move.
"""
import numpy as np
import pytest

import synth
from oracle import geometry
from oracle import fluid
from oracle.solver import Solver


def _flag_args(w, X0):
    f = w.flag
    return dict(X0=X0, length=f.length, rho=f.mass_ratio, beta=f.bending, ks=f.stretch,
                le_bc=f.le_bc)


def _small_with_bars():
    w = synth.Workload(name="t", nx=48, ny=24, nz=24, lx=6.0, ly=3.0, lz=3.0, re=300.0,
                       dt=0.0, cfl=0.4, grid=synth.Grid(x_plane=0.75, mesh=1.5, bar=0.3),
                       flag=synth.Flag(ns=8, length=1.0, x_le=2.0, y_c=1.5, z_c=1.5,
                                       bending=0.01))
    return w


@pytest.mark.parametrize("axis,shift", [(1, 3), (0, 5)])
def test_shift_symmetry(axis, shift):
    w = _small_with_bars()
    noise = synth.ic_noise(w)
    bars = geometry.grid_points_of(w)
    X0 = geometry.flag_lattice(w.flag)
    S1 = Solver(w, noise, bars, _flag_args(w, X0))
    S1.step(4)
    h = w.h
    rolled = tuple(np.roll(z, shift, axis=axis) for z in noise)
    bX = bars[0].copy()
    col = 1 if axis == 1 else 2
    L = w.ly if axis == 1 else w.lz
    bX[:, col] = np.mod(bX[:, col] + shift * h, L)
    X0s = X0.copy()
    X0s[..., col] += shift * h
    S2 = Solver(w, rolled, (bX, bars[1]), _flag_args(w, X0s))
    S2.step(4)
    for a, b in zip(S1.fields()[:3], S2.fields()[:3]):
        assert np.max(np.abs(np.roll(a, shift, axis=axis) - b)) < 1e-12
    Xs = S1.X.copy()
    Xs[:, col] += shift * h
    assert np.max(np.abs(Xs - S2.X)) < 1e-12


def test_small_flag_workload_invariants():
    w = synth.flag_64_re200()
    X0 = geometry.flag_lattice(w.flag)
    S = Solver(w, synth.ic_noise(w), None, _flag_args(w, X0))
    for _ in range(w.steps):
        S.step()
        d = fluid.divergence(S.f.u, S.f.v, S.f.w, S.h)
        assert np.max(np.abs(d)) < 1e-12
        assert abs(np.sum(S.f.u[..., -1]) - np.sum(S.f.u[..., 0])) < 1e-12 * S.f.u[..., 0].size
        assert S.flag.max_strain(S.X) < 5e-3     # impulsive start: load ~ U h / dt
    assert np.array_equal(S.X.reshape(16, 16, 3)[:, 0], X0[:, 0])
    assert np.all(np.isfinite(S.f.u))
