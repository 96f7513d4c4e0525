"""Shared set-up of the GPU parity tests: the same seeded inputs (synth) go to
the HIP library (through the C ABI binding) and to the oracle."""
import numpy as np

import synth
from oracle import geometry


def oracle_flag_args(w, X0):
    f = w.flag
    return dict(X0=X0, length=f.length, rho=f.mass_ratio, beta=f.bending, ks=f.stretch,
                le_bc=f.le_bc)


def build_pair(w, hooks=0, with_noise=True, precision=0, noise=None):
    """(gpu_run, oracle_solver) on identical inputs: the library builds its
    bodies from the workload's parameters, the oracle its own (oracle.geometry).
    precision: the library's (the oracle is FP64); noise: precomputed ic_noise."""
    import paper_2103_08246_amd as ib
    from oracle.solver import Solver
    if noise is None and with_noise:
        noise = synth.ic_noise(w)
    bars = geometry.grid_points_of(w) if w.grid is not None else None
    X0 = geometry.flag_lattice(w.flag) if w.flag is not None else None
    run = ib.create(ib.domain_from(w, flags=hooks, precision=precision), noise, grid=w.grid, flag=w.flag)
    S = Solver(w, noise, bars, oracle_flag_args(w, X0) if X0 is not None else None, hooks=hooks)
    return run, S


def rel_l2(a_list, b_list):
    num = sum(float(np.sum((np.asarray(a) - np.asarray(b)) ** 2)) for a, b in zip(a_list, b_list))
    den = sum(float(np.sum(np.asarray(b) ** 2)) for b in b_list)
    return (num / den) ** 0.5


def demean(p):
    return p - p.mean()
