"""CPU oracle for the immersed-boundary DNS time step -- TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 numpy implementation of one fractional-step time step of
the paper's method (Sec. II.B): incompressible Navier-Stokes (Eqs. 2-3) on a
staggered Cartesian mesh with second-order centred differences, Adams-Bashforth
nonlinear terms (diffusion explicit, or Crank-Nicolson with approximate
factorisation), direct-forcing immersed boundaries for the passive grid (delta
points, or Eulerian forcing at the nodes) and the flag (delta at the nodes, or
MLS at the markers of an adaptive tiling), a pressure-Poisson projection, and
the flag's spring-network structural update; virtual probes for the in-situ
statistics.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never imports it and
shares no code with it; the only common module is ``synth`` (seeded inputs
and workload parameters).  The immersed bodies are built here from the
problem statement's parameters (``geometry``), independently of the
library's own construction.

Readings of passages the paper leaves open are stated where they are used,
and collected in the design notes of the repository.

Parity pins (tests/test_oracle_*.py) tie every function here to closed
forms, invariants or brute force.  The full coupled step has no value printed
in the paper: beyond its parts, its parity is unpinned.
"""
from .delta import roma, stencil, interpolate, spread, ibm_force  # noqa: F401
from .fluid import (Fields, rhs, predictor, outlet, flux_correct, divergence,  # noqa: F401
                    project, cfl_dt)
from .poisson import solve_poisson, apply_laplacian  # noqa: F401
from .flag import FlagModel  # noqa: F401
from .probes import ProbeStats, probe_positions, station_statistics  # noqa: F401
from .grid_forcing import GridGeometry, forcing_list  # noqa: F401
from .mls import mls_stencil, build_markers, node_load  # noqa: F401
from .geometry import grid_points, grid_points_of, flag_lattice  # noqa: F401
from .solver import Solver  # noqa: F401
