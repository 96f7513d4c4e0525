"""Seeded synthetic inputs shared by the oracle and the GPU library.

This module holds only *inputs*: the workload parameters (box, Re, the
passive grid's and the flag's parameters) and the Gaussian noise of the
initial condition.  It contains none of the time step's arithmetic and builds
no geometry: the library builds its bodies from the parameters, and the
oracle builds its own (``oracle/geometry.py``).  The oracle (``oracle/``) and
the HIP library (``paper_2103_08246_amd``) never import each other.

Problem statement (paper, Sec. II.A and Fig. 1): a box with uniform inflow
(U, 0, 0), convective outflow, periodic y and z; a monoplane passive grid of
square rods of side d and spacing M placed M/2 downstream of the inlet; a
square flag of side L hinged at its leading edge, initially straight and
pitched by theta = 0.1 pi.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace
from typing import Optional

import numpy as np

SEED_BASE = 2103


@dataclass(frozen=True)
class Grid:
    """Passive grid of square rods (Sec. II.A): plane x = x_plane, mesh M, rod side d."""
    x_plane: float
    mesh: float
    bar: float


@dataclass(frozen=True)
class Flag:
    """Square flag of side L on an ns x ns node lattice (Sec. II.A)."""
    ns: int
    length: float
    x_le: float
    y_c: float
    z_c: float
    pitch: float = 0.1 * math.pi
    mass_ratio: float = 1.0
    bending: float = 1e-4
    stretch: float = 1.0e4        # in-plane spring stiffness (essentially inextensible)
    le_bc: int = 0                # 0 hinged, 1 clamped


@dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    re: float
    u_in: float = 1.0
    dt: float = 0.0               # > 0 fixed, <= 0 CFL-adaptive
    cfl: float = 0.5
    noise_amp: float = 0.05
    seed: int = SEED_BASE
    steps: int = 10
    grid: Optional[Grid] = None
    flag: Optional[Flag] = None

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def h(self) -> float:
        return self.lx / self.nx


def flag_64_re200() -> Workload:
    """Small plain-FP64 case: 4L x 2L x 2L on 64 x 32 x 32, Re 200, one 16 x 16 flag, dt 1e-3."""
    return Workload(
        name="flag_64x32x32_re200", nx=64, ny=32, nz=32, lx=4.0, ly=2.0, lz=2.0,
        re=200.0, dt=1e-3, steps=10,
        flag=Flag(ns=16, length=1.0, x_le=1.0, y_c=1.0, z_c=1.0, bending=0.01))


def grid_flag_768_re1000() -> Workload:
    """Paper-like scale: 12L x 6L x 6L on 768 x 384 x 384 (113M cells), Re 1000,
    passive grid (M = 0.5L, d = 0.1L) at x = M/2, 96 x 96 flag 6M downstream, CFL 0.5."""
    M = 0.5
    return Workload(
        name="grid_flag_768x384x384_re1000", nx=768, ny=384, nz=384, lx=12.0, ly=6.0,
        lz=6.0, re=1000.0, dt=0.0, cfl=0.5, steps=200,
        grid=Grid(x_plane=0.5 * M, mesh=M, bar=0.1),
        flag=Flag(ns=96, length=1.0, x_le=0.5 * M + 6 * M, y_c=3.0, z_c=3.0, bending=1e-3))


def grid_flag_batch_member(nx: int, r: int, dist_m: float, ns: int = 24,
                           re: float = 500.0, bending: float = 1e-3) -> Workload:
    """One member of an uneven ensemble: 12L x 6L x 6L box, nx x nx/2 x nx/2 cells."""
    M = 0.5
    return Workload(
        name=f"grid_flag_{nx}x{nx//2}x{nx//2}_d{dist_m:g}M", nx=nx, ny=nx // 2, nz=nx // 2,
        lx=12.0, ly=6.0, lz=6.0, re=re, dt=0.0, cfl=0.5, seed=SEED_BASE + r, steps=200,
        grid=Grid(x_plane=0.5 * M, mesh=M, bar=0.1),
        flag=Flag(ns=ns, length=1.0, x_le=0.5 * M + dist_m * M, y_c=3.0, z_c=3.0,
                  bending=bending))


def ensemble_24() -> list:
    """24 independent runs: 8 each of 96^, 128^ and 192^ (x by x/2 by x/2) grids,
    flag distance linspace(2M, 10M, 8) within each size group, Re 500."""
    runs = []
    r = 0
    for nx in (96, 128, 192):
        for dist in np.linspace(2.0, 10.0, 8):
            runs.append(grid_flag_batch_member(nx, r, float(dist)))
            r += 1
    return runs


def ensemble_6_384() -> list:
    """6 runs of 384 x 192 x 192 with grid bars and a 64 x 64 flag at 3..10 M, Re 1000."""
    return [grid_flag_batch_member(384, r, d, ns=64, re=1000.0)
            for r, d in enumerate((3.0, 4.0, 5.0, 6.0, 8.0, 10.0))]


def probe_layout(w: Workload, n_lags: int = 64) -> dict:
    """Virtual-probe arrangement of Sec. III on this machine: stations every M/2
    in x from x = M/2 to Lx - M/2, three by three probes 2M/3 apart around the
    centreline (M = the grid's mesh, 1 without a grid)."""
    M = w.grid.mesh if w.grid is not None else 1.0
    dx, x0 = 0.5 * M, 0.5 * M
    n_x = int(np.floor((w.lx - 0.5 * M - x0) / dx + 1e-9)) + 1
    return dict(n_x=n_x, x0=x0, dx=dx, yc=0.5 * w.ly, zc=0.5 * w.lz, dyz=2.0 * M / 3.0,
                n_lags=n_lags)


def scaled(w: Workload, nx: int, ny: int, nz: int, **kw) -> Workload:
    """Same box and physics on another mesh (keeps h isotropic if the ratios are kept)."""
    return replace(w, nx=nx, ny=ny, nz=nz, **kw)


# --------------------------------------------------------------------------------------
# Initial-condition noise
# --------------------------------------------------------------------------------------

def ic_noise(w: Workload):
    """Standard-normal noise for the initial velocity, one value per degree of freedom.

    Returns (zu, zv, zw) with shapes (nz, ny, nx+1), (nz, ny, nx), (nz, ny, nx),
    x fastest.  zu[..., 0] (the inlet face) is unused: the inlet stays at U.
    """
    rng = np.random.Generator(np.random.PCG64(w.seed))
    zu = rng.standard_normal((w.nz, w.ny, w.nx + 1))
    zv = rng.standard_normal((w.nz, w.ny, w.nx))
    zw = rng.standard_normal((w.nz, w.ny, w.nx))
    return zu, zv, zw
