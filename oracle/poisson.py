"""Pressure Poisson equation of the fractional step (oracle).

Sec. II.B: the provisional velocity is projected onto a divergence-free field
after solving the Poisson equation that enforces mass conservation.  The
discrete operator is L = D G (the 7-point Laplacian): periodic in y and z,
homogeneous Neumann in x (the boundary faces are not corrected), i.e.
phi_{-1} = phi_0 and phi_nx = phi_{nx-1}.

Solver (AFiD-type, Sec. II.B cites it): real DFT in y, complex DFT in z (library
FFTs), then for each transverse mode (m, l) the tridiagonal system in x

    phi_{i-1} + (-2 + h^2 (lam_y(m) + lam_z(l))) phi_i + phi_{i+1} = h^2 r_i,
    lam_y(m) = -(4/h^2) sin^2(pi m / ny),  lam_z(l) = -(4/h^2) sin^2(pi l / nz),

with the Neumann rows using -1 in place of -2, solved by the Thomas algorithm.
Reading for the singular (0, 0) mode: its first row is replaced by phi_0 = 0
and the x-mean of the result is removed afterwards (pressure gauge).
"""
from __future__ import annotations

import numpy as np


def eigen_shift(n: int, h: float, half: bool = False):
    """lam(m) = -(4/h^2) sin^2(pi m / n) for m = 0..n-1 (or 0..n/2 if ``half``)."""
    m = np.arange(n // 2 + 1 if half else n)
    return -(4.0 / (h * h)) * np.sin(np.pi * m / n) ** 2


def _thomas(a, b, c, d):
    """Plain Thomas algorithm, vectorised over the leading axis.

    a, b, c: (nm, n) real sub-, main and super-diagonals (a[:, 0], c[:, -1]
    unused); d: (nm, n) complex.  Returns x (nm, n).
    """
    nm, n = d.shape
    cp = np.empty((nm, n))
    dp = np.empty((nm, n), dtype=d.dtype)
    cp[:, 0] = c[:, 0] / b[:, 0]
    dp[:, 0] = d[:, 0] / b[:, 0]
    for i in range(1, n):
        den = b[:, i] - a[:, i] * cp[:, i - 1]
        cp[:, i] = c[:, i] / den
        dp[:, i] = (d[:, i] - a[:, i] * dp[:, i - 1]) / den
    x = np.empty_like(dp)
    x[:, n - 1] = dp[:, n - 1]
    for i in range(n - 2, -1, -1):
        x[:, i] = dp[:, i] - cp[:, i] * x[:, i + 1]
    return x


def solve_poisson(r, h: float):
    """Solve L phi = r.  r: (nz, ny, nx) real, compatible (sum r = 0).

    Returns phi (nz, ny, nx) with the gauge described in the module docstring.
    """
    nz, ny, nx = r.shape
    rh = np.fft.fft(np.fft.rfft(r, axis=1), axis=0)        # (nz, ny/2+1, nx)
    my = ny // 2 + 1
    lam = (eigen_shift(nz, h)[:, None] + eigen_shift(ny, h, half=True)[None, :])
    shift = (h * h) * lam.reshape(-1)                       # (nz*my,)
    d = (h * h) * rh.reshape(nz * my, nx)
    nm = nz * my
    a = np.ones((nm, nx))
    c = np.ones((nm, nx))
    b = np.empty((nm, nx))
    b[:] = -2.0 + shift[:, None]
    b[:, 0] = -1.0 + shift
    b[:, nx - 1] = -1.0 + shift
    a[:, 0] = 0.0
    c[:, nx - 1] = 0.0
    # singular (0, 0) mode: row 0 replaced by phi_0 = 0
    b[0, 0] = 1.0
    c[0, 0] = 0.0
    d[0, 0] = 0.0
    x = _thomas(a, b, c, d)
    x[0, :] -= np.mean(x[0, :])
    ph = x.reshape(nz, my, nx)
    return np.fft.irfft(np.fft.ifft(ph, axis=0), n=ny, axis=1)


def apply_laplacian(phi, h: float):
    """L phi with Neumann x ends and periodic y, z (for residual checks)."""
    nz, ny, nx = phi.shape
    g = np.concatenate([phi[..., :1], phi, phi[..., -1:]], axis=2)
    return ((g[..., 2:] + g[..., :-2] - 2.0 * phi)
            + (np.roll(phi, -1, 1) + np.roll(phi, 1, 1) - 2.0 * phi)
            + (np.roll(phi, -1, 0) + np.roll(phi, 1, 0) - 2.0 * phi)) / (h * h)
