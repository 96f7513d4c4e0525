"""Pins of the pressure-Poisson solve (oracle/poisson.py).

The discrete operator L (7-point, Neumann in x, periodic in y and z) has the
closed-form eigenvectors cos(pi m (i+1/2)/nx) exp(2 pi i (j n/ny + k l/nz))
with eigenvalues -(4/h^2)[sin^2(pi m/(2 nx)) + sin^2(pi n/ny) + sin^2(pi l/nz)];
any exact solver of L reproduces them.  A dense solve of L built entry by
entry from the stencil (with the zero-mean gauge) is a second, independent
solver at tiny sizes.
"""
import numpy as np
import pytest

from oracle import poisson

RNG = np.random.default_rng(11)


@pytest.mark.parametrize("shape", [(8, 6, 10), (12, 16, 8), (6, 6, 5)])
def test_eigenvectors(shape):
    nz, ny, nx = shape
    h = 0.37
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for (m, n, l) in [(1, 0, 0), (0, 1, 0), (0, 0, 2), (3, 2, 1), (nx - 1, ny // 2, nz // 2)]:
        phase = 2 * np.pi * (j * n / ny + k * l / nz)
        phi = np.cos(np.pi * m * (i + 0.5) / nx) * (np.cos(phase) + 0.3 * np.sin(phase))
        lam = -(4 / h ** 2) * (np.sin(np.pi * m / (2 * nx)) ** 2 + np.sin(np.pi * n / ny) ** 2
                               + np.sin(np.pi * l / nz) ** 2)
        sol = poisson.solve_poisson(lam * phi, h)
        assert np.max(np.abs(sol - phi)) < 1e-13
        assert np.max(np.abs(poisson.apply_laplacian(phi, h) - lam * phi)) < 1e-12 * abs(lam)


def _dense_L(nz, ny, nx, h):
    N = nx * ny * nz
    A = np.zeros((N, N))
    idx = lambda i, j, k: i + nx * (j + ny * k)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                r = idx(i, j, k)
                for (di, dj, dk) in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]:
                    ii, jj, kk = i + di, (j + dj) % ny, (k + dk) % nz
                    if ii < 0 or ii >= nx:
                        continue          # Neumann: the flux through the x ends is zero
                    A[r, idx(ii, jj, kk)] += 1.0 / h ** 2
                    A[r, r] -= 1.0 / h ** 2
    return A


@pytest.mark.parametrize("shape", [(4, 4, 4), (4, 4, 6), (6, 4, 3)])
def test_dense_solve(shape):
    nz, ny, nx = shape
    h = 0.5
    A = _dense_L(nz, ny, nx, h)
    r = RNG.standard_normal(shape)
    r -= r.mean()
    N = A.shape[0]
    # gauge: zero mean, imposed with a Lagrange multiplier
    B = np.zeros((N + 1, N + 1))
    B[:N, :N] = A
    B[N, :N] = 1.0
    B[:N, N] = 1.0
    x = np.linalg.solve(B, np.concatenate([r.reshape(-1), [0.0]]))[:N].reshape(shape)
    sol = poisson.solve_poisson(r, h)
    # the oracle removes the x-mean of the (0,0) mode, i.e. the global mean
    assert np.max(np.abs(sol - x)) < 1e-13 * max(1.0, np.max(np.abs(x)))


def test_random_residual():
    nz, ny, nx = 16, 12, 24
    h = 0.1
    r = RNG.standard_normal((nz, ny, nx))
    r -= r.mean()
    phi = poisson.solve_poisson(r, h)
    res = poisson.apply_laplacian(phi, h) - r
    assert np.max(np.abs(res)) < 1e-12 * np.max(np.abs(r))
    assert abs(phi.mean()) < 1e-14
