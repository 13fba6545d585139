"""Pins of the oracle's Neumann Laplacian and heat-type solve (paper §2 BC, §3 Step 1/2 solves)."""
import numpy as np
import pytest

from oracle import operators


def dense_lap_1d(n, h):
    """Textbook tridiagonal Neumann (mirror-ghost) second difference."""
    A = np.zeros((n, n))
    for i in range(n):
        if i > 0:
            A[i, i - 1] += 1.0
            A[i, i] -= 1.0
        if i < n - 1:
            A[i, i + 1] += 1.0
            A[i, i] -= 1.0
    return A / (h * h)


def dense_lap(shape, h):
    """Kronecker-sum assembly of the 3-D operator for arrays (nz, ny, nx), x fastest."""
    nz, ny, nx = shape
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    Lx, Ly, Lz = dense_lap_1d(nx, h[0]), dense_lap_1d(ny, h[1]), dense_lap_1d(nz, h[2])
    return np.kron(np.kron(Iz, Iy), Lx) + np.kron(np.kron(Iz, Ly), Ix) + np.kron(np.kron(Lz, Iy), Ix)


SHAPES = [(2, 3, 4), (1, 1, 5), (1, 1, 1), (1, 3, 2), (3, 1, 1), (4, 4, 4)]


@pytest.mark.parametrize("shape", SHAPES)
def test_laplacian_equals_assembled_matrix(shape):
    rng = np.random.default_rng(1)
    h = (0.3, 0.7, 1.3)
    u = rng.normal(size=shape)
    ref = (dense_lap(shape, h) @ u.ravel()).reshape(shape)
    assert np.allclose(operators.laplacian(u, h), ref, rtol=0, atol=1e-12)


def test_laplacian_quadratic_interior():
    # second differences of x^2 are exactly 2 away from the mirror boundary
    n, h = 9, 0.25
    x = (np.arange(n) + 0.5) * h
    u = np.broadcast_to(x ** 2, (1, 1, n)).copy()
    lap = operators.laplacian(u, (h, 1.0, 1.0))[0, 0]
    assert np.allclose(lap[1:-1], 2.0, atol=1e-12)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("c", [0.0, 0.37, 12.5])
def test_heat_solve_equals_dense_solve(shape, c):
    rng = np.random.default_rng(2)
    h = (0.3, 0.7, 1.3)
    r = rng.normal(size=shape)
    A = np.eye(r.size) - c * dense_lap(shape, h)
    ref = np.linalg.solve(A, r.ravel()).reshape(shape)
    assert np.allclose(operators.heat_solve(r, c, h), ref, rtol=0, atol=1e-13)


def test_heat_solve_preserves_constants():
    r = np.full((3, 4, 5), 2.5)
    assert np.allclose(operators.heat_solve(r, 3.0, (1.0, 2.0, 0.5)), 2.5, atol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 5, 8])
def test_cosine_modes_are_eigenvectors(n):
    h = 0.4
    A = dense_lap_1d(n, h)
    mu = operators.laplacian_eigs(n, h)
    i = np.arange(n)
    for k in range(n):
        v = np.cos(np.pi * k * (i + 0.5) / n)
        assert np.allclose(A @ v, -mu[k] * v, atol=1e-12)
