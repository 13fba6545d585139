"""Neumann Laplacian and the heat-type solve of the projection schemes (oracle).

Paper: §2, eq. (boundary-large) gives the homogeneous Neumann condition; §3.1 and
§3.2 (Step 1) define g = (I - eps dt Lap_h)^{-1}(m + dt f) and Step 2 solves
(I - alpha eps dt Lap_h) m*** = m** + alpha dt f**.  The paper does not state the
grid.  Reading: cell-centred cells x_i = (i + 1/2) h, the 7-point Lap_h with mirror
ghosts u_{-1} = u_0, u_n = u_{n-1}; an axis with a single cell contributes nothing.

``laplacian`` is that stencil written out.  ``heat_solve`` applies the exact
inverse of (I - c Lap_h) through its eigen-decomposition: the mirror-ghost
Laplacian is diagonalised by the type-II DCT with eigenvalues
-(4/h^2) sin^2(pi k / (2n)) per axis (SciPy's orthonormal DCT is the library step).
"""
import numpy as np
from scipy import fft as sfft

AXES = ((2, 0), (1, 1), (0, 2))  # (array axis, index into h) for x, y, z


def laplacian(u, h):
    """Lap_h u for a scalar field u of shape (nz, ny, nx); h = (dx, dy, dz)."""
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    for ax, hi in AXES:
        n = u.shape[ax]
        if n == 1:
            continue
        lo = np.take(u, [0], axis=ax)
        hi_edge = np.take(u, [n - 1], axis=ax)
        ext = np.concatenate([lo, u, hi_edge], axis=ax)  # mirror ghosts
        left = np.take(ext, np.arange(0, n), axis=ax)
        right = np.take(ext, np.arange(2, n + 2), axis=ax)
        out += (left - 2.0 * u + right) / (h[hi] * h[hi])
    return out


def laplacian_eigs(n, h):
    """1-D eigenvalues mu_k = (4/h^2) sin^2(pi k / (2n)) of -Lap_h (mirror ghosts)."""
    k = np.arange(n, dtype=np.float64)
    return 4.0 / (h * h) * np.sin(np.pi * k / (2.0 * n)) ** 2


def _symbol(shape, h):
    nz, ny, nx = shape
    mx = laplacian_eigs(nx, h[0])
    my = laplacian_eigs(ny, h[1])
    mz = laplacian_eigs(nz, h[2])
    return mz[:, None, None] + my[None, :, None] + mx[None, None, :]


def _active(shape):
    return [ax for ax, _ in AXES if shape[ax] > 1]


def heat_solve(r, c, h):
    """Solve (I - c Lap_h) g = r for a scalar field r (Neumann, exact inverse)."""
    r = np.asarray(r, dtype=np.float64)
    axes = _active(r.shape)
    if not axes:
        return r.copy()
    rh = sfft.dctn(r, type=2, norm="ortho", axes=axes)
    rh /= 1.0 + c * _symbol(r.shape, h)
    return sfft.idctn(rh, type=2, norm="ortho", axes=axes)


def heat_solve_vec(v, c, h):
    """Componentwise heat solve of a (3, nz, ny, nx) field."""
    return np.stack([heat_solve(v[i], c, h) for i in range(v.shape[0])])


def laplacian_vec(v, h):
    return np.stack([laplacian(v[i], h) for i in range(v.shape[0])])
