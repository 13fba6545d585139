"""Manufactured exact solutions with forcing (paper §5.1), oracle side.

1-D (§5.1): m_e = (cos X sin t, sin X sin t, cos t), X = x^2 (1 - x)^2 on [0, 1].
3-D (§5.1): the same with phi = X Y Z, Y = y^2(1-y)^2, Z = z^2(1-z)^2 on [0, 1]^3.
2-D (not in the paper; used for the 32 x 32 exchange-only film): phi = X Y.
The forcing makes m_e solve m_t = -m x h - alpha m x (m x h) + f_e with h = eps Lap m:
  f_e = dm_e/dt + eps m_e x Lap m_e + alpha eps m_e x (m_e x Lap m_e)
(the paper prints it with eps = 1).  All derivatives are in closed form; points
are cell centres x_i = (i + 1/2)/n.
"""
import numpy as np


def _p(s):
    """s^2 (1-s)^2 and its first two derivatives."""
    return s * s * (1 - s) ** 2, 2 * s * (1 - s) * (1 - 2 * s), 2 - 12 * s + 12 * s * s


def centres(n):
    return (np.arange(n) + 0.5) / n


def _phi(shape, dim):
    """phi, |grad phi|^2 and Lap phi at cell centres for the 1/2/3-D solution."""
    nz, ny, nx = shape
    X, X1, X2 = (a[None, None, :] for a in _p(centres(nx)))
    if dim == 1:
        phi, grad2, lap = X, X1 ** 2, X2
    elif dim == 2:
        Y, Y1, Y2 = (a[None, :, None] for a in _p(centres(ny)))
        phi = X * Y
        grad2 = (X1 * Y) ** 2 + (X * Y1) ** 2
        lap = X2 * Y + X * Y2
    else:
        Y, Y1, Y2 = (a[None, :, None] for a in _p(centres(ny)))
        Z, Z1, Z2 = (a[:, None, None] for a in _p(centres(nz)))
        phi = X * Y * Z
        grad2 = (X1 * Y * Z) ** 2 + (X * Y1 * Z) ** 2 + (X * Y * Z1) ** 2
        lap = X2 * Y * Z + X * Y2 * Z + X * Y * Z2
    return tuple(np.broadcast_to(a, shape).copy() for a in (phi, grad2, lap))


def exact(shape, t, dim):
    phi, _, _ = _phi(shape, dim)
    s, c = np.sin(t), np.cos(t)
    return np.stack([np.cos(phi) * s, np.sin(phi) * s, np.full(phi.shape, c)])


def lap_exact(shape, t, dim):
    """Continuum Laplacian of m_e: Lap cos(phi) = -sin(phi) Lap phi - cos(phi)|grad phi|^2 etc."""
    phi, g2, lp = _phi(shape, dim)
    s = np.sin(t)
    lc = -np.sin(phi) * lp - np.cos(phi) * g2
    ls = np.cos(phi) * lp - np.sin(phi) * g2
    return np.stack([lc * s, ls * s, np.zeros(phi.shape)])


def dt_exact(shape, t, dim):
    phi, _, _ = _phi(shape, dim)
    c = np.cos(t)
    return np.stack([np.cos(phi) * c, np.sin(phi) * c, np.full(phi.shape, -np.sin(t))])


def forcing(shape, t, dim, eps, alpha):
    me = exact(shape, t, dim)
    h = eps * lap_exact(shape, t, dim)
    mxh = np.cross(me, h, axis=0)
    return dt_exact(shape, t, dim) + mxh + alpha * np.cross(me, mxh, axis=0)
