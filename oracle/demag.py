"""Demagnetising (stray) field: Newell cell-averaged tensor and its convolution (oracle).

Paper: the stray field h_s enters the effective field of §2 and every f of §3.1 /
§3.2; the abstract and conclusions say it is evaluated by FFT, but the paper gives
no discretisation.  Reading taken (one spec shared with the GPU library, not code):

* h_s(i) = - sum_j N(r_i - r_j) m(j) over all cells j (self term included), with
  the open-boundary (non-periodic) convolution done by 2x zero padding.
* N is the cell-averaged tensor of Newell, Williams & Dunlop (JGR 98, 1993):
  N_xx from the function f, N_xy from the function g, both through the 27-point
  second-difference stencil with weights 8, -4, 2, -1, divided by 4 pi V; the
  other components by permuting the axes.
* For offsets whose largest cell index |d| exceeds R_FAR = 20 the point-dipole
  form (V / 4 pi)(delta_ab r^2 - 3 r_a r_b) / r^5 replaces the 27-point sum.  The
  sum loses digits to cancellation as the offset grows while the dipole form
  gains them; for cubic cells the two errors cross near 20 cells at about 1e-12
  (absolute, FP64), which fixes the cut-off.
* Lengths are divided by the largest cell edge before evaluation (N is scale
  free).
"""
import numpy as np
from scipy import fft as sfft

R_FAR = 20
WORKERS = 8  # threads handed to SciPy's FFT (the only parallel step)


def _safe_div(a, b):
    out = np.zeros(np.broadcast(a, b).shape)
    np.divide(a, b, out=out, where=(b != 0))
    return out


def newell_f(x, y, z):
    """Newell's f(x, y, z) (N_xx generating function)."""
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    t = (2.0 * x2 - y2 - z2) * R / 6.0
    t = t + 0.5 * y * (z2 - x2) * np.arcsinh(_safe_div(y, np.sqrt(x2 + z2)))
    t = t + 0.5 * z * (y2 - x2) * np.arcsinh(_safe_div(z, np.sqrt(x2 + y2)))
    t = t - x * y * z * np.arctan(_safe_div(y * z, x * R))
    return t


def newell_g(x, y, z):
    """Newell's g(x, y, z) (N_xy generating function)."""
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    t = -x * y * R / 3.0
    t = t + x * y * z * np.arcsinh(_safe_div(z, np.sqrt(x2 + y2)))
    t = t + y / 6.0 * (3.0 * z2 - y2) * np.arcsinh(_safe_div(x, np.sqrt(y2 + z2)))
    t = t + x / 6.0 * (3.0 * z2 - x2) * np.arcsinh(_safe_div(y, np.sqrt(x2 + z2)))
    t = t - z2 * z / 6.0 * np.arctan(_safe_div(x * y, z * R))
    t = t - z * y2 / 2.0 * np.arctan(_safe_div(x * z, y * R))
    t = t - z * x2 / 2.0 * np.arctan(_safe_div(y * z, x * R))
    return t


_W = {-1: -1.0, 0: 2.0, 1: -1.0}


def _stencil(F, X, Y, Z, a, b, c):
    acc = np.zeros(np.broadcast(X, Y, Z).shape)
    for i in (-1, 0, 1):
        for j in (-1, 0, 1):
            for k in (-1, 0, 1):
                acc += _W[i] * _W[j] * _W[k] * F(X + i * a, Y + j * b, Z + k * c)
    return acc / (4.0 * np.pi * a * b * c)


COMPONENTS = ("xx", "yy", "zz", "xy", "xz", "yz")


def newell_tensor(X, Y, Z, dx, dy, dz):
    """All six Newell components at physical offsets (X, Y, Z) for a dx x dy x dz cell."""
    return {
        "xx": _stencil(newell_f, X, Y, Z, dx, dy, dz),
        "yy": _stencil(newell_f, Y, X, Z, dy, dx, dz),
        "zz": _stencil(newell_f, Z, Y, X, dz, dy, dx),
        "xy": _stencil(newell_g, X, Y, Z, dx, dy, dz),
        "xz": _stencil(newell_g, X, Z, Y, dx, dz, dy),
        "yz": _stencil(newell_g, Y, Z, X, dy, dz, dx),
    }


def dipole_tensor(X, Y, Z, V):
    """Point-dipole demagnetising tensor (V / 4 pi)(delta_ab r^2 - 3 r_a r_b) / r^5."""
    r2 = X * X + Y * Y + Z * Z
    s = V / (4.0 * np.pi) / (r2 * r2 * np.sqrt(r2))
    return {
        "xx": s * (r2 - 3.0 * X * X),
        "yy": s * (r2 - 3.0 * Y * Y),
        "zz": s * (r2 - 3.0 * Z * Z),
        "xy": s * (-3.0 * X * Y),
        "xz": s * (-3.0 * X * Z),
        "yz": s * (-3.0 * Y * Z),
    }


def tensor_at(ix, iy, iz, h, r_far=R_FAR):
    """N_ab at integer cell offsets (arrays broadcastable), following the spec above."""
    ix, iy, iz = np.broadcast_arrays(*(np.asarray(v, dtype=np.int64) for v in (ix, iy, iz)))
    s = max(h)
    dx, dy, dz = (hh / s for hh in h)
    X, Y, Z = ix * dx, iy * dy, iz * dz
    far = np.maximum(np.maximum(np.abs(ix), np.abs(iy)), np.abs(iz)) > r_far
    out = {c: np.zeros(ix.shape) for c in COMPONENTS}
    near = ~far
    if near.any():
        tn = newell_tensor(X[near], Y[near], Z[near], dx, dy, dz)
        for c in COMPONENTS:
            out[c][near] = tn[c]
    if far.any():
        tf = dipole_tensor(X[far], Y[far], Z[far], dx * dy * dz)
        for c in COMPONENTS:
            out[c][far] = tf[c]
    return out


def padded_shape(shape):
    """Zero-padded FFT grid: 2n along every axis with n > 1, 1 otherwise."""
    return tuple(2 * n if n > 1 else 1 for n in shape)


def kernel_spectra(shape, h):
    """FFT of N_ab laid out on the zero-padded grid (offset d stored at d mod P).

    Returns (P, spectra) with spectra[c] = rfftn of the padded real kernel.
    """
    P = padded_shape(shape)
    offs = []
    for n, p in zip(shape, P):
        k = np.arange(p)
        d = np.where(k < n, k, k - p)
        valid = np.abs(d) <= n - 1
        offs.append((d, valid))
    (dz, vz), (dy, vy), (dx_, vx) = offs
    IZ, IY, IX = np.meshgrid(dz, dy, dx_, indexing="ij")
    valid = vz[:, None, None] & vy[None, :, None] & vx[None, None, :]
    comps = tensor_at(IX, IY, IZ, h)
    spectra = {}
    for c in COMPONENTS:
        arr = np.where(valid, comps[c], 0.0)
        spectra[c] = sfft.rfftn(arr, workers=WORKERS)
    return P, spectra


_PAIR = {(0, 0): "xx", (1, 1): "yy", (2, 2): "zz", (0, 1): "xy", (1, 0): "xy",
         (0, 2): "xz", (2, 0): "xz", (1, 2): "yz", (2, 1): "yz"}


def stray_field(m, spec):
    """h_s = -N (*) m for a (3, nz, ny, nx) field; ``spec`` from kernel_spectra."""
    P, spectra = spec
    shape = m.shape[1:]
    mh = [sfft.rfftn(m[b], s=P, workers=WORKERS) for b in range(3)]
    out = np.empty(m.shape)
    for a in range(3):
        acc = sum(spectra[_PAIR[(a, b)]] * mh[b] for b in range(3))
        full = sfft.irfftn(acc, s=P, workers=WORKERS)
        out[a] = -full[: shape[0], : shape[1], : shape[2]]
    return out
