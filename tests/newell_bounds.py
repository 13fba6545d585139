"""Rounding bounds of the FP64 demagnetising tensor and of FP64 FFT convolutions
(test helpers; no part of the method is computed here).

The Newell tensor of an offset d is a 27-point second difference of the
generating functions f or g, divided by 4 pi V.  The terms grow like |d|^2 while
the result falls like |d|^-3, so the sum cancels: an FP64 evaluation carries an
absolute error of about u S(d), u = 2^-53, where

    S(d) = sum over the 27 points k of |w_k F(x_k)| / (4 pi V)

is the sum of the magnitudes of the terms.  `rounding_scale_near` computes S(d)
over the Newell offsets (the point-dipole offsets beyond 20 cells do not cancel:
a few u |N(d)|);
`long_double_newell` evaluates the same formulas in x87 extended precision
(64-bit significand) to measure how many u S(d) an FP64 evaluation actually
loses.
"""
import numpy as np

from oracle import demag

U = 2.0 ** -53
# bound on |N_fp64(d) - N_exact(d)| / (u S(d)) of one FP64 evaluation (a libm
# with errors of an ulp or two); the oracle's measured worst case is about 10.5
# (test_oracle_newell_rounding_within_kappa pins it below KAPPA)
KAPPA = 16.0
# l2 rounding constant per power-of-two FFT (times u log2 P), see fft_conv_bound
FFT_C = 10.0

_W = {-1: -1.0, 0: 2.0, 1: -1.0}
# generating function, argument order and edge order of each component
_SPEC = {"xx": ("f", (0, 1, 2)), "yy": ("f", (1, 0, 2)), "zz": ("f", (2, 1, 0)),
         "xy": ("g", (0, 1, 2)), "xz": ("g", (0, 2, 1)), "yz": ("g", (1, 2, 0))}


def _stencil_abs(F, X, Y, Z, a, b, c):
    acc = np.zeros(np.broadcast(X, Y, Z).shape)
    for i in (-1, 0, 1):
        for j in (-1, 0, 1):
            for k in (-1, 0, 1):
                acc += np.abs(_W[i] * _W[j] * _W[k] * F(X + i * a, Y + j * b, Z + k * c))
    return acc / (4.0 * np.pi * a * b * c)


def _offsets_near(shape, r_far=demag.R_FAR):
    """Integer offsets (ix, iy, iz) of the grid within the Newell region."""
    nz, ny, nx = shape
    rx, ry, rz = (np.arange(-min(n - 1, r_far), min(n - 1, r_far) + 1) for n in (nx, ny, nz))
    IZ, IY, IX = np.meshgrid(rz, ry, rx, indexing="ij")
    return IX, IY, IZ


def rounding_scale_near(shape, h):
    """((IX, IY, IZ), {comp: S}) over the Newell-region offsets of the grid."""
    s = max(h)
    e = [hh / s for hh in h]
    IX, IY, IZ = _offsets_near(shape)
    P = [IX * e[0], IY * e[1], IZ * e[2]]
    out = {}
    for c, (fn, o) in _SPEC.items():
        F = demag.newell_f if fn == "f" else demag.newell_g
        out[c] = _stencil_abs(F, P[o[0]], P[o[1]], P[o[2]], e[o[0]], e[o[1]], e[o[2]])
    return (IX, IY, IZ), out


# ---- the same formulas in extended precision (for measuring FP64 rounding only)
_LD = np.longdouble


def _sdiv(a, b):
    out = np.zeros(np.broadcast(a, b).shape, dtype=_LD)
    np.divide(a, b, out=out, where=(b != 0))
    return out


def _f_ld(x, y, z):
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    t = (2 * x2 - y2 - z2) * R / 6
    t = t + y * (z2 - x2) * np.arcsinh(_sdiv(y, np.sqrt(x2 + z2))) / 2
    t = t + z * (y2 - x2) * np.arcsinh(_sdiv(z, np.sqrt(x2 + y2))) / 2
    return t - x * y * z * np.arctan(_sdiv(y * z, x * R))


def _g_ld(x, y, z):
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    t = -x * y * R / 3
    t = t + x * y * z * np.arcsinh(_sdiv(z, np.sqrt(x2 + y2)))
    t = t + y / 6 * (3 * z2 - y2) * np.arcsinh(_sdiv(x, np.sqrt(y2 + z2)))
    t = t + x / 6 * (3 * z2 - x2) * np.arcsinh(_sdiv(y, np.sqrt(x2 + z2)))
    t = t - z2 * z / 6 * np.arctan(_sdiv(x * y, z * R))
    t = t - z * y2 / 2 * np.arctan(_sdiv(x * z, y * R))
    return t - z * x2 / 2 * np.arctan(_sdiv(y * z, x * R))


def long_double_newell(IX, IY, IZ, h):
    """{comp: N_ab} at the given integer offsets, 27-point sums in long double."""
    s = max(h)
    e = [_LD(hh) / _LD(s) for hh in h]
    P = [IX.astype(_LD) * e[0], IY.astype(_LD) * e[1], IZ.astype(_LD) * e[2]]
    out = {}
    for c, (fn, o) in _SPEC.items():
        F = _f_ld if fn == "f" else _g_ld
        X, Y, Z, a, b, cc = P[o[0]], P[o[1]], P[o[2]], e[o[0]], e[o[1]], e[o[2]]
        acc = np.zeros(X.shape, dtype=_LD)
        for i in (-1, 0, 1):
            for j in (-1, 0, 1):
                for k in (-1, 0, 1):
                    acc += _LD(_W[i] * _W[j] * _W[k]) * F(X + i * a, Y + j * b, Z + k * cc)
        out[c] = acc / (_LD(4) * _LD(np.pi) * a * b * cc)
    return out


def padded_tensor(shape, h):
    """{comp: real array (Pz, Py, Px)} of the oracle tensor on the zero-padded grid,
    offset d at d mod P (the layout that demag.kernel_spectra transforms)."""
    P = demag.padded_shape(shape)
    offs = []
    for n, p in zip(shape, P):
        k = np.arange(p)
        d = np.where(k < n, k, k - p)
        offs.append((d, np.abs(d) <= n - 1))
    (dz, vz), (dy, vy), (dx, vx) = offs
    IZ, IY, IX = np.meshgrid(dz, dy, dx, indexing="ij")
    valid = vz[:, None, None] & vy[None, :, None] & vx[None, None, :]
    comps = demag.tensor_at(IX, IY, IZ, h)
    return {c: np.where(valid, comps[c], 0.0) for c in demag.COMPONENTS}, (IX, IY, IZ)


def entry_bound(shape, h, No, offsets):
    """Per-entry bound on |N_a(d) - N_b(d)| for two independent FP64 evaluations of the
    tensor: 2 KAPPA u S(d) in the Newell region, 8 u |N(d)| for the dipole offsets."""
    IX, IY, IZ = offsets
    far = np.maximum(np.maximum(np.abs(IX), np.abs(IY)), np.abs(IZ)) > demag.R_FAR
    (nx_, ny_, nz_), S = rounding_scale_near(shape, h)
    out = {}
    for c in demag.COMPONENTS:
        b = 8.0 * U * np.abs(No[c])
        near = np.zeros_like(b)
        # scatter S into the padded layout: offset d sits at d mod P
        P = demag.padded_shape(shape)
        iz = np.mod(nz_, P[0]) if P[0] > 1 else np.zeros_like(nz_)
        iy = np.mod(ny_, P[1]) if P[1] > 1 else np.zeros_like(ny_)
        ix = np.mod(nx_, P[2]) if P[2] > 1 else np.zeros_like(nx_)
        near[iz, iy, ix] = 2.0 * KAPPA * U * S[c]
        out[c] = np.where(far, b, near + b)
    return out


def fft_conv_bound(shape, spectra, m):
    """Bound on the max-abs difference of two FP64 zero-padded FFT convolutions of the
    same tensor and field: 6 FFT_C u log2(P) max |N^| ||m||_2.  A power-of-two FFT of
    length P with accurate twiddles is within C u log2(P) of the exact transform in
    the l2 norm, relative (the classical bound, C about 6 for radix 2 with correctly
    rounded twiddles; Higham, Accuracy and Stability of Numerical Algorithms, ch. 24);
    each side does three such transforms (the tensor, the field, the inverse), the
    product by the tensor spectrum scales by at most max |N^|, and the l2 norm of the
    field error bounds its max norm.  FFT_C is taken as 10: the library's radix-8
    passes with packed real pairs (two real rows per complex transform) reach up to
    about 7 on the test shapes."""
    P, sp = spectra
    ptot = int(np.prod(P))
    nmax = max(float(np.abs(v).max()) for v in sp.values())
    return 6.0 * FFT_C * U * max(1.0, np.log2(ptot)) * nmax * float(np.linalg.norm(m))
