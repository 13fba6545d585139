"""Pins of the oracle's demagnetising tensor and stray-field convolution.

Independent references: exact identities (trace, cube), brute-force quadrature of
the dipole kernel over two cells, Aharoni's closed-form prism demagnetising factor
(J. Appl. Phys. 83, 3432, 1998) and an O(N^2) direct sum.
"""
import numpy as np
import pytest

from oracle import demag


def aharoni_dz(a, b, c):
    """Demagnetising factor along z of the prism [-a,a]x[-b,b]x[-c,c] (Aharoni 1998)."""
    r = np.sqrt(a * a + b * b + c * c)
    ab, bc, ac = np.sqrt(a * a + b * b), np.sqrt(b * b + c * c), np.sqrt(a * a + c * c)
    t = (b * b - c * c) / (2 * b * c) * np.log((r - a) / (r + a))
    t += (a * a - c * c) / (2 * a * c) * np.log((r - b) / (r + b))
    t += b / (2 * c) * np.log((ab + a) / (ab - a))
    t += a / (2 * c) * np.log((ab + b) / (ab - b))
    t += c / (2 * a) * np.log((bc - b) / (bc + b))
    t += c / (2 * b) * np.log((ac - a) / (ac + a))
    t += 2 * np.arctan(a * b / (c * r))
    t += (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
    t += (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r
    t += c / (a * b) * (ac + bc)
    t -= (ab ** 3 + bc ** 3 + ac ** 3) / (3 * a * b * c)
    return t / np.pi


def test_aharoni_formula_itself():
    assert aharoni_dz(1, 1, 1) == pytest.approx(1 / 3, abs=1e-14)
    for a, b, c in [(1, 2, 3), (0.3, 1.7, 0.9)]:
        s = aharoni_dz(a, b, c) + aharoni_dz(b, c, a) + aharoni_dz(c, a, b)
        assert s == pytest.approx(1.0, abs=1e-13)


def test_cube_self_term():
    t = demag.tensor_at(0, 0, 0, (1.0, 1.0, 1.0))
    for c in ("xx", "yy", "zz"):
        assert float(t[c]) == pytest.approx(1 / 3, abs=1e-15)
    for c in ("xy", "xz", "yz"):
        assert abs(float(t[c])) < 1e-15


@pytest.mark.parametrize("h", [(1.0, 0.7, 0.5), (2.0, 1.0, 0.25), (1.0, 1.0, 3.0)])
def test_trace_identities(h):
    t0 = demag.tensor_at(0, 0, 0, h)
    assert float(t0["xx"] + t0["yy"] + t0["zz"]) == pytest.approx(1.0, abs=1e-13)
    rng = np.random.default_rng(3)
    d = rng.integers(-30, 31, size=(200, 3))
    d = d[np.any(d != 0, axis=1)]
    t = demag.tensor_at(d[:, 0], d[:, 1], d[:, 2], h)
    tr = t["xx"] + t["yy"] + t["zz"]
    # the 27-point sum cancels to a few 1e-12 (absolute, FP64) near the 20-cell
    # cut-off, more for elongated cells (up to 8:1 here) than for cubes
    assert np.all(np.abs(tr) <= 2e-11)


def test_parities():
    h = (1.0, 0.8, 0.6)
    d = np.array([[3, 2, 1], [1, 4, 2], [25, 3, 7]])
    t = demag.tensor_at(d[:, 0], d[:, 1], d[:, 2], h)
    tm = demag.tensor_at(-d[:, 0], d[:, 1], d[:, 2], h)
    for c in ("xx", "yy", "zz", "yz"):
        assert np.allclose(t[c], tm[c], rtol=1e-9, atol=1e-15)
    for c in ("xy", "xz"):
        assert np.allclose(t[c], -tm[c], rtol=1e-9, atol=1e-15)


def _quadrature_tensor(d, h, q=24):
    """Cell-averaged dipole kernel by Gauss-Legendre quadrature of the overlap form.

    N_ab(d) = (1/V) int K_ab(s) prod_a tent_a(s_a) ds, K = (delta r^2 - 3 r r)/(4 pi r^5),
    tent_a(s) = max(0, h_a - |s - d_a h_a|); valid when the two cells do not touch.
    """
    xg, wg = np.polynomial.legendre.leggauss(q)
    axes = []
    for a in range(3):
        c = d[a] * h[a]
        pts, wts = [], []
        for lo, hi in ((c - h[a], c), (c, c + h[a])):
            pts.append(0.5 * (hi - lo) * xg + 0.5 * (hi + lo))
            wts.append(0.5 * (hi - lo) * wg)
        p, w = np.concatenate(pts), np.concatenate(wts)
        axes.append((p, w * np.maximum(0.0, h[a] - np.abs(p - c))))
    X, Y, Z = np.meshgrid(axes[0][0], axes[1][0], axes[2][0], indexing="ij")
    W = axes[0][1][:, None, None] * axes[1][1][None, :, None] * axes[2][1][None, None, :]
    r2 = X * X + Y * Y + Z * Z
    k = 1.0 / (4 * np.pi * r2 ** 2.5)
    V = h[0] * h[1] * h[2]
    comp = {"xx": r2 - 3 * X * X, "yy": r2 - 3 * Y * Y, "zz": r2 - 3 * Z * Z,
            "xy": -3 * X * Y, "xz": -3 * X * Z, "yz": -3 * Y * Z}
    return {c: float(np.sum(W * k * v)) / V for c, v in comp.items()}


@pytest.mark.parametrize("d", [(2, 0, 0), (2, 1, 0), (3, -2, 1), (0, 2, 2), (4, 3, -2)])
def test_newell_matches_quadrature(d):
    h = (1.0, 0.75, 0.6)
    ref = _quadrature_tensor(d, h)
    t = demag.tensor_at(*d, h)
    for c in demag.COMPONENTS:
        assert float(t[c]) == pytest.approx(ref[c], rel=1e-9, abs=1e-12), c


def test_far_field_approaches_dipole():
    for r in (8, 16):
        d = (3 * r // 2, r, r // 2)
        t = demag.tensor_at(*d, (1.0, 1.0, 1.0), r_far=10 ** 6)
        p = demag.dipole_tensor(*(np.array(float(v)) for v in d), 1.0)
        for c in demag.COMPONENTS:
            assert abs(float(t[c]) - float(p[c])) < 1e-5 * abs(float(p["xx"])) * (8 / r) ** 2 + 2e-12


def _body_average(n, h):
    nx, ny, nz = n
    idx = np.array([(i, j, k) for k in range(nz) for j in range(ny) for i in range(nx)])
    d = idx[:, None, :] - idx[None, :, :]
    t = demag.tensor_at(d[..., 0], d[..., 1], d[..., 2], h)
    return {c: float(t[c].sum()) / len(idx) for c in t}


@pytest.mark.parametrize("n,h", [((4, 3, 2), (1.0, 0.7, 0.5)), ((3, 3, 3), (1.0, 1.0, 1.0)),
                                 ((6, 2, 1), (0.5, 1.0, 0.25))])
def test_body_average_equals_aharoni(n, h):
    a, b, c = (n[i] * h[i] / 2 for i in range(3))
    avg = _body_average(n, h)
    assert avg["zz"] == pytest.approx(aharoni_dz(a, b, c), abs=1e-12)
    assert avg["xx"] == pytest.approx(aharoni_dz(b, c, a), abs=1e-12)
    assert avg["yy"] == pytest.approx(aharoni_dz(c, a, b), abs=1e-12)
    for comp in ("xy", "xz", "yz"):
        assert abs(avg[comp]) < 1e-13


def _direct_sum(m, h):
    nz, ny, nx = m.shape[1:]
    out = np.zeros_like(m)
    pair = {(0, 0): "xx", (1, 1): "yy", (2, 2): "zz", (0, 1): "xy", (1, 0): "xy",
            (0, 2): "xz", (2, 0): "xz", (1, 2): "yz", (2, 1): "yz"}
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for kk in range(nz):
                    for jj in range(ny):
                        for ii in range(nx):
                            t = demag.tensor_at(i - ii, j - jj, k - kk, h)
                            for a in range(3):
                                for b in range(3):
                                    out[a, k, j, i] -= float(t[pair[(a, b)]]) * m[b, kk, jj, ii]
    return out


@pytest.mark.parametrize("shape", [(2, 4, 3), (1, 5, 1), (2, 2, 2), (1, 1, 1), (3, 1, 2)])
def test_fft_convolution_equals_direct_sum(shape):
    rng = np.random.default_rng(4)
    h = (1.0, 0.9, 0.7)
    m = rng.normal(size=(3,) + shape)
    spec = demag.kernel_spectra(shape, h)
    assert np.allclose(demag.stray_field(m, spec), _direct_sum(m, h), rtol=0, atol=1e-13)


def test_far_field_branch_in_convolution():
    # a strip longer than the cut-off exercises the dipole branch inside the FFT path
    shape = (1, 1, demag.R_FAR + 6)
    rng = np.random.default_rng(5)
    h = (1.0, 1.0, 1.0)
    m = rng.normal(size=(3,) + shape)
    spec = demag.kernel_spectra(shape, h)
    assert np.allclose(demag.stray_field(m, spec), _direct_sum(m, h), rtol=0, atol=1e-13)


def test_stray_operator_is_symmetric():
    rng = np.random.default_rng(6)
    shape = (3, 4, 5)
    spec = demag.kernel_spectra(shape, (1.0, 1.0, 0.5))
    u, v = rng.normal(size=(2, 3) + shape)
    assert np.sum(v * demag.stray_field(u, spec)) == pytest.approx(
        np.sum(u * demag.stray_field(v, spec)), rel=1e-12)


@pytest.mark.parametrize("h,r", [((1.0, 1.0, 1.0), 20), ((4.0, 4.0, 2.0), 12)], ids=["cubic", "flat"])
def test_oracle_newell_rounding_within_kappa(h, r):
    """The FP64 Newell sums lose digits to cancellation; measured against the same
    formulas in extended precision, the oracle's error at every offset of the octant
    up to r cells stays within KAPPA u S(d), S(d) the sum of the magnitudes of the 27
    terms.  This fixes the per-entry rounding bound the GPU parity bars are built on."""
    import newell_bounds as nb
    rr = np.arange(0, r + 1)
    IZ, IY, IX = np.meshgrid(rr, rr, rr, indexing="ij")
    n64 = demag.tensor_at(IX, IY, IZ, h, r_far=10 ** 9)
    nld = nb.long_double_newell(IX, IY, IZ, h)
    s = max(h)
    e = [hh / s for hh in h]
    P = [IX * e[0], IY * e[1], IZ * e[2]]
    worst = 0.0
    for c, (fn, o) in nb._SPEC.items():
        F = demag.newell_f if fn == "f" else demag.newell_g
        S = nb._stencil_abs(F, P[o[0]], P[o[1]], P[o[2]], e[o[0]], e[o[1]], e[o[2]])
        err = np.abs(n64[c] - nld[c].astype(np.float64))
        worst = max(worst, float((err / (nb.U * S + 1e-300)).max()))
        assert np.all(err <= nb.KAPPA * nb.U * S + 4 * nb.U * np.abs(n64[c])), c
    print(f"max FP64 Newell error / (u S): {worst:.2f}")
