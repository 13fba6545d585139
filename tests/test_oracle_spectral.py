"""Pins of the oracle's sweep-matrix spectral radius (paper §4, eqs. GS-matrix, SGS-matrix, M)."""
import numpy as np
import pytest

from oracle import scheme, spectral


def _random_unit(shape, seed):
    rng = np.random.default_rng(seed)
    m = rng.normal(size=(3,) + tuple(shape))
    return m / np.sqrt(np.sum(m * m, axis=0))


def _exchange_problem(n, dt=0.05):
    return scheme.Problem(n=n, h=(0.25, 0.25, 0.25), eps=1.0, dt=dt)


def test_matrix_forms_reproduce_the_sweeps():
    """With exchange only (the setting of §4) the matrices built from the step's own
    coefficients reproduce the step: (D - L) m* = U m^n + m^n and (D - U) m** = L m* + m^n
    cell by cell.  A wrong sign, index or coefficient fails this (the printed D - U, with
    its off-diagonal signs flipped, does)."""
    n = (8, 4, 2)
    P = _exchange_problem(n)
    m = _random_unit(n[::-1], 21)
    t = {}
    scheme.sgspm_step(P, m, 0.05, (0.0, 0.0, 0.0), tape=t)
    DL, U, DU, L = spectral.sweep_matrices(spectral.coefficients(P, t))
    mn = m.reshape(3, -1).T
    ms = np.stack([t["m1s"], t["m2s"], t["m3s"]]).reshape(3, -1).T
    mss = np.stack([t["m1ss"], t["m2ss"], t["m3s"]]).reshape(3, -1).T
    assert np.abs(np.einsum("cij,cj->ci", DL, ms) - np.einsum("cij,cj->ci", U, mn) - mn).max() <= 1e-13
    assert np.abs(np.einsum("cij,cj->ci", DU, mss) - np.einsum("cij,cj->ci", L, ms) - mn).max() <= 1e-13
    # the printed D - U (off-diagonal signs of D + U) does not
    DUp = DU.copy()
    DUp[:, 0, 1:] *= -1
    DUp[:, 1, 2] *= -1
    assert np.abs(np.einsum("cij,cj->ci", DUp, mss) - np.einsum("cij,cj->ci", L, ms) - mn).max() > 1e-6


def test_splitting_reproduces_eq_M():
    """D - L - U is the matrix A of eq. M in its Gauss-Seidel form (coefficients at n and *),
    and (D - U) - L the same form with the backward sweep's coefficients."""
    rng = np.random.default_rng(3)
    c = {s: rng.normal(size=(1, 1, 5)) for s in ("g2n", "g3n", "g1s", "g2s", "g3ss", "g2ss")}
    DL, U, DU, L = spectral.sweep_matrices(c)
    v = {s: np.ravel(c[s]) for s in c}
    one = np.ones(5)
    A = np.stack([np.stack([one, v["g3n"], -v["g2n"]], -1),
                  np.stack([-v["g3n"], one, v["g1s"]], -1),
                  np.stack([v["g2s"], -v["g1s"], one], -1)], 1)
    assert np.abs(DL - U - A).max() == 0.0
    Ab = np.stack([np.stack([one, v["g3ss"], -v["g2ss"]], -1),
                   np.stack([-v["g3ss"], one, v["g1s"]], -1),
                   np.stack([v["g2s"], -v["g1s"], one], -1)], 1)
    assert np.abs(DU - L - Ab).max() == 0.0


@pytest.mark.parametrize("which", [0, 1], ids=["gs", "sgs"])
def test_radius_is_the_iteration_convergence_rate(which):
    """rho(G) is the asymptotic rate of the iteration it describes (Gelfand's formula):
    iterating x <- G x from a generic start, |x_k|^(1/k) tends to rho."""
    rng = np.random.default_rng(4 + which)
    c = {s: 0.6 * rng.normal(size=(1, 1, 6)) for s in ("g2n", "g3n", "g1s", "g2s", "g3ss", "g2ss")}
    G = spectral.iteration_matrices(c)[which]
    rho = np.abs(np.linalg.eigvals(G)).max(axis=1)
    k = 400
    for cell in range(6):
        x = rng.normal(size=3)
        logn = 0.0
        for _ in range(k):
            x = G[cell] @ x
            s = np.linalg.norm(x)
            logn += np.log(s)
            x /= s
        assert np.exp(logn / k) == pytest.approx(rho[cell], rel=0.02, abs=1e-12)


def test_uniform_field_has_zero_radius():
    n = (4, 4, 2)
    P = _exchange_problem(n)
    m = np.zeros((3,) + n[::-1])
    m[0] = 0.6
    m[2] = 0.8
    assert spectral.spectral_radii(P, m, 0.1, (0.0, 0.0, 0.0)) == (0.0, 0.0)


def test_radii_grow_with_the_time_step():
    """Every coefficient carries a factor dt, so the radii fall as the step shrinks."""
    n = (16, 8, 1)
    m = _random_unit(n[::-1], 22)
    r = [spectral.spectral_radii(_exchange_problem(n, dt), m, 0.01, (0.0, 0.0, 0.0)) for dt in (0.02, 0.01, 0.005)]
    assert r[0][0] > r[1][0] > r[2][0] > 0.0
    assert r[0][1] > r[1][1] > r[2][1] > 0.0
