"""Pins of the oracle adjoint: dot-product test against the tangent-linear model and
central finite differences of the forward step (h = 1e-6, FP64)."""
import numpy as np
import pytest

from oracle import adjoint, scheme

CASES = [
    dict(shape=(2, 3, 4), stray=True, Q=0.3, eps=0.7),
    dict(shape=(1, 4, 6), stray=True, Q=0.1, eps=1.2),
    dict(shape=(1, 1, 5), stray=False, Q=0.0, eps=1.0),
]


def _setup(case, seed):
    rng = np.random.default_rng(seed)
    shape = case["shape"]
    P = scheme.Problem(n=shape[::-1], h=(1.0, 0.9, 0.8), eps=case["eps"], dt=0.05,
                       Q=case["Q"], stray=case["stray"])
    m = rng.normal(size=(3,) + shape)
    m /= np.linalg.norm(m, axis=0)
    return P, m, rng


@pytest.mark.parametrize("case", CASES)
def test_dot_product(case):
    P, m, rng = _setup(case, 20)
    he, alpha = np.array([0.1, -0.2, 0.05]), 0.1
    lam, dm, dhe, da = rng.normal(size=m.shape), rng.normal(size=m.shape), rng.normal(size=3), 0.7
    lm, dh, dal = adjoint.adjoint_step(P, m, alpha, he, lam)
    tl = adjoint.tangent_step(P, m, alpha, he, dm, dhe, da)
    lhs = np.sum(lam * tl)
    rhs = np.sum(lm * dm) + dh @ dhe + dal * da
    assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("case", CASES)
def test_tangent_matches_finite_differences(case):
    P, m, rng = _setup(case, 21)
    he, alpha = np.array([0.1, -0.2, 0.05]), 0.1
    dm, dhe, da = rng.normal(size=m.shape), rng.normal(size=3), 0.7
    tl = adjoint.tangent_step(P, m, alpha, he, dm, dhe, da)
    e = 1e-6
    fp = scheme.sgspm_step(P, m + e * dm, alpha + e * da, he + e * dhe)
    fm = scheme.sgspm_step(P, m - e * dm, alpha - e * da, he - e * dhe)
    fd = (fp - fm) / (2 * e)
    assert np.abs(fd - tl).max() <= 1e-6 * np.abs(tl).max()


def test_multistep_gradients_match_finite_differences():
    P, m0, rng = _setup(CASES[0], 22)
    S = 4
    he = 0.05 * rng.normal(size=(S, 3))
    alpha = 0.05
    target = rng.normal(size=m0.shape)
    L, gm, gh, ga = adjoint.run_with_grad(P, m0, alpha, he, target)

    def loss(m, a, h):
        x = m
        for n in range(S):
            x = scheme.sgspm_step(P, x, a, h[n])
        return float(np.mean((x - target) ** 2))

    e = 1e-6
    for _ in range(3):
        v = rng.normal(size=m0.shape)
        fd = (loss(m0 + e * v, alpha, he) - loss(m0 - e * v, alpha, he)) / (2 * e)
        assert fd == pytest.approx(np.sum(gm * v), rel=1e-6)
        w = rng.normal(size=he.shape)
        fd = (loss(m0, alpha, he + e * w) - loss(m0, alpha, he - e * w)) / (2 * e)
        assert fd == pytest.approx(np.sum(gh * w), rel=1e-6)
    fd = (loss(m0, alpha + e, he) - loss(m0, alpha - e, he)) / (2 * e)
    assert fd == pytest.approx(ga, rel=1e-6)
    assert L == pytest.approx(loss(m0, alpha, he), rel=1e-14)
