"""Pins of the empirical-moment oracle (eq. empiric_MOM)."""
import numpy as np

from oracle import em_oracle as O
from oracle import moments as M


def test_single_observation_is_outer_product():
    y = np.random.default_rng(0).standard_normal((1, 4, 4))
    m1, m2 = M.empirical_moments(y)
    v = y[0].reshape(-1)
    np.testing.assert_array_equal(m1, v)
    for a in range(16):
        for b in range(16):
            assert m2[a, b] == v[a] * v[b]


def test_structure():
    Y = np.random.default_rng(1).standard_normal((50, 3, 3))
    m1, m2 = M.empirical_moments(Y)
    np.testing.assert_allclose(m2, m2.T, atol=0)
    assert np.linalg.eigvalsh(m2).min() > -1e-12                      # PSD
    assert abs(np.trace(m2) - np.mean([np.sum(y * y) for y in Y])) < 1e-12
    # M2 - M1 M1^T is the covariance of the vectorised observations
    np.testing.assert_allclose(m2 - np.outer(m1, m1), np.cov(Y.reshape(50, -1).T, bias=True), atol=1e-12)


def test_closed_form_of_the_model():
    """With one noise-free observation per shift s weighted by rho1[s1] rho2[s2]
    (replicated in proportion), the empirical moments are the model's
    M1 = P C_x rho and M2 = P C_x D_rho C_x^T P^T, built here from explicit
    matrices: column s of C_x is the image translated by s (R_s x), P the
    down-sampler of eq. (model_1)."""
    Lh, K = 6, 2
    rng = np.random.default_rng(2)
    x = rng.standard_normal((Lh, Lh))
    counts1 = rng.integers(1, 4, Lh)
    counts2 = rng.integers(1, 4, Lh)
    rho = np.outer(counts1, counts2).astype(float)
    rho /= rho.sum()
    Y = []
    for s1 in range(Lh):
        for s2 in range(Lh):
            Y += [O.forward(x, K, s1, s2)] * int(counts1[s1] * counts2[s2])
    m1, m2 = M.empirical_moments(np.array(Y))
    # explicit C_x and P
    Cx = np.zeros((Lh * Lh, Lh * Lh))
    for s1 in range(Lh):
        for s2 in range(Lh):
            Cx[:, s1 * Lh + s2] = np.roll(x, (s1, s2), axis=(0, 1)).reshape(-1)   # R_s x
    Ll = Lh // K
    P = np.zeros((Ll * Ll, Lh * Lh))
    for n1 in range(Ll):
        for n2 in range(Ll):
            P[n1 * Ll + n2, (n1 * K) * Lh + n2 * K] = 1.0
    D = np.diag(rho.reshape(-1))
    np.testing.assert_allclose(m1, P @ Cx @ rho.reshape(-1), atol=1e-12)
    np.testing.assert_allclose(m2, P @ Cx @ D @ Cx.T @ P.T, atol=1e-12)
