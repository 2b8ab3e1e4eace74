"""Pins of the projected-EM oracle (Alg. 2 with the Gaussian-smoothing
projection): each checks it against something other than itself."""
import math

import numpy as np
import pytest

from oracle import em_oracle as O
from oracle import projected as P
from paper_2204_04754_amd import synth


def test_decay_schedule_closed_form():
    """eq. (decaying_function): sigma_t = 2^(-(t-1)/10), sigma_1 = 1 (to FP32 rounding)."""
    s = P.decay_schedule(41)
    t = np.arange(41)
    np.testing.assert_allclose(s, 2.0 ** (-t / 10.0), rtol=5e-6)
    assert s[0] == 1.0 and abs(s[10] - 0.5) < 1e-6 and abs(s[20] - 0.25) < 1e-6


def test_taps_definition():
    R, w = P.gaussian_taps(1.0, 64)
    assert R == 4 and w.shape == (9,)
    k = np.arange(-4, 5)
    ref = np.array([math.exp(-kk * kk / 2.0) for kk in k])
    np.testing.assert_allclose(w, ref / ref.sum(), rtol=1e-15)
    assert P.gaussian_taps(0.1, 64)[0] == 0            # below 1/8: identity
    assert P.gaussian_taps(-1.0, 64)[0] == 0 and P.gaussian_taps(float("nan"), 64)[0] == 0
    assert P.gaussian_taps(100.0, 16)[0] == 16          # clamped to Lh


@pytest.mark.parametrize("s", [0.3, 1.0, 2.7])
def test_blur_matches_fft_of_wrapped_kernel(s):
    """Independent route: the circular convolution theorem with the taps
    wrapped onto the Lh x Lh torus."""
    rng = np.random.default_rng(1)
    Lh = 24
    x = rng.standard_normal((Lh, Lh))
    R, w = P.gaussian_taps(s, Lh)
    g = np.zeros((Lh, Lh))
    for a, k1 in enumerate(range(-R, R + 1)):
        for b, k2 in enumerate(range(-R, R + 1)):
            g[k1 % Lh, k2 % Lh] += w[a] * w[b]
    ref = np.real(np.fft.ifft2(np.fft.fft2(x) * np.fft.fft2(g)))
    np.testing.assert_allclose(P.gaussian_blur_circular(x, s), ref, rtol=0, atol=1e-12)


def test_blur_is_separable_1d_passes():
    """Rows then columns with a 1-D circular convolution written independently."""
    rng = np.random.default_rng(2)
    Lh, s = 20, 1.4
    x = rng.standard_normal((Lh, Lh))
    R, w = P.gaussian_taps(s, Lh)

    def conv1(v):
        out = np.zeros_like(v)
        for n in range(Lh):
            out[n] = sum(w[j + R] * v[(n - j) % Lh] for j in range(-R, R + 1))
        return out
    ref = np.apply_along_axis(conv1, 0, x)
    ref = np.apply_along_axis(conv1, 1, ref)
    np.testing.assert_allclose(P.gaussian_blur_circular(x, s), ref, rtol=0, atol=1e-12)


def test_blur_invariants():
    rng = np.random.default_rng(3)
    Lh = 32
    x = rng.standard_normal((Lh, Lh))
    for s in (0.5, 1.0, 3.0):
        y = P.gaussian_blur_circular(x, s)
        assert abs(y.sum() - x.sum()) < 1e-10                       # weights sum to 1
        np.testing.assert_allclose(P.gaussian_blur_circular(np.full((Lh, Lh), 2.5), s), 2.5, atol=1e-13)
        u = (5, -3)
        np.testing.assert_allclose(P.gaussian_blur_circular(np.roll(x, u, (0, 1)), s),
                                   np.roll(y, u, (0, 1)), atol=1e-12)   # shift equivariance
        assert np.linalg.norm(y) <= np.linalg.norm(x)               # a low-pass filter
    np.testing.assert_array_equal(P.gaussian_blur_circular(x, 0.05), x)


def test_delta_response():
    """A unit impulse at (3, 7) spreads into the outer product of the taps."""
    Lh, s = 16, 1.0
    x = np.zeros((Lh, Lh))
    x[3, 7] = 1.0
    y = P.gaussian_blur_circular(x, s)
    R, w = P.gaussian_taps(s, Lh)
    for k1 in range(-R, R + 1):
        for k2 in range(-R, R + 1):
            assert abs(y[(3 + k1) % Lh, (7 + k2) % Lh] - w[k1 + R] * w[k2 + R]) < 1e-15


def test_projected_em_structure():
    """Identity projection = F*T plain EM steps; Gaussian projection = EM steps
    composed by hand with the blur at sigma_1, sigma_2 (Alg. 2 order)."""
    inst = synth.make_instance(16, 2, 120, 0.5, config=80)
    F, T = 2, 2
    r_id = P.projected_em(inst.y, inst.x0, inst.log_rho0, 0.5, 2, F, T, projection="identity")
    x, lr = inst.x0.astype(np.float64), inst.log_rho0.astype(np.float64)
    for _ in range(F * T):
        r = O.em_step(inst.y, x, lr, 0.5, 2)
        x, lr = r["x_new"], np.log(r["rho_new"])
    np.testing.assert_array_equal(r_id["x"], x)
    r_g = P.projected_em(inst.y, inst.x0, inst.log_rho0, 0.5, 2, F, T)
    x, lr = inst.x0.astype(np.float64), inst.log_rho0.astype(np.float64)
    for s in P.decay_schedule(T):
        for _ in range(F):
            r = O.em_step(inst.y, x, lr, 0.5, 2)
            x, lr = r["x_new"], np.log(r["rho_new"])
        x = P.gaussian_blur_circular(x, float(s))
    np.testing.assert_array_equal(r_g["x"], x)
    assert len(r_g["loglik"]) == F * T


def test_projected_em_two_outer_iterations_by_hand():
    """Alg. 2 with F = 1 and T = 2 on the Ll = 1 model (K = Lh = 4: every
    observation a scalar from a mixture of 16 Gaussians with means
    x[(-s1) mod 4, (-s2) mod 4] and weights rho1[s1] rho2[s2]), computed without
    the oracle: each EM step as a textbook known-variance mixture step
    (responsibilities from scipy.stats.norm), each projection as the 2-D
    circular blur written out with its taps exp(-k^2 / 2 s^2) normalised over
    |k| <= floor(4 s + 1/2) (reading P1), at s = 1 and then s = fl32(2^-0.1)
    (eq. decaying_function, readings P2-P3); rho carries over (P4)."""
    from scipy.stats import norm
    Lh, N, sigma = 4, 150, 0.5
    rng = np.random.default_rng(31)
    x0 = rng.standard_normal((Lh, Lh))
    r1, r2 = rng.dirichlet(np.ones(Lh)), rng.dirichlet(np.ones(Lh))
    y = rng.standard_normal(N) * 1.1
    comps = [(a, b) for a in range(Lh) for b in range(Lh)]

    def em_by_hand(x, p1, p2):
        mu = np.array([x[(-a) % Lh, (-b) % Lh] for a, b in comps])
        pi = np.array([p1[a] * p2[b] for a, b in comps])
        dens = pi[None, :] * norm.pdf(y[:, None], loc=mu[None, :], scale=sigma)
        resp = dens / dens.sum(1, keepdims=True)
        nk = resp.sum(0)
        x_new = np.empty((Lh, Lh))
        for k, (a, b) in enumerate(comps):
            x_new[(-a) % Lh, (-b) % Lh] = (resp[:, k] * y).sum() / nk[k]
        pk = (nk / N).reshape(Lh, Lh)
        return x_new, pk.sum(1), pk.sum(0)

    def blur_by_hand(x, s):
        R = min(int(np.floor(4.0 * s + 0.5)), Lh)
        taps = {k: np.exp(-k * k / (2.0 * s * s)) for k in range(-R, R + 1)}
        z = sum(taps.values())
        out = np.zeros_like(x)
        for m1 in range(Lh):
            for m2 in range(Lh):
                acc = 0.0
                for k1 in range(-R, R + 1):
                    for k2 in range(-R, R + 1):
                        acc += taps[k1] * taps[k2] / (z * z) * x[(m1 - k1) % Lh, (m2 - k2) % Lh]
                out[m1, m2] = acc
        return out

    x, p1, p2 = x0, r1, r2
    for s in (1.0, float(np.float32(np.float32(1.0) * np.float32(2.0 ** -0.1)))):
        x, p1, p2 = em_by_hand(x, p1, p2)
        x = blur_by_hand(x, s)
    r = P.projected_em(y.reshape(N, 1, 1), x0, np.log(np.stack([r1, r2])), sigma, Lh, 1, 2)
    np.testing.assert_allclose(r["x"], x, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(np.exp(r["log_rho"]), np.stack([p1, p2]), rtol=1e-9)
