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
