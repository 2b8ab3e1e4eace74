"""Pins of the reconstruction-error oracle."""
import numpy as np

from oracle import quality as Q


def _img(Lh, seed):
    return np.random.default_rng(seed).standard_normal((Lh, Lh))


def test_exact_recovery_up_to_shift():
    x = _img(12, 0)
    for u in [(0, 0), (3, 5), (11, 1)]:
        err, s = Q.shift_invariant_error(np.roll(x, u, axis=(0, 1)), x)
        assert err == 0.0
        assert s == ((-u[0]) % 12, (-u[1]) % 12)     # R_s R_u x = x for s = -u


def test_against_fft_cross_correlation():
    """||R_s a - b||^2 = ||a||^2 + ||b||^2 - 2 <R_s a, b>, the correlation for all
    s at once from the convolution theorem."""
    a, b = _img(16, 1), _img(16, 2)
    # <R_s a, b> = sum_m a[m - s] b[m] = sum_m a[m] b[m + s] = ifft(conj(A) B)[s]
    corr = np.real(np.fft.ifft2(np.conj(np.fft.fft2(a)) * np.fft.fft2(b)))
    d = (a ** 2).sum() + (b ** 2).sum() - 2 * corr
    k = np.unravel_index(np.argmin(d), d.shape)
    err, s = Q.shift_invariant_error(a, b)
    assert s == tuple(int(v) for v in k)
    assert abs(err - np.sqrt(d[k]) / np.linalg.norm(b)) < 1e-12


def test_invariants():
    x, y = _img(10, 3), _img(10, 4)
    e0, _ = Q.shift_invariant_error(x, y)
    e1, _ = Q.shift_invariant_error(np.roll(x, (2, 7), axis=(0, 1)), np.roll(y, (5, 1), axis=(0, 1)))
    assert abs(e0 - e1) < 1e-12
    assert abs(Q.shift_invariant_error(np.zeros((10, 10)), y)[0] - 1.0) < 1e-15
    e2, _ = Q.shift_invariant_error(2.0 * y, y)          # scaling error, best at s = 0
    assert abs(e2 - 1.0) < 1e-12
