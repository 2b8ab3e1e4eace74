"""FP64 CPU oracle for the projected-EM outer loop with a Gaussian-smoothing
projection.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP path.

It follows Alg. 2 (projected EM) of the paper (Shani, Tirer, Giryes, Bendory,
"Denoiser-based projections for 2D super-resolution MRA"):

* until a stopping criterion: F EM steps (eqs. weights_EM, x_EM, rho_EM, via
  em_oracle.em_step), then x <- D(x, sigma_t), then update sigma_t
* sigma_t = 2^(-1/10) sigma_(t-1), sigma_1 = 1          -- eq. (decaying_function)

Readings (the paper's denoiser, BM3D, is not implemented here):

P1  D(x, s) is a circular Gaussian blur of x whose standard deviation, in
    pixels of the L_high grid, is the denoiser's noise level s: out[m] =
    sum_k w[k1] w[k2] x[(m - k) mod Lh] over k in [-R, R]^2, with
    w[k] = exp(-k^2 / (2 s^2)) / sum_j exp(-j^2 / (2 s^2)) and
    R = min(floor(4 s + 1/2), Lh).  R = 0 (s below 1/8, or s not positive
    or not finite) is the identity.  The blur weakens as s decays, as the
    denoiser's prior term does.
P2  The stopping criterion is a fixed number T of outer iterations; the first
    projection uses sigma_1 = 1.
P3  sigma_t is a scalar state kept in FP32 and multiplied by fl32(2^(-1/10))
    after every projection (the device keeps it the same way, so both sides
    use the same s and the same R).
P4  The projection acts on x only; log rho carries over between EM steps.
"""
from __future__ import annotations

import math

import numpy as np

from . import em_oracle as O

DECAY = 2.0 ** -0.1


def decay_schedule(T: int, sigma1: float = 1.0, factor: float = DECAY) -> np.ndarray:
    """sigma_1 .. sigma_T of eq. (decaying_function), kept in FP32 (reading P3)."""
    out = np.empty(T, dtype=np.float32)
    s = np.float32(sigma1)
    f = np.float32(factor)
    for t in range(T):
        out[t] = s
        s = np.float32(s * f)
    return out


def gaussian_taps(s: float, Lh: int):
    """(R, w[-R..R]) of reading P1, in float64."""
    s = float(s)
    if not (s > 0.0) or not math.isfinite(s):
        return 0, np.ones(1)
    R = min(int(math.floor(4.0 * s + 0.5)), Lh)
    if R == 0:
        return 0, np.ones(1)
    k = np.arange(-R, R + 1, dtype=np.float64)
    w = np.exp(-k * k / (2.0 * s * s))
    return R, w / w.sum()


def gaussian_blur_circular(x, s: float) -> np.ndarray:
    """D(x, s) of reading P1 as the 2-D sum over all (2R+1)^2 taps."""
    x = np.asarray(x, dtype=np.float64)
    Lh = x.shape[0]
    R, w = gaussian_taps(s, Lh)
    out = np.zeros_like(x)
    for a, k1 in enumerate(range(-R, R + 1)):
        for b, k2 in enumerate(range(-R, R + 1)):
            out += w[a] * w[b] * np.roll(x, (k1, k2), axis=(0, 1))   # x[(m - k) mod Lh]
    return out


def projected_em(Y, x0, log_rho0, sigma: float, K: int, F: int, T: int,
                 sigma1: float = 1.0, factor: float = DECAY, projection: str = "gaussian"):
    """T outer iterations of Alg. 2 (F EM steps, then the projection, then the
    decay).  Returns the final x, log rho, rho and the log-likelihood of every
    EM step (at its input, reading R6 of em_oracle)."""
    x = np.asarray(x0, dtype=np.float64)
    lr = np.asarray(log_rho0, dtype=np.float64)
    lls, rho = [], None
    for s in decay_schedule(T, sigma1, factor):
        for _ in range(F):
            r = O.em_step(Y, x, lr, sigma, K)
            x, rho, lls = r["x_new"], r["rho_new"], lls + [r["loglik"]]
            lr = np.log(rho)
        if projection == "gaussian":
            x = gaussian_blur_circular(x, float(s))
        elif projection != "identity":
            raise ValueError(projection)
    return dict(x=x, log_rho=lr, rho=rho, loglik=np.array(lls))
