"""Seeded synthetic SR-MRA instances.

This module only *draws inputs*: a smooth random image, two shift
distributions, the shifts, the noisy observations of the forward model, and
an EM initialisation.  It contains none of the EM arithmetic (no scores, no
posteriors, no M-step) and is the one module that both the FP64 oracle's
tests and the HIP path consume, so that the two sides see bit-identical
inputs.

Forward model (paper, Sec. 1, eq. (model_1)):
    y_i[n1, n2] = x[(n1*K - s1_i) mod Lh, (n2*K - s2_i) mod Lh] + eps_i[n1, n2]
with s1_i ~ rho1 acting on axis 0 and s2_i ~ rho2 on axis 1, eps ~ N(0, sigma^2)
i.i.d. per pixel, Lh = K * Ll.

The paper measures on natural images (CBSD-68, a test portrait) and a cryo-EM
projection that are not available here; a circularly Gaussian-smoothed field
of i.i.d. normals, scaled to unit pixel standard deviation, stands in for
them (smooth, non-symmetric, no translational symmetry).

Seeds: numpy SeedSequence(220404754, spawn_key=(config, instance, role)) with
role 0 = image, 1 = rho, 2 = shifts, 3 = noise, 4 = initialisation.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

ROOT_SEED = 220404754
ROLE_IMAGE, ROLE_RHO, ROLE_SHIFTS, ROLE_NOISE, ROLE_INIT = 0, 1, 2, 3, 4


def _rng(config: int, instance: int, role: int) -> np.random.Generator:
    ss = np.random.SeedSequence(ROOT_SEED, spawn_key=(int(config), int(instance), int(role)))
    return np.random.Generator(np.random.PCG64(ss))


def smooth_image(rng: np.random.Generator, Lh: int, blur: float = 1.5) -> np.ndarray:
    """N(0,1) field, circular separable Gaussian blur (taps |k| <= ceil(4*blur)),
    divided by its population standard deviation.  Returns float64 [Lh, Lh]."""
    z = rng.standard_normal((Lh, Lh))
    r = int(np.ceil(4.0 * blur))
    taps = np.exp(-(np.arange(-r, r + 1, dtype=np.float64) ** 2) / (2.0 * blur * blur))
    taps /= taps.sum()
    out = z
    for axis in (0, 1):
        acc = np.zeros_like(out)
        for j, k in enumerate(range(-r, r + 1)):
            acc += taps[j] * np.roll(out, k, axis=axis)
        out = acc
    return out / out.std()


def observe(x: np.ndarray, s1: np.ndarray, s2: np.ndarray, K: int) -> np.ndarray:
    """Noise-free down-sampled shifted copies P R_s x (eq. (model_1)), float64 [N, Ll, Ll]."""
    Lh = x.shape[0]
    Ll = Lh // K
    n = np.arange(Ll)
    rows = (n[None, :] * K - s1[:, None]) % Lh          # [N, Ll]
    cols = (n[None, :] * K - s2[:, None]) % Lh          # [N, Ll]
    return x[rows[:, :, None], cols[:, None, :]]


@dataclass
class Instance:
    """One SR-MRA problem.  Arrays that the EM step consumes are float32; the
    oracle upcasts exactly these values to float64."""
    Lh: int
    K: int
    N: int
    sigma: float
    x_true: np.ndarray      # float32 [Lh, Lh]
    rho1: np.ndarray        # float64 [Lh]
    rho2: np.ndarray        # float64 [Lh]
    s1: np.ndarray          # int64 [N]
    s2: np.ndarray          # int64 [N]
    y: np.ndarray           # float32 [N, Ll, Ll]
    x0: np.ndarray          # float32 [Lh, Lh]
    log_rho0: np.ndarray    # float32 [2, Lh]

    @property
    def Ll(self) -> int:
        return self.Lh // self.K

    @property
    def pairs_per_step(self) -> int:
        return self.N * self.Lh * self.Lh


def make_instance(Lh: int, K: int, N: int, sigma: float, config: int = 0,
                  instance: int = 0, blur: float = 1.5,
                  chunk: int = 65536, value_range: str = "std") -> Instance:
    """value_range "std": the smooth image at zero mean and unit std;
    "unit": the same image min-max scaled to [0, 1] (mean near 0.5, like the
    paper's natural images), with the initial iterate 0.5 + 0.25 N(0, 1)."""
    if Lh % K != 0:
        raise ValueError("Lh must be a multiple of K")
    if value_range not in ("std", "unit"):
        raise ValueError("value_range must be 'std' or 'unit'")
    img = smooth_image(_rng(config, instance, ROLE_IMAGE), Lh, blur)
    if value_range == "unit":
        img = (img - img.min()) / (img.max() - img.min())
    x_true = img.astype(np.float32)
    r = _rng(config, instance, ROLE_RHO)
    rho1 = r.dirichlet(np.ones(Lh))
    rho2 = r.dirichlet(np.ones(Lh))
    rs = _rng(config, instance, ROLE_SHIFTS)
    s1 = rs.choice(Lh, size=N, p=rho1).astype(np.int64)
    s2 = rs.choice(Lh, size=N, p=rho2).astype(np.int64)
    rn = _rng(config, instance, ROLE_NOISE)
    Ll = Lh // K
    y = np.empty((N, Ll, Ll), dtype=np.float32)
    xt = x_true.astype(np.float64)
    for a in range(0, N, chunk):
        b = min(N, a + chunk)
        clean = observe(xt, s1[a:b], s2[a:b], K)
        y[a:b] = (clean + sigma * rn.standard_normal(clean.shape)).astype(np.float32)
    ri = _rng(config, instance, ROLE_INIT)
    x0 = ri.standard_normal((Lh, Lh))
    if value_range == "unit":
        x0 = 0.5 + 0.25 * x0
    x0 = x0.astype(np.float32)
    log_rho0 = np.full((2, Lh), -np.log(Lh), dtype=np.float32)
    return Instance(Lh, K, N, float(sigma), x_true, rho1, rho2, s1, s2, y, x0, log_rho0)


# Named workloads (sizes of the paper's experiments, Sec. 5, extended in N).
WORKLOADS = {
    # small case the oracle finishes in seconds: Lh 16, K 2, N 1000, sigma 0.5
    "lh16_k2_n1000": dict(Lh=16, K=2, N=1000, sigma=0.5, config=0),
    # single large instance: Lh 64, K 2, Ll 32, N 1e5, sigma 1
    "lh64_k2_n100000": dict(Lh=64, K=2, N=100_000, sigma=1.0, config=1),
    # precision study: Lh 128, K 4, Ll 32, N 2e5, sigma 0.5 and 2.0
    "lh128_k4_n200000_s0.5": dict(Lh=128, K=4, N=200_000, sigma=0.5, config=2),
    "lh128_k4_n200000_s2": dict(Lh=128, K=4, N=200_000, sigma=2.0, config=2, instance=1),
    # the serving mix's large job: Lh 256, K 4, Ll 64, N 2e4, sigma 1
    "lh256_k4_n20000": dict(Lh=256, K=4, N=20_000, sigma=1.0, config=4, instance=999),
    # single-shape measurements of the batched mix's L_low 16 and 48 classes
    "lh64_k4_n200000": dict(Lh=64, K=4, N=200_000, sigma=1.0, config=5),
    "lh96_k2_n50000": dict(Lh=96, K=2, N=50_000, sigma=1.0, config=5, instance=1),
    # robustness variant: the precision-study image min-max scaled to [0, 1]
    # (mean near 0.5), sigma 0.25 (the middle of the paper's noise levels)
    "lh128_k4_n200000_unit_s0.25": dict(Lh=128, K=4, N=200_000, sigma=0.25, config=2,
                                        value_range="unit"),
}


def workload(name: str, N: Optional[int] = None) -> Instance:
    kw = dict(WORKLOADS[name])
    if N is not None:
        kw["N"] = int(N)
    return make_instance(**kw)


def mixed_batch(count: int = 64, config: int = 3, seed_instance0: int = 0,
                n_range=(5000, 50000), sigma_range=(0.3, 2.0),
                lh_choices=(32, 48, 64, 96), k_choices=(2, 3, 4),
                large_frac: float = 0.0, large=(256, 4, 20000)):
    """Shapes for a batch of uneven instances: Lh uniform over lh_choices, K
    uniform over the divisors of Lh in k_choices, N uniform in n_range, sigma
    uniform in sigma_range.  With large_frac > 0 a fraction of the draws is
    replaced by the large shape (Lh, K, N).  Returns a list of kwargs for
    make_instance (instances are generated lazily by the caller)."""
    rng = _rng(config, 10_000 + seed_instance0, ROLE_INIT)
    out = []
    for j in range(count):
        if large_frac > 0 and rng.random() < large_frac:
            Lh, K, N = large
            sigma = float(rng.uniform(*sigma_range))
        else:
            Lh = int(rng.choice(lh_choices))
            ks = [k for k in k_choices if Lh % k == 0]
            K = int(rng.choice(ks))
            N = int(rng.integers(n_range[0], n_range[1] + 1))
            sigma = float(rng.uniform(*sigma_range))
        out.append(dict(Lh=Lh, K=K, N=N, sigma=sigma, config=config,
                        instance=seed_instance0 + j))
    return out
