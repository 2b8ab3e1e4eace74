"""Parity at full sizes, in the launch configuration bench.py times (the same
C-ABI path and partition): per-observation log-likelihood terms on seeded
samples of observations, which the oracle computes one by one, and properties
that hold at any size (every observation's posterior sums to
1, rho rows sum to 1, loglik is the sum of its terms, x' is a posterior
average of observed pixel values).  The single-instance workload is also
compared element by element with a stored full oracle step
(tests/test_gpu_golden.py)."""
import functools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import em_oracle as O  # noqa: E402
from paper_2204_04754_amd import synth  # noqa: E402
from tests.gpu_helpers import gpu_step, ll_scale, unit_roundoff  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@functools.lru_cache(maxsize=2)
def _workload(name):
    return synth.workload(name)


CASES = [("lh64_k2_n100000", "fp32_mfma"), ("lh64_k2_n100000", "fp32_plain"),
         ("lh128_k4_n200000_s0.5", "bf16_split3"), ("lh128_k4_n200000_s0.5", "fp32_mfma"),
         ("lh128_k4_n200000_s2", "bf16_split4"), ("lh256_k4_n20000", "bf16_split3"),
         ("lh64_k2_n100000", "fp32_fft"), ("lh128_k4_n200000_s0.5", "fp32_fft"),
         ("lh256_k4_n20000", "fp32_fft")]


@pytest.mark.parametrize("name,prec", CASES)
def test_full_size_sampled_and_invariants(name, prec):
    inst = _workload(name)
    N, K, s = inst.N, inst.K, inst.sigma
    g = gpu_step(inst.y, inst.x0, inst.log_rho0, s, K, prec)
    # fewer samples where the oracle's loop over Lh^2 shifts is long
    idx = np.sort(np.random.default_rng(N + K).choice(N, 128 if inst.Lh <= 128 else 32, replace=False))
    ys = inst.y[idx]
    ref = O.em_step(ys, inst.x0, inst.log_rho0, s, K)
    u = unit_roundoff(prec)
    bound = 16.0 * u * (1.0 + ll_scale(ys, inst.x0, s, K))
    d = np.abs(g["ll_obs"][idx] - ref["lse"])
    print(f"{name} {prec}: sampled ll terms max err {d.max():.2e} (bound {bound.min():.2e}..)")
    assert np.all(d <= bound)
    # every observation's posterior sums to 1: total posterior mass is N
    assert abs(g["c"].sum() - N) <= 1e-5 * N
    assert np.allclose(g["rho_new"].sum(axis=1), 1.0, atol=1e-6)
    # loglik is the sum of the per-observation terms
    assert abs(g["loglik"] - g["ll_obs"].sum()) <= 1e-5 * abs(g["loglik"])
    # x' is a posterior average of observed pixel values (where it has mass)
    assert g["x_new"].min() >= inst.y.min() - 1e-3 and g["x_new"].max() <= inst.y.max() + 1e-3
