"""GPU parity of the BF16 split-precision form at L_low 8 and 12 (score maps of
8 observations and 4 or 8 components packed into 32x32 tiles; one pass while
the components fit in one workgroup, two passes beyond) against the FP64
oracle, on every element."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import em_oracle as O  # noqa: E402
from paper_2204_04754_amd import binding as B  # noqa: E402
from paper_2204_04754_amd import synth  # noqa: E402
from tests.gpu_helpers import check_step, gpu_step, oracle_step  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# (L_high, K, N, sigma), ragged N.  L_low 8 (4 components per wave): K 1, 2
# (one block: 4 observation slots per workgroup), 3 (3 blocks, one idle wave),
# 4 (4 blocks), 5 and 8 (two passes: 7 and 16 blocks).  L_low 12 (8 components
# per wave): K 1, 2 (half a block), 3 and 4 (2 blocks), 5 (4 blocks), 6 (two
# passes, 5 blocks).
SHAPES = [(8, 1, 19, 1.0), (16, 2, 45, 1.0), (24, 3, 37, 1.0), (32, 4, 101, 1.5), (40, 5, 61, 2.0),
          (64, 8, 23, 4.0), (12, 1, 13, 1.0), (24, 2, 45, 1.0), (36, 3, 41, 1.0), (48, 4, 77, 1.5),
          (60, 5, 29, 2.0), (72, 6, 17, 3.0), (16, 2, 600, 0.5), (48, 4, 300, 0.7)]


@pytest.mark.parametrize("prec", ["bf16_split3", "bf16_split4"])
@pytest.mark.parametrize("Lh,K,N,sigma", SHAPES)
def test_shapes(Lh, K, N, sigma, prec):
    inst = synth.make_instance(Lh, K, N, sigma, config=64, instance=Lh + K)
    rng = np.random.default_rng(Lh * K + 1)
    lr = np.log(np.stack([rng.dirichlet(np.ones(Lh)), rng.dirichlet(np.ones(Lh))])).astype(np.float32)
    g = gpu_step(inst.y, inst.x0, lr, sigma, K, prec)
    ref = oracle_step(inst.y, inst.x0, lr, sigma, K)
    ex, er = check_step(inst.y, inst.x0, lr, sigma, K, g, ref, prec)
    passes = B.srmra_em_step_passes(N, Lh // K, K, prec)
    print(f"Lh {Lh} K {K} N {N} ({passes} pass): x {ex:.2e} rho {er:.2e}")


def test_passes():
    """One pass while K^2 fits in four blocks of components, two beyond."""
    for ll, K, n in ((8, 1, 1), (8, 4, 1), (8, 5, 2), (8, 8, 2), (12, 2, 1), (12, 5, 1), (12, 6, 2)):
        assert B.srmra_em_step_passes(1000, ll, K, "bf16_split3") == n, (ll, K)


def test_config0_workload_ten_steps():
    """The small parity workload (L_low 8, K 2, N 1000, sigma 0.5), ten EM
    steps in the BF16 split, each from the GPU's own iterate and compared with
    the oracle's step from that same iterate."""
    inst = synth.workload("lh16_k2_n1000")
    x, lr = inst.x0, inst.log_rho0
    for it in range(10):
        g = gpu_step(inst.y, x, lr, inst.sigma, inst.K, "bf16_split3")
        ref = oracle_step(inst.y, x, lr, inst.sigma, inst.K)
        ex, er = check_step(inst.y, x, lr, inst.sigma, inst.K, g, ref, "bf16_split3")
        x = g["x_new"].astype(np.float32)
        lr = g["log_rho_new"].astype(np.float32)
        print(f"step {it}: x {ex:.2e} rho {er:.2e}")


def test_deterministic():
    for Lh, K in ((32, 4), (72, 6)):
        inst = synth.make_instance(Lh, K, 333, 1.0, config=65)
        a = gpu_step(inst.y, inst.x0, inst.log_rho0, 1.0, K, "bf16_split3")
        b = gpu_step(inst.y, inst.x0, inst.log_rho0, 1.0, K, "bf16_split3")
        for k in ("x_new", "rho_new", "loglik", "ll_obs", "b", "c"):
            assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (Lh, K, k)


@pytest.mark.parametrize("Lh,K", [(16, 2), (32, 4), (40, 5), (24, 2), (48, 4), (72, 6)])
def test_single_observation_delta_prior(Lh, K):
    """N = 1 and a delta prior: the posterior is exactly 1 at s0, so the
    sampled pixels take the observation's values up to the split's residual
    and every other pixel keeps x exactly (one and two passes)."""
    inst = synth.make_instance(Lh, K, 1, 0.5, config=66, instance=Lh)
    lr = np.full((2, Lh), -np.inf, dtype=np.float32)
    s0 = (5, 9)
    lr[0, s0[0]] = 0.0
    lr[1, s0[1]] = 0.0
    g = gpu_step(inst.y, inst.x0, lr, 0.5, K, "bf16_split3")
    ref = O.em_step(inst.y, inst.x0, lr, 0.5, K)
    rows, cols = O.shift_downsample_indices(Lh, K, *s0)
    expect = inst.x0.astype(np.float64).copy()
    expect[np.ix_(rows, cols)] = inst.y[0]
    keep = np.ones_like(expect, dtype=bool)
    keep[np.ix_(rows, cols)] = False
    assert np.array_equal(g["x_new"][keep], expect[keep])
    np.testing.assert_allclose(g["x_new"], expect, rtol=0, atol=1e-4 * np.abs(inst.y).max())
    np.testing.assert_allclose(g["rho_new"], ref["rho_new"], atol=0)
    assert abs(g["loglik"] - ref["loglik"]) < 1e-3 * abs(ref["loglik"])
