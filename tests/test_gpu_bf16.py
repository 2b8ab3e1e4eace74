"""GPU parity of the BF16 split-precision form (L_low 24 and 32 with one 32x32
tile per score map, 48 and 64 with 2 x 2 tiles, 16 with one 16x16 tile, 48 at
K^2 <= 4 with 3 x 3 tiles of 16x16 in one pass) against the FP64 oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import em_oracle as O  # noqa: E402
from paper_2204_04754_amd import synth  # noqa: E402
from tests.gpu_helpers import check_step, gpu_step, oracle_step, rel  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# ragged N (no multiple of the 8-observation tile)
@pytest.mark.parametrize("prec", ["bf16_split3", "bf16_split4"])
@pytest.mark.parametrize("Lh,K,N,sigma", [(48, 2, 41, 2.0), (64, 2, 27, 2.0), (96, 4, 19, 2.0),
                                          (128, 4, 9, 2.0), (96, 3, 11, 2.0), (64, 2, 600, 0.7),
                                          (96, 2, 45, 2.0), (144, 3, 61, 2.0), (128, 2, 40, 2.0),
                                          (192, 3, 37, 2.0), (48, 1, 50, 2.0), (64, 1, 33, 2.0),
                                          (24, 1, 19, 2.0), (32, 2, 45, 2.0), (48, 3, 101, 2.0),
                                          (64, 4, 133, 2.0), (16, 1, 13, 2.0), (80, 5, 203, 2.0),
                                          (32, 2, 700, 0.7), (96, 2, 203, 1.0), (96, 2, 402, 0.7),
                                          (48, 1, 7, 2.0), (96, 2, 4, 1.5)])
def test_shapes(Lh, K, N, sigma, prec):
    inst = synth.make_instance(Lh, K, N, sigma, config=60, instance=Lh + K)
    rng = np.random.default_rng(Lh * K)
    lr = np.log(np.stack([rng.dirichlet(np.ones(Lh)), rng.dirichlet(np.ones(Lh))])).astype(np.float32)
    g = gpu_step(inst.y, inst.x0, lr, sigma, K, prec)
    ref = oracle_step(inst.y, inst.x0, lr, sigma, K)
    ex, er = check_step(inst.y, inst.x0, lr, sigma, K, g, ref, prec)
    print(f"Lh {Lh} K {K} N {N}: x {ex:.2e} rho {er:.2e}")


def test_wide_tiles_many_chunks():
    """L_low 64 with a ragged observation count spread over many chunks (one
    8-observation group each, the last with 3), unnormalised log rho."""
    inst = synth.make_instance(128, 2, 203, 1.0, config=62)
    lr = (inst.log_rho0 + np.float32(0.7)).astype(np.float32)
    g = gpu_step(inst.y, inst.x0, lr, 1.0, 2, "bf16_split3")
    ref = oracle_step(inst.y, inst.x0, lr, 1.0, 2)
    ex, er = check_step(inst.y, inst.x0, lr, 1.0, 2, g, ref, "bf16_split3")
    print(f"Lh 128 K 2 N 203: x {ex:.2e} rho {er:.2e}")


def test_deterministic_and_unsupported():
    inst = synth.make_instance(64, 2, 1000, 1.0, config=61)
    a = gpu_step(inst.y, inst.x0, inst.log_rho0, 1.0, 2, "bf16_split3")
    b = gpu_step(inst.y, inst.x0, inst.log_rho0, 1.0, 2, "bf16_split3")
    for k in ("x_new", "rho_new", "loglik", "ll_obs", "b", "c"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k
    inst = synth.make_instance(192, 3, 100, 1.0, config=61)
    a = gpu_step(inst.y, inst.x0, inst.log_rho0, 1.0, 3, "bf16_split3")
    b = gpu_step(inst.y, inst.x0, inst.log_rho0, 1.0, 3, "bf16_split3")
    for k in ("x_new", "rho_new", "loglik", "ll_obs", "b", "c"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k
    from paper_2204_04754_amd import binding as B
    assert B.srmra_em_step_workspace_bytes(100, 20, 2, "bf16_split3") == 0   # no L_low 20 kernel


@pytest.mark.parametrize("centre", [True, False])
def test_unit_range_images(centre):
    """Paper-like intensities (the precision-study image min-max scaled to
    [0, 1], mean near 0.5, sigma 0.25) on a 200-observation prefix.  With the
    offset mu taken off y and x the BF16 split meets the 1e-4 bound on x and
    rho; without it the scores carry the mean's magnitude, and the elements are
    held to their bounds only."""
    inst = synth.workload("lh128_k4_n200000_unit_s0.25", N=200)
    g = gpu_step(inst.y, inst.x0, inst.log_rho0, inst.sigma, 4, "bf16_split3", centre=centre)
    ref = oracle_step(inst.y, inst.x0, inst.log_rho0, inst.sigma, 4, centre=centre)
    ex, er = rel(g["x_new"], ref["x_new"]), rel(g["rho_new"], ref["rho_new"])
    ell = abs(g["loglik"] - ref["loglik"]) / abs(ref["loglik"])
    print(f"centre {centre}: x {ex:.2e} rho {er:.2e} loglik {ell:.2e}")
    if centre:
        check_step(inst.y, inst.x0, inst.log_rho0, inst.sigma, 4, g, ref, "bf16_split3")
    else:
        # element-wise bounds only (they scale with the uncentred magnitudes)
        check_step(inst.y, inst.x0, inst.log_rho0, inst.sigma, 4, g, ref, "bf16_split3",
                   centre=False, x_tol=1.0, rho_tol=1.0, bc_tol=1.0)


@pytest.mark.parametrize("prec", ["bf16_split3", "bf16_split4"])
def test_largest_supported_grid(prec):
    """L_high 1024 (L_low 64, K 16: K^2 = 256 components, the library's limits)
    in the 2 x 2-tile form.  The oracle's loop over 2^20 shifts is too slow
    here, so properties that hold at any size are checked: posteriors sum to
    1, rho rows sum to 1, loglik is the sum of its terms, x' is a posterior
    average of observed values (or keeps x), and the result is deterministic."""
    N = 5
    inst = synth.make_instance(1024, 16, N, 30.0, config=54)
    g = gpu_step(inst.y, inst.x0, inst.log_rho0, 30.0, 16, prec)
    assert abs(g["c"].sum() - N) <= 1e-5 * N
    assert np.allclose(g["rho_new"].sum(axis=1), 1.0, atol=1e-6)
    assert abs(g["loglik"] - g["ll_obs"].sum()) <= 1e-5 * abs(g["loglik"])
    assert np.all(np.isfinite(g["x_new"]))
    assert g["x_new"].min() >= min(inst.y.min(), inst.x0.min()) - 1e-3
    assert g["x_new"].max() <= max(inst.y.max(), inst.x0.max()) + 1e-3
    h = gpu_step(inst.y, inst.x0, inst.log_rho0, 30.0, 16, prec)
    assert np.array_equal(g["x_new"], h["x_new"]) and g["loglik"] == h["loglik"]


@pytest.mark.parametrize("Lh,K", [(32, 2), (48, 2), (64, 2), (96, 2), (128, 2)])
def test_single_observation_delta_prior(Lh, K):
    """N = 1 (one partial 8-observation group) and a delta prior at every
    BF16 tile layout (L_low 16, 24, 32, 48, 64): the posterior is exactly 1 at
    s0, so the sampled pixels take the observation's values up to the split's
    residual (2^-17 relative per operand) and every other pixel keeps x
    exactly."""
    inst = synth.make_instance(Lh, K, 1, 0.5, config=63, instance=Lh)
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
