"""GPU parity: the HIP EM step (through the C ABI) against the FP64 oracle on
the same seeded FP32 inputs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import em_oracle as O  # noqa: E402
from paper_2204_04754_amd import synth  # noqa: E402
from tests.bounds import W_UNDERFLOW  # noqa: E402
from tests.gpu_helpers import check_step, gpu_step, oracle_step, rel  # noqa: E402

PRECS = ["fp32_plain", "fp32_mfma"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("prec", PRECS)
def test_small_workload_trajectory(prec):
    """Lh 16, K 2, N 1000, sigma 0.5: ten EM iterations; at every iteration the
    oracle starts from the GPU's own FP32 iterate, so each step is compared
    from identical inputs."""
    inst = synth.workload("lh16_k2_n1000")
    x = inst.x0
    lr = inst.log_rho0
    for it in range(10):
        g = gpu_step(inst.y, x, lr, inst.sigma, inst.K, prec)
        ref = oracle_step(inst.y, x, lr, inst.sigma, inst.K)
        ex, er = check_step(inst.y, x, lr, inst.sigma, inst.K, g, ref, prec)
        print(f"it {it} x {ex:.2e} rho {er:.2e} ll {abs(g['loglik']-ref['loglik'])/abs(ref['loglik']):.2e}")
        x = g["x_new"].astype(np.float32)
        lr = g["log_rho_new"].astype(np.float32)


SHAPES = [  # (Lh, K, N): every supported L_low, ragged N
    (16, 2, 37), (32, 4, 53), (24, 2, 45), (48, 4, 21), (32, 2, 29), (48, 2, 19),
    (64, 2, 17), (96, 2, 6), (128, 2, 3), (64, 4, 11), (96, 4, 7), (96, 3, 5), (256, 4, 3),
    # FP32 MFMA single pass with 3 component groups rounded up to 4 (one idle
    # wave group), and K = 1 (one component, the other slot masked)
    (36, 3, 23), (48, 3, 13), (32, 1, 7),
    # the largest K^2 (256), at L_low 8
    (128, 16, 5),
]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("Lh,K,N", SHAPES)
def test_shapes(prec, Lh, K, N):
    # sigma 2 at L_low <= 48; the L_low 64 maps of 3 observations run at sigma
    # 30 (posterior near the prior), and the sharp-posterior L_low 64 cases
    # are test_low64_sharp_posterior below
    sigma = 30.0 if Lh // K >= 64 else 2.0
    inst = synth.make_instance(Lh, K, N, sigma, config=50, instance=Lh * 10 + K)
    # a non-uniform prior so that every log-prior term matters
    rng = np.random.default_rng(Lh + K)
    lr = np.log(np.stack([rng.dirichlet(np.ones(Lh)), rng.dirichlet(np.ones(Lh))])).astype(np.float32)
    g = gpu_step(inst.y, inst.x0, lr, inst.sigma, K, prec)
    ref = oracle_step(inst.y, inst.x0, lr, inst.sigma, K)
    check_step(inst.y, inst.x0, lr, inst.sigma, K, g, ref, prec)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("Lh,K,N,sigma", [(128, 2, 120, 1.0), (192, 3, 45, 2.0), (64, 1, 40, 0.5)])
def test_low64_sharp_posterior(prec, Lh, K, N, sigma):
    """L_low 64 (2 x 2 score tiles per map, two passes at K >= 2) with a
    posterior far from the prior: noise sigma <= 2 on 4096-pixel
    observations, enough of them that every component holds observations."""
    inst = synth.make_instance(Lh, K, N, sigma, config=56, instance=Lh * 10 + K)
    g = gpu_step(inst.y, inst.x0, inst.log_rho0, sigma, K, prec)
    ref = oracle_step(inst.y, inst.x0, inst.log_rho0, sigma, K)
    # most pixels sit in components that hold whole observations
    assert (ref["a"] >= 1.0).mean() >= 0.5
    ex, er = check_step(inst.y, inst.x0, inst.log_rho0, sigma, K, g, ref, prec)
    print(f"Lh {Lh} K {K} N {N} sigma {sigma}: x {ex:.2e} rho {er:.2e}")


@pytest.mark.parametrize("prec", PRECS)
def test_fp32_underflow_keeps_x(prec):
    """Reading R8 at FP32 range.  Odd shifts on axis 0 get prior mass e^-300
    (the components c1 = 1): every one of their posterior weights is below the
    smallest FP32 subnormal, so the FP32 step sees A_c = 0 and keeps x there,
    while the FP64 oracle still divides its (tiny, non-zero) sums.  At prior
    mass e^-60 the weights are normal FP32 numbers and x' = b / A is computed
    to its element-wise bound."""
    Lh, K, N = 32, 2, 64
    inst = synth.make_instance(Lh, K, N, 1.0, config=57)
    for level in (-300.0, -60.0):
        lr = np.zeros((2, Lh), np.float32)
        lr[0, 1::2] = level
        g = gpu_step(inst.y, inst.x0, lr, 1.0, K, prec)
        ref = oracle_step(inst.y, inst.x0, lr, 1.0, K)
        odd = (np.arange(Lh) % 2 == 1)
        if level == -300.0:
            assert np.all(ref["w_max"][odd, :] < W_UNDERFLOW) and np.all(ref["a"][odd, :] > 0)
            assert not np.allclose(ref["x_new"][odd, :], inst.x0[odd, :])
            assert np.array_equal(g["x_new"][odd, :], inst.x0[odd, :].astype(np.float64))
            assert np.all(g["c"][odd, :] == 0.0)
        else:
            assert np.all(ref["w_max"][odd, :] > 2.0 ** -100)
        check_step(inst.y, inst.x0, lr, 1.0, K, g, ref, prec)


def test_single_pass_covers_expected_shapes():
    """The FP32 MFMA form makes one pass where every component group of an
    observation fits one workgroup; these shapes exercise 1, 2 and 4 groups
    per workgroup and the two-pass fallback."""
    from paper_2204_04754_amd import binding as B
    passes = {(Lh, K): B.srmra_em_step_passes(N, Lh // K, K, "fp32_mfma") for Lh, K, N in SHAPES}
    assert passes[(64, 2)] == 1 and passes[(48, 3)] == 1 and passes[(96, 2)] == 1
    assert passes[(96, 3)] == 2 and passes[(128, 2)] == 2 and passes[(96, 4)] == 2


@pytest.mark.parametrize("prec", PRECS)
def test_deterministic(prec):
    inst = synth.make_instance(64, 2, 3000, 1.0, config=51)
    a = gpu_step(inst.y, inst.x0, inst.log_rho0, 1.0, 2, prec)
    b = gpu_step(inst.y, inst.x0, inst.log_rho0, 1.0, 2, prec)
    for k in ("x_new", "rho_new", "loglik", "ll_obs", "b", "c"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


@pytest.mark.parametrize("prec", PRECS)
def test_single_observation_and_delta_prior(prec):
    """N = 1 and a delta prior: all posterior mass on s0, the sampled pixels
    take the observation's values and every other pixel keeps x."""
    Lh, K = 32, 2
    inst = synth.make_instance(Lh, K, 1, 0.5, config=52)
    lr = np.full((2, Lh), -np.inf, dtype=np.float32)
    s0 = (5, 9)
    lr[0, s0[0]] = 0.0
    lr[1, s0[1]] = 0.0
    g = gpu_step(inst.y, inst.x0, lr, 0.5, K, prec)
    ref = O.em_step(inst.y, inst.x0, lr, 0.5, K)
    rows, cols = O.shift_downsample_indices(Lh, K, *s0)
    expect = inst.x0.astype(np.float64).copy()
    expect[np.ix_(rows, cols)] = inst.y[0]
    np.testing.assert_allclose(g["x_new"], expect, rtol=0, atol=1e-6)
    np.testing.assert_allclose(g["rho_new"], ref["rho_new"], atol=0)
    assert abs(g["loglik"] - ref["loglik"]) < 1e-3 * abs(ref["loglik"])


@pytest.mark.parametrize("prec", PRECS)
def test_centring_offset_invariance(prec):
    """A common offset of y and x (here +5) leaves rho', the posterior mass and
    the log-likelihood unchanged and shifts x' by the offset (the model depends
    on y - P R_s x only); with centring the GPU result at the offset matches the
    oracle at the offset, and centring on / off agree on zero-mean data."""
    inst = synth.make_instance(64, 2, 300, 1.0, config=53)
    off = np.float32(5.0)
    y5, x5 = (inst.y + off).astype(np.float32), (inst.x0 + off).astype(np.float32)
    g5 = gpu_step(y5, x5, inst.log_rho0, 1.0, 2, prec)
    ref5 = oracle_step(y5, x5, inst.log_rho0, 1.0, 2)
    check_step(y5, x5, inst.log_rho0, 1.0, 2, g5, ref5, prec)
    g0 = gpu_step(inst.y, inst.x0, inst.log_rho0, 1.0, 2, prec)
    assert rel(g5["x_new"] - off, g0["x_new"]) < 1e-4
    assert rel(g5["rho_new"], g0["rho_new"]) < 1e-5
    g_off = gpu_step(inst.y, inst.x0, inst.log_rho0, 1.0, 2, prec, centre=False)
    assert rel(g_off["x_new"], g0["x_new"]) < 1e-5
    assert abs(g_off["loglik"] - g0["loglik"]) < 1e-6 * abs(g0["loglik"])


@pytest.mark.parametrize("prec", PRECS)
def test_largest_supported_grid(prec):
    """L_high 1024 (L_low 64, K 16: K^2 = 256 components, the library's
    limits).  The oracle's explicit loop over 2^20 shifts is too slow here, so
    properties that hold at any size are checked: every observation's
    posterior sums to 1, rho rows sum to 1, loglik is the sum of its terms, x'
    keeps x where a component has no mass and is a posterior average of
    observed values elsewhere, and the result is deterministic."""
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


@pytest.mark.parametrize("prec", PRECS)
def test_large_sigma_limit(prec):
    """A step evaluated with sigma = 1000 on data of noise 1: the posterior is
    the prior up to O(||y|| ||x|| / sigma^2) = O(1e-5) terms, so rho' is the
    prior (Dirichlet here) and every component gets mass."""
    Lh, K = 32, 2
    inst = synth.make_instance(Lh, K, 50, 1.0, config=55)
    rng = np.random.default_rng(5)
    rho = np.stack([rng.dirichlet(np.ones(Lh)), rng.dirichlet(np.ones(Lh))])
    lr = np.log(rho).astype(np.float32)
    g = gpu_step(inst.y, inst.x0, lr, 1000.0, K, prec)
    ref = oracle_step(inst.y, inst.x0, lr, 1000.0, K)
    check_step(inst.y, inst.x0, lr, 1000.0, K, g, ref, prec)
    assert rel(g["rho_new"], np.exp(lr.astype(np.float64))) < 1e-4
