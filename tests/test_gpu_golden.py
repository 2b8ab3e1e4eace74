"""Parity against stored FP64 oracle results (tests/golden/*.npz, written by
tests/golden/make_goldens.py, which calls only the oracle): every element of
x', rho', b and c and the per-observation log-likelihood terms, for

* the first 2000 observations of the precision-study workload (Lh 128, K 4,
  Ll 32) at sigma 0.5 and 2, from the seeded start and from the true image
  and prior, in every precision form;
* one full step of the single-instance workload (Lh 64, K 2, Ll 32,
  N 100000, sigma 1), in the partition the benchmark times;
* the library's one-call entry point srmra_em_step (observation preparation
  inside the workspace), against the oracle and bitwise against the
  prepared-observation call.

Bounds per element: tests/bounds.py (eq. weights_EM, eq. x_EM, eq. rho_EM);
norm-wise relative error <= 1e-4 on x', rho', b and c."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2204_04754_amd import binding as B  # noqa: E402
from paper_2204_04754_amd.em import EMJob  # noqa: E402
from tests.bounds import compare_step  # noqa: E402
from tests.golden_cases import FULL_CASES, SUBSET_CASES, case_inputs, fingerprint, load  # noqa: E402
from tests.gpu_helpers import gpu_step  # noqa: E402

FORMS = ["fp32_plain", "fp32_mfma", "bf16_split3", "bf16_split4", "fp32_fft"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _case(name):
    y, x, lr, sigma, K = case_inputs(name)
    gold = load(name)
    # the stored result belongs to exactly these inputs
    assert np.allclose(gold["fingerprint"], fingerprint(y, x, lr), rtol=1e-12, atol=0)
    return y, x, lr, sigma, K, gold


@pytest.mark.parametrize("prec", FORMS)
@pytest.mark.parametrize("case", SUBSET_CASES)
def test_precision_subset(case, prec):
    y, x, lr, sigma, K, gold = _case(case)
    g = gpu_step(y, x, lr, sigma, K, prec)
    r = compare_step(g, gold, x, y, prec, K, sigma)
    print(f"{case} {prec}: x {r['x']:.2e} rho {r['rho']:.2e} b {r['b']:.2e} c {r['c']:.2e} "
          f"loglik {r['loglik']:.2e} max x err / bound {r['x_max_ratio']:.2e}")


@pytest.mark.parametrize("prec", ["fp32_mfma", "fp32_plain", "bf16_split3", "fp32_fft"])
@pytest.mark.parametrize("case", FULL_CASES)
def test_full_size_step(case, prec):
    """The whole single-instance workload in one step, compared element by
    element (the per-observation terms on the stored seeded sample).  The
    debug outputs do not change the computation: the plain prepared call gives
    bitwise the same x', rho' and loglik."""
    y, x, lr, sigma, K, gold = _case(case)
    g = gpu_step(y, x, lr, sigma, K, prec)
    r = compare_step(g, gold, x, y, prec, K, sigma, lse_idx=gold["lse_idx"])
    print(f"{case} {prec}: x {r['x']:.2e} rho {r['rho']:.2e} b {r['b']:.2e} c {r['c']:.2e} "
          f"loglik {r['loglik']:.2e} max x err / bound {r['x_max_ratio']:.2e}")
    job = EMJob(y, K, sigma, x, lr, precision=prec)
    res = job.step()
    torch.cuda.synchronize()
    assert np.array_equal(res.x_new.cpu().numpy().astype(np.float64), g["x_new"])
    assert np.array_equal(res.rho_new.cpu().numpy().astype(np.float64), g["rho_new"])
    assert float(res.loglik.item()) == g["loglik"]


@pytest.mark.parametrize("prec", ["fp32_mfma", "fp32_plain", "bf16_split3", "bf16_split4", "fp32_fft"])
def test_one_call_entry_point(prec):
    """srmra_em_step(y, N, L_low, K, x, log_rho, sigma) -> x_new, rho_new,
    loglik with the observations prepared inside the workspace: against the
    stored oracle result, and bitwise equal to srmra_em_step_prepared."""
    y, x, lr, sigma, K, gold = _case("lh128_k4_n2000_s0.5_init")
    N, Ll = y.shape[0], y.shape[1]
    Lh = K * Ll
    dev = "cuda"
    yt = torch.as_tensor(y).to(dev)
    xt = torch.as_tensor(x).to(dev)
    lrt = torch.as_tensor(lr).to(dev)
    x_new = torch.empty((Lh, Lh), dtype=torch.float32, device=dev)
    rho_new = torch.empty((2, Lh), dtype=torch.float32, device=dev)
    ll = torch.empty(1, dtype=torch.float64, device=dev)
    ws = B.empty_bytes(B.srmra_em_step_workspace_bytes(N, Ll, K, prec))
    B.srmra_em_step(yt, N, Ll, K, xt, lrt, sigma, x_new, rho_new, ll, prec, ws)
    torch.cuda.synchronize()
    g = dict(x_new=x_new.cpu().numpy().astype(np.float64),
             rho_new=rho_new.cpu().numpy().astype(np.float64), loglik=float(ll.item()))
    r = compare_step(g, gold, x, y, prec, K, sigma)
    print(f"srmra_em_step {prec}: x {r['x']:.2e} rho {r['rho']:.2e} loglik {r['loglik']:.2e}")
    job = EMJob(y, K, sigma, x, lr, precision=prec)
    res = job.step()
    torch.cuda.synchronize()
    assert np.array_equal(res.x_new.cpu().numpy().astype(np.float64), g["x_new"])
    assert np.array_equal(res.rho_new.cpu().numpy().astype(np.float64), g["rho_new"])
    assert float(res.loglik.item()) == g["loglik"]
