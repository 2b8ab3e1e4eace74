"""The allocation-free entry point srmra_em_step_noalloc (workspace in the
library's fixed per-device scratch array) against srmra_em_step with a
caller-owned workspace: bitwise the same results, on two calls in a row (the
second with a smaller input, so stale scratch content from the first call
would show), for every precision form; shapes beyond the array are refused
with SRMRA_ESCRATCH and nothing enqueued."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2204_04754_amd import binding as B  # noqa: E402
from paper_2204_04754_amd import synth  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _buffers(inst, dev="cuda"):
    Lh = inst.Lh
    return dict(y=torch.as_tensor(inst.y).to(dev), x=torch.as_tensor(inst.x0).to(dev),
                lr=torch.as_tensor(inst.log_rho0).to(dev),
                x_new=torch.empty((Lh, Lh), dtype=torch.float32, device=dev),
                rho_new=torch.empty((2, Lh), dtype=torch.float32, device=dev),
                ll=torch.empty(1, dtype=torch.float64, device=dev))


def _run(inst, prec, noalloc):
    b = _buffers(inst)
    if noalloc:
        B.srmra_em_step_noalloc(b["y"], inst.N, inst.Ll, inst.K, b["x"], b["lr"], inst.sigma,
                                b["x_new"], b["rho_new"], b["ll"], prec)
    else:
        ws = B.empty_bytes(B.srmra_em_step_workspace_bytes(inst.N, inst.Ll, inst.K, prec))
        B.srmra_em_step(b["y"], inst.N, inst.Ll, inst.K, b["x"], b["lr"], inst.sigma,
                        b["x_new"], b["rho_new"], b["ll"], prec, ws)
    torch.cuda.synchronize()
    return b["x_new"].cpu().numpy(), b["rho_new"].cpu().numpy(), float(b["ll"].item())


@pytest.mark.parametrize("prec", ["fp32_mfma", "fp32_plain", "bf16_split3", "bf16_split4", "fp32_fft"])
def test_noalloc_equals_workspace_call_twice(prec):
    big = synth.make_instance(64, 2, 1500, 1.0, config=80, instance=1)
    small = synth.make_instance(32, 2, 301, 0.7, config=80, instance=2)
    for inst in (big, small):
        assert B.srmra_em_step_workspace_bytes(inst.N, inst.Ll, inst.K, prec) <= B.SRMRA_SCRATCH_BYTES
        a = _run(inst, prec, noalloc=True)
        r = _run(inst, prec, noalloc=False)
        assert np.array_equal(a[0], r[0]) and np.array_equal(a[1], r[1]) and a[2] == r[2], inst.Lh


def test_noalloc_refuses_shapes_beyond_the_array():
    N, Ll, K = 200000, 32, 4
    need = B.srmra_em_step_workspace_bytes(N, Ll, K, "bf16_split3")
    assert need > B.SRMRA_SCRATCH_BYTES
    L = B.lib()
    Lh = K * Ll
    y = torch.empty(16, dtype=torch.float32, device="cuda")   # never read: refused on the host
    x, x_new = (torch.empty((Lh, Lh), dtype=torch.float32, device="cuda") for _ in range(2))
    lr, rho = (torch.empty((2, Lh), dtype=torch.float32, device="cuda") for _ in range(2))
    ll = torch.empty(1, dtype=torch.float64, device="cuda")
    st = L.srmra_em_step_noalloc(y.data_ptr(), N, Ll, K, x.data_ptr(), lr.data_ptr(), 1.0,
                                 x_new.data_ptr(), rho.data_ptr(), ll.data_ptr(),
                                 B.SRMRA_BF16_SPLIT3, None)
    assert st == B.SRMRA_ESCRATCH
    assert "scratch" in B.status_string(st)
