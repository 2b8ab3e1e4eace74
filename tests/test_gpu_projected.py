"""GPU parity of the projected EM (Alg. 2 with the Gaussian-smoothing
projection): the projection kernel against the oracle's 2-D tap sum, the
device noise-level schedule, the outer loop against the oracle's, and HIP
graph replays against eager execution."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import projected as P  # noqa: E402
from paper_2204_04754_amd import binding as B  # noqa: E402
from paper_2204_04754_amd import synth  # noqa: E402
from paper_2204_04754_amd.projected import ProjectedEM  # noqa: E402
from tests.gpu_helpers import rel  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("Lh", [16, 64, 96, 256])
@pytest.mark.parametrize("s", [1.0, 0.37, 2.5, 0.1, 7.0])
def test_projection_matches_oracle(Lh, s):
    rng = np.random.default_rng(Lh)
    x = rng.standard_normal((Lh, Lh)).astype(np.float32)
    xd = torch.as_tensor(x).cuda()
    out = torch.empty_like(xd)
    st = torch.full((1,), s, dtype=torch.float32, device="cuda")
    ws = B.empty_bytes(B.srmra_project_workspace_bytes(Lh))
    B.srmra_project_gaussian(xd, out, Lh, st, P.DECAY, ws)
    torch.cuda.synchronize()
    ref = P.gaussian_blur_circular(x, np.float32(s))
    assert rel(out.cpu().numpy(), ref) < 2e-6
    assert st.item() == np.float32(np.float32(s) * np.float32(P.DECAY))
    # in place (x_out = x_in) gives the same result
    st.fill_(s)
    B.srmra_project_gaussian(xd, xd, Lh, st, P.DECAY, ws)
    torch.cuda.synchronize()
    assert torch.equal(xd, out)


def test_noise_level_schedule_on_device():
    """Twelve projections in a row follow eq. (decaying_function) in FP32."""
    Lh = 32
    st = torch.ones(1, dtype=torch.float32, device="cuda")
    x = torch.zeros((Lh, Lh), device="cuda")
    ws = B.empty_bytes(B.srmra_project_workspace_bytes(Lh))
    seen = []
    for _ in range(12):
        seen.append(st.item())
        B.srmra_project_gaussian(x, x, Lh, st, P.DECAY, ws)
    np.testing.assert_array_equal(np.array(seen, np.float32), P.decay_schedule(12))


def test_projected_em_matches_oracle():
    """Two outer iterations of F = 5 EM steps on the small workload against the
    FP64 oracle's projected EM from the same start."""
    inst = synth.workload("lh16_k2_n1000")
    F, T = 5, 2
    pe = ProjectedEM(inst.y, inst.K, inst.sigma, inst.x0, inst.log_rho0, precision="fp32_mfma", F=F)
    for _ in range(T):
        pe.outer()
    torch.cuda.synchronize()
    ref = P.projected_em(inst.y, inst.x0, inst.log_rho0, inst.sigma, inst.K, F, T)
    assert rel(pe.x.cpu().numpy(), ref["x"]) < 1e-4
    assert rel(pe.job.rho.cpu().numpy(), ref["rho"]) < 1e-4
    assert abs(pe.job.loglik.item() - ref["loglik"][-1]) < 1e-5 * abs(ref["loglik"][-1])
    np.testing.assert_allclose(pe.sigma_state.item(), P.decay_schedule(T + 1)[-1], rtol=0)


def test_projected_graph_replays_match_eager():
    inst = synth.make_instance(64, 2, 3000, 1.0, config=81)
    F, T = 5, 2
    eager = ProjectedEM(inst.y, 2, 1.0, inst.x0, inst.log_rho0, F=F)
    graphed = ProjectedEM(inst.y, 2, 1.0, inst.x0, inst.log_rho0, F=F)
    g = graphed.capture(T)
    for rep in range(3):
        g.replay()
        for _ in range(T):
            eager.outer()
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.equal(graphed.x, eager.x), rep
        assert torch.equal(graphed.sigma_state, eager.sigma_state), rep
        assert torch.equal(graphed.job.loglik, eager.job.loglik), rep
    del junk


@pytest.mark.parametrize("Lh", [16, 48, 128])
def test_shift_error_matches_oracle(Lh):
    from oracle import quality as Q
    rng = np.random.default_rng(Lh + 7)
    x = rng.standard_normal((Lh, Lh)).astype(np.float32)
    xh = (np.roll(x, (3, Lh - 5), axis=(0, 1)) + 0.3 * rng.standard_normal((Lh, Lh))).astype(np.float32)
    ws = B.empty_bytes(B.srmra_shift_error_workspace_bytes(Lh))
    err = torch.empty(1, dtype=torch.float64, device="cuda")
    best = torch.empty(2, dtype=torch.int32, device="cuda")
    B.srmra_shift_error(torch.as_tensor(xh).cuda(), torch.as_tensor(x).cuda(), Lh, err, best, ws)
    torch.cuda.synchronize()
    ref, s = Q.shift_invariant_error(xh, x)
    assert abs(err.item() - ref) <= 1e-12 * ref
    assert tuple(best.cpu().tolist()) == s
    # exact recovery up to a translation reads exactly 0
    xr = torch.as_tensor(np.roll(x, (1, 2), axis=(0, 1))).cuda()
    B.srmra_shift_error(xr, torch.as_tensor(x).cuda(), Lh, err, None, ws)
    torch.cuda.synchronize()
    assert err.item() == 0.0
