"""GPU test of the serving loop: jobs that arrive while others are running are
batched with them, and each job's result is bitwise the same as when it is
served alone; a job with non-finite data fails without affecting the others."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2204_04754_amd import synth  # noqa: E402
from paper_2204_04754_amd.serve import DONE, FAILED, GPUExecutor, Job, serve  # noqa: E402


class TickClock:
    """Deterministic clock: every executor tick advances it by dt."""

    def __init__(self, dt):
        self.t, self.dt = 0.0, dt

    def __call__(self):
        return self.t

    def sleep(self, s):
        self.t += max(s, 1e-4)


class TimedExecutor(GPUExecutor):
    def __init__(self, clock, **kw):
        super().__init__(**kw)
        self.clock = clock
        self.sets = []

    def tick(self, ids):
        self.sets.append(tuple(ids))
        out = super().tick(ids)
        self.clock.t += self.clock.dt
        return out


SHAPES = [(32, 2, 400, 0.7), (48, 3, 300, 1.0), (64, 2, 250, 1.2), (96, 4, 60, 1.5),
          (48, 2, 200, 0.8), (64, 4, 150, 1.4)]


def _jobs(nan_job=None):
    jobs = []
    for j, (Lh, K, N, s) in enumerate(SHAPES):
        inst = synth.make_instance(Lh, K, N, s, config=80, instance=j)
        y = inst.y.copy()
        if j == nan_job:
            y[3, 2, 1] = np.nan
        jobs.append(Job(j, y, K, s, inst.x0, inst.log_rho0, iterations=4 + j % 3,
                        arrival=0.01 * j))
    return jobs


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("prec", ["fp32_mfma", "bf16_split3", "bf16_split3+fft", "bf16_split3+fftplan"])
def test_served_alone_equals_in_mix(prec):
    """With "+fft" every job (L_low 16, 24, 32) takes the FFT route by its own
    steps; with "+fftplan" the jobs take it inside the shared plan, as FFT
    classes."""
    prec, _, extra = prec.partition("+")
    fft = {"fft": True, "fftplan": "plan"}.get(extra, False)
    clock = TickClock(0.01)
    ex = TimedExecutor(clock, precision=prec, fft=fft)
    rep = serve(_jobs(nan_job=4), ex, hbm_budget=1 << 34, max_slots=4, clock=clock, sleep=clock.sleep)
    st = {j.job_id: j for j in rep.jobs}
    assert st[4].state == FAILED
    assert any(len(s) >= 3 for s in ex.sets)            # jobs shared ticks
    for j in (0, 1, 2, 3, 5):
        assert st[j].state == DONE
        c2 = TickClock(0.01)
        alone_ex = TimedExecutor(c2, precision=prec, fft=fft)
        job = _jobs()[j]
        job.arrival = 0.0
        r2 = serve([job], alone_ex, hbm_budget=1 << 34, max_slots=4, clock=c2, sleep=c2.sleep)
        a = r2.jobs[0].result
        b = st[j].result
        for k in ("x", "log_rho", "rho", "loglik"):
            assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), (j, k)


def test_fft_served_job_equals_its_own_steps():
    """A job routed to the FFT route by the server gets bitwise the result of
    the same number of single-problem FFT-route steps (EMJob)."""
    from paper_2204_04754_amd.em import EMJob
    j = 2                                              # Lh 64, K 2: L_low 32
    clock = TickClock(0.01)
    ex = TimedExecutor(clock, precision="bf16_split3", fft=True)
    job = _jobs()[j]
    job.arrival = 0.0
    rep = serve([job], ex, hbm_budget=1 << 34, max_slots=4, clock=clock, sleep=clock.sleep)
    got = rep.jobs[0].result
    Lh, K, N, s = SHAPES[j]
    inst = synth.make_instance(Lh, K, N, s, config=80, instance=j)
    em = EMJob(inst.y, K, s, inst.x0, inst.log_rho0, precision="fp32_fft")
    for _ in range(job.iterations):
        r = em.step()
    torch.cuda.synchronize()
    assert np.array_equal(got["x"], em.x_current.cpu().numpy())
    assert np.array_equal(got["log_rho"], em.log_rho_current.cpu().numpy())
    assert np.array_equal(got["rho"], r.rho_new.cpu().numpy())
    assert got["loglik"] == float(r.loglik.item())
