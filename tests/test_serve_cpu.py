"""CPU tests of the serving loop's policy with a fake executor and a fake
clock: admission by HBM footprint and slots, FIFO order, rejection, cancel,
failure isolation, continuous batching, latency accounting."""
import numpy as np

from paper_2204_04754_amd.serve import (ACTIVE, CANCELLED, DONE, FAILED, QUEUED, REJECTED, Job,
                                        Scheduler, serve)


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-3)


class FakeExecutor:
    """Footprint = N bytes; a tick costs `tick_s` seconds of fake time and
    reports its log-likelihoods one tick late (as the GPU executor does);
    jobs whose y contains NaN report a NaN log-likelihood."""

    def __init__(self, clock, tick_s=0.01):
        self.clock = clock
        self.tick_s = tick_s
        self.admitted = []
        self.tick_sets = []
        self.prev = {}
        self.copies = []
        self.dropped = []

    def footprint(self, job):
        return job.N

    def admit(self, job):
        self.admitted.append(job.job_id)

    def tick(self, ids):
        self.tick_sets.append(tuple(ids))
        self.clock.t += self.tick_s
        out, self.prev = self.prev, {i: (np.nan if self.nan.get(i) else -1.0) for i in ids}
        return out

    def flush(self):
        out, self.prev = self.prev, {}
        return out

    nan = {}

    def finish(self, job):
        self.copies.append(job)

    def finished(self, wait=False):
        out, self.copies = self.copies, []
        for j in out:
            j.result = {"loglik": np.nan if self.nan.get(j.job_id) else -1.0}
        return out

    def drop(self, job):
        self.dropped.append(job.job_id)


def _job(i, N, arrival=0.0, iters=3, nan=False):
    y = np.zeros((N, 8, 8), np.float32)
    if nan:
        y[0, 0, 0] = np.nan
    return Job(i, y, 2, 1.0, np.zeros((16, 16), np.float32), np.zeros((2, 16), np.float32),
               iterations=iters, arrival=arrival)


def test_admission_by_budget_and_slots_fifo():
    s = Scheduler(hbm_budget=100, max_slots=2, footprint=lambda j: j.N)
    for i, n in enumerate([40, 50, 30, 10]):
        s.submit(_job(i, n), 0.0)
    got = [j.job_id for j in s.admit(0.0)]
    assert got == [0, 1]                      # slots full after two
    assert s.used == 90
    s.retire(s.active[0], 1.0)
    got = [j.job_id for j in s.admit(1.0)]
    assert got == [2]                         # 50 + 30 <= 100
    assert [j.job_id for j in s.queue] == [3]
    assert s.active[2].state == ACTIVE and s.queue[0].state == QUEUED


def test_head_of_line_blocks_until_memory_frees():
    s = Scheduler(hbm_budget=100, max_slots=8, footprint=lambda j: j.N)
    s.submit(_job(0, 90), 0.0)
    s.submit(_job(1, 20), 0.0)
    s.submit(_job(2, 5), 0.0)
    assert [j.job_id for j in s.admit(0.0)] == [0]
    assert s.admit(0.1) == []                 # job 1 does not fit, job 2 waits behind it
    s.retire(s.active[0], 0.2)
    assert [j.job_id for j in s.admit(0.2)] == [1, 2]


def test_oversized_job_rejected_and_cancel_frees_budget():
    s = Scheduler(hbm_budget=100, max_slots=8, footprint=lambda j: j.N)
    big = _job(0, 101)
    s.submit(big, 0.0)
    assert big.state == REJECTED and big in s.finished
    s.submit(_job(1, 60), 0.0)
    s.submit(_job(2, 60), 0.0)
    s.admit(0.0)
    assert s.used == 60
    assert s.cancel(1, 0.5)
    assert s.used == 0
    assert [j.job_id for j in s.admit(0.5)] == [2]
    assert s.cancel(2, 0.6) and not s.cancel(99, 0.6)
    assert {j.job_id: j.state for j in s.finished}[2] == CANCELLED


def test_serve_loop_continuous_batching_and_failure_isolation():
    clock = FakeClock()
    ex = FakeExecutor(clock, tick_s=0.01)
    ex.nan = {2: True}
    jobs = [_job(0, 10, 0.0, iters=5), _job(1, 10, 0.025, iters=3), _job(2, 10, 0.0, iters=5, nan=True),
            _job(3, 10, 1.0, iters=2)]
    rep = serve(jobs, ex, hbm_budget=1000, max_slots=4, clock=clock, sleep=clock.sleep)
    st = {j.job_id: j for j in rep.jobs}
    assert st[0].state == DONE and st[1].state == DONE and st[3].state == DONE
    assert st[2].state == FAILED and "non-finite" in st[2].error
    assert ex.dropped == [2]           # its buffers released, the others untouched
    # job 1 arrived while job 0 was running and shared its ticks (continuous batching)
    assert any(0 in t and 1 in t for t in ex.tick_sets)
    assert st[1].t_admit >= 0.025 and st[1].t_admit < 0.05
    # latencies are arrival -> completion, and every job ran its iteration count
    for j in (0, 1, 3):
        assert st[j].iters_done == st[j].iterations
        assert st[j].latency > 0
    summ = rep.summary()
    assert summ["done"] == 3 and summ["failed"] == 1
    assert summ["p50_latency_s"] <= summ["p99_latency_s"]


def test_executor_routes_fft_jobs_and_sizes_their_footprint():
    """GPUExecutor(fft=True) sends a job at an L_low the FFT route supports
    (every L_low of the library: 8, 12, 16, 24, 32, 48, 64) to its own
    FFT-route steps, fft="plan" to the FFT route inside the plan, and without
    fft every job goes to the plan in the executor's precision; the footprint
    counts the route's prepared data and workspace (host-side library queries
    only: nothing is allocated)."""
    import pytest
    pytest.importorskip("torch")
    from paper_2204_04754_amd import binding as B
    from paper_2204_04754_amd.serve import GPUExecutor
    ex = GPUExecutor(precision="bf16_split3", device="cpu", fft=True)
    inplan = GPUExecutor(precision="bf16_split3", device="cpu", fft="plan")
    plain = GPUExecutor(precision="bf16_split3", device="cpu")
    for K, Ll in ((4, 8), (4, 16), (2, 32), (4, 64), (4, 12), (4, 24), (2, 48)):
        job = Job(0, np.zeros((1000, Ll, Ll), np.float32), K, 1.0, None, None, iterations=1)
        form, own = ex._form(job)
        assert own and form == B.SRMRA_FP32_FFT
        expect = (4 * 1000 * Ll * Ll + B.srmra_prepared_bytes(1000, Ll, K, form)
                  + B.srmra_em_step_workspace_bytes(1000, Ll, K, form))
        assert ex.footprint(job) >= expect
        assert inplan._form(job) == (B.SRMRA_FP32_FFT, False)
        assert inplan.footprint(job) == ex.footprint(job)
        assert plain._form(job) == (B.srmra_plan_form(B.SRMRA_BF16_SPLIT3, Ll), False)
    # an L_low the FFT route does not cover goes to the plan in the executor's precision
    job = Job(0, np.zeros((10, 20, 20), np.float32), 2, 1.0, None, None, iterations=1)
    assert ex._form(job) == plain._form(job)
