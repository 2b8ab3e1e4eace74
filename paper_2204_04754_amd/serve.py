"""Serving form: continuous batching of EM reconstruction jobs on one GPU.

A job is an SR-MRA instance (observations, K, sigma, initial x and log rho)
that needs a fixed number of unprojected EM iterations.  The server keeps every
admitted job's observation stack, prepared data and iterate resident in HBM
until it finishes.  Each scheduler tick:

1. moves arrived jobs into the FIFO queue (jobs whose footprint exceeds the
   whole HBM budget are rejected at once);
2. admits queued jobs in order while a slot is free and the job's footprint
   fits in the free budget: their observations are uploaded and prepared on a
   side stream, which the step stream waits for (an event) before the job's
   first step, so the upload overlaps the steps already enqueued;
3. advances every active job that still needs iterations by one EM step with
   one batched execution (the plan is rebuilt, and its descriptors uploaded
   asynchronously, only when that set changed), so jobs that arrived while
   others were running share the device with them from this tick on;
4. reads the previous tick's log-likelihoods (copied to pinned host memory
   behind that tick's work, one tick late, so the host never waits for the
   tick it has just enqueued): a job whose log-likelihood is not finite
   fails alone;
5. a job that has enqueued its last iteration has its result copied to
   pinned host memory behind it and is retired (buffers released, budget
   freed) once that copy has completed.

The admission policy (`Scheduler`) is plain Python and is tested on the CPU
with a fake clock; `GPUExecutor` does the device work through the C ABI.  An
instance's result does not depend on which jobs share its ticks (each instance
runs the same device code with a partition fixed by its own shape).
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Deque, Dict, List, Optional, Tuple

import numpy as np

QUEUED, ACTIVE, DONE, FAILED, REJECTED, CANCELLED = (
    "queued", "active", "done", "failed", "rejected", "cancelled")


@dataclass
class Job:
    job_id: int
    y: np.ndarray                 # float32 [N][Ll][Ll]
    K: int
    sigma: float
    x0: np.ndarray                # float32 [Lh][Lh]
    log_rho0: np.ndarray          # float32 [2][Lh]
    iterations: int = 20
    arrival: float = 0.0
    state: str = QUEUED
    footprint: int = 0
    iters_done: int = 0
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    result: Optional[dict] = None
    error: Optional[str] = None

    @property
    def N(self) -> int:
        return int(self.y.shape[0])

    @property
    def Ll(self) -> int:
        return int(self.y.shape[1])

    @property
    def latency(self) -> Optional[float]:
        return None if self.t_done is None else self.t_done - self.arrival


class Scheduler:
    """FIFO admission by HBM footprint and free slots (no device work)."""

    def __init__(self, hbm_budget: int, max_slots: int, footprint: Callable[[Job], int]):
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.footprint = footprint
        self.queue: Deque[Job] = deque()
        self.active: Dict[int, Job] = {}
        self.used = 0
        self.finished: List[Job] = []

    def submit(self, job: Job, now: float) -> None:
        job.footprint = int(self.footprint(job))
        if job.footprint > self.budget:
            job.state = REJECTED
            job.error = f"footprint {job.footprint} B exceeds the HBM budget {self.budget} B"
            job.t_done = now
            self.finished.append(job)
            return
        job.state = QUEUED
        self.queue.append(job)

    def cancel(self, job_id: int, now: float) -> bool:
        for j in list(self.queue):
            if j.job_id == job_id:
                self.queue.remove(j)
                j.state, j.t_done = CANCELLED, now
                self.finished.append(j)
                return True
        if job_id in self.active:
            j = self.active.pop(job_id)
            self.used -= j.footprint
            j.state, j.t_done = CANCELLED, now
            self.finished.append(j)
            return True
        return False

    def admit(self, now: float) -> List[Job]:
        """Jobs to start now, in FIFO order (head-of-line: stops at the first
        job that does not fit)."""
        out = []
        while self.queue and len(self.active) < self.max_slots:
            j = self.queue[0]
            if self.used + j.footprint > self.budget:
                break
            self.queue.popleft()
            j.state, j.t_admit = ACTIVE, now
            self.active[j.job_id] = j
            self.used += j.footprint
            out.append(j)
        return out

    def retire(self, job: Job, now: float, failed: bool = False, error: str = "") -> None:
        self.active.pop(job.job_id, None)
        self.used -= job.footprint
        job.state = FAILED if failed else DONE
        job.error = error or None
        job.t_done = now
        self.finished.append(job)

    @property
    def idle(self) -> bool:
        return not self.queue and not self.active


class GPUExecutor:
    """Device side of the server: per-job buffers and the batched plan.  With
    fft=True a job whose L_low the FFT route supports is advanced by its own
    FFT-route step (srmra_em_step_prepared, SRMRA_FP32_FFT) on the same stream
    after the plan, which holds the other jobs; with fft="plan" such a job is
    prepared for the FFT route and advanced inside the plan, whose tuning
    entries send its (L_low, K) class to the FFT route.

    Interface used by `serve`: footprint(job), admit(job), tick(ids) (enqueue
    one step of ids; returns the previous tick's {id: loglik}), finish(job)
    (enqueue the result copy), finished() (jobs whose result is on the host),
    drop(job) (release a failed job's buffers), flush() (the last tick's
    log-likelihoods)."""

    def __init__(self, precision="fp32_mfma", device="cuda", fft=False):
        import torch

        from . import binding as B
        self.torch = torch
        self.B = B
        self.device = torch.device(device)
        self.precision = B._prec(precision)
        self.fft = fft if fft == "plan" else bool(fft)
        self.buf: Dict[int, dict] = {}
        self.plan = None
        self.plan_ids: Optional[tuple] = None
        self.workspace = None
        self.old_plans: List[tuple] = []
        self.pending_ll = None          # (ids, pinned host tensor, event) of the last tick
        self.copies: List[tuple] = []   # (job, pinned results, event)
        if self.device.type == "cuda":
            self.stream = torch.cuda.current_stream(self.device)
            self.side = torch.cuda.Stream(self.device)     # default priority

    def _form(self, job_or_buf) -> Tuple[int, bool]:
        """(precision the job runs in, whether by its own FFT-route step)."""
        B = self.B
        Ll, K = (job_or_buf.Ll, job_or_buf.K) if isinstance(job_or_buf, Job) else \
            (job_or_buf["L_low"], job_or_buf["K"])
        if self.fft and B.srmra_em_step_workspace_bytes(1, Ll, K, B.SRMRA_FP32_FFT) > 0:
            return B.SRMRA_FP32_FFT, self.fft != "plan"
        return B.srmra_plan_form(self.precision, Ll), False

    def footprint(self, job: Job) -> int:
        B = self.B
        Ll, K, N = job.Ll, job.K, job.N
        form, _ = self._form(job)
        if form < 0:
            return 1 << 62
        Lh = K * Ll
        return (4 * N * Ll * Ll + B.srmra_prepared_bytes(N, Ll, K, form)
                + B.srmra_em_step_workspace_bytes(N, Ll, K, form) + 4 * (2 * Lh * Lh + 6 * Lh) + 4096)

    def admit(self, job: Job) -> None:
        """Upload and prepare on the side stream; the buffers are allocated
        there and marked as used by the step stream as well."""
        torch, B = self.torch, self.B
        f = dict(device=self.device, dtype=torch.float32)
        form, own = self._form(job)
        Lh = job.K * job.Ll
        with torch.cuda.stream(self.side):
            y = torch.as_tensor(np.ascontiguousarray(job.y, np.float32)).to(self.device, non_blocking=True)
            prep = B.empty_bytes(B.srmra_prepared_bytes(job.N, job.Ll, job.K, form), self.device)
            B.srmra_prepare_observations(y, job.N, job.Ll, job.K, form, prep, self.side)
            ws = B.empty_bytes(B.srmra_em_step_workspace_bytes(job.N, job.Ll, job.K, form), self.device) \
                if own else None
            b = dict(y=y, prep=prep, N=job.N, L_low=job.Ll, K=job.K, sigma=job.sigma, own=own, ws=ws, form=form,
                     xa=torch.as_tensor(np.asarray(job.x0, np.float32)).to(**f, non_blocking=True),
                     xb=torch.empty((Lh, Lh), **f),
                     la=torch.as_tensor(np.asarray(job.log_rho0, np.float32)).to(**f, non_blocking=True),
                     lb=torch.empty((2, Lh), **f),
                     rho_new=torch.empty((2, Lh), **f),
                     loglik=torch.empty(1, dtype=torch.float64, device=self.device),
                     cur=0, ready=torch.cuda.Event())
            b["ready"].record(self.side)
        for k in ("y", "prep", "ws", "xa", "xb", "la", "lb", "rho_new", "loglik"):
            if b[k] is not None:
                b[k].record_stream(self.stream)
        b["waited"] = False
        self.buf[job.job_id] = b

    def _problem(self, b):
        cur = b["cur"]
        return dict(y=b["y"], prep=b["prep"], N=b["N"], L_low=b["L_low"], K=b["K"],
                    sigma=b["sigma"],
                    x=b["xa"] if cur == 0 else b["xb"], x_new=b["xb"] if cur == 0 else b["xa"],
                    log_rho=b["la"] if cur == 0 else b["lb"],
                    log_rho_new=b["lb"] if cur == 0 else b["la"],
                    rho_new=b["rho_new"], loglik=b["loglik"])

    def tick(self, ids: List[int]) -> Dict[int, float]:
        """Enqueue one EM step of every job in `ids` on the step stream and
        return the log-likelihoods of the previous tick (waiting for that
        tick only, never for this one)."""
        torch, B = self.torch, self.B
        for i in ids:
            b = self.buf[i]
            if not b["waited"]:
                self.stream.wait_event(b["ready"])
                b["waited"] = True
        planned = [i for i in ids if not self.buf[i]["own"]]
        key = tuple(planned)
        if planned and (key != self.plan_ids or self.plan is None):
            if self.plan is not None:
                # released one tick later (its helper streams may still run)
                self.old_plans.append((self.plan, self.workspace))
            # classes of jobs prepared for the FFT route run there inside the plan
            fft_classes = sorted({(self.buf[i]["L_low"], self.buf[i]["K"]) for i in planned
                                  if self.buf[i]["form"] == B.SRMRA_FP32_FFT})
            table = [dict(precision=self.precision, L_low=ll, K=k, form=B.SRMRA_FP32_FFT, item_obs=0)
                     for (ll, k) in fft_classes]
            self.plan = B.Plan([self._problem(self.buf[i]) for i in planned], self.precision,
                               tuning=table or None)
            self.workspace = B.empty_bytes(self.plan.workspace_bytes, self.device)
            self.plan.upload(self.workspace, self.stream)
            self.plan_ids = key
        if planned:
            self.plan.execute(self.workspace, self.stream)
        for i in ids:
            b = self.buf[i]
            if b["own"]:
                q = self._problem(b)
                B.srmra_em_step_prepared(q["y"], q["prep"], q["N"], q["L_low"], q["K"], q["x"],
                                         q["log_rho"], q["sigma"], q["x_new"], q["rho_new"],
                                         q["log_rho_new"], q["loglik"], B.SRMRA_FP32_FFT, b["ws"],
                                         self.stream)
        for i in ids:
            self.buf[i]["cur"] ^= 1
        with torch.cuda.stream(self.stream):
            ll = torch.cat([self.buf[i]["loglik"] for i in ids])
            host = torch.empty(ll.shape, dtype=ll.dtype, pin_memory=True)
            host.copy_(ll, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.stream)
        prev, self.pending_ll = self.pending_ll, (list(ids), host, ev)
        out = self._read(prev)
        # plans replaced before the tick just read have no work left on the device
        while len(self.old_plans) > 1:
            p, _ = self.old_plans.pop(0)
            p.close()
        return out

    @staticmethod
    def _read(entry) -> Dict[int, float]:
        if entry is None:
            return {}
        ids, host, ev = entry
        ev.synchronize()
        return {i: float(v) for i, v in zip(ids, host.numpy())}

    def flush(self) -> Dict[int, float]:
        """The last tick's log-likelihoods (waits for that tick)."""
        prev, self.pending_ll = self.pending_ll, None
        return self._read(prev)

    def finish(self, job: Job) -> None:
        """Enqueue the copy of the job's result to pinned host memory behind
        its last step."""
        torch = self.torch
        b = self.buf[job.job_id]
        x = b["xa"] if b["cur"] == 0 else b["xb"]
        lr = b["la"] if b["cur"] == 0 else b["lb"]
        with torch.cuda.stream(self.stream):
            out = {}
            for k, t in (("x", x), ("log_rho", lr), ("rho", b["rho_new"]), ("loglik", b["loglik"])):
                h = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
                h.copy_(t, non_blocking=True)
                out[k] = h
            ev = torch.cuda.Event()
            ev.record(self.stream)
        self.copies.append((job, out, ev))

    def finished(self, wait: bool = False) -> List[Job]:
        """Jobs whose result copy has completed (all pending ones if wait):
        their result is set and their buffers released."""
        done, keep = [], []
        for job, out, ev in self.copies:
            if wait or ev.query():
                ev.synchronize()
                job.result = dict(x=out["x"].numpy().copy(), log_rho=out["log_rho"].numpy().copy(),
                                  rho=out["rho"].numpy().copy(), loglik=float(out["loglik"].numpy()[0]))
                self.buf.pop(job.job_id, None)
                self.plan_ids = None   # the active set changes
                done.append(job)
            else:
                keep.append((job, out, ev))
        self.copies = keep
        return done

    def drop(self, job: Job) -> None:
        """Release a failed job's buffers (the step stream still orders their
        reuse after the work already enqueued)."""
        self.buf.pop(job.job_id, None)
        self.plan_ids = None


@dataclass
class ServeReport:
    jobs: List[Job] = field(default_factory=list)
    wall: float = 0.0
    ticks: int = 0

    def summary(self) -> dict:
        done = [j for j in self.jobs if j.state == DONE]
        lat = np.array([j.latency for j in done]) if done else np.zeros(0)
        first = min((j.arrival for j in self.jobs), default=0.0)
        last = max((j.t_done for j in done), default=first)
        span = max(last - first, 1e-9)
        return dict(jobs=len(self.jobs), done=len(done),
                    failed=sum(j.state == FAILED for j in self.jobs),
                    rejected=sum(j.state == REJECTED for j in self.jobs),
                    solves_per_s=len(done) / span,
                    p50_latency_s=float(np.percentile(lat, 50)) if lat.size else None,
                    p99_latency_s=float(np.percentile(lat, 99)) if lat.size else None,
                    ticks=self.ticks, wall_s=self.wall)


def serve(jobs: List[Job], executor, hbm_budget: int, max_slots: int = 64,
          clock: Callable[[], float] = time.perf_counter, sleep=time.sleep,
          on_tick: Optional[Callable[[int, Scheduler], None]] = None) -> ServeReport:
    """Run the continuous-batching loop until every job is finished.  Job
    arrival times are relative to the start of the loop.  The executor returns
    each tick's log-likelihoods one tick later; a job is finished once its
    last step is enqueued and its result has reached the host."""
    sched = Scheduler(hbm_budget, max_slots, executor.footprint)
    pending = sorted(jobs, key=lambda j: j.arrival)
    t0 = clock()
    k = 0
    ticks = 0
    finishing = set()

    def check(lls):
        now = clock() - t0
        for i, v in lls.items():
            j = sched.active.get(i)
            if j is None or i in finishing or np.isfinite(v):
                continue
            executor.drop(j)
            sched.retire(j, now, failed=True, error="non-finite log-likelihood")

    def collect(wait=False):
        for j in executor.finished(wait):
            finishing.discard(j.job_id)
            now = clock() - t0
            if j.job_id not in sched.active:
                continue
            if not np.isfinite(j.result["loglik"]):
                j.result = None
                sched.retire(j, now, failed=True, error="non-finite log-likelihood")
            else:
                sched.retire(j, now)

    while k < len(pending) or not sched.idle:
        now = clock() - t0
        while k < len(pending) and pending[k].arrival <= now:
            sched.submit(pending[k], pending[k].arrival)
            k += 1
        for j in sched.admit(now):
            executor.admit(j)
        ids = sorted(i for i, j in sched.active.items() if i not in finishing)
        if ids:
            check(executor.tick(ids))
            ticks += 1
            for i in ids:
                j = sched.active.get(i)
                if j is None:
                    continue
                j.iters_done += 1
                if j.iters_done >= j.iterations:
                    finishing.add(i)
                    executor.finish(j)
            if on_tick:
                on_tick(ticks, sched)
        else:
            check(executor.flush())
        collect(wait=not ids)
        if not ids and not sched.active and k < len(pending):
            sleep(max(0.0, min(0.05, pending[k].arrival - (clock() - t0))))
    rep = ServeReport(jobs=sched.finished, wall=clock() - t0, ticks=ticks)
    return rep
