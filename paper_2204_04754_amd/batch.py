"""Device-buffer driver for the batched form (srmra_plan_* in the C ABI): many
independent SR-MRA instances advanced together, one persistent launch per pass
and (L_low, form) class per EM step, optionally captured as a HIP graph of
several iterations.  Marshalling and buffer ownership only."""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np
import torch

from . import binding as B


def table_form(table, precision: int, L_low: int, K: int) -> Optional[int]:
    """The form the first matching entry of a tuning table gives (L_low, K), or None."""
    for t in table or ():
        if B._prec(t["precision"]) == precision and int(t["L_low"]) == L_low and int(t["K"]) == K:
            return B._prec(t["form"])
    return None


def prepare(e: dict, form: int, stream=None) -> None:
    """(Re)prepare problem e's observations for the form it will run in (the FFT
    route keeps the observations' DFTs, the BF16 split its operand planes; a
    BF16 preparation also serves FP32 MFMA)."""
    pb = B.srmra_prepared_bytes(e["N"], e["L_low"], e["K"], form)
    if pb == 0:
        raise B.SrmraError(B.SRMRA_EUNSUPPORTED, "prepare")
    e["prep"] = B.empty_bytes(pb, e["y"].device)
    B.srmra_prepare_observations(e["y"], e["N"], e["L_low"], e["K"], form, e["prep"], stream)
    e["prep_form"] = form


class BatchedEM:
    def __init__(self, instances: Sequence[dict], precision="fp32_mfma", device="cuda",
                 stream=None, tuning=None, fft=False):
        """instances: dicts with y [N][Ll][Ll], K, sigma, x0 [Lh][Lh], log_rho0 [2][Lh]
        (NumPy or torch).  tuning: None (library defaults), a list of
        srmra_tuning entries, or "auto" (run the autotuner on this batch; with
        fft, the FFT route is one of its candidates).  Each problem is prepared
        for the form its class runs in."""
        self.device = torch.device(device)
        self.precision = B._prec(precision)
        self.stream = stream
        self.inst: List[dict] = []
        f = dict(device=self.device, dtype=torch.float32)
        table = list(tuning) if tuning and tuning != "auto" else None
        for d in instances:
            y = d["y"]
            y = torch.as_tensor(np.ascontiguousarray(y, np.float32)) if isinstance(y, np.ndarray) else y
            y = y.to(self.device, torch.float32).contiguous()
            N, Ll = int(y.shape[0]), int(y.shape[1])
            K = int(d["K"])
            Lh = K * Ll
            form = table_form(table, self.precision, Ll, K)
            if form is None:
                form = B.srmra_plan_form(self.precision, Ll)
            if form < 0:
                raise B.SrmraError(B.SRMRA_EUNSUPPORTED, "BatchedEM")
            e = dict(y=y, N=N, L_low=Ll, K=K, Lh=Lh, sigma=float(d["sigma"]), form=form,
                     x=torch.as_tensor(np.asarray(d["x0"], np.float32)).to(**f).contiguous(),
                     x_new=torch.empty((Lh, Lh), **f),
                     log_rho=torch.as_tensor(np.asarray(d["log_rho0"], np.float32)).to(**f).contiguous(),
                     log_rho_new=torch.empty((2, Lh), **f),
                     rho_new=torch.empty((2, Lh), **f),
                     loglik=torch.empty(1, dtype=torch.float64, device=self.device))
            prepare(e, form, stream)
            self.inst.append(e)
        self.tuning, self.tune_report, self.tune_seconds = None, [], 0.0
        if tuning == "auto":
            import time

            from .autotune import tune
            t0 = time.perf_counter()
            self.tuning, self.tune_report = tune(self.inst, self.precision, stream=stream, fft=fft)
            self.tune_seconds = time.perf_counter() - t0
            for e in self.inst:   # a class the tuner sent to (or from) the FFT route
                form = table_form(self.tuning, self.precision, e["L_low"], e["K"])
                if form is not None and (form == B.FP32_FFT) != (e["prep_form"] == B.FP32_FFT):
                    prepare(e, form, stream)
                    e["form"] = form
        elif tuning:
            self.tuning = list(tuning)
        self.plan = B.Plan(self.inst, self.precision, tuning=self.tuning)
        self.workspace = B.empty_bytes(self.plan.workspace_bytes, self.device)
        self.plan.upload(self.workspace, stream)
        self.executions = 0

    def step(self):
        """One EM step of every instance (enqueued on the stream)."""
        self.plan.execute(self.workspace, self.stream)
        self.executions += 1

    def reset_parity(self):
        self.plan.upload(self.workspace, self.stream)
        self.executions = 0

    def current(self, i: int):
        """(x, log_rho) of instance i after the executions so far."""
        e = self.inst[i]
        if self.executions % 2 == 0:
            return e["x"], e["log_rho"]
        return e["x_new"], e["log_rho_new"]

    def results(self, i: int) -> dict:
        e = self.inst[i]
        x, lr = self.current(i)
        return dict(x_new=x.cpu().numpy().astype(np.float64),
                    log_rho_new=lr.cpu().numpy().astype(np.float64),
                    rho_new=e["rho_new"].cpu().numpy().astype(np.float64),
                    loglik=float(e["loglik"].item()))

    def capture(self, iterations: int) -> torch.cuda.CUDAGraph:
        """Capture `iterations` (even) EM steps of every instance as one graph.
        The plan must be at parity 0; replaying the graph advances every
        instance by `iterations` steps."""
        if iterations % 2:
            raise ValueError("capture an even number of iterations (ping-pong buffers)")
        if self.plan.parity() != 0:
            raise RuntimeError("capture must start at parity 0")
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                for _ in range(iterations):
                    self.plan.execute(self.workspace, torch.cuda.current_stream())
        torch.cuda.current_stream().wait_stream(s)
        return g

    @property
    def pairs_per_step(self) -> int:
        return sum(e["N"] * e["Lh"] * e["Lh"] for e in self.inst)
