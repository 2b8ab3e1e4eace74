"""Device-buffer driver around the C ABI: holds one job's observation stack,
its prepared per-job data, the workspace and ping-pong iterates, and calls
srmra_em_step_prepared once per EM iteration.  No arithmetic happens here."""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import binding as B


@dataclass
class StepResult:
    x_new: torch.Tensor
    rho_new: torch.Tensor
    log_rho_new: torch.Tensor
    loglik: torch.Tensor


class EMJob:
    """One SR-MRA job resident on the GPU (observations, iterate, workspace)."""

    def __init__(self, y, K: int, sigma: float, x0, log_rho0, precision="fp32_mfma",
                 device="cuda", stream=None, centre: bool = True):
        y = torch.as_tensor(np.ascontiguousarray(y, dtype=np.float32)) if isinstance(y, np.ndarray) else y
        self.device = torch.device(device)
        self.y = y.to(self.device, dtype=torch.float32).contiguous()
        self.N, self.Ll = int(self.y.shape[0]), int(self.y.shape[1])
        self.K = int(K)
        self.Lh = self.K * self.Ll
        self.sigma = float(sigma)
        self.precision = B._prec(precision)
        self.stream = stream
        pb = B.srmra_prepared_bytes(self.N, self.Ll, self.K, self.precision)
        wb = B.srmra_em_step_workspace_bytes(self.N, self.Ll, self.K, self.precision)
        if pb == 0 or wb == 0:
            raise B.SrmraError(B.SRMRA_EUNSUPPORTED, "EMJob")
        self.prep = B.empty_bytes(pb, self.device)
        self.workspace = B.empty_bytes(wb, self.device)
        self.centre = bool(centre)
        B.srmra_prepare_observations_ex(self.y, self.N, self.Ll, self.K, self.precision,
                                        int(self.centre), self.prep, stream)
        f = dict(device=self.device, dtype=torch.float32)
        self.x = [torch.as_tensor(np.asarray(x0, np.float32)).to(**f).contiguous(),
                  torch.empty((self.Lh, self.Lh), **f)]
        self.log_rho = [torch.as_tensor(np.asarray(log_rho0, np.float32)).to(**f).contiguous(),
                        torch.empty((2, self.Lh), **f)]
        self.rho = torch.empty((2, self.Lh), **f)
        self.loglik = torch.empty(1, dtype=torch.float64, device=self.device)
        self.cur = 0
        self.iterations = 0

    def set_iterate(self, x, log_rho):
        self.x[self.cur].copy_(torch.as_tensor(np.asarray(x, np.float32)))
        self.log_rho[self.cur].copy_(torch.as_tensor(np.asarray(log_rho, np.float32)))

    def step(self, debug: Optional[dict] = None) -> StepResult:
        a, b = self.cur, 1 - self.cur
        if debug is None:
            B.srmra_em_step_prepared(self.y, self.prep, self.N, self.Ll, self.K, self.x[a],
                                     self.log_rho[a], self.sigma, self.x[b], self.rho,
                                     self.log_rho[b], self.loglik, self.precision, self.workspace,
                                     self.stream)
        else:
            B.srmra_em_step_debug(self.y, self.prep, self.N, self.Ll, self.K, self.x[a],
                                  self.log_rho[a], self.sigma, self.x[b], self.rho,
                                  self.log_rho[b], self.loglik, debug.get("ll_obs"),
                                  debug.get("b"), debug.get("c"), self.precision, self.workspace,
                                  self.stream)
        self.cur = b
        self.iterations += 1
        return StepResult(self.x[b], self.rho, self.log_rho[b], self.loglik)

    @property
    def x_current(self) -> torch.Tensor:
        return self.x[self.cur]

    @property
    def log_rho_current(self) -> torch.Tensor:
        return self.log_rho[self.cur]
