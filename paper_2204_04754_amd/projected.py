"""Projected EM (Alg. 2) on the device: F EM steps, then the projection
x <- D(x, s_t), then s_t <- 2^(-1/10) s_t (eq. decaying_function), repeated.
D is the library's Gaussian-smoothing stand-in for the denoiser
(srmra_project_gaussian) or the identity.  The noise level s_t lives in device
memory, so T outer iterations can be captured as one HIP graph.  Marshalling
and buffer ownership only: every step runs the library's kernels."""
from __future__ import annotations

import torch

from . import binding as B
from .em import EMJob

DECAY = 2.0 ** -0.1


class ProjectedEM:
    def __init__(self, y, K: int, sigma: float, x0, log_rho0, precision="fp32_mfma", F: int = 5,
                 sigma1: float = 1.0, decay: float = DECAY, projection: str = "gaussian",
                 device="cuda", stream=None, centre: bool = True):
        if projection not in ("gaussian", "identity"):
            raise ValueError("projection must be 'gaussian' or 'identity'")
        self.job = EMJob(y, K, sigma, x0, log_rho0, precision=precision, device=device,
                         stream=stream, centre=centre)
        self.F, self.decay, self.projection, self.stream = int(F), float(decay), projection, stream
        self.sigma_state = torch.full((1,), float(sigma1), dtype=torch.float32, device=self.job.device)
        self.pws = B.empty_bytes(B.srmra_project_workspace_bytes(self.job.Lh), self.job.device)
        self.outer_done = 0

    def project(self):
        x = self.job.x[self.job.cur]
        if self.projection == "gaussian":
            B.srmra_project_gaussian(x, x, self.job.Lh, self.sigma_state, self.decay, self.pws,
                                     self.stream)

    def outer(self):
        """One outer iteration of Alg. 2 (enqueued on the stream)."""
        for _ in range(self.F):
            self.job.step()
        self.project()
        self.outer_done += 1

    def capture(self, outer_iterations: int) -> torch.cuda.CUDAGraph:
        """`outer_iterations` outer iterations as one graph; F * outer_iterations
        must be even (ping-pong iterates).  Replaying advances the state by
        that many outer iterations, the noise level included."""
        if (self.F * outer_iterations) % 2:
            raise ValueError("F * outer_iterations must be even (ping-pong iterates)")
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream(device=self.job.device)
        s.wait_stream(torch.cuda.current_stream())
        saved = self.job.stream, self.stream
        with torch.cuda.stream(s):
            self.job.stream = self.stream = torch.cuda.current_stream()
            with torch.cuda.graph(g, stream=s):
                for _ in range(outer_iterations):
                    self.outer()
        self.job.stream, self.stream = saved
        self.outer_done -= outer_iterations   # counted when replayed
        torch.cuda.current_stream().wait_stream(s)
        return g

    @property
    def x(self) -> torch.Tensor:
        return self.job.x_current
