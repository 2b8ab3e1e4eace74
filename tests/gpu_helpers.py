"""Shared helpers of the GPU tests: run one step through the C ABI and compare
it with the FP64 oracle on the same FP32 inputs."""
import numpy as np
import torch

from oracle import em_oracle as O
from paper_2204_04754_amd import binding as B  # noqa: F401
from paper_2204_04754_amd import em
from tests.bounds import (U32, U_SPLIT, compare_step, ll_scale, obs_scale, rel,  # noqa: F401
                          unit_roundoff)

DEV = "cuda"


def gpu_step(y, x, log_rho, sigma, K, precision, debug=True, centre=True):
    """One EM step on the GPU from (x, log_rho); returns numpy results."""
    job = em.EMJob(y, K, sigma, x, log_rho, precision=precision, centre=centre)
    Lh = job.Lh
    dbg = None
    if debug:
        dbg = dict(ll_obs=torch.empty(job.N, dtype=torch.float32, device=DEV),
                   b=torch.empty((Lh, Lh), dtype=torch.float64, device=DEV),
                   c=torch.empty((Lh, Lh), dtype=torch.float64, device=DEV))
    r = job.step(dbg)
    torch.cuda.synchronize()
    out = dict(x_new=r.x_new.cpu().numpy().astype(np.float64),
               rho_new=r.rho_new.cpu().numpy().astype(np.float64),
               log_rho_new=r.log_rho_new.cpu().numpy().astype(np.float64),
               loglik=float(r.loglik.item()))
    if debug:
        out.update(ll_obs=dbg["ll_obs"].cpu().numpy().astype(np.float64),
                   b=dbg["b"].cpu().numpy(), c=dbg["c"].cpu().numpy())
    return out


def oracle_step(y, x, log_rho, sigma, K, centre=True):
    """The oracle's step with the magnitudes the element-wise bounds use."""
    return O.em_step(y, x, log_rho, sigma, K, return_details=True, return_magnitudes=True,
                     g=obs_scale(y, x, sigma, K, centre))


def check_step(y, x, log_rho, sigma, K, g, ref, precision, centre=True, **kw):
    """Compare one GPU step g with the oracle step ref (from oracle_step) on
    every element of x', rho', b, c and the per-observation terms (see
    tests/bounds.py); norm-wise relative error <= 1e-4 on x', rho', b and c.
    Returns the norm-wise (x, rho) errors."""
    r = compare_step(g, ref, x, y, precision, K, sigma, centre=centre, **kw)
    return r["x"], r["rho"]
