"""Shared helpers of the GPU tests: run one step through the C ABI and compare
it with the FP64 oracle on the same FP32 inputs."""
import numpy as np
import torch

from oracle import em_oracle as O
from paper_2204_04754_amd import binding as B
from paper_2204_04754_amd import em

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


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def score_scale(y, x, sigma, K):
    """Magnitude of the terms a = <y, R_t x_c>/sigma^2 whose FP32 rounding sets the
    attainable accuracy of the per-observation quantities: max_i ||y_i|| * max_c ||x_c|| / sigma^2,
    plus ||y_i||^2/(2 sigma^2), per observation."""
    y = np.asarray(y, np.float64)
    x = np.asarray(x, np.float64)
    xc = max(np.linalg.norm(x[a::K, b::K]) for a in range(K) for b in range(K))
    yn = np.linalg.norm(y.reshape(y.shape[0], -1), axis=1)
    return yn * xc / sigma ** 2 + yn ** 2 / (2 * sigma ** 2)


# FP32 unit roundoff
U32 = 2.0 ** -24


# residual of the BF16 hi + lo split: |v - hi - lo| <= 2^-17 |v|, so a split
# product carries a relative error of about 2^-16
U_SPLIT = 2.0 ** -16


def unit_roundoff(precision):
    return U_SPLIT if precision in ("bf16_split3", "bf16_split4") else U32


def check_step(y, x, log_rho, sigma, K, g, ref, x_tol=1e-4, rho_tol=1e-4, ll_c=16.0, u=None):
    """Compare one GPU step g with the oracle step ref.  Norm-wise relative
    error <= 1e-4 on x and rho (the accuracy target of the build); loglik and
    the per-observation terms within ll_c * u * (magnitude of the rounded
    terms), u the unit roundoff of the contraction (FP32, or the BF16 split)."""
    u = U32 if u is None else u
    xg, xr = g["x_new"], ref["x_new"]
    assert np.all(np.isfinite(xg))
    if "a" in ref:
        # x' = b / A per component (eq. x_EM).  A component whose total
        # posterior mass A_c is a small fraction of one observation is decided
        # by tail weights w << 1 only; the relative error of such a weight is
        # the full rounding error of its score a (eq. weights_EM), while that of
        # a dominant weight (w near 1) cancels against the log-sum-exp.  x'
        # there is not compared (b and c, the sufficient statistics, still
        # are): below 1e-3 of an observation for FP32 (score error ~1e-7, and
        # the weights underflow FP32), below one observation for the BF16
        # split (score error ~1e-3 at sigma 0.5).
        min_mass = 1e-3 if u <= U32 else 1.0
        keep = ref["a"] >= min_mass
        assert keep.mean() >= 0.5, "test input leaves most components without posterior mass"
        xg, xr = xg[keep], xr[keep]
    ex = rel(xg, xr)
    er = rel(g["rho_new"], ref["rho_new"])
    assert ex <= x_tol, f"x rel err {ex:.3e}"
    assert er <= rho_tol, f"rho rel err {er:.3e}"
    scale = score_scale(y, x, sigma, K)
    if "ll_obs" in g:
        d = np.abs(g["ll_obs"] - ref["lse"])
        assert np.all(d <= ll_c * u * (1 + scale)), f"ll_obs max err {d.max():.3e}"
    # the sum of the per-observation bounds (triangle inequality over the terms)
    assert abs(g["loglik"] - ref["loglik"]) <= ll_c * u * (len(scale) + scale.sum())
    return ex, er
