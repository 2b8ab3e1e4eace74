"""Error bounds for comparing one EM step computed in FP32 (or the BF16
split, or through 2-D DFTs) with the FP64 oracle, element by element.

Pure NumPy: used by the GPU parity tests and by the script that writes the
stored oracle results (for the per-observation scale g), never by the
library.

Model of the errors (Sec. 2, eq. weights_EM, eq. x_EM, eq. rho_EM):

* Every log-joint term a_is = <y_i, P R_s x>/sigma^2 + beta_s of observation
  i carries an error of at most D_i = C_LL u' g_i, where
  g_i = 1 + ||y_i - mu|| max_c ||x_c - mu|| / sigma^2 is the size of the
  centred score (mu the offset the library takes off y and x), u' the unit of
  the contraction (2^-24 in FP32; 2^-16 for the BF16 split, whose hi + lo
  residual is 2^-18 per operand) and C_LL the constant that the per-observation
  log-likelihood terms are held to (the same bound, asserted on every term).
* A weight normalised over the shifts then moves by a factor exp(e) with
  |e| <= 2 D_i (1 - w_is) (the normaliser's error is a w-weighted mean of the
  terms' errors, so it cancels against a dominant term) plus the FP32
  rounding of the weight's exponent (a - m_i) - l_i, formed from the largest
  term m_i and l_i = log sum exp(a - m_i) so that no large number is
  rounded: |a - m_i| stays below about 88 for any weight FP32 can hold, so
  this and the exponential's rounding are below 100 u.
* The sums b = sum w y, c_s = sum_i w_is and A are accumulated in FP32 per
  chunk of observations and in FP64 across chunks: a relative error of at most
  KAPPA = e_prod + 2 sqrt(n) 2^-24 + 100 * 2^-24 of the sum of absolute terms
  (random-walk growth over n terms; e_prod the relative error of one product
  of the back-projection: 0 in FP32, 1.5 * 2^-17 for the 3-product split,
  2^-17 with four products, 4 log2(Ll^2) 2^-24 through the DFTs; the last
  term the weights' own rounding above).
* A weight below the FP32 normal range may be lost entirely: an absolute
  error of up to ETA = 2^-126 per weight, n_c = N Ll^2 weights per pixel.
* Through the DFTs (the FFT route) the back-projection's error is norm-wise,
  not relative to each element's own terms: a correlation formed as
  IDFT(Y conj(W)) has ||error||_2 <= e_prod ||w||_1 ||y||_2 (each transform's
  error is relative in the 2-norm, and |W| <= ||w||_1 at every frequency), so
  every element of b_c also gets e_prod max_i ||y_i - mu|| m_c, m_c the
  component's posterior mass (taken as its largest over the components).

The oracle returns the first-order sums of the weight errors (v1, v0, c1 for
the scale g, b_abs, w_max), from which every element gets its own bound.
"""
from __future__ import annotations

import math

import numpy as np

U32 = 2.0 ** -24
U_SPLIT = 2.0 ** -16
C_LL = 16.0
ETA = 2.0 ** -126
# a pixel whose every weight lies below this (half the smallest FP32 subnormal,
# with room for the score's error) gets no weight in FP32 at all: A = 0 on the
# GPU and x' keeps x (reading R8 at FP32 range)
W_UNDERFLOW = 2.0 ** -151


def unit_roundoff(precision: str) -> float:
    return U_SPLIT if precision in ("bf16_split3", "bf16_split4") else U32


def product_error(precision: str, Ll: int) -> float:
    if precision == "bf16_split3":
        return 1.5 * 2.0 ** -17
    if precision == "bf16_split4":
        return 2.0 ** -17
    if precision == "fp32_fft":
        return 4.0 * math.log2(Ll * Ll) * U32
    return 0.0


def centre_offset(y, centre: bool = True) -> float:
    """The offset the library takes off y and x: the FP64 mean of every
    observation pixel, rounded to FP32."""
    return float(np.float32(np.asarray(y, np.float64).mean())) if centre else 0.0


def obs_scale(y, x, sigma: float, K: int, centre: bool = True) -> np.ndarray:
    """g_i = 1 + ||y_i - mu|| max_c ||x_c - mu|| / sigma^2 per observation."""
    mu = centre_offset(y, centre)
    y = np.asarray(y, np.float64) - mu
    x = np.asarray(x, np.float64) - mu
    xc = max(np.linalg.norm(x[a::K, b::K]) for a in range(K) for b in range(K))
    yn = np.linalg.norm(y.reshape(y.shape[0], -1), axis=1)
    return 1.0 + yn * xc / sigma ** 2


def ll_scale(y, x, sigma: float, K: int) -> np.ndarray:
    """Magnitude of the rounded terms of one per-observation log-likelihood
    term: ||y_i|| max_c ||x_c|| / sigma^2 + ||y_i||^2 / (2 sigma^2)."""
    y = np.asarray(y, np.float64)
    x = np.asarray(x, np.float64)
    xc = max(np.linalg.norm(x[a::K, b::K]) for a in range(K) for b in range(K))
    yn = np.linalg.norm(y.reshape(y.shape[0], -1), axis=1)
    return yn * xc / sigma ** 2 + yn ** 2 / (2 * sigma ** 2)


def rel(a, b) -> float:
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def elementwise_bounds(ref: dict, x_in, y, precision: str, K: int, centre: bool = True) -> dict:
    """Per-element bounds on |gpu - oracle| for x', rho', b and c, from the
    oracle's magnitudes (ref must carry a, c, b_abs, w_max, v1, v0, c1 computed
    with g = obs_scale(...)) and the error model of the module docstring."""
    y = np.asarray(y)
    N, Ll = y.shape[0], y.shape[1]
    u = unit_roundoff(precision)
    n_c = float(N) * Ll * Ll
    kappa = product_error(precision, Ll) + 2.0 * math.sqrt(n_c) * U32 + 100.0 * U32
    d2 = 2.0 * C_LL * u
    mu = abs(centre_offset(y, centre))
    ymax = float(np.abs(np.asarray(y, np.float64)).max())
    A, xr = ref["a"], ref["x_new"]
    xm = np.abs(xr - centre_offset(y, centre))
    fft_b = 0.0
    if precision == "fp32_fft":
        Lh = K * Ll
        comp = (-np.arange(Lh)) % K
        mass = max(float(ref["c"][np.ix_(comp == a, comp == b)].sum()) for a in range(K) for b in range(K))
        yc = np.asarray(y, np.float64) - centre_offset(y, centre)
        fft_b = product_error(precision, Ll) * float(np.linalg.norm(yc.reshape(N, -1), axis=1).max()) * mass
    with np.errstate(divide="ignore", invalid="ignore"):
        num = (d2 * (ref["v1"] + (mu + xm) * ref["v0"]) + kappa * (ref["b_abs"] + (mu + xm) * A)
               + n_c * ETA * (ymax + mu + xm) + fft_b)
        tol_x = np.where(A > 0, num / A, np.inf) + 4.0 * U32 * (np.abs(xr) + mu)
    tol_b = (d2 * (ref["v1"] + 2 * mu * ref["v0"]) + kappa * (ref["b_abs"] + 2 * mu * A)
             + n_c * ETA * (ymax + 2 * mu) + fft_b)
    tol_c = d2 * ref["c1"] + kappa * ref["c"] + N * ETA
    tot = ref["c"].sum()
    rho = ref["rho_new"]
    tc = tol_c.sum()
    tol_rho = np.stack([(tol_c.sum(axis=1) + rho[0] * tc) / tot, (tol_c.sum(axis=0) + rho[1] * tc) / tot])
    tol_rho += 4.0 * U32 * rho
    # pixels whose mass FP32 may lose to underflow by more than 1e-6 relative
    range_limited = n_c * ETA > 1e-6 * A
    underflow = ref["w_max"] < W_UNDERFLOW
    # the first-order part of the b and c bounds: the weights' logit error
    # alone (zero for exact logits)
    first_b = d2 * (ref["v1"] + 2 * mu * ref["v0"])
    first_c = d2 * ref["c1"]
    return dict(x=tol_x, b=tol_b, c=tol_c, rho=tol_rho, range_limited=range_limited,
                underflow=underflow, first_b=first_b, first_c=first_c)


def compare_step(g: dict, ref: dict, x_in, y, precision: str, K: int, sigma: float,
                 centre: bool = True, x_tol: float = 1e-4, rho_tol: float = 1e-4,
                 bc_tol: float = 1e-4, ll_c: float = C_LL, lse_idx=None) -> dict:
    """Assert the GPU step g against the oracle step ref on every element.

    * x': every pixel within its element-wise bound; a pixel with no FP32
      weight at all (every weight below W_UNDERFLOW) keeps x exactly (reading
      R8 at FP32 range); norm-wise relative error <= x_tol over all pixels
      except those whose mass is within reach of FP32 underflow (the
      underflowed ones are compared with x, kept).
    * rho', b, c: every element within its bound; rho' norm-wise <= rho_tol;
      b and c norm-wise <= bc_tol plus the norm of the first-order part of
      their bound (the logits' error), relative.
    * per-observation log-likelihood terms within ll_c u' (1 + size of the
      rounded terms); loglik within the sum of those bounds.
    Returns the measured errors."""
    x_in = np.asarray(x_in, np.float64)
    tb = elementwise_bounds(ref, x_in, y, precision, K, centre)
    xg, xr = np.asarray(g["x_new"], np.float64), ref["x_new"]
    assert np.all(np.isfinite(xg)), "non-finite x'"
    uf = tb["underflow"]
    assert np.array_equal(xg[uf], x_in[uf]), "pixels with no FP32 weight must keep x"
    dx = np.abs(xg - xr)
    bad = ~uf & ~(dx <= tb["x"])
    assert not bad.any(), (f"x' off its element-wise bound at {int(bad.sum())} pixels: "
                           f"max |d| {dx[bad].max():.3e}, bound there {tb['x'][bad][np.argmax(dx[bad])]:.3e}")
    expect = np.where(uf, x_in, xr)
    keep = ~tb["range_limited"] | uf
    ex = rel(xg[keep], expect[keep])
    assert ex <= x_tol, f"x rel err {ex:.3e}"
    rg = np.asarray(g["rho_new"], np.float64)
    drho = np.abs(rg - ref["rho_new"])
    assert np.all(drho <= tb["rho"]), f"rho' off its bound: max ratio {np.max(drho / tb['rho']):.3e}"
    er = rel(rg, ref["rho_new"])
    assert er <= rho_tol, f"rho rel err {er:.3e}"
    out = dict(x=ex, rho=er, x_max_ratio=float(np.max(np.where(uf, 0, dx / tb["x"]))),
               x_pixels_range_limited=int((tb["range_limited"] & ~uf).sum()),
               x_pixels_underflow=int(uf.sum()))
    if "b" in g:
        db = np.abs(np.asarray(g["b"]) - ref["b"])
        dc = np.abs(np.asarray(g["c"]) - ref["c"])
        assert np.all(db <= tb["b"]), f"b off its bound: max ratio {np.max(db / tb['b']):.3e}"
        assert np.all(dc <= tb["c"]), f"c off its bound: max ratio {np.max(dc / tb['c']):.3e}"
        out.update(b=rel(g["b"], ref["b"]), c=rel(g["c"], ref["c"]))
        # b and c are sums of weights: beside the 1e-4 of the outputs they
        # carry the first-order effect of the logits' error bound (a weight
        # moves by up to 2 D_i (1 - w); x' and rho', ratios of these sums, are
        # held to 1e-4 alone)
        gb = bc_tol + float(np.linalg.norm(tb["first_b"]) / np.linalg.norm(ref["b"]))
        gc = bc_tol + float(np.linalg.norm(tb["first_c"]) / np.linalg.norm(ref["c"]))
        assert out["b"] <= gb, f"b rel err {out['b']:.3e} (gate {gb:.3e})"
        assert out["c"] <= gc, f"c rel err {out['c']:.3e} (gate {gc:.3e})"
    u = unit_roundoff(precision)
    xin32 = np.asarray(x_in, np.float32)
    scale = ll_scale(y, xin32, sigma, K)
    if "ll_obs" in g:
        llg = np.asarray(g["ll_obs"], np.float64)
        if lse_idx is not None:
            llg = llg[lse_idx]
            sc = scale[lse_idx]
        else:
            sc = scale
        d = np.abs(llg - ref["lse"])
        assert np.all(d <= ll_c * u * (1 + sc)), f"ll_obs max err {d.max():.3e}"
        out["lse_max"] = float(d.max())
    assert abs(g["loglik"] - ref["loglik"]) <= ll_c * u * (len(scale) + scale.sum())
    out["loglik"] = abs(g["loglik"] - ref["loglik"]) / abs(ref["loglik"])
    return out
