"""FP64 CPU oracle for one EM step of 2-D super-resolution MRA.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP path.

It follows the paper (Shani, Tirer, Giryes, Bendory, "Denoiser-based
projections for 2D super-resolution MRA") literally, in float64 NumPy, with an
explicit loop over every one of the Lh^2 circular shifts and no polyphase,
FFT or GEMM reformulation:

* forward operator P R_s x by direct index gather        -- Sec. 1, eq. (model_1)
* log-likelihood                                         -- Sec. 2, eq. (likelihood_EM)
* posterior weights w^{i,s}, normalised over s            -- Sec. 2, eq. (weights_EM)
* E-step objective Q                                      -- Sec. 2, eq. (Q)
* M-step for x:  A x = b                                  -- Sec. 2, eq. (x_EM)
* M-step for rho                                          -- Sec. 2, eq. (rho_EM)

Readings taken where the paper is silent or ambiguous (each is listed in the
design notes of the repository):

R1  P^{-1} in A and b is read as P^T (the zero-filling up-sampler) and
    R_s^{-1} = R_s^T; these are the normal equations of Q in x.
R2  Shifts are 0-based, s in Z_Lh, taken modulo Lh.
R3  With rho = rho1 rho2^T the rho M-step returns the two marginals of the
    numerator of eq. (rho_EM), each normalised by its denominator.
R4  s1 / rho1 act on axis 0 (rows) of the row-major image, s2 / rho2 on axis 1.
R5  (R_s x)[m] = x[m - s]; so y[n] = x[nK - s].
R6  loglik is eq. (likelihood_EM) literally (no Gaussian normalising constant),
    evaluated at the *input* parameters of the step.
R8  A pixel with zero total posterior mass keeps its previous value.
R9  sigma must be > 0; the sigma -> 0 limit is provided separately as a hard
    assignment (ties broken by the lowest s1*Lh + s2).
R10 log_rho is used as given (it need not be normalised); -inf entries allowed.
"""
from __future__ import annotations

import numpy as np


def _f64(a):
    return np.asarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# Forward operator, eq. (model_1)
# --------------------------------------------------------------------------
def shift_downsample_indices(Lh: int, K: int, s1: int, s2: int):
    """Row and column indices of P R_s x: y[n1, n2] = x[(n1 K - s1) mod Lh,
    (n2 K - s2) mod Lh] for n in {0..Ll-1}^2 (eq. (model_1), readings R2, R4, R5)."""
    Ll = Lh // K
    n = np.arange(Ll)
    return (n * K - s1) % Lh, (n * K - s2) % Lh


def forward(x, K: int, s1: int, s2: int) -> np.ndarray:
    """P R_s x for one shift, by explicit gather.  Returns [Ll, Ll]."""
    x = _f64(x)
    rows, cols = shift_downsample_indices(x.shape[0], K, s1, s2)
    return x[np.ix_(rows, cols)]


# --------------------------------------------------------------------------
# E-step: log-joint terms for every (observation, shift)
# --------------------------------------------------------------------------
def log_joint(Y, x, log_rho1, log_rho2, sigma: float, K: int) -> np.ndarray:
    """L[i, s1, s2] = log rho1[s1] + log rho2[s2] - ||y_i - P R_s x||^2 / (2 sigma^2).

    The summand of eq. (likelihood_EM) in log form; rho[s] = rho1[s1] rho2[s2]
    (Sec. 2, the diagonal matrix D_rho built from rho1 rho2^T).  Explicit loop over
    all Lh^2 shifts; float64 [N, Lh, Lh]."""
    Y = _f64(Y)
    x = _f64(x)
    lr1 = _f64(log_rho1)
    lr2 = _f64(log_rho2)
    if not sigma > 0:
        raise ValueError("sigma must be > 0 (reading R9)")
    N = Y.shape[0]
    Lh = x.shape[0]
    L = np.empty((N, Lh, Lh), dtype=np.float64)
    inv2s2 = 1.0 / (2.0 * sigma * sigma)
    for s1 in range(Lh):
        for s2 in range(Lh):
            v = forward(x, K, s1, s2)                       # P R_s x
            d = ((Y - v[None, :, :]) ** 2).sum(axis=(1, 2))  # ||y_i - P R_s x||^2
            L[:, s1, s2] = lr1[s1] + lr2[s2] - d * inv2s2
    return L


def logsumexp_over_shifts(L: np.ndarray) -> np.ndarray:
    """log sum_s exp(L[i, s]) per observation, with the usual max shift."""
    Lf = L.reshape(L.shape[0], -1)
    m = Lf.max(axis=1)
    safe = np.where(np.isfinite(m), m, 0.0)
    return safe + np.log(np.exp(Lf - safe[:, None]).sum(axis=1))


def log_likelihood(Y, x, log_rho1, log_rho2, sigma: float, K: int) -> float:
    """eq. (likelihood_EM), reading R6."""
    return float(logsumexp_over_shifts(log_joint(Y, x, log_rho1, log_rho2, sigma, K)).sum())


def posterior(L: np.ndarray, lse: np.ndarray) -> np.ndarray:
    """w^{i,s} = C^i rho[s] exp(-||y_i - P R_s x||^2 / 2 sigma^2) with
    sum_s w^{i,s} = 1 (eq. (weights_EM))."""
    return np.exp(L - lse[:, None, None])


# --------------------------------------------------------------------------
# M-step, eq. (x_EM) and eq. (rho_EM)
# --------------------------------------------------------------------------
def m_step_sums(Y, w: np.ndarray, K: int):
    """Accumulate b = sum_i sum_s w^{i,s} R_s^T P^T y_i and the diagonal of
    A = sum_i sum_s w^{i,s} R_s^T P^T P R_s (eq. (x_EM), reading R1), by
    scattering every weighted observation back to the pixels it was sampled
    from.  Returns (b [Lh, Lh], a [Lh, Lh], c [Lh, Lh]) with c[s] = sum_i w^{i,s}."""
    Y = _f64(Y)
    N, Lh = w.shape[0], w.shape[1]
    b = np.zeros((Lh, Lh))
    a = np.zeros((Lh, Lh))
    c = w.sum(axis=0)
    for s1 in range(Lh):
        for s2 in range(Lh):
            rows, cols = shift_downsample_indices(Lh, K, s1, s2)
            contrib = np.tensordot(w[:, s1, s2], Y, axes=(0, 0))  # sum_i w^{i,s} y_i
            b[np.ix_(rows, cols)] += contrib
            a[np.ix_(rows, cols)] += c[s1, s2]
    return b, a, c


def em_sums(Y, x, log_rho, sigma: float, K: int, chunk: int = 256,
            magnitudes: bool = False, g=None) -> dict:
    """The E-step and the sums of the M-step over a set of observations
    (Sec. 2, eq. (likelihood_EM), eq. (weights_EM) and the sums inside
    eq. (x_EM) and eq. (rho_EM)).

    Observations are processed in chunks; this is exact because the
    per-observation normaliser only involves that observation and every other
    quantity is a sum over observations.  Sums of disjoint sets of
    observations combine with merge_sums.  Returns dict(b, a, c [Lh, Lh],
    lse [N]) and, with magnitudes, the sizes that bound a computation of the
    same step at lower precision:
      b_abs  the back-projection of |y_i| (so |b| <= b_abs);
      w_max  per pixel, the largest single weight w^{i,s} among all (i, s)
             that sample it;
    and, given g (one non-negative scale per observation), the same sums with
    the weights w^{i,s} replaced by w^{i,s} (1 - w^{i,s}) g_i:
      v1     the back-projection of |y_i| with these weights,
      v0     the diagonal of A with these weights,
      c1     per shift, the sum over observations of these weights.
    If every log-joint term of observation i carries an error of at most
    g_i (in any direction), a weight normalised over s moves by a factor
    exp(e) with |e| <= 2 g_i (1 - w^{i,s}); v1, v0 and c1 are the first-order
    sizes of the resulting changes of b, A and c."""
    Y = _f64(Y)
    x = _f64(x)
    log_rho = _f64(log_rho)
    N = Y.shape[0]
    Lh = x.shape[0]
    if Lh % K != 0 or Y.shape[1:] != (Lh // K, Lh // K):
        raise ValueError("shape mismatch")
    b = np.zeros((Lh, Lh))
    a = np.zeros((Lh, Lh))
    c = np.zeros((Lh, Lh))
    lse = np.empty(N)
    out = dict(b=b, a=a, c=c, lse=lse)
    if magnitudes:
        out.update(b_abs=np.zeros((Lh, Lh)), w_max=np.zeros((Lh, Lh)))
        if g is not None:
            g = _f64(g)
            out.update(v1=np.zeros((Lh, Lh)), v0=np.zeros((Lh, Lh)), c1=np.zeros((Lh, Lh)))
    for lo in range(0, N, chunk):
        hi = min(N, lo + chunk)
        L = log_joint(Y[lo:hi], x, log_rho[0], log_rho[1], sigma, K)
        lse[lo:hi] = logsumexp_over_shifts(L)
        w = posterior(L, lse[lo:hi])
        bb, aa, cc = m_step_sums(Y[lo:hi], w, K)
        b += bb
        a += aa
        c += cc
        if magnitudes:
            out["b_abs"] += m_step_sums(np.abs(Y[lo:hi]), w, K)[0]
            wm = w.max(axis=0)
            w_max = out["w_max"]
            for s1 in range(Lh):
                for s2 in range(Lh):
                    rows, cols = shift_downsample_indices(Lh, K, s1, s2)
                    w_max[np.ix_(rows, cols)] = np.maximum(w_max[np.ix_(rows, cols)], wm[s1, s2])
            if g is not None:
                wg = w * (1.0 - w) * g[lo:hi, None, None]
                v1, v0, c1 = m_step_sums(np.abs(Y[lo:hi]), wg, K)
                out["v1"] += v1
                out["v0"] += v0
                out["c1"] += c1
    return out


def merge_sums(parts) -> dict:
    """Combine em_sums of consecutive disjoint sets of observations (in order):
    the sums add, w_max takes the larger value, lse concatenates."""
    out = {k: parts[0][k].copy() for k in parts[0]}
    for p in parts[1:]:
        for k in ("b", "a", "c", "b_abs", "v1", "v0", "c1"):
            if k in out:
                out[k] += p[k]
        if "w_max" in out:
            out["w_max"] = np.maximum(out["w_max"], p["w_max"])
    out["lse"] = np.concatenate([p["lse"] for p in parts])
    return out


def em_finish(x, sums: dict) -> dict:
    """The M-step from the sums: eq. (x_EM) and eq. (rho_EM), and the
    log-likelihood eq. (likelihood_EM) at the input parameters (reading R6)."""
    x = _f64(x)
    b, a, c = sums["b"], sums["a"], sums["c"]
    # eq. (x_EM): A is diagonal here (reading R1), so A x = b is solved per pixel.
    x_new = np.where(a > 0, b / np.where(a > 0, a, 1.0), x)     # reading R8
    # eq. (rho_EM) with the product form (reading R3).
    tot = c.sum()
    rho_new = np.stack([c.sum(axis=1) / tot, c.sum(axis=0) / tot])
    return dict(x_new=x_new, rho_new=rho_new, loglik=float(sums["lse"].sum()), lse=sums["lse"])


def em_step(Y, x, log_rho, sigma: float, K: int, chunk: int = 256,
            return_details: bool = False, return_magnitudes: bool = False, g=None):
    """One unprojected EM step from theta_t = (x, rho) (Sec. 2, EM paragraph).

    Y: [N, Ll, Ll]; x: [Lh, Lh]; log_rho: [2, Lh] (row 0 = log rho1 on axis 0,
    row 1 = log rho2 on axis 1).

    Returns dict(x_new [Lh,Lh], rho_new [2,Lh], loglik, lse [N]) and, with
    return_details, also b, a, c (see m_step_sums); with return_magnitudes
    also the magnitudes of em_sums (v1, v0, c1 when g is given)."""
    sums = em_sums(Y, x, log_rho, sigma, K, chunk=chunk, magnitudes=return_magnitudes, g=g)
    out = em_finish(x, sums)
    if return_details:
        out.update(b=sums["b"], a=sums["a"], c=sums["c"])
    if return_magnitudes:
        out.update({k: sums[k] for k in ("b_abs", "w_max", "v1", "v0", "c1") if k in sums})
    return out


# --------------------------------------------------------------------------
# Pieces used only by the oracle's own pins
# --------------------------------------------------------------------------
def q_function(Y, x, log_rho1, log_rho2, w, sigma: float, K: int) -> float:
    """eq. (Q): sum_i sum_s w^{i,s} (log rho[s] - ||y_i - P R_s x||^2 / (2 sigma^2))."""
    L = log_joint(Y, x, log_rho1, log_rho2, sigma, K)
    wl = np.where(w > 0, w * L, 0.0)
    return float(wl.sum())


def dense_operators(Lh: int, K: int):
    """Explicit matrices for tiny sizes: P [Ll^2, Lh^2] (picks every K-th pixel in
    both axes) and a function s -> R_s [Lh^2, Lh^2] with (R_s x)[m] = x[m - s]
    (eq. (model_1), reading R5).  Vectorisation is row-major."""
    Ll = Lh // K
    P = np.zeros((Ll * Ll, Lh * Lh))
    for n1 in range(Ll):
        for n2 in range(Ll):
            P[n1 * Ll + n2, (n1 * K) * Lh + n2 * K] = 1.0

    def R(s1: int, s2: int) -> np.ndarray:
        M = np.zeros((Lh * Lh, Lh * Lh))
        for m1 in range(Lh):
            for m2 in range(Lh):
                M[m1 * Lh + m2, ((m1 - s1) % Lh) * Lh + (m2 - s2) % Lh] = 1.0
        return M

    return P, R


def dense_x_step(Y, w, K: int) -> np.ndarray:
    """eq. (x_EM) as printed, for tiny sizes: form A = sum w R_s^{-1} P^{-1} P R_s and
    b = sum w R_s^{-1} P^{-1} y_i as dense matrices (with P^{-1} := P^T and
    R_s^{-1} computed by numpy.linalg.inv) and solve A x = b with
    numpy.linalg.solve.  Returns [Lh, Lh]."""
    Y = _f64(Y)
    N, Lh = w.shape[0], w.shape[1]
    P, R = dense_operators(Lh, K)
    A = np.zeros((Lh * Lh, Lh * Lh))
    bvec = np.zeros(Lh * Lh)
    Yv = Y.reshape(N, -1)
    for s1 in range(Lh):
        for s2 in range(Lh):
            Rs = R(s1, s2)
            Rinv = np.linalg.inv(Rs)
            M = Rinv @ P.T
            ws = w[:, s1, s2]
            A += ws.sum() * (M @ P @ Rs)
            bvec += M @ (Yv.T @ ws)
    return np.linalg.solve(A, bvec).reshape(Lh, Lh)


def hard_assignment_posterior(Y, x, log_rho1, log_rho2, K: int) -> np.ndarray:
    """sigma -> 0 limit of eq. (weights_EM) (reading R9): all mass on the shifts
    with the smallest distance among those with rho[s] > 0, split in proportion
    to rho; returns the argmax shift index s1*Lh + s2 per observation (lowest
    index on ties)."""
    Y = _f64(Y)
    x = _f64(x)
    N = Y.shape[0]
    Lh = x.shape[0]
    d = np.empty((N, Lh, Lh))
    for s1 in range(Lh):
        for s2 in range(Lh):
            v = forward(x, K, s1, s2)
            d[:, s1, s2] = ((Y - v[None]) ** 2).sum(axis=(1, 2))
    allowed = np.isfinite(_f64(log_rho1))[:, None] & np.isfinite(_f64(log_rho2))[None, :]
    d = np.where(allowed[None], d, np.inf)
    return d.reshape(N, -1).argmin(axis=1)
