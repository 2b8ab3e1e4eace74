"""Write the stored expected values of one EM step under tests/golden/.

    python tests/golden/make_goldens.py [--procs 8] [--only NAME]

Every value written here comes from the FP64 oracle (oracle/em_oracle.py) on
the seeded synthetic inputs of paper_2204_04754_amd/synth.py; nothing else is
called.  The observations are split into consecutive parts that worker
processes run through oracle.em_sums, merged in order with oracle.merge_sums
and finished with oracle.em_finish (exact up to rounding order: every M-step
quantity is a sum over observations).

Cases (one EM step each, from the stated start):
  lh64_k2_n100000_init      the single-instance workload (Lh 64, K 2, Ll 32,
                            N 100000, sigma 1) from its seeded x0 and uniform rho
  lh128_k4_n2000_s0.5_init  the first 2000 observations of the precision-study
  lh128_k4_n2000_s0.5_truth workload (Lh 128, K 4, Ll 32, sigma 0.5 and 2),
  lh128_k4_n2000_s2_init    from the seeded x0 / uniform rho ("init") and from
  lh128_k4_n2000_s2_truth   the true image and prior ("truth")

Each file holds x_new, rho_new, b, a, c, the magnitudes b_abs, w_max, v1,
v0, c1 (oracle.em_sums with g = tests.bounds.obs_scale, the scale of each
observation's centred score), loglik, the
per-observation log-sum-exp terms (all of them, or a seeded sample of 4096
with their indices where N is larger), and a fingerprint of the inputs
(float64 sums of y and x) that the tests check before comparing.
"""
from __future__ import annotations

import argparse
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
os.environ.setdefault("OMP_NUM_THREADS", "1")

import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import em_oracle as O  # noqa: E402
from paper_2204_04754_amd import synth  # noqa: E402
from tests.bounds import obs_scale  # noqa: E402
from tests.golden_cases import CASES, case_inputs, fingerprint  # noqa: E402

LSE_SAMPLE = 4096


def _part(args):
    y, x, lr, sigma, K, g = args
    return O.em_sums(y, x, lr, sigma, K, magnitudes=True, g=g)


def make(name: str, procs: int) -> str:
    y, x, lr, sigma, K = case_inputs(name)
    N = y.shape[0]
    t = time.perf_counter()
    bounds = np.linspace(0, N, min(procs * 4, N) + 1).astype(int)
    g = obs_scale(y, x, sigma, K)
    work = [(y[a:b], x, lr, sigma, K, g[a:b]) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    with ProcessPoolExecutor(procs) as ex:
        parts = list(ex.map(_part, work))
    sums = O.merge_sums(parts)
    out = O.em_finish(x, sums)
    lse = sums["lse"]
    if N > LSE_SAMPLE:
        idx = np.sort(np.random.default_rng(N).choice(N, LSE_SAMPLE, replace=False))
    else:
        idx = np.arange(N)
    path = os.path.join(HERE, name + ".npz")
    np.savez_compressed(path, x_new=out["x_new"], rho_new=out["rho_new"], b=sums["b"], a=sums["a"],
                        c=sums["c"], b_abs=sums["b_abs"], w_max=sums["w_max"], v1=sums["v1"],
                        v0=sums["v0"], c1=sums["c1"],
                        loglik=np.float64(out["loglik"]), lse=lse[idx], lse_idx=idx,
                        N=np.int64(N), K=np.int64(K), sigma=np.float64(sigma),
                        fingerprint=fingerprint(y, x, lr))
    print(f"{name}: {time.perf_counter() - t:.0f} s -> {os.path.relpath(path, ROOT)}", flush=True)
    return path


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    ap.add_argument("--only", default="")
    a = ap.parse_args()
    for name in CASES:
        if a.only and name != a.only:
            continue
        make(name, a.procs)


if __name__ == "__main__":
    main()
