"""Inputs of the stored oracle results under tests/golden/ (shared by the
script that writes them and the tests that read them).  Inputs only: the
seeded synthetic workloads of paper_2204_04754_amd/synth.py, no EM arithmetic."""
from __future__ import annotations

import functools
import os

import numpy as np

from paper_2204_04754_amd import synth

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# one EM step each: the single-instance workload (Lh 64, K 2, Ll 32, N 1e5,
# sigma 1) from its seeded start, and the first 2000 observations of the
# precision-study workload (Lh 128, K 4, Ll 32, sigma 0.5 / 2) from the seeded
# start ("init") and from the true image and prior ("truth")
SUBSET_CASES = ["lh128_k4_n2000_s0.5_init", "lh128_k4_n2000_s0.5_truth",
                "lh128_k4_n2000_s2_init", "lh128_k4_n2000_s2_truth"]
FULL_CASES = ["lh64_k2_n100000_init"]
CASES = SUBSET_CASES + FULL_CASES
SUBSET_N = 2000


@functools.lru_cache(maxsize=2)
def _workload(name):
    return synth.workload(name)


def case_inputs(name: str):
    """(y, x, log_rho, sigma, K) of a named case, float32 as the GPU sees them."""
    if name == "lh64_k2_n100000_init":
        inst = _workload("lh64_k2_n100000")
        return inst.y, inst.x0, inst.log_rho0, inst.sigma, inst.K
    wl = {"s0.5": "lh128_k4_n200000_s0.5", "s2": "lh128_k4_n200000_s2"}
    _, _, _, sig, start = name.split("_")
    inst = _workload(wl[sig])
    y = np.ascontiguousarray(inst.y[:SUBSET_N])
    if start == "init":
        return y, inst.x0, inst.log_rho0, inst.sigma, inst.K
    lr = np.log(np.stack([inst.rho1, inst.rho2])).astype(np.float32)
    return y, inst.x_true, lr, inst.sigma, inst.K


def fingerprint(y, x, log_rho) -> np.ndarray:
    return np.array([np.asarray(y, np.float64).sum(), np.abs(np.asarray(y, np.float64)).sum(),
                     np.asarray(x, np.float64).sum(), np.asarray(log_rho, np.float64).sum()])


def load(name: str) -> dict:
    """The stored oracle result of a case; 'loglik' as a Python float."""
    with np.load(os.path.join(GOLDEN_DIR, name + ".npz")) as d:
        out = {k: d[k] for k in d.files}
    out["loglik"] = float(out["loglik"])
    return out
