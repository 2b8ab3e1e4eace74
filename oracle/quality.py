"""FP64 CPU oracle of the paper's reconstruction error.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP path.

error(x_hat) = min over all circular 2-D translations s of
||R_s x_hat - x||_F / ||x||_F (Sec. 5, the error measure; the model is
shift-invariant), with (R_s v)[m] = v[m - s] (reading R5 of em_oracle).
Ties in the minimum are broken by the lowest s1 * Lh + s2.
"""
from __future__ import annotations

import numpy as np


def shift_invariant_error(x_hat, x):
    """(error, (s1, s2)) by an explicit loop over the Lh^2 translations."""
    x_hat = np.asarray(x_hat, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    Lh = x.shape[0]
    best, arg = np.inf, (0, 0)
    for s1 in range(Lh):
        for s2 in range(Lh):
            d = np.sum((np.roll(x_hat, (s1, s2), axis=(0, 1)) - x) ** 2)   # x_hat[m - s]
            if d < best:
                best, arg = d, (s1, s2)
    return float(np.sqrt(best) / np.linalg.norm(x)), arg
