"""FP64 CPU oracle of the empirical moments of the observations.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP path.

eq. (empiric_MOM): M1 = (1/N) sum_i y_i and M2 = (1/N) sum_i y_i y_i^T, with
y_i vectorised row-major (pixel index l = n1 Ll + n2), M2 of size
Ll^2 x Ll^2.  The sum over observations is a library matrix product.
"""
from __future__ import annotations

import numpy as np


def empirical_moments(Y):
    """(M1 [Ll^2], M2 [Ll^2, Ll^2]) of eq. (empiric_MOM), in float64."""
    Y = np.asarray(Y, dtype=np.float64)
    V = Y.reshape(Y.shape[0], -1)
    return V.mean(axis=0), (V.T @ V) / V.shape[0]
