"""CPU checks of the stored oracle results under tests/golden/: each file
belongs to the inputs the seeded generator makes today, satisfies the
identities of one EM step (total posterior mass N, rho rows summing to 1,
x' = b / A where A > 0, |b| <= b_abs), and agrees with the current oracle on
some of its observations."""
import numpy as np
import pytest

from oracle import em_oracle as O
from tests.golden_cases import CASES, case_inputs, fingerprint, load


@pytest.mark.parametrize("case", CASES)
def test_golden_file(case):
    y, x, lr, sigma, K = case_inputs(case)
    gold = load(case)
    N = y.shape[0]
    assert int(gold["N"]) == N and int(gold["K"]) == K and float(gold["sigma"]) == sigma
    np.testing.assert_allclose(gold["fingerprint"], fingerprint(y, x, lr), rtol=1e-12, atol=0)
    assert abs(gold["c"].sum() - N) <= 1e-9 * N
    np.testing.assert_allclose(gold["rho_new"].sum(axis=1), 1.0, rtol=0, atol=1e-12)
    a = gold["a"]
    np.testing.assert_allclose(gold["x_new"][a > 0], gold["b"][a > 0] / a[a > 0], rtol=1e-15)
    assert np.all(np.abs(gold["b"]) <= gold["b_abs"] * (1 + 1e-12))
    assert np.all(gold["v0"] >= 0) and np.all(gold["c1"] >= 0) and np.all(gold["w_max"] <= 1.0)
    if len(gold["lse"]) == N:
        assert abs(gold["loglik"] - gold["lse"].sum()) <= 1e-12 * abs(gold["loglik"])
    # the current oracle gives the stored terms of the first stored observations
    j = gold["lse_idx"][:6]
    head = O.em_step(y[j], x, lr, sigma, K)
    np.testing.assert_allclose(head["lse"], gold["lse"][:6], rtol=1e-13)
