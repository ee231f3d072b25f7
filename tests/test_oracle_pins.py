"""The FP64 oracle against brute force, explicit matrices, special cases,
optimality conditions and values printed in the paper (CPU only)."""
import numpy as np
import pytest

import oracle
from paper_2511_16358_amd import workloads
from tests import pins


@pytest.mark.parametrize("check", pins.ALL_CHECKS, ids=lambda c: c.__name__)
def test_pin(check):
    check(oracle)


def test_recovery_planted30():
    """Noiseless planted 30x30x30 iFCTN tensor, matched ranks R=2, 50%
    sampling: PAM drives the error on the missing entries towards zero
    (Theorem 1 only promises a critical point; the seed is fixed)."""
    p = workloads.problem("planted30", 0, lambda d, r, G: oracle.reconstruct(G, d))
    X, G, hist = oracle.pam(p.O, p.mask, p.G0, p.dims, rho=p.rho, t_max=300, eps=0.0)
    err = oracle.rse(p.X_true.astype(np.float64), X)
    assert err < 1e-3, err
    objs = [h["objective"] for h in hist]
    assert all(b <= a * (1 + 1e-12) + 1e-15 for a, b in zip(objs, objs[1:]))
