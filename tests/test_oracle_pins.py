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


def test_tucker_workload_has_tucker_rank_5():
    """The synthetic tensor of Sec. 5: every mode unfolding has rank 5."""
    import numpy as np
    from paper_2511_16358_amd import workloads as W
    p = W.tucker_problem(seed=1, missing=0.8)
    X = p.X_true.astype(np.float64)
    assert X.shape == (20, 20, 20, 20) and abs(X.max() - 1.0) < 1e-6 and X.min() > 0
    for m in range(4):
        unf = np.moveaxis(X, m, 0).reshape(20, -1)
        assert np.linalg.matrix_rank(unf, tol=1e-5 * np.linalg.norm(unf)) == 5
    assert abs(1.0 - p.mask.mean() - 0.8) < 0.01


def test_fibre_missing_mask():
    import numpy as np
    from paper_2511_16358_amd import workloads as W
    m = W.fibre_missing_mask((40, 30, 7), 0.3, 2, seed=3)
    assert np.all(m == m[:, :, :1])                 # whole fibres along the band mode
    assert abs(1.0 - m[:, :, 0].mean() - 0.3) < 0.05
