"""GPU parity of the seeded default G^0 (ifctn_default_factors, and
ifctn_init / ifctn_complete with G0_host NULL) against the oracle's
independent implementation, through the C ABI.  The random part is exact on
both sides (the same 53-bit fractions); the scale comes from a float64
reduction over the observed entries taken in another order, so entries agree
to a few ulps."""
import numpy as np
import pytest

import oracle
from paper_2511_16358_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_2511_16358_amd import ifctn
    ifctn.lib()
    return ifctn


def ranks_of(N, upper, default=3):
    r = np.full((N, N), default, dtype=np.int64)
    np.fill_diagonal(r, 0)
    for (a, b), v in upper.items():
        r[a, b] = r[b, a] = v
    return r


def flat(G, N):
    return np.concatenate([G[key].ravel() for key in oracle.block_order(N)])


CASES = [
    ((9, 7, 5), ranks_of(3, {(0, 1): 2, (1, 2): 5}), 0.3),
    ((80, 70, 60), ranks_of(3, {}), 0.1),                   # more than 1024 x 256 entries: the grid-stride loop
    ((6, 5, 4, 7), ranks_of(4, {(0, 3): 2}), 0.5),
    ((4, 3, 5, 3, 4), ranks_of(5, {(2, 4): 4}, default=2), 0.2),
    ((5, 6, 7), ranks_of(3, {(0, 1): 12, (0, 2): 30}), 0.3),  # the large-rank route's sizes
]


@pytest.mark.parametrize("precision", [0, 1, 2], ids=["fp32", "bf16_refine", "fp64"])
@pytest.mark.parametrize("dims,ranks,keep", CASES, ids=["x".join(map(str, c[0])) for c in CASES])
def test_default_factors_match_oracle(dims, ranks, keep, precision):
    from paper_2511_16358_amd import ifctn
    rng = np.random.default_rng(sum(dims))
    O = (3.0 * rng.standard_normal(dims)).astype(np.float64 if precision == ifctn.IFCTN_FP64 else np.float32)
    mask = (rng.random(dims) < keep).astype(np.uint8)
    for seed in (0, 12345, (1 << 63) + 5):
        print(f"[case] default_factors dims={dims} seed={seed} precision={precision}", flush=True)
        got = ifctn.default_factors(O, mask, dims, ranks, seed=seed, precision=precision, packed=True)
        ref = flat(oracle.default_factors(O.astype(np.float64), mask, dims, ranks, seed), len(dims))
        assert got.shape == ref.shape
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
        # the random fractions themselves are identical: every ratio is the same scale
        ratio = got / np.where(ref == 0, 1.0, ref)
        assert np.ptp(ratio[ref != 0]) <= 1e-13


def test_default_factors_empty_and_zero_data():
    from paper_2511_16358_amd import ifctn
    dims, ranks = (7, 6, 5), ranks_of(3, {})
    O = np.zeros(dims, dtype=np.float32)
    for mask in (np.zeros(dims, np.uint8), np.ones(dims, np.uint8)):
        got = ifctn.default_factors(O, mask, dims, ranks, seed=9, packed=True)
        ref = flat(oracle.default_factors(O, mask, dims, ranks, 9), 3)   # m = 1
        assert np.max(np.abs(got - ref)) <= 1e-15


def test_init_without_g0_uses_the_seeded_default():
    """G0 NULL at ifctn_init is the default of seed 0: the sweeps equal those
    from the explicit default bitwise, and match the oracle started from its
    own default in FP64."""
    from paper_2511_16358_amd import ifctn
    p = W.random_problem((12, 10, 9), ranks_of(3, {(0, 1): 4}), seed=4, keep=0.4)
    O64 = p.O.astype(np.float64)
    j0 = ifctn.Job(O64, p.mask, None, p.dims, p.ranks, rho=p.rho, precision=ifctn.IFCTN_FP64)
    g0 = ifctn.default_factors(O64, p.mask, p.dims, p.ranks, seed=0, precision=ifctn.IFCTN_FP64, packed=True)
    j1 = ifctn.Job(O64, p.mask, g0, p.dims, p.ranks, rho=p.rho, precision=ifctn.IFCTN_FP64)
    j0.sweep(3)
    j1.sweep(3)
    X0, X1 = j0.x().cpu().numpy(), j1.x().cpu().numpy()
    j0.close()
    j1.close()
    assert np.array_equal(X0, X1)
    Go = oracle.default_factors(O64, p.mask, p.dims, p.ranks, 0)
    Xo, _, _ = oracle.pam(O64, p.mask, Go, p.dims, rho=p.rho, t_max=3, eps=0.0)
    assert np.linalg.norm(X0 - Xo) <= 1e-10 * np.linalg.norm(Xo)
    # ifctn_complete with G0 NULL runs the same iteration
    Xc, st = ifctn.complete(O64, p.mask, None, p.dims, p.ranks, t_max=3, precision=ifctn.IFCTN_FP64)
    assert np.array_equal(Xc.cpu().numpy(), X0) and st["sweeps_done"] == 3


def test_served_request_without_g0_equals_complete():
    """A served request with G0 None takes the same seeded default (drawn at
    submit) and gives X and the statistics of ifctn_complete with G0 NULL,
    bit for bit."""
    from paper_2511_16358_amd import ifctn
    p = W.random_problem((11, 9, 8, 5), ranks_of(4, {}, default=2), seed=8, keep=0.4)
    Xc, st = ifctn.complete(p.O, p.mask, None, p.dims, p.ranks, t_max=9, precision=ifctn.IFCTN_FP32)
    srv = ifctn.Server(hbm_budget_bytes=64 << 20, max_active=2, num_streams=2, sweeps_per_round=4)
    srv.submit(p.O, p.mask, None, p.dims, p.ranks, 9, precision=ifctn.IFCTN_FP32, tag=1)
    got = []
    for _ in range(300):
        got += srv.poll(8, wait_ms=100)
        if got:
            break
    srv.close()
    assert len(got) == 1 and got[0]["status"] == ifctn.IFCTN_OK
    assert np.array_equal(got[0]["X"].cpu().numpy(), Xc.cpu().numpy())
    for key in ("sweeps_done", "rel_change", "objective", "dx_norm2", "dg_norm2"):
        assert got[0]["stats"][key] == st[key], key
