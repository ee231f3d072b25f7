"""Serving runtime (ifctn_server_*, continuous batching) on the GPU.

A served request runs the same kernels in the same order as ifctn_complete
with the same parameters, and every kernel reduces in a fixed order, so the
bar for "the same alone and in the mix" is bitwise equality of X and of the
statistics.  Served FP64 requests are also checked against the oracle.
"""
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


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def mix(seed=0):
    """Requests of orders 2..5, several ranks, all three precisions, with and
    without the stop rule."""
    from paper_2511_16358_amd import ifctn
    shapes = [((13, 11, 9), 3), ((7, 6, 5, 4), 2), ((21, 17), 4), ((5, 4, 6, 3, 4), 2), ((30, 8, 12), 5),
              ((9, 10, 11), 2), ((6, 7, 8, 5), 3), ((40, 33, 3), 4), ((16, 16, 16), 6), ((4, 5, 6, 5, 4), 3)]
    precs = [ifctn.IFCTN_FP32, ifctn.IFCTN_BF16_REFINE, ifctn.IFCTN_FP64]
    reqs = []
    for q, (dims, R) in enumerate(shapes):
        p = W.random_problem(dims, W.uniform_ranks(len(dims), R), seed=seed * 100 + q, keep=0.4)
        prec = precs[q % 3]
        reqs.append(dict(p=p, precision=prec, t_max=12 + 3 * q, eps=(1e-3 if q % 2 else 0.0),
                         refine=(4 if prec == ifctn.IFCTN_BF16_REFINE else 0)))
    return reqs


def alone(r):
    from paper_2511_16358_amd import ifctn
    p = r["p"]
    O = p.O.astype(np.float64) if r["precision"] == ifctn.IFCTN_FP64 else p.O
    X, st = ifctn.complete(O, p.mask, p.G0, p.dims, p.ranks, t_max=r["t_max"], eps=r["eps"],
                           precision=r["precision"], refine_sweeps=r["refine"])
    return X.cpu().numpy(), st


def serve(reqs, **cfg):
    from paper_2511_16358_amd import ifctn
    srv = ifctn.Server(**cfg)
    for q, r in enumerate(reqs):
        p = r["p"]
        O = p.O.astype(np.float64) if r["precision"] == ifctn.IFCTN_FP64 else p.O
        srv.submit(O, p.mask, p.G0, p.dims, p.ranks, r["t_max"], eps=r["eps"], precision=r["precision"],
                   refine_sweeps=r["refine"], tag=q)
    got = {}
    for _ in range(600):
        for c in srv.poll(64, wait_ms=100):
            got[c["tag"]] = c
        if len(got) == len(reqs):
            break
    srv.close()
    assert len(got) == len(reqs), "not every request completed"
    return got


def test_alone_equals_mix_bitwise():
    from paper_2511_16358_amd import ifctn
    reqs = mix(0)
    ref = [alone(r) for r in reqs]
    got = serve(reqs, hbm_budget_bytes=256 << 20, max_active=6, num_streams=4, sweeps_per_round=3)
    for q, (X, st) in enumerate(ref):
        c = got[q]
        assert c["status"] == ifctn.IFCTN_OK, q
        Xs = c["X"].cpu().numpy()
        assert np.array_equal(Xs, X), (q, relerr(Xs, X))
        for key in ("sweeps_done", "converged", "rel_change", "objective", "dx_norm2", "dg_norm2"):
            assert c["stats"][key] == st[key], (q, key, c["stats"][key], st[key])
        assert c["t_submit"] <= c["t_admit"] <= c["t_done"]


def test_constrained_budget_admits_in_order():
    """With room for a single job the requests run one after another in
    submission order, and still give the results they give alone."""
    from paper_2511_16358_amd import ifctn
    reqs = []
    for q in range(5):
        p = W.random_problem((14, 12, 10), W.uniform_ranks(3, 3), seed=70 + q, keep=0.4)
        reqs.append(dict(p=p, precision=ifctn.IFCTN_FP32, t_max=10 + q, eps=0.0, refine=0))
    need = ifctn.workspace_bytes((14, 12, 10), W.uniform_ranks(3, 3))
    got = serve(reqs, hbm_budget_bytes=int(need * 1.5), max_active=8, num_streams=2, sweeps_per_round=4)
    admits = [got[q]["t_admit"] for q in range(len(reqs))]
    assert admits == sorted(admits)
    for q in range(1, len(reqs)):       # one resident job at a time
        assert got[q]["t_admit"] >= got[q - 1]["t_done"] - 1e-3
    for q, r in enumerate(reqs):
        X, _ = alone(r)
        assert np.array_equal(got[q]["X"].cpu().numpy(), X), q


def test_served_fp64_requests_match_oracle():
    from paper_2511_16358_amd import ifctn
    reqs = []
    for q, (dims, R) in enumerate([((10, 9, 8), 2), ((6, 5, 7, 4), 2), ((12, 11), 3)]):
        p = W.random_problem(dims, W.uniform_ranks(len(dims), R), seed=50 + q, keep=0.5)
        reqs.append(dict(p=p, precision=ifctn.IFCTN_FP64, t_max=40, eps=2e-3, refine=0))
    got = serve(reqs, hbm_budget_bytes=64 << 20, max_active=3, num_streams=3, sweeps_per_round=5)
    for q, r in enumerate(reqs):
        p = r["p"]
        Xo, _, ho = oracle.pam(p.O.astype(np.float64), p.mask, p.G0, p.dims, rho=0.1, t_max=40, eps=2e-3)
        c = got[q]
        assert c["stats"]["sweeps_done"] == len(ho)
        assert c["stats"]["converged"] == (1 if ho[-1]["rel_change"] < 2e-3 else 0)
        assert relerr(c["X"].cpu().numpy(), Xo) < 1e-10


def test_submit_refusals_and_bad_data():
    from paper_2511_16358_amd import ifctn
    p = W.random_problem((20, 20, 20), W.uniform_ranks(3, 3), seed=9)
    need = ifctn.workspace_bytes(p.dims, p.ranks)
    srv = ifctn.Server(hbm_budget_bytes=need // 2, max_active=2, num_streams=1, sweeps_per_round=2)
    with pytest.raises(ifctn.IfctnError) as e:
        srv.submit(p.O, p.mask, p.G0, p.dims, p.ranks, 5)
    assert e.value.status == ifctn.IFCTN_E_NOMEM
    bad = p.ranks.copy()
    bad[0][1] = 2
    with pytest.raises(ifctn.IfctnError) as e:
        srv.submit(p.O, p.mask, np.zeros(8000), p.dims, bad, 5)
    assert e.value.status == ifctn.IFCTN_E_INVAL
    srv.close()
    # a non-finite observed entry fails that request only
    small = W.random_problem((8, 7, 6), W.uniform_ranks(3, 2), seed=10)
    O = small.O.copy()
    i = tuple(np.argwhere(small.mask)[0])
    O[i] = np.inf
    srv = ifctn.Server(hbm_budget_bytes=32 << 20, max_active=2, num_streams=2, sweeps_per_round=2)
    srv.submit(O, small.mask, small.G0, small.dims, small.ranks, 6, tag=1)
    srv.submit(small.O, small.mask, small.G0, small.dims, small.ranks, 6, tag=2)
    got = {}
    for _ in range(100):
        for c in srv.poll(8, wait_ms=100):
            got[c["tag"]] = c
        if len(got) == 2:
            break
    srv.close()
    assert got[1]["status"] == ifctn.IFCTN_E_INVAL
    assert got[2]["status"] == ifctn.IFCTN_OK


def test_destroy_with_queued_requests_returns():
    from paper_2511_16358_amd import ifctn
    p = W.random_problem((24, 20, 16), W.uniform_ranks(3, 3), seed=11)
    need = ifctn.workspace_bytes(p.dims, p.ranks)
    srv = ifctn.Server(hbm_budget_bytes=need + 4096, max_active=1, num_streams=1, sweeps_per_round=2)
    for q in range(5):
        srv.submit(p.O, p.mask, p.G0, p.dims, p.ranks, 30, tag=q)
    srv.close()      # drops the queued ones, waits for the resident one


def test_rank_grid_batch_equals_alone():
    """Rank selection as a served batch: one observed tensor and mask shared
    by every rank matrix of the grid; each job's result is its result alone."""
    from paper_2511_16358_amd import ifctn
    p = W.random_problem((14, 12, 10), W.uniform_ranks(3, 2), seed=81, keep=0.5)
    grid = W.rank_grid_msi()
    O = torch.as_tensor(p.O).cuda()
    M = torch.as_tensor(p.mask).cuda()
    G0s = [W.initial_factors_for(p, r, seed=q) for q, r in enumerate(grid)]
    srv = ifctn.Server(64 << 20, max_active=len(grid), num_streams=4, sweeps_per_round=4)
    torch.cuda.synchronize()
    for q, (r, G0) in enumerate(zip(grid, G0s)):
        srv.submit(O, M, G0, p.dims, r, 40, eps=1e-4, tag=q)
    got = {}
    for _ in range(300):
        for c in srv.poll(16, wait_ms=100):
            got[c["tag"]] = c
        if len(got) == len(grid):
            break
    srv.close()
    assert len(got) == len(grid)
    for q, (r, G0) in enumerate(zip(grid, G0s)):
        X, st = ifctn.complete(p.O, p.mask, G0, p.dims, r, t_max=40, eps=1e-4)
        assert np.array_equal(got[q]["X"].cpu().numpy(), X.cpu().numpy()), q
        assert got[q]["stats"]["sweeps_done"] == st["sweeps_done"]


def test_served_fp64_rank_grid_matches_oracle():
    """A rank grid served as one FP64 batch (shared observed tensor and
    mask): every job against the oracle's Algorithm 1 with the same ranks and
    initial factors."""
    from paper_2511_16358_amd import ifctn
    p = W.random_problem((12, 10, 9), W.uniform_ranks(3, 2), seed=83, keep=0.5)
    grid = W.rank_grid_msi()
    O64 = p.O.astype(np.float64)
    O = torch.as_tensor(O64).cuda()
    M = torch.as_tensor(p.mask).cuda()
    G0s = [W.initial_factors_for(p, r, seed=q) for q, r in enumerate(grid)]
    srv = ifctn.Server(64 << 20, max_active=len(grid), num_streams=4, sweeps_per_round=4)
    torch.cuda.synchronize()
    for q, (r, G0) in enumerate(zip(grid, G0s)):
        srv.submit(O, M, G0, p.dims, r, 15, eps=0.0, precision=ifctn.IFCTN_FP64, tag=q)
    got = {}
    for _ in range(300):
        for c in srv.poll(16, wait_ms=100):
            got[c["tag"]] = c
        if len(got) == len(grid):
            break
    srv.close()
    assert len(got) == len(grid)
    for q, (r, G0) in enumerate(zip(grid, G0s)):
        Xo, _, ho = oracle.pam(O64, p.mask, G0, p.dims, rho=0.1, t_max=15, eps=0.0)
        assert got[q]["status"] == ifctn.IFCTN_OK
        assert relerr(got[q]["X"].cpu().numpy(), Xo) < 1e-10, (q, np.asarray(r).tolist())
        assert abs(got[q]["stats"]["objective"] - ho[-1]["objective"]) <= 1e-9 * ho[-1]["objective"]


def test_failed_admission_reports_and_server_continues():
    """A request that fails at admission (fault injection: the next
    admission reports IFCTN_E_NOMEM) is completed with that status, its slot
    and pool range are returned, and the requests after it run normally."""
    from paper_2511_16358_amd import ifctn
    p = W.random_problem((16, 14, 12), W.uniform_ranks(3, 3), seed=91)
    need = ifctn.workspace_bytes(p.dims, p.ranks)
    srv = ifctn.Server(hbm_budget_bytes=need + 4096, max_active=1, num_streams=1, sweeps_per_round=3)
    ifctn.set_option("inject_admit_failures", 1)
    try:
        for q in range(3):
            srv.submit(p.O, p.mask, p.G0, p.dims, p.ranks, 9, tag=q)
        got = {}
        for _ in range(300):
            for c in srv.poll(8, wait_ms=100):
                got[c["tag"]] = c
            if len(got) == 3:
                break
    finally:
        ifctn.set_option("inject_admit_failures", 0)
        srv.close()
    assert got[0]["status"] == ifctn.IFCTN_E_NOMEM
    X, st = ifctn.complete(p.O, p.mask, p.G0, p.dims, p.ranks, t_max=9)
    for q in (1, 2):
        assert got[q]["status"] == ifctn.IFCTN_OK
        assert np.array_equal(got[q]["X"].cpu().numpy(), X.cpu().numpy())
