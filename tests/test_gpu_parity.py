"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
the same seeded inputs and the same initial factors.

Tolerances (relative Frobenius error of X, gauge-invariant):
  * FP64 library path: 1e-10 (same algorithm, different summation order);
  * FP32 library path: 1e-5 (float32 streaming data, float64 Gram / Cholesky
    / factors / reductions).
Factors are compared too where both runs start from the same G^0: every block
is a strictly convex problem, so the trajectory is unique (no gauge freedom
between the two implementations).
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
    ifctn.lib()          # fails loudly when the library is missing
    return ifctn


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def assert_x_close(Xg, Xo, tol, what=""):
    """X within tol of the oracle's: relative Frobenius error, and every entry
    within 10 tol of the oracle's largest entry."""
    Xg = np.asarray(Xg, dtype=np.float64)
    Xo = np.asarray(Xo, dtype=np.float64)
    e = relerr(Xg, Xo)
    assert e < tol, (what, e)
    worst = float(np.max(np.abs(Xg - Xo))) if Xo.size else 0.0
    assert worst <= 10 * tol * max(float(np.max(np.abs(Xo))) if Xo.size else 0.0, 1e-300), (what, worst)


def run_both(p, sweeps, precision, batch=1):
    """`sweeps` sweeps on both sides.  The library runs them in calls of
    ifctn_sweep(batch): within a call the X step of every sweep but the last
    rides in the next sweep's first contraction launch (the fused form that
    ifctn_complete, the server and the bench run); statistics are compared
    after every call."""
    from paper_2511_16358_amd import ifctn
    print(f"[case] dims={p.dims} ranks={np.asarray(p.ranks).tolist()} sweeps={sweeps} batch={batch} "
          f"precision={precision}", flush=True)
    O64 = p.O.astype(np.float64)
    Oin = O64 if precision == ifctn.IFCTN_FP64 else p.O
    job = ifctn.Job(Oin, p.mask, p.G0, p.dims, p.ranks, rho=p.rho, precision=precision)
    Xo = oracle.initial_x(O64, p.mask)
    Go = {k: v.copy() for k, v in p.G0.items()}
    gpu_stats, ora_stats = [], []
    s = 0
    while s < sweeps:
        n = min(batch, sweeps - s)
        gpu_stats.append(job.sweep(n))
        for _ in range(n):
            Xo, Go, st = oracle.pam_sweep(Xo, Go, O64, p.mask, p.dims, p.rho)
        ora_stats.append(st)
        s += n
    Xg = job.x().cpu().numpy()
    Xh = job.xhat().cpu().numpy()
    Gg = job.factors()
    job.close()
    return dict(Xg=Xg, Xh=Xh, Gg=Gg, Xo=Xo, Go=Go, gs=gpu_stats, os=ora_stats)


SMALL = [
    ((7, 13, 5), W.uniform_ranks(3, 3)),
    ((6, 5, 7), np.array([[0, 2, 3], [2, 0, 1], [3, 1, 0]])),
    ((9, 11), W.uniform_ranks(2, 4)),
    ((5, 6, 7, 3), W.uniform_ranks(4, 2)),
    ((4, 3, 5, 2, 3), W.uniform_ranks(5, 2)),
    ((33, 17, 40), W.uniform_ranks(3, 5)),      # several tiles and ragged tails
    ((3, 1, 4), W.uniform_ranks(3, 2)),          # a mode of size 1
    ((12, 20, 3, 9), np.array([[0, 2, 3, 1], [2, 0, 2, 3], [3, 2, 0, 2], [1, 3, 2, 0]])),
    ((8, 7, 9, 6, 10), W.uniform_ranks(5, 3)),   # order 5: staged accumulation over two c-modes
    ((4, 4, 4, 4, 4), W.uniform_ranks(5, 8)),    # largest rank at order 5: 8^4 accumulators per row
]


@pytest.mark.parametrize("dims,ranks", SMALL, ids=["x".join(map(str, d)) for d, _ in SMALL])
def test_fp64_path_matches_oracle(dims, ranks):
    from paper_2511_16358_amd import ifctn
    p = W.random_problem(dims, ranks, seed=sum(dims), keep=0.5)
    r = run_both(p, 3, ifctn.IFCTN_FP64)
    assert_x_close(r["Xg"], r["Xo"], 1e-10)
    assert relerr(r["Xh"], oracle.reconstruct(r["Go"], p.dims)) < 1e-10
    for key in r["Go"]:
        assert relerr(r["Gg"][key], r["Go"][key]) < 1e-9, key
    for g, o in zip(r["gs"], r["os"]):
        assert abs(g["objective"] - o["objective"]) <= 1e-9 * max(o["objective"], 1e-30)
        assert abs(g["rel_change"] - o["rel_change"]) <= 1e-9 * max(o["rel_change"], 1e-30)
        assert abs(g["dg_norm2"] - o["dg_norm2"]) <= 1e-8 * max(o["dg_norm2"], 1e-30)
    # observed entries are exactly the data
    m = p.mask.astype(bool)
    assert np.array_equal(r["Xg"][m], p.O.astype(np.float64)[m])


@pytest.mark.parametrize("dims,ranks", SMALL, ids=["x".join(map(str, d)) for d, _ in SMALL])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_phased_factor_blocks_match_oracle(dims, ranks, precision):
    """Every factor block forced into the phased form (partial Gram matrices
    on many workgroups, then per-column solves)."""
    from paper_2511_16358_amd import ifctn
    p = W.random_problem(dims, ranks, seed=17)
    prec = ifctn.IFCTN_FP64 if precision == "fp64" else ifctn.IFCTN_FP32
    ifctn.set_option("phased_min", 0)
    ifctn.set_option("gamma", 0)
    try:
        r = run_both(p, 3, prec)
    finally:
        ifctn.set_option("phased_min", -1)
        ifctn.set_option("gamma", -1)
    tol = 1e-10 if precision == "fp64" else 1e-5
    assert_x_close(r["Xg"], r["Xo"], tol)
    for key in r["Go"]:
        assert relerr(r["Gg"][key], r["Go"][key]) < tol * 10, key
    for gs, os_ in zip(r["gs"], r["os"]):
        assert abs(gs["objective"] - os_["objective"]) <= tol * 10 * abs(os_["objective"])


@pytest.mark.parametrize("dims,ranks", SMALL, ids=["x".join(map(str, d)) for d, _ in SMALL])
def test_fp32_path_matches_oracle(dims, ranks):
    """The default FP32 path on every small shape (order-5 staged
    accumulation over float tables, rank 8 at order 5, unequal ranks, a mode
    of size 1), one sweep per call."""
    from paper_2511_16358_amd import ifctn
    p = W.random_problem(dims, ranks, seed=7 + sum(dims), keep=0.5)
    r = run_both(p, 3, ifctn.IFCTN_FP32)
    assert_x_close(r["Xg"], r["Xo"], 1e-5)
    m = p.mask.astype(bool)
    assert np.array_equal(r["Xg"][m], p.O[m].astype(np.float64))


@pytest.mark.parametrize("dims,ranks", SMALL, ids=["x".join(map(str, d)) for d, _ in SMALL])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fused_x_step_matches_oracle(dims, ranks, precision):
    """Four sweeps in one ifctn_sweep call: the X steps of the first three
    run fused into the next sweep's mode-0 contraction launch (the path of
    ifctn_complete, the server and the bench)."""
    from paper_2511_16358_amd import ifctn
    p = W.random_problem(dims, ranks, seed=41 + sum(dims), keep=0.5)
    prec = ifctn.IFCTN_FP64 if precision == "fp64" else ifctn.IFCTN_FP32
    r = run_both(p, 4, prec, batch=4)
    tol = 1e-10 if precision == "fp64" else 1e-5
    assert_x_close(r["Xg"], r["Xo"], tol)
    g, o = r["gs"][-1], r["os"][-1]
    assert abs(g["objective"] - o["objective"]) <= 10 * tol * max(o["objective"], 1e-30)
    assert abs(g["rel_change"] - o["rel_change"]) <= 10 * tol * max(o["rel_change"], 1e-30)
    for key in r["Go"]:
        assert relerr(r["Gg"][key], r["Go"][key]) < 10 * tol, key
    m = p.mask.astype(bool)
    assert np.array_equal(r["Xg"][m], p.O.astype(np.float64)[m] if prec == ifctn.IFCTN_FP64
                          else p.O[m].astype(np.float64))


@pytest.mark.parametrize("dims,ranks", SMALL, ids=["x".join(map(str, d)) for d, _ in SMALL])
def test_phased_one_launch_form_matches_oracle(dims, ranks):
    """Phased factor blocks in the one-launch form (the last workgroup of a
    column tile solves its columns); the default is two launches per sub-block."""
    from paper_2511_16358_amd import ifctn
    p = W.random_problem(dims, ranks, seed=29)
    ifctn.set_option("phased_min", 0)
    ifctn.set_option("phased_onelaunch", 1)
    ifctn.set_option("gamma", 0)
    try:
        r = run_both(p, 3, ifctn.IFCTN_FP64)
    finally:
        ifctn.set_option("phased_min", -1)
        ifctn.set_option("phased_onelaunch", -1)
        ifctn.set_option("gamma", -1)
    assert_x_close(r["Xg"], r["Xo"], 1e-10)


@pytest.mark.parametrize("dims,ranks", SMALL, ids=["x".join(map(str, d)) for d, _ in SMALL])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_gamma_route_matches_oracle(dims, ranks, precision):
    """Every factor block by the Gamma route (Gamma_k = Z_k^T Z_k built on the
    matrix cores, per-column H_j from it), three sweeps in one call."""
    from paper_2511_16358_amd import ifctn
    p = W.random_problem(dims, ranks, seed=53 + len(dims), keep=0.5)
    prec = ifctn.IFCTN_FP64 if precision == "fp64" else ifctn.IFCTN_FP32
    ifctn.set_option("gamma", 2)
    try:
        r = run_both(p, 3, prec, batch=3)
    finally:
        ifctn.set_option("gamma", -1)
    tol = 1e-10 if precision == "fp64" else 1e-5
    assert_x_close(r["Xg"], r["Xo"], tol)
    for key in r["Go"]:
        assert relerr(r["Gg"][key], r["Go"][key]) < 10 * tol, key
    g, o = r["gs"][-1], r["os"][-1]
    assert abs(g["objective"] - o["objective"]) <= 10 * tol * max(o["objective"], 1e-30)
    assert abs(g["dg_norm2"] - o["dg_norm2"]) <= 100 * tol * max(o["dg_norm2"], 1e-30)


@pytest.mark.parametrize("dims,ranks", [SMALL[3], SMALL[4], SMALL[8]], ids=["5x6x7x3", "4x3x5x2x3", "8x7x9x6x10"])
def test_gamma_overlap_is_bitwise_inline(dims, ranks):
    """Gamma_k built on the job's second stream, concurrently with the
    contraction, and in line on the job's stream: the same kernels on the same
    data, so bitwise the same X, factors and statistics."""
    from paper_2511_16358_amd import ifctn
    p = W.random_problem(dims, ranks, seed=61, keep=0.5)
    out = []
    ifctn.set_option("gamma", 2)
    try:
        for ov in (1, 0):
            ifctn.set_option("overlap", ov)
            job = ifctn.Job(p.O, p.mask, p.G0, p.dims, p.ranks, rho=p.rho, precision=ifctn.IFCTN_FP32)
            st = job.sweep(4)
            out.append((job.x().cpu().numpy(), job.factors(), st))
            job.close()
    finally:
        ifctn.set_option("overlap", -1)
        ifctn.set_option("gamma", -1)
    (xa, ga, sa), (xb, gb, sb) = out
    assert np.array_equal(xa, xb)
    for key in ga:
        assert np.array_equal(ga[key], gb[key]), key
    assert sa["objective"] == sb["objective"] and sa["dg_norm2"] == sb["dg_norm2"]


@pytest.mark.parametrize("dims,ranks", SMALL[:5], ids=["x".join(map(str, d)) for d, _ in SMALL[:5]])
def test_separate_gram_launch_matches_oracle(dims, ranks):
    """The Gram weights as a launch of their own (the default puts them in the
    contraction launch): same results."""
    from paper_2511_16358_amd import ifctn
    p = W.random_problem(dims, ranks, seed=23)
    ifctn.set_option("merge_gram", 0)
    try:
        r = run_both(p, 3, ifctn.IFCTN_FP64)
    finally:
        ifctn.set_option("merge_gram", -1)
    assert_x_close(r["Xg"], r["Xo"], 1e-10)


def test_planted30_fp32_20_sweeps():
    """The oracle-sized workload: 30^3, planted R=2, 50% sampling, 20 sweeps."""
    from paper_2511_16358_amd import ifctn
    p = W.problem("planted30", 0, lambda d, r, G: oracle.reconstruct(G, d))
    r = run_both(p, p.sweeps, ifctn.IFCTN_FP32)
    curve = []
    # per-sweep divergence is implicit in the final comparison; the stats
    # (float64 sums) follow the oracle's closely
    for g, o in zip(r["gs"], r["os"]):
        curve.append(abs(g["objective"] - o["objective"]) / max(o["objective"], 1e-30))
    print("objective divergence per sweep:", ["%.1e" % c for c in curve])
    assert_x_close(r["Xg"], r["Xo"], 1e-5)
    assert max(curve) < 1e-4


def test_planted30_fp64_20_sweeps():
    from paper_2511_16358_amd import ifctn
    p = W.problem("planted30", 0, lambda d, r, G: oracle.reconstruct(G, d))
    r = run_both(p, p.sweeps, ifctn.IFCTN_FP64)
    assert_x_close(r["Xg"], r["Xo"], 1e-10)
    for key in r["Go"]:
        assert relerr(r["Gg"][key], r["Go"][key]) < 1e-8, key


def test_deterministic_bitwise():
    from paper_2511_16358_amd import ifctn
    p = W.random_problem((33, 17, 40), W.uniform_ranks(3, 4), seed=3)
    outs = []
    for _ in range(2):
        job = ifctn.Job(p.O, p.mask, p.G0, p.dims, p.ranks)
        st = job.sweep(4)
        outs.append((job.x().cpu().numpy(), job.factors(), st))
        job.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    for key in outs[0][1]:
        assert np.array_equal(outs[0][1][key], outs[1][1][key])
    assert outs[0][2]["objective"] == outs[1][2]["objective"]


def test_sweep_batching_equals_single_sweeps():
    """ifctn_sweep(n) fuses the X step of sweep s into sweep s+1's first
    kernel; the result equals n calls of ifctn_sweep(1)."""
    from paper_2511_16358_amd import ifctn
    p = W.random_problem((20, 24, 18), W.uniform_ranks(3, 3), seed=11)
    a = ifctn.Job(p.O, p.mask, p.G0, p.dims, p.ranks, precision=ifctn.IFCTN_FP64)
    sa = a.sweep(5)
    b = ifctn.Job(p.O, p.mask, p.G0, p.dims, p.ranks, precision=ifctn.IFCTN_FP64)
    for _ in range(5):
        sb = b.sweep(1)
    assert relerr(a.x().cpu().numpy(), b.x().cpu().numpy()) < 1e-13
    assert abs(sa["objective"] - sb["objective"]) <= 1e-12 * sb["objective"]
    assert sa["sweeps_done"] == sb["sweeps_done"] == 5


def test_assemble_matches_oracle():
    from paper_2511_16358_amd import ifctn
    for dims, R in [((7, 13, 5), 3), ((5, 6, 7, 3), 2), ((9, 11), 4), ((4, 3, 5, 2, 3), 2)]:
        ranks = W.uniform_ranks(len(dims), R)
        G = {k: np.random.default_rng(5).standard_normal(s) for k, s in W.factor_shapes(dims, ranks)}
        ref = oracle.reconstruct(G, dims)
        got64 = ifctn.assemble(dims, ranks, G, precision=ifctn.IFCTN_FP64).cpu().numpy()
        got32 = ifctn.assemble(dims, ranks, G).cpu().numpy()
        assert relerr(got64, ref) < 1e-12
        assert relerr(got32, ref) < 1e-6


def test_complete_stop_rule_matches_oracle():
    """ifctn_complete stops at the first sweep with rel_change < eps."""
    from paper_2511_16358_amd import ifctn
    p = W.random_problem((10, 12, 9), W.uniform_ranks(3, 2), seed=21)
    O64 = p.O.astype(np.float64)
    _, _, hist = oracle.pam(O64, p.mask, p.G0, p.dims, rho=0.1, t_max=12, eps=0.0)
    rels = [h["rel_change"] for h in hist]
    eps = 0.5 * (rels[5] + rels[6])
    stop = next(s for s in range(12) if rels[s] < eps)
    X, st = ifctn.complete(O64, p.mask, p.G0, p.dims, p.ranks, t_max=12, eps=eps,
                           precision=ifctn.IFCTN_FP64)
    assert st["sweeps_done"] == stop + 1 and st["converged"] == 1
    Xo, _, _ = oracle.pam(O64, p.mask, p.G0, p.dims, rho=0.1, t_max=12, eps=eps)
    assert relerr(X.cpu().numpy(), Xo) < 1e-10


@pytest.mark.parametrize("target", [0, 6, 7, 8, 9, 13])
def test_device_stop_flag_at_chunk_boundaries(target):
    """The stop test runs on the device after every X step and the host reads
    the flag once per chunk of sweeps: the stop sweep must be the oracle's
    wherever it falls relative to the chunks."""
    from paper_2511_16358_amd import ifctn
    p = W.random_problem((9, 8, 10), W.uniform_ranks(3, 2), seed=33)
    O64 = p.O.astype(np.float64)
    _, _, hist = oracle.pam(O64, p.mask, p.G0, p.dims, rho=0.1, t_max=16, eps=0.0)
    rels = [h["rel_change"] for h in hist]
    lo = min(rels[:target]) if target else np.inf
    if not rels[target] < lo:
        pytest.skip("relative change not decreasing at this sweep")
    eps = 0.5 * (rels[target] + min(lo, 2 * rels[target]))
    stop = next(s for s in range(16) if rels[s] < eps)
    assert stop == target
    X, st = ifctn.complete(O64, p.mask, p.G0, p.dims, p.ranks, t_max=16, eps=eps, precision=ifctn.IFCTN_FP64)
    assert st["sweeps_done"] == stop + 1 and st["converged"] == 1
    Xo, _, ho = oracle.pam(O64, p.mask, p.G0, p.dims, rho=0.1, t_max=16, eps=eps)
    assert len(ho) == stop + 1
    assert relerr(X.cpu().numpy(), Xo) < 1e-10
    assert abs(st["rel_change"] - ho[-1]["rel_change"]) <= 1e-9 * ho[-1]["rel_change"]


def test_device_stop_never_met_runs_t_max():
    from paper_2511_16358_amd import ifctn
    p = W.random_problem((9, 8, 10), W.uniform_ranks(3, 2), seed=34)
    O64 = p.O.astype(np.float64)
    X, st = ifctn.complete(O64, p.mask, p.G0, p.dims, p.ranks, t_max=11, eps=1e-300, precision=ifctn.IFCTN_FP64)
    assert st["sweeps_done"] == 11 and st["converged"] == 0
    Xo, _, _ = oracle.pam(O64, p.mask, p.G0, p.dims, rho=0.1, t_max=11, eps=0.0)
    assert relerr(X.cpu().numpy(), Xo) < 1e-10


def test_paper_defaults_planted30():
    """Algorithm 1 with the paper's defaults (t_max = 1000, eps = 1e-5,
    rho = 0.1) on the planted 30^3 tensor: same stop sweep as the oracle."""
    from paper_2511_16358_amd import ifctn
    p = W.problem("planted30", 0, lambda d, r, G: oracle.reconstruct(G, d))
    O64 = p.O.astype(np.float64)
    Xo, _, ho = oracle.pam(O64, p.mask, p.G0, p.dims, rho=0.1, t_max=1000, eps=1e-5)
    X, st = ifctn.complete(O64, p.mask, p.G0, p.dims, p.ranks, t_max=1000, eps=1e-5, precision=ifctn.IFCTN_FP64)
    print(f"planted30 defaults: oracle stops after {len(ho)} sweeps, GPU after {st['sweeps_done']}")
    assert st["sweeps_done"] == len(ho) and st["converged"] == 1
    assert relerr(X.cpu().numpy(), Xo) < 1e-9
    X32, st32 = ifctn.complete(p.O, p.mask, p.G0, p.dims, p.ranks, t_max=1000, eps=1e-5)
    assert abs(st32["sweeps_done"] - len(ho)) <= 2
    assert relerr(X32.cpu().numpy(), p.X_true) < 2 * relerr(Xo, p.X_true) + 1e-4


def test_bf16_refine_with_stop_rule():
    """BF16_REFINE with eps: the bfloat16 phase stops on the device test,
    then the float32 refinement sweeps run."""
    from paper_2511_16358_amd import ifctn
    p = W.problem("planted30", 0, lambda d, r, G: oracle.reconstruct(G, d))
    X, st = ifctn.complete(p.O, p.mask, p.G0, p.dims, p.ranks, t_max=1000, eps=1e-3,
                           precision=ifctn.IFCTN_BF16_REFINE, refine_sweeps=20)
    assert st["converged"] == 1 and st["sweeps_done"] < 1000
    _, _, ho = oracle.pam(p.O.astype(np.float64), p.mask, p.G0, p.dims, rho=0.1, t_max=1000, eps=1e-3)
    assert abs(st["sweeps_done"] - 20 - len(ho)) <= 3
    m = p.mask.astype(bool)
    assert np.array_equal(X.cpu().numpy()[m], p.O[m])


def test_invalid_inputs_rejected():
    from paper_2511_16358_amd import ifctn
    p = W.random_problem((6, 5, 4), W.uniform_ranks(3, 2), seed=1)
    O = p.O.copy()
    O[np.argwhere(p.mask)[0][0], np.argwhere(p.mask)[0][1], np.argwhere(p.mask)[0][2]] = np.nan
    with pytest.raises(ifctn.IfctnError) as e:
        ifctn.Job(O, p.mask, p.G0, p.dims, p.ranks)
    assert e.value.status == ifctn.IFCTN_E_INVAL
    # NaN off the mask is ignored (X^0 is zero there)
    O2 = p.O.copy()
    O2[~p.mask.astype(bool)] = np.nan
    job = ifctn.Job(O2, p.mask, p.G0, p.dims, p.ranks)
    assert np.isfinite(job.sweep(2)["objective"])
    job.close()
    # parameter errors are reported before any factor is read
    flat = np.zeros(4096)
    bad = p.ranks.copy()
    bad[0][1] = 3
    with pytest.raises(ifctn.IfctnError) as e:
        ifctn.Job(p.O, p.mask, flat, p.dims, bad)
    assert e.value.status == ifctn.IFCTN_E_INVAL
    with pytest.raises(ifctn.IfctnError) as e:
        ifctn.Job(p.O, p.mask, p.G0, p.dims, p.ranks, rho=0.0)
    assert e.value.status == ifctn.IFCTN_E_INVAL
    with pytest.raises(ifctn.IfctnError) as e:
        ifctn.Job(p.O, p.mask, flat, p.dims, W.uniform_ranks(3, ifctn.IFCTN_MAX_RANK + 1))
    assert e.value.status == ifctn.IFCTN_E_UNSUPPORTED


def test_fully_observed_fixed_point():
    """O = iFCTN(G*) fully observed and G^0 = G*: a sweep keeps X and G."""
    from paper_2511_16358_amd import ifctn
    dims, ranks = (8, 9, 7), W.uniform_ranks(3, 3)
    G = {k: np.random.default_rng(2).uniform(0.2, 1.0, s) for k, s in W.factor_shapes(dims, ranks)}
    X = oracle.reconstruct(G, dims)
    mask = np.ones(dims, dtype=np.uint8)
    job = ifctn.Job(X, mask, G, dims, ranks, precision=ifctn.IFCTN_FP64)
    st = job.sweep(1)
    Gg = job.factors()
    for key in G:
        assert relerr(Gg[key], G[key]) < 1e-11
    assert np.array_equal(job.x().cpu().numpy(), X)
    assert st["objective"] < 1e-20 * float(np.sum(X * X))
    job.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_no_observed_entry(prec):
    """An empty mask: X^0 = 0, so the first relative change is infinite on
    both sides, and the iteration then follows the factors alone."""
    import dataclasses
    from paper_2511_16358_amd import ifctn
    p = W.random_problem((9, 7, 6), W.uniform_ranks(3, 2), seed=21, keep=0.5)
    p = dataclasses.replace(p, O=np.zeros(p.dims, dtype=np.float32), mask=np.zeros(p.dims, dtype=np.uint8))
    precision = ifctn.IFCTN_FP64 if prec == "fp64" else ifctn.IFCTN_FP32
    r = run_both(p, 3, precision)
    assert r["gs"][0]["rel_change"] == float("inf") and r["os"][0]["rel_change"] == float("inf")
    tol = 1e-10 if prec == "fp64" else 2e-5
    assert_x_close(r["Xg"], r["Xo"], tol)
    for key in r["Go"]:
        assert relerr(r["Gg"][key], r["Go"][key]) < 10 * tol, key


LONG = [(40000, 3), (3, 40000), (20000, 4, 3), (5, 3, 30000), (3, 4, 5, 3000)]


@pytest.mark.parametrize("dims", LONG, ids=["x".join(map(str, d)) for d in LONG])
def test_long_fibre(dims):
    """A mode too long for a fibre's LDS tables: the fibre is split into
    chunks over workgroups (each with a partial slot), or another mode serves
    as fibre.  Two FP64 and two FP32 sweeps against the oracle, one sweep per
    call, then two sweeps in one call each (the second sweep's mode-0 launch
    carries the fused X step on the chunked fibre)."""
    from paper_2511_16358_amd import ifctn
    p = W.random_problem(dims, W.uniform_ranks(len(dims), 2), seed=22, keep=0.3)
    for batch in (1, 2):
        r = run_both(p, 2, ifctn.IFCTN_FP64, batch=batch)
        assert_x_close(r["Xg"], r["Xo"], 1e-10, f"fp64 batch {batch}")
        for key in r["Go"]:
            assert relerr(r["Gg"][key], r["Go"][key]) < 1e-9, key
        r = run_both(p, 2, ifctn.IFCTN_FP32, batch=batch)
        assert_x_close(r["Xg"], r["Xo"], 2e-5, f"fp32 batch {batch}")


# --------------------------------------------------------------------------
# full-size workloads in the benchmark's launch configuration
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["msi256", "traffic214", "video144"])
def test_full_size_two_sweeps_match_oracle(name):
    """Two full sweeps at the workloads' real sizes (the oracle takes a few
    seconds per sweep here) plus properties that hold at any size."""
    from paper_2511_16358_amd import ifctn
    p = W.problem(name, 0, lambda d, r, G: oracle.reconstruct(G, d))
    r = run_both(p, 2, ifctn.IFCTN_FP32, batch=2)
    e = relerr(r["Xg"], r["Xo"])
    print(f"{name}: rel err after 2 sweeps {e:.2e}")
    assert_x_close(r["Xg"], r["Xo"], 1e-5, name)
    m = p.mask.astype(bool)
    assert np.array_equal(r["Xg"][m], p.O[m].astype(np.float64))


@pytest.mark.parametrize("name", ["msi256", "traffic214"])
def test_full_size_lemma2_every_sweep(name):
    """Lemma 2 on the GPU's own float64 statistics: the objective decreases
    by at least rho/2 (||dX||^2 + sum ||dG||^2) every sweep (slack for the
    float32 data)."""
    from paper_2511_16358_amd import ifctn
    p = W.problem(name, 0, lambda d, r, G: oracle.reconstruct(G, d))
    job = ifctn.Job(p.O, p.mask, p.G0, p.dims, p.ranks, rho=p.rho)
    Xh0 = job.xhat().cpu().numpy().astype(np.float64)
    F = 0.5 * float(np.sum((oracle.initial_x(p.O, p.mask) - Xh0) ** 2))
    for s in range(8):
        st = job.sweep(1)
        dec = F - st["objective"]
        need = 0.5 * p.rho * (st["dx_norm2"] + st["dg_norm2"])
        assert dec >= need - 1e-5 * F, (s, dec, need)
        F = st["objective"]
    job.close()


def _random_case(seed):
    rng = np.random.default_rng(1000 + seed)
    N = int(rng.integers(2, 6))
    while True:
        dims = tuple(int(x) for x in rng.integers(1, 14, size=N))
        if np.prod(dims) <= 4000:
            break
    ranks = np.zeros((N, N), dtype=np.int64)
    for a in range(N):
        for b in range(a + 1, N):
            ranks[a][b] = ranks[b][a] = int(rng.integers(1, 9 if N <= 3 else 6))
    return dims, ranks


@pytest.mark.parametrize("seed", range(16))
def test_random_shapes_fp64(seed):
    """Random orders 2-5, mode sizes 1-13 and unequal edge ranks 1-8: two
    FP64 sweeps against the oracle (a third of the cases with the phased
    per-column form forced, a third with the Gamma route forced)."""
    from paper_2511_16358_amd import ifctn
    dims, ranks = _random_case(seed)
    p = W.random_problem(dims, ranks, seed=seed, keep=0.6)
    if seed % 3 == 1:          # per-column route, phased form
        ifctn.set_option("phased_min", 0)
        ifctn.set_option("gamma", 0)
    elif seed % 3 == 2:        # Gamma route wherever it fits
        ifctn.set_option("gamma", 2)
    try:
        r = run_both(p, 2, ifctn.IFCTN_FP64)
    finally:
        ifctn.set_option("phased_min", -1)
        ifctn.set_option("gamma", -1)
    assert_x_close(r["Xg"], r["Xo"], 1e-10, (dims, ranks.tolist()))
    for key in r["Go"]:
        assert relerr(r["Gg"][key], r["Go"][key]) < 1e-9, (key, dims)


# --------------------------------------------------------------------------
# the synthetic workload of Sec. 5: 20^4 tensor of Tucker rank (5,5,5,5)
# --------------------------------------------------------------------------
def test_tucker20_fp32_sweeps_match_oracle():
    """The 20^4 Tucker-(5,5,5,5) tensor with 80% of the entries missing:
    five FP32 sweeps in one call against the oracle."""
    from paper_2511_16358_amd import ifctn
    p = W.tucker_problem(seed=0, missing=0.8)
    r = run_both(p, 5, ifctn.IFCTN_FP32, batch=5)
    assert_x_close(r["Xg"], r["Xo"], 1e-5, "tucker20")
    g, o = r["gs"][-1], r["os"][-1]
    assert abs(g["objective"] - o["objective"]) <= 1e-4 * o["objective"]


def test_tucker20_stop_sweep_matches_oracle():
    """Algorithm 1 with the paper's settings (rho = 0.1, eps = 1e-5, t_max =
    1000) on the 20^4 Tucker tensor at 80% missing: the FP32 library stops
    within two sweeps of the oracle, the FP64 library on the same sweep."""
    from paper_2511_16358_amd import ifctn
    p = W.tucker_problem(seed=0, missing=0.8)
    O64 = p.O.astype(np.float64)
    Xo, _, ho = oracle.pam(O64, p.mask, p.G0, p.dims, rho=0.1, t_max=1000, eps=1e-5)
    X64, st64 = ifctn.complete(O64, p.mask, p.G0, p.dims, p.ranks, t_max=1000, eps=1e-5,
                               precision=ifctn.IFCTN_FP64)
    X32, st32 = ifctn.complete(p.O, p.mask, p.G0, p.dims, p.ranks, t_max=1000, eps=1e-5)
    print(f"tucker20: oracle stops after {len(ho)} sweeps, FP64 library {st64['sweeps_done']}, "
          f"FP32 library {st32['sweeps_done']}")
    assert st64["sweeps_done"] == len(ho) and st64["converged"] == 1
    assert_x_close(X64.cpu().numpy(), Xo, 1e-9, "fp64")
    assert abs(st32["sweeps_done"] - len(ho)) <= 2 and st32["converged"] == 1
    assert abs(relerr(X32.cpu().numpy(), p.X_true) - relerr(Xo, p.X_true)) <= 1e-3 * relerr(Xo, p.X_true) + 1e-5
