"""Checks that pin the FP64 oracle to the paper and to mathematics.

Each ``check_*`` function raises AssertionError when the oracle module it is
given disagrees with something fixed independently of the oracle: brute-force
sums, explicit Kronecker / Khatri-Rao matrices built from the definitions,
least-squares problems solved by a library routine, optimality conditions,
closed-form special cases and values printed in the paper.  The same checks
run against deliberately broken copies of the oracle (test_oracle_mutations)
to show that each plausible mistake is caught.
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# tiny random factor sets
# --------------------------------------------------------------------------
def rand_factors(dims, ranks, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    N = len(dims)
    return {(k, i): scale * rng.standard_normal((int(ranks[k][i]), dims[k]))
            for k in range(N) for i in range(N) if i != k}


def sym_ranks(N, values):
    """Symmetric rank matrix from the upper-triangle values (a<b order)."""
    r = np.zeros((N, N), dtype=int)
    it = iter(values)
    for a in range(N):
        for b in range(a + 1, N):
            r[a][b] = r[b][a] = next(it)
    return r


# --------------------------------------------------------------------------
# independent evaluations of the decomposition
# --------------------------------------------------------------------------
def brute_force_ifctn(G, dims, ranks):
    """eq. (iFCTN) summed literally: for every entry, the sum over all tuples
    (r_{a,b})_{a<b} of the product of all N(N-1) cherry-factor entries."""
    N = len(dims)
    pairs = [(a, b) for a in range(N) for b in range(a + 1, N)]
    out = np.zeros(dims)
    for idx in itertools.product(*[range(d) for d in dims]):
        total = 0.0
        for rt in itertools.product(*[range(ranks[a][b]) for a, b in pairs]):
            r = {}
            for (a, b), v in zip(pairs, rt):
                r[(a, b)] = r[(b, a)] = v
            p = 1.0
            for k in range(N):
                for i in range(N):
                    if i != k:
                        p *= G[(k, i)][r[(k, i)], idx[k]]
            total += p
        out[idx] = total
    return out


def kr(A, B):
    """Khatri-Rao product as defined in Sec. 2.1: for A (m x r), B (n x r),
    C[(i-1)n + j, l] = A[i, l] B[j, l] (1-based)."""
    m, r = A.shape
    n, r2 = B.shape
    assert r == r2
    C = np.zeros((m * n, r))
    for i in range(m):
        for j in range(n):
            C[i * n + j, :] = A[i, :] * B[j, :]
    return C


def lin_index(idx, dims):
    """Paper's linear index (Sec. 2.1), 0-based: mode 1 fastest."""
    li, stride = 0, 1
    for i, d in zip(idx, dims):
        li += i * stride
        stride *= d
    return li


def unfold(T, k):
    """Mode-k unfolding with the paper's column order (remaining modes, the
    lowest mode fastest): shape I_k x prod_{m != k} I_m."""
    dims = T.shape
    rest = [m for m in range(T.ndim) if m != k]
    U = np.zeros((dims[k], int(np.prod([dims[m] for m in rest]))))
    for idx in itertools.product(*[range(d) for d in dims]):
        col = lin_index([idx[m] for m in rest], [dims[m] for m in rest])
        U[idx[k], col] = T[idx]
    return U


def cherry_tensor(G, dims, ranks, k):
    """Def. 1 evaluated entrywise: the mode-k cherry tensor of the factors
    {G_{k,i}}, of shape (R_{k,1}, ..., I_k, ..., R_{k,N})."""
    N = len(dims)
    shape = [dims[k] if m == k else ranks[k][m] for m in range(N)]
    T = np.zeros(shape)
    for idx in itertools.product(*[range(s) for s in shape]):
        p = 1.0
        for m in range(N):
            if m != k:
                p *= G[(k, m)][idx[m], idx[k]]
        T[idx] = p
    return T


def kr_chain_own(G, k, N):
    """(G_(k))^T = M_N (.) ... (.) M_{k+1} (.) M_{k-1} (.) ... (.) M_1 with
    M_i = G_{k,i}, each transposed so that the shared dimension I_k is the
    KR column dimension: result (prod_i R_{k,i}) x I_k."""
    mats = [G[(k, m)] for m in reversed(range(N)) if m != k]
    out = mats[0]
    for M in mats[1:]:
        out = kr(out, M)
    return out


# --------------------------------------------------------------------------
# P1 / P4: reconstruction against brute force
# --------------------------------------------------------------------------
def check_reconstruct_brute(O, cases=None, tol=1e-12):
    cases = cases or [((3, 4, 2), sym_ranks(3, [2, 3, 1])),
                      ((2, 3, 2, 2), sym_ranks(4, [2, 1, 2, 2, 1, 2])),
                      ((4, 3), sym_ranks(2, [3]))]
    for s, (dims, ranks) in enumerate(cases):
        G = rand_factors(dims, ranks, seed=100 + s)
        ref = brute_force_ifctn(G, dims, ranks)
        got = O.reconstruct(G, dims)
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        assert err < tol, f"reconstruct vs brute force {dims}: {err}"


def check_n3_remark(O, tol=1e-12):
    """The N = 3 triple sum of the remark after Def. 2."""
    dims = (3, 2, 4)
    ranks = sym_ranks(3, [2, 3, 2])
    G = rand_factors(dims, ranks, seed=7)
    ref = np.zeros(dims)
    for i1, i2, i3 in itertools.product(*[range(d) for d in dims]):
        s = 0.0
        for r12 in range(ranks[0][1]):
            for r13 in range(ranks[0][2]):
                for r23 in range(ranks[1][2]):
                    s += (G[(0, 1)][r12, i1] * G[(0, 2)][r13, i1] * G[(1, 0)][r12, i2]
                          * G[(1, 2)][r23, i2] * G[(2, 0)][r13, i3] * G[(2, 1)][r23, i3])
        ref[i1, i2, i3] = s
    got = O.reconstruct(G, dims)
    assert np.max(np.abs(got - ref)) < tol * np.max(np.abs(ref))


# --------------------------------------------------------------------------
# P2 / P3: Def. 1 and Prop. 1 with explicit matrices
# --------------------------------------------------------------------------
def check_cherry_kr(O=None):
    """(G_(k))^T from the KR chain equals the transposed unfolding of the
    entrywise cherry tensor (Def. 1 with the Sec. 2.1 conventions)."""
    dims = (3, 4, 2)
    ranks = sym_ranks(3, [2, 3, 2])
    G = rand_factors(dims, ranks, seed=11)
    for k in range(3):
        T = cherry_tensor(G, dims, ranks, k)
        lhs = unfold(T, k).T
        rhs = kr_chain_own(G, k, 3)
        assert np.allclose(lhs, rhs, rtol=0, atol=1e-13), k


def check_subnetwork(O, tol=1e-12):
    """Prop. 1: X_(k)^T = Z_k (G_(k))^T with the explicit
    Z_k = diag(vec S_k) (G_{N,k}^T (x) ... (x) G_{1,k}^T) (mode k skipped)."""
    for dims, ranks, seed in [((3, 4, 2), sym_ranks(3, [2, 3, 2]), 3),
                              ((2, 3, 2, 3), sym_ranks(4, [2, 1, 2, 2, 2, 1]), 4)]:
        N = len(dims)
        G = rand_factors(dims, ranks, seed)
        Xt = O.reconstruct(G, dims)
        for k in range(N):
            S = O.subnetwork_S(G, dims, k)
            S_t = np.squeeze(S, axis=k)
            rest = [m for m in range(N) if m != k]
            vecS = np.zeros(S_t.size)
            for idx in itertools.product(*[range(dims[m]) for m in rest]):
                vecS[lin_index(idx, [dims[m] for m in rest])] = S_t[idx]
            K = None
            for m in reversed(rest):
                K = G[(m, k)].T if K is None else np.kron(K, G[(m, k)].T)
            Z = np.diag(vecS) @ K
            lhs = unfold(Xt, k).T
            rhs = Z @ kr_chain_own(G, k, N)
            assert np.max(np.abs(lhs - rhs)) < tol * np.max(np.abs(lhs)), (dims, k)


# --------------------------------------------------------------------------
# P5 / P15: Prop. 3 and the gauge freedom of each edge
# --------------------------------------------------------------------------
def check_transposition(O, tol=1e-12):
    dims = (3, 2, 4, 2)
    ranks = sym_ranks(4, [2, 1, 3, 2, 1, 2])
    G = rand_factors(dims, ranks, seed=21)
    X = O.reconstruct(G, dims)
    for n in [(2, 0, 3, 1), (3, 2, 1, 0), (1, 0, 2, 3)]:
        dn = tuple(dims[m] for m in n)
        Gn = {(k, j): G[(n[k], n[j])] for k in range(4) for j in range(4) if k != j}
        Xn = O.reconstruct(Gn, dn)
        assert np.max(np.abs(Xn - X.transpose(n))) < tol * np.max(np.abs(X)), n


def check_gauge(O, tol=1e-11):
    dims = (3, 4, 5)
    ranks = sym_ranks(3, [3, 2, 3])
    G = rand_factors(dims, ranks, seed=5)
    X = O.reconstruct(G, dims)
    rng = np.random.default_rng(9)
    Gq = dict(G)
    for a, b in [(0, 1), (1, 2)]:
        Q = rng.standard_normal((ranks[a][b], ranks[a][b])) + 3 * np.eye(ranks[a][b])
        Gq[(a, b)] = Q @ G[(a, b)]
        Gq[(b, a)] = np.linalg.inv(Q).T @ G[(b, a)]
    Xq = O.reconstruct(Gq, dims)
    assert np.max(np.abs(Xq - X)) < tol * np.max(np.abs(X))


# --------------------------------------------------------------------------
# P6 / P7 / P8: the block sub-problem
# --------------------------------------------------------------------------
def probe_design(O, G, dims, k, i, j):
    """Columns of the design matrix of column j of G_{k,i}, obtained by
    evaluating the reconstruction with G_{k,i}(:, j) set to unit vectors."""
    R = G[(k, i)].shape[0]
    cols = []
    for r in range(R):
        Gp = dict(G)
        g = G[(k, i)].copy()
        g[:, j] = 0.0
        g[r, j] = 1.0
        Gp[(k, i)] = g
        cols.append(np.take(O.reconstruct(Gp, dims), [j], axis=k).reshape(-1))
    return np.stack(cols, axis=1)


def ridge_lstsq(A, x, g_old, rho):
    """argmin_g 1/2||A g - x||^2 + rho/2 ||g - g_old||^2 as an ordinary
    least-squares problem on the stacked system [A; sqrt(rho) I]."""
    R = A.shape[1]
    M = np.vstack([A, np.sqrt(rho) * np.eye(R)])
    y = np.concatenate([x, np.sqrt(rho) * g_old])
    return np.linalg.lstsq(M, y, rcond=None)[0]


def check_n2_ridge(O, tol=1e-10):
    """N = 2: every column update is a ridge regression against the other
    factor (proximal ALS for matrix completion)."""
    dims = (6, 5)
    ranks = sym_ranks(2, [3])
    G = rand_factors(dims, ranks, seed=31)
    rng = np.random.default_rng(32)
    X = rng.standard_normal(dims)
    rho = 0.1
    new01 = O.update_factor(X, G, dims, 0, 1, rho)
    for j in range(dims[0]):
        ref = ridge_lstsq(G[(1, 0)].T, X[j, :], G[(0, 1)][:, j], rho)
        assert np.max(np.abs(new01[:, j] - ref)) < tol * max(1, np.max(np.abs(ref)))
    new10 = O.update_factor(X, G, dims, 1, 0, rho)
    for j in range(dims[1]):
        ref = ridge_lstsq(G[(0, 1)].T, X[:, j], G[(1, 0)][:, j], rho)
        assert np.max(np.abs(new10[:, j] - ref)) < tol * max(1, np.max(np.abs(ref)))


PROBE_CASES = [((4, 4, 4), [2, 3, 2]),          # equal sizes: catches transposed operands
               ((3, 5, 4), [2, 1, 3]),
               ((3, 2, 3, 2), [2, 1, 2, 2, 1, 2])]


def check_block_probe(O, tol=1e-9):
    """Each block's columns equal the least-squares solution built from the
    probed design matrix (P7), satisfy the first-order condition and decrease
    f + rho/2 ||dG||^2 (P8)."""
    rho = 0.1
    for c, (dims, rv) in enumerate(PROBE_CASES):
        N = len(dims)
        ranks = sym_ranks(N, rv)
        G = rand_factors(dims, ranks, seed=40 + c)
        rng = np.random.default_rng(50 + c)
        X = rng.standard_normal(dims)
        for k in range(N):
            for i in range(N):
                if i == k:
                    continue
                new = O.update_factor(X, G, dims, k, i, rho)
                for j in range(dims[k]):
                    A = probe_design(O, G, dims, k, i, j)
                    x = np.take(X, [j], axis=k).reshape(-1)
                    g_old = G[(k, i)][:, j]
                    ref = ridge_lstsq(A, x, g_old, rho)
                    g = new[:, j]
                    scale = max(1.0, np.max(np.abs(ref)))
                    assert np.max(np.abs(g - ref)) < tol * scale, (dims, k, i, j)
                    grad = A.T @ (A @ g - x) + rho * (g - g_old)
                    assert np.max(np.abs(grad)) < tol * max(1.0, np.max(np.abs(A.T @ x))), \
                        (dims, k, i, j)
                Gn = dict(G)
                Gn[(k, i)] = new
                f0 = 0.5 * np.sum((X - O.reconstruct(G, dims)) ** 2)
                f1 = 0.5 * np.sum((X - O.reconstruct(Gn, dims)) ** 2)
                assert f1 + 0.5 * rho * np.sum((new - G[(k, i)]) ** 2) <= f0 * (1 + 1e-12) + 1e-12


def check_spd(O):
    """P16: H_j = A_j^T A_j + rho I has all eigenvalues >= rho."""
    dims = (3, 5, 4)
    ranks = sym_ranks(3, [2, 3, 3])
    G = rand_factors(dims, ranks, seed=61)
    X = np.random.default_rng(62).standard_normal(dims)
    rho = 0.1
    for k, i in [(0, 1), (1, 2), (2, 0)]:
        for j in range(dims[k]):
            _, _, H, _ = O.column_system(X, G, dims, k, i, j, rho)
            assert np.allclose(H, H.T, rtol=0, atol=1e-12)
            assert np.min(np.linalg.eigvalsh(H)) >= rho * (1 - 1e-10)


# --------------------------------------------------------------------------
# P10: the X step
# --------------------------------------------------------------------------
def check_x_update(O):
    rng = np.random.default_rng(71)
    dims = (5, 6, 7)
    Xs = rng.standard_normal(dims)
    Xhat = rng.standard_normal(dims)
    Obs = rng.standard_normal(dims)
    mask = rng.random(dims) < 0.4
    for rho in (0.1, 1.0, 3.0):
        Xn = O.update_x(Xs, Xhat, Obs, mask, rho)
        assert np.array_equal(Xn[mask], Obs[mask])
        # first-order condition of 1/2 (x - xhat)^2 + rho/2 (x - x_s)^2
        g = (Xn - Xhat) + rho * (Xn - Xs)
        assert np.max(np.abs(g[~mask])) < 1e-12


# --------------------------------------------------------------------------
# sweep level: Gauss-Seidel order (replay), Lemma 2, stop rule, fixed point
# --------------------------------------------------------------------------
def replay_sweep(O, X, G, Obs, mask, dims, rho):
    """One sweep rebuilt from probed least-squares blocks in the order of
    Algorithm 1, then the X step as the minimiser of its separable problem."""
    N = len(dims)
    G = {key: v.copy() for key, v in G.items()}
    for k in range(N):
        for i in range(N):
            if i == k:
                continue
            new = G[(k, i)].copy()
            for j in range(dims[k]):
                A = probe_design(O, G, dims, k, i, j)
                x = np.take(X, [j], axis=k).reshape(-1)
                new[:, j] = ridge_lstsq(A, x, G[(k, i)][:, j], rho)
            G[(k, i)] = new
    Xhat = O.reconstruct(G, dims)
    m = np.asarray(mask).astype(bool)
    # minimiser of 1/2 (x - xhat)^2 + rho/2 (x - x_s)^2 off Omega
    Xn = np.where(m, Obs, (Xhat + rho * X) / (1 + rho))
    return Xn, G


def check_sweep_replay(O, tol=1e-9):
    for c, (dims, rv) in enumerate(PROBE_CASES[:2]):
        N = len(dims)
        ranks = sym_ranks(N, rv)
        rng = np.random.default_rng(80 + c)
        G = rand_factors(dims, ranks, seed=90 + c, scale=0.7)
        Obs = rng.standard_normal(dims)
        mask = rng.random(dims) < 0.6
        X = np.where(mask, Obs, 0.0)
        Xo, Go, _ = O.pam_sweep(X, G, Obs, mask, dims, 0.1)
        Xr, Gr = replay_sweep(O, X, G, Obs, mask, dims, 0.1)
        assert np.max(np.abs(Xo - Xr)) < tol * max(1, np.max(np.abs(Xr))), dims
        for key in G:
            assert np.max(np.abs(Go[key] - Gr[key])) < tol * max(1, np.max(np.abs(Gr[key]))), key


def check_lemma2(O, sweeps=6):
    """Lemma 2: F^s - F^{s+1} >= rho/2 ||M^{s+1} - M^s||^2 for every sweep."""
    dims = (6, 5, 7)
    ranks = sym_ranks(3, [2, 2, 3])
    rng = np.random.default_rng(101)
    Obs = rng.uniform(0, 1, dims)
    mask = rng.random(dims) < 0.5
    G = rand_factors(dims, ranks, seed=102, scale=0.8)
    X = np.where(mask, Obs, 0.0)
    rho = 0.1
    F = 0.5 * np.sum((X - O.reconstruct(G, dims)) ** 2)
    for s in range(sweeps):
        Xn, Gn, st = O.pam_sweep(X, G, Obs, mask, dims, rho)
        Fn = 0.5 * np.sum((Xn - O.reconstruct(Gn, dims)) ** 2)
        dM = np.sum((Xn - X) ** 2) + sum(np.sum((Gn[key] - G[key]) ** 2) for key in G)
        assert F - Fn >= 0.5 * rho * dM - 1e-12 * max(F, 1.0), (s, F - Fn, 0.5 * rho * dM)
        assert abs(st["objective"] - Fn) <= 1e-10 * max(Fn, 1e-300)
        X, G, F = Xn, Gn, Fn


def check_stop_rule(O):
    """rel = ||X^{s+1} - X^s|| / ||X^s|| after the X step; Algorithm 1 stops at
    the first sweep below eps; eps = 0 runs all t_max sweeps."""
    dims = (5, 4, 6)
    ranks = sym_ranks(3, [2, 2, 2])
    rng = np.random.default_rng(111)
    Obs = rng.uniform(0, 1, dims)
    mask = rng.random(dims) < 0.5
    G0 = rand_factors(dims, ranks, seed=112, scale=0.8)
    snaps = []

    def cb(s, X, G, st):
        snaps.append(X.copy())

    X, G, hist = O.pam(np.where(mask, Obs, 0), mask, G0, dims, rho=0.1, t_max=8, eps=0.0,
                       callback=cb)
    assert len(hist) == 8
    prev = np.where(mask, Obs, 0.0)
    for s in range(8):
        rel = np.linalg.norm((snaps[s] - prev).ravel()) / np.linalg.norm(prev.ravel())
        assert abs(hist[s]["rel_change"] - rel) <= 1e-12 * rel, s
        prev = snaps[s]
    eps = 0.5 * (hist[3]["rel_change"] + hist[4]["rel_change"])
    stop = next(s for s in range(8) if hist[s]["rel_change"] < eps)
    _, _, h2 = O.pam(np.where(mask, Obs, 0), mask, G0, dims, rho=0.1, t_max=8, eps=eps)
    assert len(h2) == stop + 1


def check_fixed_point(O, tol=1e-12):
    """Fully observed O = iFCTN(G*) with G^0 = G*: one sweep changes nothing
    (every block's minimiser is the current value, the X step keeps O)."""
    dims = (4, 5, 3)
    ranks = sym_ranks(3, [2, 3, 2])
    G = rand_factors(dims, ranks, seed=121)
    Xs = O.reconstruct(G, dims)
    mask = np.ones(dims, dtype=bool)
    Xn, Gn, st = O.pam_sweep(Xs, G, Xs, mask, dims, 0.1)
    assert np.max(np.abs(Xn - Xs)) == 0.0
    for key in G:
        assert np.max(np.abs(Gn[key] - G[key])) < tol * max(1, np.max(np.abs(G[key]))), key
    assert st["objective"] < 1e-20 * max(1.0, float(np.sum(Xs * Xs)))


# --------------------------------------------------------------------------
# values printed in the paper
# --------------------------------------------------------------------------
def check_storage_count(O):
    g = golden()["flower_storage"]
    dims, R = g["dims"], g["rank"]
    ranks = [[0 if a == b else R for b in range(3)] for a in range(3)]
    n = O.num_parameters(dims, ranks)
    assert n == g["parameters"], n
    ratio = 100.0 * n / np.prod(dims)
    assert round(ratio, 2) == g["storage_ratio_percent"], ratio


def check_observed_rows(O):
    """The 'Observed' rows of Table 5: RSE of the zero-filled observation is
    sqrt(missing ratio) (denominator = ground truth; zero fill), and RMSE over
    the missing entries does not depend on the missing ratio."""
    g = golden()["observed_rows_guangzhou"]
    rng = np.random.default_rng(131)
    dims = (214, 61, 144)
    Xt = rng.uniform(0.2, 0.8, dims)
    rmses = []
    for miss, printed in zip(g["missing_ratio"], g["rse"]):
        mask = rng.random(dims) >= miss
        X0 = O.initial_x(np.where(mask, Xt, 7.0), mask)
        val = O.rse(Xt, X0)
        assert abs(val - printed) <= 0.0015, (miss, val, printed)
        rmses.append(O.rmse(Xt, X0, mask))
    rms = np.sqrt(np.mean(Xt * Xt))
    assert np.max(np.abs(np.array(rmses) / rms - 1.0)) < 0.01, rmses


def check_image_metrics(O):
    """MPSNR / MSSIM against closed forms and an independent route to the
    local statistics (scipy's 2-D correlation with the same window)."""
    from scipy.signal import correlate2d
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 1, size=(17, 15))
    assert abs(O.ssim_band(x, x) - 1.0) < 1e-12                     # identical images
    y = np.clip(x + rng.normal(0, 0.1, size=x.shape), 0, 1)
    assert abs(O.ssim_band(x, y) - O.ssim_band(y, x)) < 1e-14        # symmetric
    # constant offset d: variances and covariance unchanged, so each window
    # gives (2 mu (mu + d) + C1) / (mu^2 + (mu + d)^2 + C1)
    d = 0.05
    ax = np.arange(11) - 5.0
    g = np.exp(-(ax[:, None] ** 2 + ax[None, :] ** 2) / (2 * 1.5 ** 2))
    g /= g.sum()
    mu = correlate2d(x, g, mode="valid")
    c1 = 0.01 ** 2
    want = np.mean((2 * mu * (mu + d) + c1) / (mu * mu + (mu + d) ** 2 + c1))
    assert abs(O.ssim_band(x, x + d) - want) < 1e-12
    # contrast change at equal means: a window with x -> mean + a (x - mean)
    # has SSIM (2 a s^2 + C2) / ((1 + a^2) s^2 + C2); check on a flat-mean image
    z = rng.uniform(0, 1, size=(11, 11))
    gm = np.sum(g * z)
    z2 = gm + 0.5 * (z - gm)
    s2 = np.sum(g * z * z) - gm * gm
    c2 = 0.03 ** 2
    assert abs(O.ssim_band(z, z2) - (2 * 0.5 * s2 + c2) / ((1 + 0.25) * s2 + c2)) < 1e-12
    # PSNR of a constant error d is 10 log10(1 / d^2); MPSNR / MSSIM are band means
    X = rng.uniform(0, 1, size=(12, 13, 3))
    assert np.allclose(O.psnr_bands(X + d, X), 10 * np.log10(1 / d ** 2), atol=1e-9)
    assert np.allclose(O.psnr_bands(X + d, X, peak=2.0), 10 * np.log10(4 / d ** 2), atol=1e-9)
    assert abs(O.mpsnr(X + d, X) - 10 * np.log10(1 / d ** 2)) < 1e-9
    Y = np.clip(X + rng.normal(0, 0.05, size=X.shape), 0, 1)
    assert abs(O.mssim(Y, X) - np.mean([O.ssim_band(Y[:, :, b], X[:, :, b]) for b in range(3)])) < 1e-15


def check_default_factors(O):
    """The seeded default G^0: SplitMix64's published first outputs from state
    0, entry n of the block order drawn from output n, and E[iFCTN(G^0)] = m,
    the root mean square of the observed entries (averaged over 1000 seeds,
    order 3, unequal ranks)."""
    assert [int(v) for v in O.splitmix64(0, [0, 1, 2])] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                           0x06C45D188009454F]
    rng = np.random.default_rng(11)
    dims = (6, 5, 4)
    R = sym_ranks(3, [2, 3, 4])
    X = 5.0 * rng.random(dims)
    mask = rng.random(dims) < 0.3
    m = np.sqrt(np.mean(X[mask] ** 2))
    G = O.default_factors(X, mask, dims, R, seed=5)
    flat = np.concatenate([G[key].ravel() for key in O.block_order(3)])
    s = 2.0 * (m / 24.0) ** (1.0 / 6.0)
    for n in (0, flat.size - 1):
        assert flat[n] == s * float(int(O.splitmix64(5, n)) >> 11) * 2.0 ** -53
    means = [np.mean(O.reconstruct(O.default_factors(X, mask, dims, R, seed), dims)) for seed in range(1000)]
    assert abs(np.mean(means) / m - 1.0) < 0.08


ALL_CHECKS = [
    check_image_metrics,
    check_reconstruct_brute, check_n3_remark, check_cherry_kr, check_subnetwork,
    check_transposition, check_gauge, check_n2_ridge, check_block_probe, check_spd,
    check_x_update, check_sweep_replay, check_lemma2, check_stop_rule, check_fixed_point,
    check_storage_count, check_observed_rows, check_default_factors,
]
