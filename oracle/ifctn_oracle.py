"""FP64 CPU oracle for iFCTN tensor completion solved by proximal alternating
minimisation (PAM).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import or run this module.  It shares no code with the
HIP library and never imports it; the product path must not call it.

What it follows (paper: "iFCTN: an intra-block Fully-Connected Tensor Network
Decomposition for Tensor Completion", arXiv 2511.16358):

* eq. (iFCTN), Def. 2 -- the entrywise iFCTN decomposition.  Every rank index
  r_{a,b} occurs in exactly two cherry factors, G_{a,b}(r, i_a) and
  G_{b,a}(r, i_b), so the sum over rank tuples splits edge by edge into the
  Hadamard product of the edge matrices G_{a,b}^T G_{b,a}; Prop. 1 builds its
  S_k from the same reshaped products.  :func:`reconstruct` uses that form.
* Prop. 1 -- the mode-k cherry sub-network S_k (:func:`subnetwork_S`).
* Sec. 4.2, eq. (updateG) -- the column-wise closed form of the G_{k,i}
  sub-problem (:func:`update_factor`), assembled literally per column j from
  D = diag(vec S_k), y_j and G_{i,k}.
* eq. (updateX) -- the X step (:func:`update_x`).
* Algorithm 1 -- initialisation, Gauss-Seidel order, stop rule (:func:`pam`);
  its input G^0 drawn by a seeded default of the data's scale
  (:func:`default_factors`, SplitMix64 of Steele, Lea and Flood 2014).
* Sec. 5 -- RSE and RMSE (:func:`rse`, :func:`rmse`), MPSNR and MSSIM of
  image-shaped tensors (:func:`mpsnr`, :func:`mssim`; the standard
  definitions the paper cites, Wang et al. 2004 for SSIM).

Readings of the paper where it is silent or garbled: the data term carries 1/2 (consistent with f and with eq. updateG);
G_{k,m} is new for m < i and old for m > i inside block k, factors of modes
< k are new; y_j is the product of the own-side edge matrices of mode k
except the edge {k,i}; X^0 is O with zeros off Omega; RSE divides by the
norm of the ground truth; RMSE averages over the missing entries; the stop
test runs after the X step with the norm of the previous iterate.

Every function here is pinned by the CPU tests against brute force, special
cases, closed forms and values printed in the paper.

Modes are 0-based; tensors are row-major numpy arrays; a factor set is a dict
``G[(k, i)]`` of arrays of shape (R_ki, I_k).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

FactorDict = dict


# --------------------------------------------------------------------------
# eq. (iFCTN) and Prop. 1
# --------------------------------------------------------------------------
def edges(N):
    """Pairs {a, b}, a < b, of the fully connected network."""
    return [(a, b) for a in range(N) for b in range(a + 1, N)]


def edge_matrix(G, a, b):
    """Contraction of the rank index shared by G_{a,b} and G_{b,a}:
    (G_{a,b}^T G_{b,a})(i_a, i_b), shape I_a x I_b (works for a > b too)."""
    return G[(a, b)].T @ G[(b, a)]


def _on_grid(M, a, b, N):
    """Broadcast a matrix indexed (i_a, i_b) onto an N-mode grid."""
    if a < b:
        shape = [1] * N
        shape[a], shape[b] = M.shape
        return M.reshape(shape)
    return _on_grid(M.T, b, a, N)


def reconstruct(G, dims):
    """iFCTN(G) of eq. (iFCTN): the product over all edges {a,b} of the edge
    matrices, evaluated on the full index grid."""
    N = len(dims)
    X = np.ones(tuple(dims))
    for a, b in edges(N):
        X = X * _on_grid(edge_matrix(G, a, b), a, b, N)
    return X


def subnetwork_S(G, dims, k):
    """S_k of Prop. 1: the Hadamard product over edges {a,b} not containing k
    of the reshaped G_{a,b}^T G_{b,a}.  Returned on the N-mode grid with mode
    k of size 1 (S_k does not depend on i_k)."""
    N = len(dims)
    S = np.ones(tuple(1 if m == k else dims[m] for m in range(N)))
    for a, b in edges(N):
        if k in (a, b):
            continue
        S = S * _on_grid(edge_matrix(G, a, b), a, b, N)
    return S


def own_side_Y(G, dims, k, i):
    """y_j of eq. (updateG) for all j at once: Y(j, i_{-k,-i}) = prod over
    m != k, i of (G_{k,m}^T G_{m,k})(j, i_m).  Mode i has size 1."""
    N = len(dims)
    Y = np.ones(tuple(1 if m == i else dims[m] for m in range(N)))
    for m in range(N):
        if m in (k, i):
            continue
        Y = Y * _on_grid(edge_matrix(G, k, m), k, m, N)
    return Y


# --------------------------------------------------------------------------
# eq. (updateG): one block G_{k,i}, column by column
# --------------------------------------------------------------------------
def block_operands(G, dims, k, i):
    """The parts of eq. (updateG) that are shared by all columns of block
    (k, i): S_k (D = diag(vec S_k)), Y (all y_j) and G_{i,k}."""
    return subnetwork_S(G, dims, k), own_side_Y(G, dims, k, i), G[(i, k)]


def column_system(X, G, dims, k, i, j, rho, operands=None):
    """Normal equations of column j of G_{k,i}.

    The slice i_k = j of iFCTN(G) is linear in g = G_{k,i}(:, j):
    Xhat(j, i_{-k}) = sum_r A_j(i_{-k}, r) g_r with the design matrix
    A_j = D (y_j (x) G_{i,k}^T), i.e.
    A_j(i_{-k}, r) = S_k(i_{-k}) * y_j(i_{-k,-i}) * G_{i,k}(r, i_i).
    Returns (A_j, x_j, H_j, b_j) with H_j = A_j^T A_j + rho I and
    b_j = A_j^T x_j + rho g_old, x_j = X(j, i_{-k}) in the same row order.
    """
    N = len(dims)
    S, Y, Gik = operands if operands is not None else block_operands(G, dims, k, i)
    Yj = np.take(Y, [j], axis=k)                      # mode k -> size 1
    R = Gik.shape[0]
    shape = tuple(1 if m == k else dims[m] for m in range(N))
    SY = np.broadcast_to(S * Yj, shape)
    cols = []
    for r in range(R):
        g_on_i = np.broadcast_to(_axis_vector(Gik[r], i, N), shape)
        cols.append((SY * g_on_i).reshape(-1))
    A = np.stack(cols, axis=1)                        # (prod_{m!=k} I_m) x R
    x = np.take(X, [j], axis=k).reshape(-1)
    g_old = G[(k, i)][:, j]
    H = A.T @ A + rho * np.eye(R)
    b = A.T @ x + rho * g_old
    return A, x, H, b


def _axis_vector(v, axis, N):
    shape = [1] * N
    shape[axis] = v.shape[0]
    return v.reshape(shape)


def update_factor(X, G, dims, k, i, rho, map_columns=map):
    """Solve eq. (updateG) for every column j of G_{k,i} (columns are
    independent: y_j, D and G_{i,k} do not involve G_{k,i}).  The SPD system
    (H_j, b_j) is solved by a Cholesky factorisation.  ``map_columns`` maps
    the per-column solve over the columns (the built-in ``map`` by default; a
    thread pool's map runs the same arithmetic on several cores)."""
    ops = block_operands(G, dims, k, i)

    def solve(j):
        _, _, H, b = column_system(X, G, dims, k, i, j, rho, operands=ops)
        c = scipy.linalg.cho_factor(H, lower=True)
        return scipy.linalg.cho_solve(c, b)

    Gnew = G[(k, i)].copy()
    for j, g in enumerate(map_columns(solve, range(dims[k]))):
        Gnew[:, j] = g
    return Gnew


# --------------------------------------------------------------------------
# eq. (updateX), objective, metrics
# --------------------------------------------------------------------------
def update_x(X, Xhat, O, mask, rho_x):
    """eq. (updateX): O on Omega, (iFCTN(G) + rho X)/(1 + rho) off Omega."""
    m = np.asarray(mask).astype(bool)
    return np.where(m, O, (Xhat + rho_x * X) / (1.0 + rho_x))


def rse(X_true, X):
    """Relative error ||X_true - X||_F / ||X_true||_F (Sec. 5; reading: the
    denominator is the ground truth, as the Observed rows of Table 5 imply)."""
    return float(np.linalg.norm((X_true - X).ravel()) / np.linalg.norm(np.asarray(X_true).ravel()))


def rmse(X_true, X, mask):
    """Root mean square error over the T missing entries (Sec. 5)."""
    miss = ~np.asarray(mask).astype(bool)
    d = (np.asarray(X_true, dtype=np.float64) - X)[miss]
    return float(np.sqrt(np.sum(d * d) / max(d.size, 1)))


def gaussian_window(size=11, sigma=1.5):
    """Normalised size x size Gaussian window of the SSIM definition."""
    ax = np.arange(size, dtype=np.float64) - (size // 2)
    g = np.exp(-(ax[:, None] ** 2 + ax[None, :] ** 2) / (2.0 * sigma * sigma))
    return g / g.sum()


def psnr_bands(X, ref, peak=1.0):
    """PSNR of every band (last mode) of an H x W x B tensor: 10 log10(peak^2 / MSE)."""
    X = np.asarray(X, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    out = []
    for b in range(X.shape[2]):
        mse = np.mean((X[:, :, b] - ref[:, :, b]) ** 2)
        out.append(np.inf if mse == 0 else 10.0 * np.log10(peak * peak / mse))
    return np.array(out)


def ssim_band(x, y, peak=1.0, size=11, sigma=1.5):
    """SSIM of two H x W images: the mean over every position where the
    window fits of ((2 mu_x mu_y + C1)(2 s_xy + C2)) / ((mu_x^2 + mu_y^2 + C1)
    (s_x^2 + s_y^2 + C2)), local statistics weighted by the Gaussian window,
    C1 = (0.01 peak)^2, C2 = (0.03 peak)^2."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    g = gaussian_window(size, sigma)
    c1, c2 = (0.01 * peak) ** 2, (0.03 * peak) ** 2
    H, W = x.shape
    vals = []
    for h in range(H - size + 1):
        for w in range(W - size + 1):
            px = x[h:h + size, w:w + size]
            py = y[h:h + size, w:w + size]
            mx, my = np.sum(g * px), np.sum(g * py)
            vx = np.sum(g * px * px) - mx * mx
            vy = np.sum(g * py * py) - my * my
            cxy = np.sum(g * px * py) - mx * my
            vals.append(((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2)))
    return float(np.mean(vals))


def mpsnr(X, ref, peak=1.0):
    """Mean over bands of the PSNR (Sec. 5)."""
    return float(np.mean(psnr_bands(X, ref, peak)))


def mssim(X, ref, peak=1.0):
    """Mean over bands of the SSIM (Sec. 5)."""
    return float(np.mean([ssim_band(X[:, :, b], ref[:, :, b], peak) for b in range(np.shape(X)[2])]))


def num_parameters(dims, ranks):
    """Storage of the cherry factors: sum over k and i != k of R_{k,i} I_k."""
    N = len(dims)
    return int(sum(ranks[k][i] * dims[k] for k in range(N) for i in range(N) if i != k))


# --------------------------------------------------------------------------
# Algorithm 1
# --------------------------------------------------------------------------
def block_order(N):
    """Gauss-Seidel order of the factor blocks: k ascending, i ascending."""
    return [(k, i) for k in range(N) for i in range(N) if i != k]


def pam_sweep(X, G, O, mask, dims, rho, rho_x=None, map_columns=map):
    """One iteration of Algorithm 1.  Returns (X_new, G_new, stats)."""
    if rho_x is None:
        rho_x = rho
    G = {key: v.copy() for key, v in G.items()}
    dg2 = 0.0
    for k, i in block_order(len(dims)):
        new = update_factor(X, G, dims, k, i, rho, map_columns)
        dg2 += float(np.sum((new - G[(k, i)]) ** 2))
        G[(k, i)] = new
    Xhat = reconstruct(G, dims)
    X_new = update_x(X, Xhat, O, mask, rho_x)
    dx2 = float(np.sum((X_new - X) ** 2))
    x2 = float(np.sum(X * X))
    r = X_new - Xhat
    stats = dict(dx_norm2=dx2, x_norm2=x2, dg_norm2=dg2,
                 rel_change=float(np.sqrt(dx2 / x2)) if x2 > 0 else (0.0 if dx2 == 0 else np.inf),
                 objective=0.5 * float(np.sum(r * r)))
    return X_new, G, stats


def initial_x(O, mask):
    """X^0 = O on Omega and 0 elsewhere."""
    m = np.asarray(mask).astype(bool)
    return np.where(m, np.asarray(O, dtype=np.float64), 0.0)


# --------------------------------------------------------------------------
# A seeded default G^0 (Algorithm 1 takes G^0 as an input and leaves its
# distribution open)
# --------------------------------------------------------------------------
def splitmix64(seed, n):
    """Outputs n (an integer array) of SplitMix64 started from state `seed`
    (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
    OOPSLA 2014): the state advances by the odd constant 0x9E3779B97F4A7C15 per
    output, so output n mixes seed + (n + 1) * 0x9E3779B97F4A7C15 (mod 2^64) by
    z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB;
    z ^= z >> 31 (all mod 2^64)."""
    u64 = np.uint64
    with np.errstate(over="ignore"):
        z = u64(seed) + (np.asarray(n, dtype=u64) + u64(1)) * u64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> u64(30))) * u64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> u64(27))) * u64(0x94D049BB133111EB)
        return z ^ (z >> u64(31))


def default_factors(O, mask, dims, ranks, seed=0):
    """Uniform initial factors with the scale of the data.  Entry n of the
    factors taken in block order (k ascending, i ascending, each R_ki x I_k
    row-major) is s * u_n, u_n = (SplitMix64 output n >> 11) / 2^53 in [0, 1).
    Entries of mean s/2 make E[W_ab] = R_ab s^2 / 4 for every edge matrix, and
    distinct edges use distinct factors, so E[Xhat] = prod_{a<b} R_ab s^2 / 4
    (eq. (iFCTN)); s sets that to m, the root mean square of the observed
    entries (m = 1 when none is observed or all are 0):
    s = 2 (m / prod R_ab)^(1 / (2e)) over the e = N(N-1)/2 edges."""
    N = len(dims)
    vals = np.asarray(O, dtype=np.float64)[np.asarray(mask).astype(bool)]
    m = float(np.sqrt(np.mean(vals * vals))) if vals.size else 0.0
    if not (m > 0.0) or not np.isfinite(m):
        m = 1.0
    prod_r = 1.0
    for a, b in edges(N):
        prod_r *= ranks[a][b]
    s = 2.0 * (m / prod_r) ** (1.0 / (2.0 * len(edges(N))))
    G, n0 = {}, 0
    for k, i in block_order(N):
        cnt = int(ranks[k][i]) * int(dims[k])
        u = (splitmix64(seed, np.arange(n0, n0 + cnt)) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
        G[(k, i)] = s * u.reshape(int(ranks[k][i]), int(dims[k]))
        n0 += cnt
    return G


def pam(O, mask, G0, dims, rho=0.1, t_max=1000, eps=1e-5, rho_x=None, callback=None):
    """Algorithm 1: sweeps until ||X^{s+1} - X^s|| / ||X^s|| < eps or s = t_max.
    eps = 0 runs exactly t_max sweeps.  Returns (X, G, history)."""
    X = initial_x(O, mask)
    G = {key: np.asarray(v, dtype=np.float64).copy() for key, v in G0.items()}
    O64 = np.asarray(O, dtype=np.float64)
    hist = []
    for s in range(t_max):
        X, G, st = pam_sweep(X, G, O64, mask, dims, rho, rho_x)
        hist.append(st)
        if callback is not None:
            callback(s, X, G, st)
        if st["rel_change"] < eps:
            break
    return X, G, hist
