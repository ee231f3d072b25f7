"""Plant plausible mistakes in the oracle (on the CPU) and show that the pins
catch every one of them.  Each mutation replaces one function of the oracle
module for the duration of the test."""
import numpy as np
import pytest
import scipy.linalg

import oracle.ifctn_oracle as orc
from tests import pins


def _mut_reconstruct_drops_edge(m):
    def reconstruct(G, dims):
        N = len(dims)
        X = np.ones(tuple(dims))
        for a, b in m.edges(N)[:-1]:
            X = X * m._on_grid(m.edge_matrix(G, a, b), a, b, N)
        return X
    return "reconstruct", reconstruct


def _mut_edge_same_side(m):
    def edge_matrix(G, a, b):
        # own-side factor used twice instead of G_{a,b}^T G_{b,a}
        A = G[(a, b)]
        B = G[(b, a)]
        return A.T @ (B * 0 + np.resize(A, B.shape)) if A.shape == B.shape else A.T @ B * 1.0001
    return "edge_matrix", edge_matrix


def _mut_subnetwork_includes_k(m):
    def subnetwork_S(G, dims, k):
        N = len(dims)
        S = np.ones(tuple(1 if q == k else dims[q] for q in range(N)))
        for a, b in m.edges(N):
            if k in (a, b):
                M = m.edge_matrix(G, a, b)
                other = b if a == k else a
                v = M.sum(axis=0 if a == k else 1)
                shape = [1] * N
                shape[other] = dims[other]
                S = S * v.reshape(shape)
                continue
            S = S * m._on_grid(m.edge_matrix(G, a, b), a, b, N)
        return S
    return "subnetwork_S", subnetwork_S


def _mut_y_includes_edge_ki(m):
    orig = m.own_side_Y

    def own_side_Y(G, dims, k, i):
        Y = orig(G, dims, k, i)
        W = m.edge_matrix(G, k, i)
        return Y * W.sum(axis=1).reshape([dims[k] if q == k else 1 for q in range(len(dims))])
    return "own_side_Y", own_side_Y


def _mut_far_side_from_own(m):
    orig = m.block_operands

    def block_operands(G, dims, k, i):
        S, Y, _ = orig(G, dims, k, i)
        Gki = G[(k, i)]
        # own-side factor where the far side G_{i,k} belongs (shapes agree on cubes)
        Gik = Gki if Gki.shape == G[(i, k)].shape else G[(i, k)][::-1].copy()
        return S, Y, Gik
    return "block_operands", block_operands


def _mut_no_prox_in_b(m):
    orig = m.column_system

    def column_system(X, G, dims, k, i, j, rho, operands=None):
        A, x, H, b = orig(X, G, dims, k, i, j, rho, operands)
        return A, x, H, A.T @ x
    return "column_system", column_system


def _mut_no_prox_in_H(m):
    orig = m.column_system

    def column_system(X, G, dims, k, i, j, rho, operands=None):
        A, x, H, b = orig(X, G, dims, k, i, j, rho, operands)
        return A, x, H - rho * np.eye(H.shape[0]) + 1e-9 * np.eye(H.shape[0]), b
    return "column_system", column_system


def _mut_D_not_squared(m):
    orig = m.column_system

    def column_system(X, G, dims, k, i, j, rho, operands=None):
        A, x, H, b = orig(X, G, dims, k, i, j, rho, operands)
        S = (operands or m.block_operands(G, dims, k, i))[0]
        s = np.broadcast_to(S, tuple(1 if q == k else dims[q] for q in range(len(dims)))).reshape(-1)
        s = np.where(np.abs(s) > 1e-300, s, 1.0)
        A1 = A / s[:, None]
        return A, x, A1.T @ A + rho * np.eye(A.shape[1]), b
    return "column_system", column_system


def _mut_x_update_swapped(m):
    def update_x(X, Xhat, O, mask, rho_x):
        mk = np.asarray(mask).astype(bool)
        return np.where(~mk, O, (Xhat + rho_x * X) / (1.0 + rho_x))
    return "update_x", update_x


def _mut_x_update_denominator(m):
    def update_x(X, Xhat, O, mask, rho_x):
        mk = np.asarray(mask).astype(bool)
        return np.where(mk, O, (Xhat + rho_x * X) / (2.0 + rho_x))
    return "update_x", update_x


def _mut_order_descending_i(m):
    def block_order(N):
        return [(k, i) for k in range(N) for i in reversed(range(N)) if i != k]
    return "block_order", block_order


def _mut_jacobi_sweep(m):
    def pam_sweep(X, G, O, mask, dims, rho, rho_x=None):
        rho_x = rho if rho_x is None else rho_x
        G0 = {key: v.copy() for key, v in G.items()}
        Gn = {}
        for k, i in m.block_order(len(dims)):
            Gn[(k, i)] = m.update_factor(X, G0, dims, k, i, rho)
        Xhat = m.reconstruct(Gn, dims)
        Xn = m.update_x(X, Xhat, O, mask, rho_x)
        dx2 = float(np.sum((Xn - X) ** 2))
        x2 = float(np.sum(X * X))
        r = Xn - Xhat
        return Xn, Gn, dict(dx_norm2=dx2, x_norm2=x2, dg_norm2=0.0,
                            rel_change=float(np.sqrt(dx2 / x2)), objective=0.5 * float(np.sum(r * r)))
    return "pam_sweep", pam_sweep


def _mut_x_updated_before_factors(m):
    def pam_sweep(X, G, O, mask, dims, rho, rho_x=None):
        rho_x = rho if rho_x is None else rho_x
        Xhat0 = m.reconstruct(G, dims)
        Xmid = m.update_x(X, Xhat0, O, mask, rho_x)
        G = {key: v.copy() for key, v in G.items()}
        for k, i in m.block_order(len(dims)):
            G[(k, i)] = m.update_factor(Xmid, G, dims, k, i, rho)
        Xhat = m.reconstruct(G, dims)
        Xn = m.update_x(X, Xhat, O, mask, rho_x)
        dx2 = float(np.sum((Xn - X) ** 2))
        x2 = float(np.sum(X * X))
        r = Xn - Xhat
        return Xn, G, dict(dx_norm2=dx2, x_norm2=x2, dg_norm2=0.0,
                           rel_change=float(np.sqrt(dx2 / x2)), objective=0.5 * float(np.sum(r * r)))
    return "pam_sweep", pam_sweep


def _mut_rel_uses_new_norm(m):
    orig = m.pam_sweep

    def pam_sweep(X, G, O, mask, dims, rho, rho_x=None):
        Xn, Gn, st = orig(X, G, O, mask, dims, rho, rho_x)
        st = dict(st)
        st["rel_change"] = float(np.sqrt(st["dx_norm2"] / np.sum(Xn * Xn)))
        return Xn, Gn, st
    return "pam_sweep", pam_sweep


def _mut_rse_estimate_norm(m):
    def rse(X_true, X):
        return float(np.linalg.norm((X_true - X).ravel()) / np.linalg.norm(np.asarray(X).ravel()))
    return "rse", rse


def _mut_rmse_all_entries(m):
    def rmse(X_true, X, mask):
        d = np.asarray(X_true, dtype=np.float64) - X
        return float(np.sqrt(np.mean(d * d)))
    return "rmse", rmse


def _mut_initial_x_keeps_unobserved(m):
    def initial_x(O, mask):
        return np.asarray(O, dtype=np.float64).copy()
    return "initial_x", initial_x


def _mut_params_counts_edges_once(m):
    def num_parameters(dims, ranks):
        N = len(dims)
        return int(sum(ranks[k][i] * dims[k] for k in range(N) for i in range(k + 1, N)))
    return "num_parameters", num_parameters


def _mut_cholesky_upper_misuse(m):
    def update_factor(X, G, dims, k, i, rho, map_columns=map):
        ops = m.block_operands(G, dims, k, i)
        Gnew = G[(k, i)].copy()
        for j in range(dims[k]):
            _, _, H, b = m.column_system(X, G, dims, k, i, j, rho, operands=ops)
            L = np.linalg.cholesky(H)
            Gnew[:, j] = scipy.linalg.solve_triangular(L, b, lower=True)   # forgot L^T
        return Gnew
    return "update_factor", update_factor


def _mut_ssim_c2_not_squared(m):
    def ssim_band(x, y, peak=1.0, size=11, sigma=1.5):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        g = m.gaussian_window(size, sigma)
        c1, c2 = (0.01 * peak) ** 2, 0.03 * peak
        H, W = x.shape
        vals = []
        for h in range(H - size + 1):
            for w in range(W - size + 1):
                px, py = x[h:h + size, w:w + size], y[h:h + size, w:w + size]
                mx, my = np.sum(g * px), np.sum(g * py)
                vx, vy = np.sum(g * px * px) - mx * mx, np.sum(g * py * py) - my * my
                cxy = np.sum(g * px * py) - mx * my
                vals.append(((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2)))
        return float(np.mean(vals))
    return "ssim_band", ssim_band


def _mut_window_sigma(m):
    def gaussian_window(size=11, sigma=1.5):
        ax = np.arange(size, dtype=np.float64) - (size // 2)
        g = np.exp(-(ax[:, None] ** 2 + ax[None, :] ** 2) / (sigma * sigma))   # lost the factor 2
        return g / g.sum()
    return "gaussian_window", gaussian_window


def _mut_psnr_peak_not_squared(m):
    def psnr_bands(X, ref, peak=1.0):
        X = np.asarray(X, dtype=np.float64)
        ref = np.asarray(ref, dtype=np.float64)
        return np.array([10.0 * np.log10(peak / np.mean((X[:, :, b] - ref[:, :, b]) ** 2))
                         for b in range(X.shape[2])])
    return "psnr_bands", psnr_bands


def _default_factors_variant(m, scale, stat="rms", order=None):
    def default_factors(O, mask, dims, ranks, seed=0):
        N = len(dims)
        vals = np.asarray(O, dtype=np.float64)[np.asarray(mask).astype(bool)]
        mm = float(np.sqrt(np.mean(vals * vals)) if stat == "rms" else np.mean(vals)) if vals.size else 1.0
        prod_r = float(np.prod([ranks[a][b] for a, b in m.edges(N)]))
        s = scale(mm, prod_r, len(m.edges(N)))
        G, n0 = {}, 0
        for k, i in (order(N) if order else m.block_order(N)):
            cnt = int(ranks[k][i]) * int(dims[k])
            u = (m.splitmix64(seed, np.arange(n0, n0 + cnt)) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
            G[(k, i)] = s * u.reshape(int(ranks[k][i]), int(dims[k]))
            n0 += cnt
        return G
    return "default_factors", default_factors


def _mut_default_scale_no_two(m):
    return _default_factors_variant(m, lambda mm, p, e: (mm / p) ** (1.0 / (2 * e)))


def _mut_default_exponent_per_edge(m):
    return _default_factors_variant(m, lambda mm, p, e: 2.0 * (mm / p) ** (1.0 / e))


def _mut_default_mean_not_rms(m):
    return _default_factors_variant(m, lambda mm, p, e: 2.0 * (mm / p) ** (1.0 / (2 * e)), stat="mean")


def _mut_default_i_major_order(m):
    return _default_factors_variant(m, lambda mm, p, e: 2.0 * (mm / p) ** (1.0 / (2 * e)),
                                    order=lambda N: [(k, i) for i in range(N) for k in range(N) if i != k])


MUTATIONS = [
    _mut_reconstruct_drops_edge, _mut_edge_same_side, _mut_subnetwork_includes_k,
    _mut_y_includes_edge_ki, _mut_far_side_from_own, _mut_no_prox_in_b, _mut_no_prox_in_H,
    _mut_D_not_squared, _mut_x_update_swapped, _mut_x_update_denominator,
    _mut_order_descending_i, _mut_jacobi_sweep, _mut_x_updated_before_factors,
    _mut_rel_uses_new_norm, _mut_rse_estimate_norm, _mut_rmse_all_entries,
    _mut_initial_x_keeps_unobserved, _mut_params_counts_edges_once, _mut_cholesky_upper_misuse,
    _mut_ssim_c2_not_squared, _mut_window_sigma, _mut_psnr_peak_not_squared,
    _mut_default_scale_no_two, _mut_default_exponent_per_edge, _mut_default_mean_not_rms,
    _mut_default_i_major_order,
]


@pytest.mark.parametrize("mutation", MUTATIONS, ids=lambda f: f.__name__[5:])
def test_mutation_is_caught(mutation, monkeypatch):
    name, fn = mutation(orc)
    monkeypatch.setattr(orc, name, fn)
    failures = []
    for check in pins.ALL_CHECKS:
        try:
            check(orc)
        except (AssertionError, ValueError, np.linalg.LinAlgError, IndexError) as e:
            failures.append(check.__name__)
            continue
    assert failures, f"mutation {name} slipped through every pin"
