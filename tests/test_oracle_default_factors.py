"""Pins of the oracle's seeded default G^0 (Algorithm 1 takes G^0 as an input
and leaves its distribution open): the SplitMix64 stream against the
generator's published outputs, the counter form against the stepping form,
the scale against the expectation E[iFCTN(G^0)] = m that defines it, and the
block order of the factors."""
import numpy as np

import oracle


def ranks_of(N, upper, default=3):
    r = np.full((N, N), default, dtype=np.int64)
    np.fill_diagonal(r, 0)
    for (a, b), v in upper.items():
        r[a, b] = r[b, a] = v
    return r


def test_splitmix64_published_outputs():
    # the first outputs of SplitMix64 from state 0 (Steele, Lea and Flood 2014;
    # the values its reference implementation prints)
    got = [int(v) for v in oracle.splitmix64(0, [0, 1, 2])]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_splitmix64_counter_form_equals_stepping():
    """Output n taken directly equals the (n+1)-th output of the generator
    stepped one state at a time (Python integers, mod 2^64)."""
    M = (1 << 64) - 1
    seed = 0xDEADBEEF12345678
    state, seq = seed, []
    for _ in range(64):
        state = (state + 0x9E3779B97F4A7C15) & M
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        seq.append(z ^ (z >> 31))
    got = [int(v) for v in oracle.splitmix64(seed, np.arange(64))]
    assert got == seq


def test_default_factors_layout_and_range():
    dims = (5, 4, 3, 6)
    R = ranks_of(4, {(0, 1): 2, (2, 3): 4})
    rng = np.random.default_rng(0)
    O, mask = rng.random(dims), rng.random(dims) < 0.5
    G = oracle.default_factors(O, mask, dims, R, seed=7)
    assert list(G) == oracle.block_order(4)
    for (k, i), v in G.items():
        assert v.shape == (R[k][i], dims[k])
    flat = np.concatenate([G[key].ravel() for key in oracle.block_order(4)])
    assert flat.size == oracle.num_parameters(dims, R)
    m = np.sqrt(np.mean(O[mask] ** 2))
    s = 2.0 * (m / np.prod([R[a][b] for a, b in oracle.edges(4)])) ** (1.0 / 12.0)
    assert flat.min() >= 0.0 and flat.max() < s
    # entry n is s * (output n >> 11) / 2^53: the first and the last entry
    assert flat[0] == s * float(int(oracle.splitmix64(7, 0)) >> 11) * 2.0 ** -53
    n = flat.size - 1
    assert flat[n] == s * float(int(oracle.splitmix64(7, n)) >> 11) * 2.0 ** -53
    # another seed gives other factors; the same seed the same factors
    G2 = oracle.default_factors(O, mask, dims, R, seed=7)
    G3 = oracle.default_factors(O, mask, dims, R, seed=8)
    assert all(np.array_equal(G[key], G2[key]) for key in G)
    assert not np.array_equal(G[(0, 1)], G3[(0, 1)])


def test_default_factors_reconstruct_to_the_data_scale():
    """E[iFCTN(G^0)] = m (the root mean square of the observed entries) for
    every entry: averaged over 2000 seeds, the mean of the reconstruction
    is m within a few standard errors, at orders 3-5 and unequal ranks."""
    rng = np.random.default_rng(1)
    cases = [((6, 5, 4), ranks_of(3, {(0, 1): 2, (0, 2): 3, (1, 2): 4}), 0.06),
             ((4, 3, 4, 3), ranks_of(4, {(0, 3): 2, (1, 2): 5}), 0.08),
             ((3, 3, 2, 3, 2), ranks_of(5, {(0, 4): 2}, default=2), 0.15)]
    for dims, R, tol in cases:
        O = 5.0 * rng.random(dims)
        mask = rng.random(dims) < 0.3
        m = np.sqrt(np.mean(O[mask] ** 2))
        means = [np.mean(oracle.reconstruct(oracle.default_factors(O, mask, dims, R, seed), dims))
                 for seed in range(2000)]
        assert abs(np.mean(means) / m - 1.0) < tol, (dims, np.mean(means) / m)


def test_default_factors_without_observed_data():
    """No observed entry (or only zeros): the scale of m = 1."""
    dims = (4, 3, 5)
    R = ranks_of(3, {})
    O = np.zeros(dims)
    for mask in (np.zeros(dims, dtype=bool), np.ones(dims, dtype=bool)):
        G = oracle.default_factors(O, mask, dims, R, seed=3)
        G1 = oracle.default_factors(np.ones(dims), np.ones(dims, dtype=bool), dims, R, seed=3)
        assert all(np.array_equal(G[key], G1[key]) for key in G)
