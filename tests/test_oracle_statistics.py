"""End-to-end pins of the oracle sampler by the laws of multinomial sampling.

Eq. 2 of the paper draws N indices whose counts are Multinomial(N, w); these
tests check the counts' chi-square fit, their means and variances over many
seeds, and the exact probability of every count vector for M = 3, N = 2.
"""
import math
from itertools import product

import numpy as np
from scipy import stats


def test_counts_chi_square(oracle_mod):
    rng = np.random.default_rng(3)
    M, N = 40, 200000
    w = np.exp(rng.normal(0, 1, M))
    p = w / w.sum()
    r, W, u = oracle_mod.resample(w, N, seed=17)
    assert np.all(np.diff(r) >= 0)          # sorted uniforms give sorted indices
    c = np.bincount(r, minlength=M)
    assert stats.chisquare(c, N * p).pvalue > 1e-4


def test_counts_mean_variance(oracle_mod):
    w = np.array([0.05, 0.15, 0.3, 0.5])
    p = w / w.sum()
    M, N, R = 4, 30, 4000
    rr = oracle_mod.resample_repeat(w, N, 100, R)
    C = np.stack([np.bincount(x, minlength=M) for x in rr])
    mean = C.mean(0)
    var = C.var(0, ddof=1)
    ev = N * p * (1 - p)
    assert np.all(np.abs(mean - N * p) < 5 * np.sqrt(ev / R))
    # sample variance of R draws: relative s.e. about sqrt(2/(R-1))
    assert np.all(np.abs(var / ev - 1) < 6 * np.sqrt(2 / (R - 1)))
    # multinomial covariance: counts sum to N
    assert np.all(C.sum(1) == N)


def test_exact_pmf_m3_n2(oracle_mod):
    w = np.array([0.2, 0.3, 0.5])
    R = 60000
    rr = oracle_mod.resample_repeat(w, 2, 5000, R)
    keys = {}
    for row in rr:
        c = tuple(np.bincount(row, minlength=3))
        keys[c] = keys.get(c, 0) + 1
    cells = [c for c in product(range(3), repeat=3) if sum(c) == 2]
    pmf = {c: math.factorial(2) / np.prod([math.factorial(k) for k in c])
           * np.prod([w[j] ** c[j] for j in range(3)]) for c in cells}
    obs = np.array([keys.get(c, 0) for c in cells])
    exp = np.array([R * pmf[c] for c in cells])
    assert abs(exp.sum() - R) < 1e-6
    assert stats.chisquare(obs, exp).pvalue > 1e-4


def test_zero_weight_bins_never_drawn(oracle_mod):
    w = np.array([0.0, 1.0, 0.0, 0.0, 2.0, 0.0])
    r, W, u = oracle_mod.resample(w, 5000, seed=4)
    assert set(np.unique(r).tolist()) <= {1, 4}


def test_binary32_weights_promoted(oracle_mod):
    rng = np.random.default_rng(8)
    w32 = np.exp(rng.normal(0, 2, 5000)).astype(np.float32)
    r32, W32, _ = oracle_mod.resample(w32, 1000, seed=9, zkind=0)
    r64, W64, _ = oracle_mod.resample(w32.astype(np.float64), 1000, seed=9)
    assert np.array_equal(W32, W64) and np.array_equal(r32, r64)


def test_batched_equals_single(oracle_mod):
    rng = np.random.default_rng(10)
    Ms = [1, 7, 300, 50]
    Ns = [3, 1, 40, 0]
    w = np.exp(rng.normal(0, 1, sum(Ms)))
    w_off = np.concatenate([[0], np.cumsum(Ms)])
    n_off = np.concatenate([[0], np.cumsum(Ns)])
    r = oracle_mod.resample_batched(w, w_off, n_off, seed=21)
    for b in range(len(Ms)):
        rb, _, _ = oracle_mod.resample(w[w_off[b]:w_off[b + 1]], Ns[b], seed=21, stream=b)
        assert r[n_off[b]:n_off[b + 1]].tolist() == rb.tolist()


def test_binary64_weights_with_binary32_spacings(oracle_mod):
    """resample with zkind 1 on binary64 weights is the composition of the
    pinned stages: W of the weights, the binary32-form uniforms, the count
    definition of the map."""
    rng = np.random.Generator(np.random.PCG64(404))
    w = np.outer(rng.random(30), rng.random(17)).ravel()
    r, W, u = oracle_mod.resample(w, 400, seed=6, stream=2, zkind=1)
    W0, _ = oracle_mod.cumulative_weights(w)
    assert np.array_equal(W, W0)
    assert np.array_equal(u, oracle_mod.sorted_uniforms(400, 6, 2, zkind=1))
    assert np.array_equal(r, oracle_mod.inverse_cmf_count(W, u))
