"""Pins of the oracle's inverse-CMF map (Sec. I Eq. 3; Sec. II Alg. 2-4; Sec. III Alg. 5).

Nothing here re-types the oracle's formula: the map is checked against the
worked example of Fig. 1, brute force over tiny inputs, numpy's textbook
lower-bound search, and the comparison counts of Table I.
"""
import json
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig1_worked_example.json")


def _fig1():
    with open(GOLDEN) as f:
        return json.load(f)


def test_fig1_indices(oracle_mod):
    g = _fig1()
    W = np.array(g["W"])
    U = np.array(g["U"])
    # the stored values are the figure coordinates mapped to [0, 1]
    assert np.allclose(W, (np.array(g["W_x"]) + 4) / 8)
    assert np.allclose(U, (np.array(g["U_x"]) + 4) / 8)
    expect = np.array(g["r_paper_1based"]) - 1
    r, _ = oracle_mod.dac(W, U)
    assert r.tolist() == expect.tolist()
    assert oracle_mod.inverse_cmf_count(W, U).tolist() == expect.tolist()
    assert oracle_mod.ccf(W, U)[0].tolist() == expect.tolist()
    assert oracle_mod.binary_sampler(W, U)[0].tolist() == expect.tolist()


def test_fig1_recursion_trace(oracle_mod):
    """Alg. 5 must locate U3 first, then U1 and U4, then U2 and U5 (Fig. 1 steps 1-3)."""
    g = _fig1()
    _, _, tr = oracle_mod.dac(np.array(g["W"]), np.array(g["U"]), trace=True)
    steps = {}
    for depth, iu, jw in tr.tolist():
        steps.setdefault(str(depth + 1), []).append([f"U{iu + 1}", f"W{jw + 1}"])
    assert steps == g["steps_1based"]


def _random_cmf(rng, M, allow_zero=True):
    w = rng.integers(0, 4, size=M).astype(np.float64) if allow_zero else rng.random(M) + 0.1
    if w.sum() == 0:
        w[-1] = 1.0
    W = np.cumsum(w) / w.sum()   # small integers: exact sums, ties between bins possible
    return W


def test_bruteforce_tiny(oracle_mod):
    """Every sampler of the paper equals the count definition and numpy's lower bound."""
    rng = np.random.default_rng(7)
    for trial in range(3000):
        M = int(rng.integers(1, 9))
        N = int(rng.integers(1, 9))
        W = _random_cmf(rng, M)
        # uniforms: mix of exact bin edges, neighbours of edges and random values
        pool = np.concatenate([W, np.nextafter(W, 2), np.nextafter(W, -1), rng.random(4),
                               [1.0, np.nextafter(0, 1)]])
        pool = pool[(pool > 0) & (pool <= 1)]
        u = np.sort(rng.choice(pool, size=N))
        expect = np.searchsorted(W[:-1], u, side="left")       # textbook lower bound
        brute = np.array([sum(1 for j in range(M - 1) if W[j] < x) for x in u])
        assert expect.tolist() == brute.tolist()
        assert oracle_mod.inverse_cmf_count(W, u).tolist() == brute.tolist()
        assert oracle_mod.dac(W, u)[0].tolist() == brute.tolist(), (W, u)
        assert oracle_mod.ccf(W, u)[0].tolist() == brute.tolist()
        assert oracle_mod.binary_sampler(W, u)[0].tolist() == brute.tolist()


def test_edges_and_clamp(oracle_mod):
    W = np.array([0.25, 0.25, 0.5, 0.75, 0.75, 1.0])  # bins 1 and 4 have zero weight
    u = np.array([0.25, np.nextafter(0.25, 1), 0.5, 0.75, np.nextafter(0.75, 1), 1.0])
    r, _ = oracle_mod.dac(W, u)
    # u on an edge belongs to the bin that ends there; zero-width bins are never chosen
    assert r.tolist() == [0, 2, 2, 3, 5, 5]
    # uniforms above the last cumulative weight are clamped to the last bin
    W2 = np.array([0.1, 0.2, 0.9])
    u2 = np.array([0.95, 0.99])
    assert oracle_mod.dac(W2, u2)[0].tolist() == [2, 2]
    assert oracle_mod.ccf(W2, u2)[0].tolist() == [2, 2]
    assert oracle_mod.inverse_cmf_count(W2, u2).tolist() == [2, 2]


def test_binary_search_alg2(oracle_mod):
    Z = np.array([0.1, 0.2, 0.2, 0.4, 0.8])
    # first index in [a, b] with Z >= X, else b
    assert oracle_mod.binary_search(Z, 0, 4, 0.2)[0] == 1
    assert oracle_mod.binary_search(Z, 0, 4, 0.25)[0] == 3
    assert oracle_mod.binary_search(Z, 0, 4, 0.9)[0] == 4
    assert oracle_mod.binary_search(Z, 2, 3, 0.05)[0] == 2
    assert oracle_mod.binary_search(Z, 3, 3, 0.05)[0] == 3


@pytest.mark.parametrize("ratio", [1, 10, 100, 1000])
def test_table1_comparison_counts(oracle_mod, ratio):
    """Table I: CCF ~ M + N, Binary ~ N log2 M, DaC ~ N log2(M/N + 1)."""
    rng = np.random.default_rng(ratio)
    N = 2000
    M = N * ratio
    w = rng.random(M)
    W = np.cumsum(w) / w.sum()
    u = np.sort(rng.random(N))
    r_dac, c_dac = oracle_mod.dac(W, u)
    r_ccf, c_ccf = oracle_mod.ccf(W, u)
    r_bin, c_bin = oracle_mod.binary_sampler(W, u)
    assert r_dac.tolist() == r_ccf.tolist() == r_bin.tolist()
    assert c_ccf <= M + N
    assert c_ccf >= 0.5 * M
    assert abs(c_bin - N * math.log2(M)) <= N * 1.5
    # DaC does a bounded number of comparisons per sample times log2(M/N + 1)
    assert c_dac <= 3.0 * N * math.log2(M / N + 1) + 2 * N
    if ratio >= 100:
        assert c_dac < c_ccf and c_dac < c_bin


def test_batched_parallel_equals_sequential(oracle_mod):
    """The OpenMP loop over filters (the batched CPU baseline) changes no
    filter's arithmetic: its result equals the sequential loop's."""
    rng = np.random.Generator(np.random.PCG64(44))
    Mb = rng.integers(1, 6000, 40)
    Nb = rng.integers(0, 400, 40)
    w_off = np.concatenate([[0], np.cumsum(Mb)]).astype(np.int64)
    n_off = np.concatenate([[0], np.cumsum(Nb)]).astype(np.int64)
    for dtype in (np.float64, np.float32):
        w = np.exp(rng.normal(0.0, 3.0, int(w_off[-1]))).astype(dtype)
        seq = oracle_mod.resample_batched(w, w_off, n_off, 9)
        par, used = oracle_mod.resample_batched_parallel(w, w_off, n_off, 9, 3)
        assert used >= 1
        assert np.array_equal(seq, par)
