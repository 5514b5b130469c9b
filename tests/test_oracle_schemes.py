"""Pins of the oracle's stratified and systematic schemes (the sorted uniforms
of Sec. V's generalisation, through the same inverse-CMF map).

Each test checks a property that the scheme's definition fixes independently
of how the oracle writes it: strata membership in exact rational arithmetic,
the uniform law of the within-stratum offsets, the count bounds that hold for
every weight vector (|c_j - N w_j| < 1 for systematic, < 2 for stratified),
unbiasedness of the counts and the variance reduction against multinomial.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle


@pytest.mark.parametrize("scheme", ["stratified", "systematic"])
def test_strata_membership_exact(scheme):
    for N in [1, 2, 7, 1000, 4097]:
        u = oracle.scheme_uniforms(N, seed=11, stream=3, scheme=scheme)
        assert len(u) == N
        assert np.all(np.diff(u) >= 0) and u[0] > 0 and u[-1] <= 1
        for i in range(0, N, max(1, N // 257)):
            q = Fraction(float(u[i])) * N           # exact
            assert i <= q <= i + 1, (N, i, float(q))


def test_stratified_offsets_are_uniform_and_independent():
    N = 50000
    u = oracle.scheme_uniforms(N, seed=5, stream=0, scheme="stratified")
    off = u * N - np.arange(N)
    assert stats.kstest(off, "uniform").pvalue > 1e-3
    rho = np.corrcoef(off[:-1], off[1:])[0, 1]
    assert abs(rho) < 5 / np.sqrt(N)


def test_systematic_offset_shared_and_uniform_across_seeds():
    N = 3000
    u = oracle.scheme_uniforms(N, seed=8, stream=2, scheme="systematic")
    off = u * N - np.arange(N)
    assert np.ptp(off) < 1e-9
    offs = [oracle.scheme_uniforms(16, seed=s, stream=0, scheme="systematic")[0] * 16
            for s in range(2000)]
    assert stats.kstest(offs, "uniform").pvalue > 1e-3


def test_multinomial_scheme_is_alg1():
    w = np.random.Generator(np.random.PCG64(4)).random(500)
    r0, W0, u0 = oracle.resample(w, 300, seed=2, stream=1)
    r1, W1, u1 = oracle.resample_scheme(w, 300, seed=2, stream=1, scheme="multinomial")
    assert np.array_equal(r0, r1) and np.array_equal(u0, u1)


def _counts(r, M):
    return np.bincount(r, minlength=M)


@pytest.mark.parametrize("scheme,bound", [("systematic", 1.0), ("stratified", 2.0)])
def test_count_bounds_every_weight_vector(scheme, bound):
    rng = np.random.Generator(np.random.PCG64(21))
    for trial in range(20):
        M = int(rng.integers(1, 400))
        N = int(rng.integers(1, 600))
        w = np.exp(rng.normal(0, 2.5, M))
        if trial % 4 == 0:
            w[rng.random(M) < 0.3] = 0.0
            w[0] += 1.0
        r, W, u = oracle.resample_scheme(w, N, seed=trial, stream=0, scheme=scheme)
        # the map itself: the count definition on the same W and u
        assert np.array_equal(r, oracle.inverse_cmf_count(W, u))
        dW = np.diff(np.concatenate([[0.0], W]))
        c = _counts(r, M)
        assert np.all(np.abs(c - N * dW) < bound + 1e-6), (trial, np.max(np.abs(c - N * dW)))
        assert np.all(c[dW == 0] == 0)


@pytest.mark.parametrize("scheme", ["systematic", "stratified"])
def test_counts_unbiased_and_less_variable_than_multinomial(scheme):
    rng = np.random.Generator(np.random.PCG64(33))
    M, N, R = 40, 100, 600
    w = rng.dirichlet(np.full(M, 0.7))
    C = np.array([_counts(oracle.resample_scheme(w, N, seed=s, stream=0, scheme=scheme)[0], M)
                  for s in range(R)])
    Cm = np.array([_counts(oracle.resample(w, N, seed=s, stream=0)[0], M) for s in range(R)])
    mean = C.mean(0)
    # multinomial variance bounds these schemes' per-bin variance
    se = np.sqrt(N * w * (1 - w) / R) + 1e-12
    assert np.all(np.abs(mean - N * w) < 5 * se + 1e-9)
    assert C.var(0).sum() < 0.8 * Cm.var(0).sum()
