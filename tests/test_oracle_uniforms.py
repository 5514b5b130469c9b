"""Pins of the oracle's sorted uniforms (Sec. II, Alg. 1) and of its random source.

- Philox4x32-10 is compared with rocRAND's separately written implementation
  (a host-callable header shipped with ROCm), compiled here into a probe.
- The variates v are checked for their lattice and range, and for uniformity.
- The spacings z = -log v are checked against the exponential law.
- u is checked in exact rational arithmetic from the oracle's own z (this pins
  the prefix sums and the normaliser Z_N of Alg. 1), and against the laws of
  uniform order statistics: U_(i) ~ Beta(i, N+1-i), Z_N ~ Gamma(N+1, 1).
"""
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))

PROBE_SRC = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
// rocRAND's public engine: key = seed, counter words 2-3 = subsequence,
// counter words 0-1 = offset / 4; next() returns the block's four words.
int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        unsigned a = e(), b = e(), c = e(), d = e();
        std::printf("%08x %08x %08x %08x\n", a, b, c, d);
    }
    return 0;
}
"""


@pytest.mark.slow
def test_philox_matches_rocrand(oracle_mod, tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    src = tmp_path / "probe.cpp"
    src.write_text(PROBE_SRC)
    exe = tmp_path / "probe"
    subprocess.check_call([hipcc, "-O1", "-I/opt/rocm/include", "-o", str(exe), str(src)],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    rng = np.random.default_rng(5)
    # counter word 1 stays below 2^30 so that 4 * (offset) fits in 64 bits
    cases = [[0] * 6, [0xFFFFFFFF, 0x3FFFFFFF] + [0xFFFFFFFF] * 4, [1, 0, 0, 0, 0, 0],
             [0, 0, 0, 0, 1, 0]]
    rnd = rng.integers(0, 2**32, size=(60, 6), dtype=np.uint64)
    rnd[:, 1] %= 2**30
    cases += rnd.tolist()
    inp = "\n".join(" ".join(f"{x:x}" for x in c) for c in cases) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout
    got = [[int(t, 16) for t in line.split()] for line in out.strip().splitlines()]
    assert len(got) == len(cases)
    for c, g in zip(cases, got):
        mine = oracle_mod.philox4x32_10(c[:4], c[4:]).tolist()
        assert mine == g, (c, mine, g)


def test_variate_lattice_and_range(oracle_mod):
    vs = np.array([oracle_mod.uniform_open(123, 7, i) for i in range(4000)])
    assert vs.min() >= 2.0**-53 and vs.max() <= 1 - 2.0**-53
    k = vs * 2.0**53
    assert np.all(k == np.floor(k)) and np.all(k % 2 == 1)   # odd multiples of 2^-53
    assert stats.kstest(vs, "uniform").pvalue > 1e-4
    # even and odd draws of one counter are different words
    assert len(np.unique(vs)) == len(vs)


def test_variate_streams_differ(oracle_mod):
    a = [oracle_mod.uniform_open(1, 0, i) for i in range(64)]
    b = [oracle_mod.uniform_open(1, 1, i) for i in range(64)]
    c = [oracle_mod.uniform_open(2, 0, i) for i in range(64)]
    assert a != b and a != c
    assert stats.ks_2samp(a + b, c).pvalue > 1e-4


def test_spacings_are_exponential(oracle_mod):
    z = oracle_mod.exponential_spacings(200000, 99, 0)
    assert np.all(z > 0) and np.all(np.isfinite(z))
    assert stats.kstest(z, "expon").pvalue > 1e-4
    assert abs(z.mean() - 1.0) < 5 / np.sqrt(len(z))
    z32 = oracle_mod.exponential_spacings(200000, 99, 0, zkind=1)
    # binary32 form: v rounded to binary32 (absolute z error <= 2^-24) and a
    # binary32 logarithm (relative error ~2^-24)
    assert np.all(np.abs(z32 - z) <= 2.0**-23 * (1.0 + z))


@pytest.mark.parametrize("N", [1, 2, 17, 1000])
def test_u_exact_from_spacings(oracle_mod, N):
    """u_i = Z_i / Z_N with Z the exact prefix sums of the same z (reading R1)."""
    z = oracle_mod.exponential_spacings(N, 31, 3)
    u = oracle_mod.sorted_uniforms(N, 31, 3)
    fr = [Fraction(float(x)) for x in z]
    T = sum(fr, Fraction(0))
    S = Fraction(0)
    ref = []
    for i in range(N):
        S += fr[i]
        ref.append(float(S / T))
    d = np.abs(u.view(np.int64) - np.array(ref).view(np.int64))
    assert d.max() <= 1
    assert np.all(np.diff(u) >= 0) and u[0] > 0 and u[-1] <= 1


def test_u_order_statistics(oracle_mod):
    """U_(i) ~ Beta(i, N+1-i) (1-based i) and Z_N ~ Gamma(N+1, 1) over many seeds."""
    N, R = 9, 3000
    U = np.empty((R, N))
    T = np.empty(R)
    for s in range(R):
        U[s], T[s] = oracle_mod.sorted_uniforms(N, 1000 + s, 0, with_total=True)
    for i in range(1, N + 1):
        p = stats.kstest(U[:, i - 1], stats.beta(i, N + 1 - i).cdf).pvalue
        assert p > 1e-4, (i, p)
        assert abs(U[:, i - 1].mean() - i / (N + 1)) < 5 * np.sqrt(
            i * (N + 1 - i) / ((N + 1) ** 2 * (N + 2)) / R)
    assert stats.kstest(T, stats.gamma(N + 1).cdf).pvalue > 1e-4


def test_u_sorted_large(oracle_mod):
    u = oracle_mod.sorted_uniforms(1 << 18, 5, 0)
    assert np.all(np.diff(u) >= 0) and u[0] > 0 and u[-1] <= 1
    # empirical CDF of a single large sorted sample is uniform
    assert stats.kstest(u, "uniform").pvalue > 1e-4
