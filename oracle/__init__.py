"""Plain CPU reference ("oracle") for divide-and-conquer multinomial resampling.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only code that may import this package.  The GPU
library never calls it, and the two share no code.

The arithmetic lives in ``dcr_oracle.c`` (plain C, binary64, double-double
sums); this module is a ctypes wrapper around it.  Each wrapper names the part
of the paper (A. A. Popov, "A divide and conquer strategy for multinomial
particle filter resampling") that it follows.  Indices are 0-based.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dcr_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libdcr_oracle.so")
_lib = None

OK = 0
INVALID = 1
BAD_WEIGHTS = 6


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
            "-fno-fast-math", "-fopenmp", "-o", tmp, _SRC, "-lm",
        ])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    i64, u64, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
    P = ctypes.c_void_p
    lib.dcro_philox4x32_10.argtypes = [P, P, P]
    lib.dcro_philox4x32_10.restype = None
    lib.dcro_uniform_open.argtypes = [u64, u64, u64]
    lib.dcro_uniform_open.restype = ctypes.c_double
    lib.dcro_cumulative_weights.argtypes = [P, i64, P, P]
    lib.dcro_cumulative_weights.restype = i32
    lib.dcro_cumulative_weights_f32.argtypes = [P, i64, P, P]
    lib.dcro_cumulative_weights_f32.restype = i32
    lib.dcro_exponential_spacings.argtypes = [i64, u64, u64, i32, P]
    lib.dcro_exponential_spacings.restype = None
    lib.dcro_sorted_uniforms.argtypes = [i64, u64, u64, i32, P, P]
    lib.dcro_sorted_uniforms.restype = None
    lib.dcro_inverse_cmf_one.argtypes = [P, i64, ctypes.c_double]
    lib.dcro_inverse_cmf_one.restype = ctypes.c_int32
    lib.dcro_inverse_cmf_count.argtypes = [P, i64, P, i64, P]
    lib.dcro_inverse_cmf_count.restype = None
    lib.dcro_binary_search.argtypes = [P, i64, i64, ctypes.c_double, P]
    lib.dcro_binary_search.restype = i64
    lib.dcro_binary_sampler.argtypes = [P, i64, P, i64, P, P]
    lib.dcro_binary_sampler.restype = None
    lib.dcro_ccf.argtypes = [P, i64, P, i64, P, P]
    lib.dcro_ccf.restype = None
    lib.dcro_dac.argtypes = [P, i64, P, i64, P, P, P, i64]
    lib.dcro_dac.restype = i64
    lib.dcro_resample.argtypes = [P, i64, i64, u64, u64, P, P, P]
    lib.dcro_resample.restype = i32
    lib.dcro_resample_z.argtypes = [P, i64, i64, u64, u64, i32, P, P, P]
    lib.dcro_resample_z.restype = i32
    lib.dcro_resample_f32.argtypes = [P, i64, i64, u64, u64, i32, P, P, P]
    lib.dcro_resample_f32.restype = i32
    lib.dcro_resample_repeat.argtypes = [P, i64, i64, u64, i64, P]
    lib.dcro_resample_repeat.restype = i32
    lib.dcro_resample_batched.argtypes = [P, i32, P, P, i64, u64, i32, P]
    lib.dcro_resample_batched.restype = i32
    lib.dcro_resample_batched_par.argtypes = [P, i32, P, P, i64, u64, i32, i32, P, P]
    lib.dcro_resample_batched_par.restype = i32
    lib.dcro_scheme_uniforms.argtypes = [i64, u64, u64, i32, P]
    lib.dcro_scheme_uniforms.restype = i32
    lib.dcro_resample_scheme.argtypes = [P, i32, i64, i64, u64, u64, i32, P, P, P]
    lib.dcro_resample_scheme.restype = i32
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


# --------------------------------------------------------------------------
# Randomness: Philox4x32-10 and the open-interval variate (readings R2, R3)
# --------------------------------------------------------------------------
def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block function (Salmon et al., SC'11) on one counter."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().dcro_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform_open(seed: int, stream: int, i: int) -> float:
    """The i-th variate v in (0,1) of (seed, stream): (2k+1) 2^-53."""
    return _load().dcro_uniform_open(seed, stream, i)


# --------------------------------------------------------------------------
# Sec. I, Eq. 3: cumulative weights
# --------------------------------------------------------------------------
def cumulative_weights(w: np.ndarray):
    """Normalised cumulative weights W (binary64) and the total of w.

    binary32 input is promoted exactly.  Raises OracleError on negative, NaN or
    infinite weights or a zero total.
    """
    w = np.ascontiguousarray(w)
    M = w.shape[0]
    W = np.empty(M, dtype=np.float64)
    tot = ctypes.c_double(0.0)
    lib = _load()
    if w.dtype == np.float32:
        st = lib.dcro_cumulative_weights_f32(_ptr(w), M, _ptr(W), ctypes.addressof(tot))
    else:
        w = _f64(w)
        st = lib.dcro_cumulative_weights(_ptr(w), M, _ptr(W), ctypes.addressof(tot))
    if st != OK:
        raise OracleError(f"cumulative_weights: status {st}")
    return W, tot.value


# --------------------------------------------------------------------------
# Sec. II, Alg. 1: sorted uniforms by exponential spacings
# --------------------------------------------------------------------------
def exponential_spacings(N: int, seed: int, stream: int = 0, zkind: int = 0) -> np.ndarray:
    """z_i = -log v_i for i = 0..N (N+1 values).  zkind=1: -logf(fl32(v))."""
    z = np.empty(N + 1, dtype=np.float64)
    _load().dcro_exponential_spacings(N, seed, stream, zkind, _ptr(z))
    return z


def sorted_uniforms(N: int, seed: int, stream: int = 0, zkind: int = 0, with_total=False):
    """u_i = Z_i / Z_N, i = 0..N-1 (reading R1), compensated partial sums."""
    u = np.empty(max(N, 1), dtype=np.float64)
    tot = ctypes.c_double(0.0)
    _load().dcro_sorted_uniforms(N, seed, stream, zkind, _ptr(u), ctypes.addressof(tot))
    u = u[:N]
    return (u, tot.value) if with_total else u


# --------------------------------------------------------------------------
# Inverse CMF (Eq. 3) and the paper's samplers with supplied uniforms
# --------------------------------------------------------------------------
def inverse_cmf_count(W: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Eq. 3 written out: r_i = #{ j < M-1 : W_j < u_i } (O(N M))."""
    W, u = _f64(W), _f64(u)
    r = np.empty(u.shape[0], dtype=np.int32)
    _load().dcro_inverse_cmf_count(_ptr(W), W.shape[0], _ptr(u), u.shape[0], _ptr(r))
    return r


def inverse_cmf_one(W: np.ndarray, u: float) -> int:
    W = _f64(W)
    return int(_load().dcro_inverse_cmf_one(_ptr(W), W.shape[0], float(u)))


def binary_search(Z: np.ndarray, a: int, b: int, X: float):
    """Alg. 2 on Z[a..b] (inclusive); returns (index, comparisons)."""
    Z = _f64(Z)
    n = ctypes.c_int64(0)
    m = _load().dcro_binary_search(_ptr(Z), a, b, float(X), ctypes.addressof(n))
    return int(m), n.value


def binary_sampler(W: np.ndarray, u: np.ndarray):
    """Alg. 3 with the uniforms supplied; returns (r, comparisons)."""
    W, u = _f64(W), _f64(u)
    r = np.empty(u.shape[0], dtype=np.int32)
    n = ctypes.c_int64(0)
    _load().dcro_binary_sampler(_ptr(W), W.shape[0], _ptr(u), u.shape[0], _ptr(r),
                                ctypes.addressof(n))
    return r, n.value


def ccf(W: np.ndarray, u: np.ndarray):
    """Alg. 4 (CCF linear merge) with sorted uniforms supplied."""
    W, u = _f64(W), _f64(u)
    r = np.empty(u.shape[0], dtype=np.int32)
    n = ctypes.c_int64(0)
    _load().dcro_ccf(_ptr(W), W.shape[0], _ptr(u), u.shape[0], _ptr(r), ctypes.addressof(n))
    return r, n.value


def dac(W: np.ndarray, u: np.ndarray, trace: bool = False):
    """Alg. 5 (divide and conquer) with sorted uniforms supplied.

    Returns (r, comparisons) or, with trace=True, (r, comparisons, trace) where
    trace rows are (recursion depth, uniform index, weight index).
    """
    W, u = _f64(W), _f64(u)
    N = u.shape[0]
    r = np.empty(N, dtype=np.int32)
    n = ctypes.c_int64(0)
    cap = max(N, 1) if trace else 0
    tr = np.zeros((max(cap, 1), 3), dtype=np.int64)
    ln = _load().dcro_dac(_ptr(W), W.shape[0], _ptr(u), N, _ptr(r), ctypes.addressof(n),
                          _ptr(tr) if trace else None, cap)
    if trace:
        return r, n.value, tr[:ln].copy()
    return r, n.value


# --------------------------------------------------------------------------
# End to end
# --------------------------------------------------------------------------
def resample(w: np.ndarray, N: int, seed: int, stream: int = 0, zkind: int | None = None):
    """DaC sampler end to end: returns (r, W, u).

    binary32 weights are promoted exactly; zkind selects the spacings form
    (default: 0 for binary64 weights, 1 for binary32 weights; binary64 weights
    may take zkind 1, the form the binary32 outer-product path uses).
    """
    w = np.ascontiguousarray(w)
    M = w.shape[0]
    r = np.empty(max(N, 1), dtype=np.int32)
    W = np.empty(M, dtype=np.float64)
    u = np.empty(max(N, 1), dtype=np.float64)
    lib = _load()
    if w.dtype == np.float32:
        zk = 1 if zkind is None else zkind
        st = lib.dcro_resample_f32(_ptr(w), M, N, seed, stream, zk, _ptr(r), _ptr(W), _ptr(u))
    else:
        w = _f64(w)
        st = lib.dcro_resample_z(_ptr(w), M, N, seed, stream, 0 if zkind is None else zkind,
                                 _ptr(r), _ptr(W), _ptr(u))
    if st != OK:
        raise OracleError(f"resample: status {st}")
    return r[:N], W, u[:N]


# --------------------------------------------------------------------------
# Other schemes through the same map (Sec. V): stratified and systematic
# --------------------------------------------------------------------------
SCHEMES = {"multinomial": 0, "stratified": 1, "systematic": 2}


def scheme_uniforms(N: int, seed: int, stream: int = 0, scheme: str = "stratified") -> np.ndarray:
    """Sorted uniforms of a scheme: stratified (i + v_i)/N, systematic (i + v_0)/N."""
    u = np.empty(max(N, 1), dtype=np.float64)
    st = _load().dcro_scheme_uniforms(N, seed, stream, SCHEMES[scheme], _ptr(u))
    if st != OK:
        raise OracleError(f"scheme_uniforms: status {st}")
    return u[:N]


def resample_scheme(w: np.ndarray, N: int, seed: int, stream: int = 0,
                    scheme: str = "stratified"):
    """End to end with a scheme's uniforms: returns (r, W, u)."""
    w = np.ascontiguousarray(w)
    is_f32 = 1 if w.dtype == np.float32 else 0
    if not is_f32:
        w = _f64(w)
    M = w.shape[0]
    r = np.empty(max(N, 1), dtype=np.int32)
    W = np.empty(M, dtype=np.float64)
    u = np.empty(max(N, 1), dtype=np.float64)
    st = _load().dcro_resample_scheme(_ptr(w), is_f32, M, N, seed, stream, SCHEMES[scheme],
                                      _ptr(r), _ptr(W), _ptr(u))
    if st != OK:
        raise OracleError(f"resample_scheme: status {st}")
    return r[:N], W, u[:N]


def resample_repeat(w: np.ndarray, N: int, seed0: int, R: int) -> np.ndarray:
    """R independent binary64 resamples (seeds seed0..seed0+R-1): [R, N]."""
    w = _f64(w)
    r = np.empty((R, max(N, 1)), dtype=np.int32)
    st = _load().dcro_resample_repeat(_ptr(w), w.shape[0], N, seed0, R, _ptr(r))
    if st != OK:
        raise OracleError(f"resample_repeat: status {st}")
    return r[:, :N]


def resample_batched_parallel(w: np.ndarray, w_off: np.ndarray, n_off: np.ndarray, seed: int,
                              threads: int, zkind: int | None = None):
    """resample_batched with the filters spread over OpenMP threads (the same
    per-filter arithmetic); returns (r, threads used)."""
    import ctypes
    w = np.ascontiguousarray(w)
    w_off = np.ascontiguousarray(w_off, dtype=np.int64)
    n_off = np.ascontiguousarray(n_off, dtype=np.int64)
    B = w_off.shape[0] - 1
    is_f32 = 1 if w.dtype == np.float32 else 0
    if not is_f32:
        w = _f64(w)
    zk = (1 if is_f32 else 0) if zkind is None else zkind
    r = np.empty(max(int(n_off[-1]), 1), dtype=np.int32)
    used = ctypes.c_int(0)
    st = _load().dcro_resample_batched_par(_ptr(w), is_f32, _ptr(w_off), _ptr(n_off), B, seed, zk,
                                           int(threads), _ptr(r), ctypes.addressof(used))
    if st != OK:
        raise OracleError(f"resample_batched_parallel: status {st}")
    return r[: int(n_off[-1])], int(used.value)


def resample_batched(w: np.ndarray, w_off: np.ndarray, n_off: np.ndarray, seed: int,
                     zkind: int | None = None) -> np.ndarray:
    """Filter b resamples its own segment with stream id b; local indices."""
    w = np.ascontiguousarray(w)
    w_off = np.ascontiguousarray(w_off, dtype=np.int64)
    n_off = np.ascontiguousarray(n_off, dtype=np.int64)
    B = w_off.shape[0] - 1
    is_f32 = 1 if w.dtype == np.float32 else 0
    if not is_f32:
        w = _f64(w)
    zk = (1 if is_f32 else 0) if zkind is None else zkind
    r = np.empty(max(int(n_off[-1]), 1), dtype=np.int32)
    st = _load().dcro_resample_batched(_ptr(w), is_f32, _ptr(w_off), _ptr(n_off), B, seed, zk,
                                       _ptr(r))
    if st != OK:
        raise OracleError(f"resample_batched: status {st}")
    return r[: int(n_off[-1])]
