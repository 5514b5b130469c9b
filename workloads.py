"""Seeded synthetic inputs shaped like the paper's resampling workloads.

This module only draws input data (weights, batch layouts).  It holds none of
the resampling arithmetic, so both the GPU library's tests/benchmark and the
CPU oracle may use it.

The paper times its samplers on posterior weights of an ensemble Gaussian
mixture filter with M = N * N_Y weights (Sec. IV); those weights, its code and
its data are not available, so the distributions below stand in for them.
Every generator uses numpy's PCG64 with a fixed seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    M: int
    N: int
    w64: np.ndarray
    seed: int = 0                 # Philox key for the uniforms
    stream: int = 0               # Philox stream id
    description: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def w32(self) -> np.ndarray:
        """binary32 copy of the weights (round to nearest)."""
        return self.w64.astype(np.float32)


def single_lognormal(M: int = 65536, N: int = 4096, sigma: float = 2.0, data_seed: int = 1001,
                     normalise: bool = True) -> Workload:
    """w_j = exp(g_j), g_j ~ N(0, sigma^2) iid (optionally normalised)."""
    rng = np.random.Generator(np.random.PCG64(data_seed))
    w = np.exp(rng.normal(0.0, sigma, size=M))
    if normalise:
        w = w / w.sum()
    return Workload(f"lognormal_M{M}_N{N}", M, N, w,
                    description=f"w=exp(N(0,{sigma}^2)) M={M} N={N}")


def small_single(M: int = 65536, N: int = 4096) -> Workload:
    """Single distribution: M = 65536 binary64 weights exp(N(0, 2^2)), normalised; N = 4096."""
    wl = single_lognormal(M, N, 2.0, 1001, True)
    wl.name = "single_M65536_N4096"
    return wl


def engmf_step(N: int = 2000, P: int = 64, data_seed: int = 1002) -> Workload:
    """EnGMF-shaped step: M = N*P weights a_i * b_k, a ~ LogNormal(0,1), b ~ Dirichlet(0.5).

    Weight i*P + k belongs to particle i and likelihood component k (particle-major).
    """
    rng = np.random.Generator(np.random.PCG64(data_seed))
    a = rng.lognormal(0.0, 1.0, size=N)
    b = rng.dirichlet(np.full(P, 0.5))
    w = (a[:, None] * b[None, :]).reshape(-1)
    return Workload(f"engmf_N{N}_P{P}", N * P, N, w,
                    description=f"EnGMF-shaped M={N * P} (N={N} x P={P}), draw N={N}",
                    extra={"a": a, "b": b})


def sparse_mass(M: int = 1 << 26, N: int = 1 << 14, sigma: float = 5.0,
                data_seed: int = 1003) -> Workload:
    """Large sparse-mass instance: log-weights ~ N(0, 5^2), M = 2^26, N = 2^14."""
    rng = np.random.Generator(np.random.PCG64(data_seed))
    w = np.exp(rng.normal(0.0, sigma, size=M))
    return Workload(f"sparse_M{M}_N{N}", M, N, w,
                    description=f"sparse mass: w=exp(N(0,{sigma}^2)) M={M} N={N}")


def equal_size(M: int = 1 << 24, data_seed: int = 1004) -> Workload:
    """Classic equal-size case M = N = 2^24, log-weights ~ N(0, 1)."""
    rng = np.random.Generator(np.random.PCG64(data_seed))
    w = np.exp(rng.normal(0.0, 1.0, size=M))
    return Workload(f"equal_M{M}_N{M}", M, M, w, description=f"equal size M=N={M}")


@dataclass
class BatchedWorkload:
    name: str
    B: int
    w64: np.ndarray
    w_off: np.ndarray   # int64 [B+1]
    n_off: np.ndarray   # int64 [B+1]
    seed: int = 0
    description: str = ""

    @property
    def w32(self) -> np.ndarray:
        return self.w64.astype(np.float32)

    @property
    def M(self) -> np.ndarray:
        return np.diff(self.w_off)

    @property
    def N(self) -> np.ndarray:
        return np.diff(self.n_off)


def batched(B: int = 4096, m_lo: float = 1e3, m_hi: float = 1e6, p_max: int = 256,
            sigma: float = 3.0, data_seed: int = 1005) -> BatchedWorkload:
    """B independent filters: M_b log-uniform in [m_lo, m_hi], N_b = max(1, M_b // P_b),
    P_b uniform in {1..p_max}, log-weights ~ N(0, sigma^2).  Filter b uses stream id b."""
    rng = np.random.Generator(np.random.PCG64(data_seed))
    Mb = np.rint(np.exp(rng.uniform(np.log(m_lo), np.log(m_hi), size=B))).astype(np.int64)
    Mb = np.maximum(Mb, 1)
    Pb = rng.integers(1, p_max + 1, size=B)
    Nb = np.maximum(1, Mb // Pb).astype(np.int64)
    w_off = np.zeros(B + 1, dtype=np.int64)
    w_off[1:] = np.cumsum(Mb)
    n_off = np.zeros(B + 1, dtype=np.int64)
    n_off[1:] = np.cumsum(Nb)
    w = np.exp(rng.normal(0.0, sigma, size=int(w_off[-1])))
    return BatchedWorkload(f"batched_B{B}", B, w, w_off, n_off,
                           description=f"B={B} filters, M_b log-uniform [{m_lo:g},{m_hi:g}], "
                                       f"N_b=M_b/P_b, P_b in 1..{p_max}")


CONFIGS = {
    "single": small_single,
    "engmf": engmf_step,
    "sparse": sparse_mass,
    "equal": equal_size,
    "batched": batched,
}
