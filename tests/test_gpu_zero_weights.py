"""Weights of zero get empty intervals on the GPU (Sec. I, Eq. 3: a bin of
weight zero has probability zero).

The oracle's cumulative weights are exact sums, so a weight of zero repeats
the previous W exactly.  The GPU sums in blocks; the block-end rule and the
scan's handling of zero totals must give the same property: W_j == W_{j-1}
exactly wherever w_j == 0 (W_0 == 0 if w_0 == 0), whatever boundary the zero
sits on: the end or start of a block, a whole block, a whole run of blocks
that fills one scan thread's range, the array's ends.  Then no index can land
on a zero weight (the map is exact on the GPU's own W and u).  Each case also
runs the usual parity checks against the oracle.
"""
import numpy as np
import pytest

from gpu_util import DU_FP32, DU_FP64, check_against_oracle, run_case, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BLOCK = 32768


@pytest.fixture(scope="module")
def dcr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_01356_amd as m
    m.library()
    return m


def zero_pattern(M, seed, dtype, per_thread_blocks):
    """Log-normal weights with zeros on every kind of boundary."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = np.exp(rng.normal(0.0, 2.0, M))
    nb = -(-M // BLOCK)
    w[:3 * BLOCK + 17] = 0.0                       # leading zero blocks and a partial one
    for b in range(4, nb - 1, 5):                  # block ends: 1, 5, 300, 4000 zeros
        k = (1, 5, 300, 4000)[(b // 5) % 4]
        w[(b + 1) * BLOCK - k:(b + 1) * BLOCK] = 0.0
    for b in range(6, nb - 1, 7):                  # block starts
        w[b * BLOCK:b * BLOCK + 257] = 0.0
    for b in range(9, nb - 1, 11):                 # whole blocks
        w[b * BLOCK:(b + 1) * BLOCK] = 0.0
    if per_thread_blocks > 1 and nb > 4 * per_thread_blocks:
        t0 = 2 * per_thread_blocks                 # one scan thread's whole range, and the
        w[t0 * BLOCK:(t0 + per_thread_blocks) * BLOCK] = 0.0   # block after it
        w[(t0 + per_thread_blocks) * BLOCK:(t0 + per_thread_blocks) * BLOCK + 999] = 0.0
    w[rng.random(M) < 0.2] = 0.0                   # scattered zeros
    w[-(BLOCK + 100):] = 0.0                       # trailing zeros past the last block start
    w[M // 2] = 5.0                                # keep a positive total
    return w.astype(dtype)


def assert_zero_bins_empty(w, W, r):
    z = np.flatnonzero(w == 0)
    z1 = z[z > 0]
    assert np.array_equal(W[z1], W[z1 - 1]), "a zero weight moved W"
    if w[0] == 0:
        assert W[0] == 0.0
    assert not np.any(w[r] == 0), "an index landed on a zero weight"


CASES = [
    # (M, N, map the fused call takes, blocks per scan thread)
    (200_000, 3000, "finish", 1),                           # the small path (7 blocks)
    ((1 << 20) + 333, 5000, "finish", 1),
    ((1 << 21) + 3, (1 << 18) + 5, "map_fused", 1),
    (300_000, 200_000, "map_dense", 1),
    ((1 << 27) + 4 * BLOCK + 9, 3000, "map_fused", 17),    # 4101 blocks: 17 per scan thread
]


# binary64 and binary32 for every case but the largest, which runs in binary32
# only (the scan it covers is the same in both forms)
PARAMS = [(c, dt) for c in CASES for dt in (np.float64, np.float32)
          if not (c[0] > (1 << 27) and dt == np.float64)]


@pytest.mark.parametrize("case,dtype", PARAMS)
def test_zero_weights_have_empty_intervals(dcr, case, dtype):
    M, N, kind, per = case
    w = zero_pattern(M, M % 1000, dtype, per)
    print(f"  zeros: M={M} N={N} {np.dtype(dtype).name} expect {kind}", flush=True)
    out = run_case(dcr, torch.device("cuda:0"), w, N, seed=21, stream=2, expect=kind)
    assert_zero_bins_empty(w, out["W"], out["r"])
    check_against_oracle(out, w, N, 21, 2, DU_FP64 if dtype == np.float64 else DU_FP32)


def test_zero_weights_batched_and_outer(dcr):
    dev = torch.device("cuda:0")
    rng = np.random.Generator(np.random.PCG64(77))
    # batched: every filter with zero blocks and zero ends; equal to single calls
    Mb = np.array([3 * BLOCK + 5, 70_000, BLOCK, 5 * BLOCK + 1, 1000], dtype=np.int64)
    Nb = np.array([400, 60_000, 30_000, 2000, 1], dtype=np.int64)
    w_off = np.concatenate([[0], np.cumsum(Mb)]).astype(np.int64)
    n_off = np.concatenate([[0], np.cumsum(Nb)]).astype(np.int64)
    w = np.concatenate([zero_pattern(int(m), 5 + i, np.float32, 1) for i, m in enumerate(Mb)])
    r = dcr.dcr_resample_batched(to_dev(w, dev), to_dev(w_off, dev), to_dev(n_off, dev), 3,
                                 sumN_max=int(n_off[-1]))
    torch.cuda.synchronize()
    r = r.cpu().numpy()
    for b in range(len(Mb)):
        wb = w[w_off[b]:w_off[b + 1]]
        rb = r[n_off[b]:n_off[b + 1]]
        single = dcr.dcr_resample(to_dev(wb, dev), int(Nb[b]), 3, b).cpu().numpy()
        assert np.array_equal(rb, single), b
        assert not np.any(wb[rb] == 0), b
    # outer products: zero particle rows and zero component columns
    Na, P, N = 9000, 64, 9000
    a = rng.lognormal(0.0, 1.0, Na)
    b = rng.dirichlet(np.full(P, 0.5))
    a[::7] = 0.0
    a[4096:4096 + 600] = 0.0           # a whole weight block of zero rows
    b[[0, 5, 63]] = 0.0
    W = torch.empty(Na * P, dtype=torch.float64, device=dev)
    u = torch.empty(N, dtype=torch.float64, device=dev)
    ro = dcr.dcr_resample_outer(to_dev(a, dev), to_dev(b, dev), N, 4, 1, W_out=W, u_out=u)
    torch.cuda.synchronize()
    wo = np.multiply.outer(a, b).ravel()
    assert_zero_bins_empty(wo, W.cpu().numpy(), ro.cpu().numpy())
