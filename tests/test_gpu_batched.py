"""Batched GPU resampling (dcr_resample_batched) against single calls and the oracle.

- Filter b of a batch must equal, bit for bit, dcr_resample on its own weights
  with stream id b (the batched kernels run the single-distribution block code
  on each filter's view of the arrays).
- binary64: equal to the oracle's batched result exactly.  binary32 form:
  every mismatch against the oracle is a bin-edge case.
- A bad filter is reported and filled with -1 without touching the others;
  broken offsets and exceeded capacities are reported and nothing is written.
"""
import numpy as np
import pytest

import oracle
import workloads
from parity_util import classify_mismatches

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_01356_amd as dcr
    dcr.library()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def dcr():
    import paper_2604_01356_amd as m
    return m


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def small_batch(B, seed, m_lo=1.0, m_hi=2e5, p_max=64, empty_every=0):
    """Uneven filters with M_b log-uniform in [m_lo, m_hi] (M_b = 1 included),
    N_b = M_b // P_b (P_b = 1 gives the dense regime), some N_b = 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Mb = np.maximum(1, np.rint(np.exp(rng.uniform(np.log(m_lo), np.log(m_hi), B)))).astype(np.int64)
    Pb = rng.integers(1, p_max + 1, B)
    Nb = np.maximum(1, Mb // Pb).astype(np.int64)
    if empty_every:
        Nb[::empty_every] = 0
    w_off = np.concatenate([[0], np.cumsum(Mb)]).astype(np.int64)
    n_off = np.concatenate([[0], np.cumsum(Nb)]).astype(np.int64)
    w = np.exp(rng.normal(0.0, 3.0, int(w_off[-1])))
    return w, w_off, n_off


def run_batched(dcr, dev, w, w_off, n_off, seed, sumM=None, sumN=None):
    B = len(w_off) - 1
    cap = int(n_off[-1]) if sumN is None else sumN
    r = torch.full((max(cap, int(n_off[-1]), 1),), -7, dtype=torch.int32, device=dev)
    seg = torch.full((B,), -1, dtype=torch.int32, device=dev)
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    dcr.dcr_resample_batched(_t(w, dev), _t(w_off, dev), _t(n_off, dev), seed,
                             sumM_max=sumM, sumN_max=sumN if sumN is not None else r.numel(),
                             r=r, seg_status=seg, dev_status=st)
    torch.cuda.synchronize()
    return r.cpu().numpy()[: int(n_off[-1])], seg.cpu().numpy(), int(st.item())


def single_calls(dcr, dev, w, w_off, n_off, seed, filters):
    """Per-filter dcr_resample (stream id b) with W and u."""
    out = {}
    for b in filters:
        wb = _t(w[w_off[b]:w_off[b + 1]], dev)
        N = int(n_off[b + 1] - n_off[b])
        W = torch.empty(wb.numel(), dtype=torch.float64, device=dev)
        u = torch.empty(max(N, 1), dtype=torch.float64, device=dev)
        r = dcr.dcr_resample(wb, N, seed, b, W_out=W, u_out=u)
        out[b] = (r.cpu().numpy(), W.cpu().numpy(), u[:N].cpu().numpy())
    return out


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_batched_equals_single_calls(dcr, dev, dtype):
    w, w_off, n_off = small_batch(60, 11, empty_every=13)
    w = w.astype(dtype)
    seed = 5
    r, seg, st = run_batched(dcr, dev, w, w_off, n_off, seed)
    assert st == 0 and np.all(seg == 0)
    single = single_calls(dcr, dev, w, w_off, n_off, seed, range(len(w_off) - 1))
    for b, (rb, _, _) in single.items():
        assert np.array_equal(r[n_off[b]:n_off[b + 1]], rb), f"filter {b}"


def test_batched_fp64_equals_oracle(dcr, dev):
    w, w_off, n_off = small_batch(40, 12, empty_every=7)
    r, seg, st = run_batched(dcr, dev, w, w_off, n_off, 9)
    assert st == 0
    r_o = oracle.resample_batched(w, w_off, n_off, 9)
    assert np.array_equal(r, r_o)


def test_batched_fp32_against_oracle(dcr, dev):
    w, w_off, n_off = small_batch(40, 13)
    w = w.astype(np.float32)
    r, seg, st = run_batched(dcr, dev, w, w_off, n_off, 3)
    assert st == 0
    single = single_calls(dcr, dev, w, w_off, n_off, 3, range(len(w_off) - 1))
    total = 0
    for b, (rb, Wb, ub) in single.items():
        seg_r = r[n_off[b]:n_off[b + 1]]
        assert np.array_equal(seg_r, rb)
        r_o, W_o, u_o = oracle.resample(w[w_off[b]:w_off[b + 1]], len(rb), 3, b)
        n_mis, bad = classify_mismatches(seg_r, r_o, ub, u_o, Wb, W_o)
        assert not bad, f"filter {b}: mismatches away from bin edges {bad[:5]}"
        total += n_mis
    print(f"  binary32 batch: {total} bin-edge mismatches over {int(n_off[-1])} draws")


def test_batched_single_filter_and_tiny(dcr, dev):
    # B = 1 (equals a single call) and filters of one weight each
    w = np.exp(np.random.Generator(np.random.PCG64(3)).normal(0, 1, 5000))
    r, _, st = run_batched(dcr, dev, w, np.array([0, 5000]), np.array([0, 777]), 4)
    assert st == 0
    r1 = dcr.dcr_resample(_t(w, dev), 777, 4, 0).cpu().numpy()
    assert np.array_equal(r, r1)
    w_off = np.arange(0, 65, dtype=np.int64)
    n_off = np.arange(0, 65 * 3, 3, dtype=np.int64)
    r, seg, st = run_batched(dcr, dev, np.ones(64), w_off, n_off, 1)
    assert st == 0 and np.all(r == 0)


def test_batched_bad_filter_is_isolated(dcr, dev):
    w, w_off, n_off = small_batch(20, 14)
    w[w_off[3] + 1] = -1.0            # filter 3: negative weight
    w[w_off[11]] = np.nan             # filter 11: NaN
    w[w_off[16]:w_off[17]] = 0.0      # filter 16: zero total
    bad_f = (3, 11, 16)
    r, seg, st = run_batched(dcr, dev, w, w_off, n_off, 2)
    assert st == 6
    assert all(seg[b] == 6 for b in bad_f)
    assert np.all(seg[[b for b in range(20) if b not in bad_f]] == 0)
    for b in range(20):
        part = r[n_off[b]:n_off[b + 1]]
        if b in bad_f:
            assert np.all(part == -1)
        else:
            good = oracle.resample(w[w_off[b]:w_off[b + 1]], len(part), 2, b)[0]
            assert np.array_equal(part, good)


def test_batched_invalid_offsets_and_capacity(dcr, dev):
    w, w_off, n_off = small_batch(10, 15)
    bad = w_off.copy()
    bad[4] = bad[3]                    # filter 3 would have no weights
    r, _, st = run_batched(dcr, dev, w, bad, n_off, 1)
    assert st == 1 and np.all(r == -7)
    bad = n_off.copy()
    bad[0] = 1                         # offsets must start at 0
    r, _, st = run_batched(dcr, dev, w, w_off, bad, 1)
    assert st == 1
    # more draws than the stated capacity
    r, _, st = run_batched(dcr, dev, w, w_off, n_off, 1, sumN=int(n_off[-1]) + 5)
    assert st == 0
    B = len(w_off) - 1
    rt = torch.full((int(n_off[-1]),), -7, dtype=torch.int32, device=dev)
    st_t = torch.full((1,), -1, dtype=torch.int32, device=dev)
    dcr.dcr_resample_batched(_t(w, dev), _t(w_off, dev), _t(n_off, dev), 1,
                             sumN_max=int(n_off[-1]) - 1, r=rt, dev_status=st_t)
    torch.cuda.synchronize()
    assert int(st_t.item()) == 4 and bool((rt == -7).all())
    assert B == 10


def test_batched_full_size_sampled(dcr, dev):
    """The 4096-filter workload in the binary32 form: sampled filters equal
    their single calls bit for bit and the oracle up to bin-edge cases."""
    bw = workloads.batched()
    w32 = bw.w32
    r, seg, st = run_batched(dcr, dev, w32, bw.w_off, bw.n_off, 0)
    assert st == 0 and np.all(seg == 0)
    Mb = np.diff(bw.w_off)
    rng = np.random.Generator(np.random.PCG64(77))
    pick = sorted(set(rng.choice(bw.B, 24, replace=False).tolist()
                      + [int(np.argmax(Mb)), int(np.argmin(Mb)), 0, bw.B - 1]))
    single = single_calls(dcr, dev, w32, bw.w_off, bw.n_off, 0, pick)
    mism = 0
    for b in pick:
        rb, Wb, ub = single[b]
        part = r[bw.n_off[b]:bw.n_off[b + 1]]
        assert np.array_equal(part, rb), f"filter {b}"
        r_o, W_o, u_o = oracle.resample(w32[bw.w_off[b]:bw.w_off[b + 1]], len(rb), 0, b)
        n_mis, bad = classify_mismatches(part, r_o, ub, u_o, Wb, W_o)
        assert not bad
        mism += n_mis
    # every filter's indices are in range and non-decreasing
    for b in range(bw.B):
        part = r[bw.n_off[b]:bw.n_off[b + 1]]
        if len(part):
            assert part[0] >= 0 and part[-1] < Mb[b] and np.all(np.diff(part) >= 0)
    print(f"  batched B={bw.B} sumM={int(bw.w_off[-1])} sumN={int(bw.n_off[-1])}: "
          f"{mism} bin-edge mismatches in {len(pick)} sampled filters")


def test_batched_chunks_agree_and_autotune(dcr, dev, tmp_path):
    """Every map tile gives the same indices; the autotuner picks one of them
    and answers from its cache the second time."""
    w, w_off, n_off = small_batch(50, 16, empty_every=9)
    w = w.astype(np.float32)
    wt, wo, no = _t(w, dev), _t(w_off, dev), _t(n_off, dev)
    n = int(n_off[-1])
    outs = {}
    for c in (256, 512, 1024):
        r = dcr.dcr_resample_batched_ex(wt, wo, no, 6, chunk=c, sumN_max=n)
        torch.cuda.synchronize()
        outs[c] = r.cpu().numpy()[:n]
    assert np.array_equal(outs[256], outs[512]) and np.array_equal(outs[512], outs[1024])
    ref = oracle.resample_batched(w, w_off, n_off, 6)
    mism = int(np.sum(outs[512] != ref))
    assert mism <= max(10, n // 1000)          # binary32 form: bin-edge cases only
    cache = tmp_path / "tune.txt"
    c1, ms1 = dcr.dcr_batched_autotune(wt, wo, no, 6, sumN_max=n, cache_path=cache)
    assert c1 in (256, 512, 1024) and ms1 > 0
    c2, ms2 = dcr.dcr_batched_autotune(wt, wo, no, 6, sumN_max=n, cache_path=cache)
    assert c2 == c1 and ms2 == -1.0
