"""End-to-end GPU resampling (dcr_resample) against the CPU oracle.

- The fused end-to-end call must equal, bit for bit, stage 3 applied to the W
  and u of stages 1 and 2 (and the oracle's exact map on those W and u).
- Against the oracle's own end-to-end result, every index mismatch must be a
  bin-edge case (the uniform lies within |du| + max|dW| + 1 ulp of an edge
  separating the two indices); their number is reported.
"""
import numpy as np
import pytest
from scipy import stats

import oracle
import workloads
from gpu_util import DU_FP32, check_against_oracle, run_case, to_dev
from parity_util import assert_monotone_unit

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
    return to_dev(a, dev)


# (M, N): ragged edges of lanes, sub-tiles, blocks and spacing blocks; two
# sparse cases with two and four draws per quad in the finishing launch; the
# last two are dense (N >= M/4: the windowed merge) with N + 1 >= 2^18
RAGGED = [(1, 5), (3, 1), (5, 0), (100, 1000), (32769, 4097), (65537, 3), (40000, 4095),
          (300001, 8191), (4194307, 40001), (8388617, 150001), (100003, 262143),
          (70001, 300000)]


@pytest.mark.parametrize("M,N", RAGGED)
def test_ragged_fp64(dev, dcr, M, N):
    rng = np.random.default_rng(M + 31 * N)
    w = np.exp(rng.normal(0, 2, M))
    out = run_case(dcr, dev, w, N, seed=11, stream=2)
    check_against_oracle(out, w, N, 11, 2, 1e-12, 2.0**-40)


@pytest.mark.parametrize("M,N", RAGGED)
def test_ragged_fp32(dev, dcr, M, N):
    rng = np.random.default_rng(M + 37 * N)
    w = np.exp(rng.normal(0, 2, M)).astype(np.float32)
    out = run_case(dcr, dev, w, N, seed=12, stream=0)
    # the oracle consumes the same binary32 weights promoted exactly, and the
    # binary32 form of the spacings (z = -logf(fl32(v)))
    check_against_oracle(out, w, N, 12, 0, DU_FP32, 2.0**-40)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_dense_wide_spans(dev, dcr, dtype):
    """Dense regime (4N >= M) with log-weights ~ N(0, 6^2): the draws pile on a
    few heavy weights, so chunks of the dense map span far more than 64
    sub-tiles and take the per-draw quad search; the rest merge in windows."""
    M, N = (1 << 20) + 77, (1 << 18) + 99
    rng = np.random.default_rng(606)
    w = np.exp(rng.normal(0, 6, M)).astype(dtype)
    out = run_case(dcr, dev, w, N, seed=21, stream=4, expect="map_dense")
    r = out["r"]
    # every dense-map chunk is a whole number of 256-draw blocks, so a block
    # whose indices span more than 65 sub-tiles of 256 lies in a wide chunk
    spans = r[255:N:256] - r[0:N - 255:256]
    assert spans.max() > 65 * 256 and spans.min() < 16 * 256
    du_cap = 1e-12 if dtype == np.float64 else DU_FP32
    check_against_oracle(out, w, N, 21, 4, du_cap, 2.0**-40)


@pytest.mark.parametrize("maker", ["small_single", "engmf_step"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_paper_shaped_configs(dev, dcr, maker, dtype):
    wl = getattr(workloads, maker)()
    w = wl.w64 if dtype == "f64" else wl.w32
    out = run_case(dcr, dev, w, wl.N, seed=0, stream=0)
    du_cap = 1e-12 if dtype == "f64" else DU_FP32
    check_against_oracle(out, w, wl.N, 0, 0, du_cap, 2.0**-40)


def test_zero_weight_bins_never_drawn(dev, dcr):
    rng = np.random.default_rng(5)
    w = np.exp(rng.normal(0, 1, 50000))
    w[rng.random(50000) < 0.5] = 0.0
    r = dcr.dcr_resample(_t(w, dev), 20000, seed=9).cpu().numpy()
    assert np.all(w[r] > 0)


def test_counts_chi_square_gpu(dev, dcr):
    rng = np.random.default_rng(3)
    M, N = 40, 200000
    w = np.exp(rng.normal(0, 1, M))
    r = dcr.dcr_resample(_t(w, dev), N, seed=17).cpu().numpy()
    c = np.bincount(r, minlength=M)
    assert stats.chisquare(c, N * w / w.sum()).pvalue > 1e-4


@pytest.mark.parametrize("M,N", [(3000, 50000), (200000, 2000)])
def test_counts_chi_square_regimes_gpu(dev, dcr, M, N):
    """Counts pooled over seeds against N w (chi square on cells with at
    least 20 expected draws), in the dense merge and in the sparse map."""
    rng = np.random.default_rng(M)
    w = np.exp(rng.normal(0, 1.5, M))
    p = w / w.sum()
    R = 30
    wt = _t(w, dev)
    c = np.zeros(M)
    for s in range(R):
        c += np.bincount(dcr.dcr_resample(wt, N, seed=1000 + s).cpu().numpy(), minlength=M)
    exp = R * N * p
    big = exp >= 20
    obs = np.concatenate([c[big], [c[~big].sum()]])
    ex = np.concatenate([exp[big], [exp[~big].sum()]])
    assert stats.chisquare(obs, ex).pvalue > 1e-4


def test_seed_and_stream_reproducible(dev, dcr):
    w = _t(np.exp(np.random.default_rng(1).normal(0, 1, 10000)), dev)
    a = dcr.dcr_resample(w, 3000, seed=5, stream_id=2).cpu().numpy()
    b = dcr.dcr_resample(w, 3000, seed=5, stream_id=2).cpu().numpy()
    c = dcr.dcr_resample(w, 3000, seed=5, stream_id=3).cpu().numpy()
    assert np.array_equal(a, b) and not np.array_equal(a, c)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_dense_with_light_gap(dev, dcr, dtype):
    """Dense overall (N > M/4) with a long run of negligible weights: the
    workgroups whose uniforms straddle the run see a span of hundreds of
    sub-tiles and take the per-uniform search."""
    rng = np.random.default_rng(77)
    M, N = 400000, 200000
    w = np.exp(rng.normal(0, 1, M))
    w[100000:300000] *= 1e-12
    w = w.astype(dtype)
    out = run_case(dcr, dev, w, N, seed=8, stream=0)
    check_against_oracle(out, w, N, 8, 0, 1e-12 if dtype == np.float64 else DU_FP32, 2.0**-40)


@pytest.mark.parametrize("N", [3000, 262143])
def test_largest_single_launch_finish(dev, dcr, N):
    """The largest problem the single finishing launch takes: 4096 weight blocks
    (every scan thread holds 16 block totals in registers, the last block
    ragged) and, at N = 2^18 - 1, 64 spacing blocks with four draws per quad."""
    M = (1 << 27) - 7
    rng = np.random.default_rng(123)
    w = np.exp(rng.normal(0, 3, M)).astype(np.float32)
    print(f"  largest finish: M={M} N={N}", flush=True)
    out = run_case(dcr, dev, w, N, seed=6, stream=2, expect="finish")
    check_against_oracle(out, w, N, 6, 2, DU_FP32, 2.0**-40)


@pytest.mark.parametrize("which", ["sparse", "equal"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_size(dev, dcr, which, dtype):
    """The large configurations at full size, in the benchmark's launch shape."""
    wl = workloads.sparse_mass() if which == "sparse" else workloads.equal_size()
    w = wl.w64 if dtype == "f64" else wl.w32
    del wl
    N = (1 << 14) if which == "sparse" else (1 << 24)
    print(f"  full size {which} {dtype}: M={len(w)} N={N}", flush=True)
    out = run_case(dcr, dev, w, N, seed=0, stream=0)
    du_cap = 1e-12 if dtype == "f64" else DU_FP32
    n_mis = check_against_oracle(out, w, N, 0, 0, du_cap, 2.0**-40)
    assert n_mis <= max(10, N // 1000)


def test_large_n_dense(dev, dcr):
    """N = 2^26 draws from M = 2^22 binary32 weights (16 draws per weight, the
    dense merge, 64-bit draw offsets in the grid): u is sorted and agrees with
    the oracle's within the binary32 bound, r is non-decreasing, and sampled
    indices are exact on the GPU's own W and u."""
    M, N = 1 << 22, 1 << 26
    rng = np.random.default_rng(2026)
    w = np.exp(rng.normal(0, 1, M)).astype(np.float32)
    wt = _t(w, dev)
    W = torch.empty(M, dtype=torch.float64, device=dev)
    u = torch.empty(N, dtype=torch.float64, device=dev)
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    r = dcr.dcr_resample(wt, N, seed=3, stream_id=7, W_out=W, u_out=u, dev_status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    rg, Wg, ug = r.cpu().numpy(), W.cpu().numpy(), u.cpu().numpy()
    del r, W, u
    assert_monotone_unit(Wg)
    assert np.all(np.diff(ug) >= 0) and ug[0] > 0 and ug[-1] <= 1
    assert np.all(np.diff(rg) >= 0) and rg[0] >= 0 and rg[-1] < M
    idx = np.unique(np.concatenate([np.arange(0, N, 4099), [N - 1]]))
    j = rg[idx]
    assert np.all(Wg[j] >= ug[idx])
    assert np.all((j == 0) | (Wg[np.maximum(j - 1, 0)] < ug[idx]))
    u_o = oracle.sorted_uniforms(N, 3, 7, zkind=1)
    assert np.max(np.abs(ug - u_o)) <= DU_FP32


@pytest.mark.parametrize("dtype,shift", [(np.float32, 1), (np.float32, 2), (np.float32, 3),
                                         (np.float64, 1), (np.float64, 3)])
def test_weights_off_16_byte_boundary(dev, dcr, dtype, shift):
    """Weights that start off a 16-byte boundary (a view into a larger buffer)
    take other load paths; the result must equal the aligned call bit for bit,
    in the sparse and the dense regime."""
    rng = np.random.Generator(np.random.PCG64(40 + shift))
    M = 5 * 32768 + 1234                      # several full blocks and a ragged one
    w = np.exp(rng.normal(0.0, 2.0, M)).astype(dtype)
    buf = torch.zeros(M + 8, dtype=torch.from_numpy(w).dtype, device=dev)
    buf[shift:shift + M] = _t(w, dev)
    view = buf[shift:shift + M]
    assert view.data_ptr() % 16 != 0
    aligned = _t(w, dev)
    for N in (777, 120000):
        for x in (view, aligned):
            assert x.is_contiguous()
        W0 = torch.empty(M, dtype=torch.float64, device=dev)
        W1 = torch.empty(M, dtype=torch.float64, device=dev)
        r0 = dcr.dcr_resample(aligned, N, 3, 0, W_out=W0)
        r1 = dcr.dcr_resample(view, N, 3, 0, W_out=W1)
        torch.cuda.synchronize()
        assert np.array_equal(r0.cpu().numpy(), r1.cpu().numpy())
        assert np.array_equal(W0.cpu().numpy(), W1.cpu().numpy())


def test_maximum_size_properties(dev, dcr):
    """The largest M the boundary accepts (2^31 - 1 binary32 weights, 8 GB;
    indices are int32) with N = 2^20 draws.  The oracle does not run at this
    size; the fused indices are checked against the separately called stages
    instead, which are bit-consistent with them: W_{r-1} < u <= W_r for every
    draw, W non-decreasing with W_{M-1} = 1, r in range and non-decreasing."""
    M = (1 << 31) - 1
    N = 1 << 20
    g = torch.Generator(device=dev)
    g.manual_seed(9)
    w = torch.rand(M, generator=g, device=dev, dtype=torch.float32)
    w[M // 3:M // 3 + 100000] = 0.0            # a run of zero weights
    r = dcr.dcr_resample(w, N, 5, 0).long()
    W = dcr.dcr_cumulative_weights(w)
    del w
    u = dcr.dcr_sorted_uniforms(N, 5, 0, precision=dcr.DCR_FP32_COMP, device=dev)
    torch.cuda.synchronize()
    assert int(r.min()) >= 0 and int(r.max()) <= M - 1
    assert bool(torch.all(r[1:] >= r[:-1]))
    assert float(W[-1]) == 1.0
    assert bool(torch.all(W[1:] >= W[:-1]))
    Wr = W[r]
    Wprev = torch.where(r > 0, W[(r - 1).clamp(min=0)], torch.zeros_like(Wr))
    assert bool(torch.all((u <= Wr) | (r == M - 1)))
    assert bool(torch.all(Wprev < u))
    zero_run = (r >= M // 3) & (r < M // 3 + 100000)
    assert not bool(zero_run.any())
    print(f"  M={M} N={N}: r in [{int(r.min())}, {int(r.max())}]", flush=True)


def _degenerate(kind):
    M = 3 * 32768 + 77
    if kind == "one_weight_first":
        w = np.zeros(M); w[0] = 2.5
    elif kind == "one_weight_block_edge":
        w = np.zeros(M); w[32767] = 1e-3
    elif kind == "one_weight_last":
        w = np.zeros(M); w[-1] = 7.0
    elif kind == "subnormal_f64":
        rng = np.random.default_rng(3)
        w = rng.integers(0, 50, M) * 5e-324     # binary64 subnormals only
        w[w.argmax()] += 5e-324
    elif kind == "subnormal_f32":
        rng = np.random.default_rng(4)
        w = (rng.random(M) * 1e-39).astype(np.float32)   # binary32 subnormals
    elif kind == "wide_range_f64":
        rng = np.random.default_rng(5)
        w = 10.0 ** rng.uniform(-300, 300, M)
    else:
        raise ValueError(kind)
    return w


@pytest.mark.parametrize("kind", ["one_weight_first", "one_weight_block_edge", "one_weight_last",
                                  "subnormal_f64", "subnormal_f32", "wide_range_f64"])
def test_degenerate_weights(dev, dcr, kind):
    """A single nonzero weight (first, at a block edge, last), weights that
    are all subnormal, and weights over 600 decades: the fused call equals the
    stages and agrees with the oracle."""
    w = _degenerate(kind)
    for N in (5, 2000, 200000):
        out = run_case(dcr, dev, w, N, seed=21, stream=1)
        if kind.startswith("one_weight"):
            assert np.all(out["r"] == int(np.flatnonzero(w)[0]))
        du = DU_FP32 if w.dtype == np.float32 else 1e-12
        check_against_oracle(out, w, N, 21, 1, du, 2.0**-40)


def test_total_overflow_flagged(dev, dcr):
    """Finite weights whose sum overflows binary64: reported, r filled with -1."""
    w = np.ones(100000)
    w[[10, 50000, 99999]] = 1e308
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    r = dcr.dcr_resample(_t(w, dev), 300, seed=1, dev_status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 6
    assert np.all(r.cpu().numpy() == -1)
