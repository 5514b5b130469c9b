"""GPU parity of the three stages against the CPU oracle (through the C ABI).

Stage 3 is exact, so it is compared bit for bit on identical W and u.  Stages
1 and 2 are floating-point sums in a different (blocked) order, compared within
the bounds the summation orders allow: |dW| <= 2^-40 and |du| <= 1e-12 for
binary64 (the blocked sums differ from the compensated oracle by a few units
in the last place).
"""
import numpy as np
import pytest

import oracle
import workloads
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
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


# ---------------------------------------------------------------- stage 3
MAP_CASES = [
    ("tiny", 1, 1), ("M1", 1, 50), ("N_gt_M", 7, 300), ("ragged", 1000, 257),
    ("wide", 100000, 1000), ("dense", 70000, 65537), ("equal", 4096, 4096),
    # a workgroup's range near the size it stages in LDS, and a deep search
    ("stage_edge", 65536, 4096), ("deep", 3000000, 3000),
]


@pytest.mark.parametrize("name,M,N", MAP_CASES)
def test_inverse_cmf_exact(dev, dcr, name, M, N):
    rng = np.random.default_rng(M * 7 + N)
    w = np.exp(rng.normal(0, 2, M))
    w[rng.random(M) < 0.2] = 0.0
    if w.sum() == 0:
        w[-1] = 1.0
    W, _ = oracle.cumulative_weights(w)
    u = np.sort(rng.random(N))
    # put some uniforms exactly on bin edges and next to them
    k = min(N, M, 40)
    pick = rng.integers(0, M, k)
    u[:k] = W[pick]
    u[k // 2:k] = np.nextafter(W[pick[k // 2:]], 2.0)
    u = np.sort(np.clip(u, np.nextafter(0, 1), 1.0))
    r = dcr.dcr_inverse_cmf(_t(W, dev), _t(u, dev)).cpu().numpy()
    ref, _ = oracle.dac(W, u)
    assert np.array_equal(r, ref)
    assert np.array_equal(r, np.searchsorted(W[:-1], u, side="left"))


def test_inverse_cmf_fig1(dev, dcr):
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "fig1_worked_example.json")))
    r = dcr.dcr_inverse_cmf(_t(np.array(g["W"]), dev), _t(np.array(g["U"]), dev)).cpu().numpy()
    assert (r + 1).tolist() == g["r_paper_1based"]


def test_inverse_cmf_clamp(dev, dcr):
    W = np.array([0.1, 0.2, 0.9])
    u = np.array([0.05, 0.95, 1.0])
    r = dcr.dcr_inverse_cmf(_t(W, dev), _t(u, dev)).cpu().numpy()
    assert r.tolist() == [0, 2, 2]


# ---------------------------------------------------------------- stage 1
W_SIZES = [1, 2, 15, 16, 17, 255, 256, 257, 4097, 32767, 32768, 32769, 100003, 300000]


@pytest.mark.parametrize("M", W_SIZES)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_cumulative_weights(dev, dcr, M, dtype):
    rng = np.random.default_rng(M)
    w = np.exp(rng.normal(0, 3, M)).astype(dtype)
    if M > 10:
        w[rng.random(M) < 0.1] = 0
        w[-1] = 0
        if w.sum() == 0:
            w[0] = 1
    W_o, tot_o = oracle.cumulative_weights(w)
    total = torch.zeros(1, dtype=torch.float64, device=dev)
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    W_g = dcr.dcr_cumulative_weights(_t(w, dev), total=total, dev_status=st)
    W2 = dcr.dcr_cumulative_weights(_t(w, dev))
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    W_g = W_g.cpu().numpy()
    assert np.array_equal(W_g, W2.cpu().numpy()), "not reproducible"
    assert_monotone_unit(W_g)
    assert np.max(np.abs(W_g - W_o)) <= 2.0**-40
    assert abs(total.item() - tot_o) <= 1e-12 * tot_o


@pytest.mark.parametrize("bad", [-1.0, np.nan, np.inf])
def test_bad_weights_flagged(dev, dcr, bad):
    w = np.ones(70000)
    w[65000] = bad
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    r = dcr.dcr_resample(_t(w, dev), 100, seed=1, dev_status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 6
    assert np.all(r.cpu().numpy() == -1)
    st2 = torch.full((1,), -1, dtype=torch.int32, device=dev)
    dcr.dcr_cumulative_weights(_t(w, dev), dev_status=st2)
    torch.cuda.synchronize()
    assert int(st2.item()) == 6


def test_zero_total_flagged(dev, dcr):
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    r = dcr.dcr_resample(_t(np.zeros(1000), dev), 10, seed=1, dev_status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 6 and np.all(r.cpu().numpy() == -1)


# ---------------------------------------------------------------- stage 2
U_SIZES = [1, 2, 3, 4095, 4096, 4097, 10000, 70001]


@pytest.mark.parametrize("N", U_SIZES)
def test_sorted_uniforms_fp64(dev, dcr, N):
    u_g = dcr.dcr_sorted_uniforms(N, seed=77, stream_id=5, device=dev).cpu().numpy()
    u_o = oracle.sorted_uniforms(N, 77, 5)
    assert np.all(np.diff(u_g) >= 0) and u_g[0] > 0 and u_g[-1] <= 1
    assert np.max(np.abs(u_g - u_o)) <= 1e-12


@pytest.mark.parametrize("N", [1, 4097, 70001])
def test_sorted_uniforms_fp32_form(dev, dcr, N):
    u_g = dcr.dcr_sorted_uniforms(N, seed=78, stream_id=0, precision=dcr.DCR_FP32_COMP,
                                  device=dev).cpu().numpy()
    u_same = oracle.sorted_uniforms(N, 78, 0, zkind=1)   # same binary32 spacings
    u_64 = oracle.sorted_uniforms(N, 78, 0, zkind=0)
    assert np.all(np.diff(u_g) >= 0) and u_g[0] > 0 and u_g[-1] <= 1
    # the two binary32 logarithms are each within 1 ulp: |du| <= 2^-21 u
    assert np.max(np.abs(u_g - u_same)) <= 2.0**-21
    assert np.max(np.abs(u_g - u_64)) <= 2.0**-20


def test_sorted_uniforms_streams(dev, dcr):
    a = dcr.dcr_sorted_uniforms(1000, seed=1, stream_id=0, device=dev).cpu().numpy()
    b = dcr.dcr_sorted_uniforms(1000, seed=1, stream_id=1, device=dev).cpu().numpy()
    c = dcr.dcr_sorted_uniforms(1000, seed=1, stream_id=0, device=dev).cpu().numpy()
    assert not np.array_equal(a, b) and np.array_equal(a, c)


def test_inverse_cmf_dense_range_across_windows(dev, dcr):
    """Dense regime with a long run of zero weights: a workgroup whose
    uniforms straddle the run stages its range of W in several windows."""
    rng = np.random.default_rng(77)
    M, N = 100000, 50000
    w = np.exp(rng.normal(0, 1, M))
    w[20000:45000] = 0.0
    w[70000:70003] = 5e4                        # and a few heavy weights
    W, _ = oracle.cumulative_weights(w)
    u = np.sort(rng.random(N))
    r = dcr.dcr_inverse_cmf(_t(W, dev), _t(u, dev)).cpu().numpy()
    assert np.array_equal(r, np.searchsorted(W[:-1], u, side="left"))
    assert not np.any((r >= 20000) & (r < 45000))
