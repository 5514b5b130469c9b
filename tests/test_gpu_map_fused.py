"""The sparse map that runs after the separate carry scan (k_map_fused and its
outer-product twin), in every form it serves, against the oracle.

The end-to-end call takes this map when the draws are sparse (M > 4N) and the
single finishing launch cannot hold the scans: more than 4096 weight blocks
(M > 2^27) or more than 64 spacing blocks (N + 1 > 2^18).  Each case checks
through the library's per-launch profile that the map kernel it means to
cover ran, then compares with the oracle element by element (u within its
cap, every index mismatch at a bin edge) and with the separately called
stages bit for bit.  Divide-and-conquer map: Sec. III, Alg. 5; schemes:
Sec. V.
"""
import numpy as np
import pytest

import oracle
from gpu_util import (DU_FP32, DU_FP64, DW_CAP, check_against_oracle, profiled, run_case,
                      to_dev)
from parity_util import assert_monotone_unit, classify_mismatches

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BIG_M = (1 << 27) + 12345        # 4097 weight blocks: more than the finishing launch holds
WIDE_N = (1 << 18) + 5           # 65 spacing blocks: more than the finishing launch holds


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


def _weights(M, seed, sigma, dtype):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.exp(rng.normal(0.0, sigma, M)).astype(dtype)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_many_weight_blocks(dev, dcr, dtype):
    """M > 2^27: the block ends do not fit the finishing launch's LDS; the map
    keeps every second one there and ends the block search in memory."""
    w = _weights(BIG_M, 99, 4.0, dtype)
    print(f"  map_fused many blocks: M={BIG_M} N=5000 {np.dtype(dtype).name}", flush=True)
    out = run_case(dcr, dev, w, 5000, seed=4, stream=1, expect="map_fused")
    du = DU_FP64 if dtype == np.float64 else DU_FP32
    check_against_oracle(out, w, 5000, 4, 1, du)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("M", [(1 << 21) + 3, (1 << 23) + 77])
def test_many_spacing_blocks(dev, dcr, dtype, M):
    """N + 1 > 2^18 spacings with M > 4N: every block end is in LDS (one per
    entry), the uniforms are formed from the scanned spacing-block ends."""
    w = _weights(M, M, 2.0, dtype)
    print(f"  map_fused many spacing blocks: M={M} N={WIDE_N} {np.dtype(dtype).name}", flush=True)
    out = run_case(dcr, dev, w, WIDE_N, seed=13, stream=3, expect="map_fused")
    du = DU_FP64 if dtype == np.float64 else DU_FP32
    check_against_oracle(out, w, WIDE_N, 13, 3, du)


@pytest.mark.parametrize("scheme,code", [("stratified", 1), ("systematic", 2)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_schemes_many_weight_blocks(dev, dcr, scheme, code, dtype):
    """Stratified and systematic uniforms through the same map (M > 2^27; the
    schemes have no spacing scan, so only the weight side sends them here)."""
    M, N = (1 << 27) + 5, 3000
    w = _weights(M, 7 + code, 3.0, dtype)
    wt = to_dev(w, dev)
    W = torch.empty(M, dtype=torch.float64, device=dev)
    u = torch.empty(N, dtype=torch.float64, device=dev)
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    print(f"  map_fused {scheme}: M={M} N={N} {np.dtype(dtype).name}", flush=True)
    r, kinds = profiled(dcr, lambda: dcr.dcr_resample_scheme(wt, N, 3, 2, code, W_out=W, u_out=u,
                                                             dev_status=st))
    assert kinds.get("map_fused", 0) == 1, kinds
    r_plain = dcr.dcr_resample_scheme(wt, N, 3, 2, code)
    r3 = dcr.dcr_inverse_cmf(W, dcr.dcr_scheme_uniforms(N, 3, 2, code, device=dev))
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    rg, Wg, ug = r.cpu().numpy(), W.cpu().numpy(), u.cpu().numpy()
    del wt, W, u
    assert np.array_equal(rg, r_plain.cpu().numpy()) and np.array_equal(rg, r3.cpu().numpy())
    assert_monotone_unit(Wg)
    r_o, W_o, u_o = oracle.resample_scheme(w, N, 3, 2, scheme)
    assert np.array_equal(ug, u_o)                       # a closed formula: bit for bit
    assert np.max(np.abs(Wg - W_o)) <= DW_CAP
    r_exact, _ = oracle.dac(Wg, ug)
    assert np.array_equal(rg, r_exact)
    n_mis, bad = classify_mismatches(rg, r_o, ug, u_o, Wg, W_o)
    assert not bad, bad[:5]
    print(f"  bin-edge mismatches={n_mis}", flush=True)


def _factors(Na, P, seed, dtype):
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.lognormal(0.0, 1.0, Na).astype(dtype)
    b = rng.dirichlet(np.full(P, 0.5)).astype(dtype)
    return a, b


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_outer_many_spacing_blocks(dev, dcr, dtype):
    """Outer-product weights w[i*P + k] = a[i] * b[k] (never stored) through
    the outer twin of the map: Na = 8192, P = 256 (M = 2^21), N = 300000."""
    Na, P, N = 8192, 256, 300000
    a, b = _factors(Na, P, 31 + P, dtype)
    M = Na * P
    at, bt = to_dev(a, dev), to_dev(b, dev)
    W = torch.empty(M, dtype=torch.float64, device=dev)
    u = torch.empty(N, dtype=torch.float64, device=dev)
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    r, kinds = profiled(dcr, lambda: dcr.dcr_resample_outer(at, bt, N, seed=5, stream_id=2,
                                                            W_out=W, u_out=u, dev_status=st))
    assert kinds.get("map_fused", 0) == 1, kinds
    r_plain = dcr.dcr_resample_outer(at, bt, N, seed=5, stream_id=2)
    r3 = dcr.dcr_inverse_cmf(W, u)
    # the products as a caller would materialise them (exact for binary32
    # factors), through the array path
    w = np.multiply.outer(a.astype(np.float64), b.astype(np.float64)).ravel()
    r_arr = None
    if dtype == np.float64:
        r_arr = dcr.dcr_resample(to_dev(w, dev), N, seed=5, stream_id=2)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    rg, Wg, ug = r.cpu().numpy(), W.cpu().numpy(), u.cpu().numpy()
    assert np.array_equal(rg, r_plain.cpu().numpy()) and np.array_equal(rg, r3.cpu().numpy())
    if r_arr is not None:
        assert np.array_equal(rg, r_arr.cpu().numpy())
    out = dict(r=rg, W=Wg, u=ug, kinds=kinds)
    zkind = 0 if dtype == np.float64 else 1
    check_against_oracle(out, w, N, 5, 2, DU_FP64 if zkind == 0 else DU_FP32, zkind=zkind)


def test_outer_stratified_many_weight_blocks(dev, dcr):
    """Outer-product weights with more than 2^27 products and the stratified
    scheme: the outer twin of the map with the scheme's uniforms."""
    Na, P, N = (1 << 20) + 1, 128, 4000
    a, b = _factors(Na, P, 77, np.float32)
    at, bt = to_dev(a, dev), to_dev(b, dev)
    M = Na * P
    W = torch.empty(M, dtype=torch.float64, device=dev)
    u = torch.empty(N, dtype=torch.float64, device=dev)
    r, kinds = profiled(dcr, lambda: dcr.dcr_resample_outer(at, bt, N, 9, 1, dcr.DCR_STRATIFIED,
                                                            W_out=W, u_out=u))
    assert kinds.get("map_fused", 0) == 1, kinds
    torch.cuda.synchronize()
    rg, Wg, ug = r.cpu().numpy(), W.cpu().numpy(), u.cpu().numpy()
    del W, u
    w = np.multiply.outer(a.astype(np.float64), b.astype(np.float64)).ravel()
    r_o, W_o, u_o = oracle.resample_scheme(w, N, 9, 1, "stratified")
    assert np.array_equal(ug, u_o)
    assert np.max(np.abs(Wg - W_o)) <= DW_CAP
    assert np.array_equal(rg, oracle.dac(Wg, ug)[0])
    n_mis, bad = classify_mismatches(rg, r_o, ug, u_o, Wg, W_o)
    assert not bad, bad[:5]
