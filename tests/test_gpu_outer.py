"""Structured weights w[i*P + k] = a[i] * b[k] formed on the fly
(dcr_resample_outer) against the same weights materialised, and the oracle.

- binary64 factors: the products are the binary64 weights a caller would
  materialise, so every output (r, W, u) equals dcr_resample on them bit for
  bit, in each map regime.
- binary32 factors: the binary64 products are exact; the draws use the
  binary32 spacings form.  r equals stage 3 on the call's own W and u, and
  agrees with the oracle on the exact products up to bin-edge cases.
"""
import numpy as np
import pytest

import oracle
from parity_util import assert_monotone_unit, classify_mismatches

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


def _factors(Na, P, seed, dtype):
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.lognormal(0.0, 1.0, Na).astype(dtype)
    b = rng.dirichlet(np.full(P, 0.5)).astype(dtype)
    return a, b


# (Na, P, N): the EnGMF step shape and a larger sparse case (both in the single
# finishing launch), a dense case (merge), ragged sizes, and the large
# EnGMF-shaped step timed beside the main measurement.  The outer twin of the
# sparse map after a separate carry scan is covered in test_gpu_map_fused.py.
CASES = [(2000, 64, 2000), (20000, 1000, 3000), (3000, 7, 20000), (1, 1, 5), (977, 33, 1),
         (65536, 256, 65536)]


@pytest.mark.parametrize("Na,P,N", CASES)
def test_outer_fp64_equals_materialised(dev, dcr, Na, P, N):
    a, b = _factors(Na, P, Na * 31 + P, np.float64)
    w = np.multiply.outer(a, b).ravel()     # binary64 products, rounded to nearest
    M = Na * P
    outs = []
    for call in ("outer", "array"):
        W = torch.empty(M, dtype=torch.float64, device=dev)
        u = torch.empty(max(N, 1), dtype=torch.float64, device=dev)
        st = torch.full((1,), -1, dtype=torch.int32, device=dev)
        if call == "outer":
            r = dcr.dcr_resample_outer(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev), N,
                                       seed=4, stream_id=1, W_out=W, u_out=u, dev_status=st)
        else:
            r = dcr.dcr_resample(torch.from_numpy(w).to(dev), N, seed=4, stream_id=1, W_out=W,
                                 u_out=u, dev_status=st)
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        outs.append((r.cpu().numpy(), W.cpu().numpy(), u[:N].cpu().numpy()))
    for x, y in zip(outs[0], outs[1]):
        assert np.array_equal(x, y)
    r_o, W_o, u_o = oracle.resample(w, N, 4, 1)
    n_mis, bad = classify_mismatches(outs[0][0], r_o, outs[0][2], u_o, outs[0][1], W_o)
    assert not bad


@pytest.mark.parametrize("Na,P,N", CASES)
def test_outer_fp32_against_oracle(dev, dcr, Na, P, N):
    a, b = _factors(Na, P, Na * 7 + P, np.float32)
    M = Na * P
    W = torch.empty(M, dtype=torch.float64, device=dev)
    u = torch.empty(max(N, 1), dtype=torch.float64, device=dev)
    r = dcr.dcr_resample_outer(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev), N,
                               seed=9, stream_id=0, W_out=W, u_out=u)
    r_plain = dcr.dcr_resample_outer(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev), N,
                                     seed=9, stream_id=0)
    r3 = dcr.dcr_inverse_cmf(W, u[:N])
    torch.cuda.synchronize()
    rg, Wg, ug = r.cpu().numpy(), W.cpu().numpy(), u[:N].cpu().numpy()
    assert np.array_equal(rg, r_plain.cpu().numpy()) and np.array_equal(rg, r3.cpu().numpy())
    assert_monotone_unit(Wg)
    # exact binary64 products of the binary32 factors, binary32 spacings
    w = np.multiply.outer(a.astype(np.float64), b.astype(np.float64)).ravel()
    r_o, W_o, u_o = oracle.resample(w, N, 9, 0, zkind=1)
    assert np.max(np.abs(Wg - W_o)) <= 2.0**-40
    assert np.max(np.abs(ug - u_o)) <= 2.0**-21 if N else True
    n_mis, bad = classify_mismatches(rg, r_o, ug, u_o, Wg, W_o)
    assert not bad


def test_outer_schemes_and_bad_factor(dev, dcr):
    a, b = _factors(500, 40, 5, np.float64)
    w = np.multiply.outer(a, b).ravel()
    wt = torch.from_numpy(w).to(dev)
    at, bt = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    for scheme in (dcr.DCR_STRATIFIED, dcr.DCR_SYSTEMATIC):
        r1 = dcr.dcr_resample_outer(at, bt, 3000, 2, 0, scheme)
        r2 = dcr.dcr_resample_scheme(wt, 3000, 2, 0, scheme)
        torch.cuda.synchronize()
        assert np.array_equal(r1.cpu().numpy(), r2.cpu().numpy())
    a_bad = a.copy()
    a_bad[17] = -1.0
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    r = dcr.dcr_resample_outer(torch.from_numpy(a_bad).to(dev), bt, 100, 1, dev_status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 6 and bool((r == -1).all())
