"""Stratified and systematic resampling on the GPU (dcr_resample_scheme,
dcr_scheme_uniforms) against the oracle.

- The scheme's uniforms are a closed formula in binary64, so the GPU's u must
  equal the oracle's bit for bit.
- The fused call must equal, bit for bit, stage 3 on the W of stage 1 and the
  u of dcr_scheme_uniforms, in every map regime (one finishing launch, the
  sparse map after the carry scan, the dense merge).
- Against the oracle end to end, every index mismatch is a bin-edge case.
"""
import numpy as np
import pytest

import oracle
from parity_util import classify_mismatches

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SCHEMES = {"stratified": 1, "systematic": 2}


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


@pytest.mark.parametrize("scheme", sorted(SCHEMES))
@pytest.mark.parametrize("N", [1, 2, 4095, 4096, 4097, 100003])
def test_scheme_uniforms_exact(dcr, dev, scheme, N):
    u = dcr.dcr_scheme_uniforms(N, seed=7, stream_id=5, scheme=SCHEMES[scheme], device=dev)
    torch.cuda.synchronize()
    u_o = oracle.scheme_uniforms(N, 7, 5, scheme)
    assert np.array_equal(u.cpu().numpy(), u_o)


# (M, N): the single finishing launch (sparse draws, up to 4096 weight blocks;
# 1 << 27 is exactly 4096 blocks, the largest it takes); the dense merge
# (N >= M/4); ragged sizes.  The sparse map after a separate carry scan
# (more than 4096 weight blocks) is covered in test_gpu_map_fused.py.
CASES = [(5000, 700), (1000, 1), (300000, 1000), (1 << 27, 3000), (200000, 60000),
         (100003, 262143), (65536, 65536)]


@pytest.mark.parametrize("scheme", sorted(SCHEMES))
@pytest.mark.parametrize("M,N", CASES)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_scheme_resample(dcr, dev, scheme, M, N, dtype):
    rng = np.random.Generator(np.random.PCG64(M ^ N))
    w = np.exp(rng.normal(0.0, 2.0, M)).astype(dtype)
    wt = torch.from_numpy(w).to(dev)
    sc = SCHEMES[scheme]
    W = torch.empty(M, dtype=torch.float64, device=dev)
    u = torch.empty(max(N, 1), dtype=torch.float64, device=dev)
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    r = dcr.dcr_resample_scheme(wt, N, 3, 2, sc, W_out=W, u_out=u, dev_status=st)
    r_plain = dcr.dcr_resample_scheme(wt, N, 3, 2, sc)
    W1 = dcr.dcr_cumulative_weights(wt)
    u2 = dcr.dcr_scheme_uniforms(N, 3, 2, sc, device=dev)
    r3 = dcr.dcr_inverse_cmf(W1, u2)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    r, r_plain, r3 = r.cpu().numpy(), r_plain.cpu().numpy(), r3.cpu().numpy()
    Wg, ug = W.cpu().numpy(), u[:N].cpu().numpy()
    assert np.array_equal(r, r_plain) and np.array_equal(r, r3)
    assert np.array_equal(Wg, W1.cpu().numpy()) and np.array_equal(ug, u2.cpu().numpy())
    r_o, W_o, u_o = oracle.resample_scheme(w, N, 3, 2, scheme)
    assert np.array_equal(ug, u_o)
    assert np.max(np.abs(Wg - W_o)) <= 2.0**-40
    n_mis, bad = classify_mismatches(r, r_o, ug, u_o, Wg, W_o)
    assert not bad, bad[:5]
    c = np.bincount(r, minlength=M)
    dW = np.diff(np.concatenate([[0.0], Wg]))
    bound = 1.0 if scheme == "systematic" else 2.0
    assert np.all(np.abs(c - N * dW) < bound + 1e-6)
