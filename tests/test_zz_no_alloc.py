"""The allocation-free entry point (dcr_resample_noalloc) against the
workspace entry point it varies (dcr_resample_scheme), through the C ABI.

Both run the same kernels, so the indices, W and u must agree bit for bit.
Two calls follow each other on the one static scratch array of the device,
the second with a smaller problem, so that what the first call left in the
array cannot leak into the second.  The end-to-end map is Sec. III, Alg. 5.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dcr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_01356_amd as m
    m.library()
    return m


def _weights(M, seed, sigma, dtype):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.exp(rng.normal(0.0, sigma, M)).astype(dtype)


def _both(dcr, w, N, seed, stream, scheme):
    dev = w.device
    M = w.numel()
    outs = []
    for call in ("noalloc", "workspace"):
        r = torch.full((max(N, 1),), -7, dtype=torch.int32, device=dev)
        W = torch.empty(M, dtype=torch.float64, device=dev)
        u = torch.empty(max(N, 1), dtype=torch.float64, device=dev)
        st = torch.full((1,), -1, dtype=torch.int32, device=dev)
        if call == "noalloc":
            dcr.dcr_resample_noalloc(w, N, seed, stream, scheme, r=r, W_out=W, u_out=u,
                                     dev_status=st)
        else:
            dcr.dcr_resample_scheme(w, N, seed, stream, scheme, r=r, W_out=W, u_out=u,
                                    dev_status=st)
        outs.append((r[:N], W, u[:N], st))
    torch.cuda.synchronize()
    (r1, W1, u1, s1), (r2, W2, u2, s2) = outs
    assert int(s1.item()) == 0 and int(s2.item()) == 0
    assert torch.equal(r1, r2)
    assert torch.equal(W1, W2)
    assert torch.equal(u1, u2)
    return r1


# (M, N) pairs: the first call of each case is the larger one.  They cover the
# single finishing launch (sparse draws), the separate carry scan with the
# dense map (N * 4 >= M) and the largest spacing count the array holds.
CASES = [
    ((300_000, 5_000), (70_001, 1_234)),
    ((1 << 21, 1 << 21), (40_000, 39_999)),
    ((5_000_000, 3_000_000), (1 << 20, 300_000)),
]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("big,small", CASES)
def test_two_calls_second_smaller(dcr, dtype, big, small):
    dev = torch.device("cuda:0")
    for k, (M, N) in enumerate((big, small)):
        print(f"  noalloc vs workspace: M={M} N={N} {np.dtype(dtype).name} call {k + 1}",
              flush=True)
        w = torch.from_numpy(_weights(M, M + k, 3.0, dtype)).to(dev)
        r = _both(dcr, w, N, seed=11 + k, stream=k, scheme=dcr.DCR_MULTINOMIAL)
        assert r.numel() == N and bool((r[1:] >= r[:-1]).all())


@pytest.mark.parametrize("scheme", [1, 2])
def test_schemes_two_calls(dcr, scheme):
    dev = torch.device("cuda:0")
    for k, (M, N) in enumerate(((1 << 20, 200_000), (3_000, 2_999))):
        print(f"  noalloc scheme {scheme}: M={M} N={N} call {k + 1}", flush=True)
        w = torch.from_numpy(_weights(M, 5 * M + k, 2.0, np.float32)).to(dev)
        _both(dcr, w, N, seed=3, stream=k, scheme=scheme)


def test_capacity_and_arguments(dcr):
    dev = torch.device("cuda:0")
    w = torch.ones(1000, dtype=torch.float64, device=dev)
    # a spacing side larger than the static array
    with pytest.raises(dcr.DcrError) as e:
        dcr.dcr_resample_noalloc(w, 1 << 23, 0, r=torch.empty(1 << 23, dtype=torch.int32,
                                                              device=dev))
    assert e.value.code == 4
    # N = 0 draws nothing and succeeds
    r = dcr.dcr_resample_noalloc(w, 0, 0)
    torch.cuda.synchronize()
    assert r.numel() == 0
