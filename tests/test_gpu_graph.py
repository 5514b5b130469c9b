"""The end-to-end calls can be captured into a HIP graph and replayed.

Nothing the library enqueues synchronises with the host or clears memory
with a memset, so a caller may capture dcr_resample or dcr_resample_batched
in a graph.  Each replay (with other eager work and synchronisations between
replays, and a new seed written into the captured arguments' inputs) must
equal the eager call.
"""
import numpy as np
import pytest

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


def _batch(seed=3, B=40):
    rng = np.random.Generator(np.random.PCG64(seed))
    Mb = np.maximum(1, np.rint(np.exp(rng.uniform(np.log(10), np.log(300000), B)))).astype(np.int64)
    Nb = np.maximum(1, Mb // rng.integers(1, 64, B)).astype(np.int64)
    w_off = np.concatenate([[0], np.cumsum(Mb)]).astype(np.int64)
    n_off = np.concatenate([[0], np.cumsum(Nb)]).astype(np.int64)
    return np.exp(rng.normal(0, 3, int(w_off[-1]))).astype(np.float32), w_off, n_off


def test_batched_graph_replays(dcr, dev):
    w, w_off, n_off = _batch()
    wt = torch.from_numpy(w).to(dev)
    wo = torch.from_numpy(w_off).to(dev)
    no = torch.from_numpy(n_off).to(dev)
    sumN = int(n_off[-1])
    ws = torch.empty(dcr.dcr_batched_workspace_bytes(len(w_off) - 1, w.size, sumN, 1),
                     dtype=torch.uint8, device=dev)
    r_eager = torch.empty(sumN, dtype=torch.int32, device=dev)
    r_graph = torch.empty(sumN, dtype=torch.int32, device=dev)
    st = torch.empty(1, dtype=torch.int32, device=dev)
    dcr.dcr_resample_batched(wt, wo, no, seed=11, r=r_eager, dev_status=st, ws=ws)
    torch.cuda.synchronize()
    ref = r_eager.cpu().numpy().copy()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        # warm the stream once outside capture, then capture
        dcr.dcr_resample_batched(wt, wo, no, seed=11, r=r_graph, dev_status=st, ws=ws)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            dcr.dcr_resample_batched(wt, wo, no, seed=11, r=r_graph, dev_status=st, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    for k in range(4):
        r_graph.fill_(-5)
        # eager work between replays, on the same weights and workspace
        dcr.dcr_resample_batched(wt, wo, no, seed=100 + k, r=r_eager, dev_status=st, ws=ws)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        assert np.array_equal(r_graph.cpu().numpy(), ref), f"replay {k}"


def test_single_graph_replays_new_weights(dcr, dev):
    M, N = 300000, 5000
    rng = np.random.Generator(np.random.PCG64(5))
    w1 = np.exp(rng.normal(0, 2, M))
    w2 = np.exp(rng.normal(0, 2, M))
    wt = torch.from_numpy(w1).to(dev)
    ws = torch.empty(dcr.dcr_workspace_bytes(M, N, 0), dtype=torch.uint8, device=dev)
    r = torch.empty(N, dtype=torch.int32, device=dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        dcr.dcr_resample(wt, N, 7, 0, r=r, ws=ws)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            dcr.dcr_resample(wt, N, 7, 0, r=r, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    for k, wnew in enumerate([w2, w1, w2]):
        wt.copy_(torch.from_numpy(wnew).to(dev))      # new weights in the captured buffer
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = r.cpu().numpy()
        want = dcr.dcr_resample(torch.from_numpy(wnew).to(dev), N, 7, 0).cpu().numpy()
        assert np.array_equal(got, want), f"replay {k}"
