"""Batched plans (dcr_plan_*): the plan's graph against the stateless batched
call and the oracle.

A plan resamples with its own workspace and a HIP graph of the four batched
launches, whose arguments each call rewrites.  Every plan call must equal
dcr_resample_batched_ex with the plan's map tile bit for bit; the binary64
form must equal the oracle's batched result (Alg. 5 per filter, Philox stream
id b) exactly.  Calls with new weights in the same buffers, new buffers, a
smaller B, several calls in flight without a wait, a change of map tile and a
capacity overflow are covered.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dcr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_01356_amd as m
    m.library()
    return m


def _batch(seed, B, dtype, m_hi=300_000):
    rng = np.random.Generator(np.random.PCG64(seed))
    Mb = np.maximum(1, np.rint(np.exp(rng.uniform(0.0, np.log(m_hi), B)))).astype(np.int64)
    Nb = np.maximum(1, Mb // rng.integers(1, 64, B)).astype(np.int64)
    Nb[::7] = 0
    w_off = np.concatenate([[0], np.cumsum(Mb)]).astype(np.int64)
    n_off = np.concatenate([[0], np.cumsum(Nb)]).astype(np.int64)
    w = np.exp(rng.normal(0.0, 3.0, int(w_off[-1]))).astype(dtype)
    return w, w_off, n_off


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _eager(dcr, w, wo, no, seed, chunk, sumM, sumN):
    r = torch.full((sumN,), -7, dtype=torch.int32, device="cuda:0")
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
    dcr.dcr_resample_batched_ex(w, wo, no, seed, chunk=chunk, sumM_max=sumM, sumN_max=sumN,
                                r=r, dev_status=st)
    return r, st


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_plan_replays_equal_eager_and_oracle(dcr, dtype):
    B_max, sumM, sumN = 64, 6_000_000, 600_000
    prec = dcr.DCR_FP64 if dtype == np.float64 else dcr.DCR_FP32_COMP
    plan = dcr.dcr_plan_create_batched(B_max, sumM, sumN, prec)
    try:
        chunk = dcr.dcr_plan_map_chunk(plan)
        w, w_off, n_off = _batch(5, 48, dtype)
        assert w_off[-1] <= sumM and n_off[-1] <= sumN
        wt = torch.zeros(sumM, dtype=torch.from_numpy(w[:1]).dtype, device="cuda:0")
        wt[: w.size] = _dev(w)
        wo, no = _dev(w_off), _dev(n_off)
        rs = [torch.full((sumN,), -7, dtype=torch.int32, device="cuda:0") for _ in range(4)]
        st = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
        seg = torch.full((48,), -1, dtype=torch.int32, device="cuda:0")
        # four calls in flight (two graph instances, each rewritten while the
        # other may run), each into its own output, then new weights in the
        # same buffer
        print(f"  plan: {np.dtype(dtype).name} B=48 four calls without a wait", flush=True)
        for k in range(4):
            dcr.dcr_plan_resample_batched(plan, wt, wo, no, 100 + k, rs[k], seg, st)
        torch.cuda.synchronize()
        assert int(st.item()) == 0 and bool((seg == 0).all())
        nN = int(n_off[-1])
        for k in range(4):
            ref, st_e = _eager(dcr, wt, wo, no, 100 + k, chunk, sumM, sumN)
            torch.cuda.synchronize()
            assert int(st_e.item()) == 0
            assert torch.equal(rs[k][:nN], ref[:nN]), k
        if dtype == np.float64:
            r_o = oracle.resample_batched(w, w_off, n_off, 102)
            assert np.array_equal(rs[2][:nN].cpu().numpy(), r_o)
        # new weights written into the same buffer
        w2, _, _ = _batch(6, 48, dtype)
        w2 = w2[: w.size] if w2.size >= w.size else np.resize(w2, w.size)
        wt[: w.size] = _dev(w2)
        dcr.dcr_plan_resample_batched(plan, wt, wo, no, 7, rs[0], None, st)
        ref, _ = _eager(dcr, wt, wo, no, 7, chunk, sumM, sumN)
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        assert torch.equal(rs[0][:nN], ref[:nN])
        if dtype == np.float64:
            assert np.array_equal(rs[0][:nN].cpu().numpy(),
                                  oracle.resample_batched(w2, w_off, n_off, 7))
    finally:
        dcr.dcr_plan_destroy(plan)


def test_plan_new_buffers_smaller_batch_and_tile_change(dcr):
    B_max, sumM, sumN = 40, 4_000_000, 400_000
    plan = dcr.dcr_plan_create_batched(B_max, sumM, sumN, dcr.DCR_FP32_COMP)
    try:
        for k, (seed, B) in enumerate(((11, 40), (12, 9), (13, 1), (14, 33))):
            w, w_off, n_off = _batch(seed, B, np.float32, m_hi=90_000)
            wt, wo, no = _dev(w), _dev(w_off), _dev(n_off)
            r = torch.full((sumN,), -7, dtype=torch.int32, device="cuda:0")
            st = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
            print(f"  plan: new buffers B={B} call {k}", flush=True)
            dcr.dcr_plan_resample_batched(plan, wt, wo, no, seed, r, None, st)
            chunk = dcr.dcr_plan_map_chunk(plan)
            ref, _ = _eager(dcr, wt, wo, no, seed, chunk, int(w.size), sumN)
            torch.cuda.synchronize()
            assert int(st.item()) == 0
            nN = int(n_off[-1])
            assert torch.equal(r[:nN], ref[:nN])
            if k == 1:
                # the autotuner picks a tile; the graphs are rebuilt for it
                ms = dcr.dcr_plan_autotune(plan, wt, wo, no, r, seed=0)
                assert ms > 0 and dcr.dcr_plan_map_chunk(plan) in (256, 512, 1024)
    finally:
        dcr.dcr_plan_destroy(plan)


def test_plan_tune_cache_and_capacity(dcr, tmp_path):
    cache = tmp_path / "tune.txt"
    B_max, sumM, sumN = 16, 500_000, 20_000
    cache.write_text(f"{B_max} {sumM} {sumN} 1 1024 0.5\n")
    plan = dcr.dcr_plan_create_batched(B_max, sumM, sumN, dcr.DCR_FP32_COMP, tune_cache=cache)
    try:
        assert dcr.dcr_plan_map_chunk(plan) == 1024
        # offsets whose draws exceed the plan's capacity
        w, w_off, n_off = _batch(21, 16, np.float32, m_hi=30_000)
        n_off = n_off.copy()
        n_off[1:] += sumN
        r = torch.full((2 * sumN + 16,), -7, dtype=torch.int32, device="cuda:0")
        st = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
        dcr.dcr_plan_resample_batched(plan, _dev(w), _dev(w_off), _dev(n_off), 1, r, None, st)
        torch.cuda.synchronize()
        assert int(st.item()) == 4
        assert bool((r == -7).all())
        # the autotuner appends its choice under the plan's shape
        w, w_off, n_off = _batch(22, 16, np.float32, m_hi=30_000)
        dcr.dcr_plan_autotune(plan, _dev(w), _dev(w_off), _dev(n_off), r)
        lines = cache.read_text().strip().splitlines()
        assert len(lines) == 2 and lines[1].split()[:4] == [str(B_max), str(sumM), str(sumN), "1"]
    finally:
        dcr.dcr_plan_destroy(plan)
