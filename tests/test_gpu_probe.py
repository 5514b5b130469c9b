"""The bandwidth reference kernels (measurement only) move the bytes they
claim: the copy reproduces its source, the read sums it."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_stream_probe_copy_and_read():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_01356_amd as dcr
    n = (1 << 20) + 12                      # a ragged tail beyond the unrolled loop
    src = torch.arange(n, dtype=torch.float32, device="cuda:0") % 7
    dst = torch.empty_like(src)
    for unroll in (4, 8, 16):
        dst.zero_()
        dcr.dcr_stream_probe(1, src, dst, 96, unroll)
        part = torch.zeros(96, dtype=torch.float32, device="cuda:0")
        dcr.dcr_stream_probe(0, src, part, 96, unroll)
        part2 = torch.zeros(96, dtype=torch.float32, device="cuda:0")
        dcr.dcr_stream_probe(2, src, part2, 96, unroll)   # 96 runs, the last one shorter
        torch.cuda.synchronize()
        assert torch.equal(dst, src)
        assert float(part.double().sum()) == float(src.double().sum())
        assert float(part2.double().sum()) == float(src.double().sum())
    with pytest.raises(dcr.DcrError):
        dcr.dcr_stream_probe(3, src, dst, 96)
