"""Host-side state of the library: a launch reports its own status, and the
per-launch profiler belongs to the host thread that started it."""
import ctypes
import threading

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


def _weights(M, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return torch.from_numpy(np.exp(rng.normal(0.0, 2.0, M))).to("cuda:0")


def test_earlier_hip_error_is_not_reported(dcr):
    """An unrelated failed HIP call (an invalid device number) leaves an error
    that HIP keeps until someone reads it; a resample made after it reports
    its own launches' status (DCR_OK), not that error.  The C entry point is
    called directly, and the stale error is read back afterwards so that torch
    does not trip on it."""
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipSetDevice.argtypes = [ctypes.c_int]
    hip.hipGetLastError.restype = ctypes.c_int
    lib = dcr.library()
    M, N = 100_000, 5000
    w = _weights(M, 1)
    ref = dcr.dcr_resample(w, N, seed=2)
    r = torch.full((N,), -7, dtype=torch.int32, device="cuda:0")
    ws = torch.empty(dcr.dcr_workspace_bytes(M, N, dcr.DCR_FP64), dtype=torch.uint8,
                     device="cuda:0")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert hip.hipGetLastError() == 0
    assert hip.hipSetDevice(9999) != 0          # fails on the host, harmlessly
    code = lib.dcr_resample(w.data_ptr(), M, N, 2, 0, dcr.DCR_FP64, r.data_ptr(), None, None,
                            None, ws.data_ptr(), ws.numel(), stream)
    stale = hip.hipGetLastError()               # read the earlier error back
    assert code == 0, code
    assert stale != 0
    torch.cuda.synchronize()
    assert torch.equal(r, ref)


def test_profiler_counts_only_its_own_thread(dcr):
    w = _weights(300_000, 3)
    r_other = torch.empty(20_000, dtype=torch.int32, device="cuda:0")
    stop = threading.Event()
    calls = []

    def other():
        # another host thread resampling on its own stream the whole time
        torch.cuda.set_device(0)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            while not stop.is_set():
                dcr.dcr_resample(w, 20_000, seed=5, r=r_other)
                calls.append(1)
            s.synchronize()

    th = threading.Thread(target=other)
    th.start()
    try:
        dcr.dcr_profile_begin(64)
        for k in range(3):
            dcr.dcr_resample(w, 1000, seed=k)
        prof = dcr.dcr_profile_end()
    finally:
        stop.set()
        th.join()
    torch.cuda.synchronize()
    launched = {k: v[0] for k, v in prof.items() if v[0] > 0}
    # three calls of this thread: one reduce and one finishing launch each
    assert launched == {"reduce": 3, "finish": 3}, launched
    assert len(calls) > 0
