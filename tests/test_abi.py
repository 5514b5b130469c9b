"""The C ABI library loads, exports every entry point of include/dcr.h, and
rejects bad arguments on the host before anything is enqueued (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dcr.h")
LIB = os.path.join(ROOT, "paper_2604_01356_amd", "libdcr.so")

FAKE = ctypes.c_void_p(0x7F0000000000)      # never dereferenced on the host
FAKE_UNALIGNED = ctypes.c_void_p(0x7F0000000008)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libdcr.so not built")
    import paper_2604_01356_amd as dcr
    return dcr.library()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(dcr_\w+)\s*\(",
                                 text, re.M)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ["dcr_workspace_bytes", "dcr_cumulative_weights", "dcr_sorted_uniforms",
              "dcr_inverse_cmf", "dcr_resample", "dcr_status_string",
              "dcr_batched_workspace_bytes", "dcr_resample_batched", "dcr_resample_outer"]:
        assert n in names


def test_library_exports_every_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    import paper_2604_01356_amd as dcr
    for code in range(8):
        assert dcr.dcr_status_string(code)
    assert dcr.dcr_status_string(99) == "unknown status"


def test_workspace_bytes(lib):
    import paper_2604_01356_amd as dcr
    a = dcr.dcr_workspace_bytes(1, 0)
    b = dcr.dcr_workspace_bytes(1 << 20, 1 << 12)
    c = dcr.dcr_workspace_bytes(1 << 26, 1 << 14, dcr.DCR_FP32_COMP)
    assert 0 < a < b < c
    assert c % 256 == 0
    for bad in [(0, 0), (-1, 5), (1 << 31, 1), (10, -1), (10, 1 << 31)]:
        with pytest.raises(dcr.DcrError) as e:
            dcr.dcr_workspace_bytes(*bad)
        assert e.value.code == 1
    with pytest.raises(dcr.DcrError) as e:
        dcr.dcr_workspace_bytes(10, 10, 7)
    assert e.value.code == 2


def _ws(lib, M, N):
    n = ctypes.c_size_t(0)
    assert lib.dcr_workspace_bytes(M, N, 0, ctypes.byref(n)) == 0
    return n.value


def test_host_validation_resample(lib):
    ws = _ws(lib, 1000, 100)
    f = lib.dcr_resample
    # M out of range, NULL w, NULL ws, NULL r with N > 0
    assert f(FAKE, 0, 100, 1, 0, 0, FAKE, None, None, None, FAKE, ws, None) == 1
    assert f(None, 1000, 100, 1, 0, 0, FAKE, None, None, None, FAKE, ws, None) == 1
    assert f(FAKE, 1000, 100, 1, 0, 0, FAKE, None, None, None, None, ws, None) == 1
    assert f(FAKE, 1000, 100, 1, 0, 0, None, None, None, None, FAKE, ws, None) == 1
    assert f(FAKE, 1000, -1, 1, 0, 0, FAKE, None, None, None, FAKE, ws, None) == 1
    # unknown precision, unaligned or small workspace
    assert f(FAKE, 1000, 100, 1, 0, 5, FAKE, None, None, None, FAKE, ws, None) == 2
    assert f(FAKE, 1000, 100, 1, 0, 0, FAKE, None, None, None, FAKE_UNALIGNED, ws, None) == 1
    assert f(FAKE, 1000, 100, 1, 0, 0, FAKE, None, None, None, FAKE, ws - 1, None) == 3


def test_host_validation_stages(lib):
    ws = _ws(lib, 1000, 100)
    assert lib.dcr_cumulative_weights(FAKE, 0, 0, FAKE, None, None, FAKE, ws, None) == 1
    assert lib.dcr_cumulative_weights(FAKE, 1000, 0, None, None, None, FAKE, ws, None) == 1
    assert lib.dcr_cumulative_weights(FAKE, 1000, 3, FAKE, None, None, FAKE, ws, None) == 2
    assert lib.dcr_cumulative_weights(FAKE, 1000, 0, FAKE, None, None, FAKE, 16, None) == 3
    assert lib.dcr_sorted_uniforms(-1, 1, 0, 0, FAKE, FAKE, ws, None) == 1
    assert lib.dcr_sorted_uniforms(100, 1, 0, 9, FAKE, FAKE, ws, None) == 2
    assert lib.dcr_sorted_uniforms(100, 1, 0, 0, None, FAKE, ws, None) == 1
    assert lib.dcr_sorted_uniforms(100, 1, 0, 0, FAKE, FAKE, 16, None) == 3
    assert lib.dcr_sorted_uniforms(0, 1, 0, 0, None, None, 0, None) == 0   # N = 0: no-op
    assert lib.dcr_inverse_cmf(FAKE, 0, FAKE, 10, FAKE, None, 0, None) == 1
    assert lib.dcr_inverse_cmf(None, 10, FAKE, 10, FAKE, None, 0, None) == 1
    assert lib.dcr_inverse_cmf(FAKE, 10, FAKE, 0, None, None, 0, None) == 0  # N = 0: no-op


def test_batched_workspace_bytes(lib):
    import paper_2604_01356_amd as dcr
    a = dcr.dcr_batched_workspace_bytes(1, 1, 0)
    b = dcr.dcr_batched_workspace_bytes(4096, 600_000_000, 15_000_000, dcr.DCR_FP32_COMP)
    assert 0 < a < b and b % 256 == 0
    for bad in [(0, 10, 10), (-3, 10, 10), (10, 9, 10), (10, 100, -1), (1 << 25, 1 << 26, 0),
                (4, 1 << 41, 0), (4, 100, 1 << 41)]:
        with pytest.raises(dcr.DcrError) as e:
            dcr.dcr_batched_workspace_bytes(*bad)
        assert e.value.code == 1
    with pytest.raises(dcr.DcrError) as e:
        dcr.dcr_batched_workspace_bytes(4, 100, 10, 3)
    assert e.value.code == 2


def test_host_validation_batched(lib):
    n = ctypes.c_size_t(0)
    assert lib.dcr_batched_workspace_bytes(8, 1000, 100, 1, ctypes.byref(n)) == 0
    ws = n.value
    f = lib.dcr_resample_batched
    ok = (FAKE, FAKE, FAKE, 8, 1000, 100, 1, 1, FAKE, None, None, FAKE, ws, None)

    def call(**kw):
        names = ["w", "w_off", "n_off", "B", "sumM", "sumN", "seed", "p", "r", "seg", "st",
                 "ws", "ws_bytes", "stream"]
        args = dict(zip(names, ok))
        args.update(kw)
        return f(*[args[k] for k in names])

    assert call(B=0) == 1
    assert call(sumM=7) == 1                 # fewer weights than filters
    assert call(sumN=-1) == 1
    assert call(w=None) == 1
    assert call(w_off=None) == 1
    assert call(n_off=None) == 1
    assert call(r=None) == 1                 # draws requested but no output
    assert call(ws=None) == 1
    assert call(ws=FAKE_UNALIGNED) == 1
    assert call(p=4) == 2
    assert call(ws_bytes=ws - 1) == 3
    # the tuned form rejects a map tile it is not built for, before any launch
    ex = lib.dcr_resample_batched_ex
    assert ex(FAKE, FAKE, FAKE, 8, 1000, 100, 1, 1, 100, FAKE, None, None, FAKE, ws, None) == 2
    assert ex(FAKE, FAKE, FAKE, 8, 1000, 100, 1, 1, 512, FAKE, None, None, FAKE, 16, None) == 3
    at = lib.dcr_batched_autotune
    assert at(FAKE, FAKE, FAKE, 8, 1000, 100, 1, 1, FAKE, FAKE, ws, None, None, None, None) == 1


def test_host_validation_schemes(lib):
    ws = _ws(lib, 1000, 100)
    f = lib.dcr_resample_scheme
    # every call below fails on the host, before anything is enqueued
    assert f(FAKE, 1000, 100, 1, 0, 0, 3, FAKE, None, None, None, FAKE, ws, None) == 2
    assert f(FAKE, 1000, 100, 1, 0, 0, -1, FAKE, None, None, None, FAKE, ws, None) == 2
    assert f(FAKE, 0, 100, 1, 0, 0, 1, FAKE, None, None, None, FAKE, ws, None) == 1
    assert f(FAKE, 1000, 100, 1, 0, 0, 2, FAKE, None, None, None, FAKE, 16, None) == 3
    assert f(FAKE, 1000, 100, 1, 0, 0, 1, None, None, None, None, FAKE, ws, None) == 1
    g = lib.dcr_scheme_uniforms
    assert g(10, 1, 0, 0, FAKE, None) == 2          # multinomial: use dcr_sorted_uniforms
    assert g(10, 1, 0, 5, FAKE, None) == 2
    assert g(-1, 1, 0, 1, FAKE, None) == 1
    assert g(10, 1, 0, 1, None, None) == 1
    assert g(0, 1, 0, 1, None, None) == 0           # N = 0: no-op


def test_host_validation_outer(lib):
    ws = _ws(lib, 1000, 100)
    f = lib.dcr_resample_outer
    # every call below fails on the host, before anything is enqueued
    assert f(FAKE, 0, FAKE, 10, 100, 1, 0, 0, 0, FAKE, None, None, None, FAKE, ws, None) == 1
    assert f(FAKE, 10, FAKE, 0, 100, 1, 0, 0, 0, FAKE, None, None, None, FAKE, ws, None) == 1
    assert f(None, 10, FAKE, 10, 100, 1, 0, 0, 0, FAKE, None, None, None, FAKE, ws, None) == 1
    assert f(FAKE, 10, None, 10, 100, 1, 0, 0, 0, FAKE, None, None, None, FAKE, ws, None) == 1
    assert f(FAKE, 1 << 20, FAKE, 1 << 12, 100, 1, 0, 0, 0, FAKE, None, None, None, FAKE, ws,
             None) == 1                                   # Na * P above 2^31 - 1
    assert f(FAKE, 10, FAKE, 10, 100, 1, 0, 0, 7, FAKE, None, None, None, FAKE, ws, None) == 2
    assert f(FAKE, 10, FAKE, 10, 100, 1, 0, 0, 0, FAKE, None, None, None, FAKE, 16, None) == 3


def test_host_validation_noalloc(lib):
    """The allocation-free call reports every host-visible error, the size
    check against its static scratch array included, before any HIP call."""
    f = lib.dcr_resample_noalloc
    assert f(None, 1000, 100, 1, 0, 0, 0, FAKE, None, None, None, None) == 1
    assert f(FAKE, 0, 100, 1, 0, 0, 0, FAKE, None, None, None, None) == 1
    assert f(FAKE, 1000, -1, 1, 0, 0, 0, FAKE, None, None, None, None) == 1
    assert f(FAKE, 1000, 100, 1, 0, 0, 0, None, None, None, None, None) == 1
    assert f(FAKE, 1000, 100, 1, 0, 5, 0, FAKE, None, None, None, None) == 2
    assert f(FAKE, 1000, 100, 1, 0, 0, 4, FAKE, None, None, None, None) == 2
    # more spacing blocks, or more weight blocks, than the 32 MiB array holds
    assert f(FAKE, 1000, 1 << 23, 1, 0, 0, 0, FAKE, None, None, None, None) == 4
    assert f(FAKE, (1 << 31) - 1, 10, 1, 0, 1, 0, FAKE, None, None, None, None) == 4
    # the stratified scheme has no spacing side: the same N fits
    n = ctypes.c_size_t(0)
    assert lib.dcr_workspace_bytes(1 << 20, 1 << 22, 0, ctypes.byref(n)) == 0
    assert n.value > (32 << 20)


def test_host_validation_plan(lib):
    """Plan calls refuse bad arguments before any allocation or launch."""
    h = ctypes.c_void_p(0)
    f = lib.dcr_plan_create_batched
    assert f(0, 1000, 10, 1, None, ctypes.byref(h)) == 1            # B_max < 1
    assert f(8, 4, 10, 1, None, ctypes.byref(h)) == 1               # sumM_max < B_max
    assert f(8, 1000, -1, 1, None, ctypes.byref(h)) == 1
    assert f(8, 1 << 41, 10, 1, None, ctypes.byref(h)) == 1
    assert f(8, 1000, 10, 4, None, ctypes.byref(h)) == 2            # unknown precision
    assert f(8, 1000, 10, 1, None, None) == 1                       # no output handle
    assert h.value is None
    g = lib.dcr_plan_resample_batched
    assert g(None, FAKE, FAKE, FAKE, 1, 0, FAKE, None, None, None) == 1
    assert lib.dcr_plan_destroy(None) == 1
    assert lib.dcr_plan_autotune(None, FAKE, FAKE, FAKE, 1, 0, FAKE, None, None) == 1
    c = ctypes.c_int32(0)
    assert lib.dcr_plan_map_chunk(None, ctypes.byref(c)) == 1


def test_profile_api_host(lib):
    assert lib.dcr_profile_kind_count() >= 5
    names = [lib.dcr_profile_kind_name(k).decode() for k in range(lib.dcr_profile_kind_count())]
    assert "reduce" in names and "map_fused" in names
    assert lib.dcr_profile_end(0, None, None) == 1   # not started
    assert lib.dcr_profile_begin(0) == 1


def test_package_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2604_01356_amd import _binding
    monkeypatch.setattr(_binding, "_lib", None)
    monkeypatch.setattr(_binding, "_LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _binding.library()


def test_binding_rejects_host_and_mistyped_tensors(lib):
    """The Python binding checks its tensors before any call: host tensors,
    unsupported dtypes and factors of different dtypes are refused."""
    torch = pytest.importorskip("torch")
    import paper_2604_01356_amd as dcr
    w = torch.ones(100, dtype=torch.float64)            # a host tensor
    with pytest.raises(ValueError):
        dcr.dcr_resample(w, 10, seed=1)
    with pytest.raises(ValueError):
        dcr.dcr_cumulative_weights(w)
    with pytest.raises(ValueError):
        dcr.dcr_resample_outer(torch.ones(10), torch.ones(10), 5, seed=1)
    with pytest.raises(TypeError):
        dcr.precision_of(torch.ones(10, dtype=torch.int32))
    with pytest.raises(ValueError):
        dcr.dcr_resample_batched(w, torch.zeros(2, dtype=torch.int64),
                                 torch.zeros(2, dtype=torch.int64), 1, sumN_max=1)


def test_binding_rejects_weight_bound_beyond_weights(lib, monkeypatch):
    """A sumM_max larger than w would let device-checked offsets run past the
    weights: every batched wrapper refuses it before any call."""
    torch = pytest.importorskip("torch")
    import paper_2604_01356_amd as dcr
    from paper_2604_01356_amd import _binding
    # the checks run before the tensors' device is used: stand-in device tensors
    monkeypatch.setattr(_binding, "_dev_tensor", lambda *a, **k: None)
    w = torch.ones(100, dtype=torch.float32)
    off = torch.zeros(3, dtype=torch.int64)
    for fn in (dcr.dcr_resample_batched, dcr.dcr_resample_batched_ex):
        with pytest.raises(ValueError, match="exceeds"):
            fn(w, off, off, 1, sumM_max=101, sumN_max=10)
    with pytest.raises(ValueError, match="exceeds"):
        dcr.dcr_batched_autotune(w, off, off, sumM_max=101, sumN_max=10)
