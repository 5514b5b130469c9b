"""ctypes marshalling for libdcr.so (declarations in include/dcr.h).

Device arrays are torch tensors on a HIP device; their data pointers and the
current stream of their device are handed to the C ABI unchanged.  Nothing
here computes any part of the resampling.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libdcr.so")
_lib = None

DCR_FP64 = 0
DCR_FP32_COMP = 1

STATUS = {
    0: "DCR_OK",
    1: "DCR_ERR_INVALID_ARGUMENT",
    2: "DCR_ERR_UNSUPPORTED",
    3: "DCR_ERR_WORKSPACE_TOO_SMALL",
    4: "DCR_ERR_CAPACITY_EXCEEDED",
    5: "DCR_ERR_HIP",
    6: "DCR_ERR_BAD_WEIGHTS",
    7: "DCR_ERR_INTERNAL",
}


class DcrError(RuntimeError):
    def __init__(self, where: str, code: int):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)} ({_status_text(code)})")


def library_path() -> str:
    return _LIB_PATH


def library():
    """Load libdcr.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(
            f"{_LIB_PATH} is not built; run `python paper_2604_01356_amd/build.py`")
    lib = ctypes.CDLL(_LIB_PATH)
    P, i64, u64, i32, sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32,
                            ctypes.c_size_t)
    lib.dcr_status_string.argtypes = [ctypes.c_int]
    lib.dcr_status_string.restype = ctypes.c_char_p
    lib.dcr_workspace_bytes.argtypes = [i64, i64, ctypes.c_int, ctypes.POINTER(sz)]
    lib.dcr_workspace_bytes.restype = ctypes.c_int
    lib.dcr_cumulative_weights.argtypes = [P, i64, ctypes.c_int, P, P, P, P, sz, P]
    lib.dcr_cumulative_weights.restype = ctypes.c_int
    lib.dcr_sorted_uniforms.argtypes = [i64, u64, u64, ctypes.c_int, P, P, sz, P]
    lib.dcr_sorted_uniforms.restype = ctypes.c_int
    lib.dcr_inverse_cmf.argtypes = [P, i64, P, i64, P, P, sz, P]
    lib.dcr_inverse_cmf.restype = ctypes.c_int
    lib.dcr_resample.argtypes = [P, i64, i64, u64, u64, ctypes.c_int, P, P, P, P, P, sz, P]
    lib.dcr_resample.restype = ctypes.c_int
    lib.dcr_batched_workspace_bytes.argtypes = [i32, i64, i64, ctypes.c_int, ctypes.POINTER(sz)]
    lib.dcr_batched_workspace_bytes.restype = ctypes.c_int
    lib.dcr_resample_batched.argtypes = [P, P, P, i32, i64, i64, u64, ctypes.c_int, P, P, P, P,
                                         sz, P]
    lib.dcr_resample_batched.restype = ctypes.c_int
    lib.dcr_resample_batched_ex.argtypes = [P, P, P, i32, i64, i64, u64, ctypes.c_int, i32, P, P,
                                            P, P, sz, P]
    lib.dcr_resample_batched_ex.restype = ctypes.c_int
    lib.dcr_batched_autotune.argtypes = [P, P, P, i32, i64, i64, u64, ctypes.c_int, P, P, sz,
                                         ctypes.c_char_p, P, P, P]
    lib.dcr_batched_autotune.restype = ctypes.c_int
    lib.dcr_resample_scheme.argtypes = [P, i64, i64, u64, u64, ctypes.c_int, ctypes.c_int, P, P,
                                        P, P, P, sz, P]
    lib.dcr_resample_scheme.restype = ctypes.c_int
    lib.dcr_resample_outer.argtypes = [P, i64, P, i64, i64, u64, u64, ctypes.c_int, ctypes.c_int,
                                       P, P, P, P, P, sz, P]
    lib.dcr_resample_outer.restype = ctypes.c_int
    lib.dcr_scheme_uniforms.argtypes = [i64, u64, u64, ctypes.c_int, P, P]
    lib.dcr_scheme_uniforms.restype = ctypes.c_int
    lib.dcr_resample_noalloc.argtypes = [P, i64, i64, u64, u64, ctypes.c_int, ctypes.c_int, P, P,
                                         P, P, P]
    lib.dcr_resample_noalloc.restype = ctypes.c_int
    lib.dcr_plan_create_batched.argtypes = [i32, i64, i64, ctypes.c_int, ctypes.c_char_p, P]
    lib.dcr_plan_create_batched.restype = ctypes.c_int
    lib.dcr_plan_resample_batched.argtypes = [P, P, P, P, i32, u64, P, P, P, P]
    lib.dcr_plan_resample_batched.restype = ctypes.c_int
    lib.dcr_plan_autotune.argtypes = [P, P, P, P, i32, u64, P, P, P]
    lib.dcr_plan_autotune.restype = ctypes.c_int
    lib.dcr_plan_map_chunk.argtypes = [P, P]
    lib.dcr_plan_map_chunk.restype = ctypes.c_int
    lib.dcr_plan_destroy.argtypes = [P]
    lib.dcr_plan_destroy.restype = ctypes.c_int
    lib.dcr_stream_probe.argtypes = [i32, i32, P, P, sz, i32, P]
    lib.dcr_stream_probe.restype = ctypes.c_int
    lib.dcr_profile_begin.argtypes = [i32]
    lib.dcr_profile_begin.restype = ctypes.c_int
    lib.dcr_profile_end.argtypes = [i32, P, P]
    lib.dcr_profile_end.restype = ctypes.c_int
    lib.dcr_profile_kind_count.argtypes = []
    lib.dcr_profile_kind_count.restype = i32
    lib.dcr_profile_kind_name.argtypes = [i32]
    lib.dcr_profile_kind_name.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _status_text(code: int) -> str:
    try:
        return library().dcr_status_string(int(code)).decode()
    except Exception:  # pragma: no cover - library missing while formatting an error
        return ""


def _check(where: str, code: int):
    if code != 0:
        raise DcrError(where, code)


def dcr_status_string(code: int) -> str:
    return library().dcr_status_string(int(code)).decode()


def precision_of(w) -> int:
    import torch
    if w.dtype == torch.float64:
        return DCR_FP64
    if w.dtype == torch.float32:
        return DCR_FP32_COMP
    raise TypeError(f"weights must be float64 or float32, got {w.dtype}")


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev_tensor(t, name, dtype=None, numel=None):
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {numel}")


def dcr_workspace_bytes(M: int, N: int, precision: int = DCR_FP64) -> int:
    out = ctypes.c_size_t(0)
    _check("dcr_workspace_bytes",
           library().dcr_workspace_bytes(int(M), int(N), int(precision), ctypes.byref(out)))
    return int(out.value)


def _workspace(ws, M, N, precision, device):
    import torch
    need = dcr_workspace_bytes(M, N, precision)
    if ws is None:
        return torch.empty(max(need, 256), dtype=torch.uint8, device=device)
    _dev_tensor(ws, "ws")
    return ws


def dcr_cumulative_weights(w, W=None, total=None, dev_status=None, ws=None):
    """Stage 1: normalised cumulative weights of w (float64 or float32)."""
    import torch
    _dev_tensor(w, "w")
    M = w.numel()
    p = precision_of(w)
    if W is None:
        W = torch.empty(M, dtype=torch.float64, device=w.device)
    _dev_tensor(W, "W", torch.float64, M)
    _dev_tensor(total, "total", torch.float64, 1)
    _dev_tensor(dev_status, "dev_status", torch.int32, 1)
    ws = _workspace(ws, M, 0, p, w.device)
    _check("dcr_cumulative_weights", library().dcr_cumulative_weights(
        _ptr(w), M, p, _ptr(W), _ptr(total), _ptr(dev_status), _ptr(ws), ws.numel(),
        _stream(w.device)))
    return W


def dcr_sorted_uniforms(N: int, seed: int, stream_id: int = 0, precision: int = DCR_FP64,
                        u=None, ws=None, device="cuda"):
    """Stage 2: N sorted uniforms of (seed, stream_id)."""
    import torch
    if u is None:
        u = torch.empty(max(int(N), 1), dtype=torch.float64, device=device)
    _dev_tensor(u, "u", torch.float64, int(N))
    ws = _workspace(ws, 1, N, precision, u.device)
    _check("dcr_sorted_uniforms", library().dcr_sorted_uniforms(
        int(N), int(seed), int(stream_id), int(precision), _ptr(u), _ptr(ws), ws.numel(),
        _stream(u.device)))
    return u[: int(N)]


def dcr_inverse_cmf(W, u, r=None):
    """Stage 3: r_i = first j with W_j >= u_i (clamped to M-1)."""
    import torch
    _dev_tensor(W, "W", torch.float64)
    _dev_tensor(u, "u", torch.float64)
    N = u.numel()
    if r is None:
        r = torch.empty(max(N, 1), dtype=torch.int32, device=u.device)
    _dev_tensor(r, "r", torch.int32, N)
    _check("dcr_inverse_cmf", library().dcr_inverse_cmf(
        _ptr(W), W.numel(), _ptr(u), N, _ptr(r), None, 0, _stream(u.device)))
    return r[:N]


DCR_MULTINOMIAL = 0
DCR_STRATIFIED = 1
DCR_SYSTEMATIC = 2


def dcr_resample_scheme(w, N: int, seed: int, stream_id: int = 0, scheme: int = DCR_MULTINOMIAL,
                        r=None, W_out=None, u_out=None, dev_status=None, ws=None):
    """End to end with the scheme's sorted uniforms (multinomial, stratified, systematic)."""
    import torch
    _dev_tensor(w, "w")
    M = w.numel()
    p = precision_of(w)
    N = int(N)
    if r is None:
        r = torch.empty(max(N, 1), dtype=torch.int32, device=w.device)
    _dev_tensor(r, "r", torch.int32, N)
    _dev_tensor(W_out, "W_out", torch.float64, M)
    _dev_tensor(u_out, "u_out", torch.float64, N)
    _dev_tensor(dev_status, "dev_status", torch.int32, 1)
    ws = _workspace(ws, M, N, p, w.device)
    _check("dcr_resample_scheme", library().dcr_resample_scheme(
        _ptr(w), M, N, int(seed), int(stream_id), p, int(scheme), _ptr(r), _ptr(W_out),
        _ptr(u_out), _ptr(dev_status), _ptr(ws), ws.numel(), _stream(w.device)))
    return r[:N]


def dcr_resample_outer(a, b, N: int, seed: int, stream_id: int = 0,
                       scheme: int = DCR_MULTINOMIAL, r=None, W_out=None, u_out=None,
                       dev_status=None, ws=None):
    """End to end on the weights w[i*P + k] = a[i] * b[k] (a, b both float64 or
    both float32), formed on the fly."""
    import torch
    _dev_tensor(a, "a")
    _dev_tensor(b, "b")
    if a.dtype != b.dtype:
        raise TypeError("a and b must have the same dtype")
    if a.device != b.device:
        raise ValueError("a and b must be on the same device")
    p = precision_of(a)
    Na, P = a.numel(), b.numel()
    M = Na * P
    N = int(N)
    if r is None:
        r = torch.empty(max(N, 1), dtype=torch.int32, device=a.device)
    _dev_tensor(r, "r", torch.int32, N)
    _dev_tensor(W_out, "W_out", torch.float64, M)
    _dev_tensor(u_out, "u_out", torch.float64, N)
    _dev_tensor(dev_status, "dev_status", torch.int32, 1)
    ws = _workspace(ws, M, N, p, a.device)
    _check("dcr_resample_outer", library().dcr_resample_outer(
        _ptr(a), Na, _ptr(b), P, N, int(seed), int(stream_id), p, int(scheme), _ptr(r),
        _ptr(W_out), _ptr(u_out), _ptr(dev_status), _ptr(ws), ws.numel(), _stream(a.device)))
    return r[:N]


def dcr_scheme_uniforms(N: int, seed: int, stream_id: int = 0, scheme: int = DCR_STRATIFIED,
                        u=None, device="cuda"):
    """The stratified or systematic scheme's N sorted uniforms."""
    import torch
    if u is None:
        u = torch.empty(max(int(N), 1), dtype=torch.float64, device=device)
    _dev_tensor(u, "u", torch.float64, int(N))
    _check("dcr_scheme_uniforms", library().dcr_scheme_uniforms(
        int(N), int(seed), int(stream_id), int(scheme), _ptr(u), _stream(u.device)))
    return u[: int(N)]


def dcr_resample(w, N: int, seed: int, stream_id: int = 0, r=None, W_out=None, u_out=None,
                 dev_status=None, ws=None):
    """End to end: N indices drawn from the weights w (float64 or float32)."""
    import torch
    _dev_tensor(w, "w")
    M = w.numel()
    p = precision_of(w)
    N = int(N)
    if r is None:
        r = torch.empty(max(N, 1), dtype=torch.int32, device=w.device)
    _dev_tensor(r, "r", torch.int32, N)
    _dev_tensor(W_out, "W_out", torch.float64, M)
    _dev_tensor(u_out, "u_out", torch.float64, N)
    _dev_tensor(dev_status, "dev_status", torch.int32, 1)
    ws = _workspace(ws, M, N, p, w.device)
    _check("dcr_resample", library().dcr_resample(
        _ptr(w), M, N, int(seed), int(stream_id), p, _ptr(r), _ptr(W_out), _ptr(u_out),
        _ptr(dev_status), _ptr(ws), ws.numel(), _stream(w.device)))
    return r[:N]


def dcr_resample_noalloc(w, N: int, seed: int, stream_id: int = 0,
                         scheme: int = DCR_MULTINOMIAL, r=None, W_out=None, u_out=None,
                         dev_status=None):
    """dcr_resample_scheme with no workspace argument: the library's static
    scratch array of the current device serves instead (the C call allocates
    nothing; a caller that cannot allocate passes r)."""
    import torch
    _dev_tensor(w, "w")
    M = w.numel()
    p = precision_of(w)
    N = int(N)
    if r is None:
        r = torch.empty(max(N, 1), dtype=torch.int32, device=w.device)
    _dev_tensor(r, "r", torch.int32, N)
    _dev_tensor(W_out, "W_out", torch.float64, M)
    _dev_tensor(u_out, "u_out", torch.float64, N)
    _dev_tensor(dev_status, "dev_status", torch.int32, 1)
    with torch.cuda.device(w.device):
        code = library().dcr_resample_noalloc(
            _ptr(w), M, N, int(seed), int(stream_id), p, int(scheme), _ptr(r), _ptr(W_out),
            _ptr(u_out), _ptr(dev_status), _stream(w.device))
    _check("dcr_resample_noalloc", code)
    return r[:N]


def dcr_batched_workspace_bytes(B: int, sumM_max: int, sumN_max: int,
                                precision: int = DCR_FP64) -> int:
    out = ctypes.c_size_t(0)
    _check("dcr_batched_workspace_bytes", library().dcr_batched_workspace_bytes(
        int(B), int(sumM_max), int(sumN_max), int(precision), ctypes.byref(out)))
    return int(out.value)


def _batched_args(w, w_off, n_off, sumM_max, sumN_max, r, seg_status, dev_status, ws):
    import torch
    _dev_tensor(w, "w")
    _dev_tensor(w_off, "w_off", torch.int64)
    _dev_tensor(n_off, "n_off", torch.int64)
    B = w_off.numel() - 1
    if n_off.numel() != B + 1:
        raise ValueError("w_off and n_off must have the same length")
    p = precision_of(w)
    sumM = int(w.numel() if sumM_max is None else sumM_max)
    if sumM > w.numel():
        # the device checks the offsets against sumM only: a bound beyond the
        # weights would let them run past the array
        raise ValueError(f"sumM_max = {sumM} exceeds the {w.numel()} weights of w")
    if r is None:
        if sumN_max is None:
            raise ValueError("give r or sumN_max")
        r = torch.empty(max(int(sumN_max), 1), dtype=torch.int32, device=w.device)
    sumN = int(r.numel() if sumN_max is None else sumN_max)
    _dev_tensor(r, "r", torch.int32, sumN)
    _dev_tensor(seg_status, "seg_status", torch.int32, B)
    _dev_tensor(dev_status, "dev_status", torch.int32, 1)
    need = dcr_batched_workspace_bytes(B, sumM, sumN, p)
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=w.device)
    _dev_tensor(ws, "ws")
    return B, p, sumM, sumN, r, ws


def dcr_resample_batched_ex(w, w_off, n_off, seed: int, chunk: int = 0,
                            sumM_max: int | None = None, sumN_max: int | None = None, r=None,
                            seg_status=None, dev_status=None, ws=None):
    """dcr_resample_batched with `chunk` draws per map workgroup (256, 512, 1024; 0: default)."""
    B, p, sumM, sumN, r, ws = _batched_args(w, w_off, n_off, sumM_max, sumN_max, r, seg_status,
                                            dev_status, ws)
    _check("dcr_resample_batched_ex", library().dcr_resample_batched_ex(
        _ptr(w), _ptr(w_off), _ptr(n_off), B, sumM, sumN, int(seed), p, int(chunk), _ptr(r),
        _ptr(seg_status), _ptr(dev_status), _ptr(ws), ws.numel(), _stream(w.device)))
    return r


def dcr_batched_autotune(w, w_off, n_off, seed: int = 0, sumM_max: int | None = None,
                         sumN_max: int | None = None, r=None, ws=None, cache_path=None):
    """Fastest map chunk for this batch: returns (chunk, ms per call, -1 if cached)."""
    B, p, sumM, sumN, r, ws = _batched_args(w, w_off, n_off, sumM_max, sumN_max, r, None, None,
                                            ws)
    best = ctypes.c_int32(0)
    ms = ctypes.c_float(0.0)
    _check("dcr_batched_autotune", library().dcr_batched_autotune(
        _ptr(w), _ptr(w_off), _ptr(n_off), B, sumM, sumN, int(seed), p, _ptr(r), _ptr(ws),
        ws.numel(), None if cache_path is None else str(cache_path).encode(),
        ctypes.addressof(best), ctypes.addressof(ms), _stream(w.device)))
    return int(best.value), float(ms.value)


def dcr_resample_batched(w, w_off, n_off, seed: int, sumM_max: int | None = None,
                         sumN_max: int | None = None, r=None, seg_status=None, dev_status=None,
                         ws=None):
    """B filters in one call; w_off / n_off are int64 device tensors of B+1
    offsets.  sumM_max / sumN_max bound the totals (default: the size of w and
    of r; sumM_max may not exceed the size of w).  Returns r (indices local to
    each filter)."""
    B, p, sumM, sumN, r, ws = _batched_args(w, w_off, n_off, sumM_max, sumN_max, r, seg_status,
                                            dev_status, ws)
    _check("dcr_resample_batched", library().dcr_resample_batched(
        _ptr(w), _ptr(w_off), _ptr(n_off), B, sumM, sumN, int(seed), p, _ptr(r),
        _ptr(seg_status), _ptr(dev_status), _ptr(ws), ws.numel(), _stream(w.device)))
    return r


def dcr_plan_create_batched(B_max: int, sumM_max: int, sumN_max: int,
                            precision: int = DCR_FP32_COMP, tune_cache=None) -> int:
    """A batched plan on the current device (its workspace and graph); returns
    the handle, to be released with dcr_plan_destroy."""
    h = ctypes.c_void_p(0)
    _check("dcr_plan_create_batched", library().dcr_plan_create_batched(
        int(B_max), int(sumM_max), int(sumN_max), int(precision),
        None if tune_cache is None else str(tune_cache).encode(), ctypes.byref(h)))
    return int(h.value)


def _plan_args(w, w_off, n_off, r, seg_status, dev_status):
    import torch
    _dev_tensor(w, "w")
    _dev_tensor(w_off, "w_off", torch.int64)
    _dev_tensor(n_off, "n_off", torch.int64)
    B = w_off.numel() - 1
    if n_off.numel() != B + 1:
        raise ValueError("w_off and n_off must have the same length")
    _dev_tensor(r, "r", torch.int32)
    _dev_tensor(seg_status, "seg_status", torch.int32, B)
    _dev_tensor(dev_status, "dev_status", torch.int32, 1)
    return B


def dcr_plan_resample_batched(plan: int, w, w_off, n_off, seed: int, r, seg_status=None,
                              dev_status=None):
    """B filters with the plan's workspace, map tile and graph (r: int32
    device tensor holding at least the plan's sumN_max draws)."""
    B = _plan_args(w, w_off, n_off, r, seg_status, dev_status)
    with __import__("torch").cuda.device(w.device):
        code = library().dcr_plan_resample_batched(
            ctypes.c_void_p(plan), _ptr(w), _ptr(w_off), _ptr(n_off), B, int(seed), _ptr(r),
            _ptr(seg_status), _ptr(dev_status), _stream(w.device))
    _check("dcr_plan_resample_batched", code)
    return r


def dcr_plan_autotune(plan: int, w, w_off, n_off, r, seed: int = 0) -> float:
    """Times the map tiles on this batch and keeps the fastest in the plan;
    returns its milliseconds per call."""
    B = _plan_args(w, w_off, n_off, r, None, None)
    ms = ctypes.c_float(0.0)
    with __import__("torch").cuda.device(w.device):
        code = library().dcr_plan_autotune(
            ctypes.c_void_p(plan), _ptr(w), _ptr(w_off), _ptr(n_off), B, int(seed), _ptr(r),
            ctypes.addressof(ms), _stream(w.device))
    _check("dcr_plan_autotune", code)
    return float(ms.value)


def dcr_plan_map_chunk(plan: int) -> int:
    c = ctypes.c_int32(0)
    _check("dcr_plan_map_chunk", library().dcr_plan_map_chunk(ctypes.c_void_p(plan),
                                                             ctypes.addressof(c)))
    return int(c.value)


def dcr_plan_destroy(plan: int):
    _check("dcr_plan_destroy", library().dcr_plan_destroy(ctypes.c_void_p(plan)))


def dcr_stream_probe(kind: int, src, dst, grid: int, unroll: int = 8):
    """Bandwidth reference (measurement only): kind 0 reads src (dst receives
    `grid` float partial sums), kind 1 copies src to dst."""
    _dev_tensor(src, "src")
    _dev_tensor(dst, "dst")
    nbytes = src.numel() * src.element_size()
    _check("dcr_stream_probe", library().dcr_stream_probe(
        int(kind), int(unroll), _ptr(src), _ptr(dst), nbytes, int(grid), _stream(src.device)))


def dcr_profile_begin(cap: int):
    _check("dcr_profile_begin", library().dcr_profile_begin(int(cap)))


def dcr_profile_end() -> dict:
    """Stop kernel timing; returns {kind name: (launches, total ms)}."""
    lib = library()
    n = lib.dcr_profile_kind_count()
    counts = (ctypes.c_int64 * n)()
    ms = (ctypes.c_double * n)()
    _check("dcr_profile_end", lib.dcr_profile_end(n, ctypes.addressof(counts),
                                                  ctypes.addressof(ms)))
    return {lib.dcr_profile_kind_name(k).decode(): (int(counts[k]), float(ms[k]))
            for k in range(n)}
