"""Benchmark: end-to-end multinomial resampling on one MI355X.

One step = one dcr_resample call (normalising weight scan, sorted uniforms by
exponential spacings, divide-and-conquer inverse-CMF map) on synthetic
weights already resident in HBM.  The default workload is the large
sparse-mass instance (M = 2^26 weights, log-weights ~ N(0, 5^2), N = 2^14
draws) in the binary32-input form; the binary64 form of the same workload is
timed beside it.  Weight buffers are rotated so the working set exceeds the
256 MB last-level (Infinity) cache.

Prints one JSON line (rank 0).  Multi-GPU runs are not supported.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "resampled particles/s and HBM GB/s (% peak), FP32-comp vs FP64, 1 MI355X"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
LLC_BYTES = 256 << 20          # Infinity Cache
W_BLOCK = 32768
W_SUB = 256
Z_BLOCK = 4096
KERNEL_SOURCE = os.path.join(ROOT, "paper_2604_01356_amd", "csrc", "dcr_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def reduce_bytes(M: int, N: int, s_w: int) -> int:
    """Algorithmic HBM bytes of one k_reduce launch: read w once, write the
    sub-tile ends, block totals / flags and the N+1 spacings."""
    nwb = -(-M // W_BLOCK)
    nzb = -(-(N + 1) // Z_BLOCK) if N > 0 else 0
    return M * s_w + nwb * (W_BLOCK // W_SUB) * 8 + nwb * 12 + (N + 1) * 8 + nzb * 8


def step_bytes(M: int, N: int, s_w: int, touched_sub: int) -> int:
    """Algorithmic bytes of one whole step (W and u not requested): the reduce
    launch, the map's read of the in-block spacing prefixes, its re-read of the
    weight sub-tiles that hold a draw, and the index write."""
    return reduce_bytes(M, N, s_w) + 8 * N + touched_sub * W_SUB * s_w + 4 * N


def map_bytes(N: int, s_w: int, touched_sub: int) -> int:
    """Algorithmic HBM bytes of the map launch: the in-block spacing prefixes,
    the weight sub-tiles that hold a draw (re-summed) and the index write."""
    return 8 * N + touched_sub * W_SUB * s_w + 4 * N


def source_digest(kernel: str) -> str:
    """Digest of the source a kernel is built from: the device headers and the
    kernel file up to the end of the kernel's own section (everything it can
    use is defined above it), so later kernels do not change it."""
    csrc = os.path.join(ROOT, "paper_2604_01356_amd", "csrc")
    h = hashlib.sha256()
    for name in ("dcr_device.hpp", "dcr_internal.hpp"):   # what the kernels are built from
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    with open(KERNEL_SOURCE, "r") as f:
        text = f.read()
    start = text.index(f"void {kernel}(")
    end = text.find("\n// ----", start)
    h.update(text[: end if end >= 0 else len(text)].encode())
    return h.hexdigest()[:16]


def load_traffic(workload: str, precision: str, kernel: str):
    """HBM bytes per launch of `kernel` from committed rocprofv3 counter runs,
    or None if absent or taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    e = d.get(f"{workload}/{precision}/{kernel}")
    if not e or e.get("source_digest") != source_digest(KERNEL_NAMES[kernel]):
        return None
    return e.get("bytes_per_launch")


# kernel of each timed launch kind
KERNEL_NAMES = {"reduce": "k_reduce", "finish": "k_finish", "map_dense": "k_map_dense",
                "map_fused": "k_map_fused", "carries": "k_carries",
                "batch_reduce": "k_reduce_batched", "batch_map": "k_map_batched",
                "batch_carries": "k_carries_batched", "map_span": "k_dense_span"}
KIND_OF_KERNEL = {v: k for k, v in KERNEL_NAMES.items()}
COPY_KERNEL = "neg_kernel"


def _counter_rows(path: str):
    import csv
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            yield row["Kernel_Name"], row["Counter_Name"], float(row["Counter_Value"])


def _per_kernel_means(path: str, counter: str) -> dict:
    """Mean counter value per dispatch for each library kernel, keyed by
    (bare kernel name, element type or None)."""
    import re
    acc = {}
    for name, c, v in _counter_rows(path):
        if c != counter:
            continue
        m = re.search(r"dcr::(k_\w+)(?:<(\w+))?", name)
        if not m:
            continue
        acc.setdefault((m.group(1), m.group(2)), []).append(v)
    return {k: sum(v) / len(v) for k, v in acc.items()}


def _copy_mean(path: str, counter: str) -> float:
    vals = [v for k, c, v in _counter_rows(path) if c == counter and COPY_KERNEL in k]
    if not vals:
        raise SystemExit(f"{path}: no {counter} rows for the copy kernel")
    return sum(vals) / len(vals)


def write_traffic(args):
    """Turn four rocprofv3 --pmc CSV files (FETCH_SIZE and WRITE_SIZE of the
    bench command, then of --calibrate-copy) into HBM bytes per launch of
    every library kernel they cover, each counter scaled by what it reads for
    the copy of known size."""
    fetch, write, cfetch, cwrite = args.write_traffic
    copy_kib = CALIBRATE_BYTES / 1024.0
    f_scale = copy_kib / _copy_mean(cfetch, "FETCH_SIZE")
    w_scale = copy_kib / _copy_mean(cwrite, "WRITE_SIZE")
    fk = _per_kernel_means(fetch, "FETCH_SIZE")
    wk = _per_kernel_means(write, "WRITE_SIZE")
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        d = {}
    for (bare, targ), fv in sorted(fk.items(), key=lambda kv: (kv[0][0], kv[0][1] or "")):
        if bare not in KIND_OF_KERNEL or (bare, targ) not in wk:
            continue
        prec = {"float": "f32", "double": "f64"}.get(targ, args.precision)
        workload = "batched" if bare.endswith("_batched") else args.workload
        key = f"{workload}/{prec}/{KIND_OF_KERNEL[bare]}"
        d[key] = {
            "bytes_per_launch": (fv * f_scale + wk[(bare, targ)] * w_scale) * 1024.0,
            "fetch_kib_per_launch": fv * f_scale,
            "write_kib_per_launch": wk[(bare, targ)] * w_scale,
            "copy_scale_fetch": f_scale,
            "copy_scale_write": w_scale,
            "source_digest": source_digest(bare),
        }
        print(key, json.dumps(d[key]))
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
        f.write("\n")


CALIBRATE_BYTES = 1 << 30


def calibrate_copy():
    """A plain streaming copy of known size (1 GiB read, 1 GiB written) for
    scaling the HBM byte counters."""
    import torch
    n = CALIBRATE_BYTES // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "neg copy", "bytes_read": CALIBRATE_BYTES,
                      "bytes_written": CALIBRATE_BYTES}), flush=True)


def host_info() -> dict:
    """The host the CPU rows ran on: CPU model and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def measure_copy_bw(dcr, torch, dev, reps: int = 10) -> dict:
    """Streaming references measured in the same run on 1 GiB (beyond the
    Infinity Cache): the library's streaming read and copy kernels (coalesced
    16-byte loads, best of a few grid sizes) and torch's copy_, each the
    median of `reps` launches."""
    import statistics
    n = CALIBRATE_BYTES // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)

    def med(fn):
        for _ in range(2):
            fn()
        times = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) * 1e-3)
        return statistics.median(times)

    res = {"read_gbs": 0.0, "copy_gbs": 0.0}
    for unroll in (4, 8, 16):
        for grid in (1024, 2048, 4096, 8192, 16384):
            for kind, name in ((0, "grid-stride"), (2, "contiguous runs, non-temporal")):
                t = med(lambda: dcr.dcr_stream_probe(kind, src, dst, grid, unroll))
                if CALIBRATE_BYTES / t / 1e9 > res["read_gbs"]:
                    res["read_gbs"] = CALIBRATE_BYTES / t / 1e9
                    res["read_launch"] = [name, grid, unroll]
            t = med(lambda: dcr.dcr_stream_probe(1, src, dst, grid, unroll))
            if 2 * CALIBRATE_BYTES / t / 1e9 > res["copy_gbs"]:
                res["copy_gbs"], res["copy_launch"] = 2 * CALIBRATE_BYTES / t / 1e9, [grid, unroll]
    res["torch_copy_gbs"] = 2 * CALIBRATE_BYTES / med(lambda: dst.copy_(src)) / 1e9
    res["note"] = ("1 GiB: read = bytes read / time, copy = bytes read + written / time; "
                   f"median of {reps} launches; best [pattern, grid, loads in flight] of the "
                   "sweep")
    del src, dst
    torch.cuda.empty_cache()
    return res


def measure_read_same_bytes(dcr, torch, dev, nbytes: int, reps: int = 10) -> dict:
    """The library's streaming read (both patterns, the same sweep as
    measure_copy_bw) over as many bytes as the dominant kernel moves: a launch
    of a few hundred MB carries its own ramp and tail, which 1 GiB hides."""
    import statistics
    n = max(16, nbytes // 16 * 16) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    part = torch.empty(16384, dtype=torch.float32, device=dev)

    def med(fn):
        for _ in range(2):
            fn()
        times = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) * 1e-3)
        return statistics.median(times)

    res = {"bytes": 4 * n, "read_gbs": 0.0}
    for unroll in (4, 8, 16):
        for grid in (1024, 2048, 4096, 8192, 16384):
            for kind, name in ((0, "grid-stride"), (2, "contiguous runs, non-temporal")):
                t = med(lambda: dcr.dcr_stream_probe(kind, src, part, grid, unroll))
                if 4 * n / t / 1e9 > res["read_gbs"]:
                    res["read_gbs"] = 4 * n / t / 1e9
                    res["read_launch"] = [name, grid, unroll]
    del src, part
    torch.cuda.empty_cache()
    return res


def batched_reduce_bytes(w_off, n_off, s_w: int) -> int:
    """Algorithmic HBM bytes of the batched reduce launch: every filter's
    weights once, its sub-tile ends and block totals, its N_b + 1 spacing
    prefixes and block totals."""
    import numpy as np
    Mb = np.diff(w_off)
    Nb = np.diff(n_off)
    nwb = int(np.sum(-(-Mb // W_BLOCK)))
    nzb = int(np.sum(np.where(Nb > 0, -(-(Nb + 1) // Z_BLOCK), 0)))
    return int(Mb.sum()) * s_w + nwb * ((W_BLOCK // W_SUB) * 8 + 8) + int((Nb + 1).sum()) * 8 \
        + nzb * 8


def measure_batched(dcr, torch, dev, steps: int, warmup: int, cpu_seconds: float):
    """The 4096-filter workload in the binary32 form, one dcr_resample_batched
    call per step (the weights, 2.4 GB, exceed the Infinity Cache)."""
    import numpy as np

    import workloads
    bw = workloads.batched()
    w32 = bw.w32
    sumN = int(bw.n_off[-1])
    w = torch.from_numpy(w32).to(dev)
    w_off = torch.from_numpy(bw.w_off).to(dev)
    n_off = torch.from_numpy(bw.n_off).to(dev)
    r = torch.empty(sumN, dtype=torch.int32, device=dev)
    st = torch.empty(1, dtype=torch.int32, device=dev)
    ws = torch.empty(dcr.dcr_batched_workspace_bytes(bw.B, w32.size, sumN, dcr.DCR_FP32_COMP),
                     dtype=torch.uint8, device=dev)

    # the map tile for this batch, chosen by the library's autotuner
    chunk, tune_ms = dcr.dcr_batched_autotune(w, w_off, n_off, seed=0, r=r, ws=ws)

    def step(k):
        dcr.dcr_resample_batched_ex(w, w_off, n_off, seed=k, chunk=chunk, r=r, dev_status=st,
                                    ws=ws)

    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(steps):
        step(k)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    dcr.dcr_profile_begin(steps * 8)
    for k in range(steps):
        step(k)
    prof = dcr.dcr_profile_end()
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    kernels = {k: v[1] / v[0] for k, v in prof.items() if v[0] > 0}
    # the same call captured once in a HIP graph and replayed
    r_g = torch.empty_like(r)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        dcr.dcr_resample_batched_ex(w, w_off, n_off, seed=0, chunk=chunk, r=r_g, ws=ws)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=side):
            dcr.dcr_resample_batched_ex(w, w_off, n_off, seed=0, chunk=chunk, r=r_g, ws=ws)
    torch.cuda.current_stream().wait_stream(side)
    g.replay()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / steps
    step(0)
    torch.cuda.synchronize()
    graph_equal = bool(torch.equal(r_g, r))
    del g
    # the library's own plan: its workspace, tuned tile and graph (launched
    # with hipGraphLaunch, the arguments written into the graph's nodes)
    plan = dcr.dcr_plan_create_batched(bw.B, w32.size, sumN, dcr.DCR_FP32_COMP)
    try:
        r_p = torch.empty_like(r)
        dcr.dcr_plan_autotune(plan, w, w_off, n_off, r_p, seed=0)
        for k in range(warmup):
            dcr.dcr_plan_resample_batched(plan, w, w_off, n_off, k, r_p, None, st)
        torch.cuda.synchronize()
        e0.record()
        for k in range(steps):
            dcr.dcr_plan_resample_batched(plan, w, w_off, n_off, k, r_p, None, st)
        e1.record()
        torch.cuda.synchronize()
        plan_ms = e0.elapsed_time(e1) / steps
        plan_chunk = dcr.dcr_plan_map_chunk(plan)
        dcr.dcr_plan_resample_batched(plan, w, w_off, n_off, 0, r_p, None, st)
        torch.cuda.synchronize()
        plan_equal = bool(torch.equal(r_p, r)) and int(st.item()) == 0
    finally:
        dcr.dcr_plan_destroy(plan)
    r0 = r.cpu().numpy()
    red_bytes = batched_reduce_bytes(bw.w_off, bw.n_off, 4)
    achieved = red_bytes / (kernels["batch_reduce"] * 1e-3) / 1e9
    traffic = load_traffic("batched", "f32", "batch_reduce")
    out = {
        "workload": bw.description,
        "B": bw.B, "sum_M": int(w32.size), "sum_N": sumN,
        "map_chunk": chunk, "map_chunk_tuned_ms": tune_ms,
        "ms_per_step": ms,
        "value": sumN / (ms * 1e-3),
        "unit": "particles/s",
        "graph_ms_per_step": graph_ms,
        "graph_equals_eager": graph_equal,
        "plan_ms_per_step": plan_ms,
        "plan_map_chunk": plan_chunk,
        "plan_equals_eager": plan_equal,
        "weights_per_s": w32.size / (ms * 1e-3),
        "step_weight_gbs": w32.nbytes / (ms * 1e-3) / 1e9,
        "kernels_ms": kernels,
        "roofline": {"kernel": "k_reduce_batched", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "algorithmic_bytes": red_bytes,
                     "avg_launch_us": kernels["batch_reduce"] * 1e3},
    }
    if cpu_seconds > 0:
        import oracle
        # the oracle over every filter of the batch, its filters spread over
        # the host's cores by OpenMP (each filter's arithmetic unchanged)
        threads = int(os.environ.get("OMP_NUM_THREADS") or 0) or host_info()["usable_cpus"]
        t0 = time.perf_counter()
        r_or, used = oracle.resample_batched_parallel(w32, bw.w_off, bw.n_off, 0, threads)
        t = time.perf_counter() - t0
        mism = int(np.sum(r_or != r0))
        out["cpu_baseline"] = {"value": sumN / t, "unit": "particles/s", "cores": used,
                               "kind": "oracle",
                               "sample": f"oracle on all {bw.B} filters ({sumN} draws) in "
                                         f"{t:.2f} s, OpenMP over filters on {used} threads"}
        # the binary32 form against the oracle on the same binary32 weights:
        # every mismatch is a bin-edge case (device and host logf differ by an ulp)
        out["mismatches_vs_oracle"] = mism
        out["mismatch_rate_vs_oracle"] = mism / sumN
    del w, ws, r
    torch.cuda.empty_cache()
    return out


def measure_outer(dcr, torch, dev, steps: int):
    """An EnGMF-shaped step at scale: N = 65536 particles, P = 256 likelihood
    components, M = N*P = 2^24 weights w = a_i * b_k, draw N.  binary32 factors,
    weights formed on the fly (dcr_resample_outer) against the same weights
    materialised in HBM (dcr_resample); the two give identical indices."""
    import numpy as np

    import workloads
    wl = workloads.engmf_step(N=65536, P=256)
    a = wl.extra["a"].astype(np.float32)
    b = wl.extra["b"].astype(np.float32)
    Np, P = a.size, b.size
    M = Np * P
    at, bt = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    # a_i * b_k of binary32 factors is exact in binary64: the materialised array
    w = torch.from_numpy(np.multiply.outer(a.astype(np.float64), b.astype(np.float64))
                         .ravel()).to(dev)
    ws = torch.empty(dcr.dcr_workspace_bytes(M, Np, dcr.DCR_FP64), dtype=torch.uint8,
                     device=dev)
    r1 = torch.empty(Np, dtype=torch.int32, device=dev)
    r2 = torch.empty(Np, dtype=torch.int32, device=dev)
    res = {"workload": f"engmf N={Np} x P={P} (M={M}), draw N={Np}, binary32 factors"}
    a64, b64 = at.double(), bt.double()
    calls = (("outer_f32", lambda k: dcr.dcr_resample_outer(at, bt, Np, k, r=r1, ws=ws)),
             ("outer_f64", lambda k: dcr.dcr_resample_outer(a64, b64, Np, k, r=r1, ws=ws)),
             ("array_f64", lambda k: dcr.dcr_resample(w, Np, k, r=r2, ws=ws)))
    for name, fn in calls:
        for k in range(2):
            fn(k)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for k in range(steps):
            fn(k)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res[name] = {"ms_per_step": ms, "value": Np / (ms * 1e-3), "unit": "particles/s"}
    dcr.dcr_profile_begin(steps * 8)
    for k in range(steps):
        calls[0][1](k)
    prof = dcr.dcr_profile_end()
    res["outer_f32"]["kernels_ms"] = {k: v[1] / v[0] for k, v in prof.items() if v[0] > 0}
    dcr.dcr_resample_outer(a64, b64, Np, 3, r=r1, ws=ws)
    dcr.dcr_resample(w, Np, 3, r=r2, ws=ws)
    torch.cuda.synchronize()
    res["outer_f64_equals_array"] = bool(torch.equal(r1, r2))
    del w, ws
    torch.cuda.empty_cache()
    return res


def cpu_baseline(wl, w_host, seconds: float):
    import numpy as np

    import oracle
    times = []
    r0 = None
    t_end = time.perf_counter() + seconds
    while True:
        t0 = time.perf_counter()
        r, _, _ = oracle.resample(w_host, wl.N, seed=0, stream=0)
        times.append(time.perf_counter() - t0)
        if r0 is None:
            r0 = r
        if time.perf_counter() >= t_end or len(times) >= 50:
            break
    t = float(np.median(times))
    return {
        "value": wl.N / t,
        "unit": "particles/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{len(times)} full end-to-end oracle resamples of the same workload "
                  f"(M={wl.M}, N={wl.N}), median {t:.3f} s each, single thread",
    }, r0


def cpu_paper_algorithm(wl, w_host, seconds: float):
    """The paper's own sequential method on the host, for a second CPU row:
    the plain running sum of Eq. 3 divided by the total, Alg. 1 with a plain
    running sum of the oracle's spacings, and the oracle's literal Alg. 5."""
    import numpy as np

    import oracle
    w = np.asarray(w_host, dtype=np.float64)
    times = []
    t_end = time.perf_counter() + seconds
    while True:
        t0 = time.perf_counter()
        S = np.cumsum(w)
        W = S / S[-1]
        Z = np.cumsum(oracle.exponential_spacings(wl.N, seed=0, stream=0))
        u = Z[:wl.N] / Z[wl.N]
        oracle.dac(W, u)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() >= t_end or len(times) >= 50:
            break
    t = float(np.median(times))
    return {
        "value": wl.N / t,
        "unit": "particles/s",
        "cores": 1,
        "kind": "paper algorithm (plain running sums, Alg. 1, Alg. 5)",
        "sample": f"{len(times)} end-to-end runs of the same workload (M={wl.M}, N={wl.N}), "
                  f"median {t:.3f} s each, single thread",
    }


def measure_stages(dcr, torch, dev, wl, prec: str, reps: int):
    """The three stages called separately on the main workload, each
    materialising its output (W, then u, then r from that W and u)."""
    w_host = wl.w32 if prec == "f32" else wl.w64
    w = torch.from_numpy(w_host).to(dev)
    p = dcr.precision_of(w)
    ws = torch.empty(dcr.dcr_workspace_bytes(wl.M, wl.N, p), dtype=torch.uint8, device=dev)
    W = torch.empty(wl.M, dtype=torch.float64, device=dev)
    tot = torch.empty(1, dtype=torch.float64, device=dev)
    u = torch.empty(max(wl.N, 1), dtype=torch.float64, device=dev)
    r = torch.empty(max(wl.N, 1), dtype=torch.int32, device=dev)
    calls = {
        "cumulative_weights": lambda: dcr.dcr_cumulative_weights(w, W=W, total=tot, ws=ws),
        "sorted_uniforms": lambda: dcr.dcr_sorted_uniforms(wl.N, 0, 0, precision=p, u=u, ws=ws),
        "inverse_cmf": lambda: dcr.dcr_inverse_cmf(W, u[:wl.N], r=r),
    }
    res = {"workload": wl.description, "precision": prec}
    for name, fn in calls.items():
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        res[name + "_us"] = e0.elapsed_time(e1) / reps * 1e3
    s_w = 4 if prec == "f32" else 8
    res["cumulative_weights_gbs"] = (wl.M * (s_w + 8)) / (res["cumulative_weights_us"] * 1e-6) / 1e9
    res["note"] = ("stage 1 reads w and writes W (M*(s_w+8) bytes, the rate above); the fused "
                   "dcr_resample writes neither W nor u")
    del w, ws, W, u, r
    torch.cuda.empty_cache()
    return res


def measure_small(dcr, torch, dev, reps: int = 200):
    """The two small configurations are latency-bound: microseconds per
    dcr_resample call, eager and replayed from a captured HIP graph."""
    import numpy as np

    import workloads
    res = {}
    for wl in (workloads.small_single(), workloads.engmf_step()):
        for prec in ("f64", "f32"):
            w = torch.from_numpy(wl.w64 if prec == "f64" else wl.w32).to(dev)
            p = dcr.precision_of(w)
            ws = torch.empty(dcr.dcr_workspace_bytes(wl.M, wl.N, p), dtype=torch.uint8,
                             device=dev)
            r_e = torch.empty(wl.N, dtype=torch.int32, device=dev)
            r_g = torch.empty(wl.N, dtype=torch.int32, device=dev)

            def timed(fn):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    fn()
                e1.record()
                torch.cuda.synchronize()
                return e0.elapsed_time(e1) / reps * 1e3

            def single(fn, n=50):
                # one call on an idle device: events around it, median
                import statistics
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                lat = []
                for _ in range(n):
                    torch.cuda.synchronize()
                    e0.record()
                    fn()
                    e1.record()
                    torch.cuda.synchronize()
                    lat.append(e0.elapsed_time(e1) * 1e3)
                return statistics.median(lat)

            def host_issue(fn, n=200):
                # host time to enqueue one call (no wait)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(n):
                    fn()
                t1 = time.perf_counter()
                torch.cuda.synchronize()
                return (t1 - t0) / n * 1e6

            eager_fn = lambda: dcr.dcr_resample(w, wl.N, 0, r=r_e, ws=ws)  # noqa: E731
            for _ in range(3):
                eager_fn()
            torch.cuda.synchronize()
            eager_us = timed(eager_fn)
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            g = torch.cuda.CUDAGraph()
            with torch.cuda.stream(s):
                dcr.dcr_resample(w, wl.N, 0, r=r_g, ws=ws)
                torch.cuda.synchronize()
                with torch.cuda.graph(g, stream=s):
                    dcr.dcr_resample(w, wl.N, 0, r=r_g, ws=ws)
            torch.cuda.current_stream().wait_stream(s)
            g.replay()
            torch.cuda.synchronize()
            graph_us = timed(g.replay)
            res[f"{wl.name}/{prec}"] = {
                "M": wl.M, "N": wl.N,
                "us_per_call_eager": eager_us,
                "us_per_call_graph": graph_us,
                "single_call_us_eager": single(eager_fn),
                "single_call_us_graph": single(g.replay),
                "host_issue_us_eager": host_issue(eager_fn),
                "host_issue_us_graph": host_issue(g.replay),
                "graph_equals_eager": bool(torch.equal(r_g, r_e)),
            }
            del g, ws
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="sparse", choices=["sparse", "equal", "engmf", "single"])
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 4096-filter batched workload reported beside the main line")
    ap.add_argument("--no-outer", action="store_true",
                    help="skip the structured (outer-product) EnGMF workload")
    ap.add_argument("--no-stages", action="store_true",
                    help="skip the three stages timed as separate calls")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the two small, latency-bound configurations")
    ap.add_argument("--outer-only", action="store_true",
                    help="run only the structured (outer-product) EnGMF workload")
    ap.add_argument("--no-equal", action="store_true",
                    help="skip the equal-size workload reported beside the main line")
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-compare", action="store_true", help="skip the other precision")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only the copy of known size used to scale HBM counters")
    ap.add_argument("--write-traffic", nargs=4, metavar="CSV",
                    help="FETCH_SIZE, WRITE_SIZE csv of this command, then of --calibrate-copy")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(args)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: measures one MI355X only; multi-GPU runs (--gpus > 1) "
              "are not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2604_01356_amd as dcr
    import workloads

    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        calibrate_copy()
        return
    dev = torch.device("cuda:0")
    dcr.library()
    if args.outer_only:
        print(json.dumps({"engmf_outer": measure_outer(dcr, torch, dev, args.steps)}), flush=True)
        return
    wl = workloads.CONFIGS[args.workload]()

    def measure(prec: str, steps: int, warmup: int):
        w_host = wl.w32 if prec == "f32" else wl.w64
        nbytes = w_host.nbytes
        copies = max(2, -(-2 * LLC_BYTES // nbytes) + 1)
        ws_copies = [torch.from_numpy(w_host).to(dev) for _ in range(copies)]
        p = dcr.precision_of(ws_copies[0])
        ws = torch.empty(dcr.dcr_workspace_bytes(wl.M, wl.N, p), dtype=torch.uint8, device=dev)
        r = torch.empty(max(wl.N, 1), dtype=torch.int32, device=dev)
        st = torch.empty(1, dtype=torch.int32, device=dev)

        def step(k):
            dcr.dcr_resample(ws_copies[k % copies], wl.N, seed=k, stream_id=0, r=r,
                             dev_status=st, ws=ws)

        for k in range(warmup):
            step(k)
        torch.cuda.synchronize()
        # pass 1: whole-step time
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for k in range(steps):
            step(k)
        e1.record()
        torch.cuda.synchronize()
        ms_step = e0.elapsed_time(e1) / steps
        # pass 1b: every step bracketed by its own events, for the median
        import statistics
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        for k in range(steps):
            evs[k][0].record()
            step(k)
            evs[k][1].record()
        torch.cuda.synchronize()
        ms_median = statistics.median(a.elapsed_time(b) for a, b in evs)
        # pass 2: per-kernel HIP events on the launch stream
        dcr.dcr_profile_begin(steps * 8)
        for k in range(steps):
            step(k)
        prof = dcr.dcr_profile_end()
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        kernels = {k: v[1] / v[0] for k, v in prof.items() if v[0] > 0}
        # one more step with seed 0 for the parity spot check, with W
        W0 = None
        if want_w:
            W_dev = torch.empty(wl.M, dtype=torch.float64, device=dev)
            dcr.dcr_resample(ws_copies[0], wl.N, seed=0, stream_id=0, r=r, W_out=W_dev,
                             dev_status=st, ws=ws)
            W0 = W_dev.cpu().numpy()
            del W_dev
        else:
            step(0)
        r0 = r[: wl.N].cpu().numpy().copy()
        for t in ws_copies:
            del t
        del ws_copies
        torch.cuda.empty_cache()
        return ms_step, kernels, r0, w_host, W0, ms_median

    copy_bw = measure_copy_bw(dcr, torch, dev)
    want_w = not args.no_cpu and args.precision == "f32"
    ms, kernels, r_gpu, w_host, W_gpu, ms_med = measure(args.precision, args.steps, args.warmup)
    want_w = False
    s_w = 4 if args.precision == "f32" else 8
    touched = int(len(np.unique(r_gpu // W_SUB)))
    # the dominant launch kind of the step and its algorithmic bytes
    dom = max(kernels, key=kernels.get)
    if dom == "reduce":
        dom_bytes = reduce_bytes(wl.M, wl.N, s_w)
    elif dom in ("finish", "map_dense", "map_fused"):
        dom_bytes = map_bytes(wl.N, s_w, touched)
    else:
        raise SystemExit(f"bench.py: no byte model for the launch kind {dom}")
    achieved = dom_bytes / (kernels[dom] * 1e-3) / 1e9
    traffic = load_traffic(args.workload, args.precision, dom)
    read_same = measure_read_same_bytes(dcr, torch, dev, dom_bytes)
    out = {
        "metric": METRIC,
        "value": wl.N / (ms * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_per_step_median": ms_med,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "input_dtype": args.precision,
        "data": "synthetic",
        "config": {
            "workload": wl.description,
            "M": wl.M,
            "N": wl.N,
            "precision": "FP32_COMP" if args.precision == "f32" else "FP64",
        },
        "weights_per_s": wl.M / (ms * 1e-3),
        "step_hbm_gbs": step_bytes(wl.M, wl.N, s_w, touched) / (ms * 1e-3) / 1e9,
        "step_hbm_frac": step_bytes(wl.M, wl.N, s_w, touched) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "kernels_ms": kernels,
        "roofline": {
            "kernel": KERNEL_NAMES[dom],
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes": dom_bytes,
            "avg_launch_us": kernels[dom] * 1e3,
            "frac_of_copy": achieved / copy_bw["copy_gbs"],
            "frac_of_read": achieved / copy_bw["read_gbs"],
            "frac_of_read_same_bytes": achieved / read_same["read_gbs"],
        },
        "device_copy_bw": copy_bw,
        "device_read_same_bytes": read_same,
    }
    if not args.no_compare:
        other = "f64" if args.precision == "f32" else "f32"
        ms_o, kern_o, _, _, _, med_o = measure(other, max(5, args.steps // 2), 2)
        out[f"compare_{other}"] = {
            "ms_per_step": ms_o,
            "ms_per_step_median": med_o,
            "value": wl.N / (ms_o * 1e-3),
            "speedup_of_headline": ms_o / ms,
            "kernels_ms": kern_o,
        }
    if not args.no_cpu:
        cb, r_or = cpu_baseline(wl, w_host, args.cpu_seconds)
        cb["host"] = host_info()
        out["cpu_baseline"] = cb
        out["cpu_paper_algorithm"] = cpu_paper_algorithm(wl, w_host, args.cpu_seconds / 2)
        out["mismatches_vs_oracle_seed0"] = int(np.sum(r_gpu != r_or))
        out["mismatch_rate_vs_oracle_seed0"] = float(np.mean(r_gpu != r_or))
        if W_gpu is not None:
            # the binary32-input result against the oracle on the binary64 weights
            import oracle
            r64, W64, _ = oracle.resample(wl.w64, wl.N, seed=0, stream=0)
            out["fp32_vs_fp64"] = {
                "max_abs_dW": float(np.max(np.abs(W_gpu - W64))),
                "mismatches": int(np.sum(r_gpu != r64)),
                "mismatch_rate": float(np.mean(r_gpu != r64)),
                "reference": "oracle on the binary64 weights, seed 0",
            }
    if not args.no_batched:
        out["batched"] = measure_batched(dcr, torch, dev, max(5, args.steps // 5), 2,
                                         0.0 if args.no_cpu else args.cpu_seconds / 2)
    if not args.no_outer:
        out["engmf_outer"] = measure_outer(dcr, torch, dev, max(5, args.steps // 5))
    if not args.no_small:
        out["small_configs"] = measure_small(dcr, torch, dev)
    if not args.no_stages:
        out["stages"] = measure_stages(dcr, torch, dev, wl, args.precision,
                                       max(5, args.steps // 5))
    if args.workload != "equal" and not args.no_equal:
        # the equal-size instance (linear-merge limit of the map), both forms
        wl_eq = workloads.CONFIGS["equal"]()
        wl_saved = wl
        wl = wl_eq
        out["equal"] = {"workload": wl_eq.description}
        for prec in ("f32", "f64"):
            ms_e, kern_e, r_e, w_e, _, med_e = measure(prec, max(5, args.steps // 5), 2)
            row = {"ms_per_step": ms_e, "ms_per_step_median": med_e,
                   "value": wl_eq.N / (ms_e * 1e-3), "unit": "particles/s", "kernels_ms": kern_e}
            if not args.no_cpu:
                import oracle
                r_o = oracle.resample(w_e, wl_eq.N, seed=0, stream=0)[0]
                row["mismatches_vs_oracle_seed0"] = int(np.sum(r_e != r_o))
                row["mismatch_rate_vs_oracle_seed0"] = float(np.mean(r_e != r_o))
            out["equal"][prec] = row
        out["equal"]["speedup_f32_over_f64"] = (out["equal"]["f64"]["ms_per_step"] /
                                                out["equal"]["f32"]["ms_per_step"])
        wl = wl_saved
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
