"""Host-side logic of bench.py (no GPU): the multi-GPU refusal, the
algorithmic byte counts, the source digest that ties stored HBM counters to
the kernel source they were taken on, and the scaling of rocprofv3 counter
files by the copy of known size."""
import argparse
import csv
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one MI355X" in p.stderr
    assert p.stdout == ""


def test_reduce_bytes_sparse_workload():
    # M = 2^26 binary32 weights, N = 2^14: the weights once, 2048 blocks of 128
    # sub-tile ends and 12 bytes of totals and flags, N + 1 spacings and 5
    # spacing-block totals
    M, N = 1 << 26, 1 << 14
    expect = M * 4 + 2048 * 128 * 8 + 2048 * 12 + (N + 1) * 8 + 5 * 8
    assert bench.reduce_bytes(M, N, 4) == expect == 270688304
    assert bench.reduce_bytes(M, 0, 4) == M * 4 + 2048 * 128 * 8 + 2048 * 12 + 8
    assert bench.step_bytes(M, N, 4, 0) == expect + 12 * N
    assert bench.map_bytes(N, 8, 3) == 12 * N + 3 * 256 * 8


def test_source_digest_covers_the_kernel_and_what_precedes_it(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    shutil.copy(bench.KERNEL_SOURCE, src)
    text = src.read_text()
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    d_reduce, d_finish = bench.source_digest("k_reduce"), bench.source_digest("k_finish")
    # text after every kernel changes neither digest
    src.write_text(text + "\n// trailing note\n")
    assert bench.source_digest("k_reduce") == d_reduce
    assert bench.source_digest("k_finish") == d_finish
    # text between the two sections changes only the later kernel's digest
    cut = text.index("void k_finish(")
    cut = text.rindex("\n// ----", 0, cut)
    src.write_text(text[:cut] + "\n// inserted\n" + text[cut:])
    assert bench.source_digest("k_reduce") == d_reduce
    assert bench.source_digest("k_finish") != d_finish
    # text above both changes both
    src.write_text("// first line\n" + text)
    assert bench.source_digest("k_reduce") != d_reduce
    assert bench.source_digest("k_finish") != d_finish


def _counter_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_write_traffic_scales_by_the_copy(tmp_path, monkeypatch):
    copy_kib = bench.CALIBRATE_BYTES / 1024.0
    red = "void dcr::k_reduce<float, 1>(float const*, dcr::WArgs, dcr::ZArgs, int)"
    fin = "void dcr::k_finish<float, 1>(float const*, dcr::WArgs)"
    bat = "void dcr::k_reduce_batched<float, 1>(float const*, dcr::BatchArgs)"
    neg = "void at::native::neg_kernel(...)"
    _counter_csv(tmp_path / "f.csv", [(red, "FETCH_SIZE", 1000.0), (red, "FETCH_SIZE", 3000.0),
                                      (fin, "FETCH_SIZE", 40.0), (bat, "FETCH_SIZE", 500.0),
                                      (neg, "FETCH_SIZE", 7.0)])
    _counter_csv(tmp_path / "w.csv", [(red, "WRITE_SIZE", 10.0), (fin, "WRITE_SIZE", 2.0),
                                      (bat, "WRITE_SIZE", 50.0)])
    # the copy reads back half its size on FETCH_SIZE and all of it on WRITE_SIZE
    _counter_csv(tmp_path / "cf.csv", [(neg, "FETCH_SIZE", copy_kib / 2)])
    _counter_csv(tmp_path / "cw.csv", [(neg, "WRITE_SIZE", copy_kib)])
    out = tmp_path / "traffic.json"
    out.write_text(json.dumps({"other/f32/reduce": {"bytes_per_launch": 1.0}}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    args = argparse.Namespace(write_traffic=[str(tmp_path / n) for n in ("f.csv", "w.csv", "cf.csv", "cw.csv")],
                              precision="f32", workload="sparse")
    bench.write_traffic(args)
    d = json.loads(out.read_text())
    assert d["other/f32/reduce"] == {"bytes_per_launch": 1.0}   # entries of other runs kept
    e = d["sparse/f32/reduce"]
    assert e["copy_scale_fetch"] == pytest.approx(2.0) and e["copy_scale_write"] == pytest.approx(1.0)
    assert e["bytes_per_launch"] == pytest.approx((2000.0 * 2 + 10.0) * 1024)
    assert e["source_digest"] == bench.source_digest("k_reduce")
    assert d["sparse/f32/finish"]["bytes_per_launch"] == pytest.approx((40.0 * 2 + 2.0) * 1024)
    assert d["batched/f32/batch_reduce"]["bytes_per_launch"] == pytest.approx((500.0 * 2 + 50.0) * 1024)
    # a stored figure is used only while the kernel source is unchanged
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    assert bench.load_traffic("sparse", "f32", "reduce") == pytest.approx((2000.0 * 2 + 10.0) * 1024)
    assert bench.load_traffic("sparse", "f64", "reduce") is None
    src = tmp_path / "k.hip"
    src.write_text("// changed\n" + open(bench.KERNEL_SOURCE).read())
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    assert bench.load_traffic("sparse", "f32", "reduce") is None
