"""Host logic of bench.py (no GPU): the one-GPU refusal, the HBM-counter summary and its
source-hash gate."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def _csv(path, rows):
    with open(path, "w") as f:
        f.write("Kernel_Name,Counter_Name,Counter_Value\n")
        for k, c, v in rows:
            f.write(f'"{k}",{c},{v}\n')


@pytest.mark.parametrize("st", ["void alofdft::k_stencil2<float, 6, 4, 2, 1, alofdft::CGP1LOp<float> >(alofdft::Geom)",
                                "void alofdft::k_stencil2<float, 6, 8, 1, 1, alofdft::CGP1LIOp, 1>(alofdft::Geom)"])
def test_counter_summary_scales_by_the_reference_copy(tmp_path, st):
    # the copy of 256 MiB reads 131072 KiB on FETCH_SIZE (factor 2: a 128-byte read request
    # counts as 64 bytes) and 262144 KiB on WRITE_SIZE (factor 1); the CG kernels' per-dispatch
    # means are scaled by the same factor and summed over the two launches of an iteration
    # (the FP32 first half with separate p and A p arrays, or as one array of pairs)
    up = "void alofdft::k_cg_update<float, 256, true, true>(alofdft::Geom, alofdft::CGP2Op<float>)"
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    _csv(fetch, [(st, "FETCH_SIZE", 1000.0), (st, "FETCH_SIZE", 1200.0), (up, "FETCH_SIZE", 700.0),
                 ("__amd_rocclr_copyBuffer", "FETCH_SIZE", 131072.0), ("tiny copyBuffer", "FETCH_SIZE", 1.0)])
    _csv(write, [(st, "WRITE_SIZE", 500.0), (up, "WRITE_SIZE", 300.0),
                 ("__amd_rocclr_copyBuffer", "WRITE_SIZE", 262144.0)])
    out = tmp_path / "traffic.json"
    bench.summarize_counters(str(fetch), str(write), "cg_f32_test", path=str(out))
    ent = json.load(open(out))["cg_f32_test"]
    assert ent["read_bytes"] == round((1100.0 + 700.0) * 1024 * 2.0)
    assert ent["write_bytes"] == round((500.0 + 300.0) * 1024 * 1.0)
    assert ent["bytes_per_iteration"] == ent["read_bytes"] + ent["write_bytes"]
    assert ent["kernels_sha256_16"] == bench.kernel_digest()
    # the gate: the bytes are reported only while the kernel sources match
    assert bench.traffic_for("cg_f32_test", path=str(out)) == ent["bytes_per_iteration"]
    data = json.load(open(out))
    data["cg_f32_test"]["kernels_sha256_16"] = "0" * 16
    json.dump(data, open(out, "w"))
    assert bench.traffic_for("cg_f32_test", path=str(out)) is None
    assert bench.traffic_for("absent", path=str(out)) is None


def test_fifo_replay_and_percentiles():
    # the sequential baseline replays the arrivals through one FIFO server
    assert bench.fifo_latencies([0.0, 0.5, 3.0], [1.0, 1.0, 1.0]) == [1.0, 1.5, 1.0]
    v = list(range(1, 101))
    assert bench.pct(v, 0.5) == 50 and bench.pct(v, 0.99) == 99 and bench.pct([7.0], 0.99) == 7.0
