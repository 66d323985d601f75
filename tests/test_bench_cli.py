"""The measurement script's command line, without a GPU: the one-GPU rule
and the per-kernel source hashes that tie stored traffic counters to the
sources they were taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_kernel_hashes_cover_their_sources():
    sys.path.insert(0, ROOT)
    import bench
    h1 = bench.kernel_source_hash("k_batch")
    assert h1 == bench.kernel_source_hash("k_batch") and len(h1) == 16
    assert h1 != bench.kernel_source_hash("k_swarm")
    # every source a hash covers exists
    csrc = os.path.join(ROOT, "paper_1704_01077_amd", "csrc")
    for files in bench.KERNEL_SOURCES.values():
        for f in files:
            assert os.path.exists(os.path.join(csrc, f)), f


def test_stored_traffic_records_are_well_formed():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        t = json.load(f)
    for workload, kernels in t.items():
        for kernel, rec in kernels.items():
            assert len(rec["source_hash"]) == 16
            assert rec["bytes_per_launch"] == int(rec["fetch_size_bytes"] + rec["write_size_bytes"])
            assert len(rec["fetch_size_kib"]) == len(rec["write_size_kib"]) > 0


def test_traffic_records_apply_only_to_their_key(tmp_path, monkeypatch):
    """A stored counter record is used only for the same kernel, workload,
    k, mode and batch width, and only while the kernel's sources hash to
    the value stored with it."""
    sys.path.insert(0, ROOT)
    import bench
    prof = tmp_path / "profiles"
    prof.mkdir()
    key = bench.traffic_key("k_batch", 10, "hybrid", 64)
    rec = {"source_hash": bench.kernel_source_hash("k_batch"), "bytes_per_launch": 1234,
           "k": 10, "mode": "hybrid", "batch_width": 64}
    (prof / "traffic.json").write_text(json.dumps({"ba1m": {key: rec}}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda k: rec["source_hash"])
    assert bench.load_traffic("k_batch", "ba1m", 10, "hybrid", 64) == 1234
    assert bench.load_traffic("k_batch", "ba1m", 100, "hybrid", 64) is None
    assert bench.load_traffic("k_batch", "ba1m", 10, "batched", 64) is None
    assert bench.load_traffic("k_batch", "ba1m", 10, "hybrid", 128) is None
    assert bench.load_traffic("k_batch", "rmat20", 10, "hybrid", 64) is None
    assert bench.load_traffic("k_batch", "ba1m", 10, "hybrid", 64, relabel=True) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda k: "0" * 16)
    assert bench.load_traffic("k_batch", "ba1m", 10, "hybrid", 64) is None
