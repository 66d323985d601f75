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
