"""bench.py's host-side pieces (no GPU): the roofline record, the counter
record in profiles/ that it reads, and the one-GPU refusal."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_roofline_record_arithmetic_and_lookup():
    db = {"k": {"kernel_source_sha256_16": "abc", "hbm_bytes_per_launch": 123, "source": "here"}}
    # 4 launches of 1 GB each in 2 ms: 2 TB/s against the 8 TB/s peak
    r = bench.roofline_record("k", "unit", 1e9, 2.0, 4, 2, "abc", db)
    assert abs(r["avg_launch_ms"] - 0.5) < 1e-12 and abs(r["achieved"] - 2000.0) < 1e-6
    assert abs(r["frac"] - 0.25) < 1e-12 and r["peak"] == 8000.0 and r["ms_per_solve"] == 1.0
    assert r["traffic"] == 123 and r["traffic_note"] == "here"
    # counters taken for other sources are not reported
    r = bench.roofline_record("k", "unit", 1e9, 2.0, 4, 2, "other", db)
    assert r["traffic"] is None and "changed" in r["traffic_note"]
    r = bench.roofline_record("absent", "unit", 1e9, 2.0, 4, 2, "abc", db)
    assert r["traffic"] is None and r["traffic_note"] == "no counter record"


def test_counter_record_names_the_benchmarked_kernels():
    # the R-MAT scale-24 record holds the kernels bench.py names for that
    # workload (the dense step runs the 16-record instantiation there), each
    # with a hash of the kernel sources it was taken with
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["rmat_scale24_ef16"]
    for k in ("k_bin_pull<16>", "k_bin_fill<true>", "_solve"):
        assert k in rec and len(rec[k]["kernel_source_sha256_16"]) == 16
    assert rec["k_bin_pull<16>"]["hbm_bytes_per_launch"] > 0 and rec["_solve"]["hbm_bytes_per_solve"] > 0
    hashes = {rec[k]["kernel_source_sha256_16"] for k in rec}
    assert len(hashes) == 1  # one profiling run
    # while the sources are those the counters were taken with, bench.py reports them
    if hashes == {bench.kernel_source_hash()}:
        r = bench.roofline_record("k_bin_pull<16>", "u", 1.0, 1.0, 1, 1, bench.kernel_source_hash(), rec)
        assert r["traffic"] == rec["k_bin_pull<16>"]["hbm_bytes_per_launch"]


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU only" in p.stderr and p.stdout == ""
