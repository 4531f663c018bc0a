"""Host-side parts of bench.py: the one-GPU guard and the oracle baselines
of the secondary workloads (their JSON shape; the FP32 MLP one is cheap
enough to run here)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_workload_cpu_baseline_shape():
    import bench
    cb = bench.cpu_baseline_workload("mlp_f32", min_s=0.0)
    assert cb["kind"] == "oracle" and cb["unit"] == "invocations/s"
    assert cb["value"] > 0 and cb["cores"] >= 1 and "16 invocations" in cb["sample"]
    assert bench.cpu_baseline_workload("serving") is None


def test_traffic_record_matches_the_gemm_sources():
    """The committed HBM-traffic record of the headline GEMM layer is tied to
    a digest of the GEMM sources; a change to them without re-taking the
    counters would make bench.py report traffic as unknown."""
    import bench
    with open(bench.TRAFFIC_RECORD) as fh:
        recs = [l for l in fh.read().splitlines() if l.startswith("traffic-record: ")]
    assert recs, "no traffic record"
    import json
    digests = {json.loads(l[len("traffic-record: "):])["sources"] for l in recs}
    assert bench.gemm_sources_digest() in digests
