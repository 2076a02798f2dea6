"""Host-side logic of bench.py: the memory-traffic figure is taken from a committed
counter record only while the fused-kernel sources are the ones it was measured on."""
import json
import subprocess
import sys

import bench


def _write(path, sha, workload="c3", prec="bf16x3"):
    path.write_text(
        "# summary\n\n"
        f"traffic-record sources-sha256 {sha} workload {workload} precision {prec}\n"
        "traffic-record fused_fwd waves 8 read-bytes 8.0e7 written-bytes 2.7e7\n"
        "traffic-record fused_bwd waves 4 read-bytes 1.1e8 written-bytes 4.4e7\n"
        "mfma-record fused_bwd waves 4 mops-bf16 4.0e7\n")


def test_record_used_only_for_matching_sources(tmp_path, monkeypatch):
    rec = tmp_path / "rec.md"
    monkeypatch.setattr(bench, "traffic_record_path", lambda w, p: str(rec))
    get = bench.recorded_counters
    assert get("fused_bwd", "c3", "bf16x3") is None                        # no record
    _write(rec, bench.kernel_sources_sha256())
    r = get("fused_bwd", "c3", "bf16x3")
    assert (r["read"], r["written"], r["mops_bf16"]) == (1.1e8, 4.4e7, 4.0e7)
    r = get("fused_fwd", "c3", "bf16x3", 8)
    assert (r["read"], r["written"]) == (8.0e7, 2.7e7) and "mops_bf16" not in r
    assert get("fused_fwd", "c3", "bf16x3", 4) is None                     # other form
    assert get("fused_dz", "c3", "bf16x3") is None                         # not recorded
    assert get("fused_bwd", "c5", "bf16x3") is None                        # other workload
    assert get("fused_bwd", "c3", "fp32") is None                          # other precision
    _write(rec, "0" * 64)                                                  # kernels changed
    assert get("fused_bwd", "c3", "bf16x3") is None


def test_cpu_baseline_threads_and_sample(monkeypatch):
    """The oracle baseline runs whole small chains (or the first pair of large ones)
    over the host threads and reports what it ran."""
    from workloads import make
    w = make("c2", B=3)
    rate, n_thr, desc = bench.cpu_baseline(w.chains, budget_s=0.0)
    assert rate > 0 and 1 <= n_thr <= 16 and "whole chains" in desc


def test_sources_hash_covers_every_kernel_source():
    import os
    for f in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(bench.ROOT, "paper_1806_08593_amd", "csrc", f)), f
    assert len(bench.kernel_sources_sha256()) == 64


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
