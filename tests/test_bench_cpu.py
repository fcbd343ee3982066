"""bench.py's host logic: the roofline arithmetic, the traffic summaries it
reads (taken on the current kernel sources only), and the one-GPU limit."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_roofline_of_one_launch():
    # one 1920x1080 frame in 8 us: 17 B/px over 8 us
    r = bench.roofline(1920 * 1080, 8e-3, traffic=123.0)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert abs(r["achieved"] - 17 * 1920 * 1080 / 8e-6 / 1e9) < 1e-9
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-12
    assert r["traffic"] == 123.0
    q = bench.roofline_from_rate(1920 * 1080 / 8.0)   # the same rate in Mpix/s
    assert abs(q["achieved"] - r["achieved"]) < 1e-9


def test_traffic_summaries_follow_the_kernel_sources(monkeypatch, tmp_path):
    """A summary counts only for the sources and flags it was taken on."""
    rec = {"kernel_hash": "a" * 16, "hbm_bytes_per_launch": 4.5e7}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_demo.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_hash", lambda sources=None: "a" * 16)
    assert bench.load_traffic("demo", 1) == 4.5e7
    assert bench.load_traffic("missing", 1) is None
    monkeypatch.setattr(bench, "kernel_hash", lambda sources=None: "0" * 16)
    assert bench.load_traffic("demo", 1) is None


def test_kernel_hash_covers_the_compiler_flags(monkeypatch):
    from paper_2209_08241_amd import build
    h = bench.kernel_hash()
    monkeypatch.setattr(build, "HIPCC_FLAGS", build.HIPCC_FLAGS + ["-DX"])
    assert bench.kernel_hash() != h


def test_one_gpu_only():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
    assert not r.stdout.strip().startswith("{")


def test_adjoint_summary_hashes_the_adjoint_sources():
    assert bench.kernel_hash(bench.ADJOINT_SOURCES) != bench.kernel_hash()
    assert "bn_adjoint.hip" in bench.ADJOINT_SOURCES


def test_inputs_generated_up_front_and_pool_joined():
    """Every host frame comes from one process pool that is shut down before
    the function returns (so no child outlives it, and nothing forks after
    the GPU is initialised)."""
    import argparse
    import multiprocessing
    args = argparse.Namespace(workload="plain1080", distinct=2, ring=32, no_batch=True,
                              no_serve=True, quick=True)
    inp = bench.generate_inputs(args)
    assert list(inp) == ["plain"] and len(inp["plain"]) == 2
    assert [s.seed for s in inp["plain"]] == [2, 3]
    assert inp["plain"][0].depth.shape == (1080, 1920)
    assert multiprocessing.active_children() == []
