"""Host-side checks of bench.py (no GPU): the one-GPU guard and that the committed
profiles were taken on the kernel sources in the tree."""
import json
import os
import re
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_print_hash_matches_kernel_sources():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--print-hash"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0
    assert r.stdout.strip() == bench.kernel_hash()


def test_kernel_hash_ignores_comments_and_layout_but_not_code(tmp_path, monkeypatch):
    """The hash tagging the committed counter records follows the kernel code: comments and
    layout do not change it, a changed token does."""
    src = tmp_path / "k.hip"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ["k.hip"])
    src.write_text("__global__ void k(double *x)\n{\n    x[0] = 2.0 * x[1]; // twice\n}\n")
    h0 = bench.kernel_hash()
    src.write_text("/* a kernel */\n__global__ void k(double *x) {\n  x[0] = 2.0 * x[1];  // doubled\n\n}\n")
    assert bench.kernel_hash() == h0
    src.write_text("__global__ void k(double *x)\n{\n    x[0] = 3.0 * x[1]; // twice\n}\n")
    assert bench.kernel_hash() != h0


def _hashes():
    out = {}
    for name in ("traffic_large8192.json", "sq_large8192.json"):
        with open(os.path.join(ROOT, "profiles", name)) as f:
            out[name] = json.load(f)["kernel_hash"]
    with open(os.path.join(ROOT, "profiles", "tile_kernels_large8192_ktrace.txt")) as f:
        m = re.search(r"kernel sources hash ([0-9a-f]{16})", f.read())
    out["ktrace"] = m.group(1) if m else None
    return out


def test_committed_profiles_carry_a_kernel_hash_and_stale_ones_are_not_used():
    """The traffic and SQ counter summaries and the kernel trace carry the hash of the kernel
    sources they were taken on; bench.py reports traffic and FP64 rates only from summaries
    taken on the kernel sources in the tree (null otherwise)."""
    h = bench.kernel_hash()
    hs = _hashes()
    assert all(v is not None and re.fullmatch(r"[0-9a-f]{16}", v) for v in hs.values()), hs
    if hs["traffic_large8192.json"] != h:
        assert bench.iteration_traffic(8192 * 8192) is None
        assert bench.traffic_for("solve_x", 8192 * 8192) is None
    if hs["sq_large8192.json"] != h:
        assert bench.fp64_flops_for("solve_x") is None


@pytest.mark.parametrize("config,n", [("large8192", 8192), ("spinodal2048", 2048)])
def test_counter_summaries_are_usable(config, n):
    """Every sweep kernel class of the workload has fetch and write bytes per dispatch (never
    below its algorithmic bytes), the whole iteration at least 48 B per cell, and the dominant
    kernel of the 8192^2 workload an FP64 flop count (per wave instruction: 64 lanes each)."""
    path = bench.traffic_file(config)
    if not os.path.exists(path):
        pytest.skip(f"no counter summary for {config}")
    with open(path) as f:
        t = json.load(f)
    if t["kernel_hash"] != bench.kernel_hash():
        return  # a stale summary is never used (previous test)
    present = [k for k in bench.ALGO_BYTES_PER_CELL if k in t["kernels"]]
    assert {"relations_y", "solve_y"} <= set(present)
    for k in present:
        rec = t["kernels"][k]
        assert rec["fetch_kib"] > 0 and rec["write_kib"] > 0 and rec["dispatches"] > 0
        algo_kib = bench.ALGO_BYTES_PER_CELL[k] * n * n / 1024
        assert rec["fetch_kib"] + rec["write_kib"] >= algo_kib, k
    assert bench.iteration_traffic(n * n, config) >= 48 * n * n
    if config == "large8192" and os.path.exists(bench.sq_file(config)):
        with open(bench.sq_file(config)) as f:
            if json.load(f)["kernel_hash"] == bench.kernel_hash():
                flops = bench.fp64_flops_for("solve_x")
                assert flops is not None and flops > 100 * 8192 * 8192


def test_step_count_must_be_positive():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "0"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "--steps" in r.stderr
