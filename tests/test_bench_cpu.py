"""The benchmark's contract checked on the CPU: the one-GPU rule, the per-unit figures
behind its roofline line, and that the counted constants belong to the current kernels."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1912_10192_amd import configs  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_algorithmic_bytes_and_units():
    """the update's algorithmic bytes are the method's state: 320 B per zone-cycle, 128 B
    in the predictor (P^n, B^n in, P*, B* out) and 192 B in the corrector (P*, B*, P^n, B^n
    in, P^(n+1), B^(n+1) out), 160 B per cell-stage; 128 B per face for a flux kernel.
    Units over a cycle of the batched workload: two cell-stages per cell-step, faces with
    the transverse ghost rows."""
    assert bench.BYTES_PER_UNIT["update"] * 2 == 128 + 192
    assert all(bench.BYTES_PER_UNIT[f"flux{d}"] == 128 for d in (1, 2, 3))
    blocks = configs.amr_lat_blocks((512, 256, 256))
    spl = [8, 4, 2, 1]
    cell_steps = sum(b["n"][0] * b["n"][1] * b["n"][2] * spl[b["lat"]] for b in blocks)
    assert cell_steps == 3506176 * 8 + 3375104 * 4 + 4554752 * 2 + 6914048
    assert bench.units("update", blocks, spl) == 2 * cell_steps
    one = [dict(n=(32, 16, 16), lat=0)]
    assert bench.units("flux1", one, [1]) == 2 * 33 * 18 * 18
    assert bench.units("flux3", one, [1]) == 2 * 34 * 18 * 17


def test_counted_constants_belong_to_the_current_kernels():
    """the counted flops and traffic in bench.py were taken on the kernels as they stand
    (a kernel change must come with fresh counters, else the bench reports them as null)"""
    h = bench.kernel_hash()
    assert len(h) == 16 and all(ch in "0123456789abcdef" for ch in h)
    if bench.FLOPS_PER_UNIT or bench.TRAFFIC_PER_UNIT:
        assert h == bench.KERNEL_HASH


def test_cpu_sample_runs():
    """one oracle sample process (a few steps) reports its zone-cycles and seconds"""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--cpu-sample", "1"],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["zone_cycles"] == 64 * 32 * 32 and out["seconds"] > 0


@pytest.mark.parametrize("name", ["build", "smoke"])
def test_entry_points_exist(name):
    import __graft_entry__ as g

    assert callable(getattr(g, name))
