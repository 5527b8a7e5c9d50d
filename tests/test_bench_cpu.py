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
    """360 B per cell for the update: P^n, B^n faces, stage P, stage cell-centred B,
    the fluxes of 6 conserved components on one face per direction (each face is shared
    by two cells), 3 EMFs, P and B out; 128 B per face for a flux kernel.  Units per launch on the
    256x128x128 torus in 32^3 blocks: cells, and faces with the transverse ghost rows."""
    assert bench.BYTES_PER_UNIT["update"] == 360
    assert all(bench.BYTES_PER_UNIT[f"flux{d}"] == 128 for d in (1, 2, 3))
    cfg = dict(configs.TORUS_UNIFORM)
    assert bench.units_per_launch("update", cfg) == 256 * 128 * 128
    assert bench.units_per_launch("flux1", cfg) == 128 * 33 * 34 * 34
    assert bench.units_per_launch("flux3", cfg) == 128 * 34 * 34 * 33


def test_counted_constants_belong_to_the_current_kernels():
    """the counted flops and traffic in bench.py were taken on the kernels as they stand
    (a kernel change must come with fresh counters, else the bench reports them as null)"""
    h = bench.kernel_hash()
    assert len(h) == 16 and all(ch in "0123456789abcdef" for ch in h)
    assert h == bench.KERNEL_HASH


@pytest.mark.parametrize("name", ["build", "smoke"])
def test_entry_points_exist(name):
    import __graft_entry__ as g

    assert callable(getattr(g, name))
