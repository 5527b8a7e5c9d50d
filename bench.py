#!/usr/bin/env python3
"""Benchmark of the GRMHD block update on one MI355X.

Workload: one GPU's share of a uniform grid -- the Fishbone-Moncrief torus with a
single-loop field (plasma beta 100) and a seeded 2% u_g perturbation on a 256x128x128
log-spherical Kerr-Schild grid (a = 0.9375, r in [1.2, 50]), split into 128 blocks of
32^3, PPM + HLLE, FP64 midpoint steps.  Inputs are resident in HBM before the timed
region.  Prints one JSON line: zone-cycles/s (cells x steps / wall time), the roofline
position of the dominant kernel (average launch time from HIP events on the library's
stream during the timed region) and the CPU oracle's rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "zone-cycles/s on 1 MI355X: batched AMR/LAT + learned con2prim vs plain"
PEAK = {"hbm": 8.0e12, "alu": 78.6e12}        # B/s; FP64 vector flop/s

# Per-unit algorithmic figures of each kernel class (derivation in the design doc):
# bytes = the unique HBM bytes a launch must move per unit (each input read once, each
# output written once); flops = FP64 flops per unit executed by the kernel, counted with
# the SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64 counters (FMA = 2) on this workload and
# divided by the units of that launch.  Units: faces for flux kernels, interior cells
# otherwise.  FLOPS entries are valid for the kernel source hash KERNEL_HASH only.
BYTES_PER_UNIT = {
    "flux1": 8 * (5 + 2 + 1 + 8), "flux2": 8 * (5 + 2 + 1 + 8), "flux3": 8 * (5 + 2 + 1 + 8),
    "update": 8 * (5 + 3 + 5 + 3 + 6 * 3 + 3 + 5 + 3),
    "emf": 8 * (6 + 3), "bcell": 8 * (3 + 3), "dt": 8 * (5 + 3), "ghost": 8 * 2 * 8,
}
FLOPS_PER_UNIT: dict = {}
KERNEL_HASH = None
# HBM traffic per launch from rocprofv3 FETCH_SIZE/WRITE_SIZE (calibrated on the copy
# kernel), keyed like FLOPS_PER_UNIT and valid for KERNEL_HASH only.
TRAFFIC_PER_LAUNCH: dict = {}


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "device.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_1912_10192_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def units_per_launch(cls, cfg):
    nb = 1
    for d in range(3):
        nb *= cfg["n"][d] // cfg["block"][d]
    b = cfg["block"]
    if cls.startswith("flux"):
        d = int(cls[-1]) - 1
        u = 1
        for e in range(3):
            u *= b[e] + 1 if e == d else b[e] + 2
        return nb * u
    return nb * b[0] * b[1] * b[2]


def cpu_baseline(cfg, state, steps):
    """the oracle, single-threaded, on the same initial state for `steps` steps"""
    import numpy as np

    import oracle

    g = oracle.Grid(cfg)
    ng = cfg["ng"]
    N1, N2, N3 = cfg["n"]
    Pp, Bp = g.zeros()
    P, B1, B2, B3 = state
    Pp[:, ng:ng + N3, ng:ng + N2, ng:ng + N1] = P
    Bp[0, ng:ng + N3, ng:ng + N2, ng:ng + N1 + 1] = B1
    Bp[1, ng:ng + N3, ng:ng + N2 + 1, ng:ng + N1] = B2
    Bp[2, ng:ng + N3 + 1, ng:ng + N2, ng:ng + N1] = B3
    t0 = time.perf_counter()
    g.step(Pp, Bp, steps)
    dt = time.perf_counter() - t0
    assert np.isfinite(Pp).all()
    return N1 * N2 * N3 * steps / dt, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=1)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_1912_10192_amd import configs, grmhd, initdata

    cfg = dict(configs.TORUS_UNIFORM)
    print(f"[bench] building initial state {cfg['n']}", file=sys.stderr, flush=True)
    state = initdata.torus_state(cfg["n"], **configs.TORUS_INIT)
    grid = grmhd.Grid(cfg, state=state, profile=True)
    cells = cfg["n"][0] * cfg["n"][1] * cfg["n"][2]
    print(f"[bench] warmup {args.warmup} steps", file=sys.stderr, flush=True)
    if args.warmup:
        grid.step(args.warmup, stats=True)
    torch.cuda.synchronize()
    print(f"[bench] timed {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    st = grid.step(args.steps, stats=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = cells * args.steps / wall
    a_div, r_div = grid.divb()

    cls_ms = {k: st.class_ms[i] for i, k in enumerate(grmhd.KERNEL_CLASSES)}
    cls_n = {k: st.class_launches[i] for i, k in enumerate(grmhd.KERNEL_CLASSES)}
    dom = max(cls_ms, key=lambda k: cls_ms[k])
    avg_s = cls_ms[dom] / max(cls_n[dom], 1) * 1e-3
    units = units_per_launch(dom, cfg)
    khash = kernel_hash()
    fresh = KERNEL_HASH == khash
    if fresh and dom in FLOPS_PER_UNIT:
        bound, unit, peak = "alu", "TFLOP/s", PEAK["alu"]
        achieved = FLOPS_PER_UNIT[dom] * units / avg_s
        scale = 1e12
    else:
        bound, unit, peak = "hbm", "GB/s", PEAK["hbm"]
        achieved = BYTES_PER_UNIT[dom] * units / avg_s
        scale = 1e9
    traffic = TRAFFIC_PER_LAUNCH.get(dom) if fresh else None
    roofline = {"bound": bound, "achieved": achieved / scale, "peak": peak / scale, "unit": unit,
                "frac": achieved / peak, "traffic": traffic, "kernel": dom,
                "launch_ms": avg_s * 1e3, "units_per_launch": units}

    out = {
        "metric": METRIC, "value": value, "unit": "zone-cycles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "torus-256x128x128-b32-ppm-hlle", "grid": list(cfg["n"]),
                   "blocks": 128, "block": list(cfg["block"]), "recon": "PPM",
                   "riemann": "HLLE", "c2p_guess": "plain", "c2p_tol": cfg["tol"],
                   "lat_levels": 1, "path": "plain"},
        "roofline": roofline,
        "kernel_ms_per_step": {k: v / args.steps for k, v in cls_ms.items()},
        "c2p": {"tier": list(st.c2p_tier), "mean_iters": None, "floor_hits": st.floor_hits},
        "divb_rel_max": r_div, "t_sim": st.t_sim, "dt": st.dt_min,
    }
    hist = list(st.c2p_iter_hist)
    nsolve = sum(hist[:63])
    if nsolve:
        out["c2p"]["mean_iters"] = sum(i * h for i, h in enumerate(hist[:63])) / nsolve
    del grid
    if not args.no_cpu_baseline:
        print(f"[bench] oracle on host, {args.cpu_steps} step(s) of the same grid", file=sys.stderr,
              flush=True)
        rate, secs = cpu_baseline(cfg, state, args.cpu_steps)
        out["cpu_baseline"] = {"value": rate, "unit": "zone-cycles/s", "cores": 1, "kind": "oracle",
                               "sample": f"{args.cpu_steps} full step(s) of the 256x128x128 grid "
                                         f"from the same initial state, single-threaded, {secs:.1f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
