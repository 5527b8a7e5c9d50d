#!/usr/bin/env python3
"""Benchmark of the GRMHD block update on one MI355X.

Workload: one GPU's share of a uniform grid -- the Fishbone-Moncrief torus with a
single-loop field (plasma beta 100) and a seeded 2% u_g perturbation on a 256x128x128
log-spherical Kerr-Schild grid (a = 0.9375, r in [1.2, 50]), split into 128 blocks of
32^3, PPM + HLLE, FP64 midpoint steps.  Inputs are resident in HBM before the timed
region.  Three paths are timed on the same initial state:
  plain                 global time step, one launch per kernel and stage, plain guess
  lat_batched           local time stepping with 4 levels by radius, each cycle one
                        captured graph, plain guess
  lat_batched_learned   the same with the learned first guess of the inversion
  polar_smr_lat_batched_learned
                        the same effective grid with coarser polar bands (half
                        resolution within pi/4 of the poles, a quarter in phi within
                        pi/8), reported as refinement-and-LAT-effective zone-cycles/s
The headline value is the last one's LAT-effective zone-cycles/s (every cell advanced by
every finest-level step, per second of wall time).  The roofline block reports the
dominant kernel of the plain run (average launch time from HIP events on the library's
stream during its timed region); the CPU oracle is timed on a bounded sample.
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

# Per-unit algorithmic figures of each kernel class:
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
# (flux entries: the variant the autotuner picked in the profiled run -- one face per
# thread for x1, two faces per thread for x2 and x3)
FLOPS_PER_UNIT = {
    "update": 1592.1, "flux1": 1013.0, "flux2": 899.8, "flux3": 840.7, "emf": 9.8,
    "bcell": 86.2, "dt": 330.0,
}
KERNEL_HASH = "4ccf50f64ad8e3e6"
# HBM traffic per launch from rocprofv3 FETCH_SIZE/WRITE_SIZE (scaled by the reading of
# the same counters for a 1 GiB device copy: fetch x2, write x1), keyed like
# FLOPS_PER_UNIT and valid for KERNEL_HASH only.
TRAFFIC_PER_LAUNCH = {
    "update": 1.921e9, "flux1": 7.295e8, "flux2": 7.999e8, "flux3": 7.785e8, "emf": 3.782e8,
    "bcell": 3.629e8,
}


def kernel_hash() -> str:
    """hash of the sources the stage kernels are compiled from and of the compiler flags"""
    from paper_1912_10192_amd import build

    h = hashlib.sha256()
    for f in ("kernels.hip", "device.h", "internal.h", "wave.h", "mlp.h"):
        with open(os.path.join(ROOT, "paper_1912_10192_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(build.FLAGS).encode())
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


def timed(grid, cycles, sync):
    sync()
    t0 = time.perf_counter()
    st = grid.step(cycles, stats=True)
    sync()
    return st, time.perf_counter() - t0


def c2p_summary(st):
    hist = list(st.c2p_iter_hist)
    n = sum(hist[:63])
    return {"tier": list(st.c2p_tier), "floor_hits": st.floor_hits,
            "learned_guesses": st.mlp_guesses,
            "mean_newton_iters": (sum(i * h for i, h in enumerate(hist[:63])) / n) if n else None}


def train_guess(cfg, state, steps, log):
    """train the learned inversion guess on the initial cells plus synthetic states"""
    import torch

    from paper_1912_10192_amd import grmhd, learned

    t0 = time.perf_counter()
    g = grmhd.Grid(cfg, state=state)
    g.step(2)
    P, B, G = g.extract_cells()
    chunks = [(P, B, G), learned.synthetic_states(G, 1_000_000, seed=5)]
    X, Y, norm = learned.build_dataset(chunks, cfg["gam"])
    del g, chunks
    trainer, losses = learned.train(X, Y, steps=steps, batch=4096, lr=2e-3, log_every=steps // 4)
    blob = grmhd.mlp_pack(trainer.params, norm)
    torch.cuda.synchronize()
    log(f"[bench] learned guess: {X.shape[0]} pairs, {steps} steps, losses {losses}")
    return blob, {"pairs": int(X.shape[0]), "steps": steps, "final_loss": losses[-1][1],
                  "train_s": time.perf_counter() - t0}


def lat_learned_only(args, cfg, state, cells, sync, log):
    """the headline path alone: batched LAT with the learned guess on the benchmark torus"""
    from paper_1912_10192_amd import grmhd

    lats = grmhd.lat_levels_by_radius(cfg, [2.4, 4.8, 9.6])
    nsub = 2 ** max(lats)
    cycles = max(args.steps // nsub, 1)
    blob, train = train_guess(cfg, state, args.train_steps, log)
    g = grmhd.Grid(cfg, blocks=grmhd.uniform_blocks(cfg["n"], cfg["block"], lats=lats),
                   batched=True, mlp_blob=blob)
    g.set_state(*state)
    g.autotune()
    log(f"[bench] lat_batched_learned only: levels {lats}, timed {cycles} cycles")
    g.step(1, stats=True)
    st, wall = timed(g, cycles, sync)
    print(json.dumps({"metric": METRIC, "unit": "zone-cycles/s", "n_gpus": 1,
                      "steps": cycles * nsub, "value": st.lat_eff_zone_cycles / wall,
                      "ms_per_cycle": wall * 1e3 / cycles, "higher_is_better": True,
                      "dtype": "f64", "data": "synthetic", "learned_training": train,
                      "config": {"workload": "torus-256x128x128-b32-ppm-hlle",
                                 "path": "batched LAT + learned guess", "lat_levels": lats,
                                 "cells": cells}}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="finest-level steps")
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--only-plain", action="store_true")
    ap.add_argument("--only-lat-learned", action="store_true",
                    help="only the headline path (batched LAT + learned guess, with its "
                         "training), for profiling it on its own; no plain path and no roofline")
    ap.add_argument("--train-steps", type=int, default=1000)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (calibrates the "
                         "FETCH_SIZE/WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_1912_10192_amd import configs, grmhd, initdata

    log = lambda m: print(m, file=sys.stderr, flush=True)
    sync = torch.cuda.synchronize
    if args.copy_probe:
        n = args.copy_probe << 17
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        sync()
        log(f"[bench] copy probe: 3 copies of {args.copy_probe} MiB")
        return
    cfg = dict(configs.TORUS_UNIFORM)
    log(f"[bench] building initial state {cfg['n']}")
    state = initdata.torus_state(cfg["n"], **configs.TORUS_INIT)
    cells = cfg["n"][0] * cfg["n"][1] * cfg["n"][2]

    if args.only_lat_learned:
        lat_learned_only(args, cfg, state, cells, sync, log)
        return

    # ---- plain path: global time step, one launch per kernel and stage, plain guess
    grid = grmhd.Grid(cfg, state=state, profile=True)
    tune = grid.autotune()
    log(f"[bench] autotuned variants {tune}")
    log(f"[bench] plain: warmup {args.warmup}, timed {args.steps} steps")
    if args.warmup:
        grid.step(args.warmup, stats=True)
    st, wall = timed(grid, args.steps, sync)
    a_div, r_div = grid.divb()
    cls_ms = {k: st.class_ms[i] for i, k in enumerate(grmhd.KERNEL_CLASSES)}
    cls_n = {k: st.class_launches[i] for i, k in enumerate(grmhd.KERNEL_CLASSES)}
    dom = max(cls_ms, key=lambda k: cls_ms[k])
    avg_s = cls_ms[dom] / max(cls_n[dom], 1) * 1e-3
    units = units_per_launch(dom, cfg)
    khash = kernel_hash()
    fresh = KERNEL_HASH == khash
    # the binding roof: the larger of the algorithmic byte time and flop time
    alg_bytes = BYTES_PER_UNIT[dom] * units
    alg_flops = FLOPS_PER_UNIT[dom] * units if fresh and dom in FLOPS_PER_UNIT else None
    t_hbm = alg_bytes / PEAK["hbm"]
    t_alu = alg_flops / PEAK["alu"] if alg_flops is not None else 0.0
    if t_alu > t_hbm:
        bound, unit, peak, achieved, scale = "alu", "TFLOP/s", PEAK["alu"], alg_flops / avg_s, 1e12
    else:
        bound, unit, peak, achieved, scale = "hbm", "GB/s", PEAK["hbm"], alg_bytes / avg_s, 1e9
    traffic = TRAFFIC_PER_LAUNCH.get(dom) if fresh else None
    roofline = {"bound": bound, "achieved": achieved / scale, "peak": peak / scale, "unit": unit,
                "frac": achieved / peak, "traffic": traffic, "kernel": dom,
                "launch_ms": avg_s * 1e3, "units_per_launch": units, "kernel_hash": khash,
                "alg_bytes_per_unit": BYTES_PER_UNIT[dom],
                "fp64_flops_per_unit": FLOPS_PER_UNIT.get(dom) if fresh else None,
                "hbm_frac": t_hbm / avg_s,
                "alu_frac": (t_alu / avg_s) if alg_flops is not None else None}
    del grid
    # the plain path's rate from a run without the per-class HIP events (which also keep
    # the three flux directions in sequence); the profiled run above gives the classes
    grid = grmhd.Grid(cfg, state=state)
    grid.set_variants(flux=tune["flux"], update=tune["update"], split=tune["update_split"])
    if args.warmup:
        grid.step(args.warmup, stats=True)
    st_u, wall_u = timed(grid, args.steps, sync)
    del grid
    plain_value = cells * args.steps / wall_u
    plain = {"value": plain_value, "ms_per_step": wall_u * 1e3 / args.steps, "dt": st_u.dt_min,
             "profiled_ms_per_step": wall * 1e3 / args.steps, "autotune": tune,
             "c2p": c2p_summary(st), "divb_rel_max": r_div,
             "kernel_ms_per_step": {k: v / args.steps for k, v in cls_ms.items()}}

    out = {"metric": METRIC, "unit": "zone-cycles/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic"}
    if args.only_plain:
        out.update({"value": plain_value, "ms_per_step": plain["ms_per_step"],
                    "config": {"workload": "torus-256x128x128-b32-ppm-hlle", "path": "plain"},
                    "roofline": roofline, "plain": plain})
    else:
        # ---- batched local time stepping: 4 levels by radius, graph-captured cycles
        lats = grmhd.lat_levels_by_radius(cfg, [2.4, 4.8, 9.6])
        L = max(lats) + 1
        nsub = 2 ** (L - 1)
        cycles = max(args.steps // nsub, 1)
        blocks = grmhd.uniform_blocks(cfg["n"], cfg["block"], lats=lats)
        smr = configs.polar_smr_blocks(cfg["n"], cfg["block"][0], lats)
        results = {}
        blob, train = None, None
        for name, bl, learned_on in (("lat_batched", blocks, False),
                                     ("lat_batched_learned", blocks, True),
                                     ("polar_smr_lat_batched_learned", smr, True)):
            if learned_on and blob is None:
                blob, train = train_guess(cfg, state, args.train_steps, log)
            g = grmhd.Grid(cfg, blocks=bl, batched=True, mlp_blob=blob if learned_on else None)
            if bl is smr:
                lmax = [max(b["lev"][d] for b in bl) for d in range(3)]
                g.set_blocks(initdata.block_states(state, bl, lmax))
            else:
                g.set_state(*state)
            g.autotune()
            log(f"[bench] {name}: {len(bl)} blocks, levels {lats}, warmup 1 cycle, "
                f"timed {cycles} cycles of {nsub} substeps")
            g.step(1, stats=True)
            st, wall = timed(g, cycles, sync)
            results[name] = {"value_lat_effective": st.lat_eff_zone_cycles / wall,
                             "value_amr_lat_effective": st.amr_lat_eff_zone_cycles / wall,
                             "value_real": st.real_zone_cycles / wall,
                             "ms_per_cycle": wall * 1e3 / cycles, "cycles": cycles,
                             "substeps_per_cycle": nsub, "dt_min": st.dt_min,
                             "steps_per_level": list(st.steps_per_level)[:L],
                             "cells": sum(b["n"][0] * b["n"][1] * b["n"][2] for b in bl),
                             "c2p": c2p_summary(st), "divb_rel_max": g.divb()[1]}
            del g
        head = results["lat_batched_learned"]
        out.update({
            "value": head["value_lat_effective"],
            "ms_per_step": head["ms_per_cycle"] / nsub,
            "config": {"workload": "torus-256x128x128-b32-ppm-hlle", "grid": list(cfg["n"]),
                       "blocks": 128, "block": list(cfg["block"]), "recon": "PPM",
                       "riemann": "HLLE", "c2p_tol": cfg["tol"],
                       "path": "batched LAT (levels by radius, graph-captured cycle) + learned guess",
                       "lat_levels": lats, "value_definition": "LAT-effective zone-cycles/s "
                       "(all cells x finest-level steps / wall time)"},
            "roofline": roofline,
            "plain": plain,
            "lat_batched": results["lat_batched"],
            "lat_batched_learned": head,
            "polar_smr_lat_batched_learned": results["polar_smr_lat_batched_learned"],
            "learned_training": train,
            "speedup_vs_plain": head["value_lat_effective"] / plain_value,
        })
    if not args.no_cpu_baseline:
        log(f"[bench] oracle on host, {args.cpu_steps} step(s) of the same grid")
        rate, secs = cpu_baseline(cfg, state, args.cpu_steps)
        out["cpu_baseline"] = {"value": rate, "unit": "zone-cycles/s", "cores": 1, "kind": "oracle",
                               "sample": f"{args.cpu_steps} full step(s) of the 256x128x128 grid "
                                         f"from the same initial state, single-threaded, {secs:.1f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
