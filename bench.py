#!/usr/bin/env python3
"""Benchmark of the GRMHD block update with refinement and local time stepping on one
MI355X.

Workload: the batched refinement + time-level grid -- the Fishbone-Moncrief torus with a
single-loop field (plasma beta 100) and a seeded 2% u_g perturbation on an effective
512x256x256 log-spherical Kerr-Schild grid (a = 0.9375, r in [1.2, 50]) in 1344 blocks
of 64x32x32, 32x16x16 and 16x8x8 cells, phi halved per level toward each pole (3
levels), 4 time levels by radius (dt ratios 1:2:4:8), PPM + HLLE, FP64 midpoint steps,
inversion tolerance 1e-12.  A step is one LAT cycle (8 finest substeps).  Inputs are
resident in HBM before the timed region.  Paths timed on the same initial state:
  batched_learned   one launch per time level and kernel class over a work list of the
                    level's blocks, each cycle one captured graph, learned first guess
                    of the inversion (the headline)
  batched           the same with the plain (previous-state) guess
  plain             one launch per block and kernel class in the same LAT order (the
                    paper's launch structure), plain guess
  global_dt         the same blocks on one global time step, batched launches
  emf_upwind        the headline path with Gardiner & Stone's upwinded edge EMFs
  floor_drift       the headline path with the floors in the drift frame
  disk5             the large tilted thin disk (effective 1024x384x384, density-refined,
                    five time levels), batched launches + learned guess
The headline value is real zone-cycles/s (cells x their own steps / wall time), the
median of `runs` runs of exactly `steps` cycles; LAT-effective and refinement-and-LAT-
effective rates are reported beside it.  The roofline block reports the dominant kernel
class of a profiled batched run (HIP events on the library's stream), against the
algorithmic bytes of the method's state.  The CPU oracle runs on a bounded sample on the
host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "zone-cycles/s on 1 MI355X: batched AMR/LAT + learned con2prim vs plain"
PEAK = {"hbm": 8.0e12, "alu": 78.6e12}        # B/s; FP64 vector flop/s
WORKLOAD = "torus-eff512x256x256-amr-lat4-1344blocks-ppm-hlle"

# Algorithmic bytes per unit of each kernel class (units: interior cell-stages for the
# update, faces for flux kernels).  The update's figure is the method's state only: per
# zone-cycle 320 B (the predictor reads P^n, B^n and writes P*, B*: 128 B; the corrector
# reads P*, B*, P^n, B^n and writes P^(n+1), B^(n+1): 192 B), 160 B per cell-stage on
# average.  Flux kernels: the reconstructed state and the flux they write, 128 B per face
# (their traffic is an intermediate of the split design).
BYTES_PER_UNIT = {"update": 160, "flux1": 128, "flux2": 128, "flux3": 128}
# The design's own bytes per update cell-stage (P^n, B^n, stage P and cell B, the fluxes
# of six conserved components on one face per direction, 3 EMFs, P and B out).
DESIGN_BYTES_UPDATE = 8 * (5 + 3 + 5 + 3 + 6 * 3 + 3 + 5 + 3)
# FP64 flops per unit counted with SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64 (FMA = 2) on the
# kernels of hash KERNEL_HASH, and HBM traffic per unit from FETCH_SIZE / WRITE_SIZE
# (scaled by the same counters' reading for a device copy of known size); None where not
# measured on the current kernels.
FLOPS_PER_UNIT = {"update": 1458.1}
TRAFFIC_PER_UNIT = {"update": 463.4}
KERNEL_HASH = "0c259d9ef36eb724"


def kernel_hash() -> str:
    """hash of the sources the stage kernels are compiled from and of the compiler flags"""
    from paper_1912_10192_amd import build

    h = hashlib.sha256()
    for f in ("kernels.hip", "device.h", "internal.h", "wave.h", "mlp.h"):
        with open(os.path.join(ROOT, "paper_1912_10192_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(build.FLAGS).encode())
    return h.hexdigest()[:16]


def units(cls, blocks, steps_per_level):
    """units a kernel class processes over the cycles whose per-level step counts are
    given: cell-stages for the update, faces (with the transverse ghost rows the flux
    kernels also compute) for flux kernels"""
    tot = 0
    for b in blocks:
        n = b["n"]
        s = 2 * steps_per_level[b["lat"]]
        if cls == "update":
            tot += s * n[0] * n[1] * n[2]
        elif cls.startswith("flux"):
            d = int(cls[-1]) - 1
            f = 1
            for e in range(3):
                f *= n[e] + 1 if e == d else n[e] + 2
            tot += s * f
    return tot


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "cpus_available": avail}


def cpu_sample(steps):
    """one oracle process: a 64x32x32 block of the torus (the workload's largest block
    shape, PPM + HLLE, the same initial data at that resolution), `steps` steps; prints
    its zone-cycles and seconds"""
    import numpy as np

    import oracle
    from paper_1912_10192_amd import configs, initdata

    cfg = configs.scaled(configs.TORUS_UNIFORM, (64, 32, 32), ng=3)
    state = initdata.torus_state(cfg["n"], **configs.TORUS_INIT)
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
    print(json.dumps({"zone_cycles": N1 * N2 * N3 * steps, "seconds": dt}), flush=True)


def cpu_baseline(steps, procs, log):
    """the oracle as it stands (single-threaded C, one process per core) on independent
    samples, started together: aggregate zone-cycles/s over `procs` processes"""
    log(f"[bench] oracle: {procs} processes x {steps} steps of a 64x32x32 torus block")
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-sample", str(steps)]
    t0 = time.perf_counter()
    ps = [subprocess.Popen(cmd, stdout=subprocess.PIPE, text=True) for _ in range(procs)]
    outs = [p.communicate()[0] for p in ps]
    wall = time.perf_counter() - t0
    res = [json.loads(o.strip().splitlines()[-1]) for o in outs]
    zc = sum(r["zone_cycles"] for r in res)
    per = [r["zone_cycles"] / r["seconds"] for r in res]
    return {"value": zc / wall, "unit": "zone-cycles/s", "cores": procs, "kind": "oracle",
            "per_core": statistics.median(per),
            "sample": f"{procs} independent single-threaded oracle processes, each {steps} "
                      f"steps of a 64x32x32 block of the same torus (PPM + HLLE, FP64; the "
                      f"workload's largest block shape), {wall:.1f} s wall",
            "host": host_info()}


def c2p_summary(st):
    hist = list(st.c2p_iter_hist)
    n = sum(hist[:63])
    out = {"tier": list(st.c2p_tier), "floor_hits": st.floor_hits,
           "learned_guesses": st.mlp_guesses,
           "mean_newton_iters": (sum(i * h for i, h in enumerate(hist[:63])) / n) if n else None}
    tot = sum(st.c2p_tier)
    out["tier_rates"] = [t / tot for t in st.c2p_tier] if tot else None
    for q, name in ((0.5, "p50_newton_iters"), (0.99, "p99_newton_iters")):
        acc, val = 0, None
        for i, h in enumerate(hist[:63]):
            acc += h
            if n and acc >= q * n:
                val = i
                break
        out[name] = val
    return out


def train_guess(steps, log):
    """the learned inversion guess trained on the device: 5 snapshots of the uniform
    256x128x128 torus (steps 0, 50, 100, 150, 200, 2^20 seeded cells each) plus 5 M
    synthetic states"""
    import torch

    from paper_1912_10192_amd import configs, grmhd, initdata, learned

    t0 = time.perf_counter()
    cfg = dict(configs.TORUS_UNIFORM)
    state = initdata.torus_state(cfg["n"], **configs.TORUS_INIT)
    g = grmhd.Grid(cfg, state=state, batched=2)
    gen = torch.Generator(device="cpu").manual_seed(7)
    chunks = []
    for snap in range(5):
        if snap:
            g.step(50)
        P, B, G = g.extract_cells()
        idx = torch.randperm(P.shape[1], generator=gen)[:1 << 20].to(P.device)
        chunks.append((P[:, idx].contiguous(), B[:, idx].contiguous(), G[:, idx].contiguous()))
        last_G = G
    chunks.append(learned.synthetic_states(last_G, 5_000_000, seed=5))
    X, Y, norm = learned.build_dataset(chunks, cfg["gam"])
    del g, chunks, last_G
    trainer, losses = learned.train(X, Y, steps=steps, batch=4096, lr=2e-3, log_every=steps // 4)
    blob = grmhd.mlp_pack(trainer.params, norm)
    torch.cuda.synchronize()
    log(f"[bench] learned guess: {X.shape[0]} pairs, {steps} steps, losses {losses}")
    return blob, {"pairs": int(X.shape[0]), "steps": steps, "final_loss": losses[-1][1],
                  "train_s": time.perf_counter() - t0}


def run_leg(name, cfg, blocks, bs, batched, blob, steps, warmup, runs, sync, log, variants=None):
    """warmup cycles, then `runs` timed runs of exactly `steps` cycles each; the median run.
    Kernel variants: autotuned on the live state, or the given ones."""
    from paper_1912_10192_amd import grmhd

    g = grmhd.Grid(cfg, blocks=blocks, batched=batched, mlp_blob=blob)
    g.set_blocks(bs)
    if variants is None:
        tune = g.autotune()
    else:
        tune = None
        g.set_variants(flux=variants["flux"], update=variants["update"], split=variants["update_split"])
    L = max(b["lat"] for b in blocks) + 1
    log(f"[bench] {name}: {len(blocks)} blocks, {L} time levels, batched={batched}, "
        f"learned={blob is not None}; warmup {warmup}, {runs} runs of {steps} cycles")
    if warmup:
        g.step(warmup, stats=True)
    walls, stats = [], []
    for _ in range(runs):
        sync()
        t0 = time.perf_counter()
        st = g.step(steps, stats=True)
        sync()
        walls.append(time.perf_counter() - t0)
        stats.append(st)
    i = sorted(range(runs), key=lambda k: walls[k])[runs // 2]
    st, wall = stats[i], walls[i]
    out = {"value_real": st.real_zone_cycles / wall,
           "value_lat_effective": st.lat_eff_zone_cycles / wall,
           "value_amr_lat_effective": st.amr_lat_eff_zone_cycles / wall,
           "ms_per_cycle": wall * 1e3 / steps, "runs_ms_per_cycle": [w * 1e3 / steps for w in walls],
           "cycles_per_run": steps, "substeps_per_cycle": 2 ** (L - 1), "dt_min": st.dt_min,
           "steps_per_level": list(st.steps_per_level)[:L], "c2p": c2p_summary(st),
           "divb_rel_max": g.divb()[1]}
    if tune is not None:
        out["autotune"] = {"flux": tune["flux"], "update": tune["update"],
                           "update_split": tune["update_split"]}
    del g
    return out, tune


def profiled_classes(cfg, blocks, bs, blob, tune, steps, sync, log):
    """per kernel class time of the batched path (no graph; the HIP events time each class
    on the library's stream, the flux directions one after another)"""
    from paper_1912_10192_amd import grmhd

    g = grmhd.Grid(cfg, blocks=blocks, batched=2, profile=True, mlp_blob=blob)
    g.set_blocks(bs)
    g.set_variants(flux=tune["flux"], update=tune["update"], split=tune["update_split"])
    g.step(1, stats=True)
    st = g.step(steps, stats=True)
    sync()
    cls_ms = {k: st.class_ms[i] for i, k in enumerate(grmhd.KERNEL_CLASSES)}
    cls_n = {k: st.class_launches[i] for i, k in enumerate(grmhd.KERNEL_CLASSES)}
    L = max(b["lat"] for b in blocks) + 1
    spl = list(st.steps_per_level)[:L]
    log(f"[bench] profiled classes (ms per cycle): "
        + " ".join(f"{k}={v / steps:.3f}" for k, v in cls_ms.items()))
    del g
    return cls_ms, cls_n, spl


def roofline(cls_ms, cls_n, blocks, spl):
    dom = max((k for k in cls_ms if k in BYTES_PER_UNIT), key=lambda k: cls_ms[k])
    n_launch = max(cls_n[dom], 1)
    avg_s = cls_ms[dom] * 1e-3 / n_launch
    u = units(dom, blocks, spl) / n_launch                 # units per launch (mean)
    khash = kernel_hash()
    fresh = KERNEL_HASH == khash
    alg_bytes = BYTES_PER_UNIT[dom] * u
    flops = FLOPS_PER_UNIT.get(dom) if fresh else None
    t_hbm = alg_bytes / PEAK["hbm"]
    t_alu = flops * u / PEAK["alu"] if flops else 0.0
    if t_alu > t_hbm:
        bound, unit, peak, achieved, scale = "alu", "TFLOP/s", PEAK["alu"], flops * u / avg_s, 1e12
    else:
        bound, unit, peak, achieved, scale = "hbm", "GB/s", PEAK["hbm"], alg_bytes / avg_s, 1e9
    traffic = TRAFFIC_PER_UNIT.get(dom) * u if fresh and dom in TRAFFIC_PER_UNIT else None
    out = {"bound": bound, "achieved": achieved / scale, "peak": peak / scale, "unit": unit,
           "frac": achieved / peak, "traffic": traffic, "kernel": dom,
           "launch_ms": avg_s * 1e3, "launches": n_launch, "units_per_launch": u,
           "alg_bytes_per_unit": BYTES_PER_UNIT[dom], "kernel_hash": khash,
           "fp64_flops_per_unit": flops, "hbm_frac": t_hbm / avg_s,
           "alu_frac": (t_alu / avg_s) if flops else None}
    if dom == "update":
        out["design_bytes_per_unit"] = DESIGN_BYTES_UPDATE
        out["design_bytes_frac"] = DESIGN_BYTES_UPDATE * u / avg_s / PEAK["hbm"]
    return out


def regrid_leg(cfg, blocks, bs, sync, log):
    """Refinement during the run at full size (grmhd_regrid): the headline layout, after
    two cycles, regridded to its polar caps refined in phi and back.  Times the new
    layout's context set-up (planner and tables) and each regrid call; the round trip
    must return the state (prolongation along x3 followed by restriction is exact up to
    rounding, sqrt(-g) not varying along x3), and the refined layout runs a cycle."""
    import numpy as np

    from paper_1912_10192_amd import configs, grmhd

    fine = configs.refine_caps_phi(blocks)
    g = grmhd.Grid(cfg, blocks=blocks, batched=1)
    g.set_blocks(bs)
    g.step(2, stats=False)
    sync()
    t0 = time.perf_counter()
    g2 = grmhd.Grid(cfg, blocks=fine, batched=1)
    sync()
    t_init = time.perf_counter() - t0
    t0 = time.perf_counter()
    grmhd._check(grmhd.lib().grmhd_regrid(g.ctx, g2.ctx, grmhd.REGRID_PRIMITIVE))
    t_up = time.perf_counter() - t0
    g3 = grmhd.Grid(cfg, blocks=blocks, batched=1)
    sync()
    t0 = time.perf_counter()
    grmhd._check(grmhd.lib().grmhd_regrid(g2.ctx, g3.ctx, grmhd.REGRID_PRIMITIVE))
    t_down = time.perf_counter() - t0
    a, b = g.get_blocks(), g3.get_blocks()
    err = 0.0
    for x, y in zip(a, b):
        for u, v in zip(x, y):
            err = max(err, float(np.abs(u - v).max() / max(np.abs(u).max(), 1e-300)))
    _, div_rel = g2.divb()
    st = g2.step(1, stats=True)
    cells = sum(bb["n"][0] * bb["n"][1] * bb["n"][2] for bb in fine)
    log(f"[bench] regrid: caps refined in {t_up * 1e3:.1f} ms, back in {t_down * 1e3:.1f} ms, "
        f"new context {t_init:.2f} s, round trip {err:.1e}")
    del g2, g3
    # the density criterion on the evolved headline state: blocks whose densest cell
    # exceeds 0.5 split (a new finest level), the nesting rules split more; the decision,
    # the regrid and a cycle on the new layout
    from paper_1912_10192_amd import adapt

    t0 = time.perf_counter()
    rho = adapt.block_max(g)
    lay = adapt.Layout(cfg, blocks)
    new = lay.refine([1 if r > 0.5 else 0 for r in rho], max_level=3)
    # time levels from the blocks' Courant steps (a child half its parent's), at most 5
    lats = lay.time_levels(new, adapt.estimate_steps(lay.blocks, g.block_dt(), new), 5)
    t_decide = time.perf_counter() - t0
    plain = [dict({k: v for k, v in bb.items() if k != "parent"}, lat=l) for bb, l in zip(new, lats)]
    t0 = time.perf_counter()
    g4 = g.regrid(plain)
    sync()
    t_adapt = time.perf_counter() - t0
    st4 = g4.step(1, stats=True)
    cells4 = sum(bb["n"][0] * bb["n"][1] * bb["n"][2] for bb in plain)
    eff4 = list(g4.cfg["n"])
    log(f"[bench] density criterion: {sum(1 for r in rho if r > 0.5)} blocks flagged, "
        f"{len(plain)} blocks after nesting, time levels {sorted(set(lats))}, decided in "
        f"{t_decide:.2f} s, new context and regrid {t_adapt:.2f} s")
    del g, g4
    return {"layout": "headline layout <-> polar caps refined in phi (levels (0,0,0) -> (0,0,1))",
            "cells_refined_layout": cells, "context_setup_s": t_init,
            "regrid_refine_ms": t_up * 1e3, "regrid_derefine_ms": t_down * 1e3,
            "round_trip_max_rel": err, "divb_rel_refined": div_rel,
            "bad_states_next_cycle": st.bad_states,
            "density_criterion": {"threshold": 0.5, "flagged": sum(1 for r in rho if r > 0.5),
                                  "blocks_after": len(plain), "cells_after": cells4,
                                  "effective_grid_after": eff4,
                                  "time_levels_after": [lats.count(l) for l in range(max(lats) + 1)],
                                  "decide_s": t_decide, "context_and_regrid_s": t_adapt,
                                  "bad_states_next_cycle": st4.bad_states,
                                  "dt_min_next_cycle": st4.dt_min}}


def disk_leg(args, blob, sync, log):
    """the large tilted thin disk: effective 1024x384x384 on r in [1.2, 1000], density-
    refined blocks with phi-halved polar caps, five time levels (a cycle is 16 finest
    substeps), batched launches + learned guess"""
    from paper_1912_10192_amd import configs, initdata

    cfg = dict(configs.DISK5)
    blocks = configs.disk_blocks(cfg["n"])
    procs = min(16, host_info()["cpus_available"] or 1)
    t0 = time.perf_counter()
    bs = initdata.disk_block_states(cfg, blocks, procs=procs)
    log(f"[bench] disk5: {len(blocks)} blocks, initial data in {time.perf_counter() - t0:.1f} s")
    cycles = max(1, args.steps // 5)
    out, _ = run_leg("disk5_batched_learned", cfg, blocks, bs, 1, blob, cycles, 1,
                     max(3, args.runs // 2), sync, log)
    out["workload"] = cfg["name"]
    out["blocks"] = len(blocks)
    out["cells"] = sum(b["n"][0] * b["n"][1] * b["n"][2] for b in blocks)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="LAT cycles per timed run")
    ap.add_argument("--warmup", type=int, default=2, help="untimed cycles first")
    ap.add_argument("--runs", type=int, default=5, help="timed runs (the median is reported)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=40, help="oracle steps per process")
    ap.add_argument("--cpu-procs", type=int, default=0, help="oracle processes (0: the cores available, at most 16)")
    ap.add_argument("--cpu-sample", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--only-headline", action="store_true",
                    help="only the headline path (with its training) and the per-class profiled "
                         "run that gives the roofline, for profiling them alone")
    ap.add_argument("--only-regrid", action="store_true",
                    help="only the regrid leg on the headline layout (for profiling it alone)")
    ap.add_argument("--train-steps", type=int, default=1000)
    ap.add_argument("--plain-guess", action="store_true",
                    help="no learned guess: the headline path with the previous-state guess "
                         "(for hardware-counter runs)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (calibrates the "
                         "FETCH_SIZE/WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.cpu_sample:
        cpu_sample(args.cpu_sample)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_1912_10192_amd import configs, initdata

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

    cfg = dict(configs.TORUS_AMR3)
    blocks = configs.amr_lat_blocks(cfg["n"], lat_edges=cfg["lat_edges"])
    lmax = [max(b["lev"][d] for b in blocks) for d in range(3)]
    log(f"[bench] building initial state, effective {cfg['n']}, {len(blocks)} blocks")
    state = initdata.torus_state(cfg["n"], **configs.TORUS_INIT)
    bs = initdata.block_states(state, blocks, lmax)
    del state
    cells = sum(b["n"][0] * b["n"][1] * b["n"][2] for b in blocks)
    if args.only_regrid:
        print(json.dumps({"regrid": regrid_leg(cfg, blocks, bs, sync, log)}), flush=True)
        return
    blob, train = (None, None) if args.plain_guess else train_guess(args.train_steps, log)
    head, tune = run_leg("batched_learned", cfg, blocks, bs, 1, blob, args.steps, args.warmup,
                         args.runs, sync, log)
    out = {"metric": METRIC, "unit": "zone-cycles/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "runs": args.runs, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "value": head["value_real"], "ms_per_step": head["ms_per_cycle"],
           "config": {"workload": WORKLOAD, "effective_grid": list(cfg["n"]),
                      "blocks": len(blocks), "cells": cells,
                      "block_shapes": ["64x32x32", "32x16x16", "16x8x8"],
                      "time_levels": 4, "recon": "PPM", "riemann": "HLLE",
                      "c2p_tol": cfg["tol"], "step": "one LAT cycle (8 finest substeps)",
                      "path": "batched launches per time level, graph-captured cycle, "
                              "learned first guess",
                      "value_definition": "real zone-cycles/s (cells x their own steps / "
                                          "wall time), median of the timed runs"},
           "lat_effective": head["value_lat_effective"],
           "amr_lat_effective": head["value_amr_lat_effective"],
           "batched_learned": head}
    if not args.only_headline:
        batched, _ = run_leg("batched", cfg, blocks, bs, 1, None, args.steps, args.warmup,
                             args.runs, sync, log)
        plain, _ = run_leg("plain", cfg, blocks, bs, 0, None, args.steps, args.warmup,
                           args.runs, sync, log, variants=tune)
        upw, _ = run_leg("emf_upwind", dict(cfg, emf=1), blocks, bs, 1, blob, args.steps,
                         args.warmup, args.runs, sync, log, variants=tune)
        drift, _ = run_leg("floor_drift", dict(cfg, floor_frame=1), blocks, bs, 1, blob,
                           args.steps, args.warmup, args.runs, sync, log, variants=tune)
        flat = [dict(b, lat=0) for b in blocks]
        gsteps = args.steps * head["substeps_per_cycle"]
        glob, _ = run_leg("global_dt", cfg, flat, bs, 2, None, gsteps, args.warmup, args.runs,
                          sync, log)
        rg = regrid_leg(cfg, blocks, bs, sync, log)
        disk = disk_leg(args, blob, sync, log)
        cls_ms, cls_n, spl = profiled_classes(cfg, blocks, bs, blob, tune, args.steps, sync, log)
        out.update({
            "roofline": roofline(cls_ms, cls_n, blocks, spl),
            "kernel_ms_per_cycle": {k: v / args.steps for k, v in cls_ms.items()},
            "batched": batched, "plain": plain, "global_dt": glob, "disk5": disk,
            "emf_upwind": upw, "regrid": rg,
            "emf_upwind_cost": head["value_real"] / upw["value_real"],
            "floor_drift": drift,
            "floor_drift_cost": head["value_real"] / drift["value_real"],
            "speedup_vs_plain": head["value_real"] / plain["value_real"],
            "batching_gain": batched["value_real"] / plain["value_real"],
            "learned_gain": head["value_real"] / batched["value_real"],
            "speedup_vs_global_dt_real": head["value_real"] / glob["value_real"],
            "learned_training": train})
    else:
        cls_ms, cls_n, spl = profiled_classes(cfg, blocks, bs, blob, tune, args.steps, sync, log)
        out.update({"roofline": roofline(cls_ms, cls_n, blocks, spl),
                    "kernel_ms_per_cycle": {k: v / args.steps for k, v in cls_ms.items()},
                    "learned_training": train})
    if not args.no_cpu_baseline:
        avail = host_info()["cpus_available"] or 1
        procs = args.cpu_procs or min(avail, 16)
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps, procs, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
