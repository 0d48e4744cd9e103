"""Runs of the large workloads: throughput (GLUPS, fraction of the HBM
roofline) and the error of the reduced storages against the FP64 path.

    python -m paper_2301_00228_amd.workloads hole8192 --storage f16dev
    python -m paper_2301_00228_amd.workloads batch256 --storage f32dev
    python -m paper_2301_00228_amd.workloads large --storage f16dev

Prints one JSON line per run.  Every input is synthetic and seeded
(``inputs``); the state stays in HBM during the timed steps.
"""
import argparse
import json
import sys
import time

import numpy as np

from . import inputs, lbm

HBM_PEAK_GBS = 8000.0


def cases_for(name, steps):
    if name == "hole8192":
        return [inputs.plate_with_hole(n=8192, radius=1024, steps=steps)]
    if name == "batch256":
        return inputs.plate_batch(count=256, steps=steps)
    if name == "large":
        return inputs.large_batch(steps=steps)
    if name == "clamped1024":
        return [inputs.clamped_plate(n=1024, steps=steps)]
    raise ValueError(name)


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def timed(cases, storage, steps, warmup, tune=True, tiling=None, overlap=None):
    import torch
    t0 = time.perf_counter()
    ctx = lbm.context_for(cases, storage)
    setup = time.perf_counter() - t0
    print(f"context {storage}: {setup:.1f} s", file=sys.stderr, flush=True)
    ctx.step(2)
    if tiling:
        ctx.set_tiling(*tiling)
        if overlap is not None:
            ctx.use_overlap(overlap)
    elif tune:
        t1 = time.perf_counter()
        t_set = time.perf_counter()
        ctx.set_tiling(128, 16, 0, 4, 16, 2)
        t_set = time.perf_counter() - t_set
        print(f"one tiling set up in {t_set:.2f} s", file=sys.stderr, flush=True)
        # the autotuner sets up about 30 tilings
        if t_set < 4.0:
            ctx.autotune(3)
        i = ctx.info()
        print("tuned", [i["tile_lanes"], i["tile_rows"], i["tile_order"], i["tile_edge_rows"],
                        i["tile_align"], i["tile_steps"], i["tile_edge_cols"],
                        i["tile_stream_stores"]],
              f"in {time.perf_counter() - t1:.1f} s", file=sys.stderr, flush=True)
    ctx.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    info = ctx.info()
    prof = ctx.profile(4)
    # the dominant launch: with overlapped pairs the deep tiles' launch (two
    # steps of its nodes), else the first of a two-step pair (every body node
    # read and written once), else the single-step launch; achieved =
    # lattice updates x bytes per update / launch time
    kind = ("deep" if prof["deep"][1] > 0 else
            "two_step" if prof["two_step"][1] > 0 else "interior")
    i_ms, i_n = prof[kind]
    b_ms, b_n = prof["boundary"]
    per = i_ms / i_n / 1e3
    nodes = info["nodes_in_body"]
    streamed = info["nodes_deep"] if kind == "deep" else nodes
    achieved = streamed * info["bytes_per_update"] / per / 1e9

    def avg_us(k):
        return prof[k][0] / prof[k][1] * 1e3 if prof[k][1] else None
    res = {"storage": storage, "plates": info["n_plates"], "nodes": nodes, "steps": steps,
           "glups": nodes * steps / dt / 1e9, "ms_per_step": dt / steps * 1e3,
           "interior_kind": kind, "interior_us": per * 1e6, "interior_GBs": achieved,
           "interior_frac": achieved / HBM_PEAK_GBS, "boundary_us": b_ms / max(b_n, 1) * 1e3,
           "first_launch_us": avg_us("two_step"),
           "second_launch_us": avg_us("interior") if kind != "interior" else None,
           "overlap": bool(info["overlap"]), "deep_nodes": info["nodes_deep"],
           "two_step_nodes": info["nodes_two_step"],
           "bytes_per_lup": info["bytes_per_update"], "boundary_nodes": info["boundary_nodes"],
           "tile": [info["tile_lanes"], info["tile_rows"], info["tile_order"],
                    info["tile_edge_rows"], info["tile_align"], info["tile_steps"],
                    info["tile_edge_cols"], info["tile_stream_stores"]],
           "device_GB": info["device_bytes"] / 1e9, "setup_s": setup}
    return ctx, res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["hole8192", "batch256", "large", "clamped1024"])
    ap.add_argument("--storage", default="f16dev")
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--ref", default="f64",
                    help="storage of the reference run for the error ('' = no error)")
    ap.add_argument("--tiling", default="", metavar="L,R,O,E,A,S,W[,N]",
                    help="interior tiling instead of the autotuner's pick")
    ap.add_argument("--overlap", type=int, choices=(0, 1), default=None,
                    help="with --tiling: overlapped pairs on (1) or off (0); default on")
    ap.add_argument("--ref-plates", type=int, default=0,
                    help="compare only the first N plates and the last one (0 = all)")
    args = ap.parse_args()

    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    print(f"building {args.workload}", file=sys.stderr, flush=True)
    cases = cases_for(args.workload, args.warmup + args.steps)
    tiling = [int(v) for v in args.tiling.split(",")] if args.tiling else None
    overlap = None if args.overlap is None else bool(args.overlap)
    ctx, res = timed(cases, args.storage, args.steps, args.warmup, tiling=tiling, overlap=overlap)
    res["workload"] = args.workload
    print(json.dumps(res), flush=True)
    nodes_allocated = ctx.info()["nodes_allocated"]
    ctx.close()
    del ctx
    # the ceiling the state layout sets: a plain copy of the storage's own
    # arrays over as many nodes (after the context is gone, so that both
    # need not fit in memory at once)
    lc = lbm.layout_copy_rate(args.storage, nodes_allocated, 5)
    print(json.dumps({"workload": args.workload, "storage": args.storage,
                      "layout_copy_GBs": round(lc, 1),
                      "interior_frac_of_layout_copy": round(res["interior_GBs"] / lc, 4)}), flush=True)
    if args.ref:
        # Reference and reduced run plate by plate from t = 0 for the same
        # number of steps (bounds memory: the FP64 state of the whole batch
        # may not fit next to the reduced one).
        picks = list(range(len(cases)))
        if args.ref_plates and len(cases) > args.ref_plates + 1:
            picks = list(range(args.ref_plates)) + [len(cases) - 1]
        n_total = args.warmup + args.steps
        worst = {"e": 0.0, "omega": 0.0, "u": 0.0}
        per_plate = []
        for p in picks:
            outs = {}
            for st in (args.ref, args.storage):
                with lbm.context_for([cases[p]], st) as c:
                    c.step(n_total)
                    outs[st] = c.fields(0, want=("e", "omega", "u"))
            errs = {k: rel_l2(outs[args.storage][k], outs[args.ref][k]) for k in worst}
            for k in worst:
                worst[k] = max(worst[k], errs[k])
            per_plate.append((cases[p].name, errs))
            print(f"plate {cases[p].name}: {errs}", file=sys.stderr, flush=True)
        print(json.dumps({"workload": args.workload, "storage": args.storage, "ref": args.ref,
                          "steps": n_total, "plates_compared": len(picks),
                          "max_rel_l2": worst}), flush=True)


if __name__ == "__main__":
    main()
