"""Throughput benchmark of the plane-strain LBM hot path on one MI355X.

One "step" is one time step of the whole method (interior stream+collide
with the u recovery, boundary reset and accelerations, second-row rule,
synchronization every 50th step) on the workload below, with the state
resident in HBM.  Prints ONE JSON line.

Workload (the precision workload; FP64 is the headline value): 8192 x 8192
plate with a central circular hole of radius 1024 (traction-free rim), outer
edges clamped (u* = 0), nu = 0.3, a0_phi = 0.9999, one seeded Gaussian
displacement pulse (sigma 16, amplitude 1e-3) on the annulus around the
hole, synchronization every 50 steps.  The same workload is timed with the
FP32 and the reduced (deviation) storages; in an untimed leg every storage
runs on to step 2000, where the relative L2 error of e, omega and u of each
reduced storage against FP64 is taken.  The FP64 path itself is compared
with the CPU oracle on the same plate after the oracle's timed sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "hole8192"
PRECISION_STEPS = 2000
# Interior tilings (lanes, rows, order, edge rows, alignment, steps per pass,
# edge columns) and overlapped pairs (lbm_use_overlap) measured fastest for
# this workload on MI355X (sweeps of --tiling around the library
# autotuner's picks), pinned so that runs and the committed rocprofv3
# summaries use the same launches (--autotune tunes again instead).
TUNED = {"f64": ((256, 16, 3, 8, 16, 2, 16), False),
         "f32": ((256, 16, 3, 8, 16, 2, 16), False),
         "f32dev": ((256, 16, 3, 8, 16, 2, 16), False),
         "f16dev": ((256, 16, 3, 8, 16, 2, 16), False),
         "bf16dev": ((256, 16, 3, 8, 16, 2, 16), False)}
VARIANTS = ("f32", "f32dev", "f16dev", "bf16dev")
METRIC = "GLUPS + % HBM roofline, FP64 vs FP16/FP32-storage at ≤1e-3 rel L2"
KIND_NAMES = {"deep": "deep tiles of overlapped pairs", "two_step": "first launch of a two-step pair",
              "interior": "single-step launch"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("lbm_kernels.hip", "lbm_types.h", "lbm_host.cpp"):
        with open(os.path.join(ROOT, "paper_2301_00228_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(storage, kind, tile, overlap):
    """HBM bytes per launch of one interior-kernel kind from the committed
    rocprofv3 PMC summary of this workload, if it was taken on the current
    kernel and host sources (the host builds the tile lists) with the same
    tiling and overlap setting."""
    path = os.path.join(ROOT, "profiles", f"interior_{storage}_{WORKLOAD}_traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if (d.get("kernel_source_hash") != kernel_source_hash() or d.get("tile") != tile
            or d.get("overlap", False) != overlap):
        return None
    return d.get("kernels", {}).get(kind, {}).get("hbm_bytes_per_launch")


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_plate(case):
    from oracle import oracle

    p = oracle.OraclePlate(case.nx, case.ny, mask=case.mask, periodic=case.periodic,
                           lam=case.lam, mu=case.mu, rho=case.rho, dh=case.dh, dt=case.dt,
                           sync_every=case.sync_every, u0=case.u0, v0=case.v0)
    for bc in case.bcs:
        p.set_bc(bc.xy, bc.kind, bc.val, cell=bc.cell, knots=bc.knots)
    return p


def cpu_baseline(case, budget_s):
    """Time the FP64 oracle on a bounded sample of the same workload (the
    same plate from t = 0, as many steps as fit the budget, all its OpenMP
    threads; then one step on one thread).  Returns the record and the
    oracle plate (at its last step)."""
    from oracle import oracle

    t0 = time.perf_counter()
    p = oracle_plate(case)
    setup = time.perf_counter() - t0
    nodes = case.in_body_nodes()
    threads = oracle.threads()
    p.step(1)  # (thread start-up)
    t0 = time.perf_counter()
    p.step(1)
    one = time.perf_counter() - t0
    steps = max(2, int(budget_s / max(one, 1e-6)))
    t0 = time.perf_counter()
    p.step(steps)
    dt = time.perf_counter() - t0
    # one step on one thread beside it (the serial rate the threads scale from)
    oracle.set_threads(1)
    t0 = time.perf_counter()
    p.step(1)
    dt1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    rec = {"value": nodes * steps / dt / 1e9, "unit": "GLUPS", "cores": threads, "kind": "oracle",
           "sample": f"the same {case.nx}x{case.ny} holed plate from t = 0, {steps} steps "
                     f"(steps 3..{steps + 2}) timed, {dt:.1f} s wall ({setup:.0f} s set-up "
                     f"not counted)",
           "single_thread": {"value": nodes / dt1 / 1e9, "unit": "GLUPS", "steps": 1,
                             "wall_s": round(dt1, 2)},
           "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}
    return rec, p


def cpu_workloads():
    """The FP64 oracle on samples of the batched workloads (all its OpenMP
    threads): the first four plates of the 256-plate batch over 100 steps and
    the first 4096^2 plate of the 1.2 G-node batch over 20 steps, each plate
    from t = 0 after one untimed step."""
    from paper_2301_00228_amd import inputs

    out = {}
    for name, cases, steps in (("batch256", inputs.plate_batch(count=4, steps=0), 100),
                               ("large", inputs.large_batch(count=1, strip=None, steps=0), 20)):
        nodes = sum(c.in_body_nodes() for c in cases)
        plates = [oracle_plate(c) for c in cases]
        for p in plates:
            p.step(1)
        t0 = time.perf_counter()
        for p in plates:
            p.step(steps)
        dt = time.perf_counter() - t0
        out[name] = {"value": nodes * steps / dt / 1e6, "unit": "MLUPS",
                     "plates": [f"{c.nx}x{c.ny}" for c in cases], "steps": steps,
                     "wall_s": round(dt, 2)}
        del plates
    return out


def copy_rate_gbs(gib=2.0, reps=10):
    """A plain device-to-device copy (the library's copy probe) as the
    practical HBM ceiling."""
    from paper_2301_00228_amd import lbm
    return lbm.copy_rate(int(gib * 2**30), reps)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of timed oracle steps in the CPU baseline")
    ap.add_argument("--cpu-workloads", action="store_true",
                    help="also time the oracle on samples of the batched workloads")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the untimed leg to step 2000 and the rel L2 errors")
    ap.add_argument("--profile-steps", type=int, default=8)
    ap.add_argument("--storage", default="f64", help="storage of the headline run")
    ap.add_argument("--tiling", default="", metavar="L,R,O,E,A,S[,W[,N]]",
                    help="interior tiling of the headline storage (lanes, rows, order, edge "
                         "rows, alignment, steps, edge columns, stream stores) instead of the "
                         "pinned one")
    ap.add_argument("--overlap", type=int, default=-1, choices=(-1, 0, 1),
                    help="overlapped pairs of the headline storage (-1: the pinned choice)")
    ap.add_argument("--autotune", action="store_true",
                    help="run the library's autotuner instead of the pinned tilings")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="only run a plain device copy of this many GiB 5 times (counter "
                         "calibration for rocprofv3 --pmc) and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(a batch of plates would shard across GPUs with no communication)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2301_00228_amd import inputs, lbm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration > 0:
        n = int(args.copy_calibration * 2**30) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 5}))
        return
    K, W = args.steps, args.warmup
    log(f"building the {WORKLOAD} workload")
    case = inputs.plate_with_hole(n=8192, radius=1024, steps=PRECISION_STEPS)
    nodes = case.in_body_nodes()

    def timed_run(storage):
        t0 = time.perf_counter()
        ctx = lbm.context_for(case, storage)
        log(f"{storage}: context in {time.perf_counter() - t0:.1f} s")
        if args.tiling and storage == args.storage:
            ctx.set_tiling(*[int(v) for v in args.tiling.split(",")])
        elif not args.autotune:
            ctx.set_tiling(*TUNED[storage][0])
        if not args.autotune:
            ov = args.overlap if (storage == args.storage and args.overlap >= 0) else TUNED[storage][1]
            ctx.use_overlap(bool(ov))
        ctx.step(2)
        if args.autotune:
            ctx.autotune(3)
        ctx.step(W)
        # the graphs of the timed call are captured before the timer starts
        ctx.prepare_steps(K)
        before = ctx.info()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(K)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        after = ctx.info()
        window = {"first_step": before["steps_done"], "graph_steps":
                  after["steps_in_graphs"] - before["steps_in_graphs"],
                  "sync_steps": after["syncs_done"] - before["syncs_done"]}
        log(f"{storage}: {K} steps in {dt * 1e3:.2f} ms ({nodes * K / dt / 1e9:.2f} GLUPS)")
        return ctx, dt, window

    def roofline_of(ctx, storage, psteps):
        """Dominant interior launch, timed with HIP events on its stream over
        psteps eager steps (lbm_profile)."""
        info = ctx.info()
        prof = ctx.profile(psteps)
        kind = ("deep" if prof["deep"][1] > 0 else
                "two_step" if prof["two_step"][1] > 0 else "interior")
        k_ms, k_n = prof[kind]
        per = k_ms / k_n / 1e3
        bpu = info["bytes_per_update"]
        # nodes whose state the launch streams (read once, written once) and
        # the lattice updates it performs
        if kind == "deep":
            own, lups = info["nodes_deep"], 2 * info["nodes_deep"]
        elif kind == "two_step":
            own, lups = nodes, nodes + info["nodes_two_step"]
        else:
            own, lups = nodes, nodes
        return info, prof, kind, per, own, lups, bpu

    # ---- headline storage
    ctx, dt, window = timed_run(args.storage)
    ms_per_step = dt / K * 1e3
    glups = nodes * K / dt / 1e9
    info, prof, kind, per, own, lups, bpu = roofline_of(ctx, args.storage, args.profile_steps)
    tile = [info["tile_lanes"], info["tile_rows"], info["tile_order"], info["tile_edge_rows"],
            info["tile_align"], info["tile_steps"], info["tile_edge_cols"],
            info["tile_stream_stores"]]
    overlap = bool(info["overlap"])
    achieved = own * bpu / per / 1e9
    traffic = measured_traffic(args.storage, kind, tile, overlap)
    copy_gbs = copy_rate_gbs()
    layout_gbs = lbm.layout_copy_rate(args.storage, info["nodes_allocated"], 10)
    roofline = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
        "kernel": f"k_interior<{args.storage}, {info['tile_lanes']} lanes, {KIND_NAMES[kind]}>",
        "avg_launch_us": round(per * 1e6, 2),
        "algorithmic_bytes_per_launch": own * bpu,
        "bytes_per_node_pass": bpu, "nodes_per_launch": own, "lups_per_launch": lups,
        "effective_GBs": round(lups * bpu / per / 1e9, 1),
        "effective_frac": round(lups * bpu / per / 1e9 / HBM_PEAK_GBS, 4),
        "measured_GBs": round(traffic / per / 1e9, 1) if traffic else None,
        "measured_frac": round(traffic / per / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
        "copy_GBs": round(copy_gbs, 1),
        "frac_of_copy": round(achieved / copy_gbs, 4),
        "layout_copy_GBs": round(layout_gbs, 1),
        "measured_frac_of_layout_copy": (round(traffic / per / 1e9 / layout_gbs, 4)
                                         if traffic else None),
        "step_effective_GBs": round(nodes * bpu / (dt / K) / 1e9, 1),
        "step_effective_frac": round(nodes * bpu / (dt / K) / 1e9 / HBM_PEAK_GBS, 4),
    }
    for k in ("interior", "two_step", "boundary", "sync", "deep"):
        ms, n = prof[k]
        if n:
            roofline[f"{k}_launch_avg_us"] = round(ms / n * 1e3, 2)

    # ---- untimed leg: on to step 2000, the fields the errors are taken on
    # (info was read before the profiled steps: take the count as it is now)
    done = ctx.info()["steps_done"]
    fields = {}
    if not args.no_precision and done <= PRECISION_STEPS:
        ctx.step(PRECISION_STEPS - done)
        fields[args.storage] = ctx.fields(0, want=("e", "omega", "u"))
    ctx.close()
    del ctx
    torch.cuda.empty_cache()

    variants = {}
    if not args.no_variants:
        for st in VARIANTS:
            if st == args.storage:
                continue
            c2, d2, w2 = timed_run(st)
            i2, p2, k2, per2, own2, lups2, bpu2 = roofline_of(c2, st, args.profile_steps)
            ach2 = own2 * bpu2 / per2 / 1e9
            v = {"glups": round(nodes * K / d2 / 1e9, 3), "ms_per_step": round(d2 / K * 1e3, 4),
                 "speedup_vs_" + args.storage: round(dt / d2, 3), "bytes_per_lup": bpu2,
                 "kernel_avg_launch_us": round(per2 * 1e6, 2),
                 "kernel_GBs": round(ach2, 1), "kernel_frac": round(ach2 / HBM_PEAK_GBS, 4),
                 "kernel_effective_frac": round(lups2 * bpu2 / per2 / 1e9 / HBM_PEAK_GBS, 4),
                 "step_effective_frac": round(nodes * bpu2 / (d2 / K) / 1e9 / HBM_PEAK_GBS, 4),
                 "graph_steps": w2["graph_steps"],
                 "tile": [i2["tile_lanes"], i2["tile_rows"], i2["tile_order"],
                          i2["tile_edge_rows"], i2["tile_align"], i2["tile_steps"],
                          i2["tile_edge_cols"], i2["tile_stream_stores"]]}
            t2 = measured_traffic(st, k2, v["tile"], bool(i2["overlap"]))
            lc2 = lbm.layout_copy_rate(st, i2["nodes_allocated"], 10)
            v["layout_copy_GBs"] = round(lc2, 1)
            if t2:
                v["kernel_measured_frac"] = round(t2 / per2 / 1e9 / HBM_PEAK_GBS, 4)
                v["kernel_measured_frac_of_layout_copy"] = round(t2 / per2 / 1e9 / lc2, 4)
            done2 = c2.info()["steps_done"]
            if not args.no_precision and done2 <= PRECISION_STEPS:
                c2.step(PRECISION_STEPS - done2)
                fields[st] = c2.fields(0, want=("e", "omega", "u"))
            c2.close()
            del c2
            torch.cuda.empty_cache()
            variants[st] = v
        if args.storage in fields:
            ref = fields[args.storage]
            for st, v in variants.items():
                if st in fields:
                    v["rel_l2_vs_" + args.storage + f"_at_step_{PRECISION_STEPS}"] = {
                        k: rel_l2(fields[st][k], ref[k]) for k in ("e", "omega", "u")}
                    v["within_1e-3"] = all(
                        x <= 1e-3 for x in v["rel_l2_vs_" + args.storage + f"_at_step_{PRECISION_STEPS}"].values())
                    log(f"{st}: rel L2 at step {PRECISION_STEPS}: "
                        f"{v['rel_l2_vs_' + args.storage + f'_at_step_{PRECISION_STEPS}']}")
    fields.clear()

    cpu = None
    if not args.no_cpu:
        log("oracle CPU baseline")
        cpu, orc = cpu_baseline(case, args.cpu_budget)
        # the FP64 GPU path on the same plate, to the oracle's step count
        n_orc = orc.steps_done
        ref = orc.fields()
        del orc
        with lbm.context_for(case, "f64") as c3:
            c3.set_tiling(*TUNED["f64"][0])
            c3.use_overlap(TUNED["f64"][1])
            c3.step(n_orc)
            got = c3.fields(0)
        cpu["fp64_gpu_vs_oracle_rel_max"] = {
            k: float(np.abs(got[k] - ref[k]).max() / max(np.abs(ref[k]).max(), 1e-300))
            for k in ("e", "omega", "u", "v")}
        cpu["fp64_gpu_vs_oracle_step"] = n_orc
        del ref, got
        if args.cpu_workloads:
            log("oracle on samples of the batched workloads")
            cpu["workloads"] = cpu_workloads()

    line = {
        "metric": METRIC, "value": round(glups, 4), "unit": "GLUPS", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32"}.get(args.storage, "f32+f64"), "data": "synthetic",
        "config": {"workload": "plate 8192x8192 with a central circular hole of radius 1024 "
                               "(traction-free rim), outer edges clamped u*=0, nu 0.3, a0_phi "
                               "0.9999, Gaussian pulse sigma 16 amp 1e-3 on the annulus, sync "
                               f"every 50; {args.storage} storage",
                   "nodes": nodes, "storage": args.storage, "tile": tile, "overlap": overlap,
                   "graphs": window["graph_steps"] == K,
                   "timed_window": {"steps": [window["first_step"], window["first_step"] + K - 1],
                                    "steps_in_graphs": window["graph_steps"],
                                    "sync_steps": window["sync_steps"]}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
