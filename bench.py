"""Throughput benchmark of the plane-strain LBM hot path on one MI355X.

One "step" is one time step of the whole method (interior stream+collide
with the u recovery, boundary reset and accelerations, second-row rule,
synchronization every 50th step) on the workload below, with the state
resident in HBM.  Prints ONE JSON line.

Workload (FP64, the headline value): 1024 x 1024 plate, left edge clamped
(u* = 0), other edges traction free, nu = 0.3, a0_phi = 0.9999, one seeded
Gaussian displacement pulse (sigma 16, amplitude 1e-3), synchronization
every 50 steps.  The same workload is also timed with the FP32 and the
reduced (deviation) storages, each with its relative L2 error against the
FP64 run after the same number of steps.
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
# Interior tilings (lanes, rows, order, edge rows, alignment, steps per pass,
# edge columns) and overlapped pairs (lbm_use_overlap) that measured fastest
# for this workload on MI355X, pinned so that runs and the committed
# rocprofv3 summaries use the same launches (--autotune tunes again instead).
TUNED = {"f64": ((64, 8, 0, 4, 0, 2, 4), True), "f32": ((64, 8, 0, 2, 0, 2, 8), True),
         "f32dev": ((64, 8, 0, 2, 0, 2, 8), True), "f16dev": ((64, 8, 0, 2, 0, 2, 8), True),
         "bf16dev": ((64, 8, 0, 2, 0, 2, 8), True)}
METRIC = "GLUPS + % HBM roofline, FP64 vs FP16/FP32-storage at ≤1e-3 rel L2"


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("lbm_kernels.hip", "lbm_types.h"):
        with open(os.path.join(ROOT, "paper_2301_00228_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(storage, kind, tile, overlap):
    """HBM bytes per launch of one interior-kernel kind from the committed
    rocprofv3 PMC summary, if it was taken on the current kernel source with
    the same tiling and overlap setting."""
    path = os.path.join(ROOT, "profiles", f"interior_{storage}_clamped1024_traffic.json")
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


def cpu_baseline(case, budget_s=12.0, single_s=3.0):
    """Time the FP64 oracle on a bounded sample of the same workload, with
    all its OpenMP threads and with one."""
    from oracle import oracle

    p = oracle_plate(case)
    nodes = case.in_body_nodes()
    threads = oracle.threads()

    def timed(budget, done):
        p.step(1)  # (thread start-up)
        t0 = time.perf_counter()
        p.step(4)
        probe = time.perf_counter() - t0
        steps = max(4, int(budget / max(probe / 4, 1e-6)))
        t0 = time.perf_counter()
        p.step(steps)
        return steps, time.perf_counter() - t0, done + 5

    steps, dt, first = timed(budget_s, 0)
    oracle.set_threads(1)
    steps1, dt1, first1 = timed(single_s, first + steps)
    oracle.set_threads(threads)
    return {"value": nodes * steps / dt / 1e9, "unit": "GLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{case.nx}x{case.ny} plate of the same workload, {steps} steps "
                      f"(steps {first + 1}..{first + steps}), {dt:.1f} s wall",
            "single_thread_value": nodes * steps1 / dt1 / 1e9,
            "single_thread_sample": f"steps {first1 + 1}..{first1 + steps1}, {dt1:.1f} s wall",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}


def oracle_plate(case):
    from oracle import oracle

    p = oracle.OraclePlate(case.nx, case.ny, mask=case.mask, periodic=case.periodic,
                           lam=case.lam, mu=case.mu, rho=case.rho, dh=case.dh, dt=case.dt,
                           sync_every=case.sync_every, u0=case.u0, v0=case.v0)
    for bc in case.bcs:
        p.set_bc(bc.xy, bc.kind, bc.val, cell=bc.cell, knots=bc.knots)
    return p


def cpu_workload_samples():
    """The FP64 oracle on sampled subsets of the batched workloads (all its
    OpenMP threads): 4 plates of the 256-plate batch x 100 steps, and one
    4096^2 plate of the 1.2 G-node batch x 20 steps."""
    from paper_2301_00228_amd import inputs

    out = {}
    for name, cases, steps in (("batch256", inputs.plate_batch(count=256, steps=0)[:4], 100),
                               ("large", inputs.large_batch(count=1, strip=None, steps=0), 20)):
        lup, secs = 0, 0.0
        for case in cases:
            p = oracle_plate(case)
            p.step(1)
            t0 = time.perf_counter()
            p.step(steps)
            secs += time.perf_counter() - t0
            lup += case.in_body_nodes() * steps
            del p
        out[name] = {"value": lup / secs / 1e6, "unit": "MLUPS",
                     "sample": f"{len(cases)} plate(s) ({', '.join(f'{c.nx}x{c.ny}' for c in cases)})"
                               f" x {steps} steps, {secs:.1f} s"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--cpu-workloads", action="store_true",
                    help="also time the oracle on samples of the batched workloads")
    ap.add_argument("--profile-steps", type=int, default=200)
    ap.add_argument("--storage", default="f64", help="storage of the headline run")
    ap.add_argument("--tiling", default="", metavar="L,R,O,E,A,S[,W]",
                    help="interior tiling of the headline storage (lanes, rows, order, edge "
                         "rows, alignment, steps, edge columns) instead of the pinned one")
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
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(plates shard across GPUs with no communication; see DESIGN.md)", file=sys.stderr)
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
    case = inputs.clamped_plate(n=1024, steps=args.steps)
    nodes = case.in_body_nodes()
    K, W = args.steps, args.warmup

    def timed_run(storage):
        ctx = lbm.context_for(case, storage)
        if args.tiling and storage == args.storage:
            ctx.set_tiling(*[int(v) for v in args.tiling.split(",")])
        elif not args.autotune:
            ctx.set_tiling(*TUNED[storage][0])
        if not args.autotune:
            ov = args.overlap if (storage == args.storage and args.overlap >= 0) else TUNED[storage][1]
            ctx.use_overlap(bool(ov))
        ctx.step(2)
        if args.autotune:
            ctx.autotune(5)
        ctx.step(W)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(K)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return ctx, dt

    ctx, dt = timed_run(args.storage)
    ms_per_step = dt / K * 1e3
    glups = nodes * K / dt / 1e9
    info = ctx.info()
    f64_fields = ctx.fields(0)
    tile = [info["tile_lanes"], info["tile_rows"], info["tile_order"], info["tile_edge_rows"],
            info["tile_align"], info["tile_steps"], info["tile_edge_cols"]]
    # Dominant kernel: the interior launch with the most device time -- with
    # overlapped pairs the deep tiles' launch (two steps of the two-step
    # tiles away from the single-step ones, on the library's second stream
    # beside the pair's other launches), else the first launch of a two-step
    # pair (two steps of the two-step tiles, one of the others) or the
    # single-step launch.  Device time per launch from HIP events on the
    # stream it runs on, eager launches.  achieved = algorithmic bytes per
    # lattice update x the lattice updates the launch performs / its time;
    # the launch streams each of its nodes' state once, so with two steps per
    # pass this exceeds the rate at which it actually streams (min_bytes /
    # time) and the measured traffic.
    prof = ctx.profile(args.profile_steps)
    bnd_ms, bnd_n = prof["boundary"]
    bpu = info["bytes_per_update"]
    kind = ("deep" if prof["deep"][1] > 0 else
            "two_step" if prof["two_step"][1] > 0 else "interior")
    k_ms, k_n = prof[kind]
    per_launch_s = k_ms / k_n / 1e3
    if kind == "deep":
        own = info["nodes_deep"]
        lups = 2 * own
        kname = f"k_interior<{args.storage}, {info['tile_lanes']} lanes, two-step, deep tiles>"
    elif kind == "two_step":
        own = nodes
        lups = nodes + info["nodes_two_step"]
        kname = f"k_interior<{args.storage}, {info['tile_lanes']} lanes, two-step>"
    else:
        own = nodes
        lups = nodes
        kname = f"k_interior<{args.storage}, {info['tile_lanes']} lanes, single-step>"
    achieved = lups * bpu / per_launch_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(args.storage, kind, tile, bool(info["overlap"])),
                "kernel": kname,
                "bytes_per_lup": bpu, "lups_per_launch": lups,
                "avg_launch_us": round(per_launch_s * 1e6, 2),
                "min_bytes_per_launch": own * bpu,
                "min_bytes_GBs": round(own * bpu / per_launch_s / 1e9, 1),
                "boundary_kernel_avg_us": round(bnd_ms / max(bnd_n, 1) * 1e3, 2)}
    if kind in ("deep", "two_step"):
        s_ms, s_n = prof["interior"]
        roofline["two_step_nodes"] = info["nodes_two_step"]
        roofline["second_launch_avg_us"] = round(s_ms / max(s_n, 1) * 1e3, 2)
    if kind == "deep":
        f_ms, f_n = prof["two_step"]
        roofline["deep_nodes"] = info["nodes_deep"]
        roofline["frame_launch_avg_us"] = round(f_ms / max(f_n, 1) * 1e3, 2)
    # what one step per pass over HBM would have to stream at the measured
    # step rate
    roofline["effective_GBs"] = round(nodes * bpu / (dt / K) / 1e9, 1)
    ctx.close()

    variants = {}
    if not args.no_variants:
        ref_u = f64_fields["u"]
        for st in ("f32", "f32dev", "f16dev", "bf16dev"):
            c2, d2 = timed_run(st)
            fl = c2.fields(0)
            pr = c2.profile(min(args.profile_steps, 100))
            i2 = c2.info()
            bpu2 = i2["bytes_per_update"]
            if pr["deep"][1] > 0:
                i_ms, i_n = pr["deep"]
                lups2 = 2 * i2["nodes_deep"]
            elif pr["two_step"][1] > 0:
                i_ms, i_n = pr["two_step"]
                lups2 = nodes + i2["nodes_two_step"]
            else:
                i_ms, i_n = pr["interior"]
                lups2 = nodes
            ach2 = lups2 * bpu2 / (i_ms / i_n / 1e3) / 1e9
            c2.close()
            variants[st] = {
                "glups": round(nodes * K / d2 / 1e9, 3),
                "ms_per_step": round(d2 / K * 1e3, 4),
                "speedup_vs_f64": round(dt / d2, 3),
                "interior_GBs": round(ach2, 1), "interior_frac": round(ach2 / HBM_PEAK_GBS, 4),
                "bytes_per_lup": bpu2,
                "rel_l2_vs_f64": {"e": rel_l2(fl["e"], f64_fields["e"]),
                                  "omega": rel_l2(fl["omega"], f64_fields["omega"]),
                                  "u": rel_l2(fl["u"], ref_u)},
            }
        del ref_u

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(case)
        if args.cpu_workloads:
            cpu["workload_samples"] = cpu_workload_samples()

    line = {
        "metric": METRIC, "value": round(glups, 4), "unit": "GLUPS", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": {"f64": "f64", "f32": "f32"}.get(args.storage, "f32+f64"), "data": "synthetic",
        "config": {"workload": "clamped plate 1024x1024 (left edge u*=0, other edges traction "
                               "free), nu 0.3, a0_phi 0.9999, Gaussian pulse sigma 16 amp 1e-3, "
                               "sync every 50, FP64 populations and u",
                   "nodes": nodes, "storage": args.storage, "tile": tile,
                   "overlap": bool(info["overlap"]), "graphs": True},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
