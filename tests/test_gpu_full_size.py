"""The 1024^2 clamped plate at its full length (5000 steps, synchronization
every 50) against the CPU oracle: the FP64 path in the two-step tiling with
overlapped pairs (64 lanes, 8 rows, edge rows 4, edge columns 4) at the
parity bar, and the plain FP32 path within a stated relative L2 error."""
import numpy as np
import pytest

from oracle.oracle import run_case
from paper_2301_00228_amd import inputs as I
from paper_2301_00228_amd import lbm

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

# Plain FP32 (populations, u and du/dt in FP32) after 5000 steps: the
# rounding of u and of the FP32 weights accumulates; measured 2.7e-4 on this
# plate against the FP64 path.
FP32_BOUND = 1e-3


@pytest.fixture(scope="module")
def reference():
    import torch
    torch.cuda.set_device(0)
    case = I.clamped_plate(n=1024, steps=5000)
    print("oracle: clamped 1024^2, 5000 steps", flush=True)
    ref, _ = run_case(case)
    return case, ref


def test_fp64_5000_steps_two_step_overlapped(reference):
    case, ref = reference
    with lbm.context_for(case, "f64") as ctx:
        ctx.set_tiling(64, 8, 0, 4, 0, 2, 4)
        ctx.use_overlap(True)
        ctx.step(case.steps)
        got = ctx.fields(0)
        info = ctx.info()
    assert info["overlap"] == 1 and info["tile_steps"] == 2
    assert info["steps_in_graphs"] == case.steps
    for k in ("e", "omega", "u", "v"):
        err = np.abs(got[k] - ref[k]).max() / np.abs(ref[k]).max()
        print("fp64 5000 steps", k, f"{err:.3e}", flush=True)
        assert err <= 1e-12, (k, err)


def test_fp32_5000_steps(reference):
    case, ref = reference
    with lbm.context_for(case, "f32") as ctx:
        ctx.step(case.steps)
        got = ctx.fields(0)
    for k in ("e", "omega", "u"):
        err = float(np.linalg.norm(got[k] - ref[k]) / np.linalg.norm(ref[k]))
        print("fp32 5000 steps", k, f"{err:.3e}", flush=True)
        assert err <= FP32_BOUND, (k, err)


# The bench workload at full size (8192^2 plate with a hole of radius 1024,
# 63.8 M body nodes) in the launch configuration bench.py times: its pinned
# FP64 tiling, one stream, graphs.
HOLE_STEPS = 52          # two-step pairs, their second launches and one synchronization (step 50)
PRECISION_STEPS = 2000   # the step the reduced storages are held to 1e-3 at


@pytest.fixture(scope="module")
def hole8192():
    import torch
    torch.cuda.set_device(0)
    return I.plate_with_hole(n=8192, radius=1024, steps=PRECISION_STEPS)


def _bench_context(case, storage):
    from bench import TUNED
    ctx = lbm.context_for(case, storage)
    ctx.set_tiling(*TUNED[storage][0])
    ctx.use_overlap(bool(TUNED[storage][1]))
    return ctx


def test_hole8192_fp64_bench_tiling_matches_the_oracle(hole8192):
    print("oracle: 8192^2 plate with a hole, %d steps" % HOLE_STEPS, flush=True)
    ref, _ = run_case(hole8192, steps=HOLE_STEPS)
    with _bench_context(hole8192, "f64") as ctx:
        ctx.step(HOLE_STEPS)
        got = ctx.fields(0)
        info = ctx.info()
    assert info["tile_steps"] == 2 and info["syncs_done"] == 1
    for k in ("e", "omega", "u", "v"):
        err = np.abs(got[k] - ref[k]).max() / np.abs(ref[k]).max()
        print("hole8192 fp64", HOLE_STEPS, "steps", k, f"{err:.3e}", flush=True)
        assert err <= 1e-12, (k, err)


def test_hole8192_f16dev_within_1e3_of_fp64_at_step_2000(hole8192):
    # the FP64 path is the oracle's to 1e-12 (test above and the bench line);
    # the reduced storage is held to the precision bound against it
    fields = {}
    for st in ("f64", "f16dev"):
        with _bench_context(hole8192, st) as ctx:
            ctx.step(PRECISION_STEPS)
            fields[st] = ctx.fields(0, want=("e", "omega", "u"))
    for k in ("e", "omega", "u"):
        err = float(np.linalg.norm(fields["f16dev"][k] - fields["f64"][k]) / np.linalg.norm(fields["f64"][k]))
        print("hole8192 f16dev vs fp64 at", PRECISION_STEPS, k, f"{err:.3e}", flush=True)
        assert err <= 1e-3, (k, err)


# The batched workloads at full size, in the tilings their measurements use
# (the autotuner's picks, pinned): the FP64 batched path against the oracle
# plate by plate after a synchronization, and the reduced storage against it
# at its stated step count.
BATCH256_TILING = (64, 16, 3, 8, 16, 2, 16, 1)
STRIP_TILING = (128, 32, 0, 16, 16, 2, 16, 1)


def _batched(cases, storage, tiling, steps, want=("e", "omega", "u", "v")):
    with lbm.context_for(cases, storage) as ctx:
        ctx.set_tiling(*tiling)
        ctx.use_overlap(False)
        ctx.step(steps)
        return [ctx.fields(p, want=want) for p in range(len(cases))]


def test_batch256_fp64_batched_matches_the_oracle_plate_by_plate():
    import torch
    torch.cuda.set_device(0)
    cases = I.plate_batch(count=256, steps=HOLE_STEPS)
    got = _batched(cases, "f64", BATCH256_TILING, HOLE_STEPS)
    print("256 plates, %d body nodes; oracle plate by plate" % sum(c.in_body_nodes() for c in cases),
          flush=True)
    worst = 0.0
    for c, g in zip(cases, got):
        ref, _ = run_case(c, steps=HOLE_STEPS)
        for k in ("e", "omega", "u", "v"):
            err = np.abs(g[k] - ref[k]).max() / max(np.abs(ref[k]).max(), 1e-300)
            worst = max(worst, err)
            assert err <= 1e-12, (c.name, k, err)
    print("batch256 fp64 vs oracle, worst rel max-norm %.3e" % worst, flush=True)


def test_batch256_f32dev_batched_within_1e3_of_fp64_at_step_1000():
    cases = I.plate_batch(count=256, steps=1000)
    want = ("e", "omega", "u")
    ref = _batched(cases, "f64", BATCH256_TILING, 1000, want)
    got = _batched(cases, "f32dev", BATCH256_TILING, 1000, want)
    worst = {k: 0.0 for k in want}
    for c, g, r in zip(cases, got, ref):
        for k in want:
            nb = np.linalg.norm(r[k])
            err = float(np.linalg.norm(g[k] - r[k]) / (nb if nb > 0 else 1.0))
            worst[k] = max(worst[k], err)
            assert err <= 1e-3, (c.name, k, err)
    print("batch256 f32dev vs fp64 at 1000, worst", worst, flush=True)


def test_strip_with_holes_fp64_matches_the_oracle():
    # the 65536 x 2048 strip with seeded elliptic holes of the 1.2 G-node batch
    case = I.strip_with_holes(steps=20, seed_index=4)
    (got,) = _batched([case], "f64", STRIP_TILING, 20)
    print("strip: oracle, 20 steps", flush=True)
    ref, _ = run_case(case, steps=20)
    for k in ("e", "omega", "u", "v"):
        err = np.abs(got[k] - ref[k]).max() / np.abs(ref[k]).max()
        print("strip fp64 20 steps", k, f"{err:.3e}", flush=True)
        assert err <= 1e-12, (k, err)


def test_strip_with_holes_f16dev_within_1e3_of_fp64_at_step_2000():
    case = I.strip_with_holes(steps=PRECISION_STEPS, seed_index=4)
    want = ("e", "omega", "u")
    (ref,) = _batched([case], "f64", STRIP_TILING, PRECISION_STEPS, want)
    (got,) = _batched([case], "f16dev", STRIP_TILING, PRECISION_STEPS, want)
    for k in want:
        err = float(np.linalg.norm(got[k] - ref[k]) / np.linalg.norm(ref[k]))
        print("strip f16dev vs fp64 at", PRECISION_STEPS, k, f"{err:.3e}", flush=True)
        assert err <= 1e-3, (k, err)
