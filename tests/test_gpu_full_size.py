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
