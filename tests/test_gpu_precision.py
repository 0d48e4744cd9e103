"""Reduced-storage paths against the FP64 CPU oracle (or the FP64 GPU path,
which the parity tests hold to the oracle within 1e-12): relative L2 error
of e, omega and u after 2000 steps, the bar being 1e-3.

Where the bar holds: FP32, F32DEV and F16DEV on every workload below; BF16DEV
(8 significand bits, about 8x the rounding noise of FP16) on plates of
1024^2 and more.  Where it does not (measured, recorded as a limit of the
format, not asserted): BF16DEV on plates of a few hundred nodes per side
(1.4e-3 to 3.2e-3: the second-row rule keeps the non-equilibrium moments
near the edges large, and small plates are mostly near an edge) and on the
paper's load-driven shear and hole examples; F16DEV on the rotation field of
the paper's tension-with-a-hole example (0.9e-3 to 1.2e-3)."""
import numpy as np
import pytest

from oracle.oracle import run_case
from paper_2301_00228_amd import inputs as I
from paper_2301_00228_amd import lbm

pytestmark = pytest.mark.gpu

BOUND = {"f32": 1e-3, "f32dev": 1e-5, "f16dev": 1e-3}


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def errors(got, ref):
    return {k: rel_l2(got[k], ref[k]) for k in ("e", "omega", "u")}


@pytest.fixture(scope="module")
def reference():
    import torch
    torch.cuda.set_device(0)
    case = I.plate_with_hole(n=256, radius=32, sigma=8.0, steps=2000, sync_every=50)
    ref, _ = run_case(case)
    return case, ref


@pytest.mark.parametrize("storage", ["f64", "f32", "f32dev", "f16dev"])
def test_reduced_storage_error(reference, storage):
    case, ref = reference
    with lbm.context_for(case, storage) as ctx:
        ctx.step(case.steps)
        got = ctx.fields(0)
    errs = errors(got, ref)
    print(storage, {k: f"{v:.3e}" for k, v in errs.items()}, flush=True)
    bound = 1e-12 if storage == "f64" else BOUND[storage]
    assert max(errs.values()) <= bound, (storage, errs)


@pytest.mark.parametrize("storage", ["f16dev", "bf16dev"])
def test_sixteen_bit_storages_on_the_clamped_plate(storage):
    """The 1024^2 clamped plate (sigma 16 pulse, a0_phi = 0.9999, synchronization
    every 50 steps): after 2000 steps within 1e-3 relative L2 of the FP64 path."""
    import torch
    torch.cuda.set_device(0)
    case = I.clamped_plate(n=1024, steps=2000)
    with lbm.context_for(case, "f64") as ctx:
        ctx.step(case.steps)
        ref = ctx.fields(0)
    with lbm.context_for(case, storage) as ctx:
        ctx.step(case.steps)
        got = ctx.fields(0)
    errs = errors(got, ref)
    print(storage, "1024^2", {k: f"{v:.3e}" for k, v in errs.items()}, flush=True)
    assert max(errs.values()) <= 1e-3, (storage, errs)


@pytest.fixture(scope="module")
def mixed_batch_reference():
    import torch
    torch.cuda.set_device(0)
    cases = I.mixed_batch(steps=2000)
    print("mixed batch", [(c.name, c.nx, c.ny) for c in cases], flush=True)
    return cases, [run_case(c)[0] for c in cases]


@pytest.mark.parametrize("storage", ["f32dev", "f16dev"])
def test_mixed_batch_each_plate_against_the_oracle(mixed_batch_reference, storage):
    """Seven plates in one context (five rectangles with random clamped and
    free edges, a plate with an elliptic hole, a strip with ten elliptic
    holes), 2000 steps: each plate's batched output against the oracle.
    F32DEV within 1e-5, F16DEV within 1e-3.  (BF16DEV misses 1e-3 on plates
    this small: 1.4e-3 to 2.7e-3 measured; see the module docstring.)"""
    cases, refs = mixed_batch_reference
    with lbm.context_for(cases, storage) as ctx:
        ctx.step(2000)
        outs = [ctx.fields(p, want=("e", "omega", "u")) for p in range(len(cases))]
    bound = {"f32dev": 1e-5, "f16dev": 1e-3}[storage]
    for c, got, ref in zip(cases, outs, refs):
        errs = errors(got, ref)
        print(storage, c.name, {k: f"{v:.3e}" for k, v in errs.items()}, flush=True)
        assert max(errs.values()) <= bound, (storage, c.name, errs)


def test_sixteen_bit_batch_of_large_plates():
    """Six plates of about 1024^2 (one with an elliptic hole, random clamped
    and free edges, sigma 32 pulses) in one context, 2000 steps, F16DEV and
    BF16DEV: each plate within 1e-3 relative L2 of the FP64 path run on the
    same batch."""
    import torch
    torch.cuda.set_device(0)
    rng = I.rng_for(8)
    cases = [I.mixed_plate(int(rng.integers(960, 1100)), int(rng.integers(960, 1100)), rng,
                           steps=2000, name=f"p{k}") for k in range(5)]
    cases.append(I.plate_with_ellipse_hole(nx=1024, ny=960, hole=(511.0, 480.0, 160.0, 90.0, 0.4),
                                           a0_phi=0.9999, steps=2000, sync_every=50, sigma=32.0,
                                           seed_index=8))
    outs = {}
    for st in ("f64", "f16dev", "bf16dev"):
        with lbm.context_for(cases, st) as ctx:
            ctx.step(2000)
            outs[st] = [ctx.fields(p, want=("e", "omega", "u")) for p in range(len(cases))]
    for st in ("f16dev", "bf16dev"):
        for c, got, ref in zip(cases, outs[st], outs["f64"]):
            errs = errors(got, ref)
            print(st, c.name, c.nx, c.ny, {k: f"{v:.3e}" for k, v in errs.items()}, flush=True)
            assert max(errs.values()) <= 1e-3, (st, c.name, errs)


@pytest.mark.parametrize("kind,sync", [("tension", 0), ("shear", 50)])
def test_load_driven_examples_from_rest(kind, sync):
    """The paper's tension and shear examples (plates at rest driven by
    ramped tractions, L = 96, a0_phi = 0.9999) after 2000 steps against the
    oracle: F32DEV within 1e-5 and F16DEV within 1e-3 (the 16-bit scale is
    set from the loads, since the initial fields are zero)."""
    import torch
    from paper_2301_00228_amd import experiments as E
    torch.cuda.set_device(0)
    case = E.paper_case(kind, 96, sync, cells="mask", t_end=1.0)
    case.steps = 2000
    ref, _ = run_case(case)
    for st, bound in (("f32dev", 1e-5), ("f16dev", 1e-3)):
        with lbm.context_for(case, st) as ctx:
            ctx.step(case.steps)
            got = ctx.fields(0)
        errs = errors(got, ref)
        print(kind, st, {k: f"{v:.3e}" for k, v in errs.items()}, flush=True)
        assert max(errs.values()) <= bound, (kind, st, errs)
