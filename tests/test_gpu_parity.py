"""FP64 parity of the HIP library (called through the C ABI) with the CPU
oracle on identical seeded inputs: relative max-norm <= 1e-12 per field
(max |gpu - oracle| / max |oracle|), as required of the FP64 path."""
import numpy as np
import pytest

from oracle.oracle import OraclePlate, run_case
from paper_2301_00228_amd import inputs as I
from paper_2301_00228_amd import lbm

pytestmark = pytest.mark.gpu

TOL = 1e-12
FIELDS = ("e", "omega", "u", "v")


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)


def relmax(got, ref):
    scale = np.abs(ref).max()
    return np.abs(got - ref).max() / (scale if scale > 0 else 1.0)


def assert_parity(got, ref, tol=TOL, what=""):
    errs = {k: relmax(got[k], ref[k]) for k in FIELDS}
    print(what, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k in FIELDS:
        assert np.isfinite(got[k]).all(), (what, k)
        assert errs[k] <= tol, (what, k, errs[k])


def gpu_run(cases, storage="f64", steps=None, tiling=None, graphs=True):
    single = not isinstance(cases, (list, tuple))
    cs = [cases] if single else list(cases)
    with lbm.context_for(cs, storage) as ctx:
        if tiling:
            ctx.set_tiling(*tiling)
        ctx.use_graphs(graphs)
        ctx.step(cs[0].steps if steps is None else steps)
        out = [ctx.fields(p) for p in range(len(cs))]
    return out[0] if single else out


def test_periodic_square_64_full_config():
    case = I.periodic_square()
    print("case", case.name, case.steps, flush=True)
    ref, _ = run_case(case)
    assert_parity(gpu_run(case), ref, what=case.name)


@pytest.mark.parametrize("n,ny,steps", [(96, 80, 400), (3, 3, 50), (131, 7, 120), (7, 130, 120),
                                        (259, 37, 150)])
def test_clamped_plates_ragged_and_tiny(n, ny, steps):
    case = I.clamped_plate(n=n, ny=ny, sigma=max(1.0, min(n, ny) / 12), steps=steps, sync_every=50)
    print("case", case.name, steps, flush=True)
    ref, _ = run_case(case)
    assert_parity(gpu_run(case), ref, what=case.name)


def test_plate_with_hole():
    case = I.plate_with_hole(n=160, radius=24, sigma=4.0, steps=300, sync_every=50)
    print("case", case.name, flush=True)
    ref, _ = run_case(case)
    assert_parity(gpu_run(case), ref, what=case.name)


def test_batched_plates_each_match_the_oracle():
    cases = I.plate_batch(count=7, side_lo=20, side_hi=150, steps=200)
    print("case batch of", len(cases), [(c.nx, c.ny) for c in cases], flush=True)
    outs = gpu_run(cases)
    for c, got in zip(cases, outs):
        ref, _ = run_case(c)
        assert_parity(got, ref, what=c.name)


def test_elliptic_holes_strip():
    case = I.strip_with_holes(nx=600, ny=96, sigma=6.0, pulses=3, steps=150, seed_index=7)
    print("case", case.name, flush=True)
    ref, _ = run_case(case)
    assert_parity(gpu_run(case), ref, what=case.name)


def test_time_dependent_loads_and_cell_table():
    """Dirichlet ramp on the left edge, a ramped Neumann traction on the top
    edge, and an explicit cell table on the right edge."""
    n = 48
    case = I.clamped_plate(n=n, sigma=4.0, steps=0, sync_every=25)
    dt = case.dt
    left = I.edge_nodes(n, n, I.LEFT)
    top = I.edge_nodes(n, n, I.TOP)[1:-1]
    right = I.edge_nodes(n, n, I.RIGHT)[1:-1]
    bcs = [
        I.BoundaryData(left, np.full(len(left), 1, np.uint8), np.tile([1e-4, -2e-4], (len(left), 1)),
                       knots=np.array([[0.0, 0.0], [40 * dt, 1.0]])),
        I.BoundaryData(top, np.zeros(len(top), np.uint8), np.tile([3e-4, 1e-4], (len(top), 1)),
                       knots=np.array([[0.0, 0.0], [30 * dt, 1.0], [80 * dt, 0.5]])),
        I.BoundaryData(right, np.zeros(len(right), np.uint8), np.zeros((len(right), 2)),
                       cell=np.tile([0.45, 0.9, 0.5, 0.0, 0.5], (len(right), 1))),
    ]
    case.bcs = bcs
    case.steps = 150
    ref, _ = run_case(case)
    assert_parity(gpu_run(case), ref, what="loads")


def exact_cell_case(steps=600):
    """Plate with an elliptic hole, left edge clamped, exact-geometry cells on
    every Neumann node (the oracle's cells) and a ramped uniform pressure
    on the hole's rim (force -p times the rim normal integral of each cell)."""
    from oracle import geometry as G
    case = I.plate_with_ellipse_hole(nx=96, ny=80, hole=(47.3, 38.6, 15.0, 9.5, 0.5),
                                     a0_phi=0.9999, steps=steps, sync_every=50, sigma=4.0)
    xy = I.boundary_nodes(case.mask)
    xy = xy[xy[:, 0] != 0]  # the clamped left edge keeps its Dirichlet data
    cell = G.cells(case.nx, case.ny, case.shapes, xy)
    n_ext = G.rim_normal(cell)
    rim = (xy[:, 0] > 0) & (xy[:, 0] < case.nx - 1) & (xy[:, 1] > 0) & (xy[:, 1] < case.ny - 1)
    p = 2e-3
    val = np.where(rim[:, None], -p * n_ext, 0.0)
    case.bcs.append(I.BoundaryData(xy, np.zeros(len(xy), np.uint8), val, cell=cell,
                                   knots=np.array([[0.0, 0.0], [300 * case.dt, 1.0]])))
    return case


def test_exact_geometry_cells_match_the_oracle():
    case = exact_cell_case()
    print("case", case.name, "exact cells", flush=True)
    ref, _ = run_case(case)
    assert_parity(gpu_run(case), ref, what="exact cells")
    assert_parity(gpu_run(case, tiling=(64, 8, 0, 2, 0, 2)), ref, what="exact cells two-step")


def test_uniform_stress_state_stays_at_rest_with_exact_cells():
    import test_geometry as TG
    case = TG.uniform_stress_case()
    print("case uniform stress, exact cells", flush=True)
    got = gpu_run(case)
    assert np.abs(got["u"] - case.u0).max() <= 1e-13
    assert np.abs(got["v"]).max() <= 1e-13


def test_consistency_error_matches_the_oracle():
    """The consistency error map (Sec. 4) on a plate with a hole, between
    synchronizations and right after one."""
    case = I.plate_with_hole(n=96, radius=14, sigma=4.0, steps=0, sync_every=50)
    p = OraclePlate(case.nx, case.ny, mask=case.mask, periodic=case.periodic, lam=case.lam,
                    mu=case.mu, rho=case.rho, dh=case.dh, dt=case.dt, sync_every=case.sync_every,
                    u0=case.u0, v0=case.v0)
    for bc in case.bcs:
        p.set_bc(bc.xy, bc.kind, bc.val, cell=bc.cell, knots=bc.knots)
    with lbm.context_for(case, "f64") as ctx:
        for n in (37, 13):  # steps 37 and 50 (a synchronization)
            p.step(n)
            ctx.step(n)
            ref, got = p.cons_err(), ctx.consistency_error(0)
            scale = np.abs(p.fields()["e"]).max()
            print("cons_err", n, f"max {ref.max():.3e}", f"diff {np.abs(got - ref).max():.3e}",
                  flush=True)
            assert np.abs(got - ref).max() <= 1e-12 * scale
    assert ref.max() <= 1e-12 * scale  # right after a synchronization


@pytest.mark.parametrize("kind,sync", [("tension", 0), ("shear", 50), ("hole", 50)])
def test_paper_example_setups_match_the_oracle(kind, sync):
    """The Sec. 4 examples (ramped tension, growing shear with a clamped
    edge, tension with a hole and exact cells on its rim) at L = 24."""
    from oracle import geometry as G
    from paper_2301_00228_amd import experiments as E
    case = E.paper_case(kind, 24, sync, cells="exact" if kind == "hole" else "mask", t_end=0.3,
                        cell_fn=lambda nx, ny, shapes, xy: G.cells(nx, ny, shapes, xy))
    print("case", case.name, case.steps, flush=True)
    ref, p = run_case(case)
    with lbm.context_for(case, "f64") as ctx:
        ctx.step(case.steps)
        got = ctx.fields(0)
        err = ctx.consistency_error(0)
    assert_parity(got, ref, what=case.name)
    assert np.abs(err - p.cons_err()).max() <= 1e-12 * np.abs(ref["e"]).max()


@pytest.mark.parametrize("tiling", [None, (64, 8, 0, 4, 0, 2, 4), (128, 5, 1, 2, 0, 1)])
def test_central_difference_update_matches_the_oracle(tiling):
    """The central-difference displacement update (integrator 1) on a plate
    with Dirichlet and Neumann edges and on a plate with a hole."""
    cases = [I.clamped_plate(n=96, ny=80, sigma=4.0, steps=201, sync_every=50, a0_phi=0.99),
             I.plate_with_hole(n=100, radius=14, sigma=3.0, steps=150, sync_every=40)]
    for case in cases:
        case.integrator = 1
        print("case", case.name, "central difference", tiling, flush=True)
        ref, _ = run_case(case)
        assert_parity(gpu_run(case, tiling=tiling), ref, what=case.name)


def test_clamped_1024_short_run_full_size():
    case = I.clamped_plate(n=1024, steps=60)
    print("case", case.name, case.steps, flush=True)
    ref, _ = run_case(case)
    assert_parity(gpu_run(case), ref, what=case.name)


def test_tilings_graphs_and_eager_are_bitwise_identical():
    case = I.plate_with_hole(n=100, radius=14, sigma=3.0, steps=130, sync_every=50)
    base = gpu_run(case, tiling=(128, 32))
    for tiling, graphs in [((64, 1, 0), True), ((256, 7, 1), False), ((128, 64, 2), False),
                           ((64, 13, 1), True), ((128, 32, 0, 4), True), ((256, 9, 1, 2), False),
                           ((64, 16, 2, 1), True), ((64, 8, 0, 2, 16), True),
                           ((128, 5, 1, 3, 32), False), ((256, 16, 0, 0, 48), True),
                           ((64, 8, 0, 2, 0, 2), True), ((128, 16, 1, 4, 16, 2), False),
                           ((256, 5, 0, 0, 0, 2), True), ((64, 3, 0, 1, 0, 2), False),
                           ((64, 8, 0, 2, 16, 2, 8), True), ((128, 7, 1, 3, 0, 2, 5), False),
                           ((64, 8, 0, 4, 0, 1, 16), True), ((128, 16, 3, 4, 16, 2, 16), True),
                           ((64, 8, 3, 4, 16, 2, 16), False), ((256, 7, 3, 2), True),
                           ((64, 8, 3, 4, 16, 2, 16, 1), True), ((128, 16, 0, 4, 0, 2, 4, 1), False),
                           ((256, 16, 3, 8, 16, 2, 16), True), ((64, 16, 3, 8, 16, 2, 16, 1), False),
                           ((256, 8, 0, 4, 8, 2, 8, 1), True)]:
        other = gpu_run(case, tiling=tiling, graphs=graphs)
        for k in FIELDS:
            assert np.array_equal(base[k], other[k]), (tiling, graphs, k)


@pytest.mark.parametrize("first", [60, 0, 50])
def test_autotune_keeps_the_trajectory(first):
    """Tuning mid-run (also at step 0 and at a synchronization step, where the
    autotuner takes one real step first) leaves the results bitwise equal."""
    case = I.plate_batch(count=5, side_lo=30, side_hi=90, steps=120)
    base = gpu_run(case)
    with lbm.context_for(case) as ctx:
        ctx.step(first)
        ctx.autotune(2)
        info = ctx.info()
        assert info["tile_lanes"] in (64, 128, 256) and info["tile_order"] in (0, 1, 2, 3)
        assert 1 <= info["tile_edge_rows"] <= info["tile_rows"]
        assert info["tile_align"] in (0, 16) and info["tile_steps"] in (1, 2)
        assert info["tile_edge_cols"] in (0, 4, 8, 16)
        done = info["steps_done"]
        assert done in (first, first + 1), done
        if first in (0, 50):
            assert done == first + 1, done
        ctx.step(120 - done)
        tuned = [ctx.fields(p) for p in range(len(case))]
    for a, b in zip(base, tuned):
        for k in FIELDS:
            assert np.array_equal(a[k], b[k]), k


TWO_STEP = [(64, 8, 0, 2, 0, 2), (128, 16, 0, 4, 16, 2), (256, 5, 1, 0, 0, 2), (64, 8, 0, 4, 16, 2, 8),
            (128, 9, 2, 2, 0, 2, 4),
            # the 8192^2 bench plate's FP64 tiling (256-lane tiles, paired edge strips)
            (256, 16, 3, 8, 16, 2, 16),
            # the 256-plate batch's (16-row tiles, 8-row edge tiles, stream stores)
            (64, 16, 3, 8, 16, 2, 16, 1)]


@pytest.mark.parametrize("tiling", TWO_STEP)
def test_two_step_tiles_match_the_oracle(tiling):
    """Tiles away from boundaries take two steps per pass; the others take
    them in two launches; odd step counts end with a single step."""
    cases = [I.periodic_square(), I.clamped_plate(n=150, ny=97, sigma=6.0, steps=151, sync_every=50),
             I.plate_with_hole(n=160, radius=24, sigma=4.0, steps=121, sync_every=40)]
    for case in cases:
        ref, _ = run_case(case)
        got = gpu_run(case, tiling=tiling)
        assert_parity(got, ref, what=f"{case.name} {tiling}")


def test_two_step_batch_and_split_stepping_bitwise():
    cases = I.plate_batch(count=6, side_lo=20, side_hi=200, steps=0)
    base = [None] * len(cases)
    with lbm.context_for(cases) as ctx:
        ctx.step(157)
        base = [ctx.fields(p) for p in range(len(cases))]
    with lbm.context_for(cases) as ctx:
        ctx.set_tiling(64, 8, 0, 2, 0, 2)
        for n in (1, 2, 64, 50, 7, 33):
            ctx.step(n)
        got = [ctx.fields(p) for p in range(len(cases))]
    for a, b in zip(base, got):
        for k in FIELDS:
            assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("storage", ["f64", "f16dev"])
def test_overlapped_pairs_are_bitwise_identical(storage):
    """Deep two-step tiles on a second stream beside the single-step
    launches (the default) against one stream, eager and in graphs, on a
    batch with clamped and free edges and on a periodic plate (no
    single-step tiles: every two-step tile is deep)."""
    batch = I.plate_batch(count=7, side_lo=20, side_hi=300, steps=0)
    per = I.periodic_square(n=96)
    for cases, tiling in [(batch, (64, 8, 0, 4, 0, 2, 4)), (batch, (64, 16, 1, 2, 16, 2, 8)),
                          (batch, (128, 9, 2, 3, 0, 2, 4)), ([per], (64, 8, 0, 2, 0, 2))]:
        outs = []
        for overlap, graphs in [(False, False), (True, False), (True, True)]:
            with lbm.context_for(cases, storage) as ctx:
                ctx.set_tiling(*tiling)
                ctx.use_overlap(overlap)
                ctx.use_graphs(graphs)
                ctx.step(1)
                ctx.step(150)
                info = ctx.info()
                assert info["overlap"] == int(overlap)
                assert 0 < info["nodes_deep"] <= info["nodes_two_step"]
                prof = ctx.profile(20)
                assert (prof["deep"][1] > 0) == overlap, prof
                ctx.step(7)
                outs.append([ctx.fields(p) for p in range(len(cases))])
        for o in outs[1:]:
            for a, b in zip(outs[0], o):
                for k in FIELDS:
                    assert np.array_equal(a[k], b[k]), (storage, tiling, k)


@pytest.mark.parametrize("storage", ["f32", "f32dev", "bf16dev"])
def test_overlapped_pairs_other_storages_and_modes(storage):
    """Overlap on against off, bitwise: plates with elliptic holes, no
    synchronization, the central-difference update, and a plate periodic
    in x beside clamped ones."""
    big = I.plate_with_ellipse_hole(nx=260, ny=200, hole=(131.2, 99.7, 30.0, 17.0, 0.4), a0_phi=0.9999,
                                    steps=0, sync_every=0, sigma=5.0)
    cd = I.plate_with_ellipse_hole(nx=230, ny=190, hole=(80.3, 120.1, 22.0, 11.0, 1.2), a0_phi=0.9999,
                                   steps=0, sync_every=0, sigma=5.0)
    cd.integrator = 1
    per = I.clamped_plate(n=200, ny=150, sigma=5.0, steps=0, sync_every=0)
    per.periodic = (True, False)
    per.bcs = []
    outs = []
    for ov in (False, True):
        with lbm.context_for([big, cd, per], storage) as ctx:
            ctx.set_tiling(64, 8, 0, 4, 0, 2, 8)
            ctx.use_overlap(ov)
            assert ctx.info()["nodes_deep"] > 0
            ctx.step(3)
            ctx.step(120)
            outs.append([ctx.fields(p) for p in range(3)])
    for a, b in zip(*outs):
        for k in FIELDS:
            assert np.isfinite(a[k]).all()
            assert np.array_equal(a[k], b[k]), (storage, k)


def test_overlap_switched_mid_run_and_odd_step_counts():
    """Overlap switched on and off between lbm_step calls of odd lengths
    (pairs cut at synchronizations and at the end of a call), against one
    call on one stream."""
    cases = I.plate_batch(count=4, side_lo=120, side_hi=260, steps=0)
    with lbm.context_for(cases) as ctx:
        ctx.set_tiling(64, 8, 0, 4, 0, 2, 4)
        ctx.use_overlap(False)
        ctx.step(211)
        base = [ctx.fields(p) for p in range(len(cases))]
    with lbm.context_for(cases) as ctx:
        ctx.set_tiling(64, 8, 0, 4, 0, 2, 4)
        for n, ov in ((1, True), (2, True), (37, True), (10, False), (51, True), (3, False),
                      (64, True), (43, True)):
            ctx.use_overlap(ov)
            ctx.step(n)
        got = [ctx.fields(p) for p in range(len(cases))]
    for a, b in zip(base, got):
        for k in FIELDS:
            assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("storage", ["f32", "f32dev", "f16dev", "bf16dev"])
def test_reduced_storages_bitwise_across_tilings(storage):
    """The two-step pass applies the storage rounding to its intermediate
    level, so every tiling gives the same bits in every storage."""
    case = I.plate_with_hole(n=140, radius=20, sigma=4.0, steps=0, sync_every=25)
    outs = []
    for tiling in [(64, 8, 0, 2, 0, 1), (64, 8, 0, 2, 0, 2), (256, 32, 1, 4, 16, 2)]:
        with lbm.context_for(case, storage) as ctx:
            ctx.set_tiling(*tiling)
            ctx.step(83)
            outs.append(ctx.fields(0))
    for o in outs[1:]:
        for k in FIELDS:
            assert np.array_equal(outs[0][k], o[k]), (storage, k)


def test_switching_steps_per_pass_mid_run():
    """Switching to two-step tiles mid-run allocates the third buffer from
    the current state; switching back and forth keeps the trajectory."""
    case = I.plate_with_hole(n=130, radius=18, sigma=4.0, steps=0, sync_every=40)
    with lbm.context_for(case) as ctx:
        ctx.set_tiling(64, 8, 0, 2, 0, 1)
        ctx.step(97)
        base = ctx.fields(0)
    with lbm.context_for(case) as ctx:
        ctx.set_tiling(64, 8, 0, 2, 0, 1)
        ctx.step(31)
        ctx.set_tiling(128, 16, 0, 4, 16, 2)
        ctx.step(23)
        ctx.set_tiling(64, 8, 1, 2, 0, 1)
        ctx.step(20)
        ctx.set_tiling(256, 8, 0, 0, 0, 2)
        ctx.step(23)
        got = ctx.fields(0)
    for k in FIELDS:
        assert np.array_equal(base[k], got[k]), k


def test_repeat_runs_are_deterministic():
    case = I.clamped_plate(n=70, sigma=4.0, steps=90, sync_every=50)
    a, b = gpu_run(case), gpu_run(case)
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), k


def test_split_stepping_equals_one_call():
    case = I.clamped_plate(n=60, sigma=4.0, steps=0, sync_every=50)
    with lbm.context_for(case) as ctx:
        ctx.step(173)
        one = ctx.fields(0)
    with lbm.context_for(case) as ctx:
        for n in (1, 2, 64, 50, 7, 49):
            ctx.step(n)
        split = ctx.fields(0)
    for k in FIELDS:
        assert np.array_equal(one[k], split[k]), k


def test_blow_up_is_reported():
    """At the lattice stability limit the bounded scheme diverges (the paper
    needed a0_phi = 0.9999); the library must report it, not return
    garbage."""
    case = I.clamped_plate(n=32, sigma=3.0, a0_phi=0.0, steps=0, sync_every=0)
    with lbm.context_for(case) as ctx:
        with pytest.raises(lbm.LbmError) as ei:
            ctx.step(3000)
            ctx.fields(0)
        assert ei.value.code == lbm.E_NONFINITE


def test_set_bc_after_step_is_rejected():
    case = I.clamped_plate(n=20, sigma=2.0, steps=0)
    with lbm.context_for(case) as ctx:
        ctx.step(1)
        with pytest.raises(lbm.LbmError) as ei:
            ctx.set_bc(0, [[0, 3]], [1], [[0.0, 0.0]])
        assert ei.value.code == lbm.E_STATE
        with pytest.raises(lbm.LbmError) as ei:
            lbm.Context([lbm.plate_dict(case)]).set_bc(0, [[5, 5]], [1], [[0.0, 0.0]])
        assert ei.value.code == lbm.E_INVAL


@pytest.mark.parametrize("tiling,overlap", [((64, 8, 0, 4, 0, 2, 4), True),
                                            ((128, 16, 0, 4, 16, 2, 16), False),
                                            ((128, 8, 0, 2, 0, 1, 0), False)])
def test_graphs_of_any_step_count_are_bitwise_and_counted(tiling, overlap):
    """lbm_step replays a captured graph for runs of any length and starting
    phase (whole synchronization periods from aligned steps, any other run
    as a graph of its own, cached); the trajectory is bitwise that of eager
    launches, every step runs in a graph, the synchronizations are counted,
    and graphs prepared ahead are replayed without a new capture."""
    case = I.clamped_plate(n=150, ny=118, sigma=5.0, steps=0, sync_every=50)
    calls = (2, 7, 13, 50, 3, 77, 31, 50, 50, 7, 13)
    total = sum(calls)
    with lbm.context_for(case) as ctx:
        ctx.set_tiling(*tiling)
        ctx.use_overlap(overlap)
        ctx.use_graphs(False)
        ctx.step(total)
        ref = ctx.fields(0)
        assert ctx.info()["steps_in_graphs"] == 0
    with lbm.context_for(case) as ctx:
        ctx.set_tiling(*tiling)
        ctx.use_overlap(overlap)
        for m, n in enumerate(calls):
            if m % 3 == 1:
                ctx.prepare_steps(n)
                cached = ctx.info()["graphs_cached"]
                ctx.step(n)
                assert ctx.info()["graphs_cached"] == cached
            else:
                ctx.step(n)
            if m % 4 == 0:
                ctx.fields(0)  # eager work and a synchronization between replays
        got = ctx.fields(0)
        info = ctx.info()
    assert info["steps_in_graphs"] == total
    assert info["syncs_done"] == total // 50
    for k in FIELDS:
        assert np.array_equal(got[k], ref[k]), (tiling, k)


def _moving_boundary_cases(readings):
    """A plate with a hole and ramped loads on both edge kinds, and a
    clamped plate, with the given readings of eqs. correction-f / LBE_mod."""
    hole = I.plate_with_hole(n=72, radius=10, sigma=3.0, steps=140, sync_every=50, a0_phi=0.99)
    dt = hole.dt
    rim = I.boundary_nodes(hole.mask)
    rim = rim[(rim[:, 0] > 0) & (rim[:, 0] < hole.nx - 1) & (rim[:, 1] > 0) & (rim[:, 1] < hole.ny - 1)]
    rng = np.random.default_rng(11)
    hole.bcs.append(I.BoundaryData(rim, np.zeros(len(rim), np.uint8),
                                   rng.uniform(-2e-4, 2e-4, (len(rim), 2)),
                                   knots=np.array([[0.0, 0.0], [60 * dt, 1.0]])))
    clamped = I.clamped_plate(n=80, ny=66, sigma=4.0, steps=131, sync_every=50, a0_phi=0.99)
    for c in (hole, clamped):
        c.readings = readings
    return [hole, clamped]


@pytest.mark.parametrize("readings", [(1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("tiling", [None, (64, 8, 0, 4, 0, 2, 4)])
def test_reading_switches_r2_m2_match_the_oracle(readings, tiling):
    """The R2 (streamed-in flux in eq. correction-f) and M2 (old state's
    equilibrium in eq. LBE_mod) readings against the oracle's, which its pins
    fix in closed form; each plate alone and both in one batch."""
    cases = _moving_boundary_cases(readings)
    refs = [run_case(c)[0] for c in cases]
    for c, ref in zip(cases, refs):
        print("case", c.name, "readings", readings, tiling, flush=True)
        assert_parity(gpu_run(c, tiling=tiling), ref, what=f"{c.name} {readings}")
    # in one batch with a default-reading plate (which then steps the same way)
    plain = I.clamped_plate(n=40, ny=36, sigma=3.0, steps=140, sync_every=50, a0_phi=0.99)
    ref_plain, _ = run_case(plain)
    cases[1].steps = cases[0].steps
    refs[1], _ = run_case(cases[1])
    outs = gpu_run(cases + [plain], tiling=tiling)
    for got, ref, c in zip(outs, refs + [ref_plain], cases + [plain]):
        assert_parity(got, ref, what=f"batch {c.name}")


def test_reading_switches_change_the_result_and_reject_autotune():
    cases = _moving_boundary_cases((1, 1))
    base = I.plate_with_hole(n=72, radius=10, sigma=3.0, steps=140, sync_every=50, a0_phi=0.99)
    base.bcs = cases[0].bcs
    a = gpu_run(cases[0])
    b = gpu_run(base)
    assert np.abs(a["e"] - b["e"]).max() > 1e-9 * np.abs(b["e"]).max()
    with lbm.context_for(cases[0], "f64") as ctx:
        ctx.step(3)
        with pytest.raises(lbm.LbmError) as ei:
            ctx.autotune(2)
        assert ei.value.code == lbm.E_STATE


@pytest.mark.parametrize("storage", ["f64", "f32", "f32dev", "f16dev"])
def test_copy_probes_give_plausible_rates(storage):
    # a node count that is not a multiple of the probe's 8192 x 16 block
    rate = lbm.layout_copy_rate(storage, (1 << 22) + 5, 3)
    assert 100.0 < rate < 8000.0, rate
    if storage == "f64":
        assert 100.0 < lbm.copy_rate(1 << 28, 3) < 8000.0


def test_initial_state_step_zero_and_bad_indices():
    # t = 0 against the oracle, step(0) a no-op, negative counts and plate
    # indices outside the context rejected without touching the state
    case = I.plate_with_hole(n=72, radius=10, sigma=3.0, steps=0)
    ref, _ = run_case(case, steps=0)
    with lbm.context_for(case) as ctx:
        f0 = ctx.fields(0)
        ctx.step(0)
        assert ctx.info()["steps_done"] == 0
        assert lbm.library().lbm_step(ctx._h, -1) == lbm.E_INVAL
        for bad in (1, -1):
            assert lbm.library().lbm_fields(ctx._h, bad, None, None, None, None) == lbm.E_INVAL
            with pytest.raises(lbm.LbmError) as ei:
                ctx.fields(bad)
            assert ei.value.code == lbm.E_INVAL
        f1 = ctx.fields(0)
        ctx.step(3)
        assert ctx.info()["steps_done"] == 3
    for k in FIELDS:
        assert np.array_equal(f0[k], f1[k]), k
    assert_parity(f0, ref, what="t = 0")
