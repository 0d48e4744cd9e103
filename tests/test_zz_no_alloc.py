"""lbm_fields_noalloc: the fields staged through the library's fixed device
area agree with lbm_fields (which stages them in memory the context
allocates), on two calls in a row, the second with a smaller plate."""
import numpy as np
import pytest

from paper_2301_00228_amd import inputs, lbm

pytestmark = pytest.mark.gpu


def _check_same(ctx, plate):
    ref = ctx.fields(plate)
    got = ctx.fields_noalloc(plate)
    for k in ("e", "omega", "u", "v"):
        assert got[k].shape == ref[k].shape
        assert np.array_equal(got[k], ref[k]), k
    return ref


def test_fields_noalloc_matches_fields_on_two_calls():
    import torch
    torch.cuda.set_device(0)
    big = inputs.clamped_plate(n=300, ny=260, sigma=6.0, steps=70, sync_every=50)
    small = inputs.plate_with_ellipse_hole(nx=96, ny=80, steps=70)
    print("no-alloc: clamped 300x260 then ellipse-hole 96x80, f64 and f16dev", flush=True)
    for storage in ("f64", "f16dev"):
        with lbm.context_for(big, storage) as cb, lbm.context_for(small, storage) as cs:
            cb.step(big.steps)
            cs.step(small.steps)
            rb = _check_same(cb, 0)
            rs = _check_same(cs, 0)
            assert np.abs(rb["u"]).max() > 0 and np.abs(rs["u"]).max() > 0
            # a partial request (only u) after the larger call
            u_only = cb.fields_noalloc(0, want=("u",))
            assert np.array_equal(u_only["u"], rb["u"])


def test_fields_noalloc_rejects_plates_beyond_the_fixed_area():
    import torch
    torch.cuda.set_device(0)
    case = inputs.clamped_plate(n=1100, ny=1000, sigma=8.0, steps=0)
    with lbm.context_for(case, "f32dev") as ctx:
        with pytest.raises(lbm.LbmError) as ei:
            ctx.fields_noalloc(0)
        assert ei.value.code == lbm.E_INVAL
        assert "fixed area" in str(ei.value)
        # e alone (8.8 MB) fits and matches
        assert np.array_equal(ctx.fields_noalloc(0, want=("e",))["e"], ctx.fields(0, want=("e",))["e"])
