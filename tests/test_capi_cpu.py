"""C-ABI checks that need no GPU: exported symbols and host-side argument
validation (which happens before any HIP call)."""
import os
import re

import numpy as np
import pytest

from paper_2301_00228_amd import lbm
from paper_2301_00228_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", src)))


def test_header_declarations_match_binding():
    assert declared_functions() == sorted(lbm.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = lbm.library()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert b"gfx950" in L.lbm_version()


def _gpu_present():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def _plate(**kw):
    case = I.clamped_plate(n=16, sigma=2.0, steps=0)
    d = lbm.plate_dict(case)
    d.update(kw)
    return d


def test_invalid_sizes_rejected():
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Context([_plate(nx=2, u0=None, v0=None)])
    assert ei.value.code == lbm.E_INVAL


def test_thin_mask_rejected():
    m = np.ones((16, 16), np.uint8)
    m[:, 5] = 0
    m[:, 7] = 0
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Context([_plate(mask=m)])
    assert ei.value.code == lbm.E_INVAL
    assert "neighbour" in str(ei.value)


def test_unstable_time_step_rejected():
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Context([_plate(dt=I.time_step(0.3, 0.0) * 1.01)])
    assert ei.value.code == lbm.E_UNSTABLE_DT


def test_mixed_sync_periods_rejected():
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Context([_plate(sync_every=50), _plate(sync_every=10)])
    assert ei.value.code == lbm.E_INVAL


def test_unknown_storage_rejected():
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Context([_plate()], storage=9)
    assert ei.value.code == lbm.E_INVAL


@pytest.mark.skipif(_gpu_present(), reason="checks the no-GPU error path")
def test_valid_arguments_report_missing_device():
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Context([_plate()])
    assert ei.value.code == lbm.E_DEVICE


def test_unknown_integrator_rejected():
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Context([_plate(integrator=2)])
    assert ei.value.code == lbm.E_INVAL


def test_consistency_error_needs_a_context():
    L = lbm.library()
    err = np.zeros(4)
    assert L.lbm_consistency_error(None, 0, err.ctypes.data_as(lbm.C.POINTER(lbm.C.c_double))) \
        == lbm.E_INVAL


def test_switches_need_a_context():
    L = lbm.library()
    assert L.lbm_use_overlap(None, 1) == lbm.E_INVAL
    assert L.lbm_use_graphs(None, 1) == lbm.E_INVAL


def test_unknown_reading_bits_rejected():
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Context([_plate(readings=(4, 0))])
    assert ei.value.code == lbm.E_INVAL


def test_step_entry_points_need_a_context():
    L = lbm.library()
    assert L.lbm_prepare_steps(None, 10) == lbm.E_INVAL
    assert L.lbm_fields_noalloc(None, 0, None, None, None, None) == lbm.E_INVAL


def test_copy_rate_rejects_bad_arguments():
    for nbytes, reps in ((8, 1), (1 << 20, 0)):
        with pytest.raises(lbm.LbmError) as ei:
            lbm.copy_rate(nbytes, reps)
        assert ei.value.code == lbm.E_INVAL
    assert lbm.library().lbm_copy_rate(1 << 20, 1, None) == lbm.E_INVAL


@pytest.mark.skipif(_gpu_present(), reason="checks the no-GPU error path")
def test_copy_rate_reports_missing_device():
    with pytest.raises(lbm.LbmError) as ei:
        lbm.copy_rate(1 << 20, 1)
    assert ei.value.code == lbm.E_DEVICE


def test_layout_copy_rate_rejects_bad_arguments():
    for storage, nodes, reps in ((5, 1 << 20, 1), (-1, 1 << 20, 1), (0, 0, 1), (0, (1 << 32) + 1, 1),
                                 (0, 1 << 20, 0)):
        with pytest.raises(lbm.LbmError) as ei:
            lbm.layout_copy_rate(storage, nodes, reps)
        assert ei.value.code == lbm.E_INVAL
    assert lbm.library().lbm_layout_copy_rate(0, 1 << 20, 1, None) == lbm.E_INVAL


@pytest.mark.skipif(_gpu_present(), reason="checks the no-GPU error path")
def test_layout_copy_rate_reports_missing_device():
    with pytest.raises(lbm.LbmError) as ei:
        lbm.layout_copy_rate("f64", 1 << 20, 1)
    assert ei.value.code == lbm.E_DEVICE


def test_no_plates_rejected():
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Context([])
    assert ei.value.code == lbm.E_INVAL
    assert lbm.library().lbm_step(None, 1) == lbm.E_INVAL
