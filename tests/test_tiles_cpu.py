"""The interior tiling's invariants, checked on the host (no GPU).

The launched tiles (a paired tile owning the last edge strip's rows as its
second column segment) partition every plate, and each launched tile's
prologue lists hold exactly the boundary and second-row nodes of its
segments' areas and one-node rings.

Two-step tiles take two steps per pass from their two-node ring, which must
hold no boundary or second-row node; with overlapped pairs the deep two-step
tiles run beside the single-step launches, which is race-free only if no
deep tile's two-node ring holds a node of a single-step tile and no deep
tile exports.  `tiles_harness.cpp` builds the library's tiles (its host
source, with stub kernel launchers) for plates given on stdin and checks
these invariants node by node, plus that the tiles partition every plate.
"""
import hashlib
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2301_00228_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = [os.path.join(ROOT, "tests", "tiles_harness.cpp"),
           os.path.join(ROOT, "paper_2301_00228_amd", "csrc", "lbm_host.cpp"),
           os.path.join(ROOT, "paper_2301_00228_amd", "csrc", "lbm_types.h"),
           os.path.join(ROOT, "paper_2301_00228_amd", "csrc", "lbm_kernels.h"),
           os.path.join(ROOT, "include", "lbm.h")]


@pytest.fixture(scope="module")
def harness():
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    h = hashlib.sha256()
    for f in SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    exe = os.path.join(tempfile.gettempdir(), f"lbm_tiles_harness_{h.hexdigest()[:16]}")
    if not os.path.exists(exe):
        r = subprocess.run([HIPCC, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                            "-I", os.path.join(ROOT, "paper_2301_00228_amd", "csrc"),
                            SOURCES[0], "-o", exe + ".tmp"], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        os.replace(exe + ".tmp", exe)
    return exe


def check(exe, plates, tiling, overlap=True):
    """plates: list of (mask (ny, nx) 0/1, periodic (px, py))."""
    lines = [" ".join(str(v) for v in (len(plates),) + tuple(tiling) + (int(overlap),))]
    for mask, (px, py) in plates:
        ny, nx = mask.shape
        lines.append(f"{nx} {ny} {int(px)} {int(py)}")
        lines.extend(" ".join(str(int(v)) for v in row) for row in mask)
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, (tiling, overlap, r.stdout[-2000:], r.stderr[-2000:])
    last = r.stdout.strip().splitlines()[-1].split()
    return dict(zip(last[0::2], (int(v) for v in last[1::2])))


TILINGS = [(64, 8, 0, 4, 0, 2, 4), (64, 8, 0, 2, 16, 2, 8), (128, 16, 1, 4, 16, 2, 16),
           (256, 5, 2, 0, 0, 2, 0), (64, 3, 0, 1, 0, 2, 5), (128, 9, 0, 3, 0, 2, 4),
           (64, 8, 0, 4, 0, 1, 0), (128, 16, 3, 4, 16, 2, 16), (64, 8, 3, 4, 16, 2, 16)]


def full(nx, ny):
    return np.ones((ny, nx), np.uint8)


@pytest.mark.parametrize("tiling", TILINGS)
@pytest.mark.parametrize("overlap", [True, False])
def test_plate_with_hole(harness, tiling, overlap):
    case = I.plate_with_hole(n=200, radius=30, sigma=4.0, steps=0)
    got = check(harness, [(case.mask, case.periodic)], tiling, overlap)
    if tiling == TILINGS[0]:
        assert got["single"] > 0 and got["frame"] > 0 and got["deep"] > 0
    if tiling[6] > 0:  # narrow edge strips: paired
        assert got["paired"] > 0


@pytest.mark.parametrize("tiling", TILINGS[:4])
def test_batch_of_plates_with_elliptic_holes(harness, tiling):
    rng = np.random.default_rng(7)
    plates = [(full(c.nx, c.ny) if c.mask is None else c.mask, c.periodic)
              for c in I.plate_batch(count=7, side_lo=20, side_hi=300, steps=0)]
    for nx, ny in ((300, 140), (150, 260)):
        plates.append((I.ellipse_holes_mask(nx, ny, 0.05, rng, a_lo=4.0, a_hi=16.0)[0], (False, False)))
    plates.append((I.shape_mask(180, 150, [(90.3, 74.1, 80.0, 66.0, 0.3, 1), (84.0, 70.0, 20.0, 9.0, 1.1, 0)]),
                   (False, False)))
    got = check(harness, plates, tiling)
    if tiling == TILINGS[0]:
        assert got["single"] > 0 and got["frame"] > 0 and got["deep"] > 0


@pytest.mark.parametrize("tiling", TILINGS[:4])
def test_periodic_and_tiny_plates(harness, tiling):
    strip = full(260, 90)
    strip[30:52, 100:140] = 0  # a rectangular hole in a plate periodic in x
    plates = [(full(96, 96), (True, True)), (strip, (True, False)), (full(3, 3), (False, False)),
              (full(7, 130), (False, False)), (full(131, 7), (False, False)),
              (full(5, 64), (False, True))]
    got = check(harness, plates, tiling)
    assert got["tiles"] > 0
