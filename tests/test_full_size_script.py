"""tests/full_size_oracle.py (run by hand at full size) on a tiny plate: the
oracle side of the two-machine comparison writes its sampled rows, and the
comparison of a copy of them reports zero error."""
import json
import os
import shutil
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SCRIPT = os.path.join(ROOT, "tests", "full_size_oracle.py")


def test_oracle_rows_and_compare(tmp_path):
    orc = tmp_path / "oracle"
    gpu = tmp_path / "gpu"
    r = subprocess.run([sys.executable, SCRIPT, "--rows", "oracle", "--n", "96", "--radius", "12",
                        "--steps", "60", "--row-every", "8", "--out", str(orc)],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    ref = np.load(orc / "oracle.npz")
    assert list(ref["rows"]) == list(range(0, 96, 8))
    assert ref["e"].shape == (12, 96) and ref["u"].shape == (2, 12, 96)
    assert np.abs(ref["u"]).max() > 0
    gpu.mkdir()
    meta = json.loads(str(ref["meta"]))
    meta["storage"] = "copy"
    np.savez(gpu / "copy.npz", e=ref["e"], omega=ref["omega"], u=ref["u"], rows=ref["rows"],
             meta=json.dumps(meta))
    r = subprocess.run([sys.executable, SCRIPT, "--compare", str(gpu), str(orc)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["steps"] == 60 and out["sampled_rows"] == 12
    for k in ("e", "omega", "u"):
        assert out["copy"]["rel_l2"][k] == 0.0 and out["copy"]["rel_max"][k] == 0.0
