"""The launch-shape tuner: it times candidate launch shapes and both cell
orders on a sample of the field (results are bitwise the same in every case),
keeps the fastest per size bucket, and records it on disk, so a second
process reuses it without timing anything; both processes give bitwise the
same results."""
import json
import os
import pathlib
import subprocess
import sys

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = pathlib.Path(__file__).resolve().parents[1]

CHILD = r"""
import json, sys
import numpy as np
import torch
sys.path.insert(0, {root!r})
import paper_2508_16105_amd as chem
from workloads import mech_path, mech_text
from workloads.states import rde_field
T, p, Y, _ = rde_field(mech_text("m9"), 128, 128, 406)
g = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")
m = chem.Mechanism(mech_path("m9"))
Te, Ye, st = chem.integrate(m, g(T), g(p), g(Y), 5e-9, 1e-8, 1e-12, form=chem.FORM_PERSISTENT)
print(json.dumps({{"T": Te.cpu().numpy().tolist()[:4096:97], "sum": float(Ye.sum()), "failed": st["failed"]}}))
"""


def _child(tmp):
    env = dict(os.environ, CHEM_TUNE_CACHE=str(tmp), CHEM_LOG="1")
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=str(ROOT))], capture_output=True, text=True,
                       env=env, timeout=240)
    assert r.returncode == 0, r.stderr[-3000:]
    return json.loads(r.stdout.strip().splitlines()[-1]), r.stderr


def test_tuning_is_recorded_and_reused_across_processes(tmp_path):
    first, log1 = _child(tmp_path)
    tuned = [ln for ln in log1.splitlines() if "autotune block=" in ln]
    assert len(tuned) >= 2 and any("order=1" in ln for ln in tuned) and any("order=2" in ln for ln in tuned), log1
    files = list(tmp_path.glob("tune-*.txt"))
    assert len(files) == 1
    block, refill, order = (int(x) for x in files[0].read_text().split()[:3])
    assert block in (64, 128, 256) and refill in (4, 16, 32) and order in (1, 2)
    second, log2 = _child(tmp_path)
    assert "autotune cache hit" in log2 and "autotune block=" not in log2, log2
    assert first == second and first["failed"] == 0
