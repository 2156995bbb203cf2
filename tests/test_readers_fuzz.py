"""Mutation test of the three host mechanism readers, built with the host
address and undefined-behaviour sanitizers (g++, no device code): thousands
of truncated, spliced and garbled variants of the fixtures must each load or
be refused with a documented error code and a message, never crash or read
out of bounds.  No GPU."""
import pathlib
import shutil
import subprocess

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_2508_16105_amd" / "csrc"


@pytest.fixture(scope="module")
def fuzzer(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    out = tmp_path_factory.mktemp("fz") / "readers_fuzz"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-o", str(out), str(ROOT / "tests" / "readers_fuzz.cpp"), str(CSRC / "mechanism.cpp"),
           str(CSRC / "chemkin.cpp"), str(CSRC / "foam.cpp")]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


@pytest.mark.parametrize("kind,files", [
    ("native", ["workloads/mech/m13x.mech"]),
    ("chemkin", ["tests/golden/ck_small.inp"]),
    ("openfoam", ["tests/golden/foam_small/reactions", "tests/golden/foam_small/thermo"]),
])
def test_mutated_files_load_or_are_refused(fuzzer, tmp_path, kind, files):
    args = [str(fuzzer), kind] + [str(ROOT / f) for f in files] + ["7", "1500", str(tmp_path)]
    r = subprocess.run(args, capture_output=True, text=True, timeout=600,
                       env={"ASAN_OPTIONS": "detect_leaks=0", "PATH": "/usr/bin:/bin"})
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "refused" in r.stdout
