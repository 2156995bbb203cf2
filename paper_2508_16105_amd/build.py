"""Build the chemistry library in-tree.

1. Embed csrc/device/*.hip into the host library as strings (the device
   code is compiled per mechanism, with the generated mechanism-specific
   code in front of it, by hipRTC for gfx950).
2. Compile the host library libchemmi.so with hipcc (HIP runtime + hipRTC).
3. Load each mechanism under workloads/mech so its gfx950 code object is
   compiled now and stored in the kernel cache beside the library.
"""
from __future__ import annotations

import os
import pathlib
import subprocess
import sys

PKG = pathlib.Path(__file__).resolve().parent
CSRC = PKG / "csrc"
LIB = PKG / "libchemmi.so"
ROOT = PKG.parent
# (mechanism, CHEM_LANE_MAX_SPECIES at load): the default builds and the
# wave-cooperative builds of the 9- and 13-species mechanisms
PREBUILT = [("m9", None), ("m13", None), ("m32", None), ("m9", "0"), ("m13", "0"),
            ("m13x", None), ("m13x", "0"), ("m32x", None), ("m16", None)]
# CHEMKIN renderings the tests load (written into the build folder first)
PREBUILT_CHEMKIN = ["m9", "m32x"]
# OpenFOAM renderings the tests load
PREBUILT_OPENFOAM = ["m9", "m32s"]
HOST_SOURCES = ["capi.cpp", "runtime.cpp", "module.cpp", "mechanism.cpp", "chemkin.cpp", "foam.cpp", "codegen.cpp",
                "noalloc.hip"]


def embed_device_source():
    delim = "CHEMDEV"
    out = "// generated from device/*.hip by build.py; do not edit\n"
    for var, name in (("kMathSource", "math.hip"), ("kCommonSource", "common.hip"),
                      ("kIntegratorSource", "integrator.hip"), ("kWideSource", "wide.hip"),
                      ("kEulerSource", "euler.hip")):
        src = (CSRC / "device" / name).read_text()
        assert f"){delim}\"" not in src
        out += f"static const char {var}[] = R\"{delim}(\n{src}){delim}\";\n"
    target = CSRC / "_device_source.inc"
    if not target.exists() or target.read_text() != out:
        target.write_text(out)


def compile_host(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "-Wall", "-Wno-unused-result",
           "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           *[str(CSRC / s) for s in HOST_SOURCES], "-o", str(tmp), "-lhiprtc", "-ldl"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)


def prebuild_mechanisms(builds=None):
    """Compile the device code of the committed mechanisms into the cache."""
    sys.path.insert(0, str(ROOT))
    from paper_2508_16105_amd import _lib
    mdir = ROOT / "workloads" / "mech"
    old = os.environ.get("CHEM_LANE_MAX_SPECIES")
    try:
        for nm, lane_max in builds or PREBUILT:
            if lane_max is None:
                os.environ.pop("CHEM_LANE_MAX_SPECIES", None)
            else:
                os.environ["CHEM_LANE_MAX_SPECIES"] = lane_max
            _lib.load_mechanism_handle(str(mdir / f"{nm}.mech"))
        os.environ.pop("CHEM_LANE_MAX_SPECIES", None)
        _lib.load_mechanism_handle(str(ROOT / "tests" / "golden" / "ck_small.inp"))
        if builds is None:
            import tempfile
            from workloads import gen_mech
            with tempfile.TemporaryDirectory() as td:
                for nm in PREBUILT_CHEMKIN:
                    p = pathlib.Path(td) / f"{nm}.inp"
                    p.write_text(gen_mech.to_chemkin(gen_mech.build_mechanism(nm)))
                    _lib.load_mechanism_handle(str(p))
                for nm in PREBUILT_OPENFOAM:
                    r, t = gen_mech.to_openfoam(gen_mech.build_mechanism(nm))
                    rp, tp = pathlib.Path(td) / f"{nm}.foam", pathlib.Path(td) / "thermo"
                    rp.write_text(r)
                    tp.write_text(t)
                    _lib.load_mechanism_handle(str(rp), str(tp), "openfoam")
            fx = ROOT / "tests" / "golden" / "foam_small"
            _lib.load_mechanism_handle(str(fx / "reactions"), str(fx / "thermo"), "openfoam")
    finally:
        if old is None:
            os.environ.pop("CHEM_LANE_MAX_SPECIES", None)
        else:
            os.environ["CHEM_LANE_MAX_SPECIES"] = old


def prune_cache(since):
    """Drop cached code objects neither produced nor used since `since`."""
    for f in (PKG / "kcache").glob("*.co"):
        if f.stat().st_mtime < since:
            f.unlink()


def build(verbose=False, mechanisms=True):
    import time
    t0 = time.time() - 1.0
    embed_device_source()
    compile_host(verbose)
    if mechanisms:
        prebuild_mechanisms()
        prune_cache(t0)


if __name__ == "__main__":
    build(verbose=True)
