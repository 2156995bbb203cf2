"""Host build of the library's per-lane device code for the sanitizer tests.

The library writes the full device source of a mechanism (generated
mechanism code + device/*.hip) when CHEM_DUMP_SOURCE names a file; this module
rewrites the few GPU-only constructs (inline asm that only hides values from
the optimiser, the scalar address space, the dynamic-LDS declaration) into
host C++, includes it into tests/hostemu/driver.cpp together with shim.h, and
compiles it with the host clang++ and the requested sanitizer flags.  Test
infrastructure only."""
from __future__ import annotations

import os
import pathlib
import re
import subprocess
import sys

import numpy as np

ROOT = pathlib.Path(__file__).resolve().parents[1]
EMU = pathlib.Path(__file__).resolve().parent / "hostemu"
CLANG = "/opt/rocm/llvm/bin/clang++"


def dump_device_source(mech_file: str, out: pathlib.Path, lane_max=None) -> str:
    env = dict(os.environ, CHEM_DUMP_SOURCE=str(out))
    if lane_max is not None:
        env["CHEM_LANE_MAX_SPECIES"] = str(lane_max)
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2508_16105_amd import _lib\n"
            "_lib.load_mechanism_handle(%r)\n") % (str(ROOT), str(mech_file))
    subprocess.run([sys.executable, "-c", code], check=True, env=env, cwd=str(ROOT))
    return out.read_text()


def host_source(text: str) -> str:
    """The device source with its GPU-only constructs replaced (semantics kept
    for one lane): the opaque wave-uniform zero becomes 0, empty asm barriers
    vanish, the constant address space is dropped, dynamic LDS is the driver's
    buffer."""
    text = text.replace('asm volatile("s_mov_b32 %0, 0" : "=s"(z));', "z = 0;")
    text = re.sub(r'asm volatile\(""[^;]*\);', "", text)
    text = text.replace("__builtin_amdgcn_readfirstlane(", "(")
    text = text.replace("__builtin_amdgcn_rcp(", "1.0 / (")
    text = text.replace('asm("v_cvt_i32_f64 %0, %1" : "=v"(n) : "v"(nd));', "n = emu_cvt_i32_sat(nd);")
    text = text.replace("__attribute__((address_space(4)))", "")
    text = text.replace("extern __shared__ double lds[];", "double* lds = emu_lds;")
    # one lane per workgroup: the lane's LDS words are consecutive
    assert "constexpr int kLaneStride = 64;" in text
    text = text.replace("constexpr int kLaneStride = 64;", "constexpr int kLaneStride = 1;")
    assert "asm" not in re.sub(r"//.*", "", text).replace("__asm", ""), "unhandled inline asm"
    return text


def build(mech_file: str, workdir: pathlib.Path, flags: list[str], tag: str, lane_max=None) -> pathlib.Path:
    workdir.mkdir(parents=True, exist_ok=True)
    raw = workdir / f"{tag}_device.hip"
    src = workdir / f"{tag}_host.inc"
    src.write_text(host_source(dump_device_source(mech_file, raw, lane_max)))
    exe = workdir / f"{tag}_driver"
    cmd = [CLANG, "-x", "c++", "-std=c++17", "-g", *flags, f'-DEMU_SOURCE="{src}"', f"-I{EMU}",
           str(EMU / "driver.cpp"), "-o", str(exe), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def run(exe: pathlib.Path, workdir: pathlib.Path, mode: int, par, T, p, Y, dt_or_h, rtol, atol, gT=None, gY=None,
        env=None):
    n, ns = Y.shape
    nr = len(par) // 3
    inp = workdir / f"{exe.name}_{mode}.in"
    outp = workdir / f"{exe.name}_{mode}.out"
    with open(inp, "wb") as f:
        np.array([mode, n, ns, nr], dtype=np.int32).tofile(f)
        np.array([dt_or_h, rtol, atol], dtype=np.float64).tofile(f)
        for a in (par, T, p, Y) + ((gT, gY) if mode == 3 else ()):
            np.ascontiguousarray(a, dtype=np.float64).tofile(f)
    # the driver keeps its buffers to the end (no leak report wanted)
    base = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe), str(inp), str(outp)], capture_output=True, text=True, env=dict(base, **(env or {})))
    if r.returncode != 0 or r.stderr.strip():
        raise AssertionError(f"{exe.name} mode {mode}: rc {r.returncode}\n{r.stderr[-4000:]}")
    raw = np.fromfile(outp, dtype=np.uint8)
    n1 = ns + 1
    out = {}
    pos = 0

    def take(name, count, dtype):
        nonlocal pos
        size = count * np.dtype(dtype).itemsize
        out[name] = raw[pos:pos + size].view(dtype).copy()
        pos += size

    if mode == 0:
        take("T", n, np.float64); take("Y", n * ns, np.float64); take("counts", 3 * n, np.int32)
        out["Y"] = out["Y"].reshape(n, ns)
        out["status"], out["nacc"], out["nrej"] = out["counts"].reshape(3, n)
    elif mode == 1:
        take("ynew", n * n1, np.float64); take("err", n, np.float64); take("ok", n, np.int32)
        out["ynew"] = out["ynew"].reshape(n, n1)
    elif mode == 2:
        take("f", n * n1, np.float64); take("J", n * n1 * n1, np.float64)
        out["f"] = out["f"].reshape(n, n1)
        out["J"] = out["J"].reshape(n, n1, n1)
    else:
        take("gT0", n, np.float64); take("gY0", n * ns, np.float64); take("gpar", 3 * nr, np.float64)
        take("Te", n, np.float64); take("Ye", n * ns, np.float64); take("status", n, np.int32)
        out["gY0"] = out["gY0"].reshape(n, ns)
        out["Ye"] = out["Ye"].reshape(n, ns)
    assert pos == raw.size, (pos, raw.size)
    return out
