"""The library's per-lane device code run on the host under sanitizers.

The full device source the library generates for a mechanism (mechanism code
+ integrator) is compiled as host C++ through tests/hostemu/shim.h and run one
lane at a time by tests/hostemu/driver.cpp, in three builds:
  * address + undefined-behaviour sanitizers (array bounds, float-to-int
    overflow, ...), every automatic variable pre-filled with a pattern;
  * every automatic variable pre-filled with zeros (no sanitizer);
  * the memory sanitizer (reads of uninitialised values, with origins).
A clean run, bitwise-equal results of the pattern and zero builds (a read of
an uninitialised variable would make them differ) and agreement with the
oracle are required for the integration, the fixed step with its error norm,
the source terms and Jacobian, and the discrete adjoint.  This is how
undefined behaviour in the device code is looked for without a GPU: it found
that exp_poly converted a NaN exponent to int (a NaN stage of a rejected
step), which LLVM turns into poison.  No GPU."""
import pathlib
import subprocess

import numpy as np
import pytest

import hostemu_build as hb
from errnorm_ref import errnorm_bar, errnorm_with_spread
from workloads import mech_path, mech_text
from workloads.states import rde_field, uniform_cells

RU = 8.314462618
MECHS = ("m9", "m13x")
BUILDS = {
    "pattern": ["-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                "-ftrivial-auto-var-init=pattern"],
    "zero": ["-O1", "-ftrivial-auto-var-init=zero"],
    "msan": ["-O1", "-fsanitize=memory", "-fsanitize-memory-track-origins"],
}


@pytest.fixture(scope="module")
def drivers(tmp_path_factory):
    if not pathlib.Path(hb.CLANG).exists():
        pytest.skip("host clang++ not available")
    import paper_2508_16105_amd  # noqa: F401  (the library generates the source)
    wd = tmp_path_factory.mktemp("hostemu")
    procs, exes = [], {}
    for name in MECHS:
        raw = wd / f"{name}_device.hip"
        src = wd / f"{name}_host.inc"
        src.write_text(hb.host_source(hb.dump_device_source(mech_path(name), raw)))
        for tag, flags in BUILDS.items():
            exe = wd / f"{name}_{tag}"
            cmd = [hb.CLANG, "-x", "c++", "-std=c++17", "-g", *flags, f'-DEMU_SOURCE="{src}"', f"-I{hb.EMU}",
                   str(hb.EMU / "driver.cpp"), "-o", str(exe), "-lm"]
            procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True), cmd))
            exes[(name, tag)] = exe
    for pr, cmd in procs:
        out = pr.communicate()[0]
        assert pr.returncode == 0, (cmd, out[-3000:])
    return wd, exes


def _params(name):
    import paper_2508_16105_amd as chem
    a, b, e = chem.Mechanism(mech_path(name)).get_params()
    return np.concatenate([a, b, e / RU])


def _cells(name, n=48):
    """Independent cells over 300-3000 K and 0.005-2000 atm, plus RDE-shaped
    front, burnt and fresh cells: hot cells at these pressures take rejected
    steps with non-finite stages, the path where the defect was found."""
    T, p, Y = uniform_cells(mech_text(name), n, 31)
    p = 101325.0 * np.exp(np.random.default_rng(3).uniform(np.log(0.005), np.log(2000.0), n))
    Tr, pr, Yr, reg = rde_field(mech_text(name), 32, 32, 101)
    idx = np.concatenate([np.where(reg == r)[0][:6] for r in (0, 1, 2)])
    return np.concatenate([T, Tr[idx]]), np.concatenate([p, pr[idx]]), np.concatenate([Y, Yr[idx]])


@pytest.mark.parametrize("name", MECHS)
def test_integration_clean_and_matches_oracle(drivers, oracle_lib, name):
    wd, exes = drivers
    par = _params(name)
    T, p, Y = _cells(name)
    dt, rtol, atol = 1e-8, 1e-8, 1e-12
    outs = {tag: hb.run(exes[(name, tag)], wd, 0, par, T, p, Y, dt, rtol, atol) for tag in BUILDS}
    for k in ("T", "Y", "counts"):
        assert np.array_equal(outs["pattern"][k], outs["zero"][k]), k
        assert np.array_equal(outs["pattern"][k], outs["msan"][k]), k
    om = oracle_lib.Mechanism(mech_path(name))
    To, Yo, nao, nro, sto = om.integrate(T, p, Y, dt, rtol, atol)
    o = outs["pattern"]
    assert np.array_equal(o["status"], sto)
    ok = sto == 0
    assert np.all(np.abs(o["T"] - To)[ok] <= 1e-6 * To[ok])
    assert np.all(np.abs(o["Y"] - Yo)[ok] <= 1e-8)
    assert np.sum((o["nacc"] != nao) | (o["nrej"] != nro)) <= max(1, len(T) // 50)


@pytest.mark.parametrize("name", MECHS)
def test_fixed_step_and_error_norm_match_oracle(drivers, oracle_lib, name):
    wd, exes = drivers
    par = _params(name)
    T, p, Y = uniform_cells(mech_text(name), 32, 22)
    om = oracle_lib.Mechanism(mech_path(name))
    for h in (1e-12, 1e-10):
        outs = {tag: hb.run(exes[(name, tag)], wd, 1, par, T, p, Y, h, 1e-8, 1e-12) for tag in BUILDS}
        for k in ("ynew", "err", "ok"):
            assert np.array_equal(outs["pattern"][k], outs["zero"][k], equal_nan=True), k
        o = outs["pattern"]
        for i in range(len(T)):
            y0 = np.concatenate([[T[i]], Y[i]])
            eno, spread, yo, _ = errnorm_with_spread(om, p[i], y0, h, 1e-8, 1e-12)
            if not (np.all(np.isfinite(yo)) and np.isfinite(eno)):
                assert o["ok"][i] == 0
                continue
            assert o["ok"][i] == 1
            assert abs(o["ynew"][i, 0] - yo[0]) <= 1e-10 * yo[0]
            assert np.all(np.abs(o["ynew"][i, 1:] - yo[1:]) <= 1e-12)
            assert abs(o["err"][i] - eno) <= errnorm_bar(eno, spread), (i, o["err"][i], eno)


@pytest.mark.parametrize("name", MECHS)
def test_source_terms_and_jacobian_match_oracle(drivers, oracle_lib, name):
    wd, exes = drivers
    par = _params(name)
    T, p, Y = uniform_cells(mech_text(name), 24, 21)
    outs = {tag: hb.run(exes[(name, tag)], wd, 2, par, T, p, Y, 0.0, 0.0, 0.0) for tag in BUILDS}
    assert np.array_equal(outs["pattern"]["J"], outs["zero"]["J"])
    om = oracle_lib.Mechanism(mech_path(name))
    o = outs["pattern"]
    for i in range(len(T)):
        y = np.concatenate([[T[i]], Y[i]])
        fo = om.rhs(p[i], y)
        assert np.all(np.abs(o["f"][i] - fo) <= 1e-11 * np.abs(fo).max() + 1e-300)
        Jo = om.jac_cs(p[i], y)
        Ja = om.jac(p[i], y)
        sc = np.abs(Jo).max(axis=1, keepdims=True) * np.maximum(np.abs(y), 1e-3)[None, :] \
            / np.maximum(np.abs(y), 1e-3).max()
        assert np.all(np.abs(o["J"][i] - Jo) <= 1e-10 * (np.abs(Jo) + sc) + 4.0 * np.abs(Ja - Jo)), i


@pytest.mark.parametrize("name", MECHS)
def test_adjoint_clean_and_matches_oracle(drivers, oracle_lib, name):
    """The lane adjoint (checkpointed rerun, reverse sweep with dual-number
    second-order terms), where a NaN gradient once appeared on the GPU."""
    wd, exes = drivers
    par = _params(name)
    T, p, Y = _cells(name, 16)
    n, ns = Y.shape
    rng = np.random.default_rng(17)
    gT = np.full(n, 1e-3)
    gY = rng.standard_normal((n, ns))
    dt, rtol, atol = 1e-8, 1e-8, 1e-12
    outs = {tag: hb.run(exes[(name, tag)], wd, 3, par, T, p, Y, dt, rtol, atol, gT, gY) for tag in BUILDS}
    # checkpoints at every step: the reverse sweep reads the forward rerun's
    # trail instead of the segment replay's stash; bitwise the same
    trail = hb.run(exes[(name, "pattern")], wd, 3, par, T, p, Y, dt, rtol, atol, gT, gY, env={"EMU_ADJ_K": "1"})
    for k in ("gT0", "gY0", "gpar"):
        assert np.array_equal(outs["pattern"][k], outs["zero"][k]), k
        assert np.array_equal(outs["pattern"][k], outs["msan"][k]), k
        assert np.array_equal(outs["pattern"][k], trail[k], equal_nan=True), k
    o = outs["pattern"]
    om = oracle_lib.Mechanism(mech_path(name))
    oT0, oY0, oa, ob, oe = om.adjoint(T, p, Y, dt, rtol, atol, gT, gY)
    ok = o["status"] == 0
    assert ok.sum() >= n - 2
    assert np.all(np.isfinite(o["gT0"][ok])) and np.all(np.isfinite(o["gpar"]))
    relT = np.abs(o["gT0"] - oT0)[ok] / np.abs(oT0)[ok]
    relY = np.max(np.abs(o["gY0"] - oY0), axis=1)[ok] / np.max(np.abs(oY0), axis=1)[ok]
    # 1e-5 relative, as the GPU adjoint; a cell whose error estimate is
    # rounding-dominated may move by more (the GPU test bounds those by the
    # oracle's own 1-ulp spread): at most one such cell here
    assert (relT > 1e-5).sum() + (relY > 1e-5).sum() <= 1, (relT.max(), relY.max())
    if ok.all():
        nr = len(par) // 3
        for g, ref in ((o["gpar"][:nr], oa), (o["gpar"][nr:2 * nr], ob), (o["gpar"][2 * nr:], oe)):
            assert np.max(np.abs(g - ref)) <= 1e-5 * np.max(np.abs(ref))
