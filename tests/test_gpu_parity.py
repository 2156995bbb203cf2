"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances: |dT| <= 1e-6 T and |dY_k| <= 1e-8 at rtol 1e-8, atol 1e-12 for
integrated states; source terms and Jacobians to round-off (1e-11 relative to
the row scale); the persistent and plain forms bitwise."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from workloads import WORKLOADS, mech_path, mech_text  # noqa: E402
from workloads.states import rde_field, uniform_cells  # noqa: E402

from errnorm_ref import errnorm_bar, errnorm_with_spread  # noqa: E402

DT, RTOL, ATOL = 5e-9, 1e-8, 1e-12


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def chem():
    import paper_2508_16105_amd as chem
    return chem


@pytest.fixture(scope="module")
def mechs(chem, oracle_lib):
    out = {}
    for name in ("m9", "m13"):
        out[name] = (chem.Mechanism(mech_path(name)), oracle_lib.Mechanism(mech_path(name)))
    return out


def _g(a, dev):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def _assert_state_parity(Tg, Yg, To, Yo, what):
    dT = np.abs(Tg - To)
    dY = np.abs(Yg - Yo)
    bad = (dT > 1e-6 * To) | np.any(dY > 1e-8, axis=1)
    assert not bad.any(), (f"{what}: {bad.sum()} cells out of tolerance; max |dT|/T "
                           f"{(dT / To).max():.3e}, max |dY| {dY.max():.3e}")


@pytest.mark.parametrize("name", ["m9", "m13"])
def test_source_terms_and_jacobian_match_oracle(chem, mechs, dev, name):
    gm, om = mechs[name]
    T, p, Y = uniform_cells(mech_text(name), 200, 21)
    f, J = chem.eval_source(gm, _g(T, dev), _g(p, dev), _g(Y, dev))
    f, J = f.cpu().numpy(), J.cpu().numpy()
    for i in range(len(T)):
        y = np.concatenate([[T[i]], Y[i]])
        fo = om.rhs(p[i], y)
        Jo = om.jac_cs(p[i], y)
        assert np.all(np.abs(f[i] - fo) <= 1e-11 * np.abs(fo).max() + 1e-300), (i, f[i], fo)
        sc = np.abs(Jo).max(axis=1, keepdims=True) * np.maximum(np.abs(y), 1e-3)[None, :] \
            / np.maximum(np.abs(y), 1e-3).max()
        assert np.all(np.abs(J[i] - Jo) <= 1e-10 * (np.abs(Jo) + sc)), (name, i)


@pytest.mark.parametrize("name", ["m9", "m13"])
def test_source_terms_at_the_thermo_range_ends(chem, mechs, dev, name):
    """States at the ends of the NASA-7 range (200-230 K, 4500-6000 K) and
    from 0.1 to 100 atm, where the rate exponentials reach their largest
    arguments: source terms and Jacobian against the oracle (finite results
    agree to the same bar; a non-finite oracle result is non-finite here)."""
    gm, om = mechs[name]
    _, _, Y = uniform_cells(mech_text(name), 64, 24)
    rng = np.random.default_rng(25)
    T = np.concatenate([rng.uniform(200.0, 230.0, 32), rng.uniform(4500.0, 6000.0, 32)])
    p = 101325.0 * np.exp(rng.uniform(np.log(0.1), np.log(100.0), 64))
    f, J = chem.eval_source(gm, _g(T, dev), _g(p, dev), _g(Y, dev))
    f, J = f.cpu().numpy(), J.cpu().numpy()
    checked = 0
    for i in range(len(T)):
        y = np.concatenate([[T[i]], Y[i]])
        fo = om.rhs(p[i], y)
        if not np.all(np.isfinite(fo)):
            assert not np.all(np.isfinite(f[i])), i
            continue
        assert np.all(np.abs(f[i] - fo) <= 1e-11 * np.abs(fo).max() + 1e-300), (i, T[i], f[i], fo)
        Jo = om.jac_cs(p[i], y)
        Ja = om.jac(p[i], y)
        sc = np.abs(Jo).max(axis=1, keepdims=True) * np.maximum(np.abs(y), 1e-3)[None, :] \
            / np.maximum(np.abs(y), 1e-3).max()
        tol = 1e-10 * (np.abs(Jo) + sc) + 4.0 * np.abs(Ja - Jo)
        assert np.all(np.abs(J[i] - Jo) <= tol), (name, i, T[i])
        checked += 1
    assert checked >= 48


def test_fixed_step_matches_oracle(chem, mechs, dev):
    gm, om = mechs["m9"]
    T, p, Y = uniform_cells(mech_text("m9"), 128, 22)
    for h in (1e-11, 1e-9):
        yn, en, ok = chem.step_fixed(gm, _g(T, dev), _g(p, dev), _g(Y, dev), h, RTOL, ATOL)
        yn = yn.cpu().numpy()
        assert ok.cpu().numpy().all()
        en = en.cpu().numpy()
        for i in range(len(T)):
            y0 = np.concatenate([[T[i]], Y[i]])
            eno, spread, yo, eo = errnorm_with_spread(om, p[i], y0, h, RTOL, ATOL)
            assert abs(yn[i, 0] - yo[0]) <= 1e-10 * yo[0]
            assert np.all(np.abs(yn[i, 1:] - yo[1:]) <= 1e-12)
            # the embedded error estimate that decides acceptance
            assert abs(en[i] - eno) <= errnorm_bar(eno, spread), (h, i, en[i], eno, spread)


def test_integrate_uniform4k_matches_oracle(chem, mechs, dev):
    """The small parity workload in full: 4096 independent cells (64 waves, a
    ragged last tile is covered by the ragged-size test)."""
    w = WORKLOADS["uniform4k"]
    gm, om = mechs["m9"]
    T, p, Y = uniform_cells(mech_text("m9"), w["n"], w["seed"])
    Tg, Yg, stats, st, na, nr = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), w["dt"],
                                               w["rtol"], w["atol"], return_counts=True)
    To, Yo, nao, nro, sto = om.integrate(T, p, Y, w["dt"], w["rtol"], w["atol"])
    assert stats["failed"] == 0 and np.all(sto == 0) and np.all(st.cpu().numpy() == 0)
    _assert_state_parity(Tg.cpu().numpy(), Yg.cpu().numpy(), To, Yo, "uniform4k")
    na, nr = na.cpu().numpy(), nr.cpu().numpy()
    assert stats["accepted"] == na.sum() and stats["rejected"] == nr.sum()
    differ = np.sum((na != nao) | (nr != nro))
    assert differ <= 0.01 * len(T), f"{differ} cells took a different step sequence"


def test_integrate_rde_field_matches_oracle(chem, mechs, dev):
    """A 256 x 256 RDE-shaped field (fresh, front and burnt cells)."""
    gm, om = mechs["m9"]
    T, p, Y, reg = rde_field(mech_text("m9"), 256, 256, 101)
    Tg, Yg, stats = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), DT, RTOL, ATOL)
    To, Yo, _, _, sto = om.integrate(T, p, Y, DT, RTOL, ATOL)
    assert stats["failed"] == 0 and np.all(sto == 0)
    _assert_state_parity(Tg.cpu().numpy(), Yg.cpu().numpy(), To, Yo, "rde 256x256")


def test_m13_third_body_and_troe_integration(chem, mechs, dev):
    gm, om = mechs["m13"]
    T, p, Y = uniform_cells(mech_text("m13"), 1024, 31)
    Tg, Yg, stats = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), 1e-8, RTOL, ATOL)
    To, Yo, _, _, sto = om.integrate(T, p, Y, 1e-8, RTOL, ATOL)
    assert stats["failed"] == 0 and np.all(sto == 0)
    _assert_state_parity(Tg.cpu().numpy(), Yg.cpu().numpy(), To, Yo, "m13 uniform")


@pytest.mark.parametrize("name", ["m9", "m13"])
def test_persistent_is_bitwise_equal_to_plain(chem, mechs, dev, name):
    gm, _ = mechs[name]
    T, p, Y, reg = rde_field(mech_text(name), 256, 256, 101)
    Tp, Yp, sp, stp, nap, nrp = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), DT, RTOL, ATOL,
                                               return_counts=True)
    cost = (nap + nrp).contiguous()
    for block, refill, extra in ((64, 1, {}), (256, 16, {"order": chem.ORDER_NATURAL}),
                                 (128, 64, {"cost": cost}), (64, 8, {"cost": torch.zeros_like(cost)})):
        Tq, Yq, sq, stq, naq, nrq = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), DT, RTOL,
                                                   ATOL, form=chem.FORM_PERSISTENT, block=block,
                                                   refill=refill, return_counts=True, **extra)
        assert torch.equal(Tp, Tq) and torch.equal(Yp, Yq)
        assert torch.equal(nap, naq) and torch.equal(nrp, nrq) and torch.equal(stp, stq)
        assert sq["accepted"] == sp["accepted"] and sq["cells"] == sp["cells"]


def test_calls_on_two_streams_are_ordered(chem, mechs, dev):
    """Two asynchronous persistent calls on one handle from two streams share
    the handle's device workspace; the second is ordered after the first, so
    both equal the same calls made one after the other."""
    gm, _ = mechs["m9"]
    fields = [rde_field(mech_text("m9"), 256, 256, seed)[:3] for seed in (101, 202)]
    ref = [chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), DT, RTOL, ATOL,
                          form=chem.FORM_PERSISTENT)[:2] for T, p, Y in fields]
    ins = [[_g(x, dev) for x in f] for f in fields]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    outs = []
    for (T, p, Y), s in zip(ins, streams):
        with torch.cuda.stream(s):
            outs.append(chem.integrate(gm, T, p, Y, DT, RTOL, ATOL, form=chem.FORM_PERSISTENT,
                                       stats=False)[:2])
    torch.cuda.synchronize()
    for (Tr, Yr), (To, Yo) in zip(ref, outs):
        assert torch.equal(Tr, To) and torch.equal(Yr, Yo)


@pytest.mark.parametrize("name", ["m9", "m13"])
def test_batched_fields_match_per_field_plain(chem, mechs, dev, oracle_lib, name):
    gm, om = mechs[name]
    sizes = [1000, 33, 70001, 1, 4097, 64]
    fields = []
    for i, n in enumerate(sizes):
        from workloads.states import rde_field_n
        T, p, Y, _ = rde_field_n(mech_text(name), n, 500 + i)
        fields.append((T, p, Y))
    Ts = [_g(f[0], dev) for f in fields]
    ps = [_g(f[1], dev) for f in fields]
    Ys = [_g(f[2], dev) for f in fields]
    stats = chem.integrate_batched(gm, Ts, ps, Ys, DT, RTOL, ATOL)
    assert stats["cells"] == sum(sizes) and stats["failed"] == 0
    for (T, p, Y), Tb, Yb in zip(fields, Ts, Ys):
        Tr, Yr, _ = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), DT, RTOL, ATOL)
        assert torch.equal(Tr, Tb) and torch.equal(Yr, Yb)
    # oracle on a sample of every field
    rng = np.random.default_rng(0)
    for (T, p, Y), Tb, Yb in zip(fields, Ts, Ys):
        idx = rng.choice(len(T), size=min(len(T), 200), replace=False)
        To, Yo, _, _, _ = om.integrate(T[idx], p[idx], Y[idx], DT, RTOL, ATOL)
        _assert_state_parity(Tb.cpu().numpy()[idx], Yb.cpu().numpy()[idx], To, Yo, f"batched {name}")


def test_full_size_rde1m_sampled(chem, mechs, dev):
    """The headline workload at full size in both launch forms: sampled cells
    against the oracle, and properties that hold for every cell."""
    w = WORKLOADS["rde1m"]
    gm, om = mechs["m9"]
    T, p, Y, reg = rde_field(mech_text("m9"), w["width"], w["height"], w["seed"])
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(np.where(reg == r)[0], 300, replace=False) for r in (0, 1, 2)])
    To, Yo, _, _, _ = om.integrate(T[idx], p[idx], Y[idx], w["dt"], w["rtol"], w["atol"])
    out = {}
    for form in (chem.FORM_PLAIN, chem.FORM_PERSISTENT):
        Tg, Yg, stats, st, na, nr = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), w["dt"],
                                                   w["rtol"], w["atol"], form=form, return_counts=True)
        assert stats["failed"] == 0 and stats["cells"] == len(T)
        Tn, Yn = Tg.cpu().numpy(), Yg.cpu().numpy()
        _assert_state_parity(Tn[idx], Yn[idx], To, Yo, f"rde1m form {form}")
        nsub = (na + nr).cpu().numpy()
        assert np.all(np.abs(Yn.sum(1) - 1.0) <= 1e-13 * np.maximum(nsub, 1) + 1e-14)
        assert np.all(Tn > 0) and np.all(np.isfinite(Yn))
        out[form] = (Tg, Yg)
    assert torch.equal(out[chem.FORM_PLAIN][0], out[chem.FORM_PERSISTENT][0])
    assert torch.equal(out[chem.FORM_PLAIN][1], out[chem.FORM_PERSISTENT][1])


@pytest.mark.parametrize("n", [1, 63, 65, 4097])
def test_ragged_sizes(chem, mechs, dev, n):
    gm, om = mechs["m9"]
    T, p, Y = uniform_cells(mech_text("m9"), n, 40 + n)
    Tg, Yg, stats = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), 1e-8, RTOL, ATOL)
    To, Yo, _, _, _ = om.integrate(T, p, Y, 1e-8, RTOL, ATOL)
    assert stats["cells"] == n
    _assert_state_parity(Tg.cpu().numpy(), Yg.cpu().numpy(), To, Yo, f"n={n}")


def test_bad_cells_and_failure_codes(chem, mechs, dev):
    gm, om = mechs["m9"]
    T, p, Y = uniform_cells(mech_text("m9"), 8, 50)
    T[2] = -10.0
    Y[3, 4] = np.nan
    p[5] = 0.0
    Tg, Yg, stats, st, na, nr = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), 1e-8, RTOL,
                                               ATOL, return_counts=True, allow_failed=True)
    st = st.cpu().numpy()
    assert list(np.where(st == 4)[0]) == [2, 3, 5] and stats["failed"] == 3
    assert Tg[2].item() == -10.0 and np.isnan(Yg[3, 4].item())
    with pytest.raises(chem.ChemError) as e:
        chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), 1e-8, RTOL, ATOL)
    assert e.value.code == -6
    # max_substeps = 1: hot cells cannot finish
    T2, p2, Y2 = uniform_cells(mech_text("m9"), 64, 51)
    Tg, Yg, stats, st, na, nr = chem.integrate(gm, _g(T2, dev), _g(p2, dev), _g(Y2, dev), 1e-8, RTOL,
                                               ATOL, max_substeps=1, return_counts=True,
                                               allow_failed=True)
    _, _, nao, nro, sto = om.integrate(T2, p2, Y2, 1e-8, RTOL, ATOL, max_substeps=1)
    assert np.array_equal(st.cpu().numpy(), sto)
    assert np.all((na + nr).cpu().numpy() <= 1)


def test_argument_errors(chem, mechs, dev):
    gm, _ = mechs["m9"]
    T, p, Y = uniform_cells(mech_text("m9"), 8, 52)
    with pytest.raises(ValueError):
        chem.integrate(gm, torch.tensor(T), _g(p, dev), _g(Y, dev), 1e-8, RTOL, ATOL)
    import ctypes as C
    from paper_2508_16105_amd import _lib
    Th = np.ascontiguousarray(T)
    rc = _lib.lib().chem_integrate(gm.h, 8, C.c_void_p(Th.ctypes.data), C.c_void_p(_g(p, dev).data_ptr()),
                                   C.c_void_p(_g(Y, dev).data_ptr()), 1e-8, RTOL, ATOL, None, None,
                                   None, None, None, None)
    assert rc == -1 and b"device pointer" in _lib.lib().chem_last_error()


def test_h0_option(chem, mechs, dev):
    """A per-cell first trial step changes the step sequence, not the answer."""
    gm, om = mechs["m9"]
    T, p, Y = uniform_cells(mech_text("m9"), 256, 53)
    h0 = _g(np.full(256, 1e-12), dev)
    Tg, Yg, _ = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), 1e-8, RTOL, ATOL, h0=h0)
    To, Yo, _, _, _ = om.integrate(T, p, Y, 1e-8, 1e-12, 1e-16)       # near-exact reference
    # a different step sequence: agreement at the tolerance level, not bitwise
    assert np.all(np.abs(Tg.cpu().numpy() - To) <= 1e-6 * To)
    assert np.all(np.abs(Yg.cpu().numpy() - Yo) <= 1e-7)


RU = 8.314462618


def _source_terms(om, T, p, Y, Tend, Yend, dt):
    """The operator-split reaction terms of a step from its two end states
    (eqs. (20)-(21)): wdot = rho0 (Y_end - Y_0)/dt, qdot = -sum h_k(298.15 K) wdot_k."""
    W = om.weights()
    rho0 = p / (RU * T * (Y / W).sum(axis=1))
    wdot = rho0[:, None] * (Yend - Y) / dt
    _, hrt, _ = om.thermo(298.15)
    hf = RU * 298.15 * hrt / W
    return wdot, -(wdot * hf).sum(axis=1), rho0


@pytest.mark.parametrize("name,form", [("m9", "plain"), ("m9", "persistent"), ("m13", "plain")])
def test_source_mode_matches_integrate_and_oracle(chem, mechs, dev, name, form):
    """chem_integrate_source: the state it leaves equals chem_integrate's
    (bitwise); its rates equal those formed from its own end state (to
    round-off, which pins rho0, the difference and h(298.15 K)); and against
    the oracle's end state they agree to the parity bar carried through the
    formulas (|dY| <= 1e-8 gives |d wdot| <= rho0 1e-8 / dt)."""
    gm, om = mechs[name]
    f = chem.FORM_PERSISTENT if form == "persistent" else chem.FORM_PLAIN
    T, p, Y, reg = rde_field(mech_text(name), 64, 64, 105)
    Tg, Yg, wg, qg, stats, st = chem.integrate_source(gm, _g(T, dev), _g(p, dev), _g(Y, dev), DT, RTOL, ATOL,
                                                       form=f, return_status=True)
    Ti, Yi, _ = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), DT, RTOL, ATOL, form=f)
    assert torch.equal(Tg, Ti) and torch.equal(Yg, Yi)
    assert stats["failed"] == 0 and np.all(st.cpu().numpy() == 0)
    wg, qg = wg.cpu().numpy(), qg.cpu().numpy()
    ws, qs, rho0 = _source_terms(om, T, p, Y, Tg.cpu().numpy(), Yg.cpu().numpy(), DT)
    _, hrt, _ = om.thermo(298.15)
    hf = RU * 298.15 * hrt / om.weights()
    assert np.all(np.abs(wg - ws) <= 1e-12 * np.abs(ws) + 1e-300)
    assert np.all(np.abs(qg - qs) <= 1e-12 * np.abs(ws * hf).sum(axis=1) + 1e-300)
    To, Yo, _, _, sto = om.integrate(T, p, Y, DT, RTOL, ATOL)
    assert np.all(sto == 0)
    wo, qo, _ = _source_terms(om, T, p, Y, To, Yo, DT)
    bar = rho0 * 1e-8 / DT
    assert np.all(np.abs(wg - wo) <= 1.01 * bar[:, None])
    assert np.all(np.abs(qg - qo) <= 1.01 * bar * np.abs(hf).sum())


def test_source_mode_failed_cells_are_nan(chem, mechs, dev):
    gm, _ = mechs["m9"]
    T, p, Y = uniform_cells(mech_text("m9"), 8, 26)
    T[3] = -5.0
    _, _, wg, qg, stats, st = chem.integrate_source(gm, _g(T, dev), _g(p, dev), _g(Y, dev), 1e-8, RTOL, ATOL,
                                                    return_status=True, allow_failed=True)
    st, wg, qg = st.cpu().numpy(), wg.cpu().numpy(), qg.cpu().numpy()
    assert st[3] == 4 and stats["failed"] == 1
    assert np.all(np.isnan(wg[3])) and np.isnan(qg[3])
    ok = [i for i in range(8) if i != 3]
    assert np.all(np.isfinite(wg[ok])) and np.all(np.isfinite(qg[ok]))


@pytest.mark.parametrize("name,hr,nfail", [("m9", 0.01, 32), ("m32", 0.9, 8)])
def test_step_size_floor_status_matches_oracle(chem, dev, oracle_lib, name, hr, nfail):
    """CHEM_CELL_HMIN: with a step-size floor of hmin_rel dt many cells need a
    step below it (m9 at 0.01: 113 of 256; m32, whose cells take one or two
    steps, at 0.9: 11).  The status of every cell matches the oracle's, except
    where the decision sits on the floor itself (the oracle's own status
    changes when the floor moves by 1e-6 of itself); a failed cell keeps its
    last accepted state, to the parity bar.  m32 runs in the wave-cooperative
    form."""
    gm = chem.Mechanism(mech_path(name))
    om = oracle_lib.Mechanism(mech_path(name))
    T, p, Y = uniform_cells(mech_text(name), 256, 81)
    Tg, Yg, stats, st, na, nr = chem.integrate(gm, _g(T, dev), _g(p, dev), _g(Y, dev), 1e-8, RTOL, ATOL,
                                               hmin_rel=hr, return_counts=True, allow_failed=True)
    st = st.cpu().numpy()
    To, Yo, nao, nro, sto = om.integrate(T, p, Y, 1e-8, RTOL, ATOL, hmin_rel=hr)
    edge = np.zeros(len(T), dtype=bool)
    for f in (1.0 - 1e-6, 1.0 + 1e-6):
        edge |= om.integrate(T, p, Y, 1e-8, RTOL, ATOL, hmin_rel=hr * f)[4] != sto
    assert (sto == 2).sum() >= nfail and (sto == 0).sum() >= 32
    assert np.all((st == sto) | edge), np.where((st != sto) & ~edge)[0]
    assert stats["failed"] == int((st != 0).sum())
    same = st == sto
    _assert_state_parity(Tg.cpu().numpy()[same], Yg.cpu().numpy()[same], To[same], Yo[same], f"{name} hmin")
