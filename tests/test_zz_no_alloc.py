"""chem_integrate_noalloc (the allocation-free entry point) against
chem_integrate in the persistent form, through the C ABI: bitwise equal
results and counters on two calls in a row (the second on a smaller field,
so the shared scratch holds the first call's leftovers), no change of the
device's free memory across the calls, the size limit refused, and a
wave-cooperative mechanism."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from workloads import mech_path, mech_text  # noqa: E402
from workloads.states import rde_field  # noqa: E402

DT, RTOL, ATOL = 5e-9, 1e-8, 1e-12


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def _g(a, dev, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=dev)


def _reference(chem, gm, T, p, Y):
    Te, Ye, _, st, na, nr = chem.integrate(gm, T.clone(), p, Y.clone(), DT, RTOL, ATOL, form=chem.FORM_PERSISTENT,
                                           return_counts=True)
    return [x.cpu().numpy() for x in (Te, Ye, st, na, nr)]


def _noalloc(lib, gm, T, p, Y, dev):
    n = T.shape[0]
    Tw, Yw = T.clone(), Y.clone()
    st, na, nr = (torch.full((n,), -7, dtype=torch.int32, device=dev) for _ in range(3))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    rc = lib.chem_integrate_noalloc(gm.h, n, C.c_void_p(Tw.data_ptr()), C.c_void_p(p.data_ptr()),
                                    C.c_void_p(Yw.data_ptr()), DT, RTOL, ATOL, None, C.c_void_p(st.data_ptr()),
                                    C.c_void_p(na.data_ptr()), C.c_void_p(nr.data_ptr()),
                                    C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, lib.chem_last_error().decode()
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0, "device memory changed across the call"
    return [x.cpu().numpy() for x in (Tw, Yw, st, na, nr)]


@pytest.mark.parametrize("name,sizes", [("m9", (48, 48, 13)), ("m32", (24, 24, 5))])
def test_noalloc_equals_persistent_on_two_calls(dev, name, sizes):
    import paper_2508_16105_amd as chem
    from paper_2508_16105_amd import _lib
    lib = _lib.lib()
    gm = chem.Mechanism(mech_path(name))
    T, p, Y, _ = rde_field(mech_text(name), sizes[0], sizes[1], 404)
    n2 = sizes[0] * sizes[2]                   # second call: a smaller field
    for k, cnt in enumerate((len(T), n2)):
        Tg, pg, Yg = _g(T[:cnt], dev), _g(p[:cnt], dev), _g(Y[:cnt], dev)
        ref = _reference(chem, gm, Tg, pg, Yg)
        got = _noalloc(lib, gm, Tg, pg, Yg, dev)
        for r, g, what in zip(ref, got, ("T", "Y", "status", "nacc", "nrej")):
            assert np.array_equal(r, g), (name, k, cnt, what)
        assert np.all(got[2] == 0)


def test_noalloc_counters_in_scratch_and_limits(dev):
    """Without caller counters the call still runs (counters in the scratch);
    the size limit, h0 and host pointers are refused before any launch."""
    import paper_2508_16105_amd as chem
    from paper_2508_16105_amd import _lib
    lib = _lib.lib()
    gm = chem.Mechanism(mech_path("m9"))
    T, p, Y, _ = rde_field(mech_text("m9"), 16, 16, 405)
    Tg, pg, Yg = _g(T, dev), _g(p, dev), _g(Y, dev)
    ref = _reference(chem, gm, Tg, pg, Yg)
    Tw, Yw = Tg.clone(), Yg.clone()
    chem.integrate_noalloc(gm, Tw, pg, Yw, DT, RTOL, ATOL)
    torch.cuda.synchronize()
    assert np.array_equal(Tw.cpu().numpy(), ref[0]) and np.array_equal(Yw.cpu().numpy(), ref[1])
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.chem_integrate_noalloc(gm.h, _lib.NOALLOC_MAX_CELLS + 1, C.c_void_p(Tw.data_ptr()),
                                    C.c_void_p(pg.data_ptr()), C.c_void_p(Yw.data_ptr()), DT, RTOL, ATOL, None,
                                    None, None, None, s)
    assert rc == -1 and b"CHEM_NOALLOC_MAX_CELLS" in lib.chem_last_error()
    h0 = torch.full_like(Tg, 1e-12)
    with pytest.raises(chem.ChemError):
        chem.integrate_noalloc(gm, Tw, pg, Yw, DT, RTOL, ATOL, h0=h0)
    Th = np.ascontiguousarray(T)
    rc = lib.chem_integrate_noalloc(gm.h, len(T), C.c_void_p(Th.ctypes.data), C.c_void_p(pg.data_ptr()),
                                    C.c_void_p(Yw.data_ptr()), DT, RTOL, ATOL, None, None, None, None, s)
    assert rc == -1
