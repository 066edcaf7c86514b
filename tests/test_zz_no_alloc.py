"""heom_current_noalloc (the current readout with no device allocation,
its scratch in a library-owned device array) against heom_current, through
the C ABI: two calls in a row on different inputs, the second smaller
(fewer terms and a smaller d), each compared with heom_current on the same
stationary state to 1e-13 relative; then the first input again, so that a
stale term list or operator left in the shared array would show."""
import ctypes as C

import numpy as np
import pytest

from paper_2306_07522_amd import workloads as wl
from tests.helpers import library_model

pytestmark = pytest.mark.gpu


def _both(h, x, lead):
    from paper_2306_07522_amd import _lib as L, api
    lib = api.lib()
    rec = np.ascontiguousarray(np.asarray(lead, dtype=np.int32))
    a, b = np.zeros(2), np.zeros(2)
    for fn, out in ((lib.heom_current, a), (lib.heom_current_noalloc, b)):
        L.check(fn(h.handle, C.c_void_p(x.data_ptr()), int(rec.size), rec.ctypes.data_as(L.i32p),
                   out.ctypes.data_as(C.POINTER(C.c_double)), None))
    return a, b


def test_current_noalloc_matches_current():
    import torch
    from paper_2306_07522_amd import api
    assert torch.cuda.is_available()
    big = wl.siam(eps=-2.0, U=4.0, Gamma=1.0, n_exp=3, n_max=2)    # d = 4, two records per lead
    small = wl.resonant_level(eps=0.3, n_exp=2, n_max=2)             # d = 2, one record per lead
    cases = []
    for cfg, lead in ((big, [0, 1]), (small, [0]), (big, [2, 3])):
        h = library_model(cfg, parity_op=cfg["parity_op"])
        x, rep = api.steady_state(h, tol=1e-12, precond="none", restart=40, max_iter=4000)
        assert rep["status"] == 0
        cases.append((h, x, lead))
    for h, x, lead in cases:
        ref, got = _both(h, x, lead)
        assert np.all(np.isfinite(got)) and abs(ref[0]) > 1e-6, (ref, got)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max(), (ref, got)
    # unsupported size: d = 40 > 32 is refused before any device work
    from paper_2306_07522_amd._lib import HeomError
    rng = np.random.default_rng(0)
    H = rng.standard_normal((40, 40))
    D = np.zeros((40, 40), complex)
    D[0, 1] = 1.0
    b = dict(kind="fermion", op=D, eta_p=[0.1], gam_p=[1.0], eta_m=[0.1], gam_m=[1.0])
    hb = api.Hierarchy(H + H.T, [b], 0, 1)
    xb = torch.zeros((hb.N, 40, 40), dtype=torch.complex128, device="cuda")
    rec = np.zeros(1, dtype=np.int32)
    out = np.zeros(2)
    st = api.lib().heom_current_noalloc(hb.handle, C.c_void_p(xb.data_ptr()), 1, rec.ctypes.data_as(C.POINTER(C.c_int32)),
                                       out.ctypes.data_as(C.POINTER(C.c_double)), None)
    assert st == 6  # HEOM_ERR_UNSUPPORTED
