"""Host-side checks of the C-ABI library (CPU only, no device calls):
symbol exports, exponent helpers against the oracle, and the hierarchy
tables against the oracle's enumeration."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import exponents as ox
from paper_2306_07522_amd import workloads as wl
from tests.helpers import library_model, oracle_model, oracle_to_library_perm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _api():
    from paper_2306_07522_amd import api
    return api


def test_library_exports_every_declared_symbol():
    api = _api()
    lib = api.lib()
    hdr = open(os.path.join(ROOT, "include", "heom.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    names = set(re.findall(r"\b(heom_[a-z0-9_]+)\s*\(", hdr))
    assert len(names) >= 15
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_library_shares_torchs_hip_runtime():
    """Loading libheom before anything imports torch must still leave a single
    HIP runtime in the process (torch's), since torch's pointers and streams
    are passed straight through the ABI."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2306_07522_amd import _lib\n"
            "_lib.load()\n"
            "import torch, os\n"
            "print(_lib._hip_runtimes()); print(os.path.dirname(torch.__file__))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    runtimes, torch_dir = out.stdout.strip().splitlines()[-2:]
    runtimes = __import__("ast").literal_eval(runtimes)
    assert len(runtimes) == 1 and runtimes[0].startswith(torch_dir), runtimes


@pytest.mark.parametrize("kind", ["fermi", "bose"])
@pytest.mark.parametrize("n", [1, 2, 4, 6, 10])
def test_pade_params_match_oracle(kind, n):
    k, z = _api().pade_params(kind, n)
    ko, zo = ox.pade_params_rational(kind, n)
    assert np.allclose(z, zo, rtol=1e-12, atol=0)
    assert np.allclose(k, ko, rtol=1e-10, atol=0)


def test_exponent_helpers_match_oracle():
    api = _api()
    for method in ("pade", "matsubara"):
        e = api.exponents_lorentz(2.0, 10.0, 1.0, 0.5, 5, method)
        eo = ox.lorentz_fermion_exponents(2.0, 10.0, 1.0, 0.5, 5, method)
        for k in e:
            assert np.allclose(e[k], eo[k], rtol=1e-12, atol=1e-14), (method, k)
        xi, chi = api.exponents_drude_lorentz(0.1, 0.5, 0.5, 4, method)
        xo, co = ox.drude_lorentz_exponents(0.1, 0.5, 0.5, 4, method)
        assert np.allclose(xi, xo, rtol=1e-12, atol=1e-15)
        assert np.allclose(chi, co, rtol=1e-12, atol=0)


def test_argument_errors_are_reported():
    api = _api()
    from paper_2306_07522_amd._lib import HeomError
    with pytest.raises(HeomError):
        api.Hierarchy(np.array([[0, 1], [0, 0]]), [], 0, 0)           # not Hermitian
    cfg = wl.siam()
    bad = np.eye(4)                                                   # parity op that H violates? H is diagonal -> even
    with pytest.raises(HeomError):
        # a fermionic coupling that is parity-even violates the parity check
        api.Hierarchy(cfg["H"], [dict(cfg["baths"][0], op=np.diag([1.0, 0, 0, 0]))], 0, 1,
                      parity_op=cfg["parity_op"])
    with pytest.raises(HeomError):
        api.exponents_lorentz(1.0, 10.0, 0.0, -1.0, 3)                # negative temperature


def test_lindblad_argument_errors_are_reported():
    """heom_hierarchy_set_lindblad rejects parity-odd and non-finite jump
    operators, and a hierarchy with a Lindbladian cannot join a batch (all
    before any device work)."""
    api = _api()
    from paper_2306_07522_amd._lib import HeomError
    cfg = wl.siam(n_max=1, n_exp=2)
    h = api.Hierarchy(cfg["H"], cfg["baths"], 0, 1, parity_op=cfg["parity_op"])
    d_up = cfg["dops"][0]
    with pytest.raises(HeomError, match="parity-even"):
        h.set_lindblad([d_up])                      # odd: mixes the parity sectors
    bad = np.zeros((4, 4), complex)
    bad[0, 0] = np.nan
    with pytest.raises(HeomError, match="non-finite"):
        h.set_lindblad([bad])
    h.set_lindblad([0.3 * d_up.T @ d_up])           # dephasing of the up level: even
    other = api.Hierarchy(cfg["H"], cfg["baths"], 0, 1, parity_op=cfg["parity_op"])
    with pytest.raises(HeomError, match="Lindbladian"):
        api.Batch([h, other])
    h.set_lindblad([])                              # removed again


def test_current_argument_errors_are_reported():
    """heom_current rejects leads it cannot read before touching the device."""
    import ctypes as C
    api = _api()
    from paper_2306_07522_amd import _lib as L
    cfg = wl.charge_cavity(n_photon=2, n_bexp=2, n_fexp=2, m_max=1, n_max=1)
    h = api.Hierarchy(cfg["H"], cfg["baths"], cfg["m_max"], cfg["n_max"], parity_op=cfg["parity_op"])
    ho = api.Hierarchy(cfg["H"], cfg["baths"], cfg["m_max"], cfg["n_max"], parity=-1, parity_op=cfg["parity_op"])
    fake = C.c_void_p(256)     # never dereferenced: the arguments are checked first
    out = np.zeros(2)
    for hh, lead in ((h, [0]), (h, [3]), (h, [-1]), (h, [1, 1]), (ho, [1])):
        rec = np.asarray(lead, dtype=np.int32)
        st = api.lib().heom_current(hh.handle, fake, rec.size, rec.ctypes.data_as(L.i32p), out.ctypes.data_as(L.dp),
                                    None)
        assert st == 1 and b"current" in api.lib().heom_last_error(), (lead, st)


def test_solver_option_errors_are_reported():
    """Options the solvers reject before touching device memory: deflated
    restarting out of range or with the network, unknown preconditioners,
    and heom_precondition with a preconditioner that is not a fixed map."""
    import ctypes as C
    api = _api()
    from paper_2306_07522_amd import _lib as L
    cfg = wl.spin_boson()
    h = api.Hierarchy(cfg["H"], cfg["baths"], cfg["m_max"], 0)
    fake = C.c_void_p(256)     # never dereferenced: the options are checked first
    rep = L.heom_solver_report()
    for kw in (dict(deflate=32, restart=60), dict(deflate=29, restart=30), dict(deflate=-1),
               dict(deflate=4, restart=30, precond="nn"), dict(precond=5)):
        o = api.solver_opts(**kw)
        st = api.lib().heom_steady(h.handle, fake, C.byref(o), C.byref(rep), None, 0, None)
        assert st == 1, (kw, st)
        assert b"deflate" in api.lib().heom_last_error() or b"preconditioner" in api.lib().heom_last_error()
    o = api.solver_opts(deflate=4, restart=30)
    fd = C.cast(fake, L.dp)
    st = api.lib().heom_spectrum(h.handle, None, fake, 1, fd, fd, 1, fd, C.byref(o), C.byref(rep), None, 0, None)
    assert st != 0 and b"multi-shift" in api.lib().heom_last_error()   # thick restarts: multi-shift mode only
    o = api.solver_opts(deflate=29, restart=30, mode="shifted", precond="none")
    st = api.lib().heom_spectrum(h.handle, None, fake, 1, fd, fd, 1, fd, C.byref(o), C.byref(rep), None, 0, None)
    assert st == 1 and b"deflate" in api.lib().heom_last_error()
    for p in (L.HEOM_PREC_NONE, L.HEOM_PREC_NN, 7):
        st = api.lib().heom_precondition(h.handle, L.HEOM_FP64, p, fake, C.c_void_p(512), 1, None, 0, None)
        assert st == 1 and b"precondition" in api.lib().heom_last_error()
    with pytest.raises(TypeError):
        api.solver_opts(deflation=4)


@pytest.mark.parametrize("name", ["spin_boson", "siam", "charge_cavity_small", "random_mixed"])
def test_same_ado_set_and_decay_as_oracle(name):
    if name == "spin_boson":
        cfg = wl.spin_boson()
    elif name == "siam":
        cfg = wl.siam(n_max=2)
    elif name == "charge_cavity_small":
        cfg = wl.charge_cavity(n_photon=2, n_bexp=2, n_fexp=2, m_max=2, n_max=2)
    else:
        rng = np.random.default_rng(5)
        cfg = dict(H=np.diag(rng.standard_normal(3)).astype(complex),
                   baths=wl.random_raw_baths(rng, 3, n_bos_exp=3, n_ferm_exp=2), m_max=3, n_max=3)
    om = oracle_model(cfg)
    lm = library_model(cfg)
    assert lm.N == om.N
    perm = oracle_to_library_perm(om, lm)
    assert sorted(perm.tolist()) == list(range(lm.N))
    # decay c_a = sum n_k chi_k + sum gamma_q
    t = lm.tables()
    for k, (j, q) in enumerate(om.hier.ados):
        c = sum(om.bos[x]["chi"] for x in j) + sum(om.ferm[x]["gamma"] for x in q)
        assert abs(t["decay"][perm[k]] - c) < 1e-12 * max(1, abs(c))
    # neighbour sets: block columns of the oracle's block row = library edges + self
    for k in range(0, om.N, max(1, om.N // 50)):
        cols = {b for b, _, _ in om.block_terms(k)} - {k}
        a = perm[k]
        lib_cols = set(t["col"][t["row_ptr"][a]: t["row_ptr"][a + 1]].tolist())
        assert {int(perm[b]) for b in cols} == lib_cols


def test_counts_table3_and_workloads():
    from tests.conftest import golden
    g = golden("table3_ado_counts.json")
    api = _api()
    (d1,) = wl.jordan_wigner(1)
    zero = np.zeros(2)
    for n_max in (1, 2, 3, 4):
        # 56 fermionic exponents: 28 records of (nu=+1, nu=-1) pairs
        baths = [dict(kind="fermion", op=d1, eta_p=np.ones(1), gam_p=np.ones(1), eta_m=np.ones(1), gam_m=np.ones(1))
                 for _ in range(28)]
        h = api.Hierarchy(np.zeros((2, 2)), baths, 0, n_max)
        assert h.N == g["counts"][str(n_max)][-1]
    h = library_model(wl.two_orbital_anderson())
    assert h.N == 213053 and h.info.n_edges == 2 * 832512
    assert library_model(wl.spin_boson()).N == 35
    assert library_model(wl.charge_cavity()).N == 3165


def test_dictionary_lookup_and_sign():
    cfg = wl.siam(n_max=3)
    lm = library_model(cfg)
    occ, mask, lev = lm.ados()
    rng = np.random.default_rng(2)
    for a in rng.integers(0, lm.N, 40):
        ids = [k for k in range(64) if int(mask[a]) >> k & 1]
        ids_desc = sorted(ids, reverse=True)
        assert lm.index([], ids_desc) == (a, 1)
        p = list(rng.permutation(ids_desc))
        inv = sum(1 for i in range(len(p)) for j in range(i + 1, len(p)) if p[i] < p[j])
        assert lm.index([], p) == (a, (-1) ** inv)
    assert lm.index([], [0, 0])[0] == -1               # Pauli
    assert lm.index([], [0, 1, 2, 3])[0] == -1         # beyond the tier


# --------------------------------------------------------------------------- importance pruning (host build)
def _table3():
    import json, pathlib
    return json.loads((pathlib.Path(__file__).parent / "golden" / "table3_importance.json").read_text())


def _example1(n_max, th):
    t = _table3()["model"]
    d_up, d_dn = wl.jordan_wigner(2)
    baths = [wl.lorentz_lead(op, t["Gamma"], t["W"], 0.0, t["T"], t["n_terms"]) for _ in range(2)
             for op in (d_up, d_dn)]
    H = -5.0 * (d_up.T @ d_up + d_dn.T @ d_dn) + 10.0 * (d_up.T @ d_up) @ (d_dn.T @ d_dn)
    return _api().Hierarchy(H, baths, 0, n_max, importance_threshold=th)


@pytest.mark.parametrize("n_max", [2, 3, 4])
def test_library_importance_counts_table3(n_max):
    t = _table3()
    for th, want in zip(t["thresholds"], t["counts"][str(n_max)]):
        if th == 0.0 and n_max == 4:
            continue  # 396,607 ADOs: covered by the unpruned count tests
        h = _example1(n_max, th)
        assert h.N == want, (n_max, th, h.N, want)
        h.close()


@pytest.mark.parametrize("n_max", [5, 6])
def test_library_importance_counts_table3_deep(n_max):
    """Rows 5 and 6 at the thresholds whose hierarchies stay small (the
    enumeration still visits all 4.2 M / 36.7 M candidate sets)."""
    t = _table3()
    for th, want in list(zip(t["thresholds"], t["counts"][str(n_max)]))[:4]:
        h = _example1(n_max, th)
        assert h.N == want, (n_max, th, h.N, want)
        h.close()


def test_library_pruned_ados_match_oracle():
    from oracle.liouvillian import OracleHEOM
    cfg = wl.siam(n_max=3, n_exp=3)
    om = OracleHEOM(cfg["H"], ox.exponent_records(cfg["baths"]), 0, 3, importance_threshold=3e-3)
    api = _api()
    lm = api.Hierarchy(cfg["H"], cfg["baths"], 0, 3, importance_threshold=3e-3)
    full = api.Hierarchy(cfg["H"], cfg["baths"], 0, 3)
    assert 0 < lm.N == om.N < full.N
    # same ADO sets: map the oracle's sets (oracle numbering) to the library's masks
    occ, mask, _ = lm.ados()
    lib_sets = {int(m) for m in mask}
    # both sides number the fermionic exponents alike (per bath: h-major, nu = +1 then -1)
    ora_sets = set()
    for _, q in om.hier.ados:
        m = 0
        for k in q:
            m |= 1 << k
        ora_sets.add(m)
    assert lib_sets == ora_sets


def test_spectrum_chunk_rule():
    """rhs_chunk 0 (the default) lets the library choose the frequencies per
    spectrum solve: one for hierarchies of at least 2^18 elements per column,
    16 below; a positive rhs_chunk is used as given."""
    import ctypes as C
    api = _api()
    lib = api.lib()
    assert api.solver_opts().rhs_chunk == 0
    small = wl.spin_boson()
    hs = api.Hierarchy(small["H"], small["baths"], small["m_max"], small["n_max"])
    cav = wl.charge_cavity()
    hc = api.Hierarchy(cav["H"], cav["baths"], cav["m_max"], cav["n_max"], parity_op=cav["parity_op"])
    assert hc.N * hc.d * hc.d >= 1 << 18 > hs.N * hs.d * hs.d
    o = api.solver_opts()
    assert lib.heom_spectrum_chunk(hs.handle, C.byref(o)) == 16
    assert lib.heom_spectrum_chunk(hc.handle, C.byref(o)) == 1
    assert lib.heom_spectrum_chunk(hc.handle, None) == 1
    o8 = api.solver_opts(rhs_chunk=8)
    assert lib.heom_spectrum_chunk(hc.handle, C.byref(o8)) == 8
    assert lib.heom_spectrum_chunk(None, C.byref(o8)) == 0
    hs.close()
    hc.close()


def _fermionic_model(seed, d, n_baths, nf, n_max, dense=True):
    rng = np.random.default_rng(seed)
    H = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    baths = wl.random_raw_baths(rng, d, n_bos_baths=0, n_ferm_baths=n_baths, n_ferm_exp=nf, dense_ops=dense)
    return dict(H=H + H.conj().T, baths=baths, m_max=0, n_max=n_max)


@pytest.mark.parametrize("d,n_baths,nf,n_max,dense", [
    (8, 2, 2, 4, True), (16, 2, 2, 4, False), (8, 3, 2, 3, True), (8, 2, 2, 5, True), (8, 1, 4, 3, True),
])
def test_slab_plan_layout(d, n_baths, nf, n_max, dense):
    """The slab plan of purely fermionic hierarchies, built on the host: the
    build itself checks that every row's self term and every neighbour term
    is scheduled exactly once (it fails otherwise); here also that every
    top-tier ADO is read in launch A, that no job holds more parents than the
    register accumulators, and that both launches are spread over 8 XCDs."""
    cfg = _fermionic_model(300 + d + n_max, d, n_baths, nf, n_max, dense)
    lm = library_model(cfg)
    st = lm.slab_plan_stats()
    assert st is not None
    info = lm.info
    t = list(info.tier_offset)
    assert st["children"] == t[n_max + 1] - t[n_max] and st["parents"] == t[n_max] - t[n_max - 1]
    assert st["entries"][0] >= st["children"]
    assert max(st["max_vertices"]) <= 32
    assert st["jobs"][0] % 8 == 0 and st["jobs"][1] % 8 == 0


def test_slab_plan_two_orbital_tier4():
    """The two-orbital model at tier 4 (213,053 ADOs): launch A reads each
    top-tier ADO at most about 1.35 times (splitting a large slab over several
    workgroups duplicates the children they share), the XCD loads are within
    15 % of each other, and no plan exists for a model with a bosonic bath or
    with pruning."""
    cfg = wl.two_orbital_anderson()
    lm = library_model(cfg, parity_op=cfg["parity_op"])
    st = lm.slab_plan_stats()
    assert st["children"] == 194580 and st["parents"] == 17296
    assert st["children"] <= st["entries"][0] <= 1.35 * st["children"]
    assert st["entries"][1] <= 1.35 * st["children"]
    for l in range(2):
        c = st["xcd_cost"][l]
        assert max(c) <= 1.15 * min(c), (l, c)
    cav = library_model(wl.charge_cavity(n_photon=3, n_bexp=2, n_fexp=2, m_max=1, n_max=2))
    assert cav.slab_plan_stats() is None
