"""GPU parity of the electronic current readout (eq:last, heom_current).

* Readout alone: the library's current of the oracle's LU stationary state
  (mapped to the library's ADO order) against the oracle's current of the
  same vector, to 1e-12 relative; spinless and spinful leads, a mixed
  boson/fermion model (lead records after a bosonic bath record), a pruned
  hierarchy.
* End to end: the current of the GPU stationary state against the Landauer
  integral at U = 0 (1e-9) and charge conservation for an interacting
  impurity.
"""
import numpy as np
import pytest

from oracle import exponents as ox
from oracle import observables as ob
from oracle import solvers as osv
from oracle.liouvillian import OracleHEOM, to_blocks
from paper_2306_07522_amd import workloads as wl
from tests.helpers import oracle_to_library_perm

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _cases():
    return {
        "resonant_level": (wl.resonant_level(eps=0.3, n_exp=3, n_max=2), [[0], [1]], 0.0),
        "siam": (wl.siam(eps=-2.0, U=4.0, Gamma=1.0, n_exp=3, n_max=2), [[0, 1], [2, 3]], 0.0),
        "cavity": (wl.charge_cavity(n_photon=3, n_bexp=2, n_fexp=2, Gamma=0.5, lam=0.1), [[1], [2]], 0.0),
        "siam_pruned": (wl.siam(eps=-2.0, U=4.0, Gamma=1.0, n_exp=3, n_max=3), [[0, 1], [2, 3]], 1e-3),
    }


@pytest.mark.parametrize("name", ["resonant_level", "siam", "cavity", "siam_pruned"])
def test_current_readout_matches_oracle(name):
    torch = _torch()
    from paper_2306_07522_amd import api
    cfg, leads, th = _cases()[name]
    recs = ox.exponent_records(cfg["baths"])
    om = OracleHEOM(cfg["H"], recs, cfg["m_max"], cfg["n_max"], importance_threshold=th)
    lm = api.Hierarchy(cfg["H"], cfg["baths"], cfg["m_max"], cfg["n_max"], parity_op=cfg["parity_op"],
                       importance_threshold=th)
    perm = oracle_to_library_perm(om, lm)
    xs = osv.steady_state(om.assemble(), om.d)
    xl = np.empty((lm.N, lm.d, lm.d), dtype=complex)
    xl[perm] = to_blocks(xs, om.N, om.d)
    xt = torch.from_numpy(xl).cuda()
    for lead in leads:
        Io = ob.current(om, xs, recs, lead)
        Il = api.current(lm, xt, lead)
        assert abs(Il - Io) <= 1e-12 * max(abs(Io), 1e-3), (name, lead, Il, Io)


def test_current_of_gpu_steady_state_matches_landauer():
    torch = _torch()
    from paper_2306_07522_amd import api
    for eps, mus, T in [(0.0, (1.0, -1.0), 0.5), (0.4, (1.5, -0.5), 1.0)]:
        cfg = wl.resonant_level(eps=eps, mus=mus, n_exp=3, T=T, n_max=2)
        lm = api.Hierarchy(cfg["H"], cfg["baths"], 0, 2, parity_op=cfg["parity_op"])
        x, rep = api.steady_state(lm, tol=1e-13, restart=30, max_iter=2000)
        assert rep["status"] == 0
        ref = ob.landauer_current(eps, 2.0, 10.0, mus, T, 3)
        IL, IR = api.current(lm, x, [0]), api.current(lm, x, [1])
        assert abs(IL.real - ref) <= 1e-9 * abs(ref), (IL, ref)
        assert abs(IL + IR) <= 1e-11 and abs(IL.imag) <= 1e-11


def test_interacting_current_is_conserved_on_the_gpu():
    torch = _torch()
    from paper_2306_07522_amd import api
    cfg = wl.siam()                                        # tier 3, 40 exponents, U = 10
    lm = api.Hierarchy(cfg["H"], cfg["baths"], 0, cfg["n_max"], parity_op=cfg["parity_op"])
    x, rep = api.steady_state(lm, tol=1e-12, restart=40, max_iter=4000)
    assert rep["status"] == 0
    IL, IR = api.current(lm, x, [0, 1]), api.current(lm, x, [2, 3])
    assert IL.real > 0 and abs(IL + IR) <= 1e-9 * abs(IL), (IL, IR)


def test_bias_sweep_in_one_batch_matches_landauer():
    """A bias sweep (mu_L = -mu_R = Phi / 2) solved as one batch of stationary
    states: every current against the Landauer integral at U = 0, and the
    differential conductance dI/dPhi (central differences) against the same
    differences of the Landauer currents."""
    torch = _torch()
    from paper_2306_07522_amd import api
    phis = np.linspace(0.0, 3.0, 7)
    cfgs = [wl.resonant_level(eps=0.5, mus=(p / 2, -p / 2), n_exp=3, T=0.5, n_max=2) for p in phis]
    hs = [api.Hierarchy(c["H"], c["baths"], 0, 2, parity_op=c["parity_op"]) for c in cfgs]
    b = api.Batch(hs)
    x, reps = b.steady_state(tol=1e-12, restart=30, max_iter=3000, precond="block", fallback=1)
    assert all(r["status"] == 0 for r in reps), reps
    I = np.array([c.real for c in b.currents(x, [0])])
    ref = np.array([ob.landauer_current(0.5, 2.0, 10.0, (p / 2, -p / 2), 0.5, 3) for p in phis])
    assert np.abs(I - ref).max() <= 1e-9 * np.abs(ref).max(), (I, ref)
    G, Gref = np.gradient(I, phis), np.gradient(ref, phis)
    assert np.abs(G - Gref).max() <= 1e-8 * np.abs(Gref).max()
    assert abs(I[0]) <= 1e-11 and np.all(np.diff(I) > 0)
