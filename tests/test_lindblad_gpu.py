"""GPU parity of the Lindbladian add-on (eq:Lindbladian) against the oracle.

* Apply: FP64 within 1e-12 and FP32 within 1e-5 (relative) of the oracle's
  HEOMLS with the same jump operators, on a spin-boson model, a mixed
  cavity, the Anderson impurity of both parities and the two-orbital model
  (wave kernel), with several right-hand sides and per-column shifts.
* RK4 (the stage input x + kc k is fused into the Lindblad pass as in the
  apply) against the oracle's RK4 within 1e-12.
* Stationary states against the oracle's LU, and the thermal state of a
  damped oscillator in closed form.
"""
import numpy as np
import pytest

from oracle import exponents as ox
from oracle import solvers as osv
from oracle.liouvillian import OracleHEOM, from_blocks, to_blocks
from paper_2306_07522_amd import workloads as wl
from tests.helpers import oracle_to_library_perm, rel_err

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _models():
    sm = np.array([[0, 1], [0, 0]], dtype=complex)
    sz = np.diag([1.0, -1.0]).astype(complex)
    sb = wl.spin_boson()
    cav = wl.charge_cavity(n_photon=3, n_bexp=2, n_fexp=2, m_max=2, n_max=1, Gamma=0.5, lam=0.1)
    a = cav["aop"]
    siam = wl.siam(n_max=2, n_exp=2)
    nu, nd = siam["dops"][0].T @ siam["dops"][0], siam["dops"][1].T @ siam["dops"][1]
    two = wl.two_orbital_anderson(n_max=2)
    n0 = two["dops"][0].T @ two["dops"][0]
    return {
        "spin_boson": (sb, [0.3 * sm, 0.2 * sz]),
        "cavity": (cav, [np.sqrt(0.05 * 1.5) * a, np.sqrt(0.05 * 0.5) * a.conj().T]),
        "siam": (siam, [0.4 * nu, 0.3 * nd]),
        "two_orbital": (two, [0.2 * n0]),
    }


def _pair(name, parity=+1):
    from paper_2306_07522_amd import api
    cfg, ops = _models()[name]
    om = OracleHEOM(cfg["H"], ox.exponent_records(cfg["baths"]), cfg["m_max"], cfg["n_max"], parity=parity,
                    lindblad=ops)
    lm = api.Hierarchy(cfg["H"], cfg["baths"], cfg["m_max"], cfg["n_max"], parity=parity,
                       parity_op=cfg.get("parity_op"), lindblad=ops)
    return cfg, om, lm, oracle_to_library_perm(om, lm)


@pytest.mark.parametrize("name,parity", [("spin_boson", 1), ("cavity", 1), ("cavity", -1), ("siam", 1),
                                         ("siam", -1), ("two_orbital", 1)])
def test_apply_with_lindblad_matches_oracle(name, parity):
    torch = _torch()
    cfg, om, lm, perm = _pair(name, parity)
    rng = np.random.default_rng(1)
    R = 3
    shifts = np.array([0.0, 0.4j, -0.2 + 1.1j])
    xo = rng.standard_normal((om.N, om.d, om.d, R)) + 1j * rng.standard_normal((om.N, om.d, om.d, R))
    xl = np.empty_like(xo)
    xl[perm] = xo
    yo = np.stack([to_blocks(om.assemble(shift=shifts[r]) @ from_blocks(xo[..., r]), om.N, om.d)
                   for r in range(R)], axis=-1)
    sh = torch.from_numpy(shifts).cuda()
    y = lm.apply(torch.from_numpy(xl).cuda(), shift=sh, n_rhs=R).cpu().numpy()
    assert rel_err(y[perm], yo) <= 1e-12
    x32 = xl.astype(np.complex64)
    xo32 = x32.astype(np.complex128)[perm]
    yo32 = np.stack([to_blocks(om.assemble(shift=shifts[r]) @ from_blocks(xo32[..., r]), om.N, om.d)
                     for r in range(R)], axis=-1)
    y32 = lm.apply(torch.from_numpy(x32).cuda(), shift=sh.to(torch.complex64), n_rhs=R).cpu().numpy()
    assert rel_err(y32[perm].astype(np.complex128), yo32) <= 1e-5
    # one right-hand side through the single-RHS kernels too
    y1 = lm.apply(torch.from_numpy(np.ascontiguousarray(xl[..., 0])).cuda()).cpu().numpy()
    yo1 = to_blocks(om.assemble() @ from_blocks(xo[..., 0]), om.N, om.d)
    assert rel_err(y1[perm], yo1) <= 1e-12


def test_rk4_with_lindblad_matches_oracle():
    torch = _torch()
    from paper_2306_07522_amd import api
    cfg, om, lm, perm = _pair("spin_boson")
    x0o = np.zeros((om.N, om.d, om.d), complex)
    x0o[0] = cfg["rho0"]
    x0 = np.zeros_like(x0o)
    x0[perm] = x0o
    xo, _ = osv.rk4(om.assemble(), from_blocks(x0o), 0.01, 300)
    x = torch.from_numpy(x0).cuda()
    api.propagate(lm, x, 0.01, 300)
    assert rel_err(x.cpu().numpy()[perm], to_blocks(xo, om.N, om.d)) <= 1e-12
    rho = x.cpu().numpy()[0]
    assert abs(np.trace(rho) - 1.0) <= 1e-12


@pytest.mark.parametrize("name,precond", [("cavity", "block"), ("spin_boson", "none"), ("siam", "jacobi")])
def test_steady_with_lindblad_matches_oracle(name, precond):
    torch = _torch()
    from paper_2306_07522_amd import api
    cfg, om, lm, perm = _pair(name)
    xs = to_blocks(osv.steady_state(om.assemble(), om.d), om.N, om.d)
    x, rep = api.steady_state(lm, tol=1e-12, precond=precond, restart=40, max_iter=4000)
    assert rep["status"] == 0, rep
    assert rel_err(x.cpu().numpy()[perm], xs) <= 1e-9


def test_thermal_oscillator_through_the_library():
    torch = _torch()
    from paper_2306_07522_amd import api
    n_f, kappa, nbar = 9, 0.05, 0.7
    a = np.diag(np.sqrt(np.arange(1, n_f)), 1).astype(complex)
    H = a.conj().T @ a
    h = api.Hierarchy(H, [], 0, 0, lindblad=[np.sqrt(kappa * (nbar + 1)) * a, np.sqrt(kappa * nbar) * a.conj().T])
    x, rep = api.steady_state(h, tol=1e-13, precond="none", restart=30, max_iter=2000)
    p = (nbar / (nbar + 1)) ** np.arange(n_f)
    p /= p.sum()
    assert np.abs(x.cpu().numpy()[0] - np.diag(p)).max() <= 1e-11


@pytest.mark.parametrize("mode", ["fp64", "shifted"])
def test_psd_of_damped_oscillator_closed_form(mode):
    """The library's power spectrum of the thermally damped oscillator
    against S(w) = (n / pi) (kappa/2) / ((kappa/2)^2 + (w - w_c)^2), a
    Lorentzian at +w_c (quantum regression), on an asymmetric grid: per
    frequency (FP64 GMRES) and from one Krylov space (multi-shift)."""
    _torch()
    from paper_2306_07522_amd import api
    n_f, wc, kappa, nbar = 14, 1.0, 0.2, 0.05
    a = np.diag(np.sqrt(np.arange(1, n_f)), 1).astype(complex)
    h = api.Hierarchy(wc * a.conj().T @ a, [], 0, 0,
                      lindblad=[np.sqrt(kappa * (nbar + 1)) * a, np.sqrt(kappa * nbar) * a.conj().T])
    x, rep = api.steady_state(h, tol=1e-13, precond="none", restart=60, max_iter=4000)
    grid = np.linspace(0.2, 2.5, 47)
    S, rep = api.spectrum(h, None, x, a, grid, kind="psd", tol=1e-12, mode=mode, precond="none", restart=60,
                          max_iter=20000)
    ref = nbar / np.pi * (kappa / 2) / ((kappa / 2) ** 2 + (grid - wc) ** 2)
    assert np.abs(S - ref).max() <= 1e-8 * ref.max(), (mode, np.abs(S - ref).max())
