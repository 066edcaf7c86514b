"""Pins of the oracle's bath exponents (CPU only).

Each check ties the oracle to something other than itself: closed forms
derived by hand from the Methods' exponent formulas, the Pade N = 1 closed
forms, agreement of two independent Pade constructions, and the residue
evaluation against direct quadrature of eq:C_f / eq:C_b.
"""
import numpy as np
import pytest

from oracle import exponents as ox
from tests.conftest import golden


def test_pade_n1_closed_forms():
    g = golden("closed_forms.json")["pade_n1"]
    for kind in ("fermi", "bose"):
        k, z = ox.pade_params_rational(kind, 1)
        assert abs(k[0] - g[kind]["kappa"]) < 1e-14
        assert abs(z[0] - g[kind]["zeta"]) < 1e-14


@pytest.mark.parametrize("kind", ["fermi", "bose"])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_pade_two_constructions_agree(kind, n):
    k1, z1 = ox.pade_params_rational(kind, n)
    k2, z2 = ox.pade_params_tridiag(kind, n)
    assert np.allclose(z1, z2, rtol=1e-13, atol=0)
    assert np.allclose(k1, k2, rtol=1e-12, atol=0)


def test_pade_converges_to_fermi_and_bose():
    # the Pade series approaches the exact distributions as N grows
    x = np.array([0.1, 1.0, 3.0, 7.0])
    errs_f, errs_b = [], []
    for n in (2, 4, 8):
        k, z = ox.pade_params_rational("fermi", n)
        errs_f.append(np.max(np.abs(ox.fermi_pade(x, k, z) - 1 / (np.exp(x) + 1))))
        k, z = ox.pade_params_rational("bose", n)
        errs_b.append(np.max(np.abs(ox.bose_pade(x, k, z) - 1 / (np.exp(x) - 1))))
    assert errs_f[0] > errs_f[1] > errs_f[2] and errs_f[2] < 1e-9
    assert errs_b[0] > errs_b[1] > errs_b[2] and errs_b[2] < 1e-9
    # the lowest Pade poles approach the Matsubara frequencies
    k, z = ox.pade_params_rational("fermi", 8)
    assert abs(z[0] - np.pi) < 1e-12 and abs(z[1] - 3 * np.pi) < 1e-9


def test_drude_lorentz_c1_values():
    g = golden("closed_forms.json")["drude_lorentz_c1"]
    xi, chi = ox.drude_lorentz_exponents(0.1, 0.5, 0.5, 3, "matsubara")
    assert np.allclose(xi.real, g["xi_re"], atol=1e-15, rtol=1e-14)
    assert np.allclose(xi.imag, g["xi_im"], atol=1e-15)
    assert np.allclose(chi.real, g["chi"], atol=1e-15)


@pytest.mark.parametrize("method", ["pade", "matsubara"])
def test_fermion_exponents_match_quadrature(method):
    Gamma, W, mu, T, n = 2.0, 10.0, 1.0, 0.5, 5
    e = ox.lorentz_fermion_exponents(Gamma, W, mu, T, n, method)
    kappa, zeta = ox._params("fermi", n - 1, method)
    # eta is nu-independent and gamma^-nu = conj(gamma^nu) (residues)
    assert np.array_equal(e["eta_p"], e["eta_m"])
    assert np.allclose(e["gam_m"], np.conj(e["gam_p"]), atol=0)
    # tau = 0: C^nu(0) = (1/2pi) int J/2 = Gamma W / 4, real
    s0 = ox.exponent_sum(e["eta_p"], e["gam_p"], 0.0)
    assert abs(s0 - Gamma * W / 4) < 1e-12
    for tau in (0.05, 0.3, 1.7):
        for nu, eta, gam in ((+1, e["eta_p"], e["gam_p"]), (-1, e["eta_m"], e["gam_m"])):
            q = ox.fermion_correlation_quad(Gamma, W, mu, T, tau, nu, kappa, zeta)
            s = ox.exponent_sum(eta, gam, tau)
            assert abs(q - s) < 2e-9 * max(1.0, abs(s)), (tau, nu, q, s)


def test_boson_exponents_match_quadrature():
    # The J-pole term uses the exact cot (Methods, Drude-Lorentz), so the
    # exponent sum converges to the exact correlation function as terms are
    # added: Matsubara slowly, Pade fast.
    lam, gamma, T = 0.1, 0.5, 0.5
    for tau in (0.1, 0.7, 2.5):
        q = ox.boson_correlation_quad(lam, gamma, T, tau)
        xi, chi = ox.drude_lorentz_exponents(lam, gamma, T, 400, "matsubara")
        assert abs(ox.exponent_sum(xi, chi, tau) - q) < 2e-9, tau
        errs = []
        for n in (2, 4, 8):
            xi, chi = ox.drude_lorentz_exponents(lam, gamma, T, n, "pade")
            errs.append(abs(ox.exponent_sum(xi, chi, tau) - q))
        assert errs[-1] < 1e-4 and errs[-1] < errs[0], (tau, errs)
        # imaginary part is exactly -lam gamma e^{-gamma tau}
        assert abs(q.imag + lam * gamma * np.exp(-gamma * tau)) < 1e-10
