"""Pins of the oracle's electronic current (eq:last).

* U = 0: a single level with two Lorentzian leads is non-interacting, and the
  stationary particle current equals the Landauer integral with the Pade
  Fermi functions the exponents are built from (the HEOM closes exactly at
  tier 2 for U = 0, as the density of states does).
* Any model: in the stationary state the currents from all leads add up to
  zero (charge conservation), the current is real, and it vanishes at zero
  bias.
* A spinful U = 0 level carries twice the spinless current.
"""
import numpy as np
import pytest

from oracle import exponents as ox
from oracle import observables as ob
from oracle import solvers as osv
from oracle.liouvillian import OracleHEOM
from paper_2306_07522_amd import workloads as wl


def _stationary(cfg, n_max=None):
    recs = ox.exponent_records(cfg["baths"])
    om = OracleHEOM(cfg["H"], recs, cfg["m_max"], cfg["n_max"] if n_max is None else n_max)
    return om, recs, osv.steady_state(om.assemble(), om.d)


@pytest.mark.parametrize("eps,mus,n_exp,T", [(0.0, (1.0, -1.0), 3, 0.5), (0.4, (1.5, -0.5), 4, 1.0),
                                             (-0.7, (2.0, 0.5), 2, 0.25)])
def test_current_matches_landauer_at_u0(eps, mus, n_exp, T):
    cfg = wl.resonant_level(eps=eps, mus=mus, n_exp=n_exp, T=T, n_max=2)
    om, recs, x = _stationary(cfg)
    IL = ob.current(om, x, recs, [0])
    ref = ob.landauer_current(eps, 2.0, 10.0, mus, T, n_exp)
    assert abs(IL.imag) <= 1e-12
    assert abs(IL.real - ref) <= 1e-10 * abs(ref), (IL, ref)
    # the tier does not change it (U = 0 closes at tier 2)
    om3, recs3, x3 = _stationary(cfg, n_max=3)
    assert abs(ob.current(om3, x3, recs3, [0]) - IL) <= 1e-11


def test_spinful_level_carries_twice_the_current():
    cfg = wl.siam(eps=0.3, U=0.0, Gamma=2.0, W=10.0, T=0.5, mus=(1.0, -1.0), n_exp=3, n_max=2)
    om, recs, x = _stationary(cfg)
    IL = ob.current(om, x, recs, [0, 1])              # lead L: records (L, up), (L, down)
    ref = ob.landauer_current(0.3, 2.0, 10.0, (1.0, -1.0), 0.5, 3)
    assert abs(IL.real - 2.0 * ref) <= 1e-10 * abs(ref), (IL, ref)
    assert abs(ob.current(om, x, recs, [0]) - ob.current(om, x, recs, [1])) <= 1e-12


@pytest.mark.parametrize("mus", [(1.0, -1.0), (0.0, 0.0)])
def test_interacting_current_is_conserved_real_and_zero_at_zero_bias(mus):
    cfg = wl.siam(eps=-2.0, U=4.0, Gamma=1.0, W=10.0, T=0.5, mus=mus, n_exp=3, n_max=2)
    om, recs, x = _stationary(cfg)
    IL = ob.current(om, x, recs, [0, 1])
    IR = ob.current(om, x, recs, [2, 3])
    assert abs(IL + IR) <= 1e-12
    assert abs(IL.imag) <= 1e-12
    if mus[0] == mus[1]:
        assert abs(IL) <= 1e-12
    else:
        assert IL.real > 1e-4                         # electrons flow from the higher chemical potential


def test_landauer_reference_itself():
    """The Landauer integral against its wide-band limit (W -> infinity) in
    closed form: for equal leads of width g (total width 2g) the current is
    (g / 2) (n_L - n_R), with the occupation of a Lorentzian level at
    temperature T, n(mu) = 1/2 - Im psi(1/2 + (g + i (eps - mu)) / (2 pi T)) / pi
    (psi the digamma function); 19 Pade poles make f_Pade the Fermi
    function over the range that matters."""
    from scipy import special
    eps, g, mus, T = 0.2, 0.5, (1.0, -0.6), 0.1

    def n(mu):
        return 0.5 - special.digamma(0.5 + (g + 1j * (eps - mu)) / (2 * np.pi * T)).imag / np.pi

    exact = 0.5 * g * (n(mus[0]) - n(mus[1]))
    approx = ob.landauer_current(eps, g, 5000.0, mus, T, 20)
    assert abs(approx - exact) <= 2e-4 * abs(exact), (approx, exact)
