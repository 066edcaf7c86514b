"""Pins of the oracle's time-dependent Hamiltonian, H_s(t) = H + sum_k
f_k(t) V_k, in RK4.

* Pure dephasing under H(t) = A cos(W t) sigma_z (no bath): the coherence
  is rho_01(t) = rho_01(0) exp(-2 i A sin(W t) / W), populations stay.
* A constant drive equals plain RK4 with H + c V, step for step.
* With a bath, the trace of rho_0 stays 1, and f = 0 is plain RK4.
"""
import numpy as np

from oracle import exponents as ox
from oracle import solvers as osv
from oracle.liouvillian import OracleHEOM, from_blocks, to_blocks
from paper_2306_07522_amd import workloads as wl


def test_driven_dephasing_closed_form():
    sz = np.diag([1.0, -1.0]).astype(complex)
    om = OracleHEOM(np.zeros((2, 2)), [], 0, 0)
    A, W, dt, n = 0.7, 1.9, 1e-3, 4000
    rho0 = np.array([[0.6, 0.3 + 0.2j], [0.3 - 0.2j, 0.4]])
    x = osv.rk4_driven(om.assemble(), [om.drive_superop(sz)], lambda t: [A * np.cos(W * t)],
                       from_blocks(rho0[None]), 0.0, dt, n)
    rho = to_blocks(x, 1, 2)[0]
    t = n * dt
    assert abs(rho[0, 1] - rho0[0, 1] * np.exp(-2j * A * np.sin(W * t) / W)) < 1e-10
    assert abs(rho[0, 0] - 0.6) < 1e-13


def test_constant_drive_equals_static_hamiltonian():
    cfg = wl.spin_boson()
    recs = ox.exponent_records(cfg["baths"])
    sx = np.array([[0, 1], [1, 0]], dtype=complex)
    c = 0.37
    om = OracleHEOM(cfg["H"], recs, cfg["m_max"], 0)
    om2 = OracleHEOM(cfg["H"] + c * sx, recs, cfg["m_max"], 0)
    x0 = np.zeros(om.N * 4, complex)
    x0[:4] = from_blocks(cfg["rho0"][None])
    xd = osv.rk4_driven(om.assemble(), [om.drive_superop(sx)], lambda t: [c], x0, 0.0, 0.01, 200)
    xs, _ = osv.rk4(om2.assemble(), x0, 0.01, 200)
    assert np.abs(xd - xs).max() < 1e-13


def test_driven_bath_keeps_trace_and_zero_drive_is_plain():
    cfg = wl.spin_boson()
    recs = ox.exponent_records(cfg["baths"])
    sx = np.array([[0, 1], [1, 0]], dtype=complex)
    om = OracleHEOM(cfg["H"], recs, cfg["m_max"], 0)
    x0 = np.zeros(om.N * 4, complex)
    x0[:4] = from_blocks(cfg["rho0"][None])
    M = om.assemble()
    xd = osv.rk4_driven(M, [om.drive_superop(sx)], lambda t: [0.5 * np.sin(1.3 * t)], x0, 0.2, 0.01, 300)
    rho = to_blocks(xd, om.N, 2)[0]
    assert abs(np.trace(rho) - 1.0) < 1e-12
    x0d = osv.rk4_driven(M, [om.drive_superop(sx)], lambda t: [0.0], x0, 0.0, 0.01, 100)
    xp, _ = osv.rk4(M, x0, 0.01, 100)
    assert np.abs(x0d - xp).max() < 1e-15
