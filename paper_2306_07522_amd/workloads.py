"""Seeded synthetic inputs shared by the tests, the benchmark and smoke().

This module holds no HEOM arithmetic: it only builds the physical inputs of
the paper's problem statement (Fig. 1a: a system Hamiltonian, coupling
operators, spectral-density parameters, truncation tiers) for the five
workloads, plus seeded random vectors and random raw exponent lists.
Exponents, the hierarchy and everything downstream are computed separately
by the GPU library and by the oracle.

Fermionic operators use the Jordan-Wigner construction in the occupation
basis: basis state s (an integer) has mode k occupied when bit k of s is
set; d_k |s> = (-1)^{#occupied modes below k} |s - 2^k> when bit k is set.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# Operators
# ---------------------------------------------------------------------------
def jordan_wigner(n_modes: int):
    """Annihilation operators d_0..d_{n-1} on the 2^n occupation basis."""
    dim = 1 << n_modes
    ops = []
    for k in range(n_modes):
        d = np.zeros((dim, dim))
        for s in range(dim):
            if s >> k & 1:
                sign = (-1) ** bin(s & ((1 << k) - 1)).count("1")
                d[s ^ (1 << k), s] = sign
        ops.append(d)
    return ops


def boson_annihilation(n_photon: int):
    return np.diag(np.sqrt(np.arange(1, n_photon)), k=1)


def fermion_parity(n_modes: int):
    dim = 1 << n_modes
    return np.diag([(-1) ** bin(s).count("1") for s in range(dim)]).astype(float)


# ---------------------------------------------------------------------------
# Bath parameter records (physical parameters, not exponents)
# ---------------------------------------------------------------------------
def lorentz_lead(op, Gamma, W, mu, T, n_exp):
    return dict(kind="fermion", spectral="lorentz", op=np.asarray(op, dtype=np.complex128),
                Gamma=Gamma, W=W, mu=mu, T=T, n_exp=n_exp, method="pade")


def drude_lorentz_bath(op, lam, gamma, T, n_exp, method="matsubara"):
    return dict(kind="boson", spectral="drude_lorentz", op=np.asarray(op, dtype=np.complex128),
                lam=lam, gamma=gamma, T=T, n_exp=n_exp, method=method)


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------
def spin_boson():
    """d=2; H = 0.5 sz + 0.5 sx; V = sz; Drude-Lorentz lam=0.1, gamma=0.5,
    T=0.5 with the J pole and 2 Matsubara terms (3 exponents); tier 4;
    rho0 = |0><0|; RK4 dt = 0.01 over t in [0, 20]."""
    sz = np.array([[1, 0], [0, -1]], dtype=np.complex128)
    sx = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    H = 0.5 * sz + 0.5 * sx
    rho0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
    return dict(name="spin_boson", d=2, H=H, baths=[drude_lorentz_bath(sz, 0.1, 0.5, 0.5, 3)],
                m_max=4, n_max=0, rho0=rho0, dt=0.01, n_steps=2000)


def pure_dephasing():
    """Delta = 0 variant of the spin-boson model: H = 0.5 sz, V = sz,
    rho0 = |+><+| (closed-form coherence decay)."""
    sz = np.array([[1, 0], [0, -1]], dtype=np.complex128)
    rho0 = 0.5 * np.ones((2, 2), dtype=np.complex128)
    return dict(name="pure_dephasing", d=2, H=0.5 * sz, baths=[drude_lorentz_bath(sz, 0.1, 0.5, 0.5, 3)],
                rho0=rho0)


def siam(eps=-5.0, U=10.0, Gamma=2.0, W=10.0, T=0.5, mus=(1.0, -1.0), n_exp=5, n_max=3):
    """Single-impurity Anderson model, basis |0>,|up>,|dn>,|up dn> (JW modes
    0 = up, 1 = down); two Lorentzian leads with Pade exponents.  Bath order:
    for each lead, for each spin."""
    d_up, d_dn = jordan_wigner(2)
    nu, nd = d_up.T @ d_up, d_dn.T @ d_dn
    H = eps * (nu + nd) + U * nu @ nd
    baths = [lorentz_lead(op, Gamma, W, mu, T, n_exp) for mu in mus for op in (d_up, d_dn)]
    return dict(name="siam", d=4, H=H.astype(np.complex128), baths=baths, m_max=0, n_max=n_max,
                dops=[d_up, d_dn], parity_op=fermion_parity(2),
                omegas=np.linspace(-15.0, 15.0, 2000))


def resonant_level(eps=0.0, Gamma=2.0, W=10.0, T=0.5, mus=(1.0, -1.0), n_exp=3, n_max=2):
    """Spinless non-interacting level (U = 0) with two Lorentzian leads."""
    (d,) = jordan_wigner(1)
    H = eps * d.T @ d
    baths = [lorentz_lead(d, Gamma, W, mu, T, n_exp) for mu in mus]
    return dict(name="resonant_level", d=2, H=H.astype(np.complex128), baths=baths, m_max=0, n_max=n_max,
                dops=[d], eps=eps, Gamma=Gamma, W=W, mus=mus, parity_op=fermion_parity(1))


def charge_cavity(eps=-3.0, wc=1.0, g=0.5, n_photon=10, lam=0.01, gamma=0.1, T=0.1,
                  n_bexp=4, Gamma=0.01, W=10.0, mus=(3.0, -3.0), n_fexp=5, m_max=2, n_max=2):
    """Charge qubit in a cavity: H = eps d^dag d + wc a^dag a + g d^dag d (a + a^dag);
    dot (JW mode) x cavity (n_photon Fock states) -> d = 2 n_photon; cavity
    coupled to a Drude-Lorentz bath through V = a + a^dag (J pole + 3 Matsubara
    terms), dot to two Lorentzian leads (J pole + 4 Pade terms)."""
    (dq,) = jordan_wigner(1)
    a = boson_annihilation(n_photon)
    I2, Ic = np.eye(2), np.eye(n_photon)
    D = np.kron(dq, Ic)
    A = np.kron(I2, a)
    nD = D.T @ D
    H = eps * nD + wc * A.T @ A + g * nD @ (A + A.T)
    baths = [drude_lorentz_bath(A + A.T, lam, gamma, T, n_bexp)]
    baths += [lorentz_lead(D, Gamma, W, mu, T, n_fexp) for mu in mus]
    return dict(name="charge_cavity", d=2 * n_photon, H=H.astype(np.complex128), baths=baths, wc=wc,
                m_max=m_max, n_max=n_max, aop=A.astype(np.complex128), dops=[D],
                parity_op=np.kron(fermion_parity(1), Ic), omegas=2.0 * np.arange(1, 1025) / 1024,
                dt=0.01, t_final=200.0)


def two_orbital_anderson(eps=-4.0, U=8.0, t=0.5, Gamma=2.0, W=10.0, T=0.5, mus=(1.0, -1.0),
                         n_exp=3, n_max=4):
    """Two-orbital Anderson model: 2 orbitals x 2 spins = 4 JW modes (mode
    2*orb + spin), d = 16; intra-orbital U, same-spin inter-orbital hopping t;
    two leads each coupled to all four spin-orbitals (J pole + 2 Pade terms):
    2 x 4 x 2 x 3 = 48 fermionic exponents."""
    ops = jordan_wigner(4)
    n = [o.T @ o for o in ops]
    H = sum(eps * n[k] for k in range(4))
    for orb in range(2):
        H = H + U * n[2 * orb] @ n[2 * orb + 1]
    for s in range(2):
        h = ops[s].T @ ops[2 + s]
        H = H + t * (h + h.T)
    baths = [lorentz_lead(op, Gamma, W, mu, T, n_exp) for mu in mus for op in ops]
    return dict(name="two_orbital_anderson", d=16, H=H.astype(np.complex128), baths=baths, m_max=0,
                n_max=n_max, dops=ops, parity_op=fermion_parity(4),
                omegas=np.linspace(-15.0, 15.0, 4096))


def perturbed_two_orbital(seed: int, n_max=4, scale=0.1):
    """Seeded perturbation of the two-orbital model (each of eps, U, t, mu,
    Gamma multiplied by exp(scale Z))."""
    rng = np.random.default_rng(seed)
    z = np.exp(scale * rng.standard_normal(5))
    return two_orbital_anderson(eps=-4.0 * z[0], U=8.0 * z[1], t=0.5 * z[2], Gamma=2.0 * z[4],
                                mus=(1.0 * z[3], -1.0 * z[3]), n_max=n_max)


def _random_hermitian(rng, d):
    A = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    return (A + A.conj().T) / 2


def batch_instances(n_inst=512, seed=4242):
    """Seeded random instances alternating spin-boson / Anderson families.

    d ~ U{2,4,8,16}; tier ~ U{2..6}; exponent count k ~ U{3..12};
    lam = 0.1 e^{0.5 Z}, gamma = 0.5 e^{0.5 Z}, T = 0.5; H random Hermitian
    with spectral norm 1 (parity-even blocks for the Anderson family).
    Spin-boson: V = diag(linspace(1, -1, d)), Drude-Lorentz with k terms.
    Anderson: M = log2 d modes; c = min(M, 2) coupled modes; each coupled
    mode gets one Lorentzian lead with n_exp = max(1, k // (2c)) terms.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_inst):
        d = int(rng.choice([2, 4, 8, 16]))
        L = int(rng.integers(2, 7))
        k = int(rng.integers(3, 13))
        lam = 0.1 * np.exp(0.5 * rng.standard_normal())
        gam = 0.5 * np.exp(0.5 * rng.standard_normal())
        if i % 2 == 0:
            H = _random_hermitian(rng, d)
            H /= np.linalg.norm(H, 2)
            V = np.diag(np.linspace(1.0, -1.0, d)).astype(np.complex128)
            out.append(dict(family="spin_boson", d=d, H=H, m_max=L, n_max=0,
                            baths=[drude_lorentz_bath(V, lam, gam, 0.5, k)]))
        else:
            M = int(np.log2(d))
            ops = jordan_wigner(M)
            par = np.diag(fermion_parity(M))
            H = np.zeros((d, d), dtype=np.complex128)
            for sgn in (1.0, -1.0):
                idx = np.where(par == sgn)[0]
                blk = _random_hermitian(rng, len(idx))
                H[np.ix_(idx, idx)] = blk
            H /= np.linalg.norm(H, 2)
            c = min(M, 2)
            n_exp = max(1, k // (2 * c))
            baths = [lorentz_lead(ops[m], 2.0 * lam / 0.1, 10.0 * gam / 0.5, 0.0, 0.5, n_exp) for m in range(c)]
            out.append(dict(family="anderson", d=d, H=H, m_max=0, n_max=min(L, 2 * c * n_exp),
                            baths=baths, parity_op=fermion_parity(M)))
    return out


# ---------------------------------------------------------------------------
# Random raw exponent lists and vectors
# ---------------------------------------------------------------------------
def random_raw_baths(rng, d, n_bos_baths=1, n_bos_exp=2, n_ferm_baths=1, n_ferm_exp=2, dense_ops=True):
    """Random coupling operators and raw exponent lists (the paper's
    "directly providing a list of exponents" input form).  Fermionic
    coupling operators are random (not necessarily odd) dense matrices when
    dense_ops is set: the apply is linear in them, so parity tests of the
    apply need no physical structure."""
    baths = []
    for _ in range(n_bos_baths):
        V = _random_hermitian(rng, d)
        u_type = [("R", "I", "RI")[i % 3] for i in range(n_bos_exp)]
        xi = rng.standard_normal(n_bos_exp) + 1j * rng.standard_normal(n_bos_exp)
        chi = rng.uniform(0.2, 2.0, n_bos_exp) + 1j * rng.uniform(-1.0, 1.0, n_bos_exp)
        baths.append(dict(kind="boson", op=V, u_type=u_type, xi=xi, chi=chi))
    for _ in range(n_ferm_baths):
        if dense_ops:
            D = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
        else:
            D = jordan_wigner(int(np.log2(d)))[0].astype(np.complex128)
        c = lambda n: rng.standard_normal(n) + 1j * rng.standard_normal(n)
        g = lambda n: rng.uniform(0.2, 2.0, n) + 1j * rng.uniform(-1.0, 1.0, n)
        baths.append(dict(kind="fermion", op=D, eta_p=c(n_ferm_exp), gam_p=g(n_ferm_exp),
                          eta_m=c(n_ferm_exp), gam_m=g(n_ferm_exp)))
    return baths


def random_vector(rng, N, d, n_rhs=1):
    """Complex normal [N][d][d] (or [N][d][d][R]) vector."""
    shape = (N, d, d) if n_rhs == 1 else (N, d, d, n_rhs)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
