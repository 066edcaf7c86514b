"""Environmental observables of the oracle (test infrastructure only: the
product path never imports this module).

current: the electronic current from one fermionic bath into the system,
eq:last ("Electronic current" in the Methods), in units e = hbar = 1:

    I_alpha = i sum_{nu, h, sigma} (-1)^{delta_{nu,-}} Tr[d_sigma^{nu-bar} rho^{(0,1,+)}_{|{alpha,nu,h,sigma}}]

over the first-level fermionic ADOs of the stationary state, each labelled by
one exponent (alpha, nu, h, sigma).  d^{nu-bar} with nu-bar = -nu: d for
nu = +1, d^dagger for nu = -1.

landauer_current: the non-interacting (U = 0) reference for one level with
Lorentzian leads J_alpha(w) = Gamma W^2 / ((w - mu_alpha)^2 + W^2): the
particle current from lead L, int dw/(2 pi) J_L J_R |G^R|^2 (f_L - f_R),
G^R = 1 / (w - eps - sum_alpha Sigma_alpha), Sigma_alpha = (Gamma W / 2) /
(w - mu_alpha + i W) (the same self-energy as the closed-form density of
states), with the Fermi functions in the Pade form the exponents use.
"""
import numpy as np
from scipy import integrate

from oracle import exponents as ox
from oracle.liouvillian import to_blocks


def _fermionic_exponent_ranges(records):
    """Index of the first fermionic exponent of every record (None for
    bosonic records), in the oracle's flattening order (per record, per h:
    nu = +1 then nu = -1)."""
    out, base = [], 0
    for rec in records:
        if rec["kind"] == "boson":
            out.append(None)
            continue
        out.append(base)
        base += 2 * len(rec["eta_p"])
    return out


def current(om, x_ss, records, lead):
    """eq:last for the lead made of the fermionic records `lead` (indices into
    `records`, the exponent records the oracle was built from).  x_ss: the
    oracle's stationary vector (column-stacked blocks).  Returns the complex
    value; it is real for a stationary state."""
    blocks = to_blocks(x_ss, om.N, om.d)
    first = _fermionic_exponent_ranges(records)
    total = 0j
    for r in lead:
        rec = records[r]
        if rec["kind"] == "boson":
            raise ValueError("a lead is made of fermionic baths")
        d = np.asarray(rec["op"], dtype=np.complex128)
        for h in range(len(rec["eta_p"])):
            for nu, slot in ((+1, 0), (-1, 1)):
                q = first[r] + 2 * h + slot
                idx, _ = om.hier.lookup((), (q,))
                if idx is None:
                    continue
                op = d if nu == +1 else d.conj().T      # d^{nu-bar}
                sign = 1.0 if nu == +1 else -1.0        # (-1)^{delta_{nu,-}}
                total += sign * np.trace(op @ blocks[idx])
    return 1j * total


def landauer_current(eps, Gamma, W, mus, T, n_exp):
    """Particle current from lead 0 of a single level with two Lorentzian
    leads (chemical potentials mus = (mu_L, mu_R)), with the Fermi function
    of n_exp - 1 Pade poles."""
    kappa, zeta = ox.pade_params_rational("fermi", n_exp - 1) if n_exp > 1 else (np.zeros(0), np.zeros(0))

    def f(w, mu):
        return float(np.real(ox.fermi_pade((w - mu) / T, kappa, zeta)))

    def J(w, mu):
        return Gamma * W * W / ((w - mu) ** 2 + W * W)

    def integrand(w):
        sigma = sum((Gamma * W / 2.0) / (w - mu + 1j * W) for mu in mus)
        g2 = 1.0 / abs(w - eps - sigma) ** 2
        return J(w, mus[0]) * J(w, mus[1]) * g2 * (f(w, mus[0]) - f(w, mus[1])) / (2.0 * np.pi)

    # a core around the level and the chemical potentials (the sharp
    # features), then the band, then the tails
    pts = sorted({eps, *mus})
    c = 40.0 * max(T, Gamma) + 1.0
    a, b = min(pts) - c, max(pts) + c
    lo, hi = min(a, min(pts) - 50.0 * (W + T)), max(b, max(pts) + 50.0 * (W + T))
    total = 0.0
    for x0, x1, p in ((a, b, pts), (lo, a, None), (b, hi, None)):
        if x1 > x0:
            total += integrate.quad(integrand, x0, x1, points=p, limit=400, epsabs=1e-15, epsrel=1e-12)[0]
    total += integrate.quad(integrand, -np.inf, lo, limit=200, epsabs=1e-15)[0]
    total += integrate.quad(integrand, hi, np.inf, limit=200, epsabs=1e-15)[0]
    return total
