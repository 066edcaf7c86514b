"""Bath correlation exponents -- oracle (test infrastructure only).

Follows the Methods sections "Fermion correlation function with Lorentzian
spectral density" and "Boson correlation function with Drude-Lorentz
spectral density" (eq:Lorentz, eq:Drude-Lorentz and the exponent tables
printed after them), plus eq:C_f_exp, eq:C_b_exp.

The paper defers the Pade parameters kappa_h, zeta_h to its reference
[Jie2011].  They are rebuilt here two independent ways:

* ``pade_params_rational``: the [N-1/N] Pade approximant, in y = x^2, of
  (f(x) - 1/2)/x for the Fermi function (or (n(x) - 1/x + 1/2)/x for the
  Bose function), solved in exact rationals from the Bernoulli-number
  Taylor series, then split into partial fractions at high precision;
* ``pade_params_tridiag``: poles from the eigenvalues of the symmetric
  tridiagonal matrix of the truncated continued fraction of tanh (coth),
  residues from a Vandermonde solve against the same Taylor coefficients.

The two must agree; the tests check that they do.

Readings (stated where the paper is silent or garbled):
* the second line printed as "eta_{alpha,h!=1}" is the decay rate
  gamma_{alpha,h!=1} = zeta_h T - nu i mu (residue calculation);
* eta_{alpha,1} is the same for both nu, with the Pade function evaluated
  at the complex point iW/T;
* the Matsubara decomposition is the Pade form with kappa = 1 and
  zeta_l = (2l-1) pi (Fermi) or 2 l pi (Bose).
"""
from __future__ import annotations

from fractions import Fraction

import mpmath
import numpy as np
import sympy

mpmath.mp.dps = 50


# ---------------------------------------------------------------------------
# Taylor coefficients of the smooth part of the distribution functions.
# ---------------------------------------------------------------------------
def _bernoulli(n: int) -> Fraction:
    b = sympy.bernoulli(n)
    return Fraction(int(b.p), int(b.q))


def _factorial(n: int) -> int:
    out = 1
    for k in range(2, n + 1):
        out *= k
    return out


def taylor_coeffs(kind: str, n_terms: int) -> list[Fraction]:
    """Coefficients c_k of g(y) = sum_k c_k y^k with y = x^2.

    Fermi: g = (1/2 - f(x))/x = tanh(x/2)/(2x),
           c_k = (2^(2k+2) - 1) B_(2k+2) / (2k+2)!
    Bose:  g = (n(x) - 1/x + 1/2)/x = coth(x/2)/(2x) - 1/x^2,
           c_k = B_(2k+2) / (2k+2)!
    """
    out = []
    for k in range(n_terms):
        m = 2 * k + 2
        b = _bernoulli(m)
        if kind == "fermi":
            out.append(Fraction((2 ** m - 1), 1) * b / _factorial(m))
        elif kind == "bose":
            out.append(b / _factorial(m))
        else:
            raise ValueError(kind)
    return out


# ---------------------------------------------------------------------------
# Construction 1: exact-rational [N-1/N] Pade approximant in y.
# ---------------------------------------------------------------------------
def pade_params_rational(kind: str, n_poles: int):
    """Return (kappa, zeta) arrays (float64, zeta ascending), N = n_poles.

    Q(y) g(y) - P(y) = O(y^(2N)), deg P = N-1, deg Q = N, Q(0) = 1; then
    P/Q = sum_h 2 kappa_h / (y + zeta_h^2).
    """
    n = n_poles
    c = taylor_coeffs(kind, 2 * n)
    cs = [sympy.Rational(x.numerator, x.denominator) for x in c]
    # unknowns q_1..q_N from the coefficients of y^N .. y^(2N-1)
    A = sympy.zeros(n, n)
    rhs = sympy.zeros(n, 1)
    for row, k in enumerate(range(n, 2 * n)):
        rhs[row] = -cs[k]
        for j in range(1, n + 1):
            A[row, j - 1] = cs[k - j]
    qsol = A.LUsolve(rhs)
    q = [sympy.Integer(1)] + [qsol[i] for i in range(n)]
    p = [sum(q[j] * cs[k - j] for j in range(0, k + 1)) for k in range(n)]
    # poles: roots of Q(y) (expected real negative: y = -zeta^2)
    qcoef_hi_first = [mpmath.mpf(sympy.Rational(q[j]).p) / sympy.Rational(q[j]).q for j in range(n, -1, -1)]
    roots = mpmath.polyroots(qcoef_hi_first, maxsteps=400, extraprec=400)
    kappas, zetas = [], []
    for y0 in roots:
        y0 = mpmath.re(y0)
        pv = sum(mpmath.mpf(sympy.Rational(p[k]).p) / sympy.Rational(p[k]).q * y0 ** k for k in range(n))
        dq = sum(j * mpmath.mpf(sympy.Rational(q[j]).p) / sympy.Rational(q[j]).q * y0 ** (j - 1)
                 for j in range(1, n + 1))
        res = pv / dq
        zetas.append(mpmath.sqrt(-y0))
        kappas.append(res / 2)
    order = sorted(range(n), key=lambda i: zetas[i])
    return (np.array([float(kappas[i]) for i in order]),
            np.array([float(zetas[i]) for i in order]))


# ---------------------------------------------------------------------------
# Construction 2: continued-fraction eigenvalues + Vandermonde residues.
# ---------------------------------------------------------------------------
def pade_params_tridiag(kind: str, n_poles: int):
    """Poles from the tridiagonal matrix of the continued fraction.

    tanh(t)/t = 1/(1 + t^2/(3 + t^2/(5 + ...))) has partial denominators
    b_m = 2m - 1; (coth(t) - 1/t)/t has b_m = 2m + 1.  The truncated fraction
    of depth 2N is the [N-1/N] approximant in t^2; its poles are
    t = +- i / lambda for the positive eigenvalues lambda of the 2N x 2N
    symmetric tridiagonal matrix with zero diagonal and off-diagonal
    1/sqrt(b_m b_(m+1)).  With t = x/2, zeta = 2/lambda.
    """
    n = n_poles
    m = 2 * n
    b = [(2 * k - 1) if kind == "fermi" else (2 * k + 1) for k in range(1, m + 2)]
    T = mpmath.zeros(m, m)
    for k in range(m - 1):
        v = 1 / mpmath.sqrt(mpmath.mpf(b[k]) * b[k + 1])
        T[k, k + 1] = v
        T[k + 1, k] = v
    ev = mpmath.eigsy(T)[0]
    lam = sorted([ev[i] for i in range(m) if ev[i] > 0], reverse=True)
    zetas = [2 / l for l in lam]
    c = taylor_coeffs(kind, n)
    # sum_h 2 kappa_h (-1)^k zeta_h^(-2(k+1)) = c_k, k = 0..N-1
    V = mpmath.matrix(n, n)
    r = mpmath.matrix(n, 1)
    for k in range(n):
        r[k] = mpmath.mpf(c[k].numerator) / c[k].denominator
        for h in range(n):
            V[k, h] = 2 * (-1) ** k * zetas[h] ** (-2 * (k + 1))
    kap = mpmath.lu_solve(V, r)
    return (np.array([float(kap[h]) for h in range(n)]),
            np.array([float(z) for z in zetas]))


def matsubara_params(kind: str, n_poles: int):
    """kappa = 1, zeta_l = (2l-1) pi (Fermi) or 2 l pi (Bose), l = 1..N."""
    l = np.arange(1, n_poles + 1, dtype=np.float64)
    zeta = (2 * l - 1) * np.pi if kind == "fermi" else 2 * l * np.pi
    return np.ones(n_poles), zeta


def fermi_pade(x, kappa, zeta):
    """n^Pade(x) = 1/2 - sum_h 2 kappa_h x / (x^2 + zeta_h^2) (complex x ok)."""
    x = np.asarray(x, dtype=np.complex128)
    s = np.zeros_like(x)
    for k, z in zip(kappa, zeta):
        s = s + 2 * k * x / (x * x + z * z)
    return 0.5 - s


def bose_pade(x, kappa, zeta):
    """n^Pade(x) = 1/x - 1/2 + sum_l 2 kappa_l x / (x^2 + zeta_l^2)."""
    x = np.asarray(x, dtype=np.complex128)
    s = np.zeros_like(x)
    for k, z in zip(kappa, zeta):
        s = s + 2 * k * x / (x * x + z * z)
    return 1.0 / x - 0.5 + s


# ---------------------------------------------------------------------------
# Exponent lists.
# ---------------------------------------------------------------------------
def _params(kind, n_poles, method):
    if n_poles == 0:
        return np.zeros(0), np.zeros(0)
    if method == "pade":
        return pade_params_rational(kind, n_poles)
    if method == "matsubara":
        return matsubara_params(kind, n_poles)
    raise ValueError(method)


def lorentz_fermion_exponents(Gamma, W, mu, T, n_exp, method="pade"):
    """Exponents of a Lorentzian fermionic bath (Methods, Lorentzian section).

    n_exp = N_alpha terms: h = 1 is the spectral-density pole, h = 2..N_alpha
    the poles of the Pade (or Matsubara) Fermi function.  Returns
    dict(eta_p, gam_p, eta_m, gam_m): complex arrays of length n_exp for
    nu = +1 and nu = -1.
      eta_1  = (Gamma W / 2) n^Pade(i W / T),    gamma^nu_1 = W - nu i mu
      eta_h  = -i kappa_h T Gamma W^2 / (W^2 - (zeta_h T)^2),
      gamma^nu_h = zeta_h T - nu i mu.
    """
    kappa, zeta = _params("fermi", n_exp - 1, method)
    eta1 = (Gamma * W / 2.0) * complex(fermi_pade(1j * W / T, kappa, zeta))
    etas = [eta1]
    gp = [W - 1j * mu]
    gm = [W + 1j * mu]
    for k, z in zip(kappa, zeta):
        etas.append(-1j * k * T * Gamma * W * W / (W * W - (z * T) ** 2))
        gp.append(z * T - 1j * mu)
        gm.append(z * T + 1j * mu)
    etas = np.array(etas, dtype=np.complex128)
    return dict(eta_p=etas.copy(), gam_p=np.array(gp), eta_m=etas.copy(), gam_m=np.array(gm))


def drude_lorentz_exponents(lam, gamma, T, n_exp, method="matsubara"):
    """Exponents of a Drude-Lorentz bosonic bath (Methods, Drude-Lorentz).

    J(w) = 4 lam gamma w / (w^2 + gamma^2) with C = (1/2pi) int (eq:C_b),
    i.e. Delta = lam, W = gamma.  n_exp = N_beta terms:
      xi_1 = lam gamma (cot(gamma / 2T) - i),  chi_1 = gamma
      xi_l = 4 kappa_l lam gamma T (zeta_l T) / ((zeta_l T)^2 - gamma^2),
      chi_l = zeta_l T.
    All chi are real, so each term is one combined real/imaginary ("RI")
    exponent.  Returns (xi complex array, chi complex array).
    """
    kappa, zeta = _params("bose", n_exp - 1, method)
    xi = [lam * gamma * (1.0 / np.tan(gamma / (2.0 * T)) - 1j)]
    chi = [gamma + 0j]
    for k, z in zip(kappa, zeta):
        xi.append(-2.0 * k * T * 2.0 * lam * gamma * (z * T) / (gamma * gamma - (z * T) ** 2) + 0j)
        chi.append(z * T + 0j)
    return np.array(xi, dtype=np.complex128), np.array(chi, dtype=np.complex128)


# ---------------------------------------------------------------------------
# Direct evaluation of the correlation integrals (eq:C_f, eq:C_b) with a
# given distribution function, for checking the exponent sums.
# ---------------------------------------------------------------------------
def fermion_correlation_quad(Gamma, W, mu, T, tau, nu, kappa, zeta):
    """(1/2pi) int J(w) [(1-nu)/2 + nu n(w)] e^{nu i w tau} dw by quadrature,
    with n = n^Pade((w - mu)/T).  Uses u = w - mu and the even/odd split of
    J and n - 1/2 so that Fourier-weighted QUADPACK rules apply."""
    from scipy.integrate import quad

    def odd(u):
        x = u / T
        return float(np.sum(2 * kappa * x / (x * x + zeta * zeta)))

    def Jt(u):
        return Gamma * W * W / (u * u + W * W)

    # n(w) = 1/2 - odd(u); (1-nu)/2 + nu n = 1/2 - nu odd(u)
    if tau == 0.0:
        even = quad(Jt, 0, np.inf, epsabs=1e-14, epsrel=1e-13, limit=400)[0]
        val = even
    else:
        cpart = quad(Jt, 0, np.inf, weight="cos", wvar=tau, epsabs=1e-14, limlst=200)[0]
        spart = quad(lambda u: Jt(u) * odd(u), 0, np.inf, weight="sin", wvar=tau, epsabs=1e-14, limlst=200)[0]
        # int J (1/2 - nu odd) e^{nu i u tau} du = cpart - 2 i spart (both nu)
        val = cpart - 2j * spart
    return np.exp(nu * 1j * mu * tau) * val / (2 * np.pi)


def boson_correlation_quad(lam, gamma, T, tau):
    """(1/2pi) int_0^inf J [n e^{i w tau} + (n+1) e^{-i w tau}] dw by
    quadrature with the exact Bose function, J = 4 lam gamma w/(w^2+gamma^2):
    = (1/2pi) int J [coth(w/2T) cos(w tau) - i sin(w tau)] dw."""
    from scipy.integrate import quad

    def jcoth(w):
        if w < 1e-8:
            return 4 * lam * gamma * 2 * T / (gamma * gamma)
        return 4 * lam * gamma * w / np.tanh(w / (2 * T)) / (w * w + gamma * gamma)

    def Jw(w):
        return 4 * lam * gamma * w / (w * w + gamma * gamma)

    re = quad(jcoth, 0, np.inf, weight="cos", wvar=tau, epsabs=1e-14, limlst=200)[0]
    im = -quad(Jw, 0, np.inf, weight="sin", wvar=tau, epsabs=1e-14, limlst=200)[0]
    return (re + 1j * im) / (2 * np.pi)


def exponent_sum(eta, gam, tau):
    """sum_k eta_k exp(-gamma_k tau) (eq:C_f_exp / eq:C_b_exp)."""
    return complex(np.sum(np.asarray(eta) * np.exp(-np.asarray(gam) * tau)))


def exponent_records(baths):
    """Physical bath descriptions -> raw exponent records (the form
    ``liouvillian.flatten_baths`` takes).  Records that already carry raw
    exponents pass through unchanged."""
    out = []
    for b in baths:
        if b["kind"] == "fermion" and b.get("spectral") == "lorentz":
            e = lorentz_fermion_exponents(b["Gamma"], b["W"], b["mu"], b["T"], b["n_exp"], b.get("method", "pade"))
            out.append(dict(kind="fermion", op=b["op"], **e))
        elif b["kind"] == "boson" and b.get("spectral") == "drude_lorentz":
            xi, chi = drude_lorentz_exponents(b["lam"], b["gamma"], b["T"], b["n_exp"], b.get("method", "matsubara"))
            out.append(dict(kind="boson", op=b["op"], u_type=["RI"] * len(xi), xi=xi, chi=chi))
        else:
            out.append(b)
    return out
