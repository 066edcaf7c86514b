// Host-side setup: bath exponents, ADO enumeration, neighbour tables and the
// hierarchy dictionary.  Follows eq:HEOM and the superoperators defined after
// it; the exponent formulas follow the Methods sections on the Lorentzian
// fermionic and Drude-Lorentz bosonic correlation functions.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace heom {

// ============================================================== exponents
// Eigenvalues of a real symmetric matrix by cyclic Jacobi rotations.
static std::vector<double> sym_eigenvalues(int n, std::vector<double> a) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += a[p * n + q] * a[p * n + q];
    if (off < 1e-300) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = a[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double app = a[p * n + p], aqq = a[q * n + q];
        double theta = (aqq - app) / (2 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1));
        double c = 1 / std::sqrt(t * t + 1), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - s * akq;
          a[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - s * aqk;
          a[q * n + k] = s * apk + c * aqk;
        }
      }
  }
  std::vector<double> ev(n);
  for (int i = 0; i < n; ++i) ev[i] = a[i * n + i];
  return ev;
}

// [N-1/N] Pade parameters from the continued fraction of tanh (Fermi) or
// coth - 1/t (Bose): partial denominators b_k = 2k-1 (Fermi) / 2k+1 (Bose),
// depth 2N.  Poles from the eigenvalues of the Jacobi matrix of the fraction,
// residues from its numerator / denominator three-term recurrences.
static void pade_cf(int fermi, int n, double *kappa, double *zeta) {
  int m = 2 * n;
  std::vector<double> b(m + 1);
  for (int k = 1; k <= m; ++k) b[k] = fermi ? (2.0 * k - 1) : (2.0 * k + 1);
  std::vector<double> J(m * m, 0.0);
  for (int k = 0; k + 1 < m; ++k) J[k * m + k + 1] = J[(k + 1) * m + k] = 1.0 / std::sqrt(b[k + 1] * b[k + 2]);
  std::vector<double> ev = sym_eigenvalues(m, J);
  std::vector<double> lam;
  for (double v : ev)
    if (v > 0) lam.push_back(v);
  std::sort(lam.begin(), lam.end(), std::greater<double>());
  for (int h = 0; h < n; ++h) {
    double l = lam[h];
    double y = -1.0 / (l * l);  // pole in t^2
    // A_k, B_k of  1/(b_1 + y/(b_2 + y/(...)))  and dB_k/dy
    double Am1 = 1, A0 = 0, Bm1 = 0, B0 = 1, dBm1 = 0, dB0 = 0;
    for (int k = 1; k <= m; ++k) {
      double ak = (k == 1) ? 1.0 : y, dak = (k == 1) ? 0.0 : 1.0;
      double A1 = b[k] * A0 + ak * Am1;
      double B1 = b[k] * B0 + ak * Bm1;
      double dB1 = b[k] * dB0 + ak * dBm1 + dak * Bm1;
      Am1 = A0; A0 = A1; Bm1 = B0; B0 = B1; dBm1 = dB0; dB0 = dB1;
    }
    // g(x^2) = (1/4) A(x^2/4)/B(x^2/4): residue in x^2 is A/B' -> 2 kappa
    kappa[h] = 0.5 * A0 / dB0;
    zeta[h] = 2.0 / l;
  }
  // ascending zeta
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int p, int q) { return zeta[p] < zeta[q]; });
  std::vector<double> k2(n), z2(n);
  for (int i = 0; i < n; ++i) { k2[i] = kappa[idx[i]]; z2[i] = zeta[idx[i]]; }
  std::copy(k2.begin(), k2.end(), kappa);
  std::copy(z2.begin(), z2.end(), zeta);
}

static heom_status dist_params(int fermi, int method, int n, std::vector<double> &k, std::vector<double> &z) {
  k.assign(n, 0.0);
  z.assign(n, 0.0);
  if (n == 0) return HEOM_OK;
  if (method == HEOM_MATSUBARA) {
    for (int l = 1; l <= n; ++l) {
      k[l - 1] = 1.0;
      z[l - 1] = fermi ? (2.0 * l - 1) * M_PI : 2.0 * l * M_PI;
    }
    return HEOM_OK;
  }
  if (method != HEOM_PADE) return fail(HEOM_ERR_ARG, "unknown decomposition method");
  pade_cf(fermi, n, k.data(), z.data());
  return HEOM_OK;
}

}  // namespace heom

using namespace heom;

static heom_status heom_pade_params_body(int32_t kind, int32_t method, int32_t n, double *kappa, double *zeta) {
  if (n < 0 || n > 64 || (n > 0 && (!kappa || !zeta))) return fail(HEOM_ERR_ARG, "pade_params: bad n or pointers");
  if (kind != HEOM_FERMION && kind != HEOM_BOSON) return fail(HEOM_ERR_ARG, "pade_params: bad kind");
  std::vector<double> k, z;
  HEOM_TRY(dist_params(kind == HEOM_FERMION, method, n, k, z));
  for (int i = 0; i < n; ++i) { kappa[i] = k[i]; zeta[i] = z[i]; }
  return HEOM_OK;
}

extern "C" heom_status heom_pade_params(int32_t kind, int32_t method, int32_t n, double *kappa, double *zeta) {
  return guarded([&] { return heom_pade_params_body(kind, method, n, kappa, zeta); });
}

static heom_status heom_exponents_lorentz_body(double Gamma, double W, double mu, double T, int32_t n_exp,
                                              int32_t method, double *eta_p, double *gam_p, double *eta_m,
                                              double *gam_m) {
  if (n_exp < 1 || n_exp > 65 || T <= 0 || W <= 0 || !eta_p || !gam_p || !eta_m || !gam_m)
    return fail(HEOM_ERR_ARG, "exponents_lorentz: bad arguments");
  std::vector<double> k, z;
  HEOM_TRY(dist_params(1, method, n_exp - 1, k, z));
  // Pade Fermi function at the complex point i W / T
  cd x(0.0, W / T), f(0.5, 0.0);
  for (int h = 0; h < n_exp - 1; ++h) f -= 2.0 * k[h] * x / (x * x + z[h] * z[h]);
  std::vector<cd> eta(n_exp), gp(n_exp), gm(n_exp);
  eta[0] = 0.5 * Gamma * W * f;
  gp[0] = cd(W, -mu);
  gm[0] = cd(W, mu);
  for (int h = 1; h < n_exp; ++h) {
    double zt = z[h - 1] * T;
    if (std::fabs(W * W - zt * zt) < 1e-12 * W * W) return fail(HEOM_ERR_ARG, "exponents_lorentz: pole collision W = zeta T");
    eta[h] = cd(0.0, -k[h - 1] * T * Gamma * W * W / (W * W - zt * zt));
    gp[h] = cd(zt, -mu);
    gm[h] = cd(zt, mu);
  }
  for (int h = 0; h < n_exp; ++h) {
    eta_p[2 * h] = eta_m[2 * h] = eta[h].real();
    eta_p[2 * h + 1] = eta_m[2 * h + 1] = eta[h].imag();
    gam_p[2 * h] = gp[h].real(); gam_p[2 * h + 1] = gp[h].imag();
    gam_m[2 * h] = gm[h].real(); gam_m[2 * h + 1] = gm[h].imag();
  }
  return HEOM_OK;
}

extern "C" heom_status heom_exponents_lorentz(double Gamma, double W, double mu, double T, int32_t n_exp,
                                              int32_t method, double *eta_p, double *gam_p, double *eta_m,
                                              double *gam_m) {
  return guarded([&] { return heom_exponents_lorentz_body(Gamma, W, mu, T, n_exp, method, eta_p, gam_p, eta_m, gam_m); });
}

static heom_status heom_exponents_drude_lorentz_body(double lam, double gamma, double T, int32_t n_exp,
                                                    int32_t method, double *xi, double *chi) {
  if (n_exp < 1 || n_exp > 65 || T <= 0 || gamma <= 0 || !xi || !chi)
    return fail(HEOM_ERR_ARG, "exponents_drude_lorentz: bad arguments");
  std::vector<double> k, z;
  HEOM_TRY(dist_params(0, method, n_exp - 1, k, z));
  xi[0] = lam * gamma / std::tan(gamma / (2 * T));
  xi[1] = -lam * gamma;
  chi[0] = gamma;
  chi[1] = 0.0;
  for (int l = 1; l < n_exp; ++l) {
    double zt = z[l - 1] * T;
    if (std::fabs(zt * zt - gamma * gamma) < 1e-12 * gamma * gamma)
      return fail(HEOM_ERR_ARG, "exponents_drude_lorentz: pole collision gamma = zeta T");
    xi[2 * l] = 4.0 * k[l - 1] * lam * gamma * T * zt / (zt * zt - gamma * gamma);
    xi[2 * l + 1] = 0.0;
    chi[2 * l] = zt;
    chi[2 * l + 1] = 0.0;
  }
  return HEOM_OK;
}

extern "C" heom_status heom_exponents_drude_lorentz(double lam, double gamma, double T, int32_t n_exp,
                                                    int32_t method, double *xi, double *chi) {
  return guarded([&] { return heom_exponents_drude_lorentz_body(lam, gamma, T, n_exp, method, xi, chi); });
}

namespace heom {

// ============================================================== hierarchy
int64_t lookup_ado(const Hier &h, uint64_t fmask, uint64_t bcode) {
  // h.keys is sorted; h.key_index maps a sorted position to the ADO index
  auto key = std::make_pair(fmask, bcode);
  auto it = std::lower_bound(h.keys.begin(), h.keys.end(), key);
  if (it == h.keys.end() || *it != key) return -1;
  return h.key_index[it - h.keys.begin()];
}

static bool is_hermitian(const std::vector<cd> &A, int d) {
  double nrm = 0, dev = 0;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      nrm = std::max(nrm, std::abs(A[i * d + j]));
      dev = std::max(dev, std::abs(A[i * d + j] - std::conj(A[j * d + i])));
    }
  return dev <= 1e-12 * std::max(nrm, 1e-300) || nrm == 0;
}

static std::vector<cd> matmul(const std::vector<cd> &A, const std::vector<cd> &B, int d) {
  std::vector<cd> C(d * d, 0.0);
  for (int i = 0; i < d; ++i)
    for (int k = 0; k < d; ++k) {
      cd a = A[i * d + k];
      if (a == 0.0) continue;
      for (int j = 0; j < d; ++j) C[i * d + j] += a * B[k * d + j];
    }
  return C;
}

static double maxabs(const std::vector<cd> &A) {
  double m = 0;
  for (auto v : A) m = std::max(m, std::abs(v));
  return m;
}

static std::vector<cd> read_mat(const double *p, int d) {
  std::vector<cd> A(d * d);
  for (int i = 0; i < d * d; ++i) A[i] = cd(p[2 * i], p[2 * i + 1]);
  return A;
}

static std::vector<cd> dagger(const std::vector<cd> &A, int d) {
  std::vector<cd> B(d * d);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) B[j * d + i] = std::conj(A[i * d + j]);
  return B;
}

// next combination of `n` ascending indices out of K (lexicographic)
static bool next_combination(std::vector<int> &c, int K) {
  int n = (int)c.size();
  for (int i = n - 1; i >= 0; --i) {
    if (c[i] < K - n + i) {
      ++c[i];
      for (int j = i + 1; j < n; ++j) c[j] = c[j - 1] + 1;
      return true;
    }
  }
  return false;
}

// next multiset (non-decreasing) of size m over K values
static bool next_multiset(std::vector<int> &c, int K) {
  int m = (int)c.size();
  for (int i = m - 1; i >= 0; --i) {
    if (c[i] < K - 1) {
      ++c[i];
      for (int j = i + 1; j < m; ++j) c[j] = c[i];
      return true;
    }
  }
  return false;
}

heom_status build_hier(int d, const double *Hp, int n_baths, const heom_bath *baths, int m_max, int n_max,
                       int parity, const double *parity_op, double importance_threshold, std::unique_ptr<Hier> &out) {
  if (!(importance_threshold >= 0.0)) return fail(HEOM_ERR_ARG, "importance threshold must be >= 0");
  if (d < 1 || d > 64) return fail(HEOM_ERR_ARG, "d must be in [1, 64]");
  if (!Hp) return fail(HEOM_ERR_ARG, "H is NULL");
  if (parity != 1 && parity != -1) return fail(HEOM_ERR_ARG, "parity must be +1 or -1");
  if (n_baths < 0 || (n_baths > 0 && !baths)) return fail(HEOM_ERR_ARG, "bad bath list");
  if (m_max < 0 || n_max < 0) return fail(HEOM_ERR_ARG, "negative tier");
  auto h = std::make_unique<Hier>();
  h->d = d;
  h->parity = parity;
  h->H = read_mat(Hp, d);
  if (!is_hermitian(h->H, d)) return fail(HEOM_ERR_ARG, "H is not Hermitian");
  h->ops.push_back(h->H);
  std::vector<cd> P;
  if (parity_op) {
    P = read_mat(parity_op, d);
    h->parity_op = P;
    auto c = matmul(P, h->H, d), e = matmul(h->H, P, d);
    for (int i = 0; i < d * d; ++i) c[i] -= e[i];
    if (maxabs(c) > 1e-12 * std::max(1.0, maxabs(h->H))) return fail(HEOM_ERR_ARG, "H is not parity-even");
  }
  for (int bi = 0; bi < n_baths; ++bi) {
    const heom_bath &b = baths[bi];
    if (!b.op || b.n_exp < 0) return fail(HEOM_ERR_ARG, "bath " + std::to_string(bi) + ": bad operator/n_exp");
    h->bath_kind.push_back(b.kind);
    auto O = read_mat(b.op, d);
    if (b.kind == HEOM_BOSON) {
      if (b.n_exp > 0 && (!b.u_type || !b.xi || !b.chi)) return fail(HEOM_ERR_ARG, "boson bath: missing arrays");
      if (!is_hermitian(O, d)) return fail(HEOM_ERR_ARG, "boson coupling operator is not Hermitian");
      if (parity_op) {
        auto c = matmul(P, O, d), e = matmul(O, P, d);
        for (int i = 0; i < d * d; ++i) c[i] -= e[i];
        if (maxabs(c) > 1e-12 * std::max(1.0, maxabs(O))) return fail(HEOM_ERR_ARG, "boson coupling is not parity-even");
      }
      int op = (int)h->ops.size();
      h->ops.push_back(O);
      for (int l = 0; l < b.n_exp; ++l) {
        int u = b.u_type[l];
        if (u < 0 || u > 2) return fail(HEOM_ERR_ARG, "bad bosonic exponent type");
        h->bexp.push_back({op, u, cd(b.xi[2 * l], b.xi[2 * l + 1]), cd(b.chi[2 * l], b.chi[2 * l + 1])});
      }
    } else if (b.kind == HEOM_FERMION) {
      if (b.n_exp > 0 && (!b.eta_p || !b.gam_p || !b.eta_m || !b.gam_m))
        return fail(HEOM_ERR_ARG, "fermion bath: missing arrays");
      if (parity_op) {
        auto c = matmul(P, O, d), e = matmul(O, P, d);
        for (int i = 0; i < d * d; ++i) c[i] += e[i];
        if (maxabs(c) > 1e-12 * std::max(1.0, maxabs(O))) return fail(HEOM_ERR_ARG, "fermion coupling is not parity-odd");
      }
      int op_ann = (int)h->ops.size();
      h->ops.push_back(O);                // d      (nu = -1)
      h->ops.push_back(dagger(O, d));     // d^dag  (nu = +1)
      int base = (int)h->fexp.size();
      for (int k = 0; k < b.n_exp; ++k) {
        h->fexp.push_back({op_ann, +1, base + 2 * k + 1, cd(b.eta_p[2 * k], b.eta_p[2 * k + 1]),
                           cd(b.gam_p[2 * k], b.gam_p[2 * k + 1]), base + k, bi});
        h->fexp.push_back({op_ann, -1, base + 2 * k, cd(b.eta_m[2 * k], b.eta_m[2 * k + 1]),
                           cd(b.gam_m[2 * k], b.gam_m[2 * k + 1]), base + b.n_exp + k, bi});
      }
    } else {
      return fail(HEOM_ERR_ARG, "bath kind must be HEOM_BOSON or HEOM_FERMION");
    }
  }
  h->Kb = (int)h->bexp.size();
  h->Kf = (int)h->fexp.size();
  if (h->Kf > 64) return fail(HEOM_ERR_UNSUPPORTED, "more than 64 fermionic exponents");
  h->Lb = h->Kb > 0 ? m_max : 0;
  h->Lf = std::min(n_max, h->Kf);
  if (h->Lb > 255) return fail(HEOM_ERR_UNSUPPORTED, "bosonic tier above 255");
  if (h->Lb + h->Lf > 32) return fail(HEOM_ERR_UNSUPPORTED, "more than 33 tiers");
  // bosonic occupation code: base (Lb + 1) digits
  h->bos_pow.assign(h->Kb + 1, 1);
  for (int k = 0; k < h->Kb; ++k) {
    long double next = (long double)h->bos_pow[k] * (h->Lb + 1);
    if (next > 1.8e19L) return fail(HEOM_ERR_UNSUPPORTED, "bosonic occupation code overflows 64 bits");
    h->bos_pow[k + 1] = (uint64_t)next;
  }

  // ---- enumerate: tier t = m + n ascending; n ascending; fermionic subsets
  // lexicographic (ascending index tuples); bosonic multisets lexicographic.
  // With an importance threshold, ADOs beyond levels (m, n) <= (1, 1) whose
  // eq:importance value is below it are not enumerated.
  const int Kb = h->Kb, Kf = h->Kf;
  h->importance_threshold = importance_threshold;
  std::vector<int> by_rank(Kf);
  for (int k = 0; k < Kf; ++k) by_rank[h->fexp[k].rank] = k;
  auto important = [&](const std::vector<int> &bc, uint64_t mask, int m, int n) -> bool {
    if (importance_threshold <= 0.0 || (m <= 1 && n <= 1)) return true;
    double v = 1.0, sum = 0.0;
    for (int x : bc) {  // multiset in ascending exponent order
      const double rc = h->bexp[x].chi.real();
      sum += rc;
      v *= std::abs(h->bexp[x].xi) / rc / sum;
    }
    sum = 0.0;
    for (int r = 0; r < Kf; ++r) {  // fermionic exponents in importance order
      const int k = by_rank[r];
      if (!(mask >> k & 1ull)) continue;
      const double rg = h->fexp[k].gamma.real();
      sum += rg;
      v *= std::abs(h->fexp[k].eta) / rg / sum;
    }
    return !(v < importance_threshold);
  };
  std::vector<std::pair<uint64_t, uint64_t>> keys;
  h->tier_off.clear();
  for (int t = 0; t <= h->Lb + h->Lf; ++t) {
    h->tier_off.push_back((int64_t)keys.size());
    for (int n = std::max(0, t - h->Lb); n <= std::min(t, h->Lf); ++n) {
      int m = t - n;
      std::vector<int> fc(n);
      for (int i = 0; i < n; ++i) fc[i] = i;
      bool fmore = true;
      while (fmore) {
        uint64_t mask = 0;
        for (int x : fc) mask |= 1ull << x;
        std::vector<int> bc(m, 0);
        bool bmore = (m == 0) || Kb > 0;
        while (bmore) {
          uint64_t code = 0;
          for (int x : bc) code += h->bos_pow[x];
          if (important(bc, mask, m, n)) keys.push_back({mask, code});
          if ((int64_t)keys.size() >= (1ll << 31) - 1) return fail(HEOM_ERR_UNSUPPORTED, "more than 2^31 ADOs");
          bmore = (m > 0) && next_multiset(bc, Kb);
        }
        fmore = (n > 0) && next_combination(fc, Kf);
      }
    }
  }
  h->tier_off.push_back((int64_t)keys.size());
  const int64_t N = (int64_t)keys.size();
  h->N = N;
  h->bocc.assign(N * (size_t)Kb, 0);
  h->fmask.resize(N);
  h->lev.resize(2 * N);
  h->decay.resize(N);
  for (int64_t a = 0; a < N; ++a) {
    uint64_t mask = keys[a].first, code = keys[a].second;
    h->fmask[a] = mask;
    int m = 0;
    cd c = 0.0;
    for (int k = Kb - 1; k >= 0; --k) {
      int occ = (int)(code / h->bos_pow[k]);
      code -= (uint64_t)occ * h->bos_pow[k];
      h->bocc[a * Kb + k] = (uint8_t)occ;
      m += occ;
      c += (double)occ * h->bexp[k].chi;
    }
    int n = __builtin_popcountll(mask);
    for (int k = 0; k < Kf; ++k)
      if (mask >> k & 1ull) c += h->fexp[k].gamma;
    h->lev[2 * a] = m;
    h->lev[2 * a + 1] = n;
    h->decay[a] = c;
  }
  // sorted key index for the dictionary
  std::vector<int64_t> order(N);
  for (int64_t a = 0; a < N; ++a) order[a] = a;
  std::sort(order.begin(), order.end(), [&](int64_t p, int64_t q) { return keys[p] < keys[q]; });
  h->keys.resize(N);
  h->key_index.resize(N);
  for (int64_t r = 0; r < N; ++r) { h->keys[r] = keys[order[r]]; h->key_index[r] = (int32_t)order[r]; }
  auto find = [&](uint64_t mask, uint64_t code) -> int64_t { return lookup_ado(*h, mask, code); };

  // ---- coefficient table
  //  bos up   k:              (-i, +i)                            op V_k
  //  bos down k:  R:  -i xi (V x - x V);  I: xi (V x + x V);  RI: both
  //  ferm up  k', parity of n_b:  -i s [p d^{nubar} x + (-1)^{n_b} x d^{nubar}]
  //  ferm down k, parity of n_b:  -i s [p eta d^nu x - (-1)^{n_b} conj(etabar) x d^nu]
  const cd I(0.0, 1.0);
  const double p = (double)parity;
  h->coefs.clear();
  for (int k = 0; k < Kb; ++k) h->coefs.push_back({h->bexp[k].op, -I, I});
  for (int k = 0; k < Kb; ++k) {
    const auto &e = h->bexp[k];
    cd xr = 0.0, xi = 0.0;
    if (e.u == HEOM_U_R) xr = e.xi;
    else if (e.u == HEOM_U_I) xi = e.xi;
    else { xr = e.xi.real(); xi = e.xi.imag(); }
    // -i (xr [V,.] + i xi {V,.}) = (-i xr + xi) V. + (i xr + xi) .V
    h->coefs.push_back({e.op, -I * xr + xi, I * xr + xi});
  }
  auto dnu_op = [&](int k, int nu) { return nu == +1 ? h->fexp[k].op_ann + 1 : h->fexp[k].op_ann; };
  for (int k = 0; k < Kf; ++k)
    for (int par = 0; par < 2; ++par) {
      double sgn_nb = par ? -1.0 : 1.0;  // (-1)^{n_b}
      h->coefs.push_back({dnu_op(k, -h->fexp[k].nu), -I * p, -I * sgn_nb});
    }
  for (int k = 0; k < Kf; ++k)
    for (int par = 0; par < 2; ++par) {
      double sgn_nb = par ? -1.0 : 1.0;
      cd eta = h->fexp[k].eta, etabar = h->fexp[h->fexp[k].partner].eta;
      h->coefs.push_back({dnu_op(k, h->fexp[k].nu), -I * p * eta, I * sgn_nb * std::conj(etabar)});
    }
  const int cb_up = 0, cb_dn = Kb, cf_up = 2 * Kb, cf_dn = 2 * Kb + 2 * Kf;
  h->coef_H = (int)h->coefs.size();
  h->coefs.push_back({0, -I, I});

  // ---- neighbour CSR
  h->row_ptr.assign(N + 1, 0);
  h->ecol.clear();
  h->einfo.clear();
  auto push = [&](int64_t b, int coef, int mult) {
    h->ecol.push_back((int32_t)b);
    h->einfo.push_back((int32_t)(((uint32_t)coef << 8) | (uint8_t)(int8_t)mult));
  };
  int64_t n_leaf = 0;
  for (int64_t a = 0; a < N; ++a) {
    uint64_t mask = h->fmask[a];
    uint64_t code = keys[a].second;
    int m = h->lev[2 * a], n = h->lev[2 * a + 1];
    bool has_up = false;
    // fermionic up: b = a + {k}, sign = (-1)^{#{x in a: x > k}}
    if (n < h->Lf)
      for (int k = 0; k < Kf; ++k) {
        if (mask >> k & 1ull) continue;
        int64_t b = find(mask | (1ull << k), code);
        if (b < 0) continue;
        int s = (__builtin_popcountll(k + 1 < 64 ? mask >> (k + 1) : 0ull) & 1) ? -1 : 1;
        push(b, cf_up + 2 * k + ((n + 1) & 1), s);
        has_up = true;
      }
    // bosonic up
    if (m < h->Lb)
      for (int k = 0; k < Kb; ++k) {
        int64_t b = find(mask, code + h->bos_pow[k]);
        if (b < 0) continue;
        push(b, cb_up + k, 1);
        has_up = true;
      }
    // fermionic down: b = a - {k}, sign = (-1)^{#{x in b: x > k}}
    for (int k = 0; k < Kf; ++k) {
      if (!(mask >> k & 1ull)) continue;
      uint64_t bm = mask & ~(1ull << k);
      int64_t b = find(bm, code);
      if (b < 0) continue;  // left out by the importance threshold
      int s = (__builtin_popcountll(k + 1 < 64 ? bm >> (k + 1) : 0ull) & 1) ? -1 : 1;
      push(b, cf_dn + 2 * k + ((n - 1) & 1), s);
    }
    // bosonic down with multiplicity n_k
    for (int k = 0; k < Kb; ++k) {
      int occ = h->bocc[a * Kb + k];
      if (!occ) continue;
      int64_t b = find(mask, code - h->bos_pow[k]);
      if (b < 0) continue;  // left out by the importance threshold
      push(b, cb_dn + k, occ);
    }
    if (!has_up) ++n_leaf;
    h->row_ptr[a + 1] = (int64_t)h->ecol.size();
  }
  h->n_leaf = n_leaf;

  // ---- operator ELL tables (left: rows of O; right: rows of O^T)
  OpEll &E = h->ell;
  E.n_ops = (int)h->ops.size();
  E.d = d;
  int slots = 1;
  for (auto &O : h->ops)
    for (int i = 0; i < d; ++i) {
      int cl = 0, cr = 0;
      for (int k = 0; k < d; ++k) {
        if (O[i * d + k] != 0.0) ++cl;
        if (O[k * d + i] != 0.0) ++cr;
      }
      slots = std::max(slots, std::max(cl, cr));
    }
  E.slots = slots;
  E.cnt.assign((size_t)E.n_ops * 2 * d, 0);
  E.col.assign((size_t)E.n_ops * 2 * d * slots, 0);
  E.val.assign((size_t)E.n_ops * 2 * d * slots, 0.0);
  E.op_slots.assign(E.n_ops, 0);
  for (int o = 0; o < E.n_ops; ++o) {
    auto &O = h->ops[o];
    for (int side = 0; side < 2; ++side)
      for (int i = 0; i < d; ++i) {
        size_t row = ((size_t)o * 2 + side) * d + i;
        int c = 0;
        for (int k = 0; k < d; ++k) {
          cd v = side == 0 ? O[i * d + k] : O[k * d + i];
          if (v == 0.0) continue;
          E.col[row * slots + c] = k;
          E.val[row * slots + c] = v;
          ++c;
        }
        E.cnt[row] = c;
        E.op_slots[o] = std::max(E.op_slots[o], c);
      }
  }
  // compact ELL (H without its diagonal)
  E.c_off.assign(E.n_ops, 0);
  E.c_ns.assign(E.n_ops, 0);
  E.c_real.assign(E.n_ops, 1);
  E.c_col.clear();
  E.c_val.clear();
  E.hdiag.assign(d, 0.0);
  for (int i = 0; i < d; ++i) E.hdiag[i] = h->H[i * d + i];
  for (int o = 0; o < E.n_ops; ++o) {
    auto &O = h->ops[o];
    auto keep = [&](int r, int c) { return O[r * d + c] != 0.0 && !(o == 0 && r == c); };
    int ns = 0;
    for (int i = 0; i < d; ++i) {
      int cl = 0, cr = 0;
      for (int k = 0; k < d; ++k) {
        cl += keep(i, k);
        cr += keep(k, i);
      }
      ns = std::max(ns, std::max(cl, cr));
    }
    E.c_off[o] = (int32_t)E.c_col.size();
    E.c_ns[o] = ns;
    for (int side = 0; side < 2; ++side)
      for (int i = 0; i < d; ++i) {
        int c = 0;
        for (int k = 0; k < d; ++k) {
          int r0 = side == 0 ? i : k, c0 = side == 0 ? k : i;
          if (!keep(r0, c0)) continue;
          cd v = O[r0 * d + c0];
          if (v.imag() != 0.0) E.c_real[o] = 0;
          E.c_col.push_back(k);
          E.c_val.push_back(v);
          ++c;
        }
        for (; c < ns; ++c) {
          E.c_col.push_back(0);
          E.c_val.push_back(0.0);
        }
      }
  }
  out = std::move(h);
  return HEOM_OK;
}

}  // namespace heom
