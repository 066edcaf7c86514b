// GMRES with deflated restarting (GMRES-DR; R. B. Morgan, "GMRES with
// deflated restarting", SIAM J. Sci. Comput. 24 (2002) 20-37) for one
// right-hand side and a fixed right preconditioner.
//
// Restarted GMRES forgets its Krylov space at every restart.  When the
// operator has a few eigenvalues near the origin, as the HEOMLS of weakly
// coupled baths has (slow population relaxation), the residual then stalls.
// At each restart GMRES-DR keeps the k harmonic Ritz vectors of smallest
// harmonic Ritz value together with the residual.  These span a space on
// which an Arnoldi-like relation A P V_k = V_{k+1} Hbar_k holds, and the
// next cycle extends it by m - k ordinary Arnoldi steps.
//
// Device work per restart: one in-place change of basis V <- V Q of the
// m + 1 basis vectors to k + 1 (basis_rotate).  Everything else is on the
// (m + 1) x m projected matrices on the host.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "blas.h"
#include "dense.h"
#include "solvers.h"

namespace heom {

namespace {

struct Givens {
  int row;  // acts on rows (row, row + 1)
  double c;
  cd s;
};

Givens givens_zeroing(int row, cd a, cd b) {
  const double na = std::abs(a), nb = std::abs(b);
  if (nb == 0.0) return {row, 1.0, cd(0)};
  if (na == 0.0) return {row, 0.0, std::conj(b) / nb};
  const double nrm = std::hypot(na, nb);
  return {row, na / nrm, (a / na) * std::conj(b) / nrm};
}

void apply_givens(const Givens &g, cd &x, cd &y) {
  const cd t = g.c * x + g.s * y;
  y = -std::conj(g.s) * x + g.c * y;
  x = t;
}

}  // namespace

template <typename T>
heom_status Gmres<T>::solve_dr(const T2 *b, T2 *x, double tol, int max_iter, bool x_is_zero, GmresStats &st,
                               hipStream_t s) {
  const int64_t nr = n;
  const int ld = m + 1;  // leading dimension of H (m + 1 rows) and G
  std::vector<double> bnorm, beta;
  HEOM_TRY(norms(b, bnorm, s));
  const double bn = bnorm[0];
  st.converged = false;
  static const bool verbose = std::getenv("HEOMX_VERBOSE") != nullptr;

  // true residual r = b - A x into w
  auto true_residual = [&](double &rel) -> heom_status {
    if (x_is_zero) {
      HEOM_TRY((axpby<T, T>(b, 1.0, w, 0.0, nr, s)));
    } else {
      HEOM_TRY(A(x, w));
      ++st.applies;
      HEOM_TRY((axpby<T, T>(b, 1.0, w, -1.0, nr, s)));
    }
    HEOM_TRY(norms(w, beta, s));
    rel = bn > 0 ? beta[0] / bn : 0.0;
    if (!std::isfinite(rel)) return fail(HEOM_ERR_NAN, "non-finite residual in GMRES-DR");
    st.residual = rel;
    return HEOM_OK;
  };

  std::vector<cd> H((size_t)ld * m, cd(0)), c(ld, cd(0));
  int iters = 0, start = 0;
  bool fresh = true;
  double rel = 0.0;
  HEOM_TRY(true_residual(rel));
  for (int cycle = 0;; ++cycle) {
    if (verbose)
      std::fprintf(stderr, "heomx gmres-dr<%s>: cycle %d iterations %d true residual %.3e (k=%d, m=%d)\n",
                   sizeof(T) == 8 ? "fp64" : "fp32", cycle, iters, rel, deflate, m);
    if (rel <= tol) {
      st.converged = true;
      break;
    }
    if (iters >= max_iter) break;
    ++st.restarts;
    if (fresh) {  // plain restart from the true residual held in w
      double2 *sc = (double2 *)pin.p;
      sc[0] = make_double2(1.0 / beta[0], 0.0);
      HEOM_HIP_CHECK(hipMemcpyAsync(sdev, sc, sizeof(double2), hipMemcpyHostToDevice, s));
      HEOM_TRY(scale_vec<T>(w, sdev, V, n, 1, s));
      HEOM_HIP_CHECK(hipStreamSynchronize(s));
      std::fill(H.begin(), H.end(), cd(0));
      std::fill(c.begin(), c.end(), cd(0));
      c[0] = beta[0];
      start = 0;
    }

    // least squares min |c - H y| by Givens rotations on a copy: first the
    // full (start + 1) x start block kept from the last cycle, bottom-up per
    // column, then one rotation per new Hessenberg column
    std::vector<cd> Rm = H, g = c;
    std::vector<Givens> rots;
    for (int q = 0; q < start; ++q)
      for (int i = start; i > q; --i) {
        const Givens gv = givens_zeroing(i - 1, Rm[(i - 1) + (size_t)q * ld], Rm[i + (size_t)q * ld]);
        for (int col = q; col < start; ++col) apply_givens(gv, Rm[(i - 1) + (size_t)col * ld], Rm[i + (size_t)col * ld]);
        apply_givens(gv, g[i - 1], g[i]);
        Rm[i + (size_t)q * ld] = 0.0;
        rots.push_back(gv);
      }
    int kk = start;
    double est = bn > 0 ? std::abs(g[start]) / bn : 0.0;
    for (int j = start; j < m && iters < max_iter; ++j) {
      T2 *vj = V + (size_t)j * nr;
      T2 *vn = V + (size_t)(j + 1) * nr;
      T2 *zj = P ? t : vj;
      if (P) HEOM_TRY(P(vj, zj, false));
      HEOM_TRY(A(zj, vn));
      ++st.applies;
      std::vector<cd> hc;
      double hn = 0.0;
      HEOM_TRY(gram_step(j, hc, hn, s));
      ++iters;
      for (int i = 0; i <= j; ++i) H[i + (size_t)j * ld] = hc[i];
      H[(j + 1) + (size_t)j * ld] = hn;
      cd *col = &Rm[(size_t)j * ld];
      for (int i = 0; i <= j + 1; ++i) col[i] = H[i + (size_t)j * ld];
      for (const Givens &gv : rots) apply_givens(gv, col[gv.row], col[gv.row + 1]);
      const Givens gv = givens_zeroing(j, col[j], col[j + 1]);
      apply_givens(gv, col[j], col[j + 1]);
      col[j + 1] = 0.0;
      apply_givens(gv, g[j], g[j + 1]);
      rots.push_back(gv);
      kk = j + 1;
      est = bn > 0 ? std::abs(g[j + 1]) / bn : 0.0;
      if (!(hn > 1e-300) || est <= 0.5 * tol) break;
    }
    st.iterations = iters;

    // y from the triangular system, then x += P (V y)
    std::vector<cd> y(kk);
    for (int i = kk - 1; i >= 0; --i) {
      cd acc = g[i];
      for (int q = i + 1; q < kk; ++q) acc -= Rm[i + (size_t)q * ld] * y[q];
      const cd dg = Rm[i + (size_t)i * ld];
      y[i] = std::abs(dg) > 0 ? acc / dg : cd(0);
    }
    if (kk > 0) {
      double2 *yh = (double2 *)pin.p;
      for (int i = 0; i < kk; ++i) yh[i] = make_double2(y[i].real(), y[i].imag());
      HEOM_HIP_CHECK(hipMemcpyAsync(hdev, yh, sizeof(double2) * kk, hipMemcpyHostToDevice, s));
      HEOM_HIP_CHECK(hipMemsetAsync(t, 0, sizeof(T2) * nr, s));
      HEOM_TRY(basis_update<T>(V, nr, kk, hdev, t, n, 1, 1.0, s));
      if (P) {
        HEOM_TRY(P(t, w, false));
        HEOM_TRY((axpby<T, T>(w, 1.0, x, 1.0, nr, s)));
      } else {
        HEOM_TRY((axpby<T, T>(t, 1.0, x, 1.0, nr, s)));
      }
      HEOM_HIP_CHECK(hipStreamSynchronize(s));
      x_is_zero = false;
    }
    HEOM_TRY(true_residual(rel));
    if (rel <= tol || iters >= max_iter) continue;  // the loop head reports and stops

    // deflated restart needs a full cycle; otherwise restart plainly
    fresh = true;
    if (kk < m) continue;
    std::vector<cd> rc(ld);
    for (int i = 0; i < ld; ++i) {
      cd acc = c[i];
      for (int q = 0; q < m; ++q) acc -= H[i + (size_t)q * ld] * y[q];
      rc[i] = acc;
    }
    // harmonic Ritz pairs: (H_m + |h_{m+1,m}|^2 H_m^{-H} e_m e_m^T) g = theta g
    std::vector<cd> Hm((size_t)m * m), HmH((size_t)m * m), f(m, cd(0));
    for (int q = 0; q < m; ++q)
      for (int i = 0; i < m; ++i) {
        Hm[i + (size_t)q * m] = H[i + (size_t)q * ld];
        HmH[q + (size_t)i * m] = std::conj(H[i + (size_t)q * ld]);
      }
    f[m - 1] = 1.0;
    if (!lu_solve(m, HmH, f)) continue;
    const double hl2 = std::norm(H[m + (size_t)(m - 1) * ld]);
    for (int i = 0; i < m; ++i) Hm[i + (size_t)(m - 1) * m] += hl2 * f[i];
    std::vector<cd> theta, vecs;
    if (!eig_general(m, Hm, theta, vecs)) continue;
    std::vector<int> order(m);
    for (int i = 0; i < m; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b2) { return std::abs(theta[a]) < std::abs(theta[b2]); });
    const int k = deflate;
    std::vector<cd> Pm((size_t)ld * (k + 1), cd(0));
    for (int q = 0; q < k; ++q)
      for (int i = 0; i < m; ++i) Pm[i + (size_t)q * ld] = vecs[i + (size_t)order[q] * m];
    const int k1 = orthonormalise_columns(ld, k, Pm, 1e-10);
    for (int i = 0; i < ld; ++i) Pm[i + (size_t)k1 * ld] = rc[i];
    if (orthonormalise_columns(ld, k1 + 1, Pm, 1e-10) != k1 + 1 || k1 < 1) continue;
    // projected matrices of the new basis V Q (Q = Pm, ld x (k1 + 1))
    std::vector<cd> HQ((size_t)ld * k1, cd(0));  // H Q_k, ld x k1
    for (int q = 0; q < k1; ++q)
      for (int l = 0; l < m; ++l) {
        const cd ql = Pm[l + (size_t)q * ld];
        if (ql == cd(0)) continue;
        for (int i = 0; i < ld; ++i) HQ[i + (size_t)q * ld] += H[i + (size_t)l * ld] * ql;
      }
    std::vector<cd> Hn((size_t)(k1 + 1) * k1), cn(k1 + 1), Gn((size_t)(k1 + 1) * (k1 + 1));
    for (int p = 0; p <= k1; ++p) {
      for (int q = 0; q < k1; ++q) {
        cd acc(0);
        for (int i = 0; i < ld; ++i) acc += std::conj(Pm[i + (size_t)p * ld]) * HQ[i + (size_t)q * ld];
        Hn[p + (size_t)q * (k1 + 1)] = acc;
      }
      cd acc(0);
      for (int i = 0; i < ld; ++i) acc += std::conj(Pm[i + (size_t)p * ld]) * rc[i];
      cn[p] = acc;
    }
    // Gram matrix of V Q: the last basis vector's column was never measured;
    // it is orthonormal to the others to the accuracy of CGS2
    std::vector<cd> Gf((size_t)ld * ld);
    for (int q = 0; q < ld; ++q)
      for (int i = 0; i < ld; ++i)
        Gf[i + (size_t)q * ld] = (i < m && q < m) ? G[i + (size_t)q * ld] : cd(i == q ? 1.0 : 0.0);
    for (int p = 0; p <= k1; ++p)
      for (int q = 0; q <= k1; ++q) {
        cd acc(0);
        for (int i = 0; i < ld; ++i) {
          cd gq(0);
          for (int l = 0; l < ld; ++l) gq += Gf[i + (size_t)l * ld] * Pm[l + (size_t)q * ld];
          acc += std::conj(Pm[i + (size_t)p * ld]) * gq;
        }
        Gn[p + (size_t)q * (k1 + 1)] = acc;
      }
    // V_0..V_k1 <- V Q on the device
    double2 *qh = (double2 *)pin.p;
    for (int q = 0; q <= k1; ++q)
      for (int i = 0; i < ld; ++i) {
        const cd z = Pm[i + (size_t)q * ld];
        qh[i + (size_t)q * ld] = make_double2(z.real(), z.imag());
      }
    HEOM_HIP_CHECK(hipMemcpyAsync(qdev, qh, sizeof(double2) * ld * (k1 + 1), hipMemcpyHostToDevice, s));
    HEOM_TRY(basis_rotate<T>(V, nr, ld, qdev, k1 + 1, n, s));
    HEOM_HIP_CHECK(hipStreamSynchronize(s));
    std::fill(H.begin(), H.end(), cd(0));
    std::fill(c.begin(), c.end(), cd(0));
    for (int q = 0; q < k1; ++q)
      for (int p = 0; p <= k1; ++p) H[p + (size_t)q * ld] = Hn[p + (size_t)q * (k1 + 1)];
    for (int p = 0; p <= k1; ++p) c[p] = cn[p];
    for (int q = 0; q <= k1; ++q)
      for (int p = 0; p <= k1; ++p) G[p + (size_t)q * ld] = Gn[p + (size_t)q * (k1 + 1)];
    start = k1;
    fresh = false;
  }
  return HEOM_OK;
}

template heom_status Gmres<double>::solve_dr(const double2 *, double2 *, double, int, bool, GmresStats &, hipStream_t);
template heom_status Gmres<float>::solve_dr(const float2 *, float2 *, double, int, bool, GmresStats &, hipStream_t);

}  // namespace heom
