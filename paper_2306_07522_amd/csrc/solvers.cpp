// Solvers around the Liouvillian apply: fixed-step RK4 propagation, the
// stationary state and the frequency-domain spectra (Methods, "Numerical
// computation of the spectrum"), all solved with restarted right-
// preconditioned (flexible) GMRES on device vectors.
//
// GMRES keeps its Krylov basis on the device; each Arnoldi step orthogonalises
// with classical Gram-Schmidt applied twice (CGS2, two multi-dot kernels and
// two basis updates), and copies the (j+2) x R Hessenberg column to pinned
// host memory where the Givens rotations run.  That copy is the only
// synchronisation per iteration.  Right-hand sides are independent systems
// that share every apply launch ([n][R] layout).
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>

#include "blas.h"
#include "internal.h"
#include "solvers.h"

namespace heom {

// ------------------------------------------------------------- workspace
void *WsArena::take(size_t bytes) {
  size_t off = (used + 255) & ~(size_t)255;
  if (off + bytes > size) return nullptr;
  used = off + bytes;
  return base + off;
}

PinnedBuf::~PinnedBuf() {
  if (p) (void)hipHostFree(p);
}
heom_status PinnedBuf::ensure(size_t bytes) {
  if (bytes <= cap) return HEOM_OK;
  if (p) (void)hipHostFree(p);
  p = nullptr;
  cap = 0;
  HEOM_HIP_CHECK(hipHostMalloc(&p, bytes, hipHostMallocDefault));
  cap = bytes;
  return HEOM_OK;
}

size_t gmres_bytes(int64_t n, int R, int m, bool flexible, size_t w) {
  const size_t vec = (size_t)n * R * w;
  size_t b = (size_t)(m + 1) * vec + 2 * vec + 1024;
  if (flexible) b += (size_t)m * vec + 256;
  const int nch = dot_chunks(n, R);
  b += (size_t)std::max(m + 2, R == 1 ? 2 * m + 3 : 0) * nch * R * sizeof(double2) + 256;  // partials
  b += 4 * (size_t)(m + 2) * R * sizeof(double2) + 1024;   // h, scale
  b += (size_t)(m + 1) * kRotateMax * sizeof(double2) + 256;  // basis rotation (deflated restarts)
  return b;
}

// ------------------------------------------------------------- GMRES
template <typename T>
heom_status Gmres<T>::init(WsArena &ws, int64_t n_, int R_, int m_, bool flexible_) {
  n = n_;
  R = R_;
  m = m_;
  flexible = flexible_;
  const size_t vec = (size_t)n * R * sizeof(T2);
  V = (T2 *)ws.take((size_t)(m + 1) * vec);
  w = (T2 *)ws.take(vec);
  t = (T2 *)ws.take(vec);
  Z = flexible ? (T2 *)ws.take((size_t)m * vec) : nullptr;
  nchunk = dot_chunks(n, R);
  partial = (double2 *)ws.take((size_t)std::max(m + 2, R == 1 ? 2 * m + 3 : 0) * nchunk * R * sizeof(double2));
  hdev = (double2 *)ws.take((size_t)2 * (m + 2) * R * sizeof(double2));
  sdev = (double2 *)ws.take((size_t)2 * R * sizeof(double2));
  qdev = (double2 *)ws.take((size_t)(m + 1) * kRotateMax * sizeof(double2));
  if (!V || !w || !t || (flexible && !Z) || !partial || !hdev || !sdev || !qdev)
    return fail(HEOM_ERR_ARG, "solver workspace too small (see heom_workspace_size)");
  HEOM_TRY(pin.ensure(std::max((size_t)2 * (m + 2) * R, (size_t)(m + 1) * kRotateMax) * sizeof(double2)));
  HEOM_TRY(pin_up.ensure((size_t)(m + 3 + R) * sizeof(double2)));
  H.assign((size_t)R * (m + 1) * m, cd(0));
  G.assign((size_t)(m + 1) * (m + 1), cd(0));
  cs.assign((size_t)R * m, 0.0);
  sn.assign((size_t)R * m, cd(0));
  g.assign((size_t)R * (m + 1), cd(0));
  return HEOM_OK;
}

template <typename T>
heom_status Gmres<T>::norms(const T2 *v, std::vector<double> &out, hipStream_t s) {
  HEOM_TRY(mdot<T>(v, 0, 1, v, n, R, partial, nchunk, hdev, s));
  HEOM_HIP_CHECK(hipMemcpyAsync(pin.p, hdev, sizeof(double2) * R, hipMemcpyDeviceToHost, s));
  HEOM_HIP_CHECK(hipStreamSynchronize(s));
  const double2 *hp = (const double2 *)pin.p;
  out.resize(R);
  for (int r = 0; r < R; ++r) out[r] = std::sqrt(std::max(hp[r].x, 0.0));
  return HEOM_OK;
}

// One Arnoldi orthogonalisation for a single right-hand side, on
// w = V_{j+1} (already A z_j): two-pass classical Gram-Schmidt with the
// Gram matrix.  One pass over the basis gives a = V^H w, the new Gram column
// c = V^H v_j and |w|^2; the reorthogonalised coefficients follow from the
// measured Gram matrix G = V^H V as h = a + (a - G a) (the second projection
// of CGS2 without re-reading the basis), |w - V h|^2 from
// |w|^2 - 2 Re(h^H a) + h^H G h, and a second pass applies the update and
// the normalisation together.  Returns h (j + 1 entries) and |w - V h|.
template <typename T>
heom_status Gmres<T>::gram_step(int j, std::vector<cd> &hc, double &hnorm, hipStream_t s) {
  const int64_t nr = n;
  T2 *vj = V + (size_t)j * nr;
  T2 *vn = V + (size_t)(j + 1) * nr;
  double2 *h1 = hdev, *h2 = hdev + (size_t)(m + 2);
  HEOM_TRY(mdot2<T>(V, nr, j + 1, vn, vj, n, partial, nchunk, h1, s));
  HEOM_HIP_CHECK(hipMemcpyAsync(pin.p, h1, sizeof(double2) * (2 * j + 3), hipMemcpyDeviceToHost, s));
  HEOM_HIP_CHECK(hipStreamSynchronize(s));
  const double2 *pp = (const double2 *)pin.p;
  std::vector<cd> a(j + 1);
  hc.assign(j + 1, cd(0));
  for (int i = 0; i <= j; ++i) {
    a[i] = cd(pp[i].x, pp[i].y);
    const cd c(pp[j + 1 + i].x, pp[j + 1 + i].y);
    G[(size_t)j * (m + 1) + i] = c;                // G[i][j] (column j)
    G[(size_t)i * (m + 1) + j] = std::conj(c);     // G[j][i]
  }
  const double ww = pp[2 * j + 2].x;
  if (!std::isfinite(ww)) return fail(HEOM_ERR_NAN, "non-finite Arnoldi norm");
  for (int i = 0; i <= j; ++i) {
    cd ga(0);
    for (int q = 0; q <= j; ++q) ga += G[(size_t)q * (m + 1) + i] * a[q];
    hc[i] = 2.0 * a[i] - ga;
  }
  double w2 = ww;
  for (int i = 0; i <= j; ++i) w2 -= 2.0 * (std::conj(hc[i]) * a[i]).real();
  cd hgh(0);
  for (int i = 0; i <= j; ++i) {
    cd gh(0);
    for (int q = 0; q <= j; ++q) gh += G[(size_t)q * (m + 1) + i] * hc[q];
    hgh += std::conj(hc[i]) * gh;
  }
  w2 += hgh.real();
  // uploads from the solver's own pinned staging: the host writes it again
  // only after the next step's read-back synchronisation, which these copies
  // precede on the stream, so no wait is needed here
  double2 *hv = (double2 *)pin_up.p;
  double2 *scv = hv + (m + 2);
  for (int i = 0; i <= j; ++i) hv[i] = make_double2(hc[i].real(), hc[i].imag());
  HEOM_HIP_CHECK(hipMemcpyAsync(h1, hv, sizeof(double2) * (j + 1), hipMemcpyHostToDevice, s));
  *scv = make_double2(0.0, 0.0);
  if (std::isfinite(w2) && w2 > 1e-6 * ww) {
    hnorm = std::sqrt(w2);
    scv->x = hnorm > 1e-300 ? 1.0 / hnorm : 0.0;
    HEOM_HIP_CHECK(hipMemcpyAsync(sdev, scv, sizeof(double2), hipMemcpyHostToDevice, s));
    HEOM_TRY(basis_update<T>(V, nr, j + 1, h1, vn, n, 1, -1.0, s, sdev));
  } else {  // cancellation: measure the norm directly
    HEOM_TRY(basis_update<T>(V, nr, j + 1, h1, vn, n, 1, -1.0, s));
    HEOM_TRY(mdot<T>(vn, 0, 1, vn, n, 1, partial, nchunk, h2, s));
    HEOM_HIP_CHECK(hipMemcpyAsync(pin.p, h2, sizeof(double2), hipMemcpyDeviceToHost, s));
    HEOM_HIP_CHECK(hipStreamSynchronize(s));
    const double v = ((const double2 *)pin.p)[0].x;
    if (!std::isfinite(v)) return fail(HEOM_ERR_NAN, "non-finite Arnoldi norm");
    hnorm = std::sqrt(std::max(v, 0.0));
    scv->x = hnorm > 1e-300 ? 1.0 / hnorm : 0.0;
    HEOM_HIP_CHECK(hipMemcpyAsync(sdev, scv, sizeof(double2), hipMemcpyHostToDevice, s));
    HEOM_TRY(scale_vec<T>(vn, sdev, vn, n, 1, s));
  }
  return HEOM_OK;
}

template <typename T>
heom_status Gmres<T>::solve(const T2 *b, T2 *x, double tol, int max_iter, bool x_is_zero, GmresStats &st,
                            hipStream_t s) {
  if (deflate > 0) {
    if (R != 1 || flexible || deflate + 1 > kRotateMax || deflate + 2 > m)
      return fail(HEOM_ERR_ARG, "deflated restarting needs one right-hand side, a fixed preconditioner and "
                                "1 <= deflate <= min(31, restart - 2)");
    return solve_dr(b, x, tol, max_iter, x_is_zero, st, s);
  }
  const int64_t nr = n * R;
  std::vector<double> bnorm, beta;
  HEOM_TRY(norms(b, bnorm, s));
  st.converged = false;
  std::vector<int> kcol(R, 0);
  std::vector<char> done(R, 0);
  int iters = 0;
  double prev_worst = 0.0;
  for (int cycle = 0;; ++cycle) {
    // r = b - A x
    if (x_is_zero && cycle == 0) {
      HEOM_TRY((axpby<T, T>(b, 1.0, w, 0.0, nr, s)));
    } else {
      HEOM_TRY(A(x, w));
      ++st.applies;
      HEOM_TRY((axpby<T, T>(b, 1.0, w, -1.0, nr, s)));
    }
    HEOM_TRY(norms(w, beta, s));
    bool all = true;
    double worst = 0.0;
    for (int r = 0; r < R; ++r) {
      const double rel = bnorm[r] > 0 ? beta[r] / bnorm[r] : 0.0;
      if (!std::isfinite(rel)) return fail(HEOM_ERR_NAN, "non-finite residual in GMRES");
      worst = std::max(worst, rel);
      done[r] = rel <= tol;
      all = all && done[r];
    }
    st.residual = worst;
    static const bool verbose = std::getenv("HEOMX_VERBOSE") != nullptr;
    if (verbose)
      std::fprintf(stderr, "heomx gmres<%s>: cycle %d iterations %d true residual %.3e (R=%d)\n",
                   sizeof(T) == 8 ? "fp64" : "fp32", cycle, iters, worst, R);
    if (all) {
      st.converged = true;
      break;
    }
    if (iters >= max_iter) break;
    if (stall > 0.0 && cycle >= 1 && worst > stall * prev_worst) break;
    prev_worst = worst;
    ++st.restarts;
    // V0 = r / beta
    double2 *sc = (double2 *)pin.p;
    for (int r = 0; r < R; ++r) sc[r] = make_double2(beta[r] > 0 && !done[r] ? 1.0 / beta[r] : 0.0, 0.0);
    HEOM_HIP_CHECK(hipMemcpyAsync(sdev, sc, sizeof(double2) * R, hipMemcpyHostToDevice, s));
    HEOM_TRY(scale_vec<T>(w, sdev, V, n, R, s));
    std::fill(g.begin(), g.end(), cd(0));
    for (int r = 0; r < R; ++r) {
      g[(size_t)r * (m + 1)] = done[r] ? 0.0 : beta[r];
      kcol[r] = 0;
    }
    std::vector<char> active(R);
    for (int r = 0; r < R; ++r) active[r] = !done[r] && beta[r] > 0;
    int j = 0;
    for (; j < m && iters < max_iter; ++j, ++iters) {
      T2 *vj = V + (size_t)j * nr;
      T2 *vn = V + (size_t)(j + 1) * nr;  // w = A z_j is built in the next basis slot
      T2 *zj = P ? (flexible ? Z + (size_t)j * nr : t) : vj;
      if (P) HEOM_TRY(P(vj, zj, flexible));
      HEOM_TRY(A(zj, vn));
      ++st.applies;
      // One right-hand side: Gram-matrix CGS2 (gram_step).  Several:
      // classical Gram-Schmidt with selective reorthogonalisation (the test
      // of Daniel, Gragg, Kaufman and Stewart): one pass gives h = V^H w and
      // |w|^2 together, and |w - V h|^2 follows by Pythagoras.  When the
      // projection removed more than half of |w|^2 a second pass re-projects;
      // otherwise the update and the normalisation are one fused pass.
      double2 *h1 = hdev, *h2 = hdev + (size_t)(m + 2) * R;
      const size_t hb = sizeof(double2) * (size_t)(j + 2) * R;
      std::vector<double2> hv1((size_t)(j + 2) * R), hv2((size_t)(j + 2) * R, make_double2(0.0, 0.0));
      std::vector<double> hn(R, 0.0);
      // per-RHS scales, uploaded from the solver's pinned staging (slots
      // m + 3 ...): the host rewrites them only after the next iteration's
      // read-back synchronisation
      double2 *scv = (double2 *)pin_up.p + (m + 3);
      auto scales = [&]() {
        for (int r = 0; r < R; ++r) scv[r] = make_double2(active[r] && hn[r] > 1e-300 ? 1.0 / hn[r] : 0.0, 0.0);
      };
      if (R == 1) {
        std::vector<cd> hc;
        HEOM_TRY(gram_step(j, hc, hn[0], s));
        for (int i = 0; i <= j; ++i) hv1[i] = make_double2(hc[i].real(), hc[i].imag());
      } else {
        HEOM_TRY(mdot<T>(V, nr, j + 2, vn, n, R, partial, nchunk, h1, s));
        HEOM_HIP_CHECK(hipMemcpyAsync(pin.p, h1, hb, hipMemcpyDeviceToHost, s));
        HEOM_HIP_CHECK(hipStreamSynchronize(s));
        std::memcpy(hv1.data(), pin.p, hb);
        auto sumsq = [&](const std::vector<double2> &hv, int r) {
          double p = 0.0;
          for (int i = 0; i <= j; ++i) p += hv[(size_t)i * R + r].x * hv[(size_t)i * R + r].x +
                                           hv[(size_t)i * R + r].y * hv[(size_t)i * R + r].y;
          return p;
        };
        bool reorth = false;
        for (int r = 0; r < R; ++r) {
          if (!active[r]) continue;
          const double ww = hv1[(size_t)(j + 1) * R + r].x, w1 = ww - sumsq(hv1, r);
          if (!std::isfinite(ww) || !std::isfinite(w1)) return fail(HEOM_ERR_NAN, "non-finite Arnoldi norm");
          if (w1 > 0.5 * ww) hn[r] = std::sqrt(w1);
          else reorth = true;
        }
        if (!reorth) {
          scales();
          HEOM_HIP_CHECK(hipMemcpyAsync(sdev, scv, sizeof(double2) * R, hipMemcpyHostToDevice, s));
          HEOM_TRY(basis_update<T>(V, nr, j + 1, h1, vn, n, R, -1.0, s, sdev));
        } else {
          HEOM_TRY(basis_update<T>(V, nr, j + 1, h1, vn, n, R, -1.0, s));
          HEOM_TRY(mdot<T>(V, nr, j + 2, vn, n, R, partial, nchunk, h2, s));
          HEOM_HIP_CHECK(hipMemcpyAsync(pin.p, h2, hb, hipMemcpyDeviceToHost, s));
          HEOM_HIP_CHECK(hipStreamSynchronize(s));
          std::memcpy(hv2.data(), pin.p, hb);
          bool explicit_norm = false;
          for (int r = 0; r < R; ++r) {
            if (!active[r]) continue;
            const double w1 = hv2[(size_t)(j + 1) * R + r].x, w2 = w1 - sumsq(hv2, r);
            if (!std::isfinite(w2)) return fail(HEOM_ERR_NAN, "non-finite Arnoldi norm");
            if (w2 > 1e-2 * w1) hn[r] = std::sqrt(w2);
            else explicit_norm = true;  // cancellation again: measure the norm directly
          }
          if (!explicit_norm) {
            scales();
            HEOM_HIP_CHECK(hipMemcpyAsync(sdev, scv, sizeof(double2) * R, hipMemcpyHostToDevice, s));
            HEOM_TRY(basis_update<T>(V, nr, j + 1, h2, vn, n, R, -1.0, s, sdev));
          } else {
            HEOM_TRY(basis_update<T>(V, nr, j + 1, h2, vn, n, R, -1.0, s));
            HEOM_TRY(mdot<T>(vn, 0, 1, vn, n, R, partial, nchunk, h2 + (size_t)(j + 1) * R, s));
            HEOM_HIP_CHECK(hipMemcpyAsync(pin.p, h2 + (size_t)(j + 1) * R, sizeof(double2) * R, hipMemcpyDeviceToHost, s));
            HEOM_HIP_CHECK(hipStreamSynchronize(s));
            for (int r = 0; r < R; ++r) {
              const double v = ((const double2 *)pin.p)[r].x;
              if (!std::isfinite(v)) return fail(HEOM_ERR_NAN, "non-finite Arnoldi norm");
              hn[r] = std::sqrt(std::max(v, 0.0));
            }
            scales();
            HEOM_HIP_CHECK(hipMemcpyAsync(sdev, scv, sizeof(double2) * R, hipMemcpyHostToDevice, s));
            HEOM_TRY(scale_vec<T>(vn, sdev, vn, n, R, s));
          }
        }
      }
      bool all_done = true;
      for (int r = 0; r < R; ++r) {
        cd *Hc = &H[((size_t)r * (m + 1)) * m];  // column-major (m+1) x m
        for (int i = 0; i <= j; ++i) {
          Hc[(size_t)j * (m + 1) + i] = cd(hv1[(size_t)i * R + r].x + hv2[(size_t)i * R + r].x,
                                           hv1[(size_t)i * R + r].y + hv2[(size_t)i * R + r].y);
        }
        Hc[(size_t)j * (m + 1) + j + 1] = hn[r];
        const bool use = active[r] && hn[r] > 1e-300;
        if (!active[r]) continue;
        // previous rotations
        cd *col = &Hc[(size_t)j * (m + 1)];
        for (int i = 0; i < j; ++i) {
          const double c = cs[(size_t)r * m + i];
          const cd sv = sn[(size_t)r * m + i];
          const cd tmp = c * col[i] + sv * col[i + 1];
          col[i + 1] = -std::conj(sv) * col[i] + c * col[i + 1];
          col[i] = tmp;
        }
        // new rotation zeroing col[j+1]
        const cd aa = col[j], bb = col[j + 1];
        const double na = std::abs(aa), nb = std::abs(bb);
        double c;
        cd sv, rr;
        if (nb == 0.0) { c = 1.0; sv = 0.0; rr = aa; }
        else if (na == 0.0) { c = 0.0; sv = std::conj(bb) / nb; rr = nb; }
        else {
          const double nrm = std::sqrt(na * na + nb * nb);
          c = na / nrm;
          sv = (aa / na) * std::conj(bb) / nrm;
          rr = (aa / na) * nrm;
        }
        cs[(size_t)r * m + j] = c;
        sn[(size_t)r * m + j] = sv;
        col[j] = rr;
        col[j + 1] = 0.0;
        cd *gr = &g[(size_t)r * (m + 1)];
        gr[j + 1] = -std::conj(sv) * gr[j];
        gr[j] = c * gr[j];
        kcol[r] = j + 1;
        const double rel = bnorm[r] > 0 ? std::abs(gr[j + 1]) / bnorm[r] : 0.0;
        if (rel <= tol * 0.5 || !use) active[r] = 0;  // stop extending this system's basis
        all_done = all_done && !active[r];
      }
      if (all_done) { ++j; ++iters; break; }
    }
    st.iterations = iters;
    // y per RHS from the triangular system, then the update
    int kmax = 0;
    for (int r = 0; r < R; ++r) kmax = std::max(kmax, kcol[r]);
    if (kmax == 0) continue;
    double2 *yh = (double2 *)pin.p;
    for (int i = 0; i < kmax; ++i)
      for (int r = 0; r < R; ++r) yh[(size_t)i * R + r] = make_double2(0, 0);
    for (int r = 0; r < R; ++r) {
      const int k = kcol[r];
      const cd *Hc = &H[((size_t)r * (m + 1)) * m];
      std::vector<cd> y(k);
      for (int i = k - 1; i >= 0; --i) {
        cd acc = g[(size_t)r * (m + 1) + i];
        for (int q = i + 1; q < k; ++q) acc -= Hc[(size_t)q * (m + 1) + i] * y[q];
        const cd dgl = Hc[(size_t)i * (m + 1) + i];
        y[i] = std::abs(dgl) > 0 ? acc / dgl : cd(0);
      }
      for (int i = 0; i < k; ++i) yh[(size_t)i * R + r] = make_double2(y[i].real(), y[i].imag());
    }
    HEOM_HIP_CHECK(hipMemcpyAsync(hdev, yh, sizeof(double2) * kmax * R, hipMemcpyHostToDevice, s));
    if (flexible) {
      HEOM_TRY(basis_update<T>(Z, nr, kmax, hdev, x, n, R, 1.0, s));
    } else {
      HEOM_HIP_CHECK(hipMemsetAsync(t, 0, sizeof(T2) * nr, s));
      HEOM_TRY(basis_update<T>(V, nr, kmax, hdev, t, n, R, 1.0, s));
      if (P) {
        HEOM_TRY(P(t, w, false));
        HEOM_TRY((axpby<T, T>(w, 1.0, x, 1.0, nr, s)));
      } else {
        HEOM_TRY((axpby<T, T>(t, 1.0, x, 1.0, nr, s)));
      }
    }
    HEOM_HIP_CHECK(hipStreamSynchronize(s));
    x_is_zero = false;
  }
  return HEOM_OK;
}

template struct Gmres<double>;
template struct Gmres<float>;

}  // namespace heom
