// Multi-shift spectra: every frequency from one Krylov space.
//
// The spectrum solves (Methods, "Numerical computation of the spectrum") are
// (M + sigma_k) x_k = b for thousands of shifts sigma_k = +-i omega_k with
// one right-hand side b per readout.  Without a preconditioner the Krylov
// space K_m(M + sigma, b) does not depend on sigma, so one Arnoldi process
// on M serves all shifts.  Restarting uses the full orthogonalisation method
// (FOM): its residuals are all parallel to the next Arnoldi vector,
//   b - (M + sigma_k) x_k = -h_{m+1,m} (e_m^T y_k) v_{m+1},
// so the next cycle restarts every shift from the same vector with its own
// scalar weight (restarted FOM for shifted systems, Simoncini 2003).
//
// Thick restarts (deflate = k > 0) keep, besides that vector, the Schur
// vectors V_m Z_k of the k Ritz values of M nearest the negated shifts that
// are still active (the eigenvalues that stall those shifts).  With
// H_m Z_k = Z_k T_k (reordered complex Schur form of the projected matrix)
// the kept space satisfies the shift-invariant relation
//   M (V_m Z_k) = (V_m Z_k) T_k + v_{m+1} (h_{m+1,m} e_m^T Z_k),
// so Arnoldi continues from v_{m+1}, every shift's residual stays parallel to
// the last basis vector, and each cycle solves (H + sigma_k) y = gamma_k e_k
// with the full projected matrix H (Krylov-Schur restarting, Stewart 2001).
//
// The spectrum only needs the trace readout Tr[O x_k,0] of ADO 0, which is
// linear in x_k.  Each Arnoldi vector v_j therefore contributes the scalar
// Tr[O v_j,0] once, and no solution vector is ever stored: the memory is the
// Krylov basis alone, independent of the number of frequencies.  A few probe
// shifts do keep their solution vectors, so that the true residual
// |b - (M + sigma) x| / |b| is measured with the plain apply at the end.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>

#include "blas.h"
#include "dense.h"
#include "internal.h"
#include "solvers.h"

namespace heom {

namespace {

constexpr int kMaxShiftThreads = 8;  // host threads for the per-shift projected solves

struct ShiftSystem {
  std::vector<cd> sigma;  // per frequency
  int col_b = 0;          // right-hand side = ops[col_b] . x_ss
  int col_r = 0;          // readout Tr[ops[col_r] x_0]
};


}  // namespace

size_t shifted_bytes(const Hier &h, const heom_solver_opts &o) {
  const int64_t n = h.N * (int64_t)h.d * h.d;
  const size_t vec = (size_t)n * 16;
  const int m = o.restart;
  const int nprobe = 3;
  const int64_t nch = dot_chunks(n, 1);
  return (size_t)(m + 1) * vec + (size_t)(nprobe + 2) * vec + (size_t)(2 * m + 3) * nch * sizeof(double2) +
         4 * (size_t)(m + 3) * sizeof(double2) + 2 * (size_t)h.d * h.d * 16 +
         (size_t)m * (kRotateMax + kAccumMax) * sizeof(double2) + 16 * 1024;
}

// One right-hand side, all shifts: readout[k] = Tr[ops[col_r] x_k,0].
static heom_status shifted_fom(Hier &h, const double2 *x_ss, const double2 *opsd, const std::vector<double2> &ops_h,
                               const ShiftSystem &sys, const heom_solver_opts &o, std::vector<cd> &readout,
                               heom_solver_report *rep, WsArena &ws, hipStream_t s) {
  const int d = h.d;
  const int64_t n = h.N * (int64_t)d * d;
  const int K = (int)sys.sigma.size();
  const int m = o.restart;
  readout.assign(K, cd(0));
  if (K == 0) return HEOM_OK;
  const size_t vec = (size_t)n * sizeof(double2);
  double2 *V = (double2 *)ws.take((size_t)(m + 1) * vec);
  double2 *b = (double2 *)ws.take(vec);
  double2 *r = (double2 *)ws.take(vec);
  const int nprobe = std::min(3, K);
  std::vector<double2 *> xp(nprobe);
  for (int p = 0; p < nprobe; ++p) xp[p] = (double2 *)ws.take(vec);
  const int nch = dot_chunks(n, 1);
  double2 *partial = (double2 *)ws.take((size_t)(2 * m + 3) * nch * sizeof(double2));
  double2 *hdev = (double2 *)ws.take(2 * (size_t)(m + 3) * sizeof(double2));
  double2 *sdev = (double2 *)ws.take(2 * sizeof(double2));
  const int kdef = o.deflate;  // 0: plain restarts from the residual direction
  double2 *zdev = kdef > 0 ? (double2 *)ws.take((size_t)m * kRotateMax * sizeof(double2)) : nullptr;
  double2 *ydev = (double2 *)ws.take((size_t)m * kAccumMax * sizeof(double2));
  if (!V || !b || !r || !partial || !hdev || !sdev || !ydev || (kdef > 0 && !zdev))
    return fail(HEOM_ERR_ARG, "spectrum: workspace too small");
  for (double2 *p : xp)
    if (!p) return fail(HEOM_ERR_ARG, "spectrum: workspace too small");
  PinnedBuf pin;
  HEOM_TRY(pin.ensure(sizeof(double2) * ((size_t)2 * (m + 3) + (size_t)d * d)));
  double2 *ph = (double2 *)pin.p;
  double2 *pblk = ph + 2 * (m + 3);
  // b = ops[col_b] . x_ss on every ADO
  int *colb = (int *)ws.take(sizeof(int) * 2);
  if (!colb) return fail(HEOM_ERR_ARG, "spectrum: workspace too small");
  HEOM_HIP_CHECK(hipMemcpyAsync(colb, &sys.col_b, sizeof(int), hipMemcpyHostToDevice, s));
  HEOM_TRY(left_multiply<double>(x_ss, opsd, d, h.N, 1, colb, b, s));
  for (double2 *p : xp) HEOM_HIP_CHECK(hipMemsetAsync(p, 0, vec, s));
  auto norm2 = [&](const double2 *v, double &out) -> heom_status {
    HEOM_TRY(mdot<double>(v, 0, 1, v, n, 1, partial, nch, hdev, s));
    HEOM_HIP_CHECK(hipMemcpyAsync(ph, hdev, sizeof(double2), hipMemcpyDeviceToHost, s));
    HEOM_HIP_CHECK(hipStreamSynchronize(s));
    out = std::max(ph[0].x, 0.0);
    return HEOM_OK;
  };
  double bb = 0;
  HEOM_TRY(norm2(b, bb));
  const double bnorm = std::sqrt(bb);
  if (!(bnorm > 0)) return HEOM_OK;  // zero right-hand side: zero response
  // trace functional of an ADO-0 block
  const double2 *R0 = ops_h.data() + (size_t)sys.col_r * d * d;
  auto readv = [&](const double2 *v, cd &t) -> heom_status {
    HEOM_HIP_CHECK(hipMemcpyAsync(pblk, v, sizeof(double2) * d * d, hipMemcpyDeviceToHost, s));
    HEOM_HIP_CHECK(hipStreamSynchronize(s));
    cd acc(0);
    for (int i = 0; i < d; ++i)
      for (int k = 0; k < d; ++k)
        acc += cd(R0[i * d + k].x, R0[i * d + k].y) * cd(pblk[k * d + i].x, pblk[k * d + i].y);
    t = acc;
    return HEOM_OK;
  };
  // V_0 = b / |b|; every shift starts with residual gamma_k V_0, gamma_k = |b|
  double2 sc = make_double2(1.0 / bnorm, 0.0);
  HEOM_HIP_CHECK(hipMemcpyAsync(sdev, &sc, sizeof(double2), hipMemcpyHostToDevice, s));
  HEOM_TRY(scale_vec<double>(b, sdev, V, n, 1, s));
  HEOM_HIP_CHECK(hipStreamSynchronize(s));
  std::vector<cd> gamma(K, cd(bnorm));
  std::vector<char> active(K, 1);
  std::vector<int> probe_k(nprobe);
  for (int p = 0; p < nprobe; ++p) probe_k[p] = nprobe == 1 ? 0 : (int)((int64_t)p * (K - 1) / (nprobe - 1));
  std::vector<cd> H((size_t)(m + 1) * m), t(m + 1), G((size_t)(m + 1) * (m + 1));
  int iters = 0, cycles = 0;
  int64_t applies = 0;
  double worst_est = 1.0;
  int p = 0;  // basis columns kept by a thick restart; column p is the residual direction
  // Krylov-Schur restart after a full cycle of kk columns: Schur form of the
  // projected matrix, the kdef Ritz values nearest the negated active shifts
  // moved to the front, V_k <- V_kk Z_k, v_kk moved to column kdef; the
  // projected matrix, the readout weights t and the Gram matrix G follow Z.
  // The probe updates (nact columns of ydev into outs) ride on the basis read.
  auto thick_restart = [&](int kk, cd hlast, int nact, const AccumOut &outs) -> heom_status {
    std::vector<cd> Hk((size_t)kk * kk), T, Z;
    for (int c = 0; c < kk; ++c)
      for (int i = 0; i < kk; ++i) Hk[(size_t)c * kk + i] = H[(size_t)c * (m + 1) + i];
    if (!schur_complex(kk, Hk, T, Z)) {  // no Schur form: probes, then restart plainly
      if (nact > 0) HEOM_TRY(basis_accum<double>(V, n, kk, ydev, nact, outs, n, s));
      HEOM_HIP_CHECK(hipMemcpyAsync(V, V + (size_t)kk * n, vec, hipMemcpyDeviceToDevice, s));
      HEOM_HIP_CHECK(hipStreamSynchronize(s));
      p = 0;
      return HEOM_OK;
    }
    std::vector<double> dist(kk, HUGE_VAL);
    for (int i = 0; i < kk; ++i) {
      const cd th = T[(size_t)i * kk + i];
      for (int k = 0; k < K; ++k)
        if (active[k]) dist[i] = std::min(dist[i], std::abs(th + sys.sigma[k]));
    }
    std::vector<int> order(kk);
    for (int i = 0; i < kk; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return dist[a] < dist[b]; });
    std::vector<char> sel(kk, 0);
    for (int i = 0; i < kdef; ++i) sel[order[i]] = 1;
    schur_reorder(kk, T, Z, sel);
    // V[:, 0..kdef) <- V[:, 0..kk) Z[:, 0..kdef), then v_kk to column kdef
    std::vector<double2> zh((size_t)kk * kdef);
    for (int c = 0; c < kdef; ++c)
      for (int i = 0; i < kk; ++i) {
        const cd z = Z[(size_t)c * kk + i];
        zh[(size_t)c * kk + i] = make_double2(z.real(), z.imag());
      }
    HEOM_HIP_CHECK(hipMemcpyAsync(zdev, zh.data(), sizeof(double2) * zh.size(), hipMemcpyHostToDevice, s));
    HEOM_TRY(basis_rotate<double>(V, n, kk, zdev, kdef, n, s, ydev, nact, &outs));
    HEOM_HIP_CHECK(hipMemcpyAsync(V + (size_t)kdef * n, V + (size_t)kk * n, vec, hipMemcpyDeviceToDevice, s));
    // projected matrix: T_k on top, h_{kk,kk-1} e_{kk-1}^T Z_k below it
    std::vector<cd> tn(kdef), Gn((size_t)kdef * kdef);
    for (int c = 0; c < kdef; ++c) {
      cd a(0);
      for (int i = 0; i < kk; ++i) a += t[i] * Z[(size_t)c * kk + i];
      tn[c] = a;
      for (int e = 0; e < kdef; ++e) {  // (Z^H G Z)(e, c)
        cd g(0);
        for (int i = 0; i < kk; ++i) {
          cd gz(0);
          for (int q = 0; q < kk; ++q) gz += G[(size_t)q * (m + 1) + i] * Z[(size_t)c * kk + q];
          g += std::conj(Z[(size_t)e * kk + i]) * gz;
        }
        Gn[(size_t)c * kdef + e] = g;
      }
    }
    std::fill(H.begin(), H.end(), cd(0));
    for (int c = 0; c < kdef; ++c) {
      for (int i = 0; i <= c; ++i) H[(size_t)c * (m + 1) + i] = T[(size_t)c * kk + i];
      H[(size_t)c * (m + 1) + kdef] = hlast * Z[(size_t)c * kk + kk - 1];
      t[c] = tn[c];
      for (int e = 0; e < kdef; ++e) G[(size_t)c * (m + 1) + e] = Gn[(size_t)c * kdef + e];
    }
    HEOM_HIP_CHECK(hipStreamSynchronize(s));
    p = kdef;
    return HEOM_OK;
  };
  while (true) {
    // Arnoldi on M (no shift), continued from column p
    std::fill(H.begin() + (size_t)p * (m + 1), H.end(), cd(0));
    int kk = p;
    bool breakdown = false;
    for (int j = p; j < m; ++j) {
      double2 *vj = V + (size_t)j * n, *vn = V + (size_t)(j + 1) * n;
      HEOM_TRY(readv(vj, t[j]));
      ApplyArgs a;
      a.x = vj;
      a.y = vn;
      HEOM_TRY(launch_apply(h, HEOM_FP64, a, s));
      ++applies;
      ++iters;
      // Gram-matrix CGS2: one two-vector pass gives a = V^H w, the Gram
      // column V^H v_j and |w|^2; h = a + (a - G a); one fused update +
      // normalisation pass (explicit norm when the formula cancels)
      HEOM_TRY(mdot2<double>(V, n, j + 1, vn, vj, n, partial, nch, hdev, s));
      HEOM_HIP_CHECK(hipMemcpyAsync(ph, hdev, sizeof(double2) * (2 * j + 3), hipMemcpyDeviceToHost, s));
      HEOM_HIP_CHECK(hipStreamSynchronize(s));
      std::vector<cd> av(j + 1), hv(j + 1);
      for (int i = 0; i <= j; ++i) {
        av[i] = cd(ph[i].x, ph[i].y);
        const cd c(ph[j + 1 + i].x, ph[j + 1 + i].y);
        G[(size_t)j * (m + 1) + i] = c;
        G[(size_t)i * (m + 1) + j] = std::conj(c);
      }
      const double ww = ph[2 * j + 2].x;
      if (!std::isfinite(ww)) return fail(HEOM_ERR_NAN, "spectrum: non-finite Arnoldi vector");
      for (int i = 0; i <= j; ++i) {
        cd ga(0);
        for (int q = 0; q <= j; ++q) ga += G[(size_t)q * (m + 1) + i] * av[q];
        hv[i] = 2.0 * av[i] - ga;
      }
      double hn2 = ww;
      for (int i = 0; i <= j; ++i) hn2 -= 2.0 * (std::conj(hv[i]) * av[i]).real();
      for (int i = 0; i <= j; ++i) {
        cd gh(0);
        for (int q = 0; q <= j; ++q) gh += G[(size_t)q * (m + 1) + i] * hv[q];
        hn2 += (std::conj(hv[i]) * gh).real();
      }
      std::vector<double2> hup(j + 1);
      for (int i = 0; i <= j; ++i) {
        hup[i] = make_double2(hv[i].real(), hv[i].imag());
        H[(size_t)j * (m + 1) + i] = hv[i];
      }
      HEOM_HIP_CHECK(hipMemcpyAsync(hdev, hup.data(), sizeof(double2) * (j + 1), hipMemcpyHostToDevice, s));
      const bool fused = std::isfinite(hn2) && hn2 > 1e-6 * ww;
      if (!fused) {
        HEOM_TRY(basis_update<double>(V, n, j + 1, hdev, vn, n, 1, -1.0, s));
        HEOM_TRY(norm2(vn, hn2));
      }
      double hn = std::sqrt(std::max(hn2, 0.0));
      double hscale = 0;
      for (int i = 0; i <= j; ++i) hscale = std::max(hscale, std::abs(H[(size_t)j * (m + 1) + i]));
      if (!(hn > 1e-14 * std::max(hscale, 1e-300))) {
        hn = 0.0;
        breakdown = true;  // invariant subspace: the projected solutions are exact
      }
      H[(size_t)j * (m + 1) + j + 1] = hn;
      sc = make_double2(hn > 0 ? 1.0 / hn : 0.0, 0.0);
      HEOM_HIP_CHECK(hipMemcpyAsync(sdev, &sc, sizeof(double2), hipMemcpyHostToDevice, s));
      if (fused) HEOM_TRY(basis_update<double>(V, n, j + 1, hdev, vn, n, 1, -1.0, s, sdev));
      else HEOM_TRY(scale_vec<double>(vn, sdev, vn, n, 1, s));
      HEOM_HIP_CHECK(hipStreamSynchronize(s));
      kk = j + 1;
      if (breakdown || iters >= o.max_iter) break;
    }
    ++cycles;
    // per shift: (H + sigma) y = gamma e_p, readout += t . y, new residual
    // weight.  After a thick restart H is no longer Hessenberg (row p holds
    // h_{m+1,m} e_m^T Z_k); one unitary reduction H = Q Hh Q^H per cycle
    // turns every shift's system into a Hessenberg one with right-hand side
    // gamma Q^H e_p, and the readout and last-component weights into t^T Q
    // and e_kk^T Q.
    const cd hlast = H[(size_t)(kk - 1) * (m + 1) + kk];
    const bool hess = p <= 1;
    std::vector<cd> Hh, Q, qp(kk), tq(kk), ql(kk);
    if (hess) {
      for (int j = 0; j < kk; ++j) {
        qp[j] = j == p ? cd(1) : cd(0);
        tq[j] = t[j];
        ql[j] = j == kk - 1 ? cd(1) : cd(0);
      }
    } else {
      Hh.resize((size_t)kk * kk);
      Q.assign((size_t)kk * kk, cd(0));
      for (int c = 0; c < kk; ++c) {
        Q[(size_t)c * kk + c] = 1.0;
        for (int i = 0; i < kk; ++i) Hh[(size_t)c * kk + i] = H[(size_t)c * (m + 1) + i];
      }
      hessenberg_reduce(kk, Hh, Q);
      for (int j = 0; j < kk; ++j) {
        qp[j] = std::conj(Q[(size_t)j * kk + p]);
        ql[j] = Q[(size_t)j * kk + kk - 1];
        cd a(0);
        for (int i = 0; i < kk; ++i) a += t[i] * Q[(size_t)j * kk + i];
        tq[j] = a;
      }
    }
    // the shifts are independent: contiguous ranges on a few host threads
    std::vector<std::vector<cd>> yprobe(nprobe);
    auto run_shifts = [&](int k0, int k1, bool &any_l, double &worst_l, bool &singular_l) {
      HessSolver hs;
      std::vector<cd> y, rhs(kk);
      for (int k = k0; k < k1; ++k) {
        if (!active[k]) continue;
        const double gr = gamma[k].real(), gi = gamma[k].imag();
        for (int j = 0; j < kk; ++j)
          rhs[j] = cd(gr * qp[j].real() - gi * qp[j].imag(), gr * qp[j].imag() + gi * qp[j].real());
        if (!(hess ? hs.solve(H, m + 1, kk, sys.sigma[k], rhs, y) : hs.solve(Hh, kk, kk, sys.sigma[k], rhs, y))) {
          singular_l = true;
          return;
        }
        double axr = 0, axi = 0, lr = 0, li = 0;
        for (int j = 0; j < kk; ++j) {
          const double yr = y[j].real(), yi = y[j].imag();
          axr += yr * tq[j].real() - yi * tq[j].imag();
          axi += yr * tq[j].imag() + yi * tq[j].real();
          lr += yr * ql[j].real() - yi * ql[j].imag();
          li += yr * ql[j].imag() + yi * ql[j].real();
        }
        readout[k] += cd(axr, axi);
        for (int q = 0; q < nprobe; ++q)
          if (probe_k[q] == k) {
            yprobe[q] = y;
            if (!hess) {  // coefficients in the basis V: Q y
              for (int i = 0; i < kk; ++i) {
                cd v(0);
                for (int j = 0; j < kk; ++j) v += Q[(size_t)j * kk + i] * y[j];
                yprobe[q][i] = v;
              }
            }
          }
        const double hr = hlast.real(), hi = hlast.imag();
        gamma[k] = breakdown ? cd(0) : cd(-(hr * lr - hi * li), -(hr * li + hi * lr));
        const double est = std::abs(gamma[k]) / bnorm;
        if (est <= o.tol) active[k] = 0;
        else any_l = true;
        worst_l = std::max(worst_l, est);
      }
    };
    bool any = false, singular = false;
    worst_est = 0;
    {
      const int nth = (int)std::min<int64_t>(kMaxShiftThreads, std::max<int64_t>(1, (int64_t)K * kk * kk / 100000));
      std::vector<char> any_t(nth, 0), sing_t(nth, 0);
      std::vector<double> worst_t(nth, 0.0);
      std::vector<char> fail_t(nth, 0);
      auto body = [&](int t) {
        bool a = false, sg = false;
        double w = 0.0;
        try {  // nothing may escape a worker thread (that would end the process)
          run_shifts((int)((int64_t)K * t / nth), (int)((int64_t)K * (t + 1) / nth), a, w, sg);
        } catch (...) {
          fail_t[t] = 1;
        }
        any_t[t] = a;
        sing_t[t] = sg;
        worst_t[t] = w;
      };
      std::vector<std::thread> pool;
      for (int t = 1; t < nth; ++t) {
        try {
          pool.emplace_back(body, t);
        } catch (...) {  // no thread available: this range runs here
          body(t);
        }
      }
      body(0);
      for (auto &th : pool) th.join();
      for (int t = 0; t < nth; ++t) {
        if (fail_t[t]) return fail(HEOM_ERR_ALLOC, "spectrum: host memory for the projected solves");
        any = any || any_t[t];
        singular = singular || sing_t[t];
        worst_est = std::max(worst_est, worst_t[t]);
      }
    }
    if (singular) return fail(HEOM_ERR_SINGULAR, "spectrum: singular projected shifted system");
    // probes: x_p += V y_p, all from one read of the basis (at a thick
    // restart, from the read that forms the new basis)
    AccumOut outs{};
    std::vector<double2> yh;
    int nact = 0;
    for (int q = 0; q < nprobe; ++q) {
      if (yprobe[q].empty()) continue;
      for (int j = 0; j < kk; ++j) yh.push_back(make_double2(yprobe[q][j].real(), yprobe[q][j].imag()));
      outs.p[nact++] = xp[q];
    }
    if (nact > 0) HEOM_HIP_CHECK(hipMemcpyAsync(ydev, yh.data(), sizeof(double2) * yh.size(), hipMemcpyHostToDevice, s));
    const bool more = any && !breakdown && iters < o.max_iter;
    if (more && kdef > 0 && kk == m) {
      HEOM_TRY(thick_restart(kk, hlast, nact, outs));
    } else {
      if (nact > 0) HEOM_TRY(basis_accum<double>(V, n, kk, ydev, nact, outs, n, s));
      HEOM_HIP_CHECK(hipStreamSynchronize(s));
      if (!more) break;
      // restart from the common residual direction v_{kk}
      HEOM_HIP_CHECK(hipMemcpyAsync(V, V + (size_t)kk * n, vec, hipMemcpyDeviceToDevice, s));
      p = 0;
    }
  }
  // true residuals of the probes with the plain apply
  double worst_true = 0;
  for (int p = 0; p < nprobe; ++p) {
    ApplyArgs a;
    a.x = xp[p];
    a.y = r;
    a.shift0 = sys.sigma[probe_k[p]];
    HEOM_TRY(launch_apply(h, HEOM_FP64, a, s));
    ++applies;
    HEOM_TRY((axpby<double, double>(b, 1.0, r, -1.0, n, s)));
    double rr = 0;
    HEOM_TRY(norm2(r, rr));
    worst_true = std::max(worst_true, std::sqrt(rr) / bnorm);
  }
  bool conv = true;
  for (int k = 0; k < K; ++k) conv = conv && !active[k];
  if (rep) {
    rep->iterations += iters;
    rep->restarts += cycles;
    rep->applies += applies;
    rep->true_residual = std::max(rep->true_residual, std::max(worst_true, conv ? 0.0 : worst_est));
    if (!conv || worst_true > o.tol * 10) rep->status = HEOM_ERR_NOT_CONVERGED;
  }
  if (!conv) return fail(HEOM_ERR_NOT_CONVERGED, "spectrum: some shifts did not converge");
  return HEOM_OK;
}

heom_status spectrum_shifted(Hier &hs, const double2 *x_ss, int kind, const double *op, const double *omega,
                             int64_t n_omega, double *out_host, const heom_solver_opts &o, heom_solver_report *r,
                             void *ws, size_t ws_bytes, hipStream_t s) {
  const int d = hs.d;
  auto t0 = std::chrono::steady_clock::now();
  WsArena arena(ws, ws_bytes);
  double2 *opsd = (double2 *)arena.take(2 * (size_t)d * d * sizeof(double2));
  if (!opsd) return fail(HEOM_ERR_ARG, "spectrum: workspace too small");
  std::vector<double2> ops(2 * d * d);  // ops[0] = op, ops[1] = op^dagger
  for (int i = 0; i < d; ++i)
    for (int k = 0; k < d; ++k) {
      ops[i * d + k] = make_double2(op[2 * (i * d + k)], op[2 * (i * d + k) + 1]);
      ops[d * d + i * d + k] = make_double2(op[2 * (k * d + i)], -op[2 * (k * d + i) + 1]);
    }
  HEOM_HIP_CHECK(hipMemcpyAsync(opsd, ops.data(), ops.size() * sizeof(double2), hipMemcpyHostToDevice, s));
  std::vector<ShiftSystem> systems;
  if (kind == 0) {
    // (M + i w) x_+ = op^dag rho -> Tr[op x_+];  (M - i w) x_- = op rho -> Tr[op^dag x_-]
    ShiftSystem a, b;
    a.col_b = 1; a.col_r = 0;
    b.col_b = 0; b.col_r = 1;
    for (int64_t q = 0; q < n_omega; ++q) {
      a.sigma.push_back(cd(0.0, omega[q]));
      b.sigma.push_back(cd(0.0, -omega[q]));
    }
    systems = {a, b};
  } else {
    // (M - i w) x = op rho -> Tr[op^dag x]
    ShiftSystem a;
    a.col_b = 0; a.col_r = 1;
    for (int64_t q = 0; q < n_omega; ++q) a.sigma.push_back(cd(0.0, -omega[q]));
    systems = {a};
  }
  const size_t mark = arena.used;
  std::vector<double> acc(n_omega, 0.0);
  heom_status worst = HEOM_OK;
  for (const ShiftSystem &sys : systems) {
    arena.used = mark;
    std::vector<cd> ro;
    heom_status st = shifted_fom(hs, x_ss, opsd, ops, sys, o, ro, r, arena, s);
    if (st != HEOM_OK && st != HEOM_ERR_NOT_CONVERGED) return st;
    if (st != HEOM_OK) worst = st;
    for (int64_t q = 0; q < n_omega; ++q) acc[q] += -ro[q].real() / 3.14159265358979323846;
  }
  std::copy(acc.begin(), acc.end(), out_host);
  if (r) r->seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return worst == HEOM_OK ? HEOM_OK : fail(worst, "spectrum: some frequencies did not converge");
}

}  // namespace heom
