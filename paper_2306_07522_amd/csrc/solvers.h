// Solver building blocks shared by the propagate / steady / spectrum drivers.
#pragma once

#include <functional>

#include "blas.h"
#include "device_common.h"
#include "internal.h"

namespace heom {

// Bump allocator over a caller-owned device workspace.
struct WsArena {
  char *base = nullptr;
  size_t size = 0, used = 0;
  WsArena(void *p, size_t n) : base((char *)p), size(n) {}
  void *take(size_t bytes);
};

struct PinnedBuf {
  void *p = nullptr;
  size_t cap = 0;
  ~PinnedBuf();
  heom_status ensure(size_t bytes);
};

struct GmresStats {
  int iterations = 0, restarts = 0;
  int64_t applies = 0;
  double residual = 0.0;  // max relative residual of the last true-residual check
  bool converged = false;
};

size_t gmres_bytes(int64_t n, int R, int m, bool flexible, size_t elem_bytes);

// Restarted right-preconditioned GMRES (FGMRES when flexible) on [n][R]
// device vectors.  A(in, out): out = A in.  P(in, out, flexible): out =
// M^{-1} in (may be empty for no preconditioning).
template <typename T>
struct Gmres {
  using T2 = typename Cplx<T>::t;
  int64_t n = 0;
  int R = 1, m = 30;
  bool flexible = false;
  std::function<heom_status(const void *, void *)> A;
  std::function<heom_status(const void *, void *, bool)> P;
  T2 *V = nullptr, *Z = nullptr, *w = nullptr, *t = nullptr;
  double2 *partial = nullptr, *hdev = nullptr, *sdev = nullptr, *qdev = nullptr;
  int nchunk = 1;
  // > 0: give up (not converged) when a restart cycle fails to shrink the
  // worst true residual below stall * its value one cycle earlier
  double stall = 0.0;
  // > 0: deflated restarting (GMRES-DR, Morgan 2002) keeping this many
  // harmonic Ritz vectors across restarts; one right-hand side, fixed
  // preconditioner, deflate + 1 <= kRotateMax and deflate + 2 <= m
  int deflate = 0;
  PinnedBuf pin;
  // upload staging of gram_step (coefficients, then the scale at slot m + 2):
  // pinned and owned here, so the step need not wait for its copies
  PinnedBuf pin_up;
  std::vector<cd> H, sn, g;
  std::vector<cd> G;  // Gram matrix of the current basis (single right-hand side)
  std::vector<double> cs;
  heom_status init(WsArena &ws, int64_t n, int R, int m, bool flexible);
  heom_status norms(const T2 *v, std::vector<double> &out, hipStream_t s);
  // x: initial guess (ignored when x_is_zero; then x must hold zeros)
  heom_status solve(const T2 *b, T2 *x, double tol, int max_iter, bool x_is_zero, GmresStats &st, hipStream_t s);
  // one right-hand side: orthogonalise V_{j+1} against V_0..V_j (CGS2 with
  // the Gram matrix G) and normalise it; h (j + 1 entries) and the norm
  heom_status gram_step(int j, std::vector<cd> &h, double &hnorm, hipStream_t s);
  // deflated restarting (deflated.cpp)
  heom_status solve_dr(const T2 *b, T2 *x, double tol, int max_iter, bool x_is_zero, GmresStats &st, hipStream_t s);
};

// Multi-shift spectra (shifted.cpp): every frequency from one Krylov space.
size_t shifted_bytes(const Hier &h, const heom_solver_opts &o);
heom_status spectrum_shifted(Hier &hs, const double2 *x_ss, int kind, const double *op, const double *omega,
                             int64_t n_omega, double *out_host, const heom_solver_opts &o, heom_solver_report *r,
                             void *ws, size_t ws_bytes, hipStream_t s);

}  // namespace heom
