// Vector-kernel launchers used by the solvers (blas.hip).
#pragma once

#include "internal.h"

namespace heom {

// Number of chunks of the multi-dot partial sums for n elements and R
// right-hand sides (one right-hand side: about 1,024 elements per chunk, at
// most 8,192 chunks, so that the one-workgroup-per-chunk kernel has many
// workgroups per compute unit)
inline int dot_chunks(int64_t n, int R) {
  int64_t c = R == 1 ? n / 1024 : (n * R) / (256 * 64);
  if (c < 1) c = 1;
  const int64_t cap = R == 1 ? 8192 : 1024;
  if (c > cap) c = cap;
  return (int)c;
}
// out[i * R + r] = conj(V_i) . w per right-hand side (partial: k * nchunk * R scratch)
template <typename T>
heom_status mdot(const void *V, int64_t ldv, int k, const void *w, int64_t n, int R, double2 *partial, int nchunk,
                 double2 *out, hipStream_t s);
// One right-hand side: out[i] = conj(V_i) . w, out[k + i] = conj(V_i) . u
// (i < k) and out[2k] = w . w, in one pass over the basis
// (partial: (2k + 1) * nchunk scratch)
template <typename T>
heom_status mdot2(const void *V, int64_t ldv, int k, const void *w, const void *u, int64_t n, double2 *partial,
                  int nchunk, double2 *out, hipStream_t s);
// w += sign * sum_i V_i h_i (per right-hand side), then w *= post[r].x when
// post is given (fused normalisation)
template <typename T>
heom_status basis_update(const void *V, int64_t ldv, int k, const double2 *h, void *w, int64_t n, int R, double sign,
                         hipStream_t s, const double2 *post = nullptr);
// X.p[p] += sum_{i < n_in} V_i Y[i + p * n_in] for p < n_acc <= kAccumMax
// (Y: device, column-major, complex double), one read of the basis
constexpr int kAccumMax = 4;
struct AccumOut {
  void *p[kAccumMax];
};
template <typename T>
heom_status basis_accum(const void *V, int64_t ldv, int n_in, const double2 *Y, int n_acc, const AccumOut &X, int64_t n,
                        hipStream_t s);
// In-place change of basis: V_c <- sum_{i < n_in} V_i Q[i + c * n_in] for
// c < n_out <= kRotateMax (Q: device, column-major, complex double); with
// n_acc > 0 also X->p[p] += sum_i V_i Y[i + p * n_in] (p < n_acc) from the
// same read of the basis
constexpr int kRotateMax = 32;
template <typename T>
heom_status basis_rotate(void *V, int64_t ldv, int n_in, const double2 *Q, int n_out, int64_t n, hipStream_t s,
                         const double2 *Y = nullptr, int n_acc = 0, const AccumOut *X = nullptr);
template <typename T>
heom_status scale_vec(const void *w, const double2 *sc, void *out, int64_t n, int R, hipStream_t s);
template <typename TX, typename TY>
heom_status axpby(const void *x, double alpha, void *y, double beta, int64_t total, hipStream_t s);
// z = D^{-1} r with D the diagonal of (M + shift) (bordered: element (0,0) of
// ADO 0 counts 1; zeros count 1); modulus = 1 divides by |D| instead
// Block preconditioner (block_prec.hip): per ADO and right-hand side the
// exact inverse of -(c_a - z) - i[H, .] in the eigenbasis of H; d <= 32
template <typename T>
heom_status block_prec(const void *r, void *z, const Hier &h, int R, const double2 *shifts, hipStream_t s);
template <typename T>
heom_status jacobi(const void *r, void *z, const Hier &h, int R, const double2 *shifts, int border, hipStream_t s,
                   int modulus = 0);
// u = x + c k (RK4 stage input, formed once before the apply)
template <typename T>
heom_status stage_input(const void *x, const void *k, double c, void *u, int64_t total, hipStream_t s);
template <typename T>
heom_status rk4_combine(void *x, const void *k1, const void *k2, const void *k3, const void *k4, double dt,
                        int64_t total, hipStream_t s);
template <typename T>
heom_status save_rho0(const void *x, void *traj, int d2, int *counter, int64_t max_slots, hipStream_t s);
heom_status fill_int(int *p, int v, int n, hipStream_t s);
// v[0] += 1 (FP64 complex vector)
heom_status add_unit(void *v, hipStream_t s);
template <typename T>
heom_status left_multiply(const double2 *x, const double2 *ops, int d, int64_t N, int R, const int *col_op, void *b,
                          hipStream_t s);
template <typename T>
heom_status trace_readout(const void *x, const double2 *ops, int d, int R, const int *col_op, double scale,
                          double *out, hipStream_t s);

}  // namespace heom
