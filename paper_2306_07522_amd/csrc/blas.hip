// Vector kernels for the solvers: multi-dot products (Arnoldi / CGS2),
// basis updates, scaling, the Jacobi preconditioner, the RK4 combine, the
// spectrum right-hand side and its trace readout.
//
// Vectors use the multi-RHS layout [n][R] (element-major, RHS innermost),
// n = N d^2 complex elements per right-hand side.  Reductions accumulate in
// double and are deterministic (fixed two-pass order, no atomics).
#include "blas.h"
#include "device_common.h"
#include "wave_dot.h"

namespace heom {

template <typename T> struct Acc2 { double x, y; };

// --------------------------------------------------------------- multi-dot
// partial[(i * nchunk + chunk) * R + r] = sum over the chunk's elements of
// conj(V_i[e, r]) * w[e, r] for NI consecutive basis vectors i.
template <typename T, int NI>
__global__ void __launch_bounds__(256) mdot_kernel(const typename Cplx<T>::t *__restrict__ V, int64_t ldv, int k,
                                                   const typename Cplx<T>::t *__restrict__ w, int64_t n, int R,
                                                   double2 *__restrict__ partial, int nchunk) {
  using T2 = typename Cplx<T>::t;
  __shared__ double2 red[NI][256];
  const int i0 = blockIdx.y * NI;
  const int chunk = blockIdx.x;
  // thread -> (row slot, rhs); rows of the chunk are strided by rows_per_pass
  const int rt = R < 256 ? R : 256;
  const int rows_per_pass = 256 / rt;
  const int tr = threadIdx.x % rt, trow = threadIdx.x / rt;
  const int64_t e0 = n * chunk / nchunk, e1 = n * (chunk + 1) / nchunk;
  for (int rbase = 0; rbase < R; rbase += rt) {
    const int r = rbase + tr;
    double ax[NI], ay[NI];
#pragma unroll
    for (int q = 0; q < NI; ++q) ax[q] = ay[q] = 0.0;
    if (trow < rows_per_pass && r < R) {
      const bool full = i0 + NI <= k;  // whole groups load together, unguarded
      for (int64_t e = e0 + trow; e < e1; e += rows_per_pass) {
        const T2 b = w[e * R + r];
        T2 a[NI];
        if (full) {
#pragma unroll
          for (int q = 0; q < NI; ++q) a[q] = load_stream<T>(&V[(i0 + q) * ldv + e * R + r]);
        } else {
#pragma unroll
          for (int q = 0; q < NI; ++q) a[q] = i0 + q < k ? V[(i0 + q) * ldv + e * R + r] : T2{0, 0};
        }
#pragma unroll
        for (int q = 0; q < NI; ++q) {
          ax[q] += (double)a[q].x * b.x + (double)a[q].y * b.y;
          ay[q] += (double)a[q].x * b.y - (double)a[q].y * b.x;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NI; ++q) red[q][threadIdx.x] = make_double2(ax[q], ay[q]);
    __syncthreads();
    // reduce over the row slots that share the same r
    if (threadIdx.x < rt) {
#pragma unroll
      for (int q = 0; q < NI; ++q) {
        double sx = 0, sy = 0;
        for (int t = 0; t < rows_per_pass; ++t) {
          sx += red[q][t * rt + threadIdx.x].x;
          sy += red[q][t * rt + threadIdx.x].y;
        }
        const int rr = rbase + threadIdx.x;
        if (i0 + q < k && rr < R) partial[((int64_t)(i0 + q) * nchunk + chunk) * R + rr] = make_double2(sx, sy);
      }
    }
    __syncthreads();
  }
}

// Single right-hand side, two vectors in one pass over the basis:
// partial[i] = conj(V_i) . w, partial[k + i] = conj(V_i) . u (i < k) and
// partial[2k] = w . w (chunk-wise, layout [slot][chunk]).
template <typename T, int NI>
__global__ void __launch_bounds__(256) mdot2_kernel(const typename Cplx<T>::t *__restrict__ V, int64_t ldv, int k,
                                                    const typename Cplx<T>::t *__restrict__ w,
                                                    const typename Cplx<T>::t *__restrict__ u, int64_t n,
                                                    double2 *__restrict__ partial, int nchunk) {
  using T2 = typename Cplx<T>::t;
  __shared__ double2 red[2 * NI + 1][256];
  const int i0 = blockIdx.y * NI;
  const int chunk = blockIdx.x;
  const int64_t e0 = n * chunk / nchunk, e1 = n * (chunk + 1) / nchunk;
  double ax[NI], ay[NI], cx[NI], cy[NI], ww = 0.0;
#pragma unroll
  for (int q = 0; q < NI; ++q) ax[q] = ay[q] = cx[q] = cy[q] = 0.0;
  const bool full = i0 + NI <= k;  // whole groups load together, unguarded
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const T2 bw = w[e], bu = u[e];
    if (blockIdx.y == 0) ww += (double)bw.x * bw.x + (double)bw.y * bw.y;
    T2 a[NI];
    if (full) {
#pragma unroll
      for (int q = 0; q < NI; ++q) a[q] = load_stream<T>(&V[(i0 + q) * ldv + e]);
    } else {
#pragma unroll
      for (int q = 0; q < NI; ++q) a[q] = i0 + q < k ? V[(i0 + q) * ldv + e] : T2{0, 0};
    }
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      ax[q] += (double)a[q].x * bw.x + (double)a[q].y * bw.y;
      ay[q] += (double)a[q].x * bw.y - (double)a[q].y * bw.x;
      cx[q] += (double)a[q].x * bu.x + (double)a[q].y * bu.y;
      cy[q] += (double)a[q].x * bu.y - (double)a[q].y * bu.x;
    }
  }
#pragma unroll
  for (int q = 0; q < NI; ++q) {
    red[q][threadIdx.x] = make_double2(ax[q], ay[q]);
    red[NI + q][threadIdx.x] = make_double2(cx[q], cy[q]);
  }
  red[2 * NI][threadIdx.x] = make_double2(ww, 0.0);
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
#pragma unroll
      for (int q = 0; q < 2 * NI + 1; ++q) {
        red[q][threadIdx.x].x += red[q][threadIdx.x + st].x;
        red[q][threadIdx.x].y += red[q][threadIdx.x + st].y;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < NI && i0 + (int)threadIdx.x < k) {
    partial[(int64_t)(i0 + threadIdx.x) * nchunk + chunk] = red[threadIdx.x][0];
    partial[(int64_t)(k + i0 + threadIdx.x) * nchunk + chunk] = red[NI + threadIdx.x][0];
  }
  if (blockIdx.y == 0 && threadIdx.x == 0) partial[(int64_t)(2 * k) * nchunk + chunk] = red[2 * NI][0];
}

// The same two-vector multi-dot for k <= kWaveDotMaxK, reading w and u once
// whatever k is (wave_dot.h); one workgroup per chunk.
template <typename T, int P>
__global__ void __launch_bounds__(256) mdot2_wave_kernel(const typename Cplx<T>::t *__restrict__ V, int64_t ldv,
                                                         int k, const typename Cplx<T>::t *__restrict__ w,
                                                         const typename Cplx<T>::t *__restrict__ u, int64_t n,
                                                         double2 *__restrict__ partial, int nchunk) {
  __shared__ WaveDotShared sh;
  const int chunk = blockIdx.x;
  const int64_t e0 = n * chunk / nchunk, e1 = n * (chunk + 1) / nchunk;
  wave_mdot2_chunk<T, P>(sh, V, ldv, k, w, u, e0, e1, true, partial, nchunk, chunk);
}

// out[i * R + r] = sum over chunks of partial: one workgroup per output,
// each thread sums a fixed strided subset of the chunks, then a fixed-order
// tree in LDS (deterministic)
__global__ void __launch_bounds__(256) reduce_partials_kernel(const double2 *__restrict__ partial, int k, int nchunk,
                                                              int R, double2 *__restrict__ out) {
  __shared__ double sx[256], sy[256];
  const int64_t idx = blockIdx.x;
  const int t = threadIdx.x;
  const int i = (int)(idx / R), r = (int)(idx % R);
  double ax = 0.0, ay = 0.0;
  for (int c = t; c < nchunk; c += 256) {
    const double2 p = partial[((int64_t)i * nchunk + c) * R + r];
    ax += p.x;
    ay += p.y;
  }
  sx[t] = ax;
  sy[t] = ay;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      sx[t] += sx[t + h];
      sy[t] += sy[t + h];
    }
    __syncthreads();
  }
  if (t == 0) out[idx] = make_double2(sx[0], sy[0]);
}

// w[e, r] -= sum_{i < k} V_i[e, r] * h[i * R + r]   (h is complex double)
template <typename T>
__global__ void __launch_bounds__(256) basis_update_kernel(const typename Cplx<T>::t *__restrict__ V, int64_t ldv, int k,
                                                           const double2 *__restrict__ h, typename Cplx<T>::t *__restrict__ w,
                                                           int64_t n, int R, double sign,
                                                           const double2 *__restrict__ post) {
  using T2 = typename Cplx<T>::t;
  const int64_t total = n * R;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx % R);
    double sx = 0, sy = 0;
    for (int i = 0; i < k; ++i) {
      const T2 a = load_stream<T>(&V[i * ldv + idx]);
      const double2 c = h[(int64_t)i * R + r];
      sx += (double)a.x * c.x - (double)a.y * c.y;
      sy += (double)a.x * c.y + (double)a.y * c.x;
    }
    // w is streamed too: read once here, and its new value is next read by
    // the apply's gathers (FP64 GMRES-DR 1.168 -> 1.13 s with streaming
    // access to w)
    const T2 o = load_stream<T>(&w[idx]);
    double ox = (double)o.x + sign * sx, oy = (double)o.y + sign * sy;
    if (post) {  // fused normalisation: real scale per right-hand side
      ox *= post[r].x;
      oy *= post[r].x;
    }
    T *q = reinterpret_cast<T *>(&w[idx]);
    __builtin_nontemporal_store((T)ox, q);
    __builtin_nontemporal_store((T)oy, q + 1);
  }
}

// The same update for one right-hand side and k <= kUpdate1MaxK: the
// coefficients sit in LDS, and each thread issues the loads of U basis
// vectors before it uses them, so several reads per thread are in flight
// (one load and its wait per vector otherwise).  The sum runs over i in
// the same order as the general kernel.
constexpr int kUpdate1MaxK = 1024;
template <typename T, int U>
__global__ void __launch_bounds__(256) basis_update1_kernel(const typename Cplx<T>::t *__restrict__ V, int64_t ldv,
                                                            int k, const double2 *__restrict__ h,
                                                            typename Cplx<T>::t *__restrict__ w, int64_t n,
                                                            double sign, const double2 *__restrict__ post) {
  using T2 = typename Cplx<T>::t;
  __shared__ double2 hs[kUpdate1MaxK];
  for (int i = threadIdx.x; i < k; i += 256) hs[i] = h[i];
  __syncthreads();
  const double scale = post ? post[0].x : 1.0;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
    const T2 o = load_stream<T>(&w[idx]);
    double sx = 0, sy = 0;
    int i = 0;
    for (; i + U <= k; i += U) {
      T2 a[U];
#pragma unroll
      for (int q = 0; q < U; ++q) a[q] = load_stream<T>(&V[(int64_t)(i + q) * ldv + idx]);
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const double2 c = hs[i + q];
        sx += (double)a[q].x * c.x - (double)a[q].y * c.y;
        sy += (double)a[q].x * c.y + (double)a[q].y * c.x;
      }
    }
    for (; i < k; ++i) {
      const T2 a = V[(int64_t)i * ldv + idx];
      const double2 c = hs[i];
      sx += (double)a.x * c.x - (double)a.y * c.y;
      sy += (double)a.x * c.y + (double)a.y * c.x;
    }
    double ox = (double)o.x + sign * sx, oy = (double)o.y + sign * sy;
    if (post) {  // fused normalisation
      ox *= scale;
      oy *= scale;
    }
    T *q = reinterpret_cast<T *>(&w[idx]);
    __builtin_nontemporal_store((T)ox, q);
    __builtin_nontemporal_store((T)oy, q + 1);
  }
}

// V_c <- sum_i V_i Q[i, c] for c < n_out (Q column-major, n_in x n_out,
// n_out <= MAXC <= kRotateMax), in place: each thread reads all n_in entries
// of its element before it writes any, and no other thread touches that
// element.  Optionally, from the same read, X_p += sum_i V_i Y[i + p n_in]
// for p < n_acc (outputs outside V).  MAXC sizes the register accumulators.
template <typename T, int MAXC>
__global__ void __launch_bounds__(256) basis_rotate_kernel(typename Cplx<T>::t *V, int64_t ldv, int n_in,
                                                           const double2 *__restrict__ Q, int n_out,
                                                           const double2 *__restrict__ Y, int n_acc, AccumOut X,
                                                           int64_t n) {
  using T2 = typename Cplx<T>::t;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double ax[MAXC], ay[MAXC], bx[kAccumMax], by[kAccumMax];
#pragma unroll
    for (int c = 0; c < MAXC; ++c) {
      ax[c] = 0.0;
      ay[c] = 0.0;
    }
#pragma unroll
    for (int p = 0; p < kAccumMax; ++p) bx[p] = by[p] = 0.0;
    for (int i = 0; i < n_in; ++i) {
      const T2 v = load_stream<T>(&V[i * ldv + e]);
      const double vx = v.x, vy = v.y;
#pragma unroll
      for (int c = 0; c < MAXC; ++c) {
        if (c < n_out) {
          const double2 q = Q[(int64_t)c * n_in + i];
          ax[c] += vx * q.x - vy * q.y;
          ay[c] += vx * q.y + vy * q.x;
        }
      }
#pragma unroll
      for (int p = 0; p < kAccumMax; ++p) {
        if (p < n_acc) {
          const double2 q = Y[(int64_t)p * n_in + i];
          bx[p] += vx * q.x - vy * q.y;
          by[p] += vx * q.y + vy * q.x;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < MAXC; ++c)
      if (c < n_out) {
        T *q = reinterpret_cast<T *>(&V[c * ldv + e]);
        __builtin_nontemporal_store((T)ax[c], q);
        __builtin_nontemporal_store((T)ay[c], q + 1);
      }
#pragma unroll
    for (int p = 0; p < kAccumMax; ++p)
      if (p < n_acc) {
        T2 *xo = (T2 *)X.p[p];
        T2 o = xo[e];
        o.x = (T)((double)o.x + bx[p]);
        o.y = (T)((double)o.y + by[p]);
        xo[e] = o;
      }
  }
}

// X_p += sum_{i < n_in} V_i Y[i + p * n_in] for p < n_acc <= kAccumMax
// (Y: device, column-major, complex double): several combinations of the
// basis from one read of it.
template <typename T>
__global__ void __launch_bounds__(256) basis_accum_kernel(const typename Cplx<T>::t *__restrict__ V, int64_t ldv,
                                                          int n_in, const double2 *__restrict__ Y, int n_acc,
                                                          AccumOut X, int64_t n) {
  using T2 = typename Cplx<T>::t;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double ax[kAccumMax], ay[kAccumMax];
#pragma unroll
    for (int p = 0; p < kAccumMax; ++p) ax[p] = ay[p] = 0.0;
    for (int i = 0; i < n_in; ++i) {
      const T2 v = load_stream<T>(&V[i * ldv + e]);
      const double vx = v.x, vy = v.y;
#pragma unroll
      for (int p = 0; p < kAccumMax; ++p)
        if (p < n_acc) {
          const double2 q = Y[(int64_t)p * n_in + i];
          ax[p] += vx * q.x - vy * q.y;
          ay[p] += vx * q.y + vy * q.x;
        }
    }
#pragma unroll
    for (int p = 0; p < kAccumMax; ++p)
      if (p < n_acc) {
        T2 *xo = (T2 *)X.p[p];
        T2 o = xo[e];
        o.x = (T)((double)o.x + ax[p]);
        o.y = (T)((double)o.y + ay[p]);
        xo[e] = o;
      }
  }
}

// out[e, r] = w[e, r] * s[r]  (s complex double per RHS); out may alias w
template <typename T>
__global__ void scale_kernel(const typename Cplx<T>::t *__restrict__ w, const double2 *__restrict__ s,
                             typename Cplx<T>::t *out, int64_t n, int R) {
  using T2 = typename Cplx<T>::t;
  const int64_t total = n * R;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const double2 c = s[idx % R];
    const T2 a = w[idx];
    out[idx] = T2{(T)((double)a.x * c.x - (double)a.y * c.y), (T)((double)a.x * c.y + (double)a.y * c.x)};
  }
}

// y = alpha * x + beta * y  (real scalars; x and y of possibly different precision)
template <typename TX, typename TY>
__global__ void axpby_kernel(const typename Cplx<TX>::t *__restrict__ x, double alpha, typename Cplx<TY>::t *y,
                             double beta, int64_t total) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const auto a = x[idx];
    typename Cplx<TY>::t b;
    if (beta == 0.0) {  // y is write-only: it may hold anything, NaN included
      b.x = (TY)(alpha * (double)a.x);
      b.y = (TY)(alpha * (double)a.y);
    } else {
      b = y[idx];
      b.x = (TY)(alpha * (double)a.x + beta * (double)b.x);
      b.y = (TY)(alpha * (double)a.y + beta * (double)b.y);
    }
    y[idx] = b;
  }
}

// Jacobi: z = r / diag(M + shift) where the diagonal of the HEOMLS at
// element (a, i, j) is -(c_a - z_r) - i (H_ii - H_jj); the bordered row
// (ADO 0, element (0,0)) has diagonal 1; exact zeros are replaced by 1.
template <typename T>
__global__ void jacobi_kernel(const typename Cplx<T>::t *__restrict__ r, typename Cplx<T>::t *__restrict__ z,
                              const double2 *__restrict__ decay, const double2 *__restrict__ hdiag, int d, int64_t N,
                              int R, const double2 *__restrict__ shifts, int border, int modulus) {
  using T2 = typename Cplx<T>::t;
  const int64_t total = N * d * d * R;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int rr = (int)(idx % R);
    const int64_t e = idx / R;
    const int64_t a = e / (d * d);
    const int ij = (int)(e % (d * d));
    const int i = ij / d, j = ij % d;
    double2 dg;
    const double2 c = decay[a];
    const double2 zz = shifts ? shifts[rr] : make_double2(0.0, 0.0);
    const double2 hi = hdiag[i], hj = hdiag[j];
    // -(c - z) - i (hi - hj)
    dg.x = -(c.x - zz.x) + (hi.y - hj.y);
    dg.y = -(c.y - zz.y) - (hi.x - hj.x);
    if (border && e == 0) dg = make_double2(1.0, 0.0);
    const double m2 = dg.x * dg.x + dg.y * dg.y;
    if (m2 == 0.0) dg = make_double2(1.0, 0.0);
    else if (modulus) dg = make_double2(sqrt(m2), 0.0);  // |diagonal|: a positive scaling
    const double inv = 1.0 / (dg.x * dg.x + dg.y * dg.y);
    const T2 v = r[idx];
    // v / dg = v * conj(dg) / |dg|^2
    z[idx] = T2{(T)(((double)v.x * dg.x + (double)v.y * dg.y) * inv), (T)(((double)v.y * dg.x - (double)v.x * dg.y) * inv)};
  }
}

// RK4 combine: x += dt/6 (k1 + 2 k2 + 2 k3 + k4)
template <typename T>
__global__ void rk4_combine_kernel(typename Cplx<T>::t *__restrict__ x, const typename Cplx<T>::t *__restrict__ k1,
                                   const typename Cplx<T>::t *__restrict__ k2, const typename Cplx<T>::t *__restrict__ k3,
                                   const typename Cplx<T>::t *__restrict__ k4, T dt6, int64_t total) {
  using T2 = typename Cplx<T>::t;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const T2 a = k1[idx], b = k2[idx], c = k3[idx], e = k4[idx];
    T2 v = x[idx];
    v.x += dt6 * (a.x + 2 * b.x + 2 * c.x + e.x);
    v.y += dt6 * (a.y + 2 * b.y + 2 * c.y + e.y);
    x[idx] = v;
  }
}

// RK4 stage input u = x + c k, with the same fused multiply-add (in T) that
// the apply uses when it forms the stage input while gathering
template <typename T>
__global__ void stage_input_kernel(const typename Cplx<T>::t *__restrict__ x, const typename Cplx<T>::t *__restrict__ k,
                                   T c, typename Cplx<T>::t *__restrict__ u, int64_t total) {
  using T2 = typename Cplx<T>::t;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const T2 q = k[idx];
    T2 v = x[idx];
    v.x = fma(c, q.x, v.x);
    v.y = fma(c, q.y, v.y);
    u[idx] = v;
  }
}

// save ADO 0 into the trajectory slot counter[0] and advance the counter
template <typename T>
__global__ void save_rho0_kernel(const typename Cplx<T>::t *__restrict__ x, typename Cplx<T>::t *__restrict__ traj,
                                 int d2, int *counter, int64_t max_slots) {
  const int slot = *counter;
  if (slot < max_slots)
    for (int t = threadIdx.x; t < d2; t += blockDim.x) traj[(int64_t)slot * d2 + t] = x[t];
  __syncthreads();
  if (threadIdx.x == 0) *counter = slot + 1;
}

__global__ void add_unit_kernel(double2 *v) {
  if (threadIdx.x == 0) v[0].x += 1.0;
}

heom_status add_unit(void *v, hipStream_t s) {
  hipLaunchKernelGGL(add_unit_kernel, dim3(1), dim3(64), 0, s, (double2 *)v);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

__global__ void fill_int_kernel(int *p, int v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// b[(a, i, j), r] = (O_{sel(r)} x_a)[i][j]: left-multiply every ADO of the
// FP64 single-RHS vector x by one of two d x d operators (column r uses
// op[col_op[r]]).
template <typename T>
__global__ void left_multiply_kernel(const double2 *__restrict__ x, const double2 *__restrict__ ops, int d, int64_t N,
                                     int R, const int *__restrict__ col_op, typename Cplx<T>::t *__restrict__ b) {
  using T2 = typename Cplx<T>::t;
  const int64_t total = N * d * d * R;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx % R);
    const int64_t e = idx / R;
    const int64_t a = e / (d * d);
    const int ij = (int)(e % (d * d));
    const int i = ij / d, j = ij % d;
    const double2 *O = ops + (int64_t)col_op[r] * d * d;
    double sx = 0, sy = 0;
    for (int k = 0; k < d; ++k) {
      const double2 o = O[i * d + k];
      const double2 v = x[(a * d + k) * d + j];
      sx += o.x * v.x - o.y * v.y;
      sy += o.x * v.y + o.y * v.x;
    }
    b[idx] = T2{(T)sx, (T)sy};
  }
}

// out[r] = scale * Re Tr[O_{sel(r)} x_0^{(r)}]
template <typename T>
__global__ void trace_readout_kernel(const typename Cplx<T>::t *__restrict__ x, const double2 *__restrict__ ops, int d,
                                     int R, const int *__restrict__ col_op, double scale, double *__restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const double2 *O = ops + (int64_t)col_op[r] * d * d;
  double s = 0;
  for (int i = 0; i < d; ++i)
    for (int k = 0; k < d; ++k) {
      const double2 o = O[i * d + k];
      const auto v = x[((int64_t)k * d + i) * R + r];
      s += o.x * (double)v.x - o.y * (double)v.y;
    }
  out[r] = scale * s;
}

// --------------------------------------------------------------- launchers
static inline unsigned grid_for(int64_t total) {
  int64_t g = (total + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

template <typename T>
heom_status mdot(const void *V, int64_t ldv, int k, const void *w, int64_t n, int R, double2 *partial, int nchunk,
                 double2 *out, hipStream_t s) {
  if (k <= 0) return HEOM_OK;
  constexpr int NI = 4;
  dim3 g(nchunk, (k + NI - 1) / NI);
  hipLaunchKernelGGL((mdot_kernel<T, NI>), g, dim3(256), 0, s, (const typename Cplx<T>::t *)V, ldv, k,
                     (const typename Cplx<T>::t *)w, n, R, partial, nchunk);
  const int64_t kr = (int64_t)k * R;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)kr), dim3(256), 0, s, partial, k, nchunk, R, out);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename T>
heom_status mdot2(const void *V, int64_t ldv, int k, const void *w, const void *u, int64_t n, double2 *partial,
                  int nchunk, double2 *out, hipStream_t s) {
  if (k <= 0) return HEOM_OK;
  if (k <= kWaveDotMaxK) {
    hipLaunchKernelGGL((mdot2_wave_kernel<T, 4>), dim3(nchunk), dim3(256), 0, s, (const typename Cplx<T>::t *)V, ldv,
                       k, (const typename Cplx<T>::t *)w, (const typename Cplx<T>::t *)u, n, partial, nchunk);
  } else {
    constexpr int NI = 4;
    dim3 g(nchunk, (k + NI - 1) / NI);
    hipLaunchKernelGGL((mdot2_kernel<T, NI>), g, dim3(256), 0, s, (const typename Cplx<T>::t *)V, ldv, k,
                       (const typename Cplx<T>::t *)w, (const typename Cplx<T>::t *)u, n, partial, nchunk);
  }
  const int64_t kk = 2 * (int64_t)k + 1;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)kk), dim3(256), 0, s, partial, (int)kk, nchunk, 1, out);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename T>
heom_status basis_update(const void *V, int64_t ldv, int k, const double2 *h, void *w, int64_t n, int R, double sign,
                         hipStream_t s, const double2 *post) {
  if (k <= 0 && !post) return HEOM_OK;
  // FP32 gains from four reads in flight per thread; FP64 (twice the bytes
  // per element) keeps the general kernel, which measured faster there
  // (two-orbital tier-4 GMRES-DR: 1.243 s, against 1.273 s with one, two or
  // four reads in flight from this kernel)
  constexpr int U = std::is_same<T, double>::value ? 0 : 4;
  if (R == 1 && k <= kUpdate1MaxK && U > 0)
    hipLaunchKernelGGL((basis_update1_kernel<T, (U > 0 ? U : 1)>), dim3(grid_for(n)), dim3(256), 0, s,
                       (const typename Cplx<T>::t *)V, ldv, k, h, (typename Cplx<T>::t *)w, n, sign, post);
  else
    hipLaunchKernelGGL(basis_update_kernel<T>, dim3(grid_for(n * R)), dim3(256), 0, s, (const typename Cplx<T>::t *)V,
                       ldv, k, h, (typename Cplx<T>::t *)w, n, R, sign, post);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename T>
heom_status basis_rotate(void *V, int64_t ldv, int n_in, const double2 *Q, int n_out, int64_t n, hipStream_t s,
                         const double2 *Y, int n_acc, const AccumOut *X) {
  if (n_out < 1 || n_out > kRotateMax || n_in < n_out) return fail(HEOM_ERR_ARG, "basis_rotate: bad column counts");
  if (n_acc < 0 || n_acc > kAccumMax || (n_acc > 0 && (!Y || !X))) return fail(HEOM_ERR_ARG, "basis_rotate: bad outputs");
  AccumOut xo{};
  for (int p = 0; p < n_acc; ++p) {
    if (!X->p[p]) return fail(HEOM_ERR_ARG, "basis_rotate: NULL output");
    xo.p[p] = X->p[p];
  }
  if (n_out <= 8)
    hipLaunchKernelGGL((basis_rotate_kernel<T, 8>), dim3(grid_for(n)), dim3(256), 0, s, (typename Cplx<T>::t *)V, ldv,
                       n_in, Q, n_out, Y, n_acc, xo, n);
  else
    hipLaunchKernelGGL((basis_rotate_kernel<T, kRotateMax>), dim3(grid_for(n)), dim3(256), 0, s,
                       (typename Cplx<T>::t *)V, ldv, n_in, Q, n_out, Y, n_acc, xo, n);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename T>
heom_status basis_accum(const void *V, int64_t ldv, int n_in, const double2 *Y, int n_acc, const AccumOut &X, int64_t n,
                        hipStream_t s) {
  if (n_acc < 1 || n_acc > kAccumMax || n_in < 1) return fail(HEOM_ERR_ARG, "basis_accum: bad column counts");
  for (int p = 0; p < n_acc; ++p)
    if (!X.p[p]) return fail(HEOM_ERR_ARG, "basis_accum: NULL output");
  hipLaunchKernelGGL(basis_accum_kernel<T>, dim3(grid_for(n)), dim3(256), 0, s, (const typename Cplx<T>::t *)V, ldv,
                     n_in, Y, n_acc, X, n);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename T>
heom_status scale_vec(const void *w, const double2 *sc, void *out, int64_t n, int R, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel<T>, dim3(grid_for(n * R)), dim3(256), 0, s, (const typename Cplx<T>::t *)w, sc,
                     (typename Cplx<T>::t *)out, n, R);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename TX, typename TY>
heom_status axpby(const void *x, double alpha, void *y, double beta, int64_t total, hipStream_t s) {
  hipLaunchKernelGGL((axpby_kernel<TX, TY>), dim3(grid_for(total)), dim3(256), 0, s, (const typename Cplx<TX>::t *)x,
                     alpha, (typename Cplx<TY>::t *)y, beta, total);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename T>
heom_status jacobi(const void *r, void *z, const Hier &h, int R, const double2 *shifts, int border, hipStream_t s,
                   int modulus) {
  hipLaunchKernelGGL(jacobi_kernel<T>, dim3(grid_for(h.N * h.d * h.d * R)), dim3(256), 0, s,
                     (const typename Cplx<T>::t *)r, (typename Cplx<T>::t *)z, h.dev.decay64, h.dev.hdiag, h.d, h.N, R,
                     shifts, border, modulus);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename T>
heom_status stage_input(const void *x, const void *k, double c, void *u, int64_t total, hipStream_t s) {
  hipLaunchKernelGGL(stage_input_kernel<T>, dim3(grid_for(total)), dim3(256), 0, s, (const typename Cplx<T>::t *)x,
                     (const typename Cplx<T>::t *)k, (T)c, (typename Cplx<T>::t *)u, total);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename T>
heom_status rk4_combine(void *x, const void *k1, const void *k2, const void *k3, const void *k4, double dt, int64_t total,
                        hipStream_t s) {
  using T2 = typename Cplx<T>::t;
  hipLaunchKernelGGL(rk4_combine_kernel<T>, dim3(grid_for(total)), dim3(256), 0, s, (T2 *)x, (const T2 *)k1,
                     (const T2 *)k2, (const T2 *)k3, (const T2 *)k4, (T)(dt / 6.0), total);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename T>
heom_status save_rho0(const void *x, void *traj, int d2, int *counter, int64_t max_slots, hipStream_t s) {
  hipLaunchKernelGGL(save_rho0_kernel<T>, dim3(1), dim3(256), 0, s, (const typename Cplx<T>::t *)x,
                     (typename Cplx<T>::t *)traj, d2, counter, max_slots);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

heom_status fill_int(int *p, int v, int n, hipStream_t s) {
  hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename T>
heom_status left_multiply(const double2 *x, const double2 *ops, int d, int64_t N, int R, const int *col_op, void *b,
                          hipStream_t s) {
  hipLaunchKernelGGL(left_multiply_kernel<T>, dim3(grid_for(N * d * d * R)), dim3(256), 0, s, x, ops, d, N, R, col_op,
                     (typename Cplx<T>::t *)b);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename T>
heom_status trace_readout(const void *x, const double2 *ops, int d, int R, const int *col_op, double scale, double *out,
                          hipStream_t s) {
  hipLaunchKernelGGL(trace_readout_kernel<T>, dim3((R + 63) / 64), dim3(64), 0, s, (const typename Cplx<T>::t *)x, ops, d,
                     R, col_op, scale, out);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

#define HEOM_INST(T)                                                                                              \
  template heom_status mdot<T>(const void *, int64_t, int, const void *, int64_t, int, double2 *, int, double2 *, \
                               hipStream_t);                                                                       \
  template heom_status mdot2<T>(const void *, int64_t, int, const void *, const void *, int64_t, double2 *, int,     \
                                double2 *, hipStream_t);                                                          \
  template heom_status basis_update<T>(const void *, int64_t, int, const double2 *, void *, int64_t, int, double,  \
                                       hipStream_t, const double2 *);                                              \
  template heom_status scale_vec<T>(const void *, const double2 *, void *, int64_t, int, hipStream_t);             \
  template heom_status basis_rotate<T>(void *, int64_t, int, const double2 *, int, int64_t, hipStream_t,             \
                                       const double2 *, int, const AccumOut *);                                    \
  template heom_status basis_accum<T>(const void *, int64_t, int, const double2 *, int, const AccumOut &, int64_t,  \
                                      hipStream_t);                                                               \
  template heom_status jacobi<T>(const void *, void *, const Hier &, int, const double2 *, int, hipStream_t, int);  \
  template heom_status rk4_combine<T>(void *, const void *, const void *, const void *, const void *, double,      \
                                      int64_t, hipStream_t);                                                       \
  template heom_status save_rho0<T>(const void *, void *, int, int *, int64_t, hipStream_t);                       \
  template heom_status stage_input<T>(const void *, const void *, double, void *, int64_t, hipStream_t);           \
  template heom_status left_multiply<T>(const double2 *, const double2 *, int, int64_t, int, const int *, void *, \
                                        hipStream_t);                                                              \
  template heom_status trace_readout<T>(const void *, const double2 *, int, int, const int *, double, double *,    \
                                        hipStream_t);
HEOM_INST(double)
HEOM_INST(float)
template heom_status axpby<double, double>(const void *, double, void *, double, int64_t, hipStream_t);
template heom_status axpby<float, float>(const void *, double, void *, double, int64_t, hipStream_t);
template heom_status axpby<double, float>(const void *, double, void *, double, int64_t, hipStream_t);
template heom_status axpby<float, double>(const void *, double, void *, double, int64_t, hipStream_t);

}  // namespace heom
