// Batched instances: many independent hierarchies -- each with its own d,
// exponents, tiers, Hamiltonian and baths -- advanced by single launches.
//
// The batch vector is the concatenation of the instance vectors ([N_s][d_s][d_s]
// complex each, instance order).  Three device tables drive every kernel:
//   instances  one descriptor per instance (its apply tables, d, offset);
//   tiles      (instance, first task, end task): the tasks of one instance
//              that one 256-thread block computes, one thread per output
//              element (256 / d^2 ADOs per tile);
//   chunks     contiguous element ranges that never straddle two instances,
//              the unit of the segmented reductions of the batched GMRES.
// The apply is one launch that walks the tile list (one workgroup per tile,
// or a persistent grid); the preconditioners walk the same list.  Per-instance GMRES scalars (the
// Arnoldi coefficients, Givens rotations, residual norms) come from
// segmented reductions; an Arnoldi step's device work can be captured once
// per basis size into a hipGraph and replayed.  An autotuner picks the
// launch shape (tile size, kernel variant, grid, tile order, matrix-core H
// terms) by timing the batched apply.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <numeric>
#include <string>
#include <thread>

#include "apply_wave.h"
#include "blas.h"
#include "device_common.h"
#include "internal.h"
#include "tile_product.h"
#include "solvers.h"

namespace heom {

template <typename T>
struct BInst {
  using T2 = typename Cplx<T>::t;
  const int4 *tasks;
  const int4 *groups;
  const int2 *gedges;
  const int32_t *coef_op;
  const T2 *coef;
  const int32_t *ell_cnt;
  const int32_t *ell_col;
  const T2 *ell_val;
  const T2 *decay;
  const double2 *decay64;
  const double2 *hdiag64;
  const double2 *ueig;  // [d][d] eigenvectors of H, row-major (block preconditioner)
  const double *eval;   // [d] eigenvalues of H
  double delta;         // block preconditioner regularisation
  int64_t off;  // first element of the instance in the batch vector
  int slots;
  int d;
  int wave;     // 1: d in {8, 16}, computed by the wave formulation (one wavefront per ADO)
};

// ----------------------------------------------------------------- apply
// y = B x per instance (B = M, or the bordered stationary-state operator when
// border is set: element (0,0) of ADO 0 becomes Tr rho_0).  Tiles of
// instances with d in {8, 16} hold four tasks, one per wavefront, computed by
// the wave formulation with the instance's operator tables staged in LDS;
// other tiles hold 256 / d^2 tasks, one thread per output element.
template <typename T>
__device__ __forceinline__ void batch_cell_tile(const BInst<T> &I, const int4 &tl, const typename Cplx<T>::t *x,
                                                typename Cplx<T>::t *y, int border) {
  using T2 = typename Cplx<T>::t;
  const int d = I.d, cells = d * d;
  const int tpb = cells <= 256 ? 256 / cells : 1;
  const int lt = threadIdx.x / cells;
  if (lt >= tpb) return;
  const int cell = threadIdx.x - lt * cells;
  const int i = cell / d, j = cell - (cell / d) * d;
  const T2 *xs = x + I.off;
  auto in = [&](int64_t b, int ii, int jj) -> T2 { return xs[(b * d + ii) * d + jj]; };
  for (int64_t task = (int64_t)tl.y + lt; task < tl.z; task += tpb) {
    const int4 tk = I.tasks[task];
    const int64_t a = tk.x;
    T2 acc{0, 0};
    for (int g = tk.y; g < tk.z; ++g) {
      const int4 gr = I.groups[g];
      const int op = I.coef_op[gr.z];
      const size_t rowL = ((size_t)op * 2) * d + i;
      const size_t rowR = ((size_t)op * 2 + 1) * d + j;
      const int nl = I.ell_cnt[rowL], nr = I.ell_cnt[rowR];
      T2 L{0, 0}, Rv{0, 0};
      for (int e = gr.x; e < gr.y; ++e) {
        const int2 ed = I.gedges[e];
        const T w = (T)ed.y;
        T2 l{0, 0}, rr{0, 0};
        for (int q = 0; q < nl; ++q)
          l = cfma(I.ell_val[rowL * I.slots + q], in(ed.x, I.ell_col[rowL * I.slots + q], j), l);
        for (int q = 0; q < nr; ++q)
          rr = cfma(in(ed.x, i, I.ell_col[rowR * I.slots + q]), I.ell_val[rowR * I.slots + q], rr);
        L.x = fma(w, l.x, L.x); L.y = fma(w, l.y, L.y);
        Rv.x = fma(w, rr.x, Rv.x); Rv.y = fma(w, rr.y, Rv.y);
      }
      if (gr.w) acc = csub(acc, cmul(I.decay[a], in(a, i, j)));
      acc = cfma(I.coef[2 * gr.z], L, acc);
      acc = cfma(I.coef[2 * gr.z + 1], Rv, acc);
    }
    if (border && a == 0 && cell == 0) {
      T2 tr{0, 0};
      for (int ii = 0; ii < d; ++ii) tr = cadd(tr, in(0, ii, ii));
      acc = tr;
    }
    y[I.off + (a * d + i) * d + j] = acc;
  }
}

template <typename T, int D, bool MF = false, bool LT = false>
__device__ __forceinline__ void batch_wave_tile(const ApplyParams<T> &Pi, const BInst<T> &I, const int4 &tl,
                                                const typename Cplx<T>::t *x, typename Cplx<T>::t *y, int border,
                                                unsigned char *smem) {
  using T2 = typename Cplx<T>::t;
  constexpr int DD = D * D;
  ApplyParams<T> P = Pi;
  P.x = x + I.off;
  P.y = y + I.off;
  P.border = border;
  // LDS layout from byte offsets (the accesses stay LDS accesses), as in the
  // single-hierarchy wave kernel; with LT also the packed operator metadata
  // and the coefficients
  T2 *sbuf = reinterpret_cast<T2 *>(smem);
  T2 *tval = sbuf + 4 * DD;
  int *tcol = reinterpret_cast<int *>(tval + P.n_centries);
  const size_t o_thd = (4 * DD * sizeof(T2) + (size_t)P.n_centries * (sizeof(T2) + sizeof(int)) + 15) & ~(size_t)15;
  T2 *thd = reinterpret_cast<T2 *>(smem + o_thd);
  int *cmeta = reinterpret_cast<int *>(thd + D);
  const size_t o_cfs = (o_thd + D * sizeof(T2) + (size_t)P.n_coef * sizeof(int) + 15) & ~(size_t)15;
  T2 *cfs = reinterpret_cast<T2 *>(smem + o_cfs);
  __syncthreads();  // the previous tile is done with the tables
  for (int e = threadIdx.x; e < P.n_centries; e += 256) {
    tval[e] = P.c_val[e];
    tcol[e] = P.c_col[e];
  }
  if (threadIdx.x < D) thd[threadIdx.x] = P.hdiag[threadIdx.x];
  if constexpr (LT) {
    for (int e = threadIdx.x; e < P.n_coef; e += 256) {
      const int op = P.coef_op[e];
      cmeta[e] = P.c_meta[3 * op] | (P.c_meta[3 * op + 1] << 20) | ((P.c_meta[3 * op + 2] ? 1 : 0) << 30);
      cfs[2 * e] = P.coef[2 * e];
      cfs[2 * e + 1] = P.coef[2 * e + 1];
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int64_t task = (int64_t)tl.y + wave; task < tl.z; task += 4)
    wave_task<T, D, false, true, MF, false, LT>(P, task, lane, sbuf + wave * DD, tval, tcol, thd, cmeta, cfs);
}

// MF16: the d = 16 wave instances compute their own block's H terms on the
// matrix cores (a separate instantiation, so that the other keeps its
// register budget).
template <typename T, bool MF16, bool LT>
__global__ void __launch_bounds__(256) batch_apply_kernel(const BInst<T> *__restrict__ inst,
                                                          const ApplyParams<T> *__restrict__ prm,
                                                          const int4 *__restrict__ tiles, int n_tiles,
                                                          const int *__restrict__ active,
                                                          const typename Cplx<T>::t *__restrict__ x,
                                                          typename Cplx<T>::t *__restrict__ y, int border) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const int4 tl = tiles[t];
    if (active && !active[tl.x]) continue;
    const BInst<T> &I = inst[tl.x];
    if (I.wave && I.d == 16) batch_wave_tile<T, 16, MF16, LT>(prm[tl.x], I, tl, x, y, border, smem);
    else if (I.wave && I.d == 8) batch_wave_tile<T, 8, false, LT>(prm[tl.x], I, tl, x, y, border, smem);
    else batch_cell_tile<T>(I, tl, x, y, border);
  }
}

// z = D^{-1} r per instance, D the diagonal of B (zeros count as 1).
template <typename T>
__global__ void __launch_bounds__(256) batch_jacobi_kernel(const BInst<T> *__restrict__ inst,
                                                           const int4 *__restrict__ tiles, int n_tiles,
                                                           const int *__restrict__ active,
                                                           const typename Cplx<T>::t *__restrict__ r,
                                                           typename Cplx<T>::t *__restrict__ z, int border) {
  using T2 = typename Cplx<T>::t;
  for (int t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const int4 tl = tiles[t];
    if (active && !active[tl.x]) continue;
    const BInst<T> &I = inst[tl.x];
    const int d = I.d, cells = d * d;
    const int tpb = cells <= 256 ? 256 / cells : 1;
    const int lt = threadIdx.x / cells;
    if (lt >= tpb) continue;
    const int cell = threadIdx.x - lt * cells;
    const int i = cell / d, j = cell - (cell / d) * d;
    for (int64_t task = (int64_t)tl.y + lt; task < tl.z; task += tpb) {
      const int64_t a = I.tasks[task].x;
      const double2 c = I.decay64[a], hi = I.hdiag64[i], hj = I.hdiag64[j];
      double2 dg = make_double2(-c.x + (hi.y - hj.y), -c.y - (hi.x - hj.x));
      if (border && a == 0 && cell == 0) dg = make_double2(1.0, 0.0);
      if (dg.x * dg.x + dg.y * dg.y == 0.0) dg = make_double2(1.0, 0.0);
      const double inv = 1.0 / (dg.x * dg.x + dg.y * dg.y);
      const int64_t idx = I.off + a * cells + cell;
      const T2 v = r[idx];
      z[idx] = T2{(T)(((double)v.x * dg.x + (double)v.y * dg.y) * inv), (T)(((double)v.y * dg.x - (double)v.x * dg.y) * inv)};
    }
  }
}

// z = P^{-1} r per instance with the block preconditioner: per ADO the exact
// inverse of -c_a - i[H, .] in the eigenbasis of H (see block_prec.hip), four
// d x d products through LDS (d <= 16), one task per wave at a time.
template <typename T>
__global__ void __launch_bounds__(256) batch_block_kernel(const BInst<T> *__restrict__ inst,
                                                          const int4 *__restrict__ tiles, int n_tiles,
                                                          const int *__restrict__ active,
                                                          const typename Cplx<T>::t *__restrict__ r,
                                                          typename Cplx<T>::t *__restrict__ z) {
  // the eigenbasis U of the tile's instance is shared; each wave takes every
  // fourth task of the tile with its own X and W and 2 x 2 product tiles
  // (d <= 16: at most 64 tiles, one per lane)
  using T2 = typename Cplx<T>::t;
  __shared__ double2 Us[256], Xs[4][256], Ws[4][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double2 *X = Xs[wave], *W = Ws[wave];
  for (int t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const int4 tl = tiles[t];
    if (active && !active[tl.x]) continue;  // uniform over the workgroup
    const BInst<T> &I = inst[tl.x];
    const int d = I.d, dd = d * d;
    __syncthreads();  // every wave is done with the previous tile's U
    for (int e = threadIdx.x; e < dd; e += blockDim.x) Us[e] = I.ueig[e];
    __syncthreads();
    for (int64_t task = tl.y + wave; task < tl.z; task += 4) {
      const int64_t a = I.tasks[task].x;
      const int64_t base = I.off + a * dd;
      for (int e = lane; e < dd; e += 64) {
        const T2 v = r[base + e];
        X[e] = make_double2((double)v.x, (double)v.y);
      }
      wave_sync();
      // W = U^H X
      tile_product(
          d, lane, [&](int i, int k) { const double2 u = Us[k * d + i]; return make_double2(u.x, -u.y); },
          [&](int k, int j) { return X[k * d + j]; }, [&](int i, int j, double2 v) { W[i * d + j] = v; });
      wave_sync();
      // X = (W U) / D
      const double2 c = I.decay64[a];
      tile_product(
          d, lane, [&](int i, int k) { return W[i * d + k]; }, [&](int k, int j) { return Us[k * d + j]; },
          [&](int i, int j, double2 v) {
            double dx = -c.x, dy = -c.y - (I.eval[i] - I.eval[j]);
            if (dx * dx + dy * dy < I.delta * I.delta) {
              dx = -I.delta;
              dy = 0.0;
            }
            const double inv = 1.0 / (dx * dx + dy * dy);
            X[i * d + j] = make_double2((v.x * dx + v.y * dy) * inv, (v.y * dx - v.x * dy) * inv);
          });
      wave_sync();
      // W = U X
      tile_product(
          d, lane, [&](int i, int k) { return Us[i * d + k]; }, [&](int k, int j) { return X[k * d + j]; },
          [&](int i, int j, double2 v) { W[i * d + j] = v; });
      wave_sync();
      // z = W U^H
      tile_product(
          d, lane, [&](int i, int k) { return W[i * d + k]; },
          [&](int k, int j) { const double2 u = Us[j * d + k]; return make_double2(u.x, -u.y); },
          [&](int i, int j, double2 v) { z[base + i * d + j] = T2{(T)v.x, (T)v.y}; });
      wave_sync();  // X and W are rewritten by the next task
    }
  }
}

// ----------------------------------------------------------------- segmented vector kernels
// partial[i * n_chunks + c] = sum over chunk c of conj(V_i) w, i in [i0, i0 + NI)
template <typename T, int NI>
__global__ void __launch_bounds__(256) seg_mdot_kernel(const typename Cplx<T>::t *__restrict__ V, int64_t ldv, int k,
                                                       const typename Cplx<T>::t *__restrict__ w,
                                                       const int64_t *__restrict__ ch_e, const int *__restrict__ ch_seg,
                                                       int n_chunks, const int *__restrict__ active,
                                                       double2 *__restrict__ partial) {
  using T2 = typename Cplx<T>::t;
  __shared__ double2 red[NI][256];
  const int c = blockIdx.x;
  const int i0 = blockIdx.y * NI;
  const bool on = !active || active[ch_seg[c]];
  double ax[NI], ay[NI];
#pragma unroll
  for (int q = 0; q < NI; ++q) ax[q] = ay[q] = 0.0;
  const bool full = i0 + NI <= k;  // whole groups load together, unguarded
  if (on) {
    for (int64_t e = ch_e[c] + threadIdx.x; e < ch_e[c + 1]; e += 256) {
      const T2 b = w[e];
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
        ax[q] += (double)a[q].x * b.x + (double)a[q].y * b.y;
        ay[q] += (double)a[q].x * b.y - (double)a[q].y * b.x;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NI; ++q) red[q][threadIdx.x] = make_double2(ax[q], ay[q]);
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
#pragma unroll
      for (int q = 0; q < NI; ++q) {
        red[q][threadIdx.x].x += red[q][threadIdx.x + s].x;
        red[q][threadIdx.x].y += red[q][threadIdx.x + s].y;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < NI && i0 + (int)threadIdx.x < k)
    partial[(int64_t)(i0 + threadIdx.x) * n_chunks + c] = red[threadIdx.x][0];
}

// out[i * S + s] = sum of partial over the chunks of instance s
__global__ void seg_reduce_kernel(const double2 *__restrict__ partial, int k, int n_chunks,
                                  const int *__restrict__ seg_chunk, int S, double2 *__restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)k * S) return;
  const int i = (int)(idx / S), s = (int)(idx % S);
  double sx = 0, sy = 0;
  for (int c = seg_chunk[s]; c < seg_chunk[s + 1]; ++c) {
    const double2 p = partial[(int64_t)i * n_chunks + c];
    sx += p.x;
    sy += p.y;
  }
  out[idx] = make_double2(sx, sy);
}

// Two vectors in one pass over the basis, per instance:
// partial[i] = conj(V_i) . w, partial[k + i] = conj(V_i) . u (i < k), partial[2k] = w . w
template <typename T, int NI>
__global__ void __launch_bounds__(256) seg_mdot2_kernel(const typename Cplx<T>::t *__restrict__ V, int64_t ldv, int k,
                                                        const typename Cplx<T>::t *__restrict__ w,
                                                        const typename Cplx<T>::t *__restrict__ u,
                                                        const int64_t *__restrict__ ch_e, const int *__restrict__ ch_seg,
                                                        int n_chunks, const int *__restrict__ active,
                                                        double2 *__restrict__ partial) {
  using T2 = typename Cplx<T>::t;
  __shared__ double2 red[2 * NI + 1][256];
  const int c = blockIdx.x;
  const int i0 = blockIdx.y * NI;
  const bool on = !active || active[ch_seg[c]];
  double ax[NI], ay[NI], cx[NI], cy[NI], ww = 0.0;
#pragma unroll
  for (int q = 0; q < NI; ++q) ax[q] = ay[q] = cx[q] = cy[q] = 0.0;
  // a group of NI whole basis vectors loads them together, without a
  // per-vector guard (a guarded load is waited for on its own)
  const bool full = i0 + NI <= k;
  if (on) {
    for (int64_t e = ch_e[c] + threadIdx.x; e < ch_e[c + 1]; e += 256) {
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
    partial[(int64_t)(i0 + threadIdx.x) * n_chunks + c] = red[threadIdx.x][0];
    partial[(int64_t)(k + i0 + threadIdx.x) * n_chunks + c] = red[NI + threadIdx.x][0];
  }
  if (blockIdx.y == 0 && threadIdx.x == 0) partial[(int64_t)(2 * k) * n_chunks + c] = red[2 * NI][0];
}

// Per instance (one wave each): record the new Gram column c = V^H v_j
// and form the twice-projected coefficients h = a + (a - G a), a = V^H w
// (CGS2's second projection from the measured Gram matrix G = V^H V).
// red: [(2k + 1)][S] reduced a, c, |w|^2; G: [S][ldg][ldg] column-major.
// Also |w - V h|^2 = |w|^2 - 2 Re(h^H a) + h^H G h without another read:
// form[s] = (that value, 1 when it cancels), post[s].x = its inverse square
// root (0 when it cancels: the update then keeps w - V h for an explicit
// norm), flag[s] = 1 for those instances.
__global__ void __launch_bounds__(64) batch_gram_kernel(double2 *__restrict__ G, const double2 *__restrict__ red,
                                                        int j, int S, int ldg, const int *__restrict__ active,
                                                        double2 *__restrict__ hout, double2 *__restrict__ form,
                                                        double2 *__restrict__ post, int *__restrict__ flag) {
  // one wave per instance; lane l handles basis indices l, l + 64, ...
  const int s = blockIdx.x;
  const int lane = threadIdx.x;
  const int k = j + 1;
  if (active && !active[s]) {
    for (int i = lane; i < k; i += 64) hout[(int64_t)i * S + s] = make_double2(0.0, 0.0);
    if (lane == 0) {
      form[s] = make_double2(0.0, 0.0);
      post[s] = make_double2(0.0, 0.0);
      flag[s] = 0;
    }
    return;
  }
  double2 *Gs = G + (size_t)s * ldg * ldg;
  for (int i = lane; i < k; i += 64) {
    const double2 c = red[(int64_t)(k + i) * S + s];
    Gs[(size_t)j * ldg + i] = c;
    Gs[(size_t)i * ldg + j] = make_double2(c.x, -c.y);
  }
  __syncthreads();
  for (int i = lane; i < k; i += 64) {
    double gx = 0.0, gy = 0.0;  // (G a)_i
    for (int q = 0; q < k; ++q) {
      const double2 g = Gs[(size_t)q * ldg + i], a = red[(int64_t)q * S + s];
      gx += g.x * a.x - g.y * a.y;
      gy += g.x * a.y + g.y * a.x;
    }
    const double2 a = red[(int64_t)i * S + s];
    hout[(int64_t)i * S + s] = make_double2(2.0 * a.x - gx, 2.0 * a.y - gy);
  }
  __syncthreads();
  // |w - V h|^2 = |w|^2 - 2 Re(h^H a) + h^H G h
  double part = 0.0;
  for (int i = lane; i < k; i += 64) {
    const double2 h = hout[(int64_t)i * S + s], a = red[(int64_t)i * S + s];
    double gx = 0.0, gy = 0.0;  // (G h)_i
    for (int q = 0; q < k; ++q) {
      const double2 g = Gs[(size_t)q * ldg + i], hq = hout[(int64_t)q * S + s];
      gx += g.x * hq.x - g.y * hq.y;
      gy += g.x * hq.y + g.y * hq.x;
    }
    part += (h.x * gx + h.y * gy) - 2.0 * (h.x * a.x + h.y * a.y);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
  if (lane == 0) {
    const double ww = red[(int64_t)(2 * k) * S + s].x;
    const double hn2 = ww + part;
    const bool fused = isfinite(hn2) && hn2 > 1e-6 * ww;
    form[s] = make_double2(hn2, fused ? 0.0 : 1.0);
    post[s] = make_double2(fused ? 1.0 / sqrt(hn2) : 0.0, 0.0);
    flag[s] = fused ? 0 : 1;
  }
}

// w += sign * sum_{i < k} V_i h[i * S + seg]; with post, instances whose
// post[seg].x > 0 write the result times post[seg].x to vnext instead
// (fused normalisation; w is left as it was)
constexpr int kSegUpdateMaxK = 1024;  // basis columns of one batched Arnoldi step (the launcher checks)
template <typename T>
__global__ void __launch_bounds__(256) seg_update_kernel(const typename Cplx<T>::t *__restrict__ V, int64_t ldv, int k,
                                                         const double2 *__restrict__ h, int S,
                                                         typename Cplx<T>::t *__restrict__ w,
                                                         const int64_t *__restrict__ ch_e, const int *__restrict__ ch_seg,
                                                         const int *__restrict__ active, double sign,
                                                         const double2 *__restrict__ post,
                                                         typename Cplx<T>::t *__restrict__ vnext) {
  using T2 = typename Cplx<T>::t;
  // this instance's nonzero coefficients, compacted in LDS in their order
  // (columns past the instance's basis may hold garbage and are skipped), so
  // that the element loop issues four basis reads before it uses them
  __shared__ double2 hs[kSegUpdateMaxK];
  __shared__ int hi[kSegUpdateMaxK];
  __shared__ int n_nz;
  // (hs first holds all k coefficients; one thread then compacts it in
  // place, writing slot m <= the slot i it reads)
  const int c = blockIdx.x;
  const int s = ch_seg[c];
  if (active && !active[s]) return;
  const double sc = post ? post[s].x : 0.0;
  T2 *dst = sc > 0.0 ? vnext : w;
  const double f = sc > 0.0 ? sc : 1.0;
  for (int i = threadIdx.x; i < k; i += 256) hs[i] = h[(int64_t)i * S + s];  // all loads at once
  __syncthreads();
  if (threadIdx.x == 0) {
    int m = 0;
    for (int i = 0; i < k; ++i) {
      const double2 hh = hs[i];
      if (hh.x == 0.0 && hh.y == 0.0) continue;
      hs[m] = hh;
      hi[m] = i;
      ++m;
    }
    n_nz = m;
  }
  __syncthreads();
  const int m = n_nz;
  for (int64_t e = ch_e[c] + threadIdx.x; e < ch_e[c + 1]; e += 256) {
    double ax = w[e].x, ay = w[e].y;
    int j = 0;
    for (; j + 4 <= m; j += 4) {
      T2 v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = load_stream<T>(&V[hi[j + q] * ldv + e]);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double2 hh = hs[j + q];
        ax += sign * ((double)v[q].x * hh.x - (double)v[q].y * hh.y);
        ay += sign * ((double)v[q].x * hh.y + (double)v[q].y * hh.x);
      }
    }
    for (; j < m; ++j) {
      const T2 v = V[hi[j] * ldv + e];
      const double2 hh = hs[j];
      ax += sign * ((double)v.x * hh.x - (double)v.y * hh.y);
      ay += sign * ((double)v.x * hh.y + (double)v.y * hh.x);
    }
    dst[e] = T2{(T)(f * ax), (T)(f * ay)};
  }
}

// out = sc[seg] * in  (real per-instance scale; types may differ); with a
// mask, only the instances whose mask entry is set
template <typename TI, typename TO>
__global__ void __launch_bounds__(256) seg_scale_kernel(const typename Cplx<TI>::t *__restrict__ in,
                                                        const double *__restrict__ sc,
                                                        typename Cplx<TO>::t *__restrict__ out,
                                                        const int64_t *__restrict__ ch_e, const int *__restrict__ ch_seg,
                                                        const int *__restrict__ mask) {
  const int c = blockIdx.x;
  if (mask && !mask[ch_seg[c]]) return;
  const double f = sc[ch_seg[c]];
  for (int64_t e = ch_e[c] + threadIdx.x; e < ch_e[c + 1]; e += 256)
    out[e] = typename Cplx<TO>::t{(TO)(f * (double)in[e].x), (TO)(f * (double)in[e].y)};
}

// y += sc[seg] * x  (x of type TX, y of type TY)
template <typename TX, typename TY>
__global__ void __launch_bounds__(256) seg_axpy_kernel(const typename Cplx<TX>::t *__restrict__ x,
                                                       const double *__restrict__ sc,
                                                       typename Cplx<TY>::t *__restrict__ y,
                                                       const int64_t *__restrict__ ch_e, const int *__restrict__ ch_seg) {
  const int c = blockIdx.x;
  const double f = sc[ch_seg[c]];
  if (f == 0.0) return;
  for (int64_t e = ch_e[c] + threadIdx.x; e < ch_e[c + 1]; e += 256)
    y[e] = typename Cplx<TY>::t{(TY)((double)y[e].x + f * (double)x[e].x), (TY)((double)y[e].y + f * (double)x[e].y)};
}

// b = e_0 of every instance (the stationary-state right-hand side)
__global__ void seg_unit_kernel(double2 *__restrict__ b, const int64_t *__restrict__ off, int S) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < S) b[off[s]] = make_double2(1.0, 0.0);
}

template <typename T>
__global__ void seg_zero_kernel(typename Cplx<T>::t *__restrict__ v, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    v[e] = typename Cplx<T>::t{0, 0};
}

}  // namespace heom

using namespace heom;

// ----------------------------------------------------------------- batch object
struct heom_batch {
  std::vector<heom_hier *> inst;  // not owned
  int S = 0;
  int64_t n = 0;
  std::vector<int64_t> off;       // [S + 1]
  int device = -1;
  BInst<double> *inst64 = nullptr;
  BInst<float> *inst32 = nullptr;
  ApplyParams<double> *prm64 = nullptr;  // wave-formulation tables per instance
  ApplyParams<float> *prm32 = nullptr;
  size_t smem64 = 0, smem32 = 0;         // LDS of the batched apply launch
  // every wave instance has at most 64 groups and edges per task and room for
  // its packed operator metadata and coefficients: task tables in lanes
  bool lt = true;
  size_t smem64_lt = 0, smem32_lt = 0;
  int4 *tiles = nullptr;
  int n_tiles = 0;
  std::vector<int4> tiles_inst;   // instance-major order
  std::vector<int4> tiles_cost;   // interleaved, costliest instances first
  int order = 0;                  // 0: instance-major, 1: interleaved
  int grid = 0;                   // persistent grid (0: one block per tile)
  // launch shape (autotuned): tile = base(d) x mult tasks, base(d) =
  // max(4, 256 / d^2); the wave formulation for d = 8 / 16 when var8 /
  // var16 is set (and its LDS fits), else one thread per output element
  int mult_small = 1, mult_wave = 1, var8 = 1, var16 = 1;
  int mfma16 = 0;                 // d = 16 wave instances: the self group's H terms on the matrix cores
  int tuned_from_cache = 0;
  std::vector<char> wave_ok;      // per instance: the wave formulation's LDS fits
  std::vector<double> cost;       // per instance: gathers + outputs
  std::vector<BInst<double>> i64h;
  std::vector<BInst<float>> i32h;
  std::vector<ApplyParams<double>> p64h;
  std::vector<ApplyParams<float>> p32h;
  int64_t *ch_e = nullptr;        // [n_chunks + 1]
  int *ch_seg = nullptr;          // [n_chunks]
  int *seg_chunk = nullptr;       // [S + 1]
  int n_chunks = 0;
  int64_t *d_off = nullptr;       // [S + 1]
  int *active = nullptr;          // [S]
  std::vector<int> seg_chunk_h;
  ~heom_batch() {
    void *ptrs[] = {inst64, inst32, prm64, prm32, tiles, ch_e, ch_seg, seg_chunk, d_off, active};
    for (void *p : ptrs)
      if (p) (void)hipFree(p);
  }
};

namespace heom {

// Tile lists for the current launch shape: tiles of base(d) x mult tasks
// of one instance, in instance order (tiles_inst) and round-robin over
// instances, costliest per tile first (tiles_cost).  Also sets each
// instance's variant flag in the host descriptors.
static void build_tiles(heom_batch &b) {
  const int S = b.S;
  std::vector<std::vector<int4>> per(S);
  for (int s = 0; s < S; ++s) {
    const int d = b.i64h[s].d;
    const bool wave = b.wave_ok[s] && ((d == 8 && b.var8) || (d == 16 && b.var16));
    b.i64h[s].wave = b.i32h[s].wave = wave;

    const int base = std::max(4, 256 / (d * d));
    const int tpt = base * (d >= 8 ? b.mult_wave : b.mult_small);
    const int64_t N = (b.off[s + 1] - b.off[s]) / ((int64_t)d * d);
    for (int64_t t = 0; t < N; t += tpt)
      per[s].push_back(make_int4(s, (int)t, (int)std::min<int64_t>(N, t + tpt), 0));
  }
  b.tiles_inst.clear();
  b.tiles_cost.clear();
  for (int s = 0; s < S; ++s) b.tiles_inst.insert(b.tiles_inst.end(), per[s].begin(), per[s].end());
  std::vector<int> ord(S);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int p, int q) {
    return b.cost[p] / std::max<size_t>(1, per[p].size()) > b.cost[q] / std::max<size_t>(1, per[q].size());
  });
  std::vector<size_t> pos(S, 0);
  bool any = true;
  while (any) {
    any = false;
    for (int s : ord)
      if (pos[s] < per[s].size()) {
        b.tiles_cost.push_back(per[s][pos[s]++]);
        any = true;
      }
  }
  b.n_tiles = (int)b.tiles_inst.size();
}

static heom_status batch_upload_shape(heom_batch &b) {
  HEOM_HIP_CHECK(hipMemcpy(b.prm64, b.p64h.data(), sizeof(ApplyParams<double>) * b.S, hipMemcpyHostToDevice));
  HEOM_HIP_CHECK(hipMemcpy(b.prm32, b.p32h.data(), sizeof(ApplyParams<float>) * b.S, hipMemcpyHostToDevice));
  HEOM_HIP_CHECK(hipMemcpy(b.inst64, b.i64h.data(), sizeof(BInst<double>) * b.S, hipMemcpyHostToDevice));
  HEOM_HIP_CHECK(hipMemcpy(b.inst32, b.i32h.data(), sizeof(BInst<float>) * b.S, hipMemcpyHostToDevice));
  const std::vector<int4> &src = b.order == 1 ? b.tiles_cost : b.tiles_inst;
  HEOM_HIP_CHECK(hipMemcpy(b.tiles, src.data(), sizeof(int4) * src.size(), hipMemcpyHostToDevice));
  return HEOM_OK;
}

struct BatchShape {
  int mult_small, mult_wave, var8, var16, grid, order, mfma16;
  bool operator==(const BatchShape &o) const {
    return mult_small == o.mult_small && mult_wave == o.mult_wave && var8 == o.var8 && var16 == o.var16 &&
           grid == o.grid && order == o.order && mfma16 == o.mfma16;
  }
};

static heom_status set_shape(heom_batch &b, const BatchShape &sh) {
  b.mult_small = sh.mult_small;
  b.mult_wave = sh.mult_wave;
  b.var8 = sh.var8;
  b.var16 = sh.var16;
  b.grid = sh.grid;
  b.order = sh.order;
  b.mfma16 = sh.mfma16;
  build_tiles(b);
  return batch_upload_shape(b);
}



template <typename T>
static heom_status batch_apply_T(heom_batch &b, const void *x, void *y, int border, bool use_active, hipStream_t s) {
  const int grid = b.grid > 0 ? std::min(b.grid, b.n_tiles) : b.n_tiles;
  if (grid <= 0) return HEOM_OK;
  constexpr bool dbl = std::is_same<T, double>::value;
  const BInst<T> *I = dbl ? (const BInst<T> *)b.inst64 : (const BInst<T> *)b.inst32;
  const ApplyParams<T> *Pm = dbl ? (const ApplyParams<T> *)b.prm64 : (const ApplyParams<T> *)b.prm32;
  const size_t sm = b.lt ? (dbl ? b.smem64_lt : b.smem32_lt) : (dbl ? b.smem64 : b.smem32);
  const int *act = use_active ? b.active : nullptr;
  const auto *xv = (const typename Cplx<T>::t *)x;
  auto *yv = (typename Cplx<T>::t *)y;
  if (b.mfma16 && b.lt)
    hipLaunchKernelGGL((batch_apply_kernel<T, true, true>), dim3(grid), dim3(256), sm, s, I, Pm, b.tiles, b.n_tiles, act,
                       xv, yv, border);
  else if (b.mfma16)
    hipLaunchKernelGGL((batch_apply_kernel<T, true, false>), dim3(grid), dim3(256), sm, s, I, Pm, b.tiles, b.n_tiles,
                       act, xv, yv, border);
  else if (b.lt)
    hipLaunchKernelGGL((batch_apply_kernel<T, false, true>), dim3(grid), dim3(256), sm, s, I, Pm, b.tiles, b.n_tiles,
                       act, xv, yv, border);
  else
    hipLaunchKernelGGL((batch_apply_kernel<T, false, false>), dim3(grid), dim3(256), sm, s, I, Pm, b.tiles, b.n_tiles,
                       act, xv, yv, border);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename T>
static heom_status batch_block_T(heom_batch &b, const void *r, void *z, hipStream_t s) {
  const int grid = b.grid > 0 ? std::min(b.grid, b.n_tiles) : b.n_tiles;
  if (grid <= 0) return HEOM_OK;
  const BInst<T> *I = std::is_same<T, double>::value ? (const BInst<T> *)b.inst64 : (const BInst<T> *)b.inst32;
  hipLaunchKernelGGL(batch_block_kernel<T>, dim3(grid), dim3(256), 0, s, I, b.tiles, b.n_tiles, b.active,
                     (const typename Cplx<T>::t *)r, (typename Cplx<T>::t *)z);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename T>
static heom_status batch_jacobi_T(heom_batch &b, const void *r, void *z, int border, hipStream_t s) {
  const int grid = b.grid > 0 ? std::min(b.grid, b.n_tiles) : b.n_tiles;
  if (grid <= 0) return HEOM_OK;
  const BInst<T> *I = std::is_same<T, double>::value ? (const BInst<T> *)b.inst64 : (const BInst<T> *)b.inst32;
  hipLaunchKernelGGL(batch_jacobi_kernel<T>, dim3(grid), dim3(256), 0, s, I, b.tiles, b.n_tiles, b.active,
                     (const typename Cplx<T>::t *)r, (typename Cplx<T>::t *)z, border);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

// out[i * S + s] = conj(V_i) . w per instance, i < k
template <typename T>
static heom_status seg_mdot(heom_batch &b, const void *V, int64_t ldv, int k, const void *w, double2 *partial,
                            double2 *out, hipStream_t s, const int *mask = nullptr) {  // mask: instead of active
  using T2 = typename Cplx<T>::t;
  constexpr int NI = 4;
  dim3 grid(b.n_chunks, (k + NI - 1) / NI);
  hipLaunchKernelGGL((seg_mdot_kernel<T, NI>), grid, dim3(256), 0, s, (const T2 *)V, ldv, k, (const T2 *)w, b.ch_e,
                     b.ch_seg, b.n_chunks, mask ? mask : b.active, partial);
  HEOM_HIP_CHECK(hipGetLastError());
  const int64_t tot = (int64_t)k * b.S;
  hipLaunchKernelGGL(seg_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, partial, k, b.n_chunks,
                     b.seg_chunk, b.S, out);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename T>
static heom_status seg_mdot2(heom_batch &b, const void *V, int64_t ldv, int k, const void *w, const void *u,
                             double2 *partial, double2 *out, hipStream_t s) {
  using T2 = typename Cplx<T>::t;
  // (the one-read wave variant of the single-hierarchy solver was measured
  // here and is slower: the per-instance chunks are mostly small, and one
  // workgroup walking all groups of four basis vectors serially loses to a
  // workgroup per group)
  constexpr int NI = 4;
  dim3 grid(b.n_chunks, (k + NI - 1) / NI);
  hipLaunchKernelGGL((seg_mdot2_kernel<T, NI>), grid, dim3(256), 0, s, (const T2 *)V, ldv, k, (const T2 *)w,
                     (const T2 *)u, b.ch_e, b.ch_seg, b.n_chunks, b.active, partial);
  HEOM_HIP_CHECK(hipGetLastError());
  const int kk = 2 * k + 1;
  const int64_t tot = (int64_t)kk * b.S;
  hipLaunchKernelGGL(seg_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, partial, kk, b.n_chunks,
                     b.seg_chunk, b.S, out);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename T>
static heom_status seg_update(heom_batch &b, const void *V, int64_t ldv, int k, const double2 *h, void *w,
                              double sign, hipStream_t s, const double2 *post = nullptr, void *vnext = nullptr) {
  using T2 = typename Cplx<T>::t;
  if (k > kSegUpdateMaxK) return fail(HEOM_ERR_UNSUPPORTED, "batch: Krylov basis too large for the segmented update");
  hipLaunchKernelGGL(seg_update_kernel<T>, dim3(b.n_chunks), dim3(256), 0, s, (const T2 *)V, ldv, k, h, b.S, (T2 *)w,
                     b.ch_e, b.ch_seg, b.active, sign, post, (T2 *)vnext);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename TI, typename TO>
static heom_status seg_scale(heom_batch &b, const void *in, const double *sc, void *out, hipStream_t s,
                             const int *mask = nullptr) {
  hipLaunchKernelGGL((seg_scale_kernel<TI, TO>), dim3(b.n_chunks), dim3(256), 0, s,
                     (const typename Cplx<TI>::t *)in, sc, (typename Cplx<TO>::t *)out, b.ch_e, b.ch_seg, mask);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename TX, typename TY>
static heom_status seg_axpy(heom_batch &b, const void *x, const double *sc, void *y, hipStream_t s) {
  hipLaunchKernelGGL((seg_axpy_kernel<TX, TY>), dim3(b.n_chunks), dim3(256), 0, s,
                     (const typename Cplx<TX>::t *)x, sc, (typename Cplx<TY>::t *)y, b.ch_e, b.ch_seg);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename T>
static heom_status seg_zero(void *v, int64_t n, hipStream_t s) {
  const int64_t g = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536));
  hipLaunchKernelGGL(seg_zero_kernel<T>, dim3((unsigned)g), dim3(256), 0, s, (typename Cplx<T>::t *)v, n);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

// ----------------------------------------------------------------- batched GMRES
// Restarted right-preconditioned (Jacobi) GMRES on every instance at once:
// one Arnoldi step is one batched apply + segmented CGS2 for all active
// instances; the small least-squares problems are solved per instance on
// the host.  Instances leave the active set when they converge.
template <typename T>
struct BatchGmres {
  using T2 = typename Cplx<T>::t;
  heom_batch *b = nullptr;
  int m = 30;
  T2 *V = nullptr, *Z = nullptr, *w = nullptr;
  double2 *partial = nullptr, *hdev = nullptr, *gram = nullptr;
  double *sdev = nullptr;
  int *flag = nullptr;            // [S] 1: the Gram formula cancelled, explicit norm
  double *pin_sc = nullptr;       // host pinned [S]
  double2 *pin_h = nullptr;       // host pinned: step coefficients [(m + 1) S] and norms [S]
  PinnedBuf pin;
  bool use_graph = false;
  int prec = HEOM_PREC_JACOBI;         // HEOM_PREC_NONE: Z aliases V
  std::vector<hipGraphExec_t> graphs;  // one per Arnoldi step j
  hipStream_t cap = nullptr;
  ~BatchGmres() {
    for (hipGraphExec_t g : graphs)
      if (g) (void)hipGraphExecDestroy(g);
    if (cap) (void)hipStreamDestroy(cap);
  }

  static size_t bytes(const heom_batch &b, int m, bool jac) {  // jac: any preconditioner (Z kept)
    const size_t vec = (size_t)b.n * sizeof(T2);
    return (size_t)(m + 1) * vec + (jac ? (size_t)m * vec : 0) + vec + (size_t)(2 * m + 3) * b.n_chunks * sizeof(double2) +
           (size_t)(3 * m + 7) * b.S * sizeof(double2) + (size_t)b.S * (m + 1) * (m + 1) * sizeof(double2) +
           (size_t)b.S * sizeof(double) + (size_t)b.S * sizeof(int) + 9 * 256;
  }

  heom_status init(heom_batch &bb, WsArena &ws, int m_, bool graph, int prec_) {
    b = &bb;
    m = m_;
    use_graph = graph;
    prec = prec_;
    const size_t vec = (size_t)b->n * sizeof(T2);
    V = (T2 *)ws.take((size_t)(m + 1) * vec);
    Z = prec != HEOM_PREC_NONE ? (T2 *)ws.take((size_t)m * vec) : V;
    w = (T2 *)ws.take(vec);
    partial = (double2 *)ws.take((size_t)(2 * m + 3) * b->n_chunks * sizeof(double2));
    // hdev: [0, (2m+3) S) reduced a, c, |w|^2;  then h [(m+1) S], the
    // explicit |w'|^2 [S], the Gram-formula |w'|^2 and its flag [S], and the
    // fused normalisation scale [S]
    hdev = (double2 *)ws.take((size_t)(3 * m + 7) * b->S * sizeof(double2));
    gram = (double2 *)ws.take((size_t)b->S * (m + 1) * (m + 1) * sizeof(double2));
    sdev = (double *)ws.take((size_t)b->S * sizeof(double));
    flag = (int *)ws.take((size_t)b->S * sizeof(int));
    if (!V || !Z || !w || !partial || !hdev || !gram || !sdev || !flag)
      return fail(HEOM_ERR_ARG, "batch: workspace too small");
    HEOM_TRY(pin.ensure((size_t)(m + 3) * b->S * sizeof(double2) + (size_t)(m + 1) * b->S * sizeof(double2) +
                        (size_t)b->S * sizeof(double)));
    pin_h = (double2 *)pin.p;
    pin_sc = (double *)(pin_h + (size_t)(2 * m + 4) * b->S);
    graphs.assign(m, nullptr);
    if (use_graph) HEOM_HIP_CHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    return HEOM_OK;
  }

  double2 *h_out() const { return hdev + (size_t)(2 * m + 3) * b->S; }   // [(m+1)][S] coefficients
  double2 *n_out() const { return h_out() + (size_t)(m + 1) * b->S; }    // [S] |w'|^2 (explicit, flagged only)
  double2 *f_out() const { return n_out() + b->S; }                      // [S] (formula |w'|^2, flag)
  double2 *post() const { return f_out() + b->S; }                       // [S] fused scale

  // Device work of Arnoldi step j: z_j = P v_j, w = B z_j, then CGS2 in two
  // passes over the basis: one two-vector multi-dot (a = V^H w, the Gram
  // column V^H v_j, |w|^2), the per-instance Gram correction with the norm
  // |w - V h| from the Gram matrix, one update that writes v_{j+1} already
  // normalised; only instances whose norm formula cancelled keep w - V h in
  // w and get an explicit |w|^2; then the copy of the coefficients to the
  // host.
  heom_status step_device(int j, int border, hipStream_t s) {
    const int64_t n = b->n;
    T2 *vj = V + (size_t)j * n;
    T2 *zj = Z + (size_t)j * n;
    if (prec == HEOM_PREC_JACOBI) HEOM_TRY(batch_jacobi_T<T>(*b, vj, zj, border, s));
    if (prec == HEOM_PREC_BLOCK) HEOM_TRY(batch_block_T<T>(*b, vj, zj, s));
    HEOM_TRY(batch_apply_T<T>(*b, zj, w, border, true, s));
    HEOM_TRY(seg_mdot2<T>(*b, V, n, j + 1, w, vj, partial, hdev, s));
    hipLaunchKernelGGL(batch_gram_kernel, dim3(b->S), dim3(64), 0, s, gram, hdev, j, b->S, m + 1, b->active, h_out(),
                       f_out(), post(), flag);
    HEOM_HIP_CHECK(hipGetLastError());
    HEOM_TRY(seg_update<T>(*b, V, n, j + 1, h_out(), w, -1.0, s, post(), V + (size_t)(j + 1) * n));
    HEOM_TRY(seg_mdot<T>(*b, w, 0, 1, w, partial, n_out(), s, flag));
    HEOM_HIP_CHECK(hipMemcpyAsync(pin_h, h_out(), sizeof(double2) * (m + 3) * b->S, hipMemcpyDeviceToHost, s));
    return HEOM_OK;
  }

  heom_status step(int j, int border, hipStream_t s) {
    if (!use_graph) return step_device(j, border, s);
    if (!graphs[j]) {
      hipGraph_t g = nullptr;
      HEOM_HIP_CHECK(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
      heom_status st = step_device(j, border, cap);
      hipGraph_t got = nullptr;
      hipError_t e = hipStreamEndCapture(cap, &got);
      g = got;
      if (st != HEOM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return fail(HEOM_ERR_HIP, std::string("batch graph capture: ") + hipGetErrorString(e));
      hipGraphExec_t ex = nullptr;
      e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return fail(HEOM_ERR_HIP, std::string("batch graph instantiate: ") + hipGetErrorString(e));
      graphs[j] = ex;
    }
    HEOM_HIP_CHECK(hipGraphLaunch(graphs[j], s));
    return HEOM_OK;
  }

  heom_status norms(const T2 *v, std::vector<double> &out, hipStream_t s) {
    HEOM_TRY(seg_mdot<T>(*b, v, 0, 1, v, partial, hdev, s));
    HEOM_HIP_CHECK(hipMemcpyAsync(pin_h, hdev, sizeof(double2) * b->S, hipMemcpyDeviceToHost, s));
    HEOM_HIP_CHECK(hipStreamSynchronize(s));
    out.resize(b->S);
    for (int q = 0; q < b->S; ++q) out[q] = std::sqrt(std::max(pin_h[q].x, 0.0));
    return HEOM_OK;
  }

  heom_status set_active(const std::vector<char> &act, hipStream_t s) {
    std::vector<int> a(b->S);
    for (int q = 0; q < b->S; ++q) a[q] = act[q] ? 1 : 0;
    HEOM_HIP_CHECK(hipMemcpyAsync(b->active, a.data(), sizeof(int) * b->S, hipMemcpyHostToDevice, s));
    HEOM_HIP_CHECK(hipStreamSynchronize(s));
    return HEOM_OK;
  }

  // Solve B x = rhs per instance for the instances flagged in `want` (others
  // untouched); x holds the initial guess (zero when x_is_zero).  iters[q] and
  // res[q] report per instance; conv[q] = 1 when res[q] <= tol.
  heom_status solve(const T2 *rhs, T2 *x, const std::vector<char> &want, double tol, int max_iter, int border,
                    bool x_is_zero, std::vector<int> &iters, std::vector<double> &res, std::vector<char> &conv,
                    int64_t &applies, hipStream_t s) {
    const int S = b->S;
    const int64_t n = b->n;
    std::vector<double> bnorm, beta;
    std::vector<char> act(want);
    HEOM_TRY(set_active(act, s));
    HEOM_TRY(norms(rhs, bnorm, s));
    iters.assign(S, 0);
    res.assign(S, 0.0);
    conv.assign(S, 0);
    std::vector<cd> H((size_t)S * (m + 1) * m), sn((size_t)S * m), g((size_t)S * (m + 1));
    std::vector<double> cs((size_t)S * m);
    std::vector<int> kcol(S);
    int it_total = 0;
    for (int cycle = 0;; ++cycle) {
      // w = rhs - B x on the active instances
      if (x_is_zero && cycle == 0) {
        HEOM_HIP_CHECK(hipMemcpyAsync(w, rhs, sizeof(T2) * n, hipMemcpyDeviceToDevice, s));
      } else {
        // (inactive instances keep stale values in w; their reductions are masked)
        HEOM_TRY(batch_apply_T<T>(*b, x, w, border, true, s));
        ++applies;
        HEOM_TRY((axpby<T, T>(rhs, 1.0, w, -1.0, n, s)));
      }
      HEOM_TRY(norms(w, beta, s));
      bool any = false;
      for (int q = 0; q < S; ++q) {
        if (!act[q]) continue;
        const double rel = bnorm[q] > 0 ? beta[q] / bnorm[q] : 0.0;
        if (!std::isfinite(rel)) return fail(HEOM_ERR_NAN, "batch: non-finite residual");
        res[q] = rel;
        if (rel <= tol) {
          conv[q] = 1;
          act[q] = 0;
        } else if (iters[q] >= max_iter) {
          act[q] = 0;
        }
        any = any || act[q];
      }
      if (!any) break;
      HEOM_TRY(set_active(act, s));
      // V0 = w / beta
      for (int q = 0; q < S; ++q) pin_sc[q] = act[q] && beta[q] > 0 ? 1.0 / beta[q] : 0.0;
      HEOM_HIP_CHECK(hipMemcpyAsync(sdev, pin_sc, sizeof(double) * S, hipMemcpyHostToDevice, s));
      HEOM_TRY((seg_scale<T, T>(*b, w, sdev, V, s)));
      std::fill(g.begin(), g.end(), cd(0));
      for (int q = 0; q < S; ++q) {
        g[(size_t)q * (m + 1)] = act[q] ? beta[q] : 0.0;
        kcol[q] = 0;
      }
      std::vector<char> ext(act);  // still extending its basis this cycle
      int j = 0;
      for (; j < m; ++j) {
        HEOM_TRY(step(j, border, s));
        ++applies;
        ++it_total;
        HEOM_HIP_CHECK(hipStreamSynchronize(s));
        const double2 *hp1 = pin_h, *hnrm = pin_h + (size_t)(m + 1) * S, *hform = hnrm + S;
        bool more = false, stopped = false, explicit_norm = false;
        for (int q = 0; q < S; ++q) {
          pin_sc[q] = 0.0;
          if (!ext[q]) continue;
          ++iters[q];
          cd *Hc = &H[((size_t)q * (m + 1)) * m];
          for (int i = 0; i <= j; ++i) Hc[(size_t)j * (m + 1) + i] = cd(hp1[(size_t)i * S + q].x, hp1[(size_t)i * S + q].y);
          const bool flagged = hform[q].y != 0.0;  // v_{j+1} not yet written: scale w below
          const double hn = std::sqrt(std::max(flagged ? hnrm[q].x : hform[q].x, 0.0));
          if (!std::isfinite(hn)) return fail(HEOM_ERR_NAN, "batch: non-finite Arnoldi norm");
          Hc[(size_t)j * (m + 1) + j + 1] = hn;
          cd *col = &Hc[(size_t)j * (m + 1)];
          for (int i = 0; i < j; ++i) {
            const double c = cs[(size_t)q * m + i];
            const cd sv = sn[(size_t)q * m + i];
            const cd tmp = c * col[i] + sv * col[i + 1];
            col[i + 1] = -std::conj(sv) * col[i] + c * col[i + 1];
            col[i] = tmp;
          }
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
          cs[(size_t)q * m + j] = c;
          sn[(size_t)q * m + j] = sv;
          col[j] = rr;
          col[j + 1] = 0.0;
          cd *gr = &g[(size_t)q * (m + 1)];
          gr[j + 1] = -std::conj(sv) * gr[j];
          gr[j] = c * gr[j];
          kcol[q] = j + 1;
          const double rel = bnorm[q] > 0 ? std::abs(gr[j + 1]) / bnorm[q] : 0.0;
          if (rel <= tol * 0.5 || hn <= 1e-300 || iters[q] >= max_iter) {
            ext[q] = 0;
            stopped = true;
          } else if (flagged) {
            pin_sc[q] = 1.0 / hn;
            explicit_norm = true;
          }
          more = more || ext[q];
        }
        if (!more) { ++j; break; }
        // instances that stop leave the active set; v_{j+1} = w / hn for the
        // flagged instances still extending (the others have it already)
        if (stopped) HEOM_TRY(set_active(ext, s));
        if (explicit_norm) {
          HEOM_HIP_CHECK(hipMemcpyAsync(sdev, pin_sc, sizeof(double) * S, hipMemcpyHostToDevice, s));
          HEOM_TRY((seg_scale<T, T>(*b, w, sdev, V + (size_t)(j + 1) * n, s, flag)));
        }
      }
      // x += Z y per instance
      int kmax = 0;
      for (int q = 0; q < S; ++q) kmax = std::max(kmax, kcol[q]);
      if (kmax > 0) {
        std::vector<double2> yh((size_t)kmax * S, make_double2(0, 0));
        for (int q = 0; q < S; ++q) {
          const int k = kcol[q];
          const cd *Hc = &H[((size_t)q * (m + 1)) * m];
          std::vector<cd> y(k);
          for (int i = k - 1; i >= 0; --i) {
            cd acc = g[(size_t)q * (m + 1) + i];
            for (int p = i + 1; p < k; ++p) acc -= Hc[(size_t)p * (m + 1) + i] * y[p];
            const cd dgl = Hc[(size_t)i * (m + 1) + i];
            y[i] = std::abs(dgl) > 0 ? acc / dgl : cd(0);
          }
          for (int i = 0; i < k; ++i) yh[(size_t)i * S + q] = make_double2(y[i].real(), y[i].imag());
        }
        std::vector<char> upd(S);
        for (int q = 0; q < S; ++q) upd[q] = kcol[q] > 0;
        HEOM_TRY(set_active(upd, s));
        HEOM_HIP_CHECK(hipMemcpyAsync(hdev, yh.data(), sizeof(double2) * kmax * S, hipMemcpyHostToDevice, s));
        HEOM_TRY(seg_update<T>(*b, Z, n, kmax, hdev, x, 1.0, s));
        HEOM_HIP_CHECK(hipStreamSynchronize(s));
      }
      x_is_zero = false;
      for (int q = 0; q < S; ++q)
        if (kcol[q] == 0 && act[q]) act[q] = 0;  // no progress possible (breakdown)
      HEOM_TRY(set_active(act, s));
    }
    (void)it_total;
    return HEOM_OK;
  }
};

static heom_status batch_check(const heom_batch *b) {
  if (!b) return fail(HEOM_ERR_ARG, "batch: NULL handle");
  int dev = 0;
  HEOM_HIP_CHECK(hipGetDevice(&dev));
  if (dev != b->device) return fail(HEOM_ERR_ARG, "batch: tables live on another device");
  return HEOM_OK;
}

}  // namespace heom

// ----------------------------------------------------------------- ABI
extern "C" {

static heom_status heom_batch_create_body(int32_t n_inst, heom_hier *const *inst, heom_batch **out) {
  if (!out || n_inst <= 0 || !inst) return fail(HEOM_ERR_ARG, "batch_create: bad arguments");
  *out = nullptr;
  for (int s = 0; s < n_inst; ++s) {  // argument checks before any device work
    if (!inst[s]) return fail(HEOM_ERR_ARG, "batch_create: NULL instance");
    const Hier &h = *inst[s]->impl;
    if (h.d > 16) return fail(HEOM_ERR_UNSUPPORTED, "batch_create: instances need d <= 16");
    if (!h.lind.empty()) return fail(HEOM_ERR_UNSUPPORTED, "batch_create: instances with a Lindbladian are not batched");
  }
  std::unique_ptr<heom_batch> b(new heom_batch());
  b->S = n_inst;
  b->inst.assign(inst, inst + n_inst);
  HEOM_HIP_CHECK(hipGetDevice(&b->device));
  b->off.assign(n_inst + 1, 0);
  std::vector<BInst<double>> i64(n_inst);
  std::vector<BInst<float>> i32(n_inst);
  std::vector<ApplyParams<double>> p64(n_inst);
  std::vector<ApplyParams<float>> p32(n_inst);
  std::vector<double> cost(n_inst);
  constexpr size_t kLdsMax = 64 * 1024;
  for (int s = 0; s < n_inst; ++s) {
    Hier &h = *inst[s]->impl;
    HEOM_TRY(ensure_device(h));
    const DeviceTables &D = h.dev;
    b->off[s + 1] = b->off[s] + h.N * (int64_t)h.d * h.d;
    BInst<double> a{};
    a.tasks = D.base.tasks; a.groups = D.base.groups; a.gedges = D.base.gedges;
    a.coef_op = D.coef_op; a.coef = D.coef64; a.ell_cnt = D.ell_cnt; a.ell_col = D.ell_col;
    a.ell_val = D.ell_val64; a.decay = D.decay64; a.decay64 = D.decay64; a.hdiag64 = D.hdiag;
    a.ueig = D.ueig; a.eval = D.eval; a.delta = h.block_delta;
    a.off = b->off[s]; a.slots = h.ell.slots; a.d = h.d;
    i64[s] = a;
    BInst<float> f{};
    f.tasks = D.base.tasks; f.groups = D.base.groups; f.gedges = D.base.gedges;
    f.coef_op = D.coef_op; f.coef = D.coef32; f.ell_cnt = D.ell_cnt; f.ell_col = D.ell_col;
    f.ell_val = D.ell_val32; f.decay = D.decay32; f.decay64 = D.decay64; f.hdiag64 = D.hdiag;
    f.ueig = D.ueig; f.eval = D.eval; f.delta = h.block_delta;
    f.off = b->off[s]; f.slots = h.ell.slots; f.d = h.d;
    i32[s] = f;
    cost[s] = (double)h.row_ptr.back() * h.d * h.d + (double)h.N * h.d * h.d;
    // wave formulation for d in {8, 16}: its LDS (4 staging blocks, the
    // compact operator tables and the H diagonal) must fit
    const size_t nce = h.ell.c_col.size();
    const size_t lds64 = 4 * (size_t)h.d * h.d * 16 + nce * (16 + 4) + 16 + (size_t)h.d * 16;
    const size_t lds32 = 4 * (size_t)h.d * h.d * 8 + nce * (8 + 4) + 16 + (size_t)h.d * 8;
    const bool wave = (h.d == 8 || h.d == 16) && lds64 <= kLdsMax;
    i64[s].wave = i32[s].wave = wave;
    if (wave) {
      b->smem64 = std::max(b->smem64, lds64);
      b->smem32 = std::max(b->smem32, lds32);
      const size_t nco = h.coefs.size();
      const size_t lt64 = lds64 + nco * 4 + 16 + 2 * nco * 16, lt32 = lds32 + nco * 4 + 16 + 2 * nco * 8;
      if (D.base.max_groups > 64 || D.base.max_edges > 64 || nce >= (1u << 20) || lt64 > kLdsMax) b->lt = false;
      b->smem64_lt = std::max(b->smem64_lt, lt64);
      b->smem32_lt = std::max(b->smem32_lt, lt32);
    }
    ApplyParams<double> q{};
    q.tasks = D.base.tasks; q.n_tasks = h.N; q.groups = D.base.groups; q.gedges = D.base.gedges;
    q.decay = D.decay64; q.ell_cnt = D.ell_cnt; q.ell_col = D.ell_col; q.ell_val = D.ell_val64;
    q.op_slots = D.op_slots; q.slots = h.ell.slots; q.c_meta = D.c_meta; q.c_col = D.c_col; q.c_val = D.c_val64;
    q.n_centries = (int)nce; q.hdiag = D.hdiag; q.coef_op = D.coef_op; q.coef = D.coef64; q.d = h.d; q.R = 1;
    q.n_coef = (int)h.coefs.size();
    q.hoff = D.hoff64;
    p64[s] = q;
    ApplyParams<float> r{};
    r.tasks = D.base.tasks; r.n_tasks = h.N; r.groups = D.base.groups; r.gedges = D.base.gedges;
    r.decay = D.decay32; r.ell_cnt = D.ell_cnt; r.ell_col = D.ell_col; r.ell_val = D.ell_val32;
    r.op_slots = D.op_slots; r.slots = h.ell.slots; r.c_meta = D.c_meta; r.c_col = D.c_col; r.c_val = D.c_val32;
    r.n_centries = (int)nce; r.hdiag = D.hdiag32; r.coef_op = D.coef_op; r.coef = D.coef32; r.d = h.d; r.R = 1;
    r.n_coef = (int)h.coefs.size();
    r.hoff = D.hoff32;
    p32[s] = r;
  }
  b->n = b->off[n_inst];
  b->i64h = i64;
  b->i32h = i32;
  b->p64h = p64;
  b->p32h = p32;
  b->cost = cost;
  b->wave_ok.assign(n_inst, 0);
  for (int s = 0; s < n_inst; ++s) b->wave_ok[s] = i64[s].wave;
  build_tiles(*b);
  const size_t max_tiles = b->tiles_inst.size();  // mult = 1: the most tiles any shape makes
  // chunks of at most 16384 elements inside each instance
  std::vector<int64_t> che{0};
  std::vector<int> chs;
  b->seg_chunk_h.assign(n_inst + 1, 0);
  for (int s = 0; s < n_inst; ++s) {
    b->seg_chunk_h[s] = (int)chs.size();
    for (int64_t e = b->off[s]; e < b->off[s + 1]; e += 16384) {
      chs.push_back(s);
      che.push_back(std::min<int64_t>(b->off[s + 1], e + 16384));
    }
  }
  b->seg_chunk_h[n_inst] = (int)chs.size();
  b->n_chunks = (int)chs.size();
  HEOM_HIP_CHECK(hipMalloc(&b->inst64, sizeof(BInst<double>) * n_inst));
  HEOM_HIP_CHECK(hipMalloc(&b->inst32, sizeof(BInst<float>) * n_inst));
  HEOM_HIP_CHECK(hipMalloc(&b->prm64, sizeof(ApplyParams<double>) * n_inst));
  HEOM_HIP_CHECK(hipMalloc(&b->prm32, sizeof(ApplyParams<float>) * n_inst));
  HEOM_HIP_CHECK(hipMemcpy(b->prm64, p64.data(), sizeof(ApplyParams<double>) * n_inst, hipMemcpyHostToDevice));
  HEOM_HIP_CHECK(hipMemcpy(b->prm32, p32.data(), sizeof(ApplyParams<float>) * n_inst, hipMemcpyHostToDevice));
  HEOM_HIP_CHECK(hipMalloc(&b->tiles, sizeof(int4) * std::max<size_t>(1, max_tiles)));
  HEOM_HIP_CHECK(hipMalloc(&b->ch_e, sizeof(int64_t) * che.size()));
  HEOM_HIP_CHECK(hipMalloc(&b->ch_seg, sizeof(int) * std::max<size_t>(1, chs.size())));
  HEOM_HIP_CHECK(hipMalloc(&b->seg_chunk, sizeof(int) * (n_inst + 1)));
  HEOM_HIP_CHECK(hipMalloc(&b->d_off, sizeof(int64_t) * (n_inst + 1)));
  HEOM_HIP_CHECK(hipMalloc(&b->active, sizeof(int) * n_inst));
  HEOM_HIP_CHECK(hipMemcpy(b->inst64, i64.data(), sizeof(BInst<double>) * n_inst, hipMemcpyHostToDevice));
  HEOM_HIP_CHECK(hipMemcpy(b->inst32, i32.data(), sizeof(BInst<float>) * n_inst, hipMemcpyHostToDevice));
  HEOM_HIP_CHECK(hipMemcpy(b->ch_e, che.data(), sizeof(int64_t) * che.size(), hipMemcpyHostToDevice));
  if (!chs.empty()) HEOM_HIP_CHECK(hipMemcpy(b->ch_seg, chs.data(), sizeof(int) * chs.size(), hipMemcpyHostToDevice));
  HEOM_HIP_CHECK(hipMemcpy(b->seg_chunk, b->seg_chunk_h.data(), sizeof(int) * (n_inst + 1), hipMemcpyHostToDevice));
  HEOM_HIP_CHECK(hipMemcpy(b->d_off, b->off.data(), sizeof(int64_t) * (n_inst + 1), hipMemcpyHostToDevice));
  std::vector<int> ones(n_inst, 1);
  HEOM_HIP_CHECK(hipMemcpy(b->active, ones.data(), sizeof(int) * n_inst, hipMemcpyHostToDevice));
  HEOM_TRY(batch_upload_shape(*b));
  *out = b.release();
  return HEOM_OK;
}

heom_status heom_batch_create(int32_t n_inst, heom_hier *const *inst, heom_batch **out) {
  return guarded([&] { return heom_batch_create_body(n_inst, inst, out); });
}

void heom_batch_free(heom_batch *b) { delete b; }

heom_status heom_batch_shape(const heom_batch *b, int32_t *shape) {
  if (!b || !shape) return fail(HEOM_ERR_ARG, "batch_shape: NULL argument");
  shape[0] = b->mult_small;
  shape[1] = b->mult_wave;
  shape[2] = b->var8;
  shape[3] = b->var16;
  shape[4] = b->grid;
  shape[5] = b->order;
  shape[6] = b->mfma16;
  shape[7] = b->tuned_from_cache;
  return HEOM_OK;
}

heom_status heom_batch_set_shape(heom_batch *b, const int32_t *shape) {
  return guarded([&]() -> heom_status {
    HEOM_TRY(batch_check(b));
    if (!shape) return fail(HEOM_ERR_ARG, "batch_set_shape: NULL shape");
    const BatchShape sh{shape[0], shape[1], shape[2], shape[3], shape[4], shape[5], shape[6]};
    auto mult_ok = [](int m) { return m == 1 || m == 2 || m == 4 || m == 8; };
    if (!mult_ok(sh.mult_small) || !mult_ok(sh.mult_wave) || (sh.var8 != 0 && sh.var8 != 1) ||
        (sh.var16 != 0 && sh.var16 != 1) || sh.grid < 0 || (sh.order != 0 && sh.order != 1) ||
        (sh.mfma16 != 0 && sh.mfma16 != 1))
      return fail(HEOM_ERR_ARG, "batch_set_shape: multipliers in {1, 2, 4, 8}, flags in {0, 1}, grid >= 0");
    b->tuned_from_cache = 0;
    return set_shape(*b, sh);
  });
}

heom_status heom_batch_info(const heom_batch *b, int64_t *offsets, int64_t *n_tiles, int32_t *grid, int32_t *order) {
  if (!b) return fail(HEOM_ERR_ARG, "batch_info: NULL handle");
  if (offsets) std::copy(b->off.begin(), b->off.end(), offsets);
  if (n_tiles) *n_tiles = b->n_tiles;
  if (grid) *grid = b->grid;
  if (order) *order = b->order;
  return HEOM_OK;
}

static heom_status heom_batch_apply_body(heom_batch *b, int32_t precision, const void *x_dev, void *y_dev, int32_t border,
                             void *stream) {
  HEOM_TRY(batch_check(b));
  if (!x_dev || !y_dev) return fail(HEOM_ERR_ARG, "batch_apply: NULL vector");
  hipStream_t s = (hipStream_t)stream;
  if (precision == HEOM_FP64) return batch_apply_T<double>(*b, x_dev, y_dev, border != 0, false, s);
  if (precision == HEOM_FP32) return batch_apply_T<float>(*b, x_dev, y_dev, border != 0, false, s);
  return fail(HEOM_ERR_ARG, "batch_apply: precision must be FP64 or FP32");
}

heom_status heom_batch_apply(heom_batch *b, int32_t precision, const void *x_dev, void *y_dev, int32_t border,
                             void *stream) {
  return guarded([&] { return heom_batch_apply_body(b, precision, x_dev, y_dev, border, stream); });
}

// ----------------------------------------------------------------- autotuner
// Cache key: the device, the precision and every instance's shape (N, d,
// operator-table size, wave eligibility), FNV-1a 64.
static std::string tune_key(const heom_batch &b, int precision, const hipDeviceProp_t &p) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    for (int k = 0; k < 8; ++k) {
      h ^= (v >> (8 * k)) & 0xff;
      h *= 1099511628211ull;
    }
  };
  for (const char *c = p.gcnArchName; *c; ++c) mix((uint64_t)(unsigned char)*c);
  mix((uint64_t)p.multiProcessorCount);
  mix((uint64_t)precision);
  mix((uint64_t)b.S);
  for (int s = 0; s < b.S; ++s) {
    mix((uint64_t)(b.off[s + 1] - b.off[s]));
    mix((uint64_t)b.i64h[s].d);
    mix((uint64_t)b.wave_ok[s]);
    mix((uint64_t)b.inst[s]->impl->ell.c_col.size());
  }
  char buf[32];
  std::snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)h);
  return buf;
}

static bool cache_lookup(const char *path, const std::string &key, BatchShape &sh) {
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    char k[64];
    BatchShape t{};
    if (std::sscanf(line, "heomx-batch-shape 2 %63s %d %d %d %d %d %d %d", k, &t.mult_small, &t.mult_wave, &t.var8,
                    &t.var16, &t.grid, &t.order, &t.mfma16) == 8 &&
        key == k && t.mult_small >= 1 && t.mult_wave >= 1 && t.grid >= 0 && (t.order == 0 || t.order == 1) &&
        (t.mfma16 == 0 || t.mfma16 == 1)) {
      sh = t;  // the last entry for the key wins
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

static void cache_store(const char *path, const std::string &key, const BatchShape &sh, double ms_def, double ms_best) {
  FILE *f = std::fopen(path, "a");
  if (!f) return;  // a cache that cannot be written only costs the next search
  std::fprintf(f, "heomx-batch-shape 2 %s %d %d %d %d %d %d %d %.4f %.4f\n", key.c_str(), sh.mult_small, sh.mult_wave,
               sh.var8, sh.var16, sh.grid, sh.order, sh.mfma16, ms_def, ms_best);
  std::fclose(f);
}

static heom_status heom_batch_tune_body(heom_batch *b, int32_t precision, const void *x_dev, void *y_dev, int32_t reps,
                            double *ms_default, double *ms_best, void *stream) {
  HEOM_TRY(batch_check(b));
  if (!x_dev || !y_dev || reps < 1) return fail(HEOM_ERR_ARG, "batch_tune: bad arguments");
  if (precision != HEOM_FP64 && precision != HEOM_FP32) return fail(HEOM_ERR_ARG, "batch_tune: precision");
  hipStream_t s = (hipStream_t)stream;
  hipDeviceProp_t prop;
  HEOM_HIP_CHECK(hipGetDeviceProperties(&prop, b->device));
  const int cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  hipEvent_t e0, e1;
  HEOM_HIP_CHECK(hipEventCreate(&e0));
  HEOM_HIP_CHECK(hipEventCreate(&e1));
  struct Ev {
    hipEvent_t a, b;
    ~Ev() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  } ev{e0, e1};
  auto timeit = [&](const BatchShape &sh, double &ms) -> heom_status {
    HEOM_TRY(set_shape(*b, sh));
    for (int r = 0; r < 2; ++r) HEOM_TRY(heom_batch_apply(b, precision, x_dev, y_dev, 0, stream));
    HEOM_HIP_CHECK(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) HEOM_TRY(heom_batch_apply(b, precision, x_dev, y_dev, 0, stream));
    HEOM_HIP_CHECK(hipEventRecord(e1, s));
    HEOM_HIP_CHECK(hipEventSynchronize(e1));
    float f = 0.f;
    HEOM_HIP_CHECK(hipEventElapsedTime(&f, e0, e1));
    ms = f / reps;
    return HEOM_OK;
  };
  const BatchShape def{1, 1, 1, 1, 0, 0, 0};
  double t_def = 0.0;
  HEOM_TRY(timeit(def, t_def));
  BatchShape best = def;
  double t_best = t_def;
  const char *path = std::getenv("HEOMX_TUNE_CACHE");
  const std::string key = tune_key(*b, precision, prop);
  BatchShape cached{};
  b->tuned_from_cache = 0;
  if (path && *path && cache_lookup(path, key, cached)) {
    double t = 0.0;
    HEOM_TRY(timeit(cached, t));
    best = cached;
    t_best = t;
    b->tuned_from_cache = 1;
  } else {
    // coordinate descent over the launch shape, two sweeps; a candidate
    // replaces the best only when it is faster
    bool has8 = false, has16 = false;
    for (int q = 0; q < b->S; ++q) {
      has8 = has8 || (b->wave_ok[q] && b->i64h[q].d == 8);
      has16 = has16 || (b->wave_ok[q] && b->i64h[q].d == 16);
    }
    const std::vector<int> mults = {1, 2, 4, 8};
    const std::vector<int> grids = {0, 2 * cus, 4 * cus, 8 * cus, 16 * cus};
    for (int sweep = 0; sweep < 2; ++sweep) {
      for (int param = 0; param < 7; ++param) {
        std::vector<int> cand;
        if (param == 0) cand = mults;
        else if (param == 1) cand = mults;
        else if (param == 2) { if (has8) cand = {0, 1}; }
        else if (param == 3) { if (has16) cand = {0, 1}; }
        else if (param == 4) cand = grids;
        else if (param == 5) cand = {0, 1};
        else if (has16 && best.var16) cand = {0, 1};  // the matrix-core self group: wave kernel only
        for (int v : cand) {
          BatchShape t = best;
          int *field[] = {&t.mult_small, &t.mult_wave, &t.var8, &t.var16, &t.grid, &t.order, &t.mfma16};
          *field[param] = v;
          if (t == best) continue;
          double ms = 0.0;
          HEOM_TRY(timeit(t, ms));
          if (ms < t_best) { t_best = ms; best = t; }
        }
      }
    }
    if (path && *path) cache_store(path, key, best, t_def, t_best);
  }
  HEOM_TRY(set_shape(*b, best));
  if (ms_default) *ms_default = t_def;
  if (ms_best) *ms_best = t_best;
  return HEOM_OK;
}

heom_status heom_batch_tune(heom_batch *b, int32_t precision, const void *x_dev, void *y_dev, int32_t reps,
                            double *ms_default, double *ms_best, void *stream) {
  return guarded([&] { return heom_batch_tune_body(b, precision, x_dev, y_dev, reps, ms_default, ms_best, stream); });
}

// The fallback pass re-solves an instance that missed the tolerance on its
// own: FP64 GMRES with the block preconditioner and a restart length of
// 8 x the batch's (at least 240, at most 1000), cut so that the instance's
// Krylov basis stays within kFallbackBasisBytes.
static constexpr size_t kFallbackBasisBytes = (size_t)2 << 30;
static constexpr int kFallbackWorkers = 8;

static heom_solver_opts fallback_opts(const heom_batch &b, int q, const heom_solver_opts &o) {
  heom_solver_opts f = o;
  f.mode = HEOM_SOLVE_FP64;
  f.precond = HEOM_PREC_BLOCK;
  f.deflate = 0;
  f.use_x0 = 0;
  f.fallback = 0;
  f.nn = nullptr;
  const size_t vec = (size_t)(b.off[q + 1] - b.off[q]) * 16;
  const int64_t cap = (int64_t)(kFallbackBasisBytes / std::max<size_t>(2 * vec, 1));
  f.restart = (int)std::max<int64_t>(o.restart, std::min<int64_t>({std::max(8 * o.restart, 240), 1000, cap}));
  return f;
}

heom_status heom_batch_workspace_size(const heom_batch *b, const heom_solver_opts *o, size_t *bytes) {
  if (!b || !bytes) return fail(HEOM_ERR_ARG, "batch_workspace_size: NULL argument");
  heom_solver_opts d;
  if (!o) { heom_default_opts(&d); o = &d; }
  const size_t v64 = (size_t)b->n * 16, v32 = (size_t)b->n * 8;
  size_t need = v64 + 4096;  // right-hand side
  const bool jac = o->precond != HEOM_PREC_NONE;
  size_t pass1 = 0;
  if (o->mode == HEOM_SOLVE_FP32_IR) pass1 = v64 + 2 * v32 + BatchGmres<float>::bytes(*b, o->restart, jac);
  else pass1 = BatchGmres<double>::bytes(*b, o->restart, jac);
  size_t pass2 = 0;
  if (o->fallback) {
    size_t w_max = 0;
    for (int q = 0; q < b->S; ++q) {
      const heom_solver_opts f = fallback_opts(*b, q, *o);
      size_t w = 0;
      HEOM_TRY(heom_workspace_size(b->inst[q], HEOM_OP_STEADY, &f, 0, &w));
      w_max = std::max(w_max, (w + 255) & ~(size_t)255);
    }
    pass2 = (size_t)std::min(kFallbackWorkers, b->S) * w_max;
  }
  need += std::max(pass1, pass2);
  need += (size_t)b->S * sizeof(double) + 256;
  *bytes = need + 8 * 256;
  return HEOM_OK;
}

static heom_status heom_batch_steady_body(heom_batch *b, void *x_dev, const heom_solver_opts *o, heom_solver_report *r,
                              int32_t use_graph, void *ws, size_t ws_bytes, void *stream) {
  HEOM_TRY(batch_check(b));
  if (!x_dev || !o || !ws) return fail(HEOM_ERR_ARG, "batch_steady: NULL argument");
  if (o->restart < 1 || o->restart > 1000 || o->max_iter < 1 || !(o->tol > 0)) return fail(HEOM_ERR_ARG, "batch_steady: bad options");
  if (o->precond != HEOM_PREC_JACOBI && o->precond != HEOM_PREC_NONE && o->precond != HEOM_PREC_BLOCK)
    return fail(HEOM_ERR_UNSUPPORTED, "batch_steady: Jacobi, block or no preconditioning only");
  const int prec1 = o->precond;
  if (o->mode != HEOM_SOLVE_FP64 && o->mode != HEOM_SOLVE_FP32_IR) return fail(HEOM_ERR_ARG, "batch_steady: mode");
  if (o->deflate != 0) return fail(HEOM_ERR_UNSUPPORTED, "batch_steady: no deflated restarting");
  for (heom_hier *h : b->inst)
    if (h->impl->parity != 1) return fail(HEOM_ERR_ARG, "batch_steady: every instance must be even parity");
  hipStream_t s = (hipStream_t)stream;
  const int S = b->S;
  const int64_t n = b->n;
  auto t0 = std::chrono::steady_clock::now();
  WsArena arena(ws, ws_bytes);
  double2 *rhs = (double2 *)arena.take(sizeof(double2) * n);
  if (!rhs) return fail(HEOM_ERR_ARG, "batch_steady: workspace too small");
  HEOM_TRY(seg_zero<double>(rhs, n, s));
  hipLaunchKernelGGL(seg_unit_kernel, dim3((S + 255) / 256), dim3(256), 0, s, rhs, b->d_off, S);
  HEOM_HIP_CHECK(hipGetLastError());
  std::vector<int> iters(S, 0), refines(S, 0);
  std::vector<double> res(S, 0.0);
  std::vector<char> conv(S, 0);
  int64_t applies = 0;
  // With the fallback on, the batched pass gives each instance at most 20
  // restart cycles; the instances it leaves are solved on their own with the
  // full max_iter.  (The 512-instance workload: 90 % of the instances converge
  // within 480 iterations at restart 30, and a few stagnating ones would
  // otherwise keep the batch running to max_iter on a tiny active set.)
  const int pass_max = o->fallback ? std::min(o->max_iter, 20 * o->restart) : o->max_iter;
  // One pass solves the instances flagged in `want` (from zero unless
  // from_x) with preconditioner prec_pass.
  auto run_pass = [&](int prec_pass, std::vector<char> want, bool from_x) -> heom_status {
    WsArena arena2(ws, ws_bytes);
    arena2.take(sizeof(double2) * n);  // rhs
    if (o->mode == HEOM_SOLVE_FP64) {
      BatchGmres<double> gm;
      HEOM_TRY(gm.init(*b, arena2, o->restart, use_graph != 0, prec_pass));
      std::vector<int> it;
      std::vector<double> rs;
      std::vector<char> cv;
      HEOM_TRY(gm.solve(rhs, (double2 *)x_dev, want, o->tol, pass_max, 1, !from_x, it, rs, cv, applies, s));
      for (int q = 0; q < S; ++q)
        if (want[q]) { iters[q] += it[q]; res[q] = rs[q]; conv[q] = cv[q]; }
      return HEOM_OK;
    }
    double2 *r64 = (double2 *)arena2.take(sizeof(double2) * n);
    float2 *r32 = (float2 *)arena2.take(sizeof(float2) * n);
    float2 *d32 = (float2 *)arena2.take(sizeof(float2) * n);
    if (!r64 || !r32 || !d32) return fail(HEOM_ERR_ARG, "batch_steady: workspace too small");
    BatchGmres<float> gm;
    HEOM_TRY(gm.init(*b, arena2, o->restart, use_graph != 0, prec_pass));
    const std::vector<double> bn(S, 1.0);  // |e_0| = 1 for every instance
    std::vector<int> it0(S, 0);
    for (int ref = 0;; ++ref) {
      // r64 = rhs - B x (FP64) on every instance still refining
      HEOM_TRY(gm.set_active(want, s));
      HEOM_TRY(batch_apply_T<double>(*b, x_dev, r64, 1, true, s));
      ++applies;
      HEOM_TRY((axpby<double, double>(rhs, 1.0, r64, -1.0, n, s)));
      HEOM_TRY(seg_mdot<double>(*b, r64, 0, 1, r64, gm.partial, gm.hdev, s));
      HEOM_HIP_CHECK(hipMemcpyAsync(gm.pin_h, gm.hdev, sizeof(double2) * S, hipMemcpyDeviceToHost, s));
      HEOM_HIP_CHECK(hipStreamSynchronize(s));
      bool any = false;
      for (int q = 0; q < S; ++q) {
        if (!want[q]) continue;
        const double rel = std::sqrt(std::max(gm.pin_h[q].x, 0.0)) / bn[q];
        if (!std::isfinite(rel)) return fail(HEOM_ERR_NAN, "batch_steady: non-finite residual");
        res[q] = rel;
        if (rel <= o->tol) { conv[q] = 1; want[q] = 0; }
        else if (ref >= o->max_refine || it0[q] >= pass_max) want[q] = 0;
        any = any || want[q];
      }
      if (!any) break;
      // r32 = r64 / |r64| per instance, d32 = 0, inner FP32 solve, x += |r64| d32
      for (int q = 0; q < S; ++q) {
        const double nr = res[q] * bn[q];
        gm.pin_sc[q] = want[q] && nr > 0 ? 1.0 / nr : 0.0;
      }
      HEOM_HIP_CHECK(hipMemcpyAsync(gm.sdev, gm.pin_sc, sizeof(double) * S, hipMemcpyHostToDevice, s));
      HEOM_TRY((seg_scale<double, float>(*b, r64, gm.sdev, r32, s)));
      HEOM_TRY(seg_zero<float>(d32, n, s));
      std::vector<int> it_in;
      std::vector<double> res_in;
      std::vector<char> conv_in;
      const int cap = std::max(4 * o->restart, 120);
      HEOM_TRY(gm.solve(r32, d32, want, o->inner_tol, cap, 1, true, it_in, res_in, conv_in, applies, s));
      for (int q = 0; q < S; ++q) {
        if (!want[q]) { gm.pin_sc[q] = 0.0; continue; }
        iters[q] += it_in[q];
        it0[q] += it_in[q];
        ++refines[q];
        gm.pin_sc[q] = res[q] * bn[q];
      }
      HEOM_HIP_CHECK(hipMemcpyAsync(gm.sdev, gm.pin_sc, sizeof(double) * S, hipMemcpyHostToDevice, s));
      HEOM_TRY((seg_axpy<float, double>(*b, d32, gm.sdev, x_dev, s)));
    }
    return HEOM_OK;
  };
  if (!o->use_x0) HEOM_TRY(seg_zero<double>(x_dev, n, s));
  HEOM_TRY(run_pass(prec1, std::vector<char>(S, 1), o->use_x0 != 0));
  std::vector<char> fell(S, 0);
  if (o->fallback) {
    // Instances that missed the tolerance: each again from zero on its own,
    // FP64 with the block preconditioner and a longer restart (the batch
    // pass keeps one restart length for all; the hard instances are those
    // whose GMRES(m) stagnates at that length).
    HEOM_HIP_CHECK(hipStreamSynchronize(s));
    std::vector<int> ones(S, 1);
    HEOM_HIP_CHECK(hipMemcpy(b->active, ones.data(), sizeof(int) * S, hipMemcpyHostToDevice));
    const size_t off_ws = (sizeof(double2) * (size_t)n + 255) & ~(size_t)255;  // after rhs
    std::vector<int> todo;
    std::vector<heom_solver_opts> fo(S);
    size_t w_max = 0;
    for (int q = 0; q < S; ++q) {
      if (conv[q]) continue;
      fo[q] = fallback_opts(*b, q, *o);
      size_t w = 0;
      HEOM_TRY(heom_workspace_size(b->inst[q], HEOM_OP_STEADY, &fo[q], 0, &w));
      w_max = std::max(w_max, (w + 255) & ~(size_t)255);
      todo.push_back(q);
    }
    // The solves are independent and mostly small (latency-bound): up to
    // kFallbackWorkers host threads run them at once, each on its own
    // stream with its own slice of the workspace.
    const size_t avail = ws_bytes > off_ws ? ws_bytes - off_ws : 0;
    const int n_work = (int)std::min<size_t>({(size_t)kFallbackWorkers, todo.size(), w_max ? avail / w_max : 0});
    if (!todo.empty() && n_work < 1) return fail(HEOM_ERR_ARG, "batch_steady: workspace too small for the fallback pass");
    std::atomic<size_t> next{0};
    std::vector<heom_status> wst(n_work, HEOM_OK);
    std::vector<std::string> wmsg(n_work);
    std::vector<heom_solver_report> rep(S);
    std::vector<heom_status> qst(S, HEOM_OK);
    auto worker = [&](int k) {
      hipStream_t ks = nullptr;
      if (hipSetDevice(b->device) != hipSuccess || hipStreamCreateWithFlags(&ks, hipStreamNonBlocking) != hipSuccess) {
        wst[k] = HEOM_ERR_HIP;
        wmsg[k] = "batch_steady: fallback stream";
        return;
      }
      unsigned char *wk = (unsigned char *)ws + off_ws + (size_t)k * w_max;
      for (size_t i = next++; i < todo.size(); i = next++) {
        const int q = todo[i];
        std::memset(&rep[q], 0, sizeof(rep[q]));
        qst[q] = heom_steady(b->inst[q], (double2 *)x_dev + b->off[q], &fo[q], &rep[q], wk, w_max, ks);
        if (qst[q] != HEOM_OK && qst[q] != HEOM_ERR_NOT_CONVERGED) {
          wst[k] = qst[q];
          wmsg[k] = heom_last_error();
          break;
        }
      }
      if (hipStreamSynchronize(ks) != hipSuccess && wst[k] == HEOM_OK) {
        wst[k] = HEOM_ERR_HIP;
        wmsg[k] = "batch_steady: fallback stream synchronisation";
      }
      (void)hipStreamDestroy(ks);
    };
    std::vector<std::thread> pool;
    for (int k = 1; k < n_work; ++k) pool.emplace_back(worker, k);
    if (n_work > 0) worker(0);
    for (auto &t : pool) t.join();
    for (int k = 0; k < n_work; ++k)
      if (wst[k] != HEOM_OK) return fail(wst[k], wmsg[k]);
    for (int q : todo) {
      fell[q] = 1;
      iters[q] += rep[q].iterations;
      applies += rep[q].applies;
      res[q] = rep[q].true_residual;
      conv[q] = qst[q] == HEOM_OK;
    }
  }
  HEOM_HIP_CHECK(hipStreamSynchronize(s));
  std::vector<int> ones(S, 1);
  HEOM_HIP_CHECK(hipMemcpy(b->active, ones.data(), sizeof(int) * S, hipMemcpyHostToDevice));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  bool ok = true;
  for (int q = 0; q < S; ++q) {
    ok = ok && conv[q];
    if (r) {
      std::memset(&r[q], 0, sizeof(r[q]));
      r[q].status = conv[q] ? HEOM_OK : HEOM_ERR_NOT_CONVERGED;
      r[q].iterations = iters[q];
      r[q].refinements = refines[q];
      r[q].true_residual = res[q];
      r[q].seconds = secs;
      r[q].applies = applies;
      r[q].fell_back = fell[q];
    }
  }
  return ok ? HEOM_OK : fail(HEOM_ERR_NOT_CONVERGED, "batch_steady: some instances did not reach the tolerance");
}

heom_status heom_batch_steady(heom_batch *b, void *x_dev, const heom_solver_opts *o, heom_solver_report *r,
                              int32_t use_graph, void *ws, size_t ws_bytes, void *stream) {
  return guarded([&] { return heom_batch_steady_body(b, x_dev, o, r, use_graph, ws, ws_bytes, stream); });
}

}  // extern "C"
