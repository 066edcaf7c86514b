// Wave formulation of the Liouvillian apply, shared by the single-hierarchy
// kernels (apply.hip) and the batched launch (batch.hip).
#pragma once

#include "device_common.h"
#include "internal.h"

namespace heom {

template <typename T>
struct ApplyParams {
  using T2 = typename Cplx<T>::t;
  const int4 *tasks;
  int64_t n_tasks;
  const int4 *groups;
  const int2 *gedges;
  const T2 *decay;
  const int32_t *ell_cnt;
  const int32_t *ell_col;
  const T2 *ell_val;
  const int32_t *op_slots;  // per operator: padded ELL width (entries beyond a row's count are zero)
  int slots;
  // compact operator tables (wave kernel)
  const int32_t *c_meta;
  const int32_t *c_col;
  const T2 *c_val;
  int n_centries;
  const T2 *hdiag;
  int tpw;  // tasks per wave
  int xchunk;  // XCD remap super-chunk in blocks (multiple of 8; 0 = off)
  const int32_t *coef_op;
  const T2 *coef;
  int n_coef;  // coefficient entries (coef holds two per entry)
  const T2 *x;
  const T2 *kvec;
  T kc;
  T2 *y;
  int d;
  int R;
  const T2 *shifts;
  T2 shift0;
  int border;
  // self group on the matrix cores (d = 16; the kernel instantiation with
  // MF set): H with its diagonal zeroed, row-major
  const T2 *hoff;
  int hmfma;  // launch choice, read on the host
  // epilogue: y = eacc * acc + sum_j ec[j] * ev[j] (ev[j] may alias y), and
  // when y2 is set also y2 = eacc2 * acc + sum_j ec2[j] * ev[j]
  int epi;
  const T2 *ev[4];
  T ec[4];
  T eacc;
  T2 *y2;
  T ec2[4];
  T eacc2;
};

// Stores one output element, through the epilogue when EPI is set and the
// launch asks for one (kernels built without EPI store plainly).
template <bool EPI, typename T>
__device__ __forceinline__ void store_out(const ApplyParams<T> &P, int64_t idx, typename Cplx<T>::t v) {
  if constexpr (!EPI) {
    // a streaming store: y is not read again by this launch, and keeping it
    // out of the way leaves L2 to the neighbour blocks (two-orbital tier 4:
    // 0.918 -> 0.906 ms FP64, 1.5 % less fetched)
    T *q = reinterpret_cast<T *>(&P.y[idx]);
    __builtin_nontemporal_store(v.x, q);
    __builtin_nontemporal_store(v.y, q + 1);
    return;
  }
  if (!P.epi) {
    P.y[idx] = v;
    return;
  }
  typename Cplx<T>::t r{P.eacc * v.x, P.eacc * v.y};
  typename Cplx<T>::t r2{P.eacc2 * v.x, P.eacc2 * v.y};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (!P.ev[j]) continue;
    const typename Cplx<T>::t q = P.ev[j][idx];
    r.x = fma(P.ec[j], q.x, r.x);
    r.y = fma(P.ec[j], q.y, r.y);
    r2.x = fma(P.ec2[j], q.x, r2.x);
    r2.y = fma(P.ec2[j], q.y, r2.y);
  }
  P.y[idx] = r;
  if (P.y2) P.y2[idx] = r2;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int D>
struct WaveShape {
  static constexpr int DD = D * D;
  static constexpr int EPL = (DD + 63) / 64;   // elements per lane
  static constexpr bool FULL = DD % 64 == 0;   // no masked tail
  static constexpr bool UJ = 64 % D == 0;      // column index the same for all of a lane's elements
  static __device__ __forceinline__ bool on(int lane, int s) { return FULL || lane + 64 * s < DD; }
  static __device__ __forceinline__ int col(int lane, int s) { return UJ ? lane % D : (lane + 64 * s) % D; }
};

// Element of the d x d block that lane `lane` holds in slot s: lane + 64 s,
// or, for FP32 blocks that fill whole waves with an even number of elements
// per lane, pairs of neighbouring elements 2 lane + (s & 1) + 128 (s >> 1),
// so that a lane's two elements are one 16-byte access like an FP64 element.
template <typename T, int D>
struct LaneMap {
  using W = WaveShape<D>;
  static constexpr bool PAIR = sizeof(T) == 4 && W::EPL % 2 == 0 && W::FULL;
  static __device__ __forceinline__ int elem(int lane, int s) {
    return PAIR ? 2 * lane + (s & 1) + 128 * (s >> 1) : lane + 64 * s;
  }
  static __device__ __forceinline__ bool on(int lane, int s) { return PAIR ? true : W::on(lane, s); }
  static __device__ __forceinline__ int col(int lane, int s) { return PAIR ? elem(lane, s) % D : W::col(lane, s); }
};

template <typename T, int D, bool FUSE>
__device__ __forceinline__ void load_block(const ApplyParams<T> &P, int64_t b, int lane,
                                           typename Cplx<T>::t (&v)[WaveShape<D>::EPL]) {
  using W = WaveShape<D>;
  using M = LaneMap<T, D>;
  constexpr int DD = D * D;
  const typename Cplx<T>::t *xb = P.x + b * DD;
  if constexpr (M::PAIR) {
#pragma unroll
    for (int s = 0; s < W::EPL; s += 2) {
      const float4 q = *reinterpret_cast<const float4 *>(xb + M::elem(lane, s));
      v[s] = typename Cplx<T>::t{q.x, q.y};
      v[s + 1] = typename Cplx<T>::t{q.z, q.w};
    }
    if (FUSE) {
      const typename Cplx<T>::t *kb = P.kvec + b * DD;
#pragma unroll
      for (int s = 0; s < W::EPL; s += 2) {
        const float4 q = *reinterpret_cast<const float4 *>(kb + M::elem(lane, s));
        v[s].x = fma(P.kc, q.x, v[s].x);
        v[s].y = fma(P.kc, q.y, v[s].y);
        v[s + 1].x = fma(P.kc, q.z, v[s + 1].x);
        v[s + 1].y = fma(P.kc, q.w, v[s + 1].y);
      }
    }
  } else {
#pragma unroll
    for (int s = 0; s < W::EPL; ++s) v[s] = W::on(lane, s) ? xb[lane + 64 * s] : typename Cplx<T>::t{0, 0};
    if (FUSE) {
      const typename Cplx<T>::t *kb = P.kvec + b * DD;
#pragma unroll
      for (int s = 0; s < W::EPL; ++s) {
        if (!W::on(lane, s)) continue;
        const typename Cplx<T>::t q = kb[lane + 64 * s];
        v[s].x = fma(P.kc, q.x, v[s].x);
        v[s].y = fma(P.kc, q.y, v[s].y);
      }
    }
  }
}

// acc += w (cl O X + cr X O) for the coefficient pair and operator of
// coefficient entry cid, with X a d x d block staged in LDS (row-major) and
// acc in the lane layout of LaneMap.  O gathers through the compact tables.
template <typename T, int D>
__device__ __forceinline__ void op_terms(const ApplyParams<T> &P, int cid, T w, int lane,
                                         const typename Cplx<T>::t *X, const typename Cplx<T>::t *tval,
                                         const int *tcol, typename Cplx<T>::t (&acc)[WaveShape<D>::EPL]) {
  using T2 = typename Cplx<T>::t;
  constexpr int EPL = WaveShape<D>::EPL;
  const int op = P.coef_op[cid];
  const int off = P.c_meta[3 * op], ns = P.c_meta[3 * op + 1], isreal = P.c_meta[3 * op + 2];
  if (ns <= 0) return;
  T2 cl = P.coef[2 * cid], cr = P.coef[2 * cid + 1];
  cl.x *= w; cl.y *= w; cr.x *= w; cr.y *= w;
#pragma unroll
  for (int s = 0; s < EPL; ++s) {
    if (!LaneMap<T, D>::on(lane, s)) continue;
    const int i = LaneMap<T, D>::elem(lane, s) / D;
    const int j = LaneMap<T, D>::col(lane, s);
    const int rbase = off + (D + j) * ns;
    const int lbase = off + i * ns;
    T2 L{0, 0}, Rv{0, 0};
    if (isreal) {
#pragma unroll 1
      for (int t = 0; t < ns; ++t) {
        const T vl = tval[lbase + t].x, vr = tval[rbase + t].x;
        const T2 bl = X[tcol[lbase + t] * D + j];
        const T2 br = X[i * D + tcol[rbase + t]];
        L.x = fma(vl, bl.x, L.x); L.y = fma(vl, bl.y, L.y);
        Rv.x = fma(vr, br.x, Rv.x); Rv.y = fma(vr, br.y, Rv.y);
      }
    } else {
#pragma unroll 1
      for (int t = 0; t < ns; ++t) {
        L = cfma(tval[lbase + t], X[tcol[lbase + t] * D + j], L);
        Rv = cfma(X[i * D + tcol[rbase + t]], tval[rbase + t], Rv);
      }
    }
    acc[s] = cfma(cl, L, acc[s]);
    acc[s] = cfma(cr, Rv, acc[s]);
  }
}

typedef double mfma_d4 __attribute__((ext_vector_type(4)));
typedef float mfma_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ mfma_d4 mfma16x16x4(double a, double b, mfma_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ mfma_f4 mfma16x16x4(float a, float b, mfma_f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// The H terms of the self group (the first line of eq:HEOM) on the matrix
// cores, d = 16: acc += cl H' X + cr X H' with H' = H without its diagonal
// (the diagonal is applied with the decay) and X staged row-major in LDS.
// Each complex product is four real 16 x 16 x 16 products, four K-steps of
// the 16 x 16 x 4 MFMA each.  Operand layout of that instruction (both
// precisions): lane l holds A[l % 16][l / 16] and B[l / 16][l % 16] of the
// K-step.  Result: FP64 lane l, register r holds row l / 16 + 4 r, column
// l % 16 -- the element of slot r in the FP64 lane layout; FP32 holds row
// 4 (l / 16) + r, column l % 16, which goes through LDS to the lane layout.
template <typename T>
__device__ __forceinline__ void self_h_mfma16(const ApplyParams<T> &P, int cid, int lane, typename Cplx<T>::t *X,
                                              typename Cplx<T>::t (&acc)[WaveShape<16>::EPL]) {
  using T2 = typename Cplx<T>::t;
  using V4 = T __attribute__((ext_vector_type(4)));
  const T2 cl = P.coef[2 * cid], cr = P.coef[2 * cid + 1];
  const int q = lane >> 4, c = lane & 15;
  // two passes (H' X, then X H') so that only one complex accumulator pair
  // is live at a time
  T2 v[4];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    V4 Pr = {0, 0, 0, 0}, Pi = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int k = 4 * ks + q;
      // side 0: A = H'[c][k], B = X[k][c]; side 1: A = X[c][k], B = H'[k][c]
      const T2 a = side == 0 ? P.hoff[c * 16 + k] : X[c * 16 + k];
      const T2 b = side == 0 ? X[k * 16 + c] : P.hoff[k * 16 + c];
      Pr = mfma16x16x4(a.x, b.x, Pr);
      Pr = mfma16x16x4(-a.y, b.y, Pr);
      Pi = mfma16x16x4(a.x, b.y, Pi);
      Pi = mfma16x16x4(a.y, b.x, Pi);
    }
    const T2 cf = side == 0 ? cl : cr;
    if constexpr (sizeof(T) == 8) {
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = cfma(cf, T2{Pr[r], Pi[r]}, acc[r]);
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = side == 0 ? cmul(cf, T2{Pr[r], Pi[r]}) : cfma(cf, T2{Pr[r], Pi[r]}, v[r]);
    }
  }
  if constexpr (sizeof(T) == 4) {
    wave_sync();  // every lane has read its operands from X
#pragma unroll
    for (int r = 0; r < 4; ++r) X[(4 * q + r) * 16 + c] = v[r];
    wave_sync();
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[s] = cadd(acc[s], X[LaneMap<T, 16>::elem(lane, s)]);
  }
}

// One group's terms, with the group sum u (in the lane layout) in hand: the
// decay and the diagonal of H for the self group, then cl O u + cr u O
// through the wave's LDS slice (and the trace of ADO 0 for the bordered
// operator).
template <typename T, int D, bool MF = false>
__device__ __forceinline__ void group_terms(const ApplyParams<T> &P, const int4 &gr, int64_t a, int lane,
                                            const typename Cplx<T>::t (&u)[WaveShape<D>::EPL],
                                            typename Cplx<T>::t *buf, const typename Cplx<T>::t *tval,
                                            const int *tcol, const typename Cplx<T>::t *thd,
                                            typename Cplx<T>::t (&acc)[WaveShape<D>::EPL],
                                            typename Cplx<T>::t &trace) {
  using T2 = typename Cplx<T>::t;
  constexpr int EPL = WaveShape<D>::EPL;
  if (gr.w) {
    // self group: u = x_a.  -(c_a - z) x - i (H_ii - H_jj) x
    const T2 z = P.shifts ? P.shifts[0] : P.shift0;
    const T2 c = csub(P.decay[a], z);
#pragma unroll
    for (int s = 0; s < EPL; ++s) {
      const T2 dh = csub(thd[LaneMap<T, D>::elem(lane, s) / D], thd[LaneMap<T, D>::col(lane, s)]);
      const T2 f{c.x - dh.y, c.y + dh.x};  // c + i (H_ii - H_jj)
      acc[s] = csub(acc[s], cmul(f, u[s]));
    }
  }
  const int cid = gr.z;
  const int op = P.coef_op[cid];
  const int ns = P.c_meta[3 * op + 1];
  const bool need_trace = gr.w && P.border && a == 0;
  if (ns > 0 || need_trace) {
#pragma unroll
    for (int s = 0; s < EPL; ++s)
      if (LaneMap<T, D>::on(lane, s)) buf[LaneMap<T, D>::elem(lane, s)] = u[s];
    wave_sync();
    if (need_trace && lane == 0)
      for (int i = 0; i < D; ++i) trace = cadd(trace, buf[i * (D + 1)]);
    if constexpr (D == 16 && MF) {
      if (gr.w) {
        self_h_mfma16<T>(P, cid, lane, buf, acc);
        wave_sync();
        return;
      }
    }
    op_terms<T, D>(P, cid, (T)1, lane, buf, tval, tcol, acc);
    wave_sync();
  }
}

// The groups of one task added to acc, then acc written to the task's output
// ADO (see wave_task).
// PAIRS = false streams multi-edge groups one block at a time (fewer
// registers; for callers that hold other blocks in registers meanwhile).
template <typename T, int D, bool FUSE, bool PAIRS = true, bool MF = false>
__device__ __forceinline__ void wave_task_add(const ApplyParams<T> &P, int64_t task, int lane, typename Cplx<T>::t *buf,
                                              const typename Cplx<T>::t *tval, const int *tcol,
                                              const typename Cplx<T>::t *thd,
                                              typename Cplx<T>::t (&acc)[WaveShape<D>::EPL]) {
  using T2 = typename Cplx<T>::t;
  using W = WaveShape<D>;
  constexpr int DD = D * D;
  constexpr int EPL = W::EPL;
  const int4 tk = P.tasks[task];
  const int64_t a = tk.x;
  const int flags = tk.w;
  const int64_t abase = a * DD;
  T2 trace{0, 0};
  int g = tk.y;
  if (g < tk.z) {
    int4 gr = P.groups[g];
    T2 vnext[EPL];
    load_block<T, D, FUSE>(P, P.gedges[gr.x].x, lane, vnext);
    for (; g < tk.z; ++g) {
      T2 u[EPL];
      {
        const T w0 = (T)P.gedges[gr.x].y;
#pragma unroll
        for (int s = 0; s < EPL; ++s) u[s] = T2{w0 * vnext[s].x, w0 * vnext[s].y};
      }
      int4 grn = gr;
      if (g + 1 < tk.z) {  // prefetch the next group's first neighbour block
        grn = P.groups[g + 1];
        load_block<T, D, FUSE>(P, P.gedges[grn.x].x, lane, vnext);
      }
      int e = gr.x + 1;
      for (; PAIRS && e + 1 < gr.y; e += 2) {
        const int2 e0 = P.gedges[e], e1 = P.gedges[e + 1];
        T2 v0[EPL], v1[EPL];
        load_block<T, D, FUSE>(P, e0.x, lane, v0);
        load_block<T, D, FUSE>(P, e1.x, lane, v1);
        const T w0 = (T)e0.y, w1 = (T)e1.y;
#pragma unroll
        for (int s = 0; s < EPL; ++s) {
          u[s].x = fma(w0, v0[s].x, fma(w1, v1[s].x, u[s].x));
          u[s].y = fma(w0, v0[s].y, fma(w1, v1[s].y, u[s].y));
        }
      }
      if constexpr (PAIRS) {
        // at most one edge is left
        if (e < gr.y) {
          const int2 e0 = P.gedges[e];
          T2 v0[EPL];
          load_block<T, D, FUSE>(P, e0.x, lane, v0);
          const T w0 = (T)e0.y;
#pragma unroll
          for (int s = 0; s < EPL; ++s) {
            u[s].x = fma(w0, v0[s].x, u[s].x);
            u[s].y = fma(w0, v0[s].y, u[s].y);
          }
        }
      } else {
        for (; e < gr.y; ++e) {
          const int2 e0 = P.gedges[e];
          T2 v0[EPL];
          load_block<T, D, FUSE>(P, e0.x, lane, v0);
          const T w0 = (T)e0.y;
#pragma unroll
          for (int s = 0; s < EPL; ++s) {
            u[s].x = fma(w0, v0[s].x, u[s].x);
            u[s].y = fma(w0, v0[s].y, u[s].y);
          }
        }
      }
      group_terms<T, D, MF>(P, gr, a, lane, u, buf, tval, tcol, thd, acc, trace);
      gr = grn;
    }
  }
#pragma unroll
  for (int s = 0; s < EPL; ++s) {
    if (!LaneMap<T, D>::on(lane, s)) continue;
    T2 v = acc[s];
    if (s == 0 && lane == 0 && P.border && a == 0 && (flags & TASK_DIAG)) v = trace;  // element 0 in both maps
    const int64_t idx = abase + LaneMap<T, D>::elem(lane, s);
    store_out<true>(P, idx, v);
  }
}

// One output ADO (task) of the pull kernel, as a single body: the task's
// groups stream their neighbour blocks (the next group's first block
// prefetched while the current one is finished, multi-edge groups two blocks
// at a time), each group sum is staged in the wave's LDS slice `buf`, and the
// operator products gather from it through the compact tables (tval, tcol)
// and the H diagonal (thd) held in LDS.  It computes what wave_task_add does;
// the split form (op_terms / group_terms, which the slab kernel uses)
// compiled to a pull apply 10 % slower on the
// two-orbital tier-4 model (1.39 against 1.25 ms FP64, 0.87 against 0.76 ms
// FP32, same box), so the hot path keeps this form.
template <typename T, int D, bool FUSE, bool MF = false, bool EPI = false, bool LT = false>
__device__ __forceinline__ void wave_task_pull(const ApplyParams<T> &P, int64_t task, int lane, typename Cplx<T>::t *buf,
                                          const typename Cplx<T>::t *tval, const int *tcol,
                                          const typename Cplx<T>::t *thd, const int *cmeta = nullptr,
                                          const typename Cplx<T>::t *cfs = nullptr) {
  using T2 = typename Cplx<T>::t;
  using W = WaveShape<D>;
  constexpr int DD = D * D;
  constexpr int EPL = W::EPL;
  const int4 tk = P.tasks[task];
  const int64_t a = tk.x;
  const int flags = tk.w;
  const int64_t abase = a * DD;
  T2 acc[EPL];
#pragma unroll
  for (int s = 0; s < EPL; ++s)
    acc[s] = (flags & TASK_ACC) && LaneMap<T, D>::on(lane, s) ? P.y[abase + LaneMap<T, D>::elem(lane, s)] : T2{0, 0};
  T2 trace{0, 0};
  // LT: the self group's c_a - z is read here, ahead of the block loads
  T2 cself{0, 0};
  if constexpr (LT) cself = csub(P.decay[a], P.shifts ? P.shifts[0] : P.shift0);
  int g = tk.y;
  if (g < tk.z) {
    // LT: the task's group entries and edges sit one per lane (at most 64
    // of each, checked on the host) and are read with readlane, so no
    // dependent table load stalls the group loop.
    int4 lg{0, 0, 0, 0};
    int2 le{0, 0};
    int e_first = 0;
    if constexpr (LT) {
      const int ng = tk.z - tk.y;
      if (lane < ng) lg = P.groups[tk.y + lane];
      e_first = __builtin_amdgcn_readlane(lg.x, 0);
      const int e_end = __builtin_amdgcn_readlane(lg.y, ng - 1);
      if (lane < e_end - e_first) le = P.gedges[e_first + lane];
    }
    auto group_at = [&](int gg) -> int4 {
      if constexpr (LT) {
        const int k = gg - tk.y;
        return make_int4(__builtin_amdgcn_readlane(lg.x, k), __builtin_amdgcn_readlane(lg.y, k),
                         __builtin_amdgcn_readlane(lg.z, k), __builtin_amdgcn_readlane(lg.w, k));
      } else {
        return P.groups[gg];
      }
    };
    auto edge_at = [&](int e) -> int2 {
      if constexpr (LT) {
        const int k = e - e_first;
        return make_int2(__builtin_amdgcn_readlane(le.x, k), __builtin_amdgcn_readlane(le.y, k));
      } else {
        return P.gedges[e];
      }
    };
    int4 gr = group_at(g);
    T2 vnext[EPL];
    load_block<T, D, FUSE>(P, edge_at(gr.x).x, lane, vnext);
    for (; g < tk.z; ++g) {
      T2 u[EPL];
      {
        const T w0 = (T)edge_at(gr.x).y;
#pragma unroll
        for (int s = 0; s < EPL; ++s) u[s] = T2{w0 * vnext[s].x, w0 * vnext[s].y};
      }
      int4 grn = gr;
      if constexpr (LT) {
        // prefetch the next group's first neighbour block; the last group
        // loads its own first block again (a cache hit), so that no branch
        // joins ahead of the edge loop and the prefetch stays in flight
        const bool more = g + 1 < tk.z;
        grn = group_at(more ? g + 1 : g);
        load_block<T, D, FUSE>(P, edge_at(grn.x).x, lane, vnext);
      } else if (g + 1 < tk.z) {  // prefetch the next group's first neighbour block
        grn = P.groups[g + 1];
        load_block<T, D, FUSE>(P, P.gedges[grn.x].x, lane, vnext);
      }
      int e = gr.x + 1;
      for (; e + 1 < gr.y; e += 2) {
        const int2 e0 = edge_at(e), e1 = edge_at(e + 1);
        T2 v0[EPL], v1[EPL];
        load_block<T, D, FUSE>(P, e0.x, lane, v0);
        load_block<T, D, FUSE>(P, e1.x, lane, v1);
        const T w0 = (T)e0.y, w1 = (T)e1.y;
#pragma unroll
        for (int s = 0; s < EPL; ++s) {
          u[s].x = fma(w0, v0[s].x, fma(w1, v1[s].x, u[s].x));
          u[s].y = fma(w0, v0[s].y, fma(w1, v1[s].y, u[s].y));
        }
      }
      if (e < gr.y) {
        const int2 e0 = edge_at(e);
        T2 v0[EPL];
        load_block<T, D, FUSE>(P, e0.x, lane, v0);
        const T w0 = (T)e0.y;
#pragma unroll
        for (int s = 0; s < EPL; ++s) {
          u[s].x = fma(w0, v0[s].x, u[s].x);
          u[s].y = fma(w0, v0[s].y, u[s].y);
        }
      }
      if (gr.w) {
        // self group: u = x_a.  -(c_a - z) x - i (H_ii - H_jj) x
        T2 c;
        if constexpr (LT) c = cself;
        else c = csub(P.decay[a], P.shifts ? P.shifts[0] : P.shift0);
#pragma unroll
        for (int s = 0; s < EPL; ++s) {
          const T2 dh = csub(thd[LaneMap<T, D>::elem(lane, s) / D], thd[LaneMap<T, D>::col(lane, s)]);
          const T2 f{c.x - dh.y, c.y + dh.x};  // c + i (H_ii - H_jj)
          acc[s] = csub(acc[s], cmul(f, u[s]));
        }
      }
      const int cid = gr.z;
      int off, ns, isreal;
      if constexpr (LT) {  // the operator's table slot, width and realness, packed in LDS
        const int m = cmeta[cid];
        off = m & 0xfffff;
        ns = (m >> 20) & 0x3ff;
        isreal = (m >> 30) & 1;
      } else {
        const int op = P.coef_op[cid];
        off = P.c_meta[3 * op];
        ns = P.c_meta[3 * op + 1];
        isreal = P.c_meta[3 * op + 2];
      }
      const bool need_trace = gr.w && P.border && a == 0;
      if (ns > 0 || need_trace) {
#pragma unroll
        for (int s = 0; s < EPL; ++s)
          if (LaneMap<T, D>::on(lane, s)) buf[LaneMap<T, D>::elem(lane, s)] = u[s];
        wave_sync();
        if (need_trace && lane == 0)
          for (int i = 0; i < D; ++i) trace = cadd(trace, buf[i * (D + 1)]);
        bool on_mfma = false;
        if constexpr (MF && D == 16) {
          if (gr.w) {  // the H terms on the matrix cores
            self_h_mfma16<T>(P, cid, lane, buf, acc);
            on_mfma = true;
          }
        }
        if (ns > 0 && !on_mfma) {
          const T2 cl = LT ? cfs[2 * cid] : P.coef[2 * cid], cr = LT ? cfs[2 * cid + 1] : P.coef[2 * cid + 1];
#pragma unroll
          for (int s = 0; s < EPL; ++s) {
            if (!LaneMap<T, D>::on(lane, s)) continue;
            const int i = LaneMap<T, D>::elem(lane, s) / D;
            const int j = LaneMap<T, D>::col(lane, s);
            const int rbase = off + (D + j) * ns;
            const int lbase = off + i * ns;
            T2 L{0, 0}, Rv{0, 0};
            if (isreal) {
#pragma unroll 1
              for (int t = 0; t < ns; ++t) {
                const T vl = tval[lbase + t].x, vr = tval[rbase + t].x;
                const T2 bl = buf[tcol[lbase + t] * D + j];
                const T2 br = buf[i * D + tcol[rbase + t]];
                L.x = fma(vl, bl.x, L.x); L.y = fma(vl, bl.y, L.y);
                Rv.x = fma(vr, br.x, Rv.x); Rv.y = fma(vr, br.y, Rv.y);
              }
            } else {
#pragma unroll 1
              for (int t = 0; t < ns; ++t) {
                L = cfma(tval[lbase + t], buf[tcol[lbase + t] * D + j], L);
                Rv = cfma(buf[i * D + tcol[rbase + t]], tval[rbase + t], Rv);
              }
            }
            acc[s] = cfma(cl, L, acc[s]);
            acc[s] = cfma(cr, Rv, acc[s]);
          }
        }
        wave_sync();
      }
      gr = grn;
    }
  }
#pragma unroll
  for (int s = 0; s < EPL; ++s) {
    if (!LaneMap<T, D>::on(lane, s)) continue;
    T2 v = acc[s];
    if (s == 0 && lane == 0 && P.border && a == 0 && (flags & TASK_DIAG)) v = trace;  // element 0 in both maps
    const int64_t idx = abase + LaneMap<T, D>::elem(lane, s);
    store_out<EPI>(P, idx, v);
  }
}

// One output ADO (task) of the wave formulation, computed by one wavefront:
// the task's groups stream their neighbour blocks (the next group's first
// block prefetched while the current one is finished, multi-edge groups two
// blocks at a time), each group sum is staged in the wave's LDS slice `buf`,
// and the operator products gather from it through the compact tables
// (tval, tcol) and the H diagonal (thd) held in LDS.  A task flagged
// TASK_ACC adds to the output instead of overwriting it.
template <typename T, int D, bool FUSE, bool PAIRS = true, bool MF = false, bool EPI = false, bool LT = false>
__device__ __forceinline__ void wave_task(const ApplyParams<T> &P, int64_t task, int lane, typename Cplx<T>::t *buf,
                                          const typename Cplx<T>::t *tval, const int *tcol,
                                          const typename Cplx<T>::t *thd, const int *cmeta = nullptr,
                                          const typename Cplx<T>::t *cfs = nullptr) {
  if constexpr (PAIRS) {
    wave_task_pull<T, D, FUSE, MF, EPI, LT>(P, task, lane, buf, tval, tcol, thd, cmeta, cfs);
    return;
  }
  using T2 = typename Cplx<T>::t;
  constexpr int DD = D * D;
  constexpr int EPL = WaveShape<D>::EPL;
  const int4 tk = P.tasks[task];
  const int64_t abase = (int64_t)tk.x * DD;
  T2 acc[EPL];
#pragma unroll
  for (int s = 0; s < EPL; ++s)
    acc[s] = (tk.w & TASK_ACC) && LaneMap<T, D>::on(lane, s) ? P.y[abase + LaneMap<T, D>::elem(lane, s)] : T2{0, 0};
  wave_task_add<T, D, FUSE, PAIRS, MF>(P, task, lane, buf, tval, tcol, thd, acc);
}

}  // namespace heom
