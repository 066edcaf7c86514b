// Matrix-free HEOM Liouvillian apply (eq:HEOM), y = (M + shift) x.
//
// Every output ADO a is one task, and a task is a run of edge groups.  A
// group names one operator O (H, a bosonic V, or a fermionic d / d^dagger)
// and one coefficient pair (cl, cr) -- the superoperator A, B, C or D of
// eq:HEOM with the parity projector folded in -- and contributes
//     cl * O u + cr * u O,    u = sum_e w_e x_{b_e}
// where w_e is the edge's integer multiplier (bosonic multiplicity or
// fermionic reorder sign).  All fermionic "up" terms of an ADO that share
// d^{nubar} form a single group, so the operator product is done once per
// distinct operator rather than once per neighbour.  The self group
// (op H, cl = -i, cr = +i) also carries the decay -(c_a - z) x_a.
// Operators are stored in ELL form: the signed-permutation coupling
// operators of fermionic models cost one gather per element.
//
// Two kernels:
//   wave kernel   (d in {8, 16}, one right-hand side): one wavefront per
//                 task; neighbour blocks are streamed with coalesced loads
//                 into registers, the group sum u is staged once in the
//                 wave's own LDS slice, and the operator gathers read LDS.
//   cell kernel   (any d <= 32, any number of right-hand sides): one thread
//                 per (i, j, r) cell, gathers straight from global memory.
// Layout: x, y are [N][d][d][R] complex, R innermost.
#include "device_common.h"
#include "internal.h"

namespace heom {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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
  const T2 *x;
  const T2 *kvec;
  T kc;
  T2 *y;
  int d;
  int R;
  const T2 *shifts;
  T2 shift0;
  int border;
};

// ----------------------------------------------------------------- wave kernel
template <int D>
struct WaveShape {
  static constexpr int DD = D * D;
  static constexpr int EPL = (DD + 63) / 64;   // elements per lane
  static constexpr bool FULL = DD % 64 == 0;   // no masked tail
  static constexpr bool UJ = 64 % D == 0;      // column index the same for all of a lane's elements
  static __device__ __forceinline__ bool on(int lane, int s) { return FULL || lane + 64 * s < DD; }
  static __device__ __forceinline__ int col(int lane, int s) { return UJ ? lane % D : (lane + 64 * s) % D; }
};

template <typename T, int D, bool FUSE>
__device__ __forceinline__ void load_block(const ApplyParams<T> &P, int64_t b, int lane,
                                           typename Cplx<T>::t (&v)[WaveShape<D>::EPL]) {
  using W = WaveShape<D>;
  constexpr int DD = D * D;
  const typename Cplx<T>::t *xb = P.x + b * DD;
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

// One wave processes tasks first, first + 4, ... (tpw of them).  Blocks are
// remapped inside super-chunks of xchunk blocks so that each XCD (block b
// runs on XCD b % 8) walks a contiguous run of tasks, which share parents.  Within a
// task the next group's first neighbour block is prefetched while the
// current group is finished; multi-edge groups stream two blocks at a time.
template <typename T, int D, bool FUSE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WaveShape<D>::EPL > 4 ? 2 : 4)))
apply_wave_kernel(ApplyParams<T> P) {
  using T2 = typename Cplx<T>::t;
  using W = WaveShape<D>;
  constexpr int DD = D * D;
  constexpr int EPL = W::EPL;
  extern __shared__ __align__(16) unsigned char smem[];
  T2 *sbuf = reinterpret_cast<T2 *>(smem);              // [4][DD] group staging, one slice per wave
  T2 *tval = sbuf + 4 * DD;                             // compact operator values
  int *tcol = reinterpret_cast<int *>(tval + P.n_centries);
  // H diagonal, after the column table (16-byte aligned)
  T2 *thd = reinterpret_cast<T2 *>((reinterpret_cast<uintptr_t>(tcol + P.n_centries) + 15) & ~(uintptr_t)15);
  for (int e = threadIdx.x; e < P.n_centries; e += 256) {
    tval[e] = P.c_val[e];
    tcol[e] = P.c_col[e];
  }
  if (threadIdx.x < D) thd[threadIdx.x] = P.hdiag[threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  // the task index is uniform across the wave: keep every table lookup scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  T2 *buf = sbuf + wave * DD;
  int64_t blk = blockIdx.x;
  if (P.xchunk > 0 && (int64_t)(blockIdx.x / P.xchunk + 1) * P.xchunk <= (int64_t)gridDim.x) {
    // XCD-aware remap inside super-chunks of xchunk blocks: block b runs on
    // XCD b % 8, which then walks a contiguous slice of the super-chunk
    const int64_t sup = blockIdx.x / P.xchunk, r = blockIdx.x % P.xchunk;
    blk = sup * P.xchunk + (r % 8) * (P.xchunk / 8) + r / 8;
  }
  const int64_t first = (blk * 4 * P.tpw) + wave;
  for (int it = 0; it < P.tpw; ++it) {
    const int64_t task = first + 4 * it;
    if (task >= P.n_tasks) break;
    const int4 tk = P.tasks[task];
    const int64_t a = tk.x;
    const int flags = tk.w;
    const int64_t abase = a * DD;
    T2 acc[EPL];
#pragma unroll
    for (int s = 0; s < EPL; ++s) acc[s] = (flags & TASK_ACC) && W::on(lane, s) ? P.y[abase + lane + 64 * s] : T2{0, 0};
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
        for (; e + 1 < gr.y; e += 2) {
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
        if (gr.w) {
          // self group: u = x_a.  -(c_a - z) x - i (H_ii - H_jj) x
          const T2 z = P.shifts ? P.shifts[0] : P.shift0;
          const T2 c = csub(P.decay[a], z);
#pragma unroll
          for (int s = 0; s < EPL; ++s) {
            const T2 dh = csub(thd[(lane + 64 * s) / D], thd[W::col(lane, s)]);
            const T2 f{c.x - dh.y, c.y + dh.x};  // c + i (H_ii - H_jj)
            acc[s] = csub(acc[s], cmul(f, u[s]));
          }
        }
        const int cid = gr.z;
        const int op = P.coef_op[cid];
        const int off = P.c_meta[3 * op], ns = P.c_meta[3 * op + 1], isreal = P.c_meta[3 * op + 2];
        const bool need_trace = gr.w && P.border && a == 0;
        if (ns > 0 || need_trace) {
#pragma unroll
          for (int s = 0; s < EPL; ++s)
            if (W::on(lane, s)) buf[lane + 64 * s] = u[s];
          wave_sync();
          if (need_trace && lane == 0)
            for (int i = 0; i < D; ++i) trace = cadd(trace, buf[i * (D + 1)]);
          if (ns > 0) {
            const T2 cl = P.coef[2 * cid], cr = P.coef[2 * cid + 1];
#pragma unroll
            for (int s = 0; s < EPL; ++s) {
              if (!W::on(lane, s)) continue;
              const int i = (lane + 64 * s) / D;
              const int j = W::col(lane, s);
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
      if (!W::on(lane, s)) continue;
      T2 v = acc[s];
      if (s == 0 && lane == 0 && P.border && a == 0 && (flags & TASK_DIAG)) v = trace;
      P.y[abase + lane + 64 * s] = v;
    }
  }
}

// ----------------------------------------------------------------- cell kernel
template <typename T, int D>
__global__ void __launch_bounds__(256) apply_cell_kernel(ApplyParams<T> P) {
  using T2 = typename Cplx<T>::t;
  const int d = D > 0 ? D : P.d;
  const int R = P.R;
  const int cells = d * d * R;
  int64_t task;
  int cell, cell_stride;
  if (cells <= 256) {
    const int tpb = 256 / cells;
    const int lt = threadIdx.x / cells;
    if (lt >= tpb) return;
    task = (int64_t)blockIdx.x * tpb + lt;
    cell = threadIdx.x - lt * cells;
    cell_stride = cells;
  } else {
    task = blockIdx.x;
    cell = threadIdx.x;
    cell_stride = 256;
  }
  if (task >= P.n_tasks) return;
  const int4 tk = P.tasks[task];
  const int64_t a = tk.x;
  const int flags = tk.w;
  const int dR = d * R;
  for (; cell < cells; cell += cell_stride) {
    const int i = cell / dR;
    const int rem = cell - i * dR;
    const int j = rem / R;
    const int r = rem - j * R;
    auto in = [&](int64_t b, int ii, int jj) -> T2 {
      const int64_t idx = ((b * d + ii) * d + jj) * R + r;
      T2 v = P.x[idx];
      if (P.kvec) {
        const T2 k = P.kvec[idx];
        v.x = fma(P.kc, k.x, v.x);
        v.y = fma(P.kc, k.y, v.y);
      }
      return v;
    };
    const int64_t out = ((a * d + i) * d + j) * R + r;
    T2 acc = (flags & TASK_ACC) ? P.y[out] : T2{0, 0};
    for (int g = tk.y; g < tk.z; ++g) {
      const int4 gr = P.groups[g];
      const int op = P.coef_op[gr.z];
      const size_t rowL = ((size_t)op * 2) * d + i;
      const size_t rowR = ((size_t)op * 2 + 1) * d + j;
      const int nl = P.ell_cnt[rowL], nr = P.ell_cnt[rowR];
      T2 L{0, 0}, Rv{0, 0};
      for (int e = gr.x; e < gr.y; ++e) {
        const int2 ed = P.gedges[e];
        const T w = (T)ed.y;
        T2 l{0, 0}, rr{0, 0};
        for (int t = 0; t < nl; ++t)
          l = cfma(P.ell_val[rowL * P.slots + t], in(ed.x, P.ell_col[rowL * P.slots + t], j), l);
        for (int t = 0; t < nr; ++t)
          rr = cfma(in(ed.x, i, P.ell_col[rowR * P.slots + t]), P.ell_val[rowR * P.slots + t], rr);
        L.x = fma(w, l.x, L.x); L.y = fma(w, l.y, L.y);
        Rv.x = fma(w, rr.x, Rv.x); Rv.y = fma(w, rr.y, Rv.y);
      }
      if (gr.w) {
        const T2 z = P.shifts ? P.shifts[r] : P.shift0;
        acc = csub(acc, cmul(csub(P.decay[a], z), in(a, i, j)));
      }
      acc = cfma(P.coef[2 * gr.z], L, acc);
      acc = cfma(P.coef[2 * gr.z + 1], Rv, acc);
    }
    if (P.border && a == 0 && i == 0 && j == 0 && (flags & TASK_DIAG)) {
      T2 tr{0, 0};
      for (int ii = 0; ii < d; ++ii) tr = cadd(tr, in(0, ii, ii));
      acc = tr;
    }
    P.y[out] = acc;
  }
}

// ----------------------------------------------------------------- small-system RK4
// Whole RK4 steps of a hierarchy with N d^2 <= 1024 elements in one
// workgroup: thread t owns one output element (task t / d^2, cell t % d^2)
// and keeps x, the RK4 accumulator and the stage result in registers; only
// the stage input lives in LDS, where the neighbour gathers of the apply
// read it.  One launch runs many steps, so a step costs four barriers
// instead of five kernel launches (small systems are launch-latency bound).
template <typename T>
__global__ void __launch_bounds__(1024) rk4_small_kernel(ApplyParams<T> P, typename Cplx<T>::t *__restrict__ x, T dt, int64_t steps,
                                                         int64_t save_every, int64_t step0, int64_t n_saves,
                                                         typename Cplx<T>::t *__restrict__ traj) {
  using T2 = typename Cplx<T>::t;
  extern __shared__ __align__(16) unsigned char smem[];
  T2 *u = reinterpret_cast<T2 *>(smem);
  const int d = P.d, dd = d * d;
  const int t = threadIdx.x;
  const int64_t n = P.n_tasks * dd;
  const bool own = t < n;
  int64_t a = 0;
  int i = 0, j = 0, g0 = 0, g1 = 0;
  if (own) {
    const int4 tk = P.tasks[t / dd];
    a = tk.x;
    g0 = tk.y;
    g1 = tk.z;
    i = (t % dd) / d;
    j = (t % dd) % d;
  }
  const int64_t e = a * dd + (int64_t)i * d + j;
  T2 xv = own ? x[e] : T2{0, 0};
  auto stage = [&](const T2 &in) -> T2 {
    __syncthreads();  // previous readers of u are done
    if (own) u[e] = in;
    __syncthreads();
    T2 acc{0, 0};
    if (!own) return acc;
    for (int g = g0; g < g1; ++g) {
      const int4 gr = P.groups[g];
      const int op = P.coef_op[gr.z];
      const size_t rowL = ((size_t)op * 2) * d + i;
      const size_t rowR = ((size_t)op * 2 + 1) * d + j;
      const int nl = P.ell_cnt[rowL], nr = P.ell_cnt[rowR];
      T2 L{0, 0}, Rv{0, 0};
      for (int ed = gr.x; ed < gr.y; ++ed) {
        const int2 edge = P.gedges[ed];
        const T w = (T)edge.y;
        const T2 *ub = u + (int64_t)edge.x * dd;
        T2 l{0, 0}, rr{0, 0};
        for (int q = 0; q < nl; ++q) l = cfma(P.ell_val[rowL * P.slots + q], ub[P.ell_col[rowL * P.slots + q] * d + j], l);
        for (int q = 0; q < nr; ++q) rr = cfma(ub[i * d + P.ell_col[rowR * P.slots + q]], P.ell_val[rowR * P.slots + q], rr);
        L.x = fma(w, l.x, L.x); L.y = fma(w, l.y, L.y);
        Rv.x = fma(w, rr.x, Rv.x); Rv.y = fma(w, rr.y, Rv.y);
      }
      if (gr.w) acc = csub(acc, cmul(P.decay[a], u[e]));
      acc = cfma(P.coef[2 * gr.z], L, acc);
      acc = cfma(P.coef[2 * gr.z + 1], Rv, acc);
    }
    return acc;
  };
  const T h2 = dt / 2, h6 = dt / 6, h3 = dt / 3;
  for (int64_t st = 0; st < steps; ++st) {
    const T2 k1 = stage(xv);
    T2 acc{xv.x + h6 * k1.x, xv.y + h6 * k1.y};
    const T2 k2 = stage(T2{xv.x + h2 * k1.x, xv.y + h2 * k1.y});
    acc.x += h3 * k2.x; acc.y += h3 * k2.y;
    const T2 k3 = stage(T2{xv.x + h2 * k2.x, xv.y + h2 * k2.y});
    acc.x += h3 * k3.x; acc.y += h3 * k3.y;
    const T2 k4 = stage(T2{xv.x + dt * k3.x, xv.y + dt * k3.y});
    acc.x += h6 * k4.x; acc.y += h6 * k4.y;
    xv = acc;
    const int64_t gs = step0 + st + 1;
    if (save_every > 0 && gs % save_every == 0 && own && a == 0) {
      const int64_t slot = gs / save_every - 1;
      if (slot < n_saves) traj[slot * dd + (int64_t)i * d + j] = xv;
    }
  }
  if (own) x[e] = xv;
}

template <typename T>
static heom_status launch_rk4_small_T(Hier &h, void *x, double dt, int64_t steps, int64_t save_every, int64_t step0,
                                      int64_t n_saves, void *traj, hipStream_t s) {
  using T2 = typename Cplx<T>::t;
  DeviceTables &D = h.dev;
  constexpr bool dbl = std::is_same<T, double>::value;
  ApplyParams<T> P{};
  P.tasks = D.base.tasks;
  P.n_tasks = D.base.task_off.back();
  P.groups = D.base.groups;
  P.gedges = D.base.gedges;
  P.decay = dbl ? (const T2 *)D.decay64 : (const T2 *)D.decay32;
  P.ell_cnt = D.ell_cnt;
  P.ell_col = D.ell_col;
  P.ell_val = dbl ? (const T2 *)D.ell_val64 : (const T2 *)D.ell_val32;
  P.slots = h.ell.slots;
  P.coef_op = D.coef_op;
  P.coef = dbl ? (const T2 *)D.coef64 : (const T2 *)D.coef32;
  P.d = h.d;
  P.R = 1;
  const size_t smem = (size_t)h.N * h.d * h.d * sizeof(T2);
  hipLaunchKernelGGL(rk4_small_kernel<T>, dim3(1), dim3(1024), smem, s, P, (typename Cplx<T>::t *)x, (T)dt, steps, save_every, step0,
                     n_saves, (T2 *)traj);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

bool rk4_small_fits(const Hier &h) { return h.N * (int64_t)h.d * h.d <= 1024; }

heom_status launch_rk4_small(Hier &h, int precision, void *x, double dt, int64_t steps, int64_t save_every,
                             int64_t step0, int64_t n_saves, void *traj, hipStream_t s) {
  HEOM_TRY(ensure_device(h));
  if (!rk4_small_fits(h)) return fail(HEOM_ERR_UNSUPPORTED, "rk4_small: more than 1024 elements");
  if (precision == HEOM_FP64) return launch_rk4_small_T<double>(h, x, dt, steps, save_every, step0, n_saves, traj, s);
  return launch_rk4_small_T<float>(h, x, dt, steps, save_every, step0, n_saves, traj, s);
}

template <typename T>
static heom_status launch_T(Hier &h, const ApplyArgs &a, const Plan &pl, int64_t t0, int64_t t1, hipStream_t s) {
  using T2 = typename Cplx<T>::t;
  DeviceTables &D = h.dev;
  const int64_t n_tasks = t1 - t0;
  if (n_tasks <= 0) return HEOM_OK;
  constexpr bool dbl = std::is_same<T, double>::value;
  ApplyParams<T> P{};
  P.tasks = pl.tasks + t0;
  P.n_tasks = n_tasks;
  P.groups = pl.groups;
  P.gedges = pl.gedges;
  P.decay = dbl ? (const T2 *)D.decay64 : (const T2 *)D.decay32;
  P.ell_cnt = D.ell_cnt;
  P.ell_col = D.ell_col;
  P.ell_val = dbl ? (const T2 *)D.ell_val64 : (const T2 *)D.ell_val32;
  P.op_slots = D.op_slots;
  P.c_meta = D.c_meta;
  P.c_col = D.c_col;
  P.c_val = dbl ? (const T2 *)D.c_val64 : (const T2 *)D.c_val32;
  P.n_centries = (int)h.ell.c_col.size();
  P.hdiag = dbl ? (const T2 *)D.hdiag : (const T2 *)D.hdiag32;
  P.slots = h.ell.slots;
  P.coef_op = D.coef_op;
  P.coef = dbl ? (const T2 *)D.coef64 : (const T2 *)D.coef32;
  P.x = (const T2 *)a.x;
  P.kvec = (const T2 *)a.k;
  P.kc = (T)a.kc;
  P.y = (T2 *)a.y;
  P.d = h.d;
  P.R = a.n_rhs;
  P.shifts = (const T2 *)a.shifts;
  P.shift0 = T2{(T)a.shift0.real(), (T)a.shift0.imag()};
  P.border = a.border;
  const int d = h.d;
  const size_t tab_bytes = (size_t)P.n_centries * (sizeof(T2) + sizeof(int)) + 16 + (size_t)d * sizeof(T2);
  const size_t smem = 4 * (size_t)d * d * sizeof(T2) + tab_bytes;
  if (a.n_rhs == 1 && (d == 8 || d == 16 || d == 20) && smem <= 48 * 1024) {
    P.tpw = 1;
    P.xchunk = 64;
    const int64_t grid = (n_tasks + 4 * P.tpw - 1) / (4 * P.tpw);
    if (grid > 0x7fffffff) return fail(HEOM_ERR_UNSUPPORTED, "apply grid too large");
    dim3 g((unsigned)grid), b(256);
    if (d == 8) {
      if (P.kvec) hipLaunchKernelGGL((apply_wave_kernel<T, 8, true>), g, b, smem, s, P);
      else hipLaunchKernelGGL((apply_wave_kernel<T, 8, false>), g, b, smem, s, P);
    } else if (d == 20) {
      if (P.kvec) hipLaunchKernelGGL((apply_wave_kernel<T, 20, true>), g, b, smem, s, P);
      else hipLaunchKernelGGL((apply_wave_kernel<T, 20, false>), g, b, smem, s, P);
    } else {
      if (P.kvec) hipLaunchKernelGGL((apply_wave_kernel<T, 16, true>), g, b, smem, s, P);
      else hipLaunchKernelGGL((apply_wave_kernel<T, 16, false>), g, b, smem, s, P);
    }
  } else {
    const int cells = d * d * a.n_rhs;
    const int64_t grid = cells <= 256 ? (n_tasks + (256 / cells) - 1) / (256 / cells) : n_tasks;
    if (grid > 0x7fffffff) return fail(HEOM_ERR_UNSUPPORTED, "apply grid too large");
    dim3 g((unsigned)grid), b(256);
    switch (d) {
      case 2: hipLaunchKernelGGL((apply_cell_kernel<T, 2>), g, b, 0, s, P); break;
      case 4: hipLaunchKernelGGL((apply_cell_kernel<T, 4>), g, b, 0, s, P); break;
      case 8: hipLaunchKernelGGL((apply_cell_kernel<T, 8>), g, b, 0, s, P); break;
      case 16: hipLaunchKernelGGL((apply_cell_kernel<T, 16>), g, b, 0, s, P); break;
      default: hipLaunchKernelGGL((apply_cell_kernel<T, 0>), g, b, 0, s, P); break;
    }
  }
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

static heom_status check_apply(Hier &h, int precision, const ApplyArgs &a) {
  if (precision != HEOM_FP64 && precision != HEOM_FP32) return fail(HEOM_ERR_ARG, "precision must be FP64 or FP32");
  if (!a.x || !a.y) return fail(HEOM_ERR_ARG, "apply: NULL vector");
  if (a.n_rhs < 1 || a.n_rhs > 4096) return fail(HEOM_ERR_ARG, "apply: n_rhs must be in [1, 4096]");
  if (h.d > 32) return fail(HEOM_ERR_UNSUPPORTED, "apply: d > 32");
  return ensure_device(h);
}

static heom_status run_plan(Hier &h, int precision, const ApplyArgs &a, const Plan &pl, hipStream_t s) {
  for (size_t l = 0; l + 1 < pl.task_off.size(); ++l) {
    if (precision == HEOM_FP64) HEOM_TRY(launch_T<double>(h, a, pl, pl.task_off[l], pl.task_off[l + 1], s));
    else HEOM_TRY(launch_T<float>(h, a, pl, pl.task_off[l], pl.task_off[l + 1], s));
  }
  return HEOM_OK;
}

heom_status launch_apply(Hier &h, int precision, const ApplyArgs &a, hipStream_t s) {
  HEOM_TRY(check_apply(h, precision, a));
  return run_plan(h, precision, a, h.dev.base, s);
}

heom_status launch_apply_tiled(Hier &h, int precision, const ApplyArgs &a, int n_chunks, hipStream_t s) {
  HEOM_TRY(check_apply(h, precision, a));
  if (n_chunks <= 0) {
    // keep each chunk's leaf blocks around 96 MB so they stay in the
    // 256 MB last-level cache while the lower tiers re-read them
    const double w = precision == HEOM_FP64 ? 16.0 : 8.0;
    double leaf_bytes = (double)h.n_leaf * h.d * h.d * w * a.n_rhs;
    n_chunks = (int)std::ceil(leaf_bytes / (96.0 * 1024 * 1024));
    if (n_chunks < 1) n_chunks = 1;
  }
  HEOM_TRY(ensure_tiled_plan(h, n_chunks));
  return run_plan(h, precision, a, h.dev.tiled, s);
}

}  // namespace heom
