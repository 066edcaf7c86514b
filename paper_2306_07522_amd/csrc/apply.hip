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
#include "apply_wave.h"

namespace heom {

// ----------------------------------------------------------------- wave kernel
// One wave processes tasks first, first + 4, ... (tpw of them).  Blocks are
// remapped inside super-chunks of xchunk blocks so that each XCD (block b
// runs on XCD b % 8) walks a contiguous run of tasks, which share parents.  Within a
// task the next group's first neighbour block is prefetched while the
// current group is finished; multi-edge groups stream two blocks at a time.
template <typename T, int D, bool FUSE, bool MF = false, bool EPI = false, bool LT = false>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(WaveShape<D>::EPL > 4 ? 2 : (MF && sizeof(T) == 8 ? 3 : 4))))
apply_wave_kernel(ApplyParams<T> P) {
  using T2 = typename Cplx<T>::t;
  constexpr int DD = D * D;
  extern __shared__ __align__(16) unsigned char smem[];
  // The LDS layout is built from byte offsets into smem (no integer round
  // trip of the addresses), so every access below stays an LDS access; a
  // generic (flat) access would also wait on the outstanding block loads.
  T2 *sbuf = reinterpret_cast<T2 *>(smem);              // [4][DD] group staging, one slice per wave
  T2 *tval = sbuf + 4 * DD;                             // compact operator values
  int *tcol = reinterpret_cast<int *>(tval + P.n_centries);
  // H diagonal, after the column table (16-byte aligned)
  const size_t o_thd = (4 * DD * sizeof(T2) + (size_t)P.n_centries * (sizeof(T2) + sizeof(int)) + 15) & ~(size_t)15;
  T2 *thd = reinterpret_cast<T2 *>(smem + o_thd);
  for (int e = threadIdx.x; e < P.n_centries; e += 256) {
    tval[e] = P.c_val[e];
    tcol[e] = P.c_col[e];
  }
  if (threadIdx.x < D) thd[threadIdx.x] = P.hdiag[threadIdx.x];
  // LT: per coefficient entry, the operator's packed table slot / width /
  // realness and the two coefficients, after the H diagonal
  int *cmeta = reinterpret_cast<int *>(thd + D);
  const size_t o_cfs = (o_thd + D * sizeof(T2) + (size_t)P.n_coef * sizeof(int) + 15) & ~(size_t)15;
  T2 *cfs = reinterpret_cast<T2 *>(smem + o_cfs);
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
    wave_task<T, D, FUSE, true, MF, EPI, LT>(P, task, lane, buf, tval, tcol, thd, cmeta, cfs);
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
    store_out<true>(P, out, acc);
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

bool rk4_small_fits(const Hier &h) { return h.N * (int64_t)h.d * h.d <= 1024 && h.lind.empty(); }

heom_status launch_rk4_small(Hier &h, int precision, void *x, double dt, int64_t steps, int64_t save_every,
                             int64_t step0, int64_t n_saves, void *traj, hipStream_t s) {
  HEOM_TRY(ensure_device(h));
  if (!rk4_small_fits(h)) return fail(HEOM_ERR_UNSUPPORTED, "rk4_small: more than 1024 elements");
  if (precision == HEOM_FP64) return launch_rk4_small_T<double>(h, x, dt, steps, save_every, step0, n_saves, traj, s);
  return launch_rk4_small_T<float>(h, x, dt, steps, save_every, step0, n_saves, traj, s);
}

// One instantiation of the wave kernel: the stage-input form (kvec), or the
// plain or epilogue form, each with the task tables in lanes when every task
// of the plan has at most 64 groups and 64 edges.
template <typename T, int D, bool MF>
static void launch_wave(dim3 g, dim3 b, size_t smem, hipStream_t s, const ApplyParams<T> &P, bool lt) {
  if (P.kvec) hipLaunchKernelGGL((apply_wave_kernel<T, D, true, MF>), g, b, smem, s, P);
  else if (P.epi && lt) hipLaunchKernelGGL((apply_wave_kernel<T, D, false, MF, true, true>), g, b, smem, s, P);
  else if (P.epi) hipLaunchKernelGGL((apply_wave_kernel<T, D, false, MF, true, false>), g, b, smem, s, P);
  else if (lt) hipLaunchKernelGGL((apply_wave_kernel<T, D, false, MF, false, true>), g, b, smem, s, P);
  else hipLaunchKernelGGL((apply_wave_kernel<T, D, false, MF, false, false>), g, b, smem, s, P);
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
  P.hoff = dbl ? (const T2 *)D.hoff64 : (const T2 *)D.hoff32;
  P.hmfma = a.hmfma;
  P.epi = a.epi ? 1 : 0;
  for (int j = 0; j < 4; ++j) {
    P.ev[j] = (const T2 *)a.ev[j];
    P.ec[j] = (T)a.ec[j];
  }
  P.eacc = (T)a.eacc;
  P.y2 = (T2 *)a.y2;
  for (int j = 0; j < 4; ++j) P.ec2[j] = (T)a.ec2[j];
  P.eacc2 = (T)a.eacc2;
  const int d = h.d;
  const size_t tab_bytes = (size_t)P.n_centries * (sizeof(T2) + sizeof(int)) + 16 + (size_t)d * sizeof(T2);
  const size_t smem = 4 * (size_t)d * d * sizeof(T2) + tab_bytes;
  if (a.n_rhs == 1 && (d == 8 || d == 16 || d == 20) && smem <= 48 * 1024) {
    // two tasks per wave for the FP32 and the RK4-stage (epilogue) kernels on
    // large plans: each workgroup's table staging then serves eight tasks.
    // Two-orbital tier 4, same box: FP32 apply 0.505 -> 0.494 ms, FP64 RK4
    // step 4.43 -> 4.25 ms; the plain FP64 apply keeps one task per wave
    // (0.913 against 0.932 ms with two), and small plans keep one so that
    // every CU gets work.
    P.tpw = n_tasks >= (int64_t)1 << 16 && (sizeof(T) == 4 || a.epi) ? 2 : 1;
    P.xchunk = 64;
    const int64_t grid = (n_tasks + 4 * P.tpw - 1) / (4 * P.tpw);
    if (grid > 0x7fffffff) return fail(HEOM_ERR_UNSUPPORTED, "apply grid too large");
    dim3 g((unsigned)grid), b(256);
    // the epilogue (never together with a stage-input vector) has kernels of
    // its own, so that the plain apply carries none of its code
    // task tables in lanes when every task has at most 64 groups and edges,
    // and the packed operator metadata fits (20-bit slot, 10-bit width) along
    // with the coefficients in the LDS budget
    P.n_coef = (int)h.coefs.size();
    const size_t smem_lt = smem + (size_t)P.n_coef * sizeof(int) + 16 + 2 * (size_t)P.n_coef * sizeof(T2);
    const bool lt = pl.max_groups <= 64 && pl.max_edges <= 64 && P.n_centries < (1 << 20) && d < 1024 &&
                    smem_lt <= 48 * 1024;
    const size_t sm = lt ? smem_lt : smem;
    if (d == 8) launch_wave<T, 8, false>(g, b, sm, s, P, lt);
    else if (d == 20) launch_wave<T, 20, false>(g, b, sm, s, P, lt);
    else if (P.hmfma) launch_wave<T, 16, true>(g, b, sm, s, P, lt);
    else launch_wave<T, 16, false>(g, b, sm, s, P, lt);
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

heom_status launch_plan_range(Hier &h, int precision, const ApplyArgs &a, const Plan &pl, int64_t t0, int64_t t1,
                              hipStream_t s) {
  if (precision == HEOM_FP64) return launch_T<double>(h, a, pl, t0, t1, s);
  return launch_T<float>(h, a, pl, t0, t1, s);
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

// Off-diagonal entries of H per row (the compact table's width) from which
// the matrix-core H terms beat the gathers at d = 16, per precision.
// Measured on a d = 16 spin-boson hierarchy (6,435 ADOs) with banded random
// H (median of 20 applies): the MFMA apply takes the same time at every
// width, 48.5-50 us FP64 and 36.5-37.5 us FP32 (it runs at 3 and 4 waves per
// SIMD against 4 and 6 for the gathers); the gathers take 42-44 / 46 / 47 /
// 53-59 us FP64 at 1-2 / 4 / 6 / 8-15 entries, and 28-29 / 31 / 33 / 37 /
// 40-41 us FP32 at 1-2 / 4 / 6 / 8-10 / 12-15.
constexpr int kMfmaMinOffdiag64 = 8, kMfmaMinOffdiag32 = 12;

// The wave kernel (which carries the matrix-core path) runs for this hierarchy
static bool mfma_fits(const Hier &h, int precision) {
  const size_t w = precision == HEOM_FP64 ? 16 : 8;
  const size_t smem = 4 * (size_t)h.d * h.d * w + h.ell.c_col.size() * (w + 4) + 16 + (size_t)h.d * 16;
  return smem <= 48 * 1024;
}

heom_status launch_apply_plan(Hier &h, int precision, const ApplyArgs &a, int plan, hipStream_t s) {
  HEOM_TRY(check_apply(h, precision, a));
  const bool have_slab = h.dev.slab.built;
  bool slab = false;
  switch (plan) {
    case HEOM_PLAN_AUTO:
      // the pull plan (measured faster than the slab plan on the two-orbital
      // model); its H terms on the matrix cores when d = 16 and H has at
      // least the cut-over's off-diagonal entries in some row or column
      if (h.d == 16 && a.n_rhs == 1 && mfma_fits(h, precision) &&
          h.ell.c_ns[0] >= (precision == HEOM_FP64 ? kMfmaMinOffdiag64 : kMfmaMinOffdiag32))
        return launch_apply_plan(h, precision, a, HEOM_PLAN_PULL_MFMA, s);
      break;
    case HEOM_PLAN_PULL:
      break;
    case HEOM_PLAN_PULL_MFMA: {
      if (h.d != 16 || a.n_rhs != 1 || !mfma_fits(h, precision))
        return fail(HEOM_ERR_UNSUPPORTED, "apply: the MFMA self group needs d = 16 and one right-hand side");
      ApplyArgs m = a;
      m.hmfma = 1;
      if (m.epi && (!h.lind.empty() || m.k))
        return fail(HEOM_ERR_UNSUPPORTED, "apply: the epilogue needs the pull plan, one right-hand side, no Lindblad terms");
      HEOM_TRY(run_plan(h, precision, m, h.dev.base, s));
      return launch_lindblad(h, precision, m, s);
    }
    case HEOM_PLAN_SLAB:
      if (!have_slab || a.n_rhs != 1)
        return fail(HEOM_ERR_UNSUPPORTED,
                    "apply: the slab plan needs one right-hand side and a purely fermionic, unpruned hierarchy "
                    "with n_max >= 3 and d = 8 or 16");
      slab = true;
      break;
    default:
      return fail(HEOM_ERR_ARG, "apply: unknown plan");
  }
  if (a.epi && (slab || a.n_rhs != 1 || !h.lind.empty() || a.k))
    return fail(HEOM_ERR_UNSUPPORTED, "apply: the epilogue needs the pull plan, one right-hand side, no Lindblad terms");
  if (slab) HEOM_TRY(launch_apply_slab(h, precision, a, s));
  else HEOM_TRY(run_plan(h, precision, a, h.dev.base, s));
  return launch_lindblad(h, precision, a, s);
}

heom_status launch_apply(Hier &h, int precision, const ApplyArgs &a, hipStream_t s) {
  return launch_apply_plan(h, precision, a, HEOM_PLAN_AUTO, s);
}

heom_status launch_apply_tiled(Hier &h, int precision, const ApplyArgs &a, int n_chunks, hipStream_t s) {
  HEOM_TRY(check_apply(h, precision, a));
  if (a.epi) return fail(HEOM_ERR_UNSUPPORTED, "apply: the tiled plan has no epilogue");
  if (n_chunks <= 0) {
    // keep each chunk's leaf blocks around 96 MB so they stay in the
    // 256 MB last-level cache while the lower tiers re-read them
    const double w = precision == HEOM_FP64 ? 16.0 : 8.0;
    double leaf_bytes = (double)h.n_leaf * h.d * h.d * w * a.n_rhs;
    n_chunks = (int)std::ceil(leaf_bytes / (96.0 * 1024 * 1024));
    if (n_chunks < 1) n_chunks = 1;
  }
  const Plan *pl = nullptr;
  HEOM_TRY(ensure_tiled_plan(h, n_chunks, &pl));
  HEOM_TRY(run_plan(h, precision, a, *pl, s));
  return launch_lindblad(h, precision, a, s);
}

}  // namespace heom
