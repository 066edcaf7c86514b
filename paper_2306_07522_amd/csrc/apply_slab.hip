// Slab launches of the matrix-free HEOM Liouvillian apply (eq:HEOM) for
// purely fermionic hierarchies: the top tier's up-terms (the C-type terms,
// d^{nubar} acting on the ADO one level higher) are summed by the parents'
// workgroups while each child block passes through LDS once.
//
// Three launches: the rows launch (the ordinary wave kernel) computes the
// lower tiers and every top-tier ADO's own row (self and down terms); the
// prefix launch writes every tier-(L-1) parent's prefix part of its up-terms
// to y; the suffix launch adds the suffix part and the rest of each parent's
// row (self, down terms, any up-terms of neither part) on top.
//
// One workgroup (8 waves) of a slab launch runs one job: a share of a label
// slab's parents (vertices) and the slab's children that touch them.
// Vertex v's accumulator lives in the registers of wave v % 8 (slot v / 8).
// The children come in sub-rounds of at most kSlabSub: within a sub-round no
// two children share a parent, so every accumulator takes at most one term
// per sub-round and no two waves ever add to the same accumulator.  Each wave
// loads its share of the next sub-round into registers while the current one
// is consumed from LDS (double buffering), then parks it in the other LDS
// buffer.  The coefficient pairs and operator metadata of every term sit in
// LDS beside the operators' compact tables.
#include "apply_wave.h"

namespace heom {

struct SlabArgs {
  const int4 *jobs;
  const int32_t *sub;
  const int4 *ent;
  const int2 *vert;
  int n_coef;
};

template <typename T, int D, bool FUSE, bool FIN>
__global__ void __launch_bounds__(kSlabWaves * 64) __attribute__((amdgpu_waves_per_eu(2, 2)))
apply_slab_kernel(ApplyParams<T> P, SlabArgs S) {
  using T2 = typename Cplx<T>::t;
  using M = LaneMap<T, D>;
  constexpr int DD = D * D;
  constexpr int EPL = WaveShape<D>::EPL;
  constexpr int NW = kSlabWaves, SUB = kSlabSub, PRE = (kSlabSub + kSlabWaves - 1) / kSlabWaves, VM = kSlabVmax;
  static_assert(2 * SUB >= NW, "the sub-round buffers double as the finishing tasks' staging");
  extern __shared__ __align__(16) unsigned char smem[];
  T2 *rbuf = reinterpret_cast<T2 *>(smem);  // [2][SUB][DD] sub-round children
  T2 *ccoef = rbuf + 2 * SUB * DD;          // [n_coef][2] (cl, cr)
  int4 *cmeta = reinterpret_cast<int4 *>(ccoef + 2 * S.n_coef);  // [n_coef] (off, ns, real, -)
  T2 *tval = reinterpret_cast<T2 *>(cmeta + S.n_coef);
  int *tcol = reinterpret_cast<int *>(tval + P.n_centries);
  T2 *thd = reinterpret_cast<T2 *>((reinterpret_cast<uintptr_t>(tcol + P.n_centries) + 15) & ~(uintptr_t)15);
  for (int e = threadIdx.x; e < P.n_centries; e += NW * 64) {
    tval[e] = P.c_val[e];
    tcol[e] = P.c_col[e];
  }
  for (int c = threadIdx.x; c < S.n_coef; c += NW * 64) {
    const int op = P.coef_op[c];
    cmeta[c] = make_int4(P.c_meta[3 * op], P.c_meta[3 * op + 1], P.c_meta[3 * op + 2], 0);
    ccoef[2 * c] = P.coef[2 * c];
    ccoef[2 * c + 1] = P.coef[2 * c + 1];
  }
  if (threadIdx.x < D) thd[threadIdx.x] = P.hdiag[threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int4 job = S.jobs[blockIdx.x];
  if (job.y <= 0) return;  // empty slot of the XCD layout
  // vertex accumulators and prefetched children stay in registers: every
  // index into acc and pre below is a compile-time constant after unrolling
  T2 acc[VM][EPL];
#pragma unroll
  for (int q = 0; q < VM; ++q)
#pragma unroll
    for (int s = 0; s < EPL; ++s) acc[q][s] = T2{0, 0};
  T2 pre[PRE][EPL];
  // the entries of a sub-round sit one per lane (lane < kSlabSub), loaded a
  // sub-round ahead with one vector load and read back with readlane
  static_assert(SUB <= 64, "one entry per lane");
  int4 ecur = make_int4(0, 0, 0, 0);
  // this wave's children of sub-round si are entries e0 + wave + NW q
  if (job.w > 0) {
    const int e0 = S.sub[job.z], e1 = S.sub[job.z + 1];
    if (lane < e1 - e0) ecur = S.ent[e0 + lane];
#pragma unroll
    for (int q = 0; q < PRE; ++q) {
      const int i = wave + NW * q;
      if (e0 + i < e1) {
        load_block<T, D, FUSE>(P, S.ent[e0 + i].x, lane, pre[q]);
#pragma unroll
        for (int s = 0; s < EPL; ++s)
          if (M::on(lane, s)) rbuf[i * DD + M::elem(lane, s)] = pre[q][s];
      }
    }
  }
  __syncthreads();
  for (int si = 0; si < job.w; ++si) {
    const T2 *cur = rbuf + (si & 1) * SUB * DD;
    const int e0 = S.sub[job.z + si], e1 = S.sub[job.z + si + 1];
    const bool more = si + 1 < job.w;
    const int f0 = more ? S.sub[job.z + si + 1] : 0, f1 = more ? S.sub[job.z + si + 2] : 0;
#pragma unroll
    for (int q = 0; q < PRE; ++q) {  // the next sub-round's children, in flight meanwhile
      const int i = wave + NW * q;
      if (f0 + i < f1) load_block<T, D, FUSE>(P, S.ent[f0 + i].x, lane, pre[q]);
    }
    int4 enext = make_int4(0, 0, 0, 0);
    if (lane < f1 - f0) enext = S.ent[f0 + lane];
    // each child's terms on those of its two parents that this wave holds
    for (int i = 0; i < e1 - e0; ++i) {
      const int ez = __builtin_amdgcn_readlane(ecur.z, i), ew = __builtin_amdgcn_readlane(ecur.w, i);
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int info = side ? ew : ez;
        const int slot = (info >> 24) & 127;
        if (slot == 127 || slot % NW != wave) continue;
        const int q = slot / NW;
        const int cid = info & 0x7fffff;
        const int4 mt = cmeta[cid];
        if (mt.y <= 0) continue;
        const T w = (info >> 23) & 1 ? (T)-1 : (T)1;
        T2 cl = ccoef[2 * cid], cr = ccoef[2 * cid + 1];
        cl.x *= w; cl.y *= w; cr.x *= w; cr.y *= w;
        const T2 *X = cur + i * DD;
#pragma unroll
        for (int s = 0; s < EPL; ++s) {
          if (!M::on(lane, s)) continue;
          const int ii = M::elem(lane, s) / D, jj = M::col(lane, s);
          const int lbase = mt.x + ii * mt.y, rbase = mt.x + (D + jj) * mt.y;
          T2 L{0, 0}, Rv{0, 0};
#pragma unroll 1
          for (int t = 0; t < mt.y; ++t) {
            L = cfma(tval[lbase + t], X[tcol[lbase + t] * D + jj], L);
            Rv = cfma(X[ii * D + tcol[rbase + t]], tval[rbase + t], Rv);
          }
          T2 c = cmul(cl, L);
          c = cfma(cr, Rv, c);
#pragma unroll
          for (int qq = 0; qq < VM; ++qq)
            if (qq == q) acc[qq][s] = cadd(acc[qq][s], c);
        }
      }
    }
    T2 *nxt = rbuf + ((si + 1) & 1) * SUB * DD;
#pragma unroll
    for (int q = 0; q < PRE; ++q) {
      const int i = wave + NW * q;
      if (f0 + i < f1)
#pragma unroll
        for (int s = 0; s < EPL; ++s)
          if (M::on(lane, s)) nxt[i * DD + M::elem(lane, s)] = pre[q][s];
    }
    ecur = enext;
    __syncthreads();
  }
  // the vertices: wave w holds vertices w, w + NW, ...; the sub-round
  // buffers are free now and serve as the waves' staging slices
  T2 *buf = rbuf + wave * DD;
#pragma unroll
  for (int q = 0; q < VM; ++q) {
    const int v = wave + NW * q;
    if (v >= job.y) break;
    const int2 vx = S.vert[job.x + v];
    const int64_t base = (int64_t)vx.x * DD;
    if (FIN) {
      T2 r[EPL];
#pragma unroll
      for (int s = 0; s < EPL; ++s) r[s] = M::on(lane, s) ? cadd(acc[q][s], P.y[base + M::elem(lane, s)]) : acc[q][s];
      wave_task_add<T, D, FUSE, false>(P, vx.y, lane, buf, tval, tcol, thd, r);
    } else {
#pragma unroll
      for (int s = 0; s < EPL; ++s)
        if (M::on(lane, s)) P.y[base + M::elem(lane, s)] = acc[q][s];
    }
  }
}

template <typename T, int D, bool FUSE, bool FIN>
static heom_status launch_slab_pass(const ApplyParams<T> &P, const SlabPass &sp, int n_coef, size_t smem, hipStream_t s) {
  if (sp.n_jobs == 0) return HEOM_OK;
  if (sp.n_jobs > 0x7fffffff) return fail(HEOM_ERR_UNSUPPORTED, "slab apply: too many jobs");
  auto kern = apply_slab_kernel<T, D, FUSE, FIN>;
  // grant the full LDS once per kernel (a repeated grant from a racing thread is harmless)
  static std::atomic<bool> granted{false};
  if (!granted.load(std::memory_order_acquire)) {
    HEOM_HIP_CHECK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    granted.store(true, std::memory_order_release);
  }
  SlabArgs S{sp.jobs, sp.sub, sp.ent, sp.vert, n_coef};
  hipLaunchKernelGGL(kern, dim3((unsigned)sp.n_jobs), dim3(kSlabWaves * 64), smem, s, P, S);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template <typename T, int D, bool FUSE>
static heom_status run_slab(const ApplyParams<T> &P, const SlabPlan &pl, int n_coef, size_t smem, hipStream_t s) {
  HEOM_TRY((launch_slab_pass<T, D, FUSE, false>(P, pl.pass[0], n_coef, smem, s)));
  return launch_slab_pass<T, D, FUSE, true>(P, pl.pass[1], n_coef, smem, s);
}

template <typename T>
static heom_status launch_slab_T(Hier &h, const ApplyArgs &a, hipStream_t s) {
  using T2 = typename Cplx<T>::t;
  DeviceTables &Dv = h.dev;
  const SlabPlan &pl = Dv.slab;
  constexpr bool dbl = std::is_same<T, double>::value;
  ApplyParams<T> P{};
  P.tasks = pl.tasks.tasks;
  P.n_tasks = pl.tasks.task_off.back();
  P.groups = pl.tasks.groups;
  P.gedges = pl.tasks.gedges;
  P.decay = dbl ? (const T2 *)Dv.decay64 : (const T2 *)Dv.decay32;
  P.c_meta = Dv.c_meta;
  P.c_col = Dv.c_col;
  P.c_val = dbl ? (const T2 *)Dv.c_val64 : (const T2 *)Dv.c_val32;
  P.n_centries = (int)h.ell.c_col.size();
  P.hdiag = dbl ? (const T2 *)Dv.hdiag : (const T2 *)Dv.hdiag32;
  P.slots = h.ell.slots;
  P.coef_op = Dv.coef_op;
  P.coef = dbl ? (const T2 *)Dv.coef64 : (const T2 *)Dv.coef32;
  P.x = (const T2 *)a.x;
  P.kvec = (const T2 *)a.k;
  P.kc = (T)a.kc;
  P.y = (T2 *)a.y;
  P.d = h.d;
  P.R = 1;
  P.shifts = (const T2 *)a.shifts;
  P.shift0 = T2{(T)a.shift0.real(), (T)a.shift0.imag()};
  P.border = a.border;
  const int d = h.d;
  const int n_coef = (int)h.coefs.size();
  const size_t smem = (size_t)2 * kSlabSub * d * d * sizeof(T2) + (size_t)n_coef * (2 * sizeof(T2) + sizeof(int4)) +
                      (size_t)P.n_centries * (sizeof(T2) + sizeof(int)) + 16 + (size_t)d * sizeof(T2);
  if (smem > 160 * 1024) return fail(HEOM_ERR_UNSUPPORTED, "slab apply: LDS tables too large");
  if (d == 16) {
    if (P.kvec) return run_slab<T, 16, true>(P, pl, n_coef, smem, s);
    return run_slab<T, 16, false>(P, pl, n_coef, smem, s);
  }
  if (d == 8) {
    if (P.kvec) return run_slab<T, 8, true>(P, pl, n_coef, smem, s);
    return run_slab<T, 8, false>(P, pl, n_coef, smem, s);
  }
  return fail(HEOM_ERR_UNSUPPORTED, "slab apply: d must be 8 or 16");
}

heom_status launch_apply_slab(Hier &h, int precision, const ApplyArgs &a, hipStream_t s) {
  if (!h.dev.slab.built) return fail(HEOM_ERR_UNSUPPORTED, "slab apply: no slab plan for this hierarchy");
  if (a.n_rhs != 1) return fail(HEOM_ERR_UNSUPPORTED, "slab apply: one right-hand side only");
  // rows launch: lower tiers and the top tier's own rows
  HEOM_TRY(launch_plan_range(h, precision, a, h.dev.slab.tasks, 0, h.dev.slab.n_rows, s));
  if (precision == HEOM_FP64) return launch_slab_T<double>(h, a, s);
  return launch_slab_T<float>(h, a, s);
}

}  // namespace heom
