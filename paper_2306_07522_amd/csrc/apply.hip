// Matrix-free HEOM Liouvillian apply (eq:HEOM), y = (M + shift) x.
//
// Every output ADO a is one task.  A task accumulates, for each element
// (i, j) of rho_a and each right-hand side r,
//   diag:  -(c_a - z_r) x_a[i][j] - i (H x_a)[i][j] + i (x_a H)[i][j]
//   edges: sum over neighbours b of  cl (O x_b)[i][j] + cr (x_b O)[i][j]
// where each edge names a coefficient-table entry (operator O and the two
// complex coefficients of the superoperator A, B, C or D with the parity
// projector folded in) and a small integer multiplier (bosonic multiplicity
// or fermionic reorder sign).  Operators are stored in ELL form so that the
// signed-permutation coupling operators of fermionic models cost one gather
// per element, and dense ones cost d.
//
// Layout: x, y are [N][d][d][R] complex, R innermost; one thread owns one
// (i, j, r) cell of one task.
#include "device_common.h"
#include "internal.h"

namespace heom {

template <typename T, int D>
__global__ void __launch_bounds__(256)
apply_kernel(const int4 *__restrict__ tasks, int64_t n_tasks, const int64_t *__restrict__ row_ptr,
             const int2 *__restrict__ edges, const typename Cplx<T>::t *__restrict__ decay,
             const int32_t *__restrict__ ell_cnt, const int32_t *__restrict__ ell_col,
             const typename Cplx<T>::t *__restrict__ ell_val, int slots,
             const int32_t *__restrict__ coef_op, const typename Cplx<T>::t *__restrict__ coef,
             const typename Cplx<T>::t *__restrict__ x, const typename Cplx<T>::t *__restrict__ kvec, T kc,
             typename Cplx<T>::t *__restrict__ y, int d_rt, int R, const typename Cplx<T>::t *__restrict__ shifts,
             typename Cplx<T>::t shift0, int border) {
  using T2 = typename Cplx<T>::t;
  const int d = D > 0 ? D : d_rt;
  const int cells = d * d * R;
  int64_t task;
  int cell, cell_stride;
  if (cells <= 256) {
    const int tpb = 256 / cells;
    const int lt = threadIdx.x / cells;
    if (lt >= tpb) return;
    task = (int64_t)blockIdx.x * tpb + lt;
    cell = threadIdx.x - lt * cells;
    cell_stride = cells;  // single pass
  } else {
    task = blockIdx.x;
    cell = threadIdx.x;
    cell_stride = 256;
  }
  if (task >= n_tasks) return;
  int64_t a, e0, e1;
  int flags;
  if (tasks) {
    int4 t = tasks[task];
    a = t.x; e0 = t.y; e1 = t.z; flags = t.w;
  } else {
    a = task; e0 = row_ptr[task]; e1 = row_ptr[task + 1]; flags = TASK_DIAG;
  }
  const int dR = d * R;
  for (; cell < cells; cell += cell_stride) {
    const int i = cell / dR;
    const int rem = cell - i * dR;
    const int j = rem / R;
    const int r = rem - j * R;
    auto in = [&](int64_t b, int ii, int jj) -> T2 {
      int64_t idx = ((b * d + ii) * d + jj) * R + r;
      T2 v = x[idx];
      if (kvec) {
        T2 k = kvec[idx];
        v.x = fma(kc, k.x, v.x);
        v.y = fma(kc, k.y, v.y);
      }
      return v;
    };
    const int64_t out = ((a * d + i) * d + j) * R + r;
    T2 acc = (flags & TASK_ACC) ? y[out] : T2{0, 0};
    if (flags & TASK_DIAG) {
      T2 xa = in(a, i, j);
      T2 z = shifts ? shifts[r] : shift0;
      T2 c = csub(decay[a], z);
      acc = csub(acc, cmul(c, xa));
      // -i (H x)[i][j] + i (x H)[i][j]; operator 0 is H
      T2 hl{0, 0}, hr{0, 0};
      {
        const int nl = ell_cnt[i];
        const int32_t *cl = ell_col + (size_t)i * slots;
        const T2 *vl = ell_val + (size_t)i * slots;
        for (int s = 0; s < nl; ++s) hl = cfma(vl[s], in(a, cl[s], j), hl);
        const int nr = ell_cnt[d + j];
        const int32_t *cr = ell_col + (size_t)(d + j) * slots;
        const T2 *vr = ell_val + (size_t)(d + j) * slots;
        for (int s = 0; s < nr; ++s) hr = cfma(in(a, i, cr[s]), vr[s], hr);
      }
      T2 dlt = csub(hr, hl);  // i (hr - hl)
      acc.x -= dlt.y;
      acc.y += dlt.x;
    }
    for (int64_t e = e0; e < e1; ++e) {
      const int2 ed = edges[e];
      const int64_t b = ed.x;
      const int cid = (int)((uint32_t)ed.y >> 8);
      const T mult = (T)(int8_t)(ed.y & 0xff);
      const int op = coef_op[cid];
      const T2 cl = cscale(coef[2 * cid], mult);
      const T2 cr = cscale(coef[2 * cid + 1], mult);
      const size_t rowL = ((size_t)op * 2) * d + i;
      const size_t rowR = ((size_t)op * 2 + 1) * d + j;
      T2 L{0, 0}, Rv{0, 0};
      const int nl = ell_cnt[rowL];
      for (int s = 0; s < nl; ++s) L = cfma(ell_val[rowL * slots + s], in(b, ell_col[rowL * slots + s], j), L);
      const int nr = ell_cnt[rowR];
      for (int s = 0; s < nr; ++s) Rv = cfma(in(b, i, ell_col[rowR * slots + s]), ell_val[rowR * slots + s], Rv);
      acc = cfma(cl, L, acc);
      acc = cfma(cr, Rv, acc);
    }
    if (border && a == 0 && i == 0 && j == 0 && (flags & TASK_DIAG)) {
      T2 tr{0, 0};
      for (int ii = 0; ii < d; ++ii) tr = cadd(tr, in(0, ii, ii));
      acc = tr;
    }
    y[out] = acc;
  }
}

template <typename T>
static heom_status launch_T(Hier &h, const ApplyArgs &a, const int4 *tasks, int64_t n_tasks, const int2 *edges,
                            hipStream_t s) {
  using T2 = typename Cplx<T>::t;
  DeviceTables &D = h.dev;
  const int d = h.d;
  const int R = a.n_rhs;
  const int cells = d * d * R;
  if (n_tasks == 0) return HEOM_OK;
  int64_t grid = cells <= 256 ? (n_tasks + (256 / cells) - 1) / (256 / cells) : n_tasks;
  if (grid > 0x7fffffff) return fail(HEOM_ERR_UNSUPPORTED, "apply grid too large");
  const T2 *decay = std::is_same<T, double>::value ? (const T2 *)D.decay64 : (const T2 *)D.decay32;
  const T2 *ev = std::is_same<T, double>::value ? (const T2 *)D.ell_val64 : (const T2 *)D.ell_val32;
  const T2 *cf = std::is_same<T, double>::value ? (const T2 *)D.coef64 : (const T2 *)D.coef32;
  T2 sh0{(T)a.shift0.real(), (T)a.shift0.imag()};
  dim3 g((unsigned)grid), b(256);
#define HEOM_LAUNCH(DD)                                                                                    \
  hipLaunchKernelGGL((apply_kernel<T, DD>), g, b, 0, s, tasks, n_tasks, D.row_ptr, edges, decay, D.ell_cnt, \
                     D.ell_col, ev, h.ell.slots, D.coef_op, cf, (const T2 *)a.x, (const T2 *)a.k, (T)a.kc,    \
                     (T2 *)a.y, d, R, (const T2 *)a.shifts, sh0, a.border)
  switch (d) {
    case 2: HEOM_LAUNCH(2); break;
    case 4: HEOM_LAUNCH(4); break;
    case 8: HEOM_LAUNCH(8); break;
    case 16: HEOM_LAUNCH(16); break;
    default: HEOM_LAUNCH(0); break;
  }
#undef HEOM_LAUNCH
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

heom_status launch_apply(Hier &h, int precision, const ApplyArgs &a, hipStream_t s) {
  HEOM_TRY(check_apply(h, precision, a));
  if (precision == HEOM_FP64) return launch_T<double>(h, a, nullptr, h.N, h.dev.edges, s);
  return launch_T<float>(h, a, nullptr, h.N, h.dev.edges, s);
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
  DeviceTables &D = h.dev;
  for (size_t l = 0; l + 1 < D.task_off.size(); ++l) {
    const int64_t t0 = D.task_off[l], t1 = D.task_off[l + 1];
    if (precision == HEOM_FP64) HEOM_TRY(launch_T<double>(h, a, D.tasks + t0, t1 - t0, D.tedges, s));
    else HEOM_TRY(launch_T<float>(h, a, D.tasks + t0, t1 - t0, D.tedges, s));
  }
  return HEOM_OK;
}

}  // namespace heom
