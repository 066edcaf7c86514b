// Upload of the hierarchy tables to the device, and the apply launch plans.
#include <algorithm>
#include <cmath>

#include "dense.h"
#include "internal.h"
#include "device_common.h"

namespace heom {

template <typename P>
static heom_status upload(P **dst, const void *src, size_t bytes, size_t &total) {
  if (bytes == 0) bytes = 16;
  HEOM_HIP_CHECK(hipMalloc((void **)dst, bytes));
  if (src) HEOM_HIP_CHECK(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
  total += bytes;
  return HEOM_OK;
}

void free_plan(Plan &p) {
  if (p.tasks) (void)hipFree(p.tasks);
  if (p.groups) (void)hipFree(p.groups);
  if (p.gedges) (void)hipFree(p.gedges);
  p = Plan();
}

void free_device(Hier &h) {
  DeviceTables &D = h.dev;
  if (D.device < 0) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(D.device);
  void *ptrs[] = {D.decay64, D.decay32, D.ell_cnt, D.ell_col, D.op_slots, D.ell_val64, D.ell_val32,
                  D.coef_op, D.coef64, D.coef32, D.hdiag, D.hdiag32, D.lev, D.c_meta, D.c_col, D.c_val64, D.c_val32,
                  D.ueig, D.eval, D.lind_f, D.lind_g};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  free_plan(D.base);
  free_plan(D.tiled);
  (void)hipSetDevice(cur);
  D = DeviceTables();
}

// One task's edges -> groups.  Edges that share an operator and an
// identical coefficient pair form one group (weight = the edge's integer
// multiplier); a self group (the H commutator and the decay) leads when the
// task owns its diagonal.
struct PlanBuilder {
  const Hier &h;
  std::vector<int4> tasks, groups;
  std::vector<int2> gedges;
  explicit PlanBuilder(const Hier &hh) : h(hh) {}

  void add_task(int64_t a, const std::vector<int64_t> &edge_ids, bool self, bool acc) {
    const int64_t g0 = (int64_t)groups.size();
    if (self) {
      groups.push_back(make_int4((int)gedges.size(), (int)gedges.size() + 1, h.coef_H, 1));
      gedges.push_back(make_int2((int)a, 1));
    }
    std::vector<int64_t> es(edge_ids);
    auto cid = [&](int64_t e) { return (int)((uint32_t)h.einfo[e] >> 8); };
    auto key_less = [&](int64_t p, int64_t q) {
      const CoefEntry &A = h.coefs[cid(p)], &B = h.coefs[cid(q)];
      if (A.op != B.op) return A.op < B.op;
      double ka[4] = {A.cl.real(), A.cl.imag(), A.cr.real(), A.cr.imag()};
      double kb[4] = {B.cl.real(), B.cl.imag(), B.cr.real(), B.cr.imag()};
      for (int t = 0; t < 4; ++t)
        if (ka[t] != kb[t]) return ka[t] < kb[t];
      return h.ecol[p] < h.ecol[q];
    };
    auto same = [&](int64_t p, int64_t q) {
      const CoefEntry &A = h.coefs[cid(p)], &B = h.coefs[cid(q)];
      return A.op == B.op && A.cl == B.cl && A.cr == B.cr;
    };
    std::sort(es.begin(), es.end(), key_less);
    size_t i = 0;
    while (i < es.size()) {
      size_t j = i + 1;
      while (j < es.size() && same(es[i], es[j])) ++j;
      const int e0 = (int)gedges.size();
      for (size_t t = i; t < j; ++t)
        gedges.push_back(make_int2(h.ecol[es[t]], (int)(int8_t)(h.einfo[es[t]] & 0xff)));
      groups.push_back(make_int4(e0, (int)gedges.size(), cid(es[i]), 0));
      i = j;
    }
    const int flags = (self ? TASK_DIAG : 0) | (acc ? TASK_ACC : 0);
    tasks.push_back(make_int4((int)a, (int)g0, (int)groups.size(), flags));
  }

  heom_status upload_to(Plan &P, size_t &tot) {
    if (gedges.size() > 0x7fffffffull || groups.size() > 0x7fffffffull)
      return fail(HEOM_ERR_UNSUPPORTED, "apply plan too large");
    HEOM_TRY(upload(&P.tasks, tasks.data(), sizeof(int4) * tasks.size(), tot));
    HEOM_TRY(upload(&P.groups, groups.data(), sizeof(int4) * groups.size(), tot));
    HEOM_TRY(upload(&P.gedges, gedges.data(), sizeof(int2) * gedges.size(), tot));
    P.bytes = sizeof(int4) * (tasks.size() + groups.size()) + sizeof(int2) * gedges.size();
    return HEOM_OK;
  }
};

heom_status ensure_device(Hier &h) {
  int dev = 0;
  HEOM_HIP_CHECK(hipGetDevice(&dev));
  DeviceTables &D = h.dev;
  if (D.device == dev) return HEOM_OK;
  if (D.device >= 0) return fail(HEOM_ERR_ARG, "hierarchy tables live on another device");
  D.device = dev;
  size_t tot = 0;
  const int64_t N = h.N;
  std::vector<double2> dc64(N);
  std::vector<float2> dc32(N);
  for (int64_t a = 0; a < N; ++a) {
    dc64[a] = make_double2(h.decay[a].real(), h.decay[a].imag());
    dc32[a] = make_float2((float)h.decay[a].real(), (float)h.decay[a].imag());
  }
  const OpEll &L = h.ell;
  std::vector<double2> ev64(L.val.size());
  std::vector<float2> ev32(L.val.size());
  for (size_t i = 0; i < L.val.size(); ++i) {
    ev64[i] = make_double2(L.val[i].real(), L.val[i].imag());
    ev32[i] = make_float2((float)L.val[i].real(), (float)L.val[i].imag());
  }
  const size_t nc = h.coefs.size();
  std::vector<int32_t> cop(nc);
  std::vector<double2> c64(2 * nc);
  std::vector<float2> c32(2 * nc);
  for (size_t c = 0; c < nc; ++c) {
    cop[c] = h.coefs[c].op;
    c64[2 * c] = make_double2(h.coefs[c].cl.real(), h.coefs[c].cl.imag());
    c64[2 * c + 1] = make_double2(h.coefs[c].cr.real(), h.coefs[c].cr.imag());
    c32[2 * c] = make_float2((float)h.coefs[c].cl.real(), (float)h.coefs[c].cl.imag());
    c32[2 * c + 1] = make_float2((float)h.coefs[c].cr.real(), (float)h.coefs[c].cr.imag());
  }
  std::vector<double2> hd(h.d);
  std::vector<float2> hd32(h.d);
  for (int i = 0; i < h.d; ++i) {
    hd[i] = make_double2(L.hdiag[i].real(), L.hdiag[i].imag());
    hd32[i] = make_float2((float)L.hdiag[i].real(), (float)L.hdiag[i].imag());
  }
  // eigen-decomposition of H for the block preconditioner (column-major copy in)
  std::vector<cd> Hc((size_t)h.d * h.d), Ucol;
  std::vector<double> Ev;
  for (int i = 0; i < h.d; ++i)
    for (int j = 0; j < h.d; ++j) Hc[i + (size_t)j * h.d] = h.H[(size_t)i * h.d + j];
  if (!eigh_jacobi(h.d, Hc, Ev, Ucol)) return fail(HEOM_ERR_NAN, "eigen-decomposition of H did not converge");
  std::vector<double2> ue((size_t)h.d * h.d);
  for (int i = 0; i < h.d; ++i)
    for (int k = 0; k < h.d; ++k) ue[(size_t)i * h.d + k] = make_double2(Ucol[i + (size_t)k * h.d].real(),
                                                                         Ucol[i + (size_t)k * h.d].imag());
  {
    double dmin = 0.0;
    for (const auto &b : h.bexp)
      if (b.chi.real() > 0 && (dmin == 0.0 || b.chi.real() < dmin)) dmin = b.chi.real();
    for (const auto &f : h.fexp)
      if (f.gamma.real() > 0 && (dmin == 0.0 || f.gamma.real() < dmin)) dmin = f.gamma.real();
    h.block_delta = dmin > 0 ? dmin : 1.0;
  }
  // Lindblad jump operators and G = sum_k F_k^dagger F_k
  std::vector<double2> lf, lg;
  if (!h.lind.empty()) {
    const int d = h.d;
    std::vector<cd> G((size_t)d * d, cd(0));
    for (const auto &F : h.lind) {
      for (int e = 0; e < d * d; ++e) lf.push_back(make_double2(F[e].real(), F[e].imag()));
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
          cd acc(0);
          for (int l = 0; l < d; ++l) acc += std::conj(F[(size_t)l * d + i]) * F[(size_t)l * d + j];
          G[(size_t)i * d + j] += acc;
        }
    }
    for (const cd &z : G) lg.push_back(make_double2(z.real(), z.imag()));
  }
  std::vector<int32_t> meta(3 * L.n_ops);
  for (int o = 0; o < L.n_ops; ++o) { meta[3 * o] = L.c_off[o]; meta[3 * o + 1] = L.c_ns[o]; meta[3 * o + 2] = L.c_real[o]; }
  std::vector<double2> cv64(L.c_val.size());
  std::vector<float2> cv32(L.c_val.size());
  for (size_t i = 0; i < L.c_val.size(); ++i) {
    cv64[i] = make_double2(L.c_val[i].real(), L.c_val[i].imag());
    cv32[i] = make_float2((float)L.c_val[i].real(), (float)L.c_val[i].imag());
  }
  PlanBuilder pb(h);
  std::vector<int64_t> es;
  std::vector<int64_t> order(N);
  for (int64_t a = 0; a < N; ++a) order[a] = a;
  {
    // Task order: ADOs grouped into windows by their largest exponent label
    // (stable, so tiers stay ascending inside a window).  A top-tier ADO and
    // three of its four parents share its window, so the parents' up-term
    // gathers find it in cache shortly after (or before) its own task.
    std::vector<int> key(N, -1);
    for (int64_t a = 0; a < N; ++a) {
      int k = -1;
      const uint64_t m = h.fmask[a];
      if (m) k = 63 - __builtin_clzll(m);
      for (int b = h.Kb - 1; b >= 0; --b)
        if (h.bocc[(size_t)a * h.Kb + b]) { k = std::max(k, h.Kf + b); break; }
      key[a] = k;
    }
    std::stable_sort(order.begin(), order.end(), [&](int64_t p, int64_t q) { return key[p] < key[q]; });
  }
  for (int64_t oi = 0; oi < N; ++oi) {
    const int64_t a = order[oi];
    es.clear();
    for (int64_t e = h.row_ptr[a]; e < h.row_ptr[a + 1]; ++e) es.push_back(e);
    pb.add_task(a, es, true, false);
  }
  heom_status st;
  if ((st = upload(&D.decay64, dc64.data(), sizeof(double2) * N, tot)) ||
      (st = upload(&D.decay32, dc32.data(), sizeof(float2) * N, tot)) ||
      (st = upload(&D.ell_cnt, L.cnt.data(), sizeof(int32_t) * L.cnt.size(), tot)) ||
      (st = upload(&D.ell_col, L.col.data(), sizeof(int32_t) * L.col.size(), tot)) ||
      (st = upload(&D.op_slots, L.op_slots.data(), sizeof(int32_t) * L.op_slots.size(), tot)) ||
      (st = upload(&D.ell_val64, ev64.data(), sizeof(double2) * ev64.size(), tot)) ||
      (st = upload(&D.ell_val32, ev32.data(), sizeof(float2) * ev32.size(), tot)) ||
      (st = upload(&D.coef_op, cop.data(), sizeof(int32_t) * nc, tot)) ||
      (st = upload(&D.coef64, c64.data(), sizeof(double2) * 2 * nc, tot)) ||
      (st = upload(&D.coef32, c32.data(), sizeof(float2) * 2 * nc, tot)) ||
      (st = upload(&D.hdiag, hd.data(), sizeof(double2) * h.d, tot)) ||
      (st = upload(&D.hdiag32, hd32.data(), sizeof(float2) * h.d, tot)) ||
      (st = upload(&D.lev, h.lev.data(), sizeof(int2) * N, tot)) ||
      (st = upload(&D.ueig, ue.data(), sizeof(double2) * ue.size(), tot)) ||
      (st = upload(&D.eval, Ev.data(), sizeof(double) * Ev.size(), tot)) ||
      (!lf.empty() && (st = upload(&D.lind_f, lf.data(), sizeof(double2) * lf.size(), tot))) ||
      (!lg.empty() && (st = upload(&D.lind_g, lg.data(), sizeof(double2) * lg.size(), tot))) ||
      (st = upload(&D.c_meta, meta.data(), sizeof(int32_t) * meta.size(), tot)) ||
      (st = upload(&D.c_col, L.c_col.data(), sizeof(int32_t) * L.c_col.size(), tot)) ||
      (st = upload(&D.c_val64, cv64.data(), sizeof(double2) * cv64.size(), tot)) ||
      (st = upload(&D.c_val32, cv32.data(), sizeof(float2) * cv32.size(), tot)) ||
      (st = pb.upload_to(D.base, tot))) {
    free_device(h);
    return st;
  }
  D.base.task_off = {0, (int64_t)pb.tasks.size()};
  D.bytes = tot;
  return HEOM_OK;
}

// Tiled plan.  The leaf ADOs (no higher-tier neighbour: the last tier) are
// split into n_chunks contiguous column blocks.  Launch 0 computes every
// non-leaf row without its leaf neighbours; launch k computes the leaf rows
// of chunk k in full and adds, to every non-leaf row, the terms whose
// neighbour lies in chunk k.  Each launch therefore streams one chunk of
// leaf blocks once and re-reads it from cache.
heom_status ensure_tiled_plan(Hier &h, int n_chunks) {
  DeviceTables &D = h.dev;
  const int64_t N = h.N;
  const int64_t leaf0 = h.tier_off[h.tier_off.size() - 2];
  const int64_t nleaf = N - leaf0;
  n_chunks = (int)std::max<int64_t>(1, std::min<int64_t>(n_chunks, std::max<int64_t>(nleaf, 1)));
  if (D.tiled.tasks && D.tiled.n_chunks == n_chunks) return HEOM_OK;
  free_plan(D.tiled);
  PlanBuilder pb(h);
  std::vector<int64_t> task_off{0};
  std::vector<int64_t> es;
  for (int64_t a = 0; a < leaf0; ++a) {
    es.clear();
    for (int64_t e = h.row_ptr[a]; e < h.row_ptr[a + 1]; ++e)
      if (h.ecol[e] < leaf0) es.push_back(e);
    pb.add_task(a, es, true, false);
  }
  task_off.push_back((int64_t)pb.tasks.size());
  for (int c = 0; c < n_chunks; ++c) {
    const int64_t c0 = leaf0 + nleaf * c / n_chunks, c1 = leaf0 + nleaf * (c + 1) / n_chunks;
    for (int64_t a = c0; a < c1; ++a) {
      es.clear();
      for (int64_t e = h.row_ptr[a]; e < h.row_ptr[a + 1]; ++e) es.push_back(e);
      pb.add_task(a, es, true, false);
    }
    for (int64_t a = 0; a < leaf0; ++a) {
      es.clear();
      for (int64_t e = h.row_ptr[a]; e < h.row_ptr[a + 1]; ++e)
        if (h.ecol[e] >= c0 && h.ecol[e] < c1) es.push_back(e);
      if (!es.empty()) pb.add_task(a, es, false, true);
    }
    task_off.push_back((int64_t)pb.tasks.size());
  }
  size_t tot = 0;
  HEOM_TRY(pb.upload_to(D.tiled, tot));
  D.tiled.task_off = task_off;
  D.tiled.n_chunks = n_chunks;
  return HEOM_OK;
}

}  // namespace heom
