// Upload of the hierarchy tables to the device, and the tiled apply plan.
#include <algorithm>
#include <cmath>

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

void free_device(Hier &h) {
  DeviceTables &D = h.dev;
  if (D.device < 0) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(D.device);
  void *ptrs[] = {D.row_ptr, D.edges, D.decay64, D.decay32, D.ell_cnt, D.ell_col, D.ell_val64,
                  D.ell_val32, D.coef_op, D.coef64, D.coef32, D.hdiag_re, D.tasks, D.tedges};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  (void)hipSetDevice(cur);
  D = DeviceTables();
}

heom_status ensure_device(Hier &h) {
  int dev = 0;
  HEOM_HIP_CHECK(hipGetDevice(&dev));
  DeviceTables &D = h.dev;
  if (D.device == dev) return HEOM_OK;
  if (D.device >= 0) return fail(HEOM_ERR_ARG, "hierarchy tables live on another device");
  D.device = dev;
  size_t tot = 0;
  const int64_t N = h.N;
  const int64_t E = (int64_t)h.ecol.size();
  std::vector<int2> edges(E);
  for (int64_t e = 0; e < E; ++e) edges[e] = make_int2(h.ecol[e], h.einfo[e]);
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
  std::vector<double> hd(h.d);
  for (int i = 0; i < h.d; ++i) hd[i] = h.H[i * h.d + i].real();
  heom_status st;
  if ((st = upload(&D.row_ptr, h.row_ptr.data(), sizeof(int64_t) * (N + 1), tot)) ||
      (st = upload(&D.edges, edges.data(), sizeof(int2) * E, tot)) ||
      (st = upload(&D.decay64, dc64.data(), sizeof(double2) * N, tot)) ||
      (st = upload(&D.decay32, dc32.data(), sizeof(float2) * N, tot)) ||
      (st = upload(&D.ell_cnt, L.cnt.data(), sizeof(int32_t) * L.cnt.size(), tot)) ||
      (st = upload(&D.ell_col, L.col.data(), sizeof(int32_t) * L.col.size(), tot)) ||
      (st = upload(&D.ell_val64, ev64.data(), sizeof(double2) * ev64.size(), tot)) ||
      (st = upload(&D.ell_val32, ev32.data(), sizeof(float2) * ev32.size(), tot)) ||
      (st = upload(&D.coef_op, cop.data(), sizeof(int32_t) * nc, tot)) ||
      (st = upload(&D.coef64, c64.data(), sizeof(double2) * 2 * nc, tot)) ||
      (st = upload(&D.coef32, c32.data(), sizeof(float2) * 2 * nc, tot)) ||
      (st = upload(&D.hdiag_re, hd.data(), sizeof(double) * h.d, tot))) {
    free_device(h);
    return st;
  }
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
  if (D.tasks && D.n_chunks == n_chunks) return HEOM_OK;
  if (D.tasks) { (void)hipFree(D.tasks); D.tasks = nullptr; }
  if (D.tedges) { (void)hipFree(D.tedges); D.tedges = nullptr; }
  const int64_t N = h.N;
  const int64_t leaf0 = h.tier_off[h.tier_off.size() - 2];
  const int64_t nleaf = N - leaf0;
  n_chunks = (int)std::max<int64_t>(1, std::min<int64_t>(n_chunks, std::max<int64_t>(nleaf, 1)));
  std::vector<int4> tasks;
  std::vector<int2> te;
  D.task_off.assign(1, 0);
  // launch 0
  for (int64_t a = 0; a < leaf0; ++a) {
    int64_t e0 = (int64_t)te.size();
    for (int64_t e = h.row_ptr[a]; e < h.row_ptr[a + 1]; ++e)
      if (h.ecol[e] < leaf0) te.push_back(make_int2(h.ecol[e], h.einfo[e]));
    tasks.push_back(make_int4((int)a, (int)e0, (int)te.size(), TASK_DIAG));
  }
  D.task_off.push_back((int64_t)tasks.size());
  for (int c = 0; c < n_chunks; ++c) {
    const int64_t c0 = leaf0 + nleaf * c / n_chunks, c1 = leaf0 + nleaf * (c + 1) / n_chunks;
    for (int64_t a = c0; a < c1; ++a) {
      int64_t e0 = (int64_t)te.size();
      for (int64_t e = h.row_ptr[a]; e < h.row_ptr[a + 1]; ++e) te.push_back(make_int2(h.ecol[e], h.einfo[e]));
      tasks.push_back(make_int4((int)a, (int)e0, (int)te.size(), TASK_DIAG));
    }
    for (int64_t a = 0; a < leaf0; ++a) {
      int64_t e0 = (int64_t)te.size();
      for (int64_t e = h.row_ptr[a]; e < h.row_ptr[a + 1]; ++e)
        if (h.ecol[e] >= c0 && h.ecol[e] < c1) te.push_back(make_int2(h.ecol[e], h.einfo[e]));
      if ((int64_t)te.size() > e0) tasks.push_back(make_int4((int)a, (int)e0, (int)te.size(), TASK_ACC));
    }
    D.task_off.push_back((int64_t)tasks.size());
  }
  if (te.size() > 0x7fffffffull) return fail(HEOM_ERR_UNSUPPORTED, "tiled plan too large");
  size_t tot = 0;
  HEOM_TRY(upload(&D.tasks, tasks.data(), sizeof(int4) * tasks.size(), tot));
  HEOM_TRY(upload(&D.tedges, te.data(), sizeof(int2) * te.size(), tot));
  D.n_chunks = n_chunks;
  return HEOM_OK;
}

}  // namespace heom
