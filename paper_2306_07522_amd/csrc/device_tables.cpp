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
  free_plan(D.slab);
  for (auto &kv : D.tiled) free_plan(kv.second);
  (void)hipSetDevice(cur);
  D = DeviceTables();
  h.dev_ready.store(-1, std::memory_order_release);
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

static heom_status build_slab_plan(Hier &h, Plan &out, size_t &tot);

// Upload of every table and launch plan to device `dev`; runs once per
// handle, under h.dev_mu.
static heom_status upload_tables(Hier &h, int dev) {
  DeviceTables &D = h.dev;
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
      (st = pb.upload_to(D.base, tot)) ||
      (st = build_slab_plan(h, D.slab, tot))) {
    free_device(h);
    return st;
  }
  D.base.task_off = {0, (int64_t)pb.tasks.size()};
  D.bytes = tot;
  return HEOM_OK;
}

heom_status ensure_device(Hier &h) {
  int dev = 0;
  HEOM_HIP_CHECK(hipGetDevice(&dev));
  if (h.dev_ready.load(std::memory_order_acquire) == dev) return HEOM_OK;
  std::lock_guard<std::mutex> lock(h.dev_mu);
  const int ready = h.dev_ready.load(std::memory_order_relaxed);
  if (ready == dev) return HEOM_OK;
  if (ready >= 0) return fail(HEOM_ERR_ARG, "hierarchy tables live on another device");
  HEOM_TRY(upload_tables(h, dev));
  h.dev_ready.store(dev, std::memory_order_release);
  return HEOM_OK;
}

// ---------------------------------------------------------------- slab plan
// For a purely fermionic hierarchy cut at tier L = n_max, every top-tier ADO
// c (an L-subset of exponent labels) feeds the up-terms of its L parents
// c \ {u} (eq:HEOM, the C-type terms).  The single-launch plan has every
// parent gather its children, so each child block is fetched once for its
// own row and once per parent; the parents' child sets overlap like an
// expander graph, and the cache sees little of that reuse.
//
// The slab plan splits each tier-(L-1) parent P's up-terms by the position
// the added label u takes in the child:
//  * prefix part, u above the second largest label of P: the child then
//    shares its L - 2 smallest labels (its prefix core) with P minus max(P);
//  * suffix part, every other u: for L = 4 the child shares its L - 2
//    largest labels (its suffix core) with P minus min(P).
// A slab is the set of parents and children with one core.  Launch A runs
// the tiers below L - 1 in full and then, slab by slab, the prefix parts of
// the slab's parents (written to y) followed by the full rows of its
// children (self and down terms).  Launch B runs, slab by slab, the rest of
// each parent's row (self, down terms, suffix part) and adds it to y.  A
// slab's children are read by the slab's parents and children close
// together in time; each XCD walks a contiguous run of slabs, so those
// re-reads stay in its L2 and a top-tier block leaves HBM about once per
// launch instead of once per parent.
static bool slab_applicable(const Hier &h) {
  const int L = h.Lf;
  return h.Kb == 0 && h.importance_threshold <= 0.0 && L >= 3 && (int)h.tier_off.size() == L + 2 &&
         h.tier_off[L + 1] > h.tier_off[L];
}

// Cuts tasks [0, n) with costs c into 8 contiguous runs of similar cost,
// at unit boundaries (unit_start[t] = true where a slab begins).
static std::vector<int64_t> xcd_split(const std::vector<int64_t> &cost, const std::vector<char> &unit_start) {
  const int64_t n = (int64_t)cost.size();
  std::vector<int64_t> pre(n + 1, 0);
  for (int64_t t = 0; t < n; ++t) pre[t + 1] = pre[t] + cost[t];
  std::vector<int64_t> off(9, 0);
  off[8] = n;
  int64_t t = 0;
  for (int k = 1; k < 8; ++k) {
    const double target = (double)pre[n] * k / 8.0;
    t = std::max(t, off[k - 1]);
    while (t < n && (double)pre[t + 1] <= target) ++t;  // pre[t] <= target < pre[t + 1]
    // nearest unit boundary at or around t
    int64_t lo = t, hi = t;
    while (lo > off[k - 1] && !unit_start[lo]) --lo;
    while (hi < n && !unit_start[hi]) ++hi;
    off[k] = (target - (double)pre[lo] <= (double)pre[hi] - target) ? lo : hi;
    if (off[k] < off[k - 1]) off[k] = off[k - 1];
  }
  return off;
}

static heom_status build_slab_plan(Hier &h, Plan &out, size_t &tot) {
  if (!slab_applicable(h)) return HEOM_OK;
  const int L = h.Lf;
  const int64_t v0 = h.tier_off[L - 1], c0 = h.tier_off[L], c1 = h.tier_off[L + 1];
  const int64_t k0 = h.tier_off[L - 2];
  const int64_t n_core = v0 - k0;
  auto top_bit = [](uint64_t m) { return 63 - __builtin_clzll(m); };
  auto low_bit = [](uint64_t m) { return __builtin_ctzll(m); };
  auto core_of = [&](uint64_t m) -> int64_t {
    const int64_t a = lookup_ado(h, m, 0);
    return (a >= k0 && a < v0) ? a - k0 : -1;
  };
  std::vector<std::vector<int64_t>> pv(n_core), pc(n_core), sv(n_core);
  for (int64_t P = v0; P < c0; ++P) {
    const uint64_t m = h.fmask[P];
    const int64_t kp = core_of(m & ~(1ull << top_bit(m))), ks = core_of(m & ~(1ull << low_bit(m)));
    if (kp < 0 || ks < 0) return fail(HEOM_ERR_ARG, "slab plan: missing core ADO");
    pv[kp].push_back(P);
    sv[ks].push_back(P);
  }
  for (int64_t c = c0; c < c1; ++c) {
    uint64_t m = h.fmask[c];
    m &= ~(1ull << top_bit(m));
    m &= ~(1ull << top_bit(m));
    const int64_t kp = core_of(m);
    if (kp < 0) return fail(HEOM_ERR_ARG, "slab plan: missing core ADO");
    pc[kp].push_back(c);
  }
  // up edge e of parent P belongs to the prefix part when its added label
  // lies above the second largest label of P
  auto prefix_part = [&](int64_t P, int64_t e) {
    const uint64_t m = h.fmask[P];
    const int64_t c = h.ecol[e];
    if (c < c0) return false;  // down edge
    const int u = low_bit(h.fmask[c] & ~m);
    const int second = top_bit(m & ~(1ull << top_bit(m)));
    return u > second;
  };
  PlanBuilder pb(h);
  std::vector<int64_t> es, cost;
  std::vector<char> ustart;
  int64_t n_edges = 0, n_self = 0;
  auto add = [&](int64_t a, bool self, bool acc, bool first) {
    pb.add_task(a, es, self, acc);
    cost.push_back(1 + (int64_t)es.size());
    ustart.push_back(first);
    n_edges += (int64_t)es.size();
    n_self += self;
  };
  // launch A
  for (int64_t a = 0; a < v0; ++a) {
    es.clear();
    for (int64_t e = h.row_ptr[a]; e < h.row_ptr[a + 1]; ++e) es.push_back(e);
    add(a, true, false, true);
  }
  for (int64_t k = 0; k < n_core; ++k) {
    bool first = true;
    for (int64_t P : pv[k]) {
      es.clear();
      for (int64_t e = h.row_ptr[P]; e < h.row_ptr[P + 1]; ++e)
        if (prefix_part(P, e)) es.push_back(e);
      add(P, false, false, first);
      first = false;
    }
    for (int64_t c : pc[k]) {
      es.clear();
      for (int64_t e = h.row_ptr[c]; e < h.row_ptr[c + 1]; ++e) es.push_back(e);
      add(c, true, false, first);
      first = false;
    }
  }
  const int64_t nA = (int64_t)pb.tasks.size();
  std::vector<int64_t> costA(cost.begin(), cost.end());
  std::vector<char> ustartA(ustart.begin(), ustart.end());
  cost.clear();
  ustart.clear();
  // launch B
  for (int64_t k = 0; k < n_core; ++k) {
    bool first = true;
    for (int64_t P : sv[k]) {
      es.clear();
      for (int64_t e = h.row_ptr[P]; e < h.row_ptr[P + 1]; ++e)
        if (!prefix_part(P, e)) es.push_back(e);
      add(P, true, true, first);
      first = false;
    }
  }
  const int64_t nB = (int64_t)pb.tasks.size() - nA;
  // every ADO's row exactly once: one self group per ADO, every edge once
  if (nB != c0 - v0 || nA != c1 - (c0 - v0) || n_self != h.N || n_edges != h.row_ptr[h.N])
    return fail(HEOM_ERR_ARG, "slab plan: rows not covered exactly once");
  HEOM_TRY(pb.upload_to(out, tot));
  out.task_off = {0, nA, nA + nB};
  out.xcd_off = {xcd_split(costA, ustartA), xcd_split(cost, ustart)};
  return HEOM_OK;
}

// Tiled plan.  The leaf ADOs (no higher-tier neighbour: the last tier) are
// split into n_chunks contiguous column blocks.  Launch 0 computes every
// non-leaf row without its leaf neighbours; launch k computes the leaf rows
// of chunk k in full and adds, to every non-leaf row, the terms whose
// neighbour lies in chunk k.  Each launch therefore streams one chunk of
// leaf blocks once and re-reads it from cache.
heom_status ensure_tiled_plan(Hier &h, int n_chunks, const Plan **out) {
  HEOM_TRY(ensure_device(h));
  std::lock_guard<std::mutex> lock(h.dev_mu);
  DeviceTables &D = h.dev;
  const int64_t N = h.N;
  const int64_t leaf0 = h.tier_off[h.tier_off.size() - 2];
  const int64_t nleaf = N - leaf0;
  n_chunks = (int)std::max<int64_t>(1, std::min<int64_t>(n_chunks, std::max<int64_t>(nleaf, 1)));
  auto it = D.tiled.find(n_chunks);
  if (it != D.tiled.end()) {
    *out = &it->second;
    return HEOM_OK;
  }
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
  Plan pl;
  heom_status st = pb.upload_to(pl, tot);
  if (st != HEOM_OK) {
    free_plan(pl);
    return st;
  }
  pl.task_off = task_off;
  pl.n_chunks = n_chunks;
  Plan &slot = D.tiled[n_chunks];
  slot = pl;
  *out = &slot;
  return HEOM_OK;
}

}  // namespace heom
