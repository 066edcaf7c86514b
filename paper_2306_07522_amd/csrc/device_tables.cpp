// Upload of the hierarchy tables to the device, and the apply launch plans.
#include <algorithm>
#include <cmath>
#include <map>

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
                  D.ueig, D.eval, D.lind_f, D.lind_g, D.hoff64, D.hoff32};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  free_plan(D.base);
  free_slab_plan(D.slab);
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
    P.max_groups = P.max_edges = 0;
    for (const int4 &t : tasks) {
      if (t.z <= t.y) continue;
      P.max_groups = std::max(P.max_groups, t.z - t.y);
      P.max_edges = std::max(P.max_edges, groups[t.z - 1].y - groups[t.y].x);
    }
    return HEOM_OK;
  }
};

static heom_status build_slab_plan(const Hier &h, SlabPlan *out, size_t &tot, heom_slab_stats *stats);

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
  std::vector<double2> ho((size_t)h.d * h.d);
  std::vector<float2> ho32((size_t)h.d * h.d);
  for (int i = 0; i < h.d; ++i)
    for (int j = 0; j < h.d; ++j) {
      const cd v = i == j ? cd(0.0) : h.H[(size_t)i * h.d + j];
      ho[(size_t)i * h.d + j] = make_double2(v.real(), v.imag());
      ho32[(size_t)i * h.d + j] = make_float2((float)v.real(), (float)v.imag());
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
  constexpr double kCacheResidentBytes = 64.0 * 1024 * 1024;  // FP64 vector size below which the caches hold it
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
    if ((double)N * h.d * h.d * 16 < kCacheResidentBytes) {
      // A hierarchy whose vector stays in the caches gains nothing from the
      // windows; there the last round of waves decides the time, so the
      // tasks run longest first (most edges first) and the short ones fill
      // the tail.  Charge cavity, 3,165 ADOs of 20 x 20: 52.9 -> 44.0 us per
      // FP64 apply, 235 -> 197 us per RK4 step.
      std::stable_sort(order.begin(), order.end(), [&](int64_t p, int64_t q) {
        return h.row_ptr[p + 1] - h.row_ptr[p] > h.row_ptr[q + 1] - h.row_ptr[q];
      });
    }
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
      (st = upload(&D.hoff64, ho.data(), sizeof(double2) * ho.size(), tot)) ||
      (st = upload(&D.hoff32, ho32.data(), sizeof(float2) * ho32.size(), tot)) ||
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
      (st = build_slab_plan(h, &D.slab, tot, nullptr))) {
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
// c (an L-subset of exponent labels) feeds the up-terms (the C-type terms of
// eq:HEOM) of its L parents c \ {u}.  In the single-launch plan every parent
// gathers its children, so a child block leaves memory once for its own row
// and once per parent, and the parents' child sets overlap like an expander
// graph, so the caches see little of that reuse.
//
// The slab plan splits each tier-(L-1) parent P's up-terms by the position
// the added label u takes in the child:
//  * prefix part, u above the second largest label of P: the child then has
//    the same L - 2 smallest labels (its prefix core) as P minus max(P);
//  * suffix part, u below the second smallest label of P: the child has the
//    same L - 2 largest labels (its suffix core) as P minus min(P);
//  * for L >= 5 the positions in between stay with plain gathers.
// A slab is one core with its parents (core + one label beyond it) and its
// children (core + two labels beyond it), so a child is a pair of the slab's
// parents and feeds exactly those two.  Launch A runs the prefix slabs: per
// slab workgroup, the children arrive in sub-rounds of a round-robin pairing
// of the parents (no parent twice in a sub-round), are read once into LDS,
// add their terms to both parents' register accumulators from there, and
// have their own rows (self and down terms) computed; at the end the
// parents' prefix parts are written to y.  Launch A also runs the tiers
// below L - 1.  Launch B runs the suffix slabs the same way and finishes each
// parent's row (self, down terms, the rest of its up-terms) on top of y.  A
// top-tier block thus leaves memory once per launch.
static bool slab_applicable(const Hier &h) {
  const int L = h.Lf;
  // LDS of a slab workgroup in FP64: staging, two sub-round buffers, operator tables
  const size_t lds = (size_t)2 * kSlabSub * h.d * h.d * 16 + h.ell.c_col.size() * 20 + h.coefs.size() * 48 + 32 + h.d * 16;
  return h.Kb == 0 && h.importance_threshold <= 0.0 && L >= 3 && (int)h.tier_off.size() == L + 2 &&
         h.tier_off[L + 1] > h.tier_off[L] && (h.d == 8 || h.d == 16) && lds <= 160 * 1024;
}

// Round-robin pairing of n items (circle method): rounds of disjoint pairs
// covering every pair once.
static std::vector<std::vector<std::pair<int, int>>> round_robin(int n) {
  std::vector<std::vector<std::pair<int, int>>> rounds;
  const int m = n + (n & 1);  // a dummy item when n is odd
  for (int r = 0; r + 1 < m; ++r) {
    std::vector<std::pair<int, int>> pr;
    auto push = [&](int a, int b) {
      if (a < n && b < n) pr.push_back({std::min(a, b), std::max(a, b)});
    };
    push(r, m - 1);
    for (int k = 1; k < m / 2; ++k) push((r + k) % (m - 1), (r - k + (m - 1)) % (m - 1));
    rounds.push_back(pr);
  }
  return rounds;
}

struct SlabJob {
  std::vector<int2> vert;                 // {ADO, finalize task}
  std::vector<std::vector<int4>> subs;    // sub-rounds of entries
  int64_t cost = 0;
  int64_t group = 0;                      // jobs sharing a group read the same parents
  int64_t slab = 0, slab_cost = 0;        // parts of one slab share the children between them
};

struct PassHost {
  std::vector<int4> jt;
  std::vector<int32_t> sub;
  std::vector<int4> ent;
  std::vector<int2> vert;
  std::vector<int64_t> load;
  int max_vert = 0;
};

static heom_status layout_pass(std::vector<SlabJob> &jobs, PassHost &H) {
  // XCD assignment: groups (by cost) onto the 8 XCDs, least loaded first;
  // each XCD then runs its jobs costliest first.  Workgroup b runs on XCD
  // b % 8, so job i of XCD k sits at position 8 i + k.
  std::map<int64_t, int64_t> gcost;
  for (auto &j : jobs) gcost[j.group] += j.cost;
  std::vector<std::pair<int64_t, int64_t>> gl(gcost.begin(), gcost.end());
  std::stable_sort(gl.begin(), gl.end(), [](auto &a, auto &b) { return a.second > b.second; });
  std::map<int64_t, int> gx;
  std::vector<int64_t> load(8, 0);
  for (auto &g : gl) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    gx[g.first] = k;
    load[k] += g.second;
  }
  std::vector<std::vector<int>> lists(8);
  for (int i = 0; i < (int)jobs.size(); ++i) lists[gx[jobs[i].group]].push_back(i);
  size_t most = 0;
  for (auto &l : lists) {
    // costliest slabs first; the parts of one slab next to each other, so
    // that the children they share are still in L2 for the second part
    std::stable_sort(l.begin(), l.end(), [&](int a, int b) {
      if (jobs[a].slab_cost != jobs[b].slab_cost) return jobs[a].slab_cost > jobs[b].slab_cost;
      if (jobs[a].group != jobs[b].group) return jobs[a].group < jobs[b].group;
      return jobs[a].slab < jobs[b].slab;
    });
    most = std::max(most, l.size());
  }
  std::vector<int4> &jt = H.jt;
  std::vector<int32_t> &sub = H.sub;
  std::vector<int4> &ent = H.ent;
  std::vector<int2> &vert = H.vert;
  jt.assign(8 * most, make_int4(0, 0, 0, 0));
  for (size_t i = 0; i < most; ++i)
    for (int k = 0; k < 8; ++k) {
      if (i >= lists[k].size()) continue;
      SlabJob &J = jobs[lists[k][i]];
      if (J.vert.empty() && J.subs.empty()) continue;
      int4 &o = jt[8 * i + k];
      if (J.subs.empty() && !J.vert.empty() && J.vert[0].x < 0) {  // plain job
        o = make_int4(J.vert[0].y, -(int)J.vert.size(), 0, 0);
        continue;
      }
      o.x = (int)vert.size();
      o.y = (int)J.vert.size();
      o.z = (int)sub.size();
      o.w = (int)J.subs.size();
      H.max_vert = std::max(H.max_vert, (int)J.vert.size());
      for (auto &v : J.vert) vert.push_back(v);
      for (auto &sr : J.subs) {
        sub.push_back((int)ent.size());
        for (auto &e : sr) ent.push_back(e);
      }
      sub.push_back((int)ent.size());
    }
  if (ent.size() > 0x7fffffffull) return fail(HEOM_ERR_UNSUPPORTED, "slab plan too large");
  H.load = load;
  return HEOM_OK;
}

static heom_status upload_pass(const PassHost &H, SlabPass &P, size_t &tot) {
  HEOM_TRY(upload(&P.jobs, H.jt.data(), sizeof(int4) * H.jt.size(), tot));
  HEOM_TRY(upload(&P.sub, H.sub.data(), sizeof(int32_t) * H.sub.size(), tot));
  HEOM_TRY(upload(&P.ent, H.ent.data(), sizeof(int4) * H.ent.size(), tot));
  HEOM_TRY(upload(&P.vert, H.vert.data(), sizeof(int2) * H.vert.size(), tot));
  P.n_jobs = (int64_t)H.jt.size();
  P.cost = H.load;
  return HEOM_OK;
}

void free_slab_plan(SlabPlan &p) {
  free_plan(p.tasks);
  for (auto &q : p.pass) {
    for (void *ptr : {(void *)q.jobs, (void *)q.sub, (void *)q.ent, (void *)q.vert})
      if (ptr) (void)hipFree(ptr);
    q = SlabPass();
  }
  p.built = false;
}

// Host side of the slab plan: companion tasks and the job layout of both
// launches, with the coverage checks.  Uploaded when `out` is given.
static heom_status build_slab_plan(const Hier &h, SlabPlan *out, size_t &tot, heom_slab_stats *stats) {
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
  // vertices of each slab, in ascending order of their extra label
  std::vector<std::vector<int64_t>> pv(n_core), sv(n_core);
  for (int64_t P = v0; P < c0; ++P) {
    const uint64_t m = h.fmask[P];
    const int64_t kp = core_of(m & ~(1ull << top_bit(m))), ks = core_of(m & ~(1ull << low_bit(m)));
    if (kp < 0 || ks < 0) return fail(HEOM_ERR_ARG, "slab plan: missing core ADO");
    pv[kp].push_back(P);
    sv[ks].push_back(P);
  }
  // edge of row P that reaches ADO c
  auto edge_to = [&](int64_t P, int64_t c) -> int64_t {
    for (int64_t e = h.row_ptr[P]; e < h.row_ptr[P + 1]; ++e)
      if (h.ecol[e] == c) return e;
    return -1;
  };
  auto part_of = [&](int64_t P, int64_t e) -> int {  // 0 prefix, 1 suffix, 2 plain gather, -1 not an up edge
    const int64_t c = h.ecol[e];
    if (c < c0) return -1;
    const uint64_t m = h.fmask[P];
    const int u = low_bit(h.fmask[c] & ~m);
    const int second_top = top_bit(m & ~(1ull << top_bit(m)));
    const int second_low = low_bit(m & ~(1ull << low_bit(m)));
    if (u > second_top) return 0;
    if (u < second_low) return 1;
    return 2;
  };
  PlanBuilder pb(h);
  std::vector<int64_t> es;
  int64_t n_cov = 0, n_self = 0;  // coverage check: every edge and every self term exactly once
  int64_t n_own = 0, n_vert[2] = {0, 0};  // every child row scheduled once, every parent once per launch
  auto task_row = [&](int64_t a, bool self, bool acc) {
    pb.add_task(a, es, self, acc);
    n_cov += (int64_t)es.size();
    n_self += self;
    return (int)pb.tasks.size() - 1;
  };
  // companion tasks, in launch order.  The rows launch (the ordinary wave
  // kernel) runs the tiers below L - 1 and the children's own rows (self and
  // down terms), the latter in windows of their largest label: three of a
  // child's four parents hold that label too, so the window's parents are
  // re-read from cache.
  for (int64_t a = 0; a < v0; ++a) {
    es.clear();
    for (int64_t e = h.row_ptr[a]; e < h.row_ptr[a + 1]; ++e) es.push_back(e);
    task_row(a, true, false);
  }
  {
    std::vector<std::pair<int64_t, int64_t>> order;
    order.reserve(c1 - c0);
    for (int64_t c = c0; c < c1; ++c) order.push_back({top_bit(h.fmask[c]), c});
    std::stable_sort(order.begin(), order.end());
    for (auto &oc : order) {
      es.clear();
      for (int64_t e = h.row_ptr[oc.second]; e < h.row_ptr[oc.second + 1]; ++e) es.push_back(e);
      task_row(oc.second, true, false);
      ++n_own;
    }
  }
  const int64_t n_rows = (int64_t)pb.tasks.size();
  // companion tasks finishing the parents' rows (launch B)
  std::vector<int> fin_task(c0 - v0, -1);
  for (int64_t P = v0; P < c0; ++P) {
    es.clear();
    for (int64_t e = h.row_ptr[P]; e < h.row_ptr[P + 1]; ++e) {
      const int pt = part_of(P, e);
      if (pt == -1 || pt == 2) es.push_back(e);
    }
    fin_task[P - v0] = task_row(P, true, true);
  }
  std::vector<SlabJob> jobsA, jobsB;
  int64_t costA = 0, costB = 0;
  // one slab -> jobs.  side_part: which part of the parents' up-terms this
  // launch owns (0 prefix, 1 suffix).
  auto slab_jobs = [&](const std::vector<int64_t> &V, uint64_t core, int side_part, int64_t group, int64_t slab_id,
                       std::vector<SlabJob> &out_jobs, int64_t max_cost) -> heom_status {
    const int m = (int)V.size();
    if (m == 0) return HEOM_OK;
    const size_t first_job = out_jobs.size();
    std::vector<int> extra(m);
    for (int t = 0; t < m; ++t) extra[t] = low_bit(h.fmask[V[t]] & ~core);
    auto rounds = round_robin(m);
    // cost of the whole slab decides the split into vertex ranges
    const int64_t n_pairs = (int64_t)m * (m - 1) / 2;
    const int64_t whole = n_pairs + (int64_t)m * (side_part == 0 ? 1 : 8);
    int G = (int)std::max<int64_t>(1, (whole + max_cost - 1) / std::max<int64_t>(max_cost, 1));
    G = std::max(G, (m + kSlabWaves * kSlabVmax - 1) / (kSlabWaves * kSlabVmax));
    G = std::min(G, std::max(1, m / 4));
    // split points: equal numbers of vertices
    std::vector<int> cut(G + 1, m);
    cut[0] = 0;
    {
      std::vector<int64_t> wsum(m + 1, 0);
      for (int t = 0; t < m; ++t) wsum[t + 1] = wsum[t] + 1;
      for (int g = 1; g < G; ++g) {
        int t = cut[g - 1] + 1;
        while (t < m && wsum[t] * G < wsum[m] * g) ++t;
        cut[g] = std::min(t, m - (G - g));
      }
    }
    for (int g = 0; g < G; ++g) {
      const int lo = cut[g], hi = cut[g + 1];
      if (hi - lo > kSlabWaves * kSlabVmax) return fail(HEOM_ERR_ARG, "slab plan: too many vertices in one job");
      SlabJob J;
      J.group = group;
      for (int t = lo; t < hi; ++t) J.vert.push_back(make_int2((int)V[t], side_part == 1 ? fin_task[V[t] - v0] : -1));
      for (auto &rd : rounds) {
        std::vector<int4> cur;
        for (auto &pr : rd) {
          const int a = pr.first, b = pr.second;
          const bool ma = a >= lo && a < hi, mb = b >= lo && b < hi;
          if (!ma && !mb) continue;
          const uint64_t cm = core | (1ull << extra[a]) | (1ull << extra[b]);
          const int64_t c = lookup_ado(h, cm, 0);
          if (c < c0 || c >= c1) return fail(HEOM_ERR_ARG, "slab plan: missing child ADO");
          // a side is this job's when its vertex is and its edge belongs to
          // this launch's part (for L = 3 a suffix-slab pair feeds only its
          // upper vertex: the lower one takes that child in its prefix part)
          auto side = [&](int t, bool mine) -> int {
            if (!mine) return 127 << 24;
            const int64_t e = edge_to(V[t], c);
            if (e < 0) return -1;
            if (part_of(V[t], e) != side_part) return 127 << 24;
            const int cid = (int)((uint32_t)h.einfo[e] >> 8);
            const int mult = (int)(int8_t)(h.einfo[e] & 0xff);
            if (cid >= (1 << 23) || (mult != 1 && mult != -1)) return -1;
            n_cov += 1;
            return ((t - lo) << 24) | (mult < 0 ? (1 << 23) : 0) | cid;
          };
          const int sa = side(a, ma), sb = side(b, mb);
          if (sa < 0 || sb < 0) return fail(HEOM_ERR_ARG, "slab plan: inconsistent edge");
          if (sa == (127 << 24) && sb == (127 << 24)) continue;
          cur.push_back(make_int4((int)c, -1, sa, sb));
          J.cost += 1;
          if ((int)cur.size() == kSlabSub) {
            J.subs.push_back(cur);
            cur.clear();
          }
        }
        if (!cur.empty()) J.subs.push_back(cur);
      }
      J.cost += (int64_t)J.vert.size() * (side_part == 0 ? 1 : 8);
      n_vert[side_part] += (int64_t)J.vert.size();
      J.slab = slab_id;
      out_jobs.push_back(std::move(J));
    }
    int64_t sc = 0;
    for (size_t q = first_job; q < out_jobs.size(); ++q) sc += out_jobs[q].cost;
    for (size_t q = first_job; q < out_jobs.size(); ++q) out_jobs[q].slab_cost = sc;
    return HEOM_OK;
  };
  // target job cost: about two jobs per compute unit
  const int64_t n_pair_total = c1 - c0;
  const int64_t maxA = std::max<int64_t>(64, (n_pair_total + (c0 - v0)) / 512);
  const int64_t maxB = std::max<int64_t>(64, (n_pair_total * 1 + (c0 - v0) * 8) / 512);
  for (int64_t k = 0; k < n_core; ++k) {
    const uint64_t core = h.fmask[k0 + k];
    // jobs that read the same non-local parents share a group: the core minus its smallest label
    const int64_t group = (int64_t)(core & ~(core ? (1ull << low_bit(core)) : 0ull));
    HEOM_TRY(slab_jobs(pv[k], core, 0, group, k, jobsA, maxA));
    HEOM_TRY(slab_jobs(sv[k], core, 1, group, k, jobsB, maxB));
  }
  for (auto &j : jobsA) costA += j.cost;
  for (auto &j : jobsB) costB += j.cost;
  if (n_self != h.N || n_cov != h.row_ptr[h.N] || n_own != c1 - c0 || n_vert[0] != c0 - v0 || n_vert[1] != c0 - v0)
    return fail(HEOM_ERR_ARG, "slab plan: rows not covered exactly once");
  PassHost HA, HB;
  HEOM_TRY(layout_pass(jobsA, HA));
  HEOM_TRY(layout_pass(jobsB, HB));
  if (stats) {
    stats->built = 1;
    stats->children = c1 - c0;
    stats->parents = c0 - v0;
    const PassHost *hp[2] = {&HA, &HB};
    for (int l = 0; l < 2; ++l) {
      stats->jobs[l] = (int64_t)hp[l]->jt.size();
      stats->entries[l] = (int64_t)hp[l]->ent.size();
      stats->max_vertices[l] = hp[l]->max_vert;
      for (int k = 0; k < 8; ++k) stats->xcd_cost[l][k] = hp[l]->load[k];
    }
    stats->cost[0] = costA;
    stats->cost[1] = costB;
  }
  if (!out) return HEOM_OK;
  HEOM_TRY(pb.upload_to(out->tasks, tot));
  out->tasks.task_off = {0, (int64_t)pb.tasks.size()};
  out->n_rows = n_rows;
  HEOM_TRY(upload_pass(HA, out->pass[0], tot));
  HEOM_TRY(upload_pass(HB, out->pass[1], tot));
  out->built = true;
  return HEOM_OK;
}

}  // namespace heom

extern "C" heom_status heom_slab_plan_stats(const heom_hier *hw, heom_slab_stats *out) {
  using namespace heom;
  return guarded([&]() -> heom_status {
    if (!hw || !out) return fail(HEOM_ERR_ARG, "slab_plan_stats: NULL argument");
    *out = heom_slab_stats{};
    size_t tot = 0;
    return build_slab_plan(*hw->impl, nullptr, tot, out);
  });
}

namespace heom {

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
