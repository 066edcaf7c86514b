// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <complex>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "heom.h"

namespace heom {

using cd = std::complex<double>;

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
heom_status fail(heom_status s, const std::string &msg);

// Runs the body of a C entry point so that no C++ exception crosses the C
// boundary: host allocation failures become HEOM_ERR_ALLOC, anything else
// HEOM_ERR_ARG with its message.
template <class F>
heom_status guarded(F &&body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc &) {
    return fail(HEOM_ERR_ALLOC, "host allocation failed");
  } catch (const std::exception &e) {
    return fail(HEOM_ERR_ARG, e.what());
  } catch (...) {
    return fail(HEOM_ERR_ARG, "unexpected host error");
  }
}

#define HEOM_HIP_CHECK(expr)                                                         \
  do {                                                                               \
    hipError_t _e = (expr);                                                          \
    if (_e != hipSuccess)                                                            \
      return ::heom::fail(HEOM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

#define HEOM_TRY(expr)                \
  do {                                \
    heom_status _s = (expr);          \
    if (_s != HEOM_OK) return _s;     \
  } while (0)

// ---------------------------------------------------------------- tables
// Edge coefficient entry: the term  cl * O x_b + cr * x_b O  with O = ops[op];
// the per-edge multiplier (bosonic multiplicity or fermionic reorder sign) is
// applied on top.
struct CoefEntry {
  int op;
  cd cl, cr;
};

// ELL form of every operator, left (rows of O) and right (rows of O^T).
struct OpEll {
  int n_ops = 0, d = 0, slots = 0;
  std::vector<int32_t> op_slots;  // [n_ops]
  std::vector<int32_t> cnt;  // [n_ops][2][d]
  std::vector<int32_t> col;  // [n_ops][2][d][slots]
  std::vector<cd> val;       // [n_ops][2][d][slots]
  // compact form for the wave kernel: op o owns entries [off[o], off[o] +
  // 2 d ns[o]) laid out [side][row][slot]; operator 0 (H) keeps only its
  // off-diagonal entries, its diagonal goes to hdiag.
  std::vector<int32_t> c_off, c_ns, c_real;
  std::vector<int32_t> c_col;
  std::vector<cd> c_val;
  std::vector<cd> hdiag;
};

// A launch plan: tasks (one output ADO each), each a run of edge groups.
// A group shares one operator and one coefficient pair (cl, cr); its edges
// carry a small integer weight, so the group contributes
//   cl * O u + cr * u O,   u = sum_e w_e x_{b_e}.
struct Plan {
  int n_chunks = -1;             // -1: untiled single launch
  int4 *tasks = nullptr;         // {a, g0, g1, flags}
  int4 *groups = nullptr;        // {e0, e1, coef_id, self}
  int2 *gedges = nullptr;        // {b, w}
  std::vector<int64_t> task_off; // [n_launch + 1]
  size_t bytes = 0;
  int max_groups = 0;            // largest number of groups of one task
  int max_edges = 0;             // largest number of edges of one task
};

// Slab passes of the apply (built in device_tables.cpp, run by
// apply_slab.hip).  A job is one workgroup's share of a label slab: the
// slab's parents (vertices) whose up-term accumulators the workgroup keeps in
// registers, and the slab's children, fed to it in sub-rounds (disjoint pairs
// of vertices, so no two children of a sub-round touch the same vertex) that
// are staged once in LDS and serve both of their parents from there.
//   jobs: {vert_off, n_vert, sub_off, n_sub}; n_vert < 0 marks a plain job
//         running companion tasks [vert_off, vert_off - n_vert) one per wave;
//   sub:  entry boundaries, sub[sub_off + s] .. sub[sub_off + s + 1];
//   ent:  {child ADO, companion task of the child's own row or -1,
//          side A, side B}, a side packing the coefficient entry (bits
//          0..22), a negative reorder sign (bit 23) and the job-local vertex
//          slot (bits 24..30; 127 = not this job's vertex);
//   vert: {ADO, companion task finishing the vertex's row or -1}.
struct SlabPass {
  int4 *jobs = nullptr;
  int32_t *sub = nullptr;
  int4 *ent = nullptr;
  int2 *vert = nullptr;
  int64_t n_jobs = 0;
  std::vector<int64_t> cost;    // per XCD, for the record
};
constexpr int kSlabWaves = 8;   // waves per slab workgroup
constexpr int kSlabSub = 16;    // children per sub-round
constexpr int kSlabVmax = 4;    // vertex accumulators per wave
struct SlabPlan {
  Plan tasks;                   // companion tasks, groups and edges
  int64_t n_rows = 0;           // companion tasks [0, n_rows): the rows launch
  SlabPass pass[2];
  bool built = false;
};

// Device copies of the tables, one set per precision for the values.
struct DeviceTables {
  int device = -1;
  double2 *decay64 = nullptr;   // [N]
  float2 *decay32 = nullptr;
  int32_t *ell_cnt = nullptr;
  int32_t *ell_col = nullptr;
  int32_t *op_slots = nullptr;  // [n_ops] max row count of each operator
  double2 *ell_val64 = nullptr;
  float2 *ell_val32 = nullptr;
  int32_t *coef_op = nullptr;   // [n_coef]
  double2 *coef64 = nullptr;    // [n_coef][2] (cl, cr)
  float2 *coef32 = nullptr;
  double2 *hdiag = nullptr;     // [d] diagonal of H
  double2 *hoff64 = nullptr;    // [d][d] H with its diagonal zeroed, row-major (MFMA self group)
  float2 *hoff32 = nullptr;
  int2 *lev = nullptr;          // [N] (m, n) levels of every ADO
  float2 *hdiag32 = nullptr;
  double2 *ueig = nullptr;      // [d][d] row-major eigenvectors of H (H = U diag(E) U^H)
  double *eval = nullptr;       // [d] eigenvalues of H, ascending
  double2 *lind_f = nullptr;    // [n_lind][d][d] Lindblad jump operators, row-major
  double2 *lind_g = nullptr;    // [d][d] sum_k F_k^dagger F_k
  int32_t *c_meta = nullptr;    // [n_ops][3] (off, ns, real) of the compact ELL
  int32_t *c_col = nullptr;
  double2 *c_val64 = nullptr;
  float2 *c_val32 = nullptr;
  Plan base;                    // untiled, one launch: every ADO gathers all its neighbours
  SlabPlan slab;                // two launches over label slabs (built = false when not applicable)
  std::map<int, Plan> tiled;    // top tier split into chunks, by chunk count
  size_t bytes = 0;
};

struct Hier {
  int d = 0, Kb = 0, Kf = 0, Lb = 0, Lf = 0, parity = 1;
  double importance_threshold = 0.0;
  // block preconditioner: denominators of modulus below this are replaced by
  // -block_delta (the slowest bath decay rate, min Re chi / Re gamma)
  double block_delta = 1.0;
  std::vector<cd> H;  // d*d row-major
  struct BosExp { int op, u; cd xi, chi; };
  // rank: position in the order eq:importance runs over (per bath: nu = +1
  // terms h = 1.., then nu = -1 terms)
  // bath: index of the input bath record the exponent came from
  struct FermExp { int op_ann, nu, partner; cd eta, gamma; int rank; int bath; };
  std::vector<BosExp> bexp;
  std::vector<FermExp> fexp;
  std::vector<int> bath_kind;  // per input bath record: HEOM_BOSON or HEOM_FERMION
  std::vector<cd> parity_op;   // d*d row-major, empty when none was given
  // Lindbladian add-on (eq:Lindbladian): jump operators, each d*d row-major
  std::vector<std::vector<cd>> lind;
  std::vector<std::vector<cd>> ops;  // ops[0] = H
  // ADOs
  int64_t N = 0;
  std::vector<uint8_t> bocc;       // [N][Kb]
  std::vector<uint64_t> fmask;     // [N]
  std::vector<int32_t> lev;        // [N][2] (m, n)
  std::vector<int64_t> tier_off;   // [n_tiers+1]
  std::vector<cd> decay;           // [N]
  std::vector<int64_t> row_ptr;    // [N+1]
  std::vector<int32_t> ecol;       // [E]
  std::vector<int32_t> einfo;      // [E] coef_id << 8 | (uint8) mult
  std::vector<CoefEntry> coefs;   // last entry: the H commutator (op 0, -i, +i)
  int coef_H = 0;
  OpEll ell;
  int64_t n_leaf = 0;
  // device upload: done once, on first use, under dev_mu; dev_ready holds the
  // device id once every table and plan is in place (-1 before)
  std::mutex dev_mu;
  std::atomic<int> dev_ready{-1};
  // bosonic code for dictionary lookups
  std::vector<uint64_t> bos_pow;
  std::vector<std::pair<uint64_t, uint64_t>> keys;  // sorted (fmask, bos code)
  std::vector<int32_t> key_index;                   // ADO index of keys[r]
  DeviceTables dev;
};

// host builder (host_hierarchy.cpp)
heom_status build_hier(int d, const double *H, int n_baths, const heom_bath *baths, int m_max, int n_max,
                       int parity, const double *parity_op, double importance_threshold, std::unique_ptr<Hier> &out);
int64_t lookup_ado(const Hier &h, uint64_t fmask, uint64_t bcode);

// device upload / kernels (device.hip)
heom_status ensure_device(Hier &h);
// the tiled plan of n_chunks chunks (built on first request, kept until heom_free)
heom_status ensure_tiled_plan(Hier &h, int n_chunks, const Plan **out);
void free_device(Hier &h);
void free_plan(Plan &p);

struct ApplyArgs {
  const void *x = nullptr;      // input vector
  const void *k = nullptr;      // optional: input is x + kc * k
  double kc = 0.0;
  void *y = nullptr;
  int n_rhs = 1;
  const void *shifts = nullptr; // device complex[n_rhs] of the precision, or null
  cd shift0 = 0.0;              // used when shifts == null
  int border = 0;               // 1: replace y[0][0][0] by Tr rho_0 (steady-state row)
  // Optional epilogue (one right-hand side, pull plan, no Lindblad terms):
  // y = eacc * (M x) + sum_j ec[j] * ev[j], elementwise, and when y2 is set
  // also y2 = eacc2 * (M x) + sum_j ec2[j] * ev[j].  An ev[j] may be y itself
  // (each element is read before it is written, by the same lane).
  int hmfma = 0;                // 1: the self group's H terms on the matrix cores (d = 16, wave kernel)
  bool epi = false;
  const void *ev[4] = {nullptr, nullptr, nullptr, nullptr};
  double ec[4] = {0.0, 0.0, 0.0, 0.0};
  double eacc = 1.0;
  void *y2 = nullptr;
  double ec2[4] = {0.0, 0.0, 0.0, 0.0};
  double eacc2 = 0.0;
};
heom_status launch_apply(Hier &h, int precision, const ApplyArgs &a, hipStream_t s);
// as launch_apply with an explicit plan (HEOM_PLAN_*)
heom_status launch_apply_plan(Hier &h, int precision, const ApplyArgs &a, int plan, hipStream_t s);
// the three slab launches (apply_slab.hip)
heom_status launch_apply_slab(Hier &h, int precision, const ApplyArgs &a, hipStream_t s);
// the wave kernel over tasks [t0, t1) of a plan (apply.hip)
heom_status launch_plan_range(Hier &h, int precision, const ApplyArgs &a, const Plan &pl, int64_t t0, int64_t t1,
                              hipStream_t s);
void free_slab_plan(SlabPlan &p);
// whole RK4 steps in one workgroup for hierarchies of at most 1024 elements
bool rk4_small_fits(const Hier &h);
heom_status launch_rk4_small(Hier &h, int precision, void *x, double dt, int64_t steps, int64_t save_every,
                             int64_t step0, int64_t n_saves, void *traj, hipStream_t s);
heom_status launch_apply_tiled(Hier &h, int precision, const ApplyArgs &a, int n_chunks, hipStream_t s);
// y += sum_k J(F_k)[x (+ kc k)] on every ADO (after the apply proper); no-op without jump operators
heom_status launch_lindblad(Hier &h, int precision, const ApplyArgs &a, hipStream_t s);
constexpr int kLindbladMaxD = 32;

}  // namespace heom

struct heom_hier {
  std::unique_ptr<heom::Hier> impl;
};
