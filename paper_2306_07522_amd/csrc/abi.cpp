// C ABI entry points: handles, dictionary, apply.
#include <cstring>
#include <string>

#include "internal.h"

namespace heom {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

heom_status fail(heom_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

}  // namespace heom

using namespace heom;

extern "C" {

const char *heom_version(void) { return "heomx 0.1 (gfx950)"; }

const char *heom_last_error(void) { return g_last_error.c_str(); }

const char *heom_status_string(heom_status s) {
  switch (s) {
    case HEOM_OK: return "ok";
    case HEOM_ERR_ARG: return "invalid argument";
    case HEOM_ERR_ALLOC: return "allocation failed";
    case HEOM_ERR_HIP: return "HIP runtime error";
    case HEOM_ERR_NOT_CONVERGED: return "not converged";
    case HEOM_ERR_SINGULAR: return "singular / breakdown";
    case HEOM_ERR_UNSUPPORTED: return "unsupported";
    case HEOM_ERR_NAN: return "non-finite value";
    default: return "unknown status";
  }
}

heom_status heom_build_hierarchy(int32_t d, const double *H, int32_t n_baths, const heom_bath *baths,
                                 int32_t m_max, int32_t n_max, int32_t parity, const double *parity_op,
                                 heom_hier **out) {
  if (!out) return fail(HEOM_ERR_ARG, "out is NULL");
  *out = nullptr;
  try {
    std::unique_ptr<Hier> h;
    HEOM_TRY(build_hier(d, H, n_baths, baths, m_max, n_max, parity, parity_op, 0.0, h));
    auto *w = new heom_hier;
    w->impl = std::move(h);
    *out = w;
    return HEOM_OK;
  } catch (const std::bad_alloc &) {
    return fail(HEOM_ERR_ALLOC, "host allocation failed while building the hierarchy");
  } catch (const std::exception &e) {
    return fail(HEOM_ERR_ARG, e.what());
  }
}

heom_status heom_build_hierarchy_pruned(int32_t d, const double *H, int32_t n_baths, const heom_bath *baths,
                                        int32_t m_max, int32_t n_max, int32_t parity, const double *parity_op,
                                        double importance_threshold, heom_hier **out) {
  if (!out) return fail(HEOM_ERR_ARG, "out is NULL");
  *out = nullptr;
  try {
    std::unique_ptr<Hier> h;
    HEOM_TRY(build_hier(d, H, n_baths, baths, m_max, n_max, parity, parity_op, importance_threshold, h));
    auto *w = new heom_hier;
    w->impl = std::move(h);
    *out = w;
    return HEOM_OK;
  } catch (const std::bad_alloc &) {
    return fail(HEOM_ERR_ALLOC, "host allocation failed while building the hierarchy");
  } catch (const std::exception &e) {
    return fail(HEOM_ERR_ARG, e.what());
  }
}

void heom_free(heom_hier *h) {
  if (!h) return;
  free_device(*h->impl);
  delete h;
}

heom_status heom_hierarchy_info(const heom_hier *hw, heom_info *o) {
  if (!hw || !o) return fail(HEOM_ERR_ARG, "NULL argument");
  const Hier &h = *hw->impl;
  std::memset(o, 0, sizeof(*o));
  o->n_ado = h.N;
  o->d = h.d;
  o->n_bos_exp = h.Kb;
  o->n_ferm_exp = h.Kf;
  o->m_max = h.Lb;
  o->n_max = h.Lf;
  o->parity = h.parity;
  o->n_ops = (int32_t)h.ops.size();
  o->n_edges = (int64_t)h.ecol.size();
  o->n_leaf = h.n_leaf;
  o->n_tiers = (int32_t)h.tier_off.size() - 1;
  for (size_t t = 0; t < h.tier_off.size() && t < 34; ++t) o->tier_offset[t] = h.tier_off[t];
  o->table_bytes = (int64_t)(sizeof(int64_t) * (h.N + 1) + 8 * h.ecol.size() + 24 * h.N);
  o->vector_bytes_fp64 = h.N * (int64_t)h.d * h.d * 16;
  return HEOM_OK;
}

heom_status heom_hierarchy_ados(const heom_hier *hw, int32_t *bos_occ, uint64_t *ferm_mask, int32_t *level) {
  if (!hw) return fail(HEOM_ERR_ARG, "NULL handle");
  const Hier &h = *hw->impl;
  for (int64_t a = 0; a < h.N; ++a) {
    if (bos_occ)
      for (int k = 0; k < h.Kb; ++k) bos_occ[a * h.Kb + k] = h.bocc[a * h.Kb + k];
    if (ferm_mask) ferm_mask[a] = h.fmask[a];
    if (level) { level[2 * a] = h.lev[2 * a]; level[2 * a + 1] = h.lev[2 * a + 1]; }
  }
  return HEOM_OK;
}

heom_status heom_ado_index(const heom_hier *hw, const int32_t *bos_occ, const int32_t *ferm_ids, int32_t n_f,
                           int64_t *idx, int32_t *sign) {
  if (!hw || !idx || !sign || n_f < 0 || (n_f > 0 && !ferm_ids)) return fail(HEOM_ERR_ARG, "NULL argument");
  const Hier &h = *hw->impl;
  *idx = -1;
  *sign = 0;
  uint64_t code = 0;
  int m = 0;
  for (int k = 0; k < h.Kb; ++k) {
    int o = bos_occ ? bos_occ[k] : 0;
    if (o < 0) return fail(HEOM_ERR_ARG, "negative occupation");
    if (o > h.Lb) return HEOM_OK;
    m += o;
    code += (uint64_t)o * h.bos_pow[k];
  }
  if (m > h.Lb || n_f > h.Lf) return HEOM_OK;
  uint64_t mask = 0;
  int s = 1;
  for (int i = 0; i < n_f; ++i) {
    int q = ferm_ids[i];
    if (q < 0 || q >= h.Kf) return fail(HEOM_ERR_ARG, "fermionic exponent index out of range");
    if (mask >> q & 1ull) return HEOM_OK;  // Pauli: repeated exponent
    // moving q (at list position i) past the later, larger indices
    for (int j = i + 1; j < n_f; ++j)
      if (ferm_ids[j] > q) s = -s;
    mask |= 1ull << q;
  }
  int64_t a = lookup_ado(h, mask, code);
  if (a < 0) return HEOM_OK;
  *idx = a;
  *sign = s;
  return HEOM_OK;
}

heom_status heom_hierarchy_tables(const heom_hier *hw, double *decay, int64_t *row_ptr, int32_t *col, int32_t *kind,
                                  int32_t *expo, int32_t *mult) {
  if (!hw) return fail(HEOM_ERR_ARG, "NULL handle");
  const Hier &h = *hw->impl;
  if (decay)
    for (int64_t a = 0; a < h.N; ++a) { decay[2 * a] = h.decay[a].real(); decay[2 * a + 1] = h.decay[a].imag(); }
  if (row_ptr)
    for (int64_t a = 0; a <= h.N; ++a) row_ptr[a] = h.row_ptr[a];
  const int Kb = h.Kb, Kf = h.Kf;
  for (size_t e = 0; e < h.ecol.size(); ++e) {
    if (col) col[e] = h.ecol[e];
    int cid = (int)((uint32_t)h.einfo[e] >> 8);
    int mu = (int)(int8_t)(h.einfo[e] & 0xff);
    int k, x;
    if (cid < Kb) { k = 0; x = cid; }
    else if (cid < 2 * Kb) { k = 1; x = cid - Kb; }
    else if (cid < 2 * Kb + 2 * Kf) { k = 2; x = (cid - 2 * Kb) / 2; }
    else { k = 3; x = (cid - 2 * Kb - 2 * Kf) / 2; }
    if (kind) kind[e] = k;
    if (expo) expo[e] = x;
    if (mult) mult[e] = mu;
  }
  return HEOM_OK;
}

static heom_status heom_apply_body(heom_hier *hw, int32_t precision, const void *x_dev, void *y_dev, int32_t n_rhs,
                       const double *shift, void *stream) {
  if (!hw) return fail(HEOM_ERR_ARG, "NULL handle");
  if (x_dev == y_dev) return fail(HEOM_ERR_ARG, "apply: x and y must not alias");
  ApplyArgs a;
  a.x = x_dev;
  a.y = y_dev;
  a.n_rhs = n_rhs;
  a.shift0 = shift ? cd(shift[0], shift[1]) : cd(0.0);
  return launch_apply(*hw->impl, precision, a, (hipStream_t)stream);
}

heom_status heom_apply(heom_hier *hw, int32_t precision, const void *x_dev, void *y_dev, int32_t n_rhs,
                       const double *shift, void *stream) {
  return guarded([&] { return heom_apply_body(hw, precision, x_dev, y_dev, n_rhs, shift, stream); });
}

static heom_status heom_apply_plan_body(heom_hier *hw, int32_t precision, const void *x_dev, void *y_dev,
                                        int32_t n_rhs, const double *shift, int32_t plan, void *stream) {
  if (!hw) return fail(HEOM_ERR_ARG, "NULL handle");
  if (x_dev == y_dev) return fail(HEOM_ERR_ARG, "apply: x and y must not alias");
  ApplyArgs a;
  a.x = x_dev;
  a.y = y_dev;
  a.n_rhs = n_rhs;
  a.shift0 = shift ? cd(shift[0], shift[1]) : cd(0.0);
  return launch_apply_plan(*hw->impl, precision, a, plan, (hipStream_t)stream);
}

heom_status heom_apply_plan(heom_hier *hw, int32_t precision, const void *x_dev, void *y_dev, int32_t n_rhs,
                            const double *shift, int32_t plan, void *stream) {
  return guarded([&] { return heom_apply_plan_body(hw, precision, x_dev, y_dev, n_rhs, shift, plan, stream); });
}

static heom_status heom_apply_shifted_body(heom_hier *hw, int32_t precision, const void *x_dev, void *y_dev, int32_t n_rhs,
                               const void *shifts_dev, void *stream) {
  if (!hw) return fail(HEOM_ERR_ARG, "NULL handle");
  if (x_dev == y_dev) return fail(HEOM_ERR_ARG, "apply: x and y must not alias");
  if (!shifts_dev) return fail(HEOM_ERR_ARG, "apply_shifted: NULL shifts");
  ApplyArgs a;
  a.x = x_dev;
  a.y = y_dev;
  a.n_rhs = n_rhs;
  a.shifts = shifts_dev;
  return launch_apply(*hw->impl, precision, a, (hipStream_t)stream);
}

heom_status heom_apply_shifted(heom_hier *hw, int32_t precision, const void *x_dev, void *y_dev, int32_t n_rhs,
                               const void *shifts_dev, void *stream) {
  return guarded([&] { return heom_apply_shifted_body(hw, precision, x_dev, y_dev, n_rhs, shifts_dev, stream); });
}

static heom_status heom_apply_steady_operator_body(heom_hier *hw, int32_t precision, const void *x_dev, void *y_dev,
                                       void *stream) {
  if (!hw) return fail(HEOM_ERR_ARG, "NULL handle");
  if (x_dev == y_dev) return fail(HEOM_ERR_ARG, "apply: x and y must not alias");
  ApplyArgs a;
  a.x = x_dev;
  a.y = y_dev;
  a.n_rhs = 1;
  a.border = 1;
  return launch_apply(*hw->impl, precision, a, (hipStream_t)stream);
}

heom_status heom_apply_steady_operator(heom_hier *hw, int32_t precision, const void *x_dev, void *y_dev,
                                       void *stream) {
  return guarded([&] { return heom_apply_steady_operator_body(hw, precision, x_dev, y_dev, stream); });
}

static heom_status heom_apply_tiled_body(heom_hier *hw, int32_t precision, const void *x_dev, void *y_dev, int32_t n_rhs,
                             const double *shift, int32_t n_chunks, void *stream) {
  if (!hw) return fail(HEOM_ERR_ARG, "NULL handle");
  Hier &h = *hw->impl;
  if (x_dev == y_dev) return fail(HEOM_ERR_ARG, "apply: x and y must not alias");
  ApplyArgs a;
  a.x = x_dev;
  a.y = y_dev;
  a.n_rhs = n_rhs;
  a.shift0 = shift ? cd(shift[0], shift[1]) : cd(0.0);
  return launch_apply_tiled(h, precision, a, n_chunks, (hipStream_t)stream);
}

heom_status heom_apply_tiled(heom_hier *hw, int32_t precision, const void *x_dev, void *y_dev, int32_t n_rhs,
                             const double *shift, int32_t n_chunks, void *stream) {
  return guarded([&] { return heom_apply_tiled_body(hw, precision, x_dev, y_dev, n_rhs, shift, n_chunks, stream); });
}

heom_status heom_prepare(heom_hier *hw) {
  return guarded([&]() -> heom_status {
    if (!hw) return fail(HEOM_ERR_ARG, "prepare: NULL handle");
    return ensure_device(*hw->impl);
  });
}

}  // extern "C"
