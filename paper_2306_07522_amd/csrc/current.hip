// Electronic current from a fermionic lead into the system (eq:last): a
// readout of the first-level fermionic ADOs of a stationary state.
//
//   I_alpha = i sum_{nu, h, sigma} (-1)^{delta_{nu,-}} Tr[d_sigma^{nu-bar} rho_{|{alpha,nu,h,sigma}}]
//
// (e = hbar = 1).  The host resolves every exponent of the lead's bath records
// to the index of its single-exponent ADO through the hierarchy dictionary and
// prepares the matrices i (-1)^{delta_{nu,-}} d^{nu-bar}; one workgroup sums
// Tr[O_t X_{a_t}] over all terms with a fixed-order reduction.
#include <mutex>
#include <vector>

#include "device_common.h"
#include "internal.h"

namespace heom {

// out = sum_t sum_{i,j} O_t[i][j] X_{a_t}[j][i]  (X row-major d x d blocks).
// With neg = NULL the O_t carry their coefficient; otherwise O_t is the
// plain operator times i, or times -i where neg[t] is set.
__global__ void __launch_bounds__(256) current_kernel(const double2 *__restrict__ x, int d, int n_terms,
                                                      const int64_t *__restrict__ ado, const double2 *__restrict__ ops,
                                                      const int32_t *__restrict__ neg, double2 *__restrict__ out) {
  __shared__ double sx[256], sy[256];
  const int dd = d * d;
  const int64_t total = (int64_t)n_terms * dd;
  double ax = 0.0, ay = 0.0;
  for (int64_t k = threadIdx.x; k < total; k += blockDim.x) {
    const int t = (int)(k / dd), e = (int)(k % dd);
    const int i = e / d, j = e % d;
    double2 o = ops[k];
    if (neg) o = neg[t] ? make_double2(o.y, -o.x) : make_double2(-o.y, o.x);  // -i O or i O
    const double2 v = x[ado[t] * dd + j * d + i];
    ax += o.x * v.x - o.y * v.y;
    ay += o.x * v.y + o.y * v.x;
  }
  sx[threadIdx.x] = ax;
  sy[threadIdx.x] = ay;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sx[threadIdx.x] += sx[threadIdx.x + h];
      sy[threadIdx.x] += sy[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = make_double2(sx[0], sy[0]);
}

}  // namespace heom

using namespace heom;

static heom_status check_current_args(heom_hier *hw, const void *x_dev, int32_t n_rec, const int32_t *records,
                                      double *out) {
  if (!hw || !x_dev || !records || !out || n_rec < 1) return fail(HEOM_ERR_ARG, "current: NULL argument");
  Hier &h = *hw->impl;
  if (h.parity != 1) return fail(HEOM_ERR_ARG, "current: needs the even-parity hierarchy of the stationary state");
  for (int r = 0; r < n_rec; ++r) {
    const int b = records[r];
    if (b < 0 || b >= (int)h.bath_kind.size()) return fail(HEOM_ERR_ARG, "current: bath index out of range");
    if (h.bath_kind[b] != HEOM_FERMION) return fail(HEOM_ERR_ARG, "current: a lead is made of fermionic baths");
    for (int q = 0; q < r; ++q)
      if (records[q] == b) return fail(HEOM_ERR_ARG, "current: repeated bath index");
  }
  return HEOM_OK;
}

static heom_status heom_current_body(heom_hier *hw, const void *x_dev, int32_t n_rec, const int32_t *records,
                                    double *out, void *stream) {
  HEOM_TRY(check_current_args(hw, x_dev, n_rec, records, out));
  Hier &h = *hw->impl;
  out[0] = out[1] = 0.0;
  const int d = h.d, dd = d * d;
  std::vector<int64_t> ado;
  std::vector<double2> ops;
  for (int q = 0; q < h.Kf; ++q) {
    const auto &f = h.fexp[q];
    bool in_lead = false;
    for (int r = 0; r < n_rec; ++r) in_lead = in_lead || f.bath == records[r];
    if (!in_lead) continue;
    const int64_t a = lookup_ado(h, 1ull << q, 0);
    if (a < 0) continue;  // n_max = 0: no first-level ADOs
    // d^{nu-bar}: d for nu = +1, d^dagger for nu = -1; coefficient i (-1)^{delta_{nu,-}}
    const std::vector<cd> &O = h.ops[f.nu == +1 ? f.op_ann : f.op_ann + 1];
    const cd coef = f.nu == +1 ? cd(0, 1) : cd(0, -1);
    ado.push_back(a);
    for (int e = 0; e < dd; ++e) {
      const cd v = coef * O[e];
      ops.push_back(make_double2(v.real(), v.imag()));
    }
  }
  if (ado.empty()) return HEOM_OK;
  HEOM_TRY(ensure_device(h));
  hipStream_t s = (hipStream_t)stream;
  int64_t *d_ado = nullptr;
  double2 *d_ops = nullptr, *d_out = nullptr;
  heom_status st = HEOM_OK;
  if (hipMalloc(&d_ado, sizeof(int64_t) * ado.size()) != hipSuccess ||
      hipMalloc(&d_ops, sizeof(double2) * ops.size()) != hipSuccess || hipMalloc(&d_out, sizeof(double2)) != hipSuccess) {
    st = fail(HEOM_ERR_ALLOC, "current: device allocation failed");
  } else {
    double2 res = make_double2(0.0, 0.0);
    if (hipMemcpyAsync(d_ado, ado.data(), sizeof(int64_t) * ado.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(d_ops, ops.data(), sizeof(double2) * ops.size(), hipMemcpyHostToDevice, s) != hipSuccess) {
      st = fail(HEOM_ERR_HIP, "current: copy to the device failed");
    } else {
      hipLaunchKernelGGL(current_kernel, dim3(1), dim3(256), 0, s, (const double2 *)x_dev, d, (int)ado.size(), d_ado,
                         d_ops, (const int32_t *)nullptr, d_out);
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(&res, d_out, sizeof(double2), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        st = fail(HEOM_ERR_HIP, "current: kernel or copy failed");
    }
    out[0] = res.x;
    out[1] = res.y;
  }
  if (d_ado) (void)hipFree(d_ado);
  if (d_ops) (void)hipFree(d_ops);
  if (d_out) (void)hipFree(d_out);
  return st;
}

extern "C" heom_status heom_current(heom_hier *hw, const void *x_dev, int32_t n_rec, const int32_t *records,
                                    double *out, void *stream) {
  return guarded([&] { return heom_current_body(hw, x_dev, n_rec, records, out, stream); });
}

// ------------------------------------------------------------------ no-allocation variant
// heom_current_noalloc keeps the term list and the terms' operators in a
// file-scope device array instead of per-call allocations: at most
// kCurTerms terms (every fermionic exponent is at most one term, and there
// are at most 64) of d <= kCurMaxD.  Layout: ado[kCurTerms] (int64),
// neg[kCurTerms] (int32), the result (double2), then the operators,
// kCurTerms x d^2 double2 (row-major, term-major).
namespace heom {
constexpr int kCurTerms = 64, kCurMaxD = 32;
constexpr size_t kCurOpsOff = 1024;  // past ado (512 B), neg (256 B) and the result, 256-byte aligned
constexpr size_t kCurScratchBytes = kCurOpsOff + (size_t)kCurTerms * kCurMaxD * kCurMaxD * sizeof(double2);
}  // namespace heom

static __device__ __align__(256) unsigned char scratch[heom::kCurScratchBytes];

namespace heom {
// device address of `scratch` on each device, taken once per device with
// that device current (each device holds its own copy of the array)
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64] = {};

static heom_status scratch_on_current_device(unsigned char **ptr) {
  int dev = 0;
  HEOM_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(HEOM_ERR_UNSUPPORTED, "current_noalloc: device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HEOM_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(HEOM_ERR_HIP, "current_noalloc: no device address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *ptr = (unsigned char *)g_scratch_ptr[dev];
  return HEOM_OK;
}
}  // namespace heom

static heom_status heom_current_noalloc_body(heom_hier *hw, const void *x_dev, int32_t n_rec, const int32_t *records,
                                            double *out, void *stream) {
  HEOM_TRY(check_current_args(hw, x_dev, n_rec, records, out));
  Hier &h = *hw->impl;
  out[0] = out[1] = 0.0;
  const int d = h.d, dd = d * d;
  if (d > kCurMaxD) return fail(HEOM_ERR_UNSUPPORTED, "current_noalloc: d above 32 exceeds the scratch array");
  // the terms, staged on the stack: ADO, sign of the coefficient, operator
  int64_t ado[kCurTerms];
  int32_t neg[kCurTerms];
  const std::vector<cd> *opm[kCurTerms];
  int n_terms = 0;
  for (int q = 0; q < h.Kf; ++q) {
    const auto &f = h.fexp[q];
    bool in_lead = false;
    for (int r = 0; r < n_rec; ++r) in_lead = in_lead || f.bath == records[r];
    if (!in_lead) continue;
    const int64_t a = lookup_ado(h, 1ull << q, 0);
    if (a < 0) continue;
    if (n_terms >= kCurTerms) return fail(HEOM_ERR_UNSUPPORTED, "current_noalloc: more than 64 terms");
    ado[n_terms] = a;
    neg[n_terms] = f.nu == +1 ? 0 : 1;  // coefficient i for nu = +1, -i for nu = -1
    opm[n_terms] = &h.ops[f.nu == +1 ? f.op_ann : f.op_ann + 1];
    ++n_terms;
  }
  if (n_terms == 0) return HEOM_OK;
  unsigned char *base = nullptr;
  HEOM_TRY(scratch_on_current_device(&base));
  int64_t *d_ado = (int64_t *)base;
  int32_t *d_neg = (int32_t *)(base + kCurTerms * sizeof(int64_t));
  double2 *d_out = (double2 *)(base + kCurTerms * (sizeof(int64_t) + sizeof(int32_t)));
  double2 *d_ops = (double2 *)(base + kCurOpsOff);
  hipStream_t s = (hipStream_t)stream;
  HEOM_HIP_CHECK(hipMemcpyAsync(d_ado, ado, sizeof(int64_t) * n_terms, hipMemcpyHostToDevice, s));
  HEOM_HIP_CHECK(hipMemcpyAsync(d_neg, neg, sizeof(int32_t) * n_terms, hipMemcpyHostToDevice, s));
  for (int t = 0; t < n_terms; ++t)  // std::complex<double> is laid out as (re, im)
    HEOM_HIP_CHECK(hipMemcpyAsync(d_ops + (size_t)t * dd, opm[t]->data(), sizeof(double2) * dd,
                                  hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(current_kernel, dim3(1), dim3(256), 0, s, (const double2 *)x_dev, d, n_terms,
                     (const int64_t *)d_ado, (const double2 *)d_ops, (const int32_t *)d_neg, d_out);
  HEOM_HIP_CHECK(hipGetLastError());
  double2 res = make_double2(0.0, 0.0);
  HEOM_HIP_CHECK(hipMemcpyAsync(&res, d_out, sizeof(double2), hipMemcpyDeviceToHost, s));
  HEOM_HIP_CHECK(hipStreamSynchronize(s));
  out[0] = res.x;
  out[1] = res.y;
  return HEOM_OK;
}

extern "C" heom_status heom_current_noalloc(heom_hier *hw, const void *x_dev, int32_t n_rec, const int32_t *records,
                                            double *out, void *stream) {
  return guarded([&] { return heom_current_noalloc_body(hw, x_dev, n_rec, records, out, stream); });
}
