// Lindbladian add-on (eq:Lindbladian): every ADO X gets
//
//   sum_k J(F_k)[X] = sum_k F_k X F_k^dagger - 1/2 (G X + X G),  G = sum_k F_k^dagger F_k,
//
// added to y after the apply proper (the ADO space does not grow).  One
// workgroup per (ADO, right-hand side): X staged in LDS (with the fused RK4
// stage input x + kc k), the anticommutator with G, then per jump operator
// W = X F^dagger through a second LDS buffer and F W.  d <= 32.
#include <vector>

#include "device_common.h"
#include "internal.h"

namespace heom {

template <typename T>
__global__ void __launch_bounds__(256) lindblad_kernel(const typename Cplx<T>::t *__restrict__ x,
                                                       const typename Cplx<T>::t *__restrict__ kv, double kc,
                                                       typename Cplx<T>::t *__restrict__ y,
                                                       const double2 *__restrict__ F, const double2 *__restrict__ G,
                                                       int n_ops, int d, int64_t N, int R, int border) {
  using T2 = typename Cplx<T>::t;
  constexpr int kPer = (kLindbladMaxD * kLindbladMaxD + 255) / 256;  // elements per thread
  __shared__ double2 X[kLindbladMaxD * kLindbladMaxD], W[kLindbladMaxD * kLindbladMaxD];
  const int dd = d * d;
  const int64_t tasks = N * R;
  for (int64_t task = blockIdx.x; task < tasks; task += gridDim.x) {
    const int64_t a = task / R;
    const int r = (int)(task % R);
    const int64_t base = a * dd;
    __syncthreads();  // the previous task is done with X and W
    for (int e = threadIdx.x; e < dd; e += blockDim.x) {
      const int64_t idx = (base + e) * R + r;
      const T2 v = x[idx];
      double vx = (double)v.x, vy = (double)v.y;
      if (kv) {
        const T2 q = kv[idx];
        vx += kc * (double)q.x;
        vy += kc * (double)q.y;
      }
      X[e] = make_double2(vx, vy);
    }
    __syncthreads();
    double ax[kPer], ay[kPer];
#pragma unroll
    for (int s = 0; s < kPer; ++s) {
      ax[s] = 0.0;
      ay[s] = 0.0;
      const int e = threadIdx.x + 256 * s;
      if (e >= dd) continue;
      const int i = e / d, j = e % d;
      for (int l = 0; l < d; ++l) {  // -1/2 (G X + X G)
        const double2 g1 = G[i * d + l], x1 = X[l * d + j];
        const double2 x2 = X[i * d + l], g2 = G[l * d + j];
        ax[s] -= 0.5 * (g1.x * x1.x - g1.y * x1.y + x2.x * g2.x - x2.y * g2.y);
        ay[s] -= 0.5 * (g1.x * x1.y + g1.y * x1.x + x2.x * g2.y + x2.y * g2.x);
      }
    }
    for (int k = 0; k < n_ops; ++k) {
      const double2 *Fk = F + (size_t)k * dd;
      for (int e = threadIdx.x; e < dd; e += blockDim.x) {  // W = X F^dagger
        const int i = e / d, j = e % d;
        double sx = 0.0, sy = 0.0;
        for (int l = 0; l < d; ++l) {
          const double2 xv = X[i * d + l], f = Fk[j * d + l];  // X[i][l] conj(F[j][l])
          sx += xv.x * f.x + xv.y * f.y;
          sy += xv.y * f.x - xv.x * f.y;
        }
        W[e] = make_double2(sx, sy);
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < kPer; ++s) {  // += F W
        const int e = threadIdx.x + 256 * s;
        if (e >= dd) continue;
        const int i = e / d, j = e % d;
        for (int l = 0; l < d; ++l) {
          const double2 f = Fk[i * d + l], w = W[l * d + j];
          ax[s] += f.x * w.x - f.y * w.y;
          ay[s] += f.x * w.y + f.y * w.x;
        }
      }
      __syncthreads();  // W is rewritten by the next jump operator
    }
#pragma unroll
    for (int s = 0; s < kPer; ++s) {
      const int e = threadIdx.x + 256 * s;
      if (e >= dd) continue;
      if (border && a == 0 && e == 0) continue;  // the trace row of the stationary-state operator
      const int64_t idx = (base + e) * R + r;
      T2 o = y[idx];
      o.x = (T)((double)o.x + ax[s]);
      o.y = (T)((double)o.y + ay[s]);
      y[idx] = o;
    }
  }
}

heom_status launch_lindblad(Hier &h, int precision, const ApplyArgs &a, hipStream_t s) {
  if (h.lind.empty()) return HEOM_OK;
  if (!h.dev.lind_f || !h.dev.lind_g) return fail(HEOM_ERR_ARG, "Lindbladian: device tables missing");
  const int64_t tasks = h.N * (int64_t)a.n_rhs;
  const unsigned grid = (unsigned)std::min<int64_t>(std::max<int64_t>(tasks, 1), 16384);
  const int n_ops = (int)h.lind.size();
  if (precision == HEOM_FP64)
    hipLaunchKernelGGL(lindblad_kernel<double>, dim3(grid), dim3(256), 0, s, (const double2 *)a.x,
                       (const double2 *)a.k, a.kc, (double2 *)a.y, h.dev.lind_f, h.dev.lind_g, n_ops, h.d, h.N,
                       a.n_rhs, a.border);
  else
    hipLaunchKernelGGL(lindblad_kernel<float>, dim3(grid), dim3(256), 0, s, (const float2 *)a.x, (const float2 *)a.k,
                       a.kc, (float2 *)a.y, h.dev.lind_f, h.dev.lind_g, n_ops, h.d, h.N, a.n_rhs, a.border);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

}  // namespace heom

using namespace heom;

static heom_status heom_hierarchy_set_lindblad_body(heom_hier *hw, int32_t n_ops, const double *F) {
  if (!hw || n_ops < 0 || (n_ops > 0 && !F)) return fail(HEOM_ERR_ARG, "set_lindblad: NULL argument");
  Hier &h = *hw->impl;
  const int d = h.d;
  if (n_ops > 0 && d > kLindbladMaxD) return fail(HEOM_ERR_UNSUPPORTED, "set_lindblad: d must be at most 32");
  std::vector<std::vector<cd>> ops;
  for (int k = 0; k < n_ops; ++k) {
    std::vector<cd> M((size_t)d * d);
    for (int e = 0; e < d * d; ++e) {
      const double re = F[2 * ((size_t)k * d * d + e)], im = F[2 * ((size_t)k * d * d + e) + 1];
      if (!std::isfinite(re) || !std::isfinite(im)) return fail(HEOM_ERR_ARG, "set_lindblad: non-finite entry");
      M[e] = cd(re, im);
    }
    if (!h.parity_op.empty()) {  // the jump operator must keep the parity sectors apart
      const std::vector<cd> &P = h.parity_op;
      double diff = 0.0, scale = 0.0;
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
          cd pm(0), mp(0);
          for (int l = 0; l < d; ++l) {
            pm += P[(size_t)i * d + l] * M[(size_t)l * d + j];
            mp += M[(size_t)i * d + l] * P[(size_t)l * d + j];
          }
          diff = std::max(diff, std::abs(pm - mp));
          scale = std::max(scale, std::abs(M[(size_t)i * d + j]));
        }
      if (diff > 1e-12 * std::max(1.0, scale)) return fail(HEOM_ERR_ARG, "set_lindblad: jump operator is not parity-even");
    }
    ops.push_back(std::move(M));
  }
  free_device(h);  // tables are uploaded again, with the jump operators, on the next use
  h.lind = std::move(ops);
  return HEOM_OK;
}

extern "C" heom_status heom_hierarchy_set_lindblad(heom_hier *hw, int32_t n_ops, const double *F) {
  return guarded([&] { return heom_hierarchy_set_lindblad_body(hw, n_ops, F); });
}
