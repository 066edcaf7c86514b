// Time-dependent system Hamiltonian in RK4: H_s(t) = H + sum_k f_k(t) V_k
// (the paper allows H_s(t) in the dynamics, "Package architecture").  Each
// RK4 stage applies M (with H) and then adds, on every ADO X of the stage
// input, -i sum_k f_k(t_stage) [V_k, X]; the coefficients come from a host
// callback at the stage times t, t + dt/2, t + dt/2, t + dt and travel to
// the kernel as launch arguments, so every stage keeps its own values.
#include <vector>

#include "blas.h"
#include "device_common.h"
#include "internal.h"
#include "solvers.h"

namespace heom {

constexpr int kMaxDrive = 8;
struct DriveCoef {
  double c[kMaxDrive];
};

// y += -i sum_k c_k [V_k, X], X = x (+ kc k) per ADO; one workgroup per ADO
template <typename T>
__global__ void __launch_bounds__(256) drive_kernel(const typename Cplx<T>::t *__restrict__ x,
                                                    const typename Cplx<T>::t *__restrict__ kv, double kc,
                                                    typename Cplx<T>::t *__restrict__ y, const double2 *__restrict__ V,
                                                    DriveCoef cf, int n_drive, int d, int64_t N) {
  using T2 = typename Cplx<T>::t;
  __shared__ double2 X[kLindbladMaxD * kLindbladMaxD];
  const int dd = d * d;
  for (int64_t a = blockIdx.x; a < N; a += gridDim.x) {
    const int64_t base = a * dd;
    __syncthreads();
    for (int e = threadIdx.x; e < dd; e += blockDim.x) {
      const T2 v = x[base + e];
      double vx = (double)v.x, vy = (double)v.y;
      if (kv) {
        const T2 q = kv[base + e];
        vx += kc * (double)q.x;
        vy += kc * (double)q.y;
      }
      X[e] = make_double2(vx, vy);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < dd; e += blockDim.x) {
      const int i = e / d, j = e % d;
      double sx = 0.0, sy = 0.0;  // sum_k c_k (V_k X - X V_k)[i][j]
      for (int k = 0; k < n_drive; ++k) {
        const double2 *Vk = V + (size_t)k * dd;
        double px = 0.0, py = 0.0;
        for (int l = 0; l < d; ++l) {
          const double2 v1 = Vk[i * d + l], x1 = X[l * d + j];
          const double2 x2 = X[i * d + l], v2 = Vk[l * d + j];
          px += v1.x * x1.x - v1.y * x1.y - (x2.x * v2.x - x2.y * v2.y);
          py += v1.x * x1.y + v1.y * x1.x - (x2.x * v2.y + x2.y * v2.x);
        }
        sx += cf.c[k] * px;
        sy += cf.c[k] * py;
      }
      T2 o = y[base + e];  // -i (sx + i sy) = sy - i sx
      o.x = (T)((double)o.x + sy);
      o.y = (T)((double)o.y - sx);
      y[base + e] = o;
    }
  }
}

static heom_status launch_drive(const Hier &h, int precision, const ApplyArgs &a, const double2 *V, int n_drive,
                                const DriveCoef &cf, hipStream_t s) {
  const unsigned grid = (unsigned)std::min<int64_t>(std::max<int64_t>(h.N, 1), 16384);
  if (precision == HEOM_FP64)
    hipLaunchKernelGGL(drive_kernel<double>, dim3(grid), dim3(256), 0, s, (const double2 *)a.x, (const double2 *)a.k,
                       a.kc, (double2 *)a.y, V, cf, n_drive, h.d, h.N);
  else
    hipLaunchKernelGGL(drive_kernel<float>, dim3(grid), dim3(256), 0, s, (const float2 *)a.x, (const float2 *)a.k,
                       a.kc, (float2 *)a.y, V, cf, n_drive, h.d, h.N);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

}  // namespace heom

using namespace heom;

static heom_status heom_propagate_driven_body(heom_hier *hw, int32_t precision, void *x_dev, double t0, double dt,
                                             int64_t n_steps, int64_t save_every, void *traj_dev, int32_t n_drive,
                                             const double *V_host, heom_drive_fn f, void *ctx, void *ws,
                                             size_t ws_bytes, void *stream) {
  if (!hw || !x_dev || n_steps < 0 || !std::isfinite(dt) || !std::isfinite(t0))
    return fail(HEOM_ERR_ARG, "propagate_driven: bad arguments");
  if (precision != HEOM_FP64 && precision != HEOM_FP32) return fail(HEOM_ERR_ARG, "bad precision");
  if (save_every < 0 || (save_every > 0 && !traj_dev)) return fail(HEOM_ERR_ARG, "propagate_driven: bad trajectory args");
  if (n_drive < 1 || n_drive > kMaxDrive || !V_host || !f)
    return fail(HEOM_ERR_ARG, "propagate_driven: 1 to 8 drive operators and a coefficient callback");
  Hier &h = *hw->impl;
  const int d = h.d, dd = d * d;
  if (d > kLindbladMaxD) return fail(HEOM_ERR_UNSUPPORTED, "propagate_driven: d must be at most 32");
  std::vector<double2> Vd((size_t)n_drive * dd);
  for (int k = 0; k < n_drive; ++k) {
    const double *Vk = V_host + 2 * (size_t)k * dd;
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        const cd vij(Vk[2 * (i * d + j)], Vk[2 * (i * d + j) + 1]), vji(Vk[2 * (j * d + i)], Vk[2 * (j * d + i) + 1]);
        if (!std::isfinite(vij.real()) || !std::isfinite(vij.imag()) || std::abs(vij - std::conj(vji)) > 1e-12 * (1.0 + std::abs(vij)))
          return fail(HEOM_ERR_ARG, "propagate_driven: drive operators must be Hermitian");
        Vd[(size_t)k * dd + i * d + j] = make_double2(vij.real(), vij.imag());
      }
    if (!h.parity_op.empty()) {
      const std::vector<cd> &P = h.parity_op;
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
          cd pm(0), mp(0);
          for (int l = 0; l < d; ++l) {
            const double2 a1 = Vd[(size_t)k * dd + l * d + j], a2 = Vd[(size_t)k * dd + i * d + l];
            pm += P[(size_t)i * d + l] * cd(a1.x, a1.y);
            mp += cd(a2.x, a2.y) * P[(size_t)l * d + j];
          }
          if (std::abs(pm - mp) > 1e-12) return fail(HEOM_ERR_ARG, "propagate_driven: drive operator is not parity-even");
        }
    }
  }
  HEOM_TRY(ensure_device(h));
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = h.N * (int64_t)dd;
  const size_t w = precision == HEOM_FP64 ? 16 : 8;
  WsArena arena(ws, ws_bytes);
  void *k[4];
  for (int i = 0; i < 4; ++i) k[i] = arena.take((size_t)n * w);
  void *u = arena.take((size_t)n * w);  // stage input x + c k, formed once per stage
  int *counter = (int *)arena.take(256);
  if (!k[0] || !k[1] || !k[2] || !k[3] || !u || !counter)
    return fail(HEOM_ERR_ARG, "propagate_driven: workspace too small");
  double2 *Vdev = nullptr;
  if (hipMalloc(&Vdev, sizeof(double2) * Vd.size()) != hipSuccess) return fail(HEOM_ERR_ALLOC, "propagate_driven: allocation");
  struct Free {
    double2 *p;
    ~Free() { (void)hipFree(p); }
  } guard{Vdev};
  HEOM_HIP_CHECK(hipMemcpyAsync(Vdev, Vd.data(), sizeof(double2) * Vd.size(), hipMemcpyHostToDevice, s));
  HEOM_TRY(fill_int(counter, 0, 1, s));
  const int64_t n_saves = save_every > 0 ? n_steps / save_every : 0;
  auto coef = [&](double t, DriveCoef &cf) -> heom_status {
    for (int q = 0; q < kMaxDrive; ++q) cf.c[q] = 0.0;
    f(t, cf.c, ctx);
    for (int q = 0; q < n_drive; ++q)
      if (!std::isfinite(cf.c[q])) return fail(HEOM_ERR_NAN, "propagate_driven: non-finite drive coefficient");
    return HEOM_OK;
  };
  double t = t0;
  for (int64_t step = 0; step < n_steps; ++step) {
    const double ts[4] = {t, t + 0.5 * dt, t + 0.5 * dt, t + dt};
    const double cs[3] = {0.5 * dt, 0.5 * dt, dt};
    for (int st = 0; st < 4; ++st) {
      ApplyArgs a;
      a.n_rhs = 1;
      a.x = x_dev;
      a.y = k[st];
      if (st > 0) {  // one pass forms x + c k for both the apply and the drive term
        if (precision == HEOM_FP64) HEOM_TRY(stage_input<double>(x_dev, k[st - 1], cs[st - 1], u, n, s));
        else HEOM_TRY(stage_input<float>(x_dev, k[st - 1], cs[st - 1], u, n, s));
        a.x = u;
      }
      DriveCoef cf;
      HEOM_TRY(coef(ts[st], cf));
      HEOM_TRY(launch_apply(h, precision, a, s));
      HEOM_TRY(launch_drive(h, precision, a, Vdev, n_drive, cf, s));
    }
    if (precision == HEOM_FP64) HEOM_TRY(rk4_combine<double>(x_dev, k[0], k[1], k[2], k[3], dt, n, s));
    else HEOM_TRY(rk4_combine<float>(x_dev, k[0], k[1], k[2], k[3], dt, n, s));
    if (save_every > 0 && (step + 1) % save_every == 0) {
      if (precision == HEOM_FP64) HEOM_TRY(save_rho0<double>(x_dev, traj_dev, dd, counter, n_saves, s));
      else HEOM_TRY(save_rho0<float>(x_dev, traj_dev, dd, counter, n_saves, s));
    }
    t = t0 + (double)(step + 1) * dt;
  }
  HEOM_HIP_CHECK(hipStreamSynchronize(s));  // the drive operators are freed on return
  return HEOM_OK;
}

extern "C" heom_status heom_propagate_driven(heom_hier *hw, int32_t precision, void *x_dev, double t0, double dt,
                                             int64_t n_steps, int64_t save_every, void *traj_dev, int32_t n_drive,
                                             const double *V_host, heom_drive_fn f, void *ctx, void *ws,
                                             size_t ws_bytes, void *stream) {
  return guarded([&] { return heom_propagate_driven_body(hw, precision, x_dev, t0, dt, n_steps, save_every, traj_dev, n_drive, V_host, f, ctx, ws, ws_bytes, stream); });
}
