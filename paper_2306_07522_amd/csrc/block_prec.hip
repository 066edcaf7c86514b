// Block (ADO-local) preconditioner: the exact inverse of the part of the
// HEOMLS that acts within one ADO, -(c_a - z) X - i [H, X] (the first line
// of eq:HEOM).  In the eigenbasis of H = U diag(E) U^H it is diagonal:
//
//   X -> U ( (U^H X U) / D_a ) U^H,  D_a[i][j] = -(c_a - z) - i (E_i - E_j),
//
// with |D_a[i][j]| < delta replaced by -delta (tier 0 has c_a = 0, so its
// populations would divide by zero).  Jacobi keeps only the diagonal of H in
// the original basis; this keeps all of the coherent part of the ADO's own
// dynamics, which is what restarted GMRES struggles with when the baths are
// weak: the spectrum then hugs the imaginary axis, out to the width of H's
// spectrum.
//
// One workgroup per (ADO, right-hand side), four d x d complex products
// through LDS, accumulated in double.  Each thread computes a 2 x 2 tile of
// a product, so every operand read from LDS serves two multiply-adds (the
// products are bound by LDS reads, two per multiply-add without tiling).
#include "blas.h"
#include "device_common.h"
#include "tile_product.h"

namespace heom {

constexpr int kBlockPrecMaxD = 32;

template <typename T>
__global__ void __launch_bounds__(256) block_prec_kernel(const typename Cplx<T>::t *__restrict__ r,
                                                         typename Cplx<T>::t *__restrict__ z,
                                                         const double2 *__restrict__ U, const double *__restrict__ E,
                                                         const double2 *__restrict__ decay, int d, int64_t N, int R,
                                                         const double2 *__restrict__ shifts, double delta) {
  using T2 = typename Cplx<T>::t;
  extern __shared__ double2 lds[];
  const int dd = d * d;
  // LDS rows padded to d + 1 entries: with d entries (320 B for d = 20) the
  // rows two apart that a tile's lanes read fall on the same banks
  const int p = d + 1, pd = d * p;
  double2 *Us = lds;           // U, row-major
  double2 *X = lds + pd;       // working block
  double2 *W = lds + 2 * pd;   // second working block
  for (int e = threadIdx.x; e < dd; e += blockDim.x) Us[(e / d) * p + e % d] = U[e];
  const int64_t tasks = N * R;
  for (int64_t task = blockIdx.x; task < tasks; task += gridDim.x) {
    const int64_t a = task / R;
    const int rr = (int)(task % R);
    const int64_t base = a * dd;
    __syncthreads();  // U staged; the previous task is done with X and W
    for (int e = threadIdx.x; e < dd; e += blockDim.x) {
      const T2 v = r[(base + e) * R + rr];
      X[(e / d) * p + e % d] = make_double2((double)v.x, (double)v.y);
    }
    __syncthreads();
    // W = U^H X
    tile_product(
        d, (int)threadIdx.x, [&](int i, int k) { const double2 u = Us[k * p + i]; return make_double2(u.x, -u.y); },
        [&](int k, int j) { return X[k * p + j]; }, [&](int i, int j, double2 v) { W[i * p + j] = v; });
    __syncthreads();
    // X = (W U) / D_a
    const double2 c = decay[a];
    const double2 sh = shifts ? shifts[rr] : make_double2(0.0, 0.0);
    tile_product(
        d, (int)threadIdx.x, [&](int i, int k) { return W[i * p + k]; }, [&](int k, int j) { return Us[k * p + j]; },
        [&](int i, int j, double2 v) {
          double dx = -(c.x - sh.x), dy = -(c.y - sh.y) - (E[i] - E[j]);
          if (dx * dx + dy * dy < delta * delta) {
            dx = -delta;
            dy = 0.0;
          }
          const double inv = 1.0 / (dx * dx + dy * dy);
          X[i * p + j] = make_double2((v.x * dx + v.y * dy) * inv, (v.y * dx - v.x * dy) * inv);
        });
    __syncthreads();
    // W = U X
    tile_product(
        d, (int)threadIdx.x, [&](int i, int k) { return Us[i * p + k]; }, [&](int k, int j) { return X[k * p + j]; },
        [&](int i, int j, double2 v) { W[i * p + j] = v; });
    __syncthreads();
    // z = W U^H
    tile_product(
        d, (int)threadIdx.x, [&](int i, int k) { return W[i * p + k]; },
        [&](int k, int j) { const double2 u = Us[j * p + k]; return make_double2(u.x, -u.y); },
        [&](int i, int j, double2 v) { z[(base + i * d + j) * R + rr] = T2{(T)v.x, (T)v.y}; });
  }
}

template <typename T>
heom_status block_prec(const void *r, void *z, const Hier &h, int R, const double2 *shifts, hipStream_t s) {
  if (h.d > kBlockPrecMaxD) return fail(HEOM_ERR_UNSUPPORTED, "block preconditioner: d must be at most 32");
  if (!h.dev.ueig || !h.dev.eval) return fail(HEOM_ERR_ARG, "block preconditioner: device tables missing");
  const int64_t tasks = h.N * (int64_t)R;
  const unsigned grid = (unsigned)std::min<int64_t>(std::max<int64_t>(tasks, 1), 8192);
  const size_t lds = sizeof(double2) * 3 * h.d * (h.d + 1);
  // one thread per 2 x 2 tile, whole waves: 128 threads for d = 20, 256 for d = 32
  const int tiles = ((h.d + 1) / 2) * ((h.d + 1) / 2);
  const unsigned threads = (unsigned)std::min(256, (tiles + 63) / 64 * 64);
  hipLaunchKernelGGL(block_prec_kernel<T>, dim3(grid), dim3(threads), lds, s, (const typename Cplx<T>::t *)r,
                     (typename Cplx<T>::t *)z, h.dev.ueig, h.dev.eval, h.dev.decay64, h.d, h.N, R, shifts,
                     h.block_delta);
  HEOM_HIP_CHECK(hipGetLastError());
  return HEOM_OK;
}

template heom_status block_prec<double>(const void *, void *, const Hier &, int, const double2 *, hipStream_t);
template heom_status block_prec<float>(const void *, void *, const Hier &, int, const double2 *, hipStream_t);

}  // namespace heom
