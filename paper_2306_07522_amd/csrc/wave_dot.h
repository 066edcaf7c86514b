// One-read two-vector multi-dot over one chunk of elements, shared by the
// single-hierarchy solver (blas.hip) and the batched one (batch.hip).
//
// For k <= kWaveDotMaxK basis vectors V_i it forms, over elements
// [e0, e1): conj(V_i) . w, conj(V_i) . u and w . w, reading w and u once
// whatever k is.  The four waves of the workgroup walk sub-blocks of 64 * P
// elements, holding w and u there in registers, and take the basis vectors
// four at a time.  The 16 per-lane values of four vectors (Re and Im of
// conj(V_q).w and conj(V_q).u) are summed over the wave by recursive
// halving: after exchanges at lane distances 32, 16, 8, 4 each lane holds
// one of the 16 values summed over half, a quarter, ... of the wave, and two
// more exchanges (2, 1) finish the sum, so lane l ends with value
// 8 b5 + 4 b4 + 2 b3 + b2 of the bits of l.  Each lane accumulates its
// value of group g in acc[g] over the sub-blocks; |w|^2 stays lane-local
// until the end.  The four waves then combine through LDS in a fixed order
// (deterministic).  Output layout [slot][chunk]: slots i < k (w), k + i (u),
// 2k (w . w).
#pragma once

#include "device_common.h"

namespace heom {

constexpr int kWaveDotMaxK = 64;

struct WaveDotShared {
  double red[4][kWaveDotMaxK / 4][16];
  double redw[4][64];
};

// Called by all 256 threads of the workgroup; on = false writes zeros.
template <typename T, int P>
__device__ __forceinline__ void wave_mdot2_chunk(WaveDotShared &sh, const typename Cplx<T>::t *__restrict__ V,
                                                 int64_t ldv, int k, const typename Cplx<T>::t *__restrict__ w,
                                                 const typename Cplx<T>::t *__restrict__ u, int64_t e0, int64_t e1,
                                                 bool on, double2 *__restrict__ partial, int nchunk, int chunk) {
  using T2 = typename Cplx<T>::t;
  constexpr int G = kWaveDotMaxK / 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ng = (k + 3) / 4;
  double acc[G];
#pragma unroll
  for (int g = 0; g < G; ++g) acc[g] = 0.0;
  double ww = 0.0;
  if (!on) e1 = e0;  // no sub-blocks: zeros
  for (int64_t base = e0 + (int64_t)wave * 64 * P; base < e1; base += (int64_t)4 * 64 * P) {
    // a whole sub-block (every sub-block but the ragged last) loads without
    // per-element guards, so its P loads per vector are in flight together
    // instead of one guarded load at a time
    const bool full = base + 64 * P <= e1;
    double wx[P], wy[P], ux[P], uy[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int64_t e = base + lane + 64 * p;
      wx[p] = wy[p] = ux[p] = uy[p] = 0.0;
      if (full || e < e1) {
        const T2 bw = w[e], bu = u[e];
        wx[p] = bw.x; wy[p] = bw.y; ux[p] = bu.x; uy[p] = bu.y;
        ww += wx[p] * wx[p] + wy[p] * wy[p];
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (g >= ng) break;
      double v[16];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int q = 4 * g + c;
        double dx = 0.0, dy = 0.0, fx = 0.0, fy = 0.0;
        if (q < k) {
          T2 a[P];
          if (full) {
#pragma unroll
            for (int p = 0; p < P; ++p) a[p] = load_stream<T>(&V[(int64_t)q * ldv + base + lane + 64 * p]);
          } else {
#pragma unroll
            for (int p = 0; p < P; ++p) {
              const int64_t e = base + lane + 64 * p;
              a[p] = e < e1 ? V[(int64_t)q * ldv + e] : T2{0, 0};
            }
          }
#pragma unroll
          for (int p = 0; p < P; ++p) {
            const double ax = a[p].x, ay = a[p].y;
            dx += ax * wx[p] + ay * wy[p];
            dy += ax * wy[p] - ay * wx[p];
            fx += ax * ux[p] + ay * uy[p];
            fy += ax * uy[p] - ay * ux[p];
          }
        }
        v[4 * c] = dx; v[4 * c + 1] = dy; v[4 * c + 2] = fx; v[4 * c + 3] = fy;
      }
      // recursive halving: at distance 32 the lanes with bit 5 set keep
      // values 8..15, the others 0..7, and each adds its partner's copy
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const bool hi = lane & 32;
        const double send = hi ? v[r] : v[8 + r];
        const double keep = hi ? v[8 + r] : v[r];
        v[r] = keep + __shfl_xor(send, 32);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool hi = lane & 16;
        const double send = hi ? v[r] : v[4 + r];
        const double keep = hi ? v[4 + r] : v[r];
        v[r] = keep + __shfl_xor(send, 16);
      }
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const bool hi = lane & 8;
        const double send = hi ? v[r] : v[2 + r];
        const double keep = hi ? v[2 + r] : v[r];
        v[r] = keep + __shfl_xor(send, 8);
      }
      {
        const bool hi = lane & 4;
        const double send = hi ? v[0] : v[1];
        const double keep = hi ? v[1] : v[0];
        v[0] = keep + __shfl_xor(send, 4);
      }
      v[0] += __shfl_xor(v[0], 2);
      v[0] += __shfl_xor(v[0], 1);
      acc[g] += v[0];
    }
  }
  // lane l holds value j = 8 b5 + 4 b4 + 2 b3 + b2 of every group (bits of l)
  const int j = ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1);
  if ((lane & 3) == 0) {
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (g < ng) sh.red[wave][g][j] = acc[g];
  }
  sh.redw[wave][lane] = ww;
  __syncthreads();
  // value j of group g: vector q = 4g + j / 4, component j % 4 (Re, Im of
  // the w product, then of the u product)
  for (int q = threadIdx.x; q < k; q += 256) {
    const int g = q >> 2, c = q & 3;
    double t[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      t[i] = ((sh.red[0][g][4 * c + i] + sh.red[1][g][4 * c + i]) + sh.red[2][g][4 * c + i]) + sh.red[3][g][4 * c + i];
    partial[(int64_t)q * nchunk + chunk] = make_double2(t[0], t[1]);
    partial[(int64_t)(k + q) * nchunk + chunk] = make_double2(t[2], t[3]);
  }
  if (wave == 0) {
    double sw = ((sh.redw[0][lane] + sh.redw[1][lane]) + sh.redw[2][lane]) + sh.redw[3][lane];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sw += __shfl_xor(sw, off);
    if (lane == 0) partial[(int64_t)(2 * k) * nchunk + chunk] = make_double2(sw, 0.0);
  }
}

}  // namespace heom
