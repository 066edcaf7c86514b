// Device-side helpers shared by the HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

namespace heom {

template <typename T> struct Cplx;
template <> struct Cplx<double> { using t = double2; };
template <> struct Cplx<float> { using t = float2; };

// A streaming read of one complex element: marked non-temporal, so that a
// pass over a Krylov basis (read once per Arnoldi step, gigabytes apart)
// does not push reusable lines out of the caches.
template <typename T>
__device__ __forceinline__ typename Cplx<T>::t load_stream(const typename Cplx<T>::t *p) {
  const T *q = reinterpret_cast<const T *>(p);
  return typename Cplx<T>::t{__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1)};
}

template <typename T2> __device__ __forceinline__ T2 cadd(T2 a, T2 b) { return T2{a.x + b.x, a.y + b.y}; }
template <typename T2> __device__ __forceinline__ T2 csub(T2 a, T2 b) { return T2{a.x - b.x, a.y - b.y}; }
template <typename T2> __device__ __forceinline__ T2 cmul(T2 a, T2 b) {
  return T2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * b + c
template <typename T2> __device__ __forceinline__ T2 cfma(T2 a, T2 b, T2 c) {
  return T2{fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y))};
}
template <typename T2, typename T> __device__ __forceinline__ T2 cscale(T2 a, T s) { return T2{a.x * s, a.y * s}; }

// task flags
enum : int { TASK_DIAG = 1, TASK_ACC = 2 };

}  // namespace heom
