// Device-side entry points replaced for the host-only sanitizer build of the
// library's host files (host_hierarchy.cpp, device_tables.cpp, abi.cpp):
// every kernel launch request fails with HEOM_ERR_UNSUPPORTED, as it would
// without a usable GPU, and device memory is host memory (hipMalloc is
// malloc), so the one-time table upload runs under the sanitizers.
#include <atomic>
#include <cstdlib>
#include <cstring>

#include "internal.h"

static std::atomic<long> g_mallocs{0};

extern "C" {
long stub_device_allocations(void) { return g_mallocs.load(); }
hipError_t hipMalloc(void **p, size_t n) {
  *p = std::malloc(n ? n : 1);
  if (!*p) return hipErrorOutOfMemory;
  g_mallocs.fetch_add(1);
  return hipSuccess;
}
hipError_t hipFree(void *p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind) {
  if (n) std::memcpy(dst, src, n);
  return hipSuccess;
}
hipError_t hipGetDevice(int *d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
const char *hipGetErrorString(hipError_t) { return "host-only stub"; }
}

namespace heom {

heom_status launch_apply(Hier &, int, const ApplyArgs &, hipStream_t) {
  return fail(HEOM_ERR_UNSUPPORTED, "host-only build: no device code");
}

heom_status launch_apply_plan(Hier &, int, const ApplyArgs &, int, hipStream_t) {
  return fail(HEOM_ERR_UNSUPPORTED, "host-only build: no device code");
}

heom_status launch_apply_tiled(Hier &, int, const ApplyArgs &, int, hipStream_t) {
  return fail(HEOM_ERR_UNSUPPORTED, "host-only build: no device code");
}

}  // namespace heom
