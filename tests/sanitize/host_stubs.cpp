// Device-side entry points replaced for the host-only sanitizer build of the
// library's host files (host_hierarchy.cpp, abi.cpp): every device request
// fails with HEOM_ERR_UNSUPPORTED, as it would without a usable GPU.
#include "internal.h"

namespace heom {

void free_device(Hier &) {}

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
