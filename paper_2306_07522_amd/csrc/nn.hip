// Learned block preconditioner: placeholder until the MLP kernels land.
#include "nn.h"

namespace heom {

size_t nn_workspace_bytes(const Hier &, int, size_t) { return 0; }

heom_status NnApply::init(const heom_nn *, const Hier &, int, const double2 *, int, WsArena &, size_t) {
  return fail(HEOM_ERR_UNSUPPORTED, "learned preconditioner not built");
}

template <typename T>
heom_status NnApply::apply(const void *, void *, hipStream_t) {
  return fail(HEOM_ERR_UNSUPPORTED, "learned preconditioner not built");
}

template heom_status NnApply::apply<double>(const void *, void *, hipStream_t);
template heom_status NnApply::apply<float>(const void *, void *, hipStream_t);

}  // namespace heom
