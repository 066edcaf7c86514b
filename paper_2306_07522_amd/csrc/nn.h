// Learned block preconditioner (interface used by the solvers).
#pragma once

#include "internal.h"
#include "solvers.h"

namespace heom {

size_t nn_workspace_bytes(const Hier &h, int R, size_t elem_bytes);

// One use of a trained network as the variable right preconditioner of
// FGMRES: z = J r + |J r|_a * g(features_a) blockwise, where J is the Jacobi
// preconditioner and g the MLP.
struct NnApply {
  const heom_nn *net = nullptr;
  const Hier *h = nullptr;
  int R = 1;
  const double2 *shifts = nullptr;
  int border = 0;
  bool fell_back = false;
  void *scratch = nullptr;
  heom_status init(const heom_nn *net, const Hier &h, int R, const double2 *shifts, int border, WsArena &ws,
                   size_t elem_bytes);
  template <typename T>
  heom_status apply(const void *in, void *out, hipStream_t s);
};

}  // namespace heom
