// Learned block preconditioner: a small MLP applied to every ADO block of the
// residual, used as the variable right preconditioner of FGMRES.  Weights
// are FP32 masters with BF16 copies; every matrix product runs on BF16 MFMA
// with FP32 accumulation.
#pragma once

#include "internal.h"
#include "solvers.h"

struct heom_nn {
  int d = 0, hidden = 0;
  int f_in = 0, k1 = 0;      // features 2 d^2 + 6, padded to a multiple of 32
  int f_out = 0, o_pad = 0;  // outputs 2 d^2, padded to a multiple of 32
  int device = -1;
  // layer l: W [rows_l x cols_l] row-major, b [rows_l]
  int rows[3] = {0, 0, 0}, cols[3] = {0, 0, 0};
  float *W[3] = {nullptr, nullptr, nullptr}, *b[3] = {nullptr, nullptr, nullptr};
  uint16_t *Wb[3] = {nullptr, nullptr, nullptr};  // BF16 copies of W
  float *mW[3] = {nullptr, nullptr, nullptr}, *vW[3] = {nullptr, nullptr, nullptr};
  float *mb[3] = {nullptr, nullptr, nullptr}, *vb[3] = {nullptr, nullptr, nullptr};
  int64_t adam_step = 0;
};

namespace heom {

size_t nn_workspace_bytes(const Hier &h, int R, size_t elem_bytes);

// One use of a trained network as the variable right preconditioner:
// z = r + |r_a| * g(features_a) blockwise.
struct NnApply {
  const heom_nn *net = nullptr;
  const Hier *h = nullptr;
  int R = 1;
  const double2 *shifts = nullptr;
  int border = 0;
  bool fell_back = false;
  double cscale = 1.0;
  uint16_t *X = nullptr, *H1 = nullptr, *H2 = nullptr;
  float *O = nullptr, *nu = nullptr;
  heom_status init(const heom_nn *net, const Hier &h, int R, const double2 *shifts, int border, WsArena &ws,
                   size_t elem_bytes);
  template <typename T>
  heom_status apply(const void *in, void *out, hipStream_t s);
};

// BF16 GEMM with FP32 accumulation: C = op(A) op(B) (+ epilogue), see nn.hip
enum { EPI_F32 = 0, EPI_BIAS_F32 = 1, EPI_BIAS_RELU_BF16 = 2, EPI_MASK_BF16 = 3 };
heom_status gemm_bf16(bool ta, bool tb, int epi, const uint16_t *A, int lda, const uint16_t *B, int ldb, int M, int N,
                      int K, float *Cf, uint16_t *Cb, int ldc, const float *bias, const float *pre, int ldp,
                      hipStream_t s);

}  // namespace heom
