// Launch-plan structs of the paper's memory unit (SwiGLU fast network,
// dot-product inner loss with token-wise step sizes; Supp. A, Sec. 4.2
// Eq. 8-10): forward step, update, operand preparation, and the reverse mode.
#pragma once
#include <stdint.h>

namespace ttt {

// Weights of the SwiGLU fast network per head: W1 [d][h], W2 [h][d], W3 [d][h]
// at w1/w2/w3 + head * stride.
struct AmuWeights {
  const float* w1;
  const float* w2;
  const float* w3;
  int64_t stride;
};

// Operand copies per head (ttt_amu_prep), n_prep matrices of D*h elements in
// the matrix-core type: 0 W1 as [hid][d], 1 W3 as [hid][d], 2 W2 as [hid][d],
// 3 W2 as [d][hid]; with n_prep = 6 also 4 W1 as [d][hid], 5 W3 as [d][hid].
enum { AMU_W1T = 0, AMU_W3T = 1, AMU_W2N = 2, AMU_W2D = 3, AMU_W1D = 4, AMU_W3D = 5 };

// One chunk step of one sequence, every head: gradient of chunk s over a
// token shard (work-group = head * G + shard) and apply of chunk s-1.
struct AmuStepArgs {
  const void* Q;
  const void* K;
  const void* V;
  void* O;
  const float* eta_tok;  // [N][H] token-wise step sizes
  int64_t stride_tok, stride_head;
  int32_t H;
  uint32_t flags;
  int32_t G;
  const void* prep;      // [H][n_prep][D*h] operand copies (ttt_amu_prep)
  int32_t n_prep;
  float* partial;        // [H*G][3*D*h]: grad W1 | grad W2 | grad W3
  int64_t grad_start;
  int32_t grad_len;
  int64_t app_start;
  int32_t app_len;
};

struct AmuUpdArgs {
  AmuWeights src;
  const float* partial;
  int32_t G, H, h;
  float* w_dst;          // [H][3*D*h] packed W1 | W2 | W3
  float* wT1;            // final split copies, nullable
  float* wT2;
  float* wT3;
};

struct AmuPrepArgs {
  AmuWeights src;
  void* prep;
  int32_t n_mats;        // 4 or 6 (see the operand-copy list above)
  int32_t H, h;
};

// Reverse mode over a token range [start, start+len) of every head, work-group
// = head * G + shard.  Apply adjoint (X = Q, Y = dO): dQ and the adjoint of
// the weights the queries were mapped with.  Update adjoint (X = K, Y = V):
// dK, dV, d eta_i and the second-order contribution -(dG/dW)^T Wh of one
// update W' = W - G(W) given the adjoint Wh of W'.
struct AmuBwdArgs {
  const void* X;
  const void* Y;
  void* dX;
  void* dY;                // update only
  const float* eta_tok;    // update only, [N][H]
  float* deta_tok;         // update only, [N][H]
  int64_t stride_tok, stride_head;
  int32_t H;
  uint32_t flags;
  int32_t G;
  const void* prep_w;      // [H][6][D*h] operand copies of the weights
  const void* prep_a;      // [H][6][D*h] operand copies of Wh (update only)
  float* partial;          // [H*G][3*D*h] contributions to the weights' adjoint
  int64_t start;
  int32_t len;
};

// dst = base + sum over the G shard partials in shard order (base nullable);
// split copies of the result when out1..3 are set.  Packed [H][3*D*h].
struct AmuPsumArgs {
  const float* partial;
  int32_t G, H, h;
  const float* base;
  float* dst;
  float* out1;
  float* out2;
  float* out3;
};

}  // namespace ttt
