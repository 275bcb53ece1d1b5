// Host-side declarations shared by the kernel translation units and the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/ttt.h"
#include "ttt_amu.h"
#include "ttt_common.h"

namespace ttt {
// Chunk step at large state sizes (d >= 256): the chunk's rows are read from
// the token tensors (head offset applied), every product is a GEMM over
// operands streamed from HBM.
struct LargeNormArgs {
  const void* K;
  const void* V;
  const void* Q;
  int64_t stride_tok;
  uint32_t flags;
  int32_t rows, d;
  void* Kn;
  float* Vn;
  void* Qn;
};
// Row normalisation of a large-state chunk (K, V, Q; the flags select which).
hipError_t launch_large_norm(const LargeNormArgs& a, bool io_bf16, bool mma_bf16, hipStream_t st);
struct LargeStepArgs {
  const void* K;  // first token of the chunk, head offset applied
  const void* V;
  const void* Q;
  void* O;        // nullable: no apply
  int64_t stride_tok;
  uint32_t flags;
  int32_t rows, d, h;
  int32_t grad;   // 1: gradient of the chunk and the update
  int32_t masters_only;  // 1: the update leaves the operand copies (a sum of gradients at W0)
  float eta;
  void* Kn;       // [rows][d] operand type
  void* Qn;
  void* E;
  void* A;        // [rows][h] operand type
  void* D;
  void* Aq;
  float* Vn;      // [rows][d] FP32
  void* S1;       // operand type: SiLU'(Z), tile-native (whole 128-row tiles) in the forward step
  float* W1;      // FP32 masters [d][h], [h][d], updated in place
  float* W2;
  void* W1op;     // operand copies of the masters
  void* W2op;
  float* loss_part;  // [d/128 * ceil(rows/128)]
  float* loss;       // nullable: the chunk's loss
};
hipError_t launch_large_step(const LargeStepArgs& a, bool io_bf16, bool mma_bf16, hipStream_t st);
// Reverse step of one chunk of the MSE unit at large state sizes (the apply
// adjoint at W_{c+1}, then the update adjoint at W_c along the carried
// adjoint Wh, which it replaces by the adjoint of W_c).
struct LargeBwdArgs {
  const void* K;  // first token of the chunk, head offset applied (io type)
  const void* V;
  const void* Q;
  const void* dO;
  void* dQ;       // written: gradients w.r.t. the raw rows (io type)
  void* dK;
  void* dV;
  int64_t stride_tok;
  uint32_t flags;
  int32_t rows, d, h;
  float eta;
  void* Kn;       // [rows][d] operand type
  void* Qn;
  void* E;
  void* dOn;
  void* dY;
  float* Vn;      // [rows][d] FP32
  float* dq;
  float* dk;
  float* dv;
  float* dE;
  void* A;        // [rows][h] operand type
  void* S1;
  void* S2;
  void* P;
  void* D;
  void* Aq;
  void* Sq1;
  void* dZq;
  void* dP;
  void* dZa;
  void* EWh;
  void* dZ;
  const void* W1op;   // W_c
  const void* W2op;
  const void* W1nop;  // W_{c+1}
  const void* W2nop;
  float* Wh1;         // carried adjoint: FP32 masters and operand copies
  float* Wh2;
  void* Wh1op;
  void* Wh2op;
  float* Acc1;        // where the update adjoint's weight terms are added (the
  float* Acc2;        // carried adjoint itself for the chain) and their
  void* Acc1op;       // operand copies (nullable)
  void* Acc2op;
  int32_t apply;      // 1: the apply adjoint of the chunk (dQ written)
  int32_t update;     // 1: the update adjoint of the chunk (dK, dV written)
  float* deta_part;   // per-tile partials of the step-size derivative
  float* deta;        // this head's running d/d eta (one float)
};
hipError_t launch_large_bwd_step(const LargeBwdArgs& a, bool io_bf16, bool mma_bf16, hipStream_t st);
// Reverse step of one chunk of the paper's memory unit at large state sizes
// (apply adjoint at W' = W_{c+1} and/or update adjoint at W = W_c along the
// adjoint Wh of W'; weight terms of the update adjoint added to Acc).
struct LargeAmuBwdArgs {
  const void* K;  // first token of the chunk, head offset applied (io type)
  const void* V;
  const void* Q;
  const void* dO;
  void* dQ;
  void* dK;
  void* dV;
  int64_t stride_tok;
  const float* eta;    // step size of the chunk's first token for this head
  float* deta;         // its derivative (same layout)
  int64_t eta_stride;  // between consecutive tokens (the head count)
  uint32_t flags;
  int32_t rows, d, h;
  int32_t apply, update;
  void* Kn;      // [rows][d] operand type
  void* Qn;
  void* E;
  void* dOn;
  float* Vn;     // [rows][d] FP32
  float* Ydot;
  float* dq;
  float* dk;
  float* dv;
  void* Z3;      // [rows][h] operand type
  void* S;
  void* S1;
  void* S2;
  void* Hd;
  void* Zd3;
  void* Sd;
  void* Hdot;
  void* T2;
  void* dHh;
  void* aZ1;
  void* aZ3;
  void* aZd1;
  void* aZd3;
  const void* Wop[3];   // W (W1, W2, W3 operand copies)
  const void* Wnop[3];  // W'
  float* Wh[3];         // adjoint of W': FP32 masters and operand copies
  void* Whop[3];
  float* Acc[3];        // where the update adjoint's weight terms go, and
  void* Accop[3];       // their operand copies (nullable)
};
hipError_t launch_large_amu_bwd_step(const LargeAmuBwdArgs& a, bool io_bf16, bool mma_bf16, hipStream_t st);
// Fill n floats with zero.
hipError_t launch_large_zero(float* p, int64_t n, hipStream_t st);
// dst[i] += src[i] for n floats.
hipError_t launch_large_add(const float* src, float* dst, int64_t n, hipStream_t st);
// Chunk step of the paper's memory unit (SwiGLU network, dot-product loss
// with token-wise step sizes) at large state sizes.
struct LargeAmuArgs {
  const void* K;  // first token of the chunk, head offset applied
  const void* V;
  const void* Q;
  void* O;        // nullable: no apply
  int64_t stride_tok;
  const float* eta;    // step size of the chunk's first token for this head
  int64_t eta_stride;  // between consecutive tokens (the head count)
  uint32_t flags;
  int32_t rows, d, h;
  int32_t grad;      // 1: gradient of the chunk and the update of the masters
  int32_t write_op;  // 1: the update also rewrites the operand copies
  void* Kn;          // [rows][d] operand type
  void* Qn;
  void* E;
  float* Vn;         // [rows][d] FP32
  void* Z3;          // [rows][h] operand type: x W3
  void* Hd;          // SiLU(x W1) * (x W3)
  void* G1;          // Z3 * SiLU'(Z1)
  void* G3;          // SiLU(Z1)
  void* D1;          // hidden adjoint times G1
  void* D3;          // hidden adjoint times G3
  float* W1;         // FP32 masters [d][h], [h][d], [d][h], updated in place
  float* W2;
  float* W3;
  void* W1op;        // operand copies of the masters
  void* W2op;
  void* W3op;
};
hipError_t launch_large_amu_step(const LargeAmuArgs& a, bool io_bf16, bool mma_bf16, hipStream_t st);
// Operand copy (BF16 or FP32) of n FP32 values.
hipError_t launch_large_cast(const float* src, void* dst, int64_t n, bool mma_bf16, hipStream_t st);
// One projection of the layer around the memory unit (token rows in the io
// type, D = H * d features): kind 0, [Q | K | V] = X W (+ bias) with W
// [D][3D]; kind 1, Y = alpha * (O W (+ bias)) + X with W [D][D].
struct GcmGemmArgs {
  int32_t kind;
  int32_t D;
  int64_t rows;
  const void* x;   // [rows][D]
  const void* w;   // kind 0: [D][3D]; kind 1: [D][D] (io type)
  const float* bias;   // nullable: [3D] or [D]
  const float* alpha;  // kind 1: [D]
  void* q;         // kind 0 outputs, [rows][D] each
  void* k;
  void* v;
  const void* o;   // kind 1: the memory unit's output [rows][D]
  void* y;         // kind 1 output [rows][D]
};
hipError_t launch_gcm_gemm(const GcmGemmArgs& a, bool io_bf16, hipStream_t st);
// Reverse mode of the layer around the unit, in three phases around the
// unit's own forward and reverse calls (N = rows, D features, token tensors
// in the io type):
//   phase 0  P = X Wqkv (+ bqkv)                      [N][3D], pitch 3D
//   phase 1  G = O Wo (+ bo) (FP32), dG = alpha dY, dalpha = sum G dY,
//            dbo = sum dG, dWo = O^T dG, dO = dG Wo^T  (O, dO pitch 3D)
//   phase 2  dWqkv = X^T dP, dbqkv = sum dP, dX = dY + dP Wqkv^T   (dP pitch 3D)
struct GcmBwdArgs {
  int32_t phase;
  int32_t D;
  int64_t rows;
  const void* X;
  const void* Wqkv;
  const float* bqkv;   // nullable
  const void* Wo;
  const float* bo;     // nullable
  const float* alpha;
  const void* dY;
  void* P;             // [N][3D]
  void* O;             // [N][3D], the first D columns used
  float* G;            // [N][D]
  void* dG;            // [N][D]
  void* dO;            // [N][3D], the first D columns used
  const void* dP;      // [N][3D]
  float* part;         // column partial sums [ceil(N / 256)][3D]
  void* dX;
  float* dWqkv;        // [D][3D]
  float* dbqkv;        // [3D], nullable
  float* dWo;          // [D][D]
  float* dbo;          // [D], nullable
  float* dalpha;       // [D]
};
hipError_t launch_gcm_bwd(const GcmBwdArgs& a, bool io_bf16, hipStream_t st);
hipError_t launch_large_init(const float* w1, const float* w2, float* m1, float* m2, void* o1, void* o2, int64_t n,
                             bool mma_bf16, hipStream_t st);
hipError_t launch_fwd_step(const FwdStepArgs& a, int n_blocks, int h, bool io_bf16, bool mma_bf16, hipStream_t st);
hipError_t launch_update(const UpdStepArgs& a, int n_blocks, hipStream_t st);
hipError_t persist_occupancy(int h, bool io_bf16, bool mma_bf16, int* blocks_per_cu, int* threads);
hipError_t launch_fwd_persist(const PersistArgs& a, int n_blocks, int h, bool io_bf16, bool mma_bf16,
                              hipStream_t st);
hipError_t launch_zero_words(uint32_t* p, int n, hipStream_t st);
hipError_t launch_bwd_step(const BwdStepArgs& a, int n_blocks, int h, bool io_bf16, bool mma_bf16, hipStream_t st);
hipError_t launch_bwd_step_bf(const BwdStepArgs& a, int n_blocks, int h, bool io_bf16, hipStream_t st);
hipError_t launch_bwd_reduce(const BwdReduceArgs& a, int n_blocks, hipStream_t st);
hipError_t launch_bwd_prep(const BwdPrepArgs& a, int n_active, bool mma_bf16, hipStream_t st);
hipError_t launch_bwd_sum(const BwdSumArgs& a, hipStream_t st);
hipError_t launch_amu_step(const AmuStepArgs& a, int n_blocks, int h, bool io_bf16, bool mma_bf16, hipStream_t st);
hipError_t launch_amu_update(const AmuUpdArgs& a, hipStream_t st);
hipError_t launch_amu_prep(const AmuPrepArgs& a, bool mma_bf16, hipStream_t st);
hipError_t launch_amu_bwd_apply(const AmuBwdArgs& a, int n_blocks, int h, bool io_bf16, bool mma_bf16, hipStream_t st);
hipError_t launch_amu_bwd_update(const AmuBwdArgs& a, int n_blocks, int h, bool io_bf16, bool mma_bf16,
                                 hipStream_t st);
hipError_t launch_amu_psum(const AmuPsumArgs& a, hipStream_t st);
// ttt_chunk_fwd on a caller workspace (fixed_scratch null), or on a fixed
// scratch buffer of ws_bytes with a forward-only layout whose device address
// fixed_scratch() returns (called after validation; null on failure).
ttt_status_t chunk_fwd_impl(const ttt_problem_t* p, const void* Q, const void* K, const void* V, const float* W1_0,
                            const float* W2_0, void* O, float* W1_T, float* W2_T, float* ckpt, float* loss, void* ws,
                            size_t ws_bytes, void* (*fixed_scratch)(), hipStream_t st);
}  // namespace ttt
