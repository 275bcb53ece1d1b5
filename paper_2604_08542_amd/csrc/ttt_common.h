// Device-side building blocks shared by the forward and backward kernels:
// vector types, matrix-core wrappers for gfx950, the SiLU family, token-row
// loading with per-token L2 normalisation, and the launch-plan structs.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace ttt {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

constexpr int D = 64;   // head dimension (the only one supported)
constexpr int TT = 32;  // tokens per tile
constexpr int MAXS = 64;  // sequences per launch descriptor
constexpr float NORM_EPS = 1e-12f;

// ----------------------------------------------------------------- matrix cores
// Lane layouts (verified on gfx950):
//  32x32xK: A operand lane l holds A[l%32][kgrp(l/32)], B lane l holds
//           B[kgrp(l/32)][l%32]; result register r of lane l holds
//           C[8*(r/4) + 4*(l/32) + (r%4)][l%32].
//  16x16xK: A lane l holds A[l%16][kgrp(l/16)], B lane l holds
//           B[kgrp(l/16)][l%16]; result register r holds C[4*(l/16)+r][l%16].
//  kgrp(g) is the g-th group of K/2 (32x32) or K/4 (16x16) contraction slots:
//  8 consecutive slots for bf16, 1 slot for f32.
__device__ __forceinline__ f32x16 mma32(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Two floats to a bf16 pair (one v_cvt_pk_bf16_f32, round to nearest even).
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2_t));
}
__device__ __forceinline__ bf16x8 as_bf16x8(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  return __builtin_bit_cast(bf16x8, (u32x4){a, b, c, d});
}

// Row index held by result register r of a 32x32 block in lane-half hf.
__device__ __forceinline__ constexpr int c32_row(int r, int hf) { return 8 * (r >> 2) + 4 * hf + (r & 3); }

// ----------------------------------------------------------------- shard sums
// s + part[0] + part[stride] + ... + part[(G-1) stride], added one shard at
// a time in shard order.  The loads of 8 shards are issued before their
// additions so that they are in flight together; the additions, and so the
// result, are those of the plain loop.
__device__ __forceinline__ f32x4 add_shards(f32x4 s, const f32x4* part, int64_t stride, int G) {
  int gg = 0;
  for (; gg + 8 <= G; gg += 8) {
    f32x4 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = part[(int64_t)(gg + q) * stride];
#pragma unroll
    for (int q = 0; q < 8; ++q) s += v[q];
  }
  for (; gg < G; ++gg) s += part[(int64_t)gg * stride];
  return s;
}

// ----------------------------------------------------------------- SiLU family
// sigma(z) from one exp2 and one reciprocal (both hardware transcendentals).
__device__ __forceinline__ float sigmoid(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}

// ----------------------------------------------------------------- io helpers
template <typename T> __device__ __forceinline__ float to_f(T x) { return (float)x; }
template <typename T> __device__ __forceinline__ T from_f(float x) { return (T)x; }

// Load n (4 or 8) consecutive io elements as floats.
template <typename IOT, int N>
__device__ __forceinline__ void load_vec(const IOT* p, float (&x)[N]) {
  if constexpr (std::is_same_v<IOT, float>) {
#pragma unroll
    for (int i = 0; i < N; i += 4) {
      f32x4 v = *reinterpret_cast<const f32x4*>(p + i);
      x[i] = v[0]; x[i + 1] = v[1]; x[i + 2] = v[2]; x[i + 3] = v[3];
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; i += 4) {
      bf16x4 v = *reinterpret_cast<const bf16x4*>(p + i);
      x[i] = (float)v[0]; x[i + 1] = (float)v[1]; x[i + 2] = (float)v[2]; x[i + 3] = (float)v[3];
    }
  }
}

template <typename IOT, int N>
__device__ __forceinline__ void store_vec(IOT* p, const float (&x)[N]) {
  if constexpr (std::is_same_v<IOT, float>) {
#pragma unroll
    for (int i = 0; i < N; i += 4) {
      f32x4 v = {x[i], x[i + 1], x[i + 2], x[i + 3]};
      *reinterpret_cast<f32x4*>(p + i) = v;
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; i += 4) {
      bf16x4 v = {(bf16)x[i], (bf16)x[i + 1], (bf16)x[i + 2], (bf16)x[i + 3]};
      *reinterpret_cast<bf16x4*>(p + i) = v;
    }
  }
}

// Sum over each aligned group of N consecutive lanes (N = 1, 2, 4, 8, 16),
// returned in every lane of the group.  DPP lane moves folded into the adds:
// lane^1 and lane^2 within a quad, then the mirror within 8 and within 16
// lanes (after the quad sums, the mirrored lane holds the other quad's / the
// other half's sum).  Both lanes of every pair add the same two values, so
// all lanes of a group get the bitwise-same result.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int N>
__device__ __forceinline__ float lane_group_sum(float x) {
  static_assert(N == 1 || N == 2 || N == 4 || N == 8 || N == 16, "groups of 1 to 16 lanes");
  if constexpr (N >= 2) x += dpp_move<0xB1>(x);   // quad_perm [1,0,3,2]
  if constexpr (N >= 4) x += dpp_move<0x4E>(x);   // quad_perm [2,3,0,1]
  if constexpr (N >= 8) x += dpp_move<0x141>(x);  // row_half_mirror
  if constexpr (N >= 16) x += dpp_move<0x140>(x); // row_mirror
  return x;
}

// One token row of D elements is spread over TPR = D/EPT consecutive lanes,
// EPT elements each.  Loads the row (zeros for masked rows) and, when asked,
// divides by max(||row||_2, eps); `inv` returns that divisor's reciprocal
// (1 when not normalising) and `nrm` the raw row norm.
template <typename IOT, int EPT>
__device__ __forceinline__ void load_row_norm(const IOT* rowp, bool valid, bool do_norm, float (&x)[EPT],
                                              float& inv) {
  constexpr int TPR = D / EPT;
  if (valid) {
    load_vec<IOT, EPT>(rowp, x);
  } else {
#pragma unroll
    for (int i = 0; i < EPT; ++i) x[i] = 0.f;
  }
  inv = 1.f;
  if (do_norm) {
    float ss = 0.f;
#pragma unroll
    for (int i = 0; i < EPT; ++i) ss = fmaf(x[i], x[i], ss);
    ss = lane_group_sum<TPR>(ss);
    inv = 1.0f / fmaxf(sqrtf(ss), NORM_EPS);
#pragma unroll
    for (int i = 0; i < EPT; ++i) x[i] *= inv;
  }
}

// XCD-aware block order: work-groups are dealt round-robin over the 8 XCDs,
// so consecutive logical blocks (the work-groups of one chain) are mapped to
// one XCD to share its L2.  Identity when the grid is not a multiple of 8.
__device__ __forceinline__ int xcd_linear_block() {
  const int nb = gridDim.x, bid = blockIdx.x;
  return (nb % 8 == 0) ? (bid % 8) * (nb / 8) + bid / 8 : bid;
}

// ----------------------------------------------------------------- launch plans
// One chunk step of the forward for a list of active sequences: the gradient
// partials of chunk s and the apply of chunk s-1 (both use the weights W_s).
struct FwdStepArgs {
  const void* Q;
  const void* K;
  const void* V;
  void* O;
  int64_t stride_tok, stride_head;
  const float* w1_src;  // W1 of chain c at w1_src + (c % w_mod) * w_cstride, [D][h]
  const float* w2_src;  // W2 likewise, [h][D]
  int64_t w_cstride;
  int32_t w_mod;
  int32_t H;
  uint32_t flags;
  int32_t G;        // work-groups per chain
  float* partial;   // [n_slots][2*D*h] gradient partials (slot = active chain * G + g)
  float* partial_loss;  // [n_slots]
  int32_t n_active;
  int32_t seq_id[MAXS];
  int64_t grad_start[MAXS];
  int32_t grad_len[MAXS];  // 0: no gradient chunk this step
  int64_t app_start[MAXS];
  int32_t app_len[MAXS];   // 0: no apply chunk this step
};

// What one work-group computes in one chunk step of one chain: the gradient
// partial of its token shard of chunk s (tiles g, g+G, g+2G, ... of the
// chunk) and the apply of its shard of chunk s-1, both with the weights W_s.
struct StepCtx {
  const void* Q;
  const void* K;
  const void* V;
  void* O;
  int64_t stride_tok, stride_head;
  uint32_t flags;
  const float* W1;   // W_s of the chain: [D][h]
  const float* W2;   // [h][D]
  int32_t head, g, G;
  int64_t gs;        // first token of the gradient chunk
  int32_t gl;        // its length (0: no gradient this step)
  int64_t as0;       // first token of the apply chunk
  int32_t al;        // its length (0: no apply this step)
  float* part;       // this work-group's gradient partial [2*D*h] (written iff gl > 0)
  float* part_loss;  // this work-group's loss partial
};

// The whole forward of many chains in one launch.  Work-groups form groups of
// G; a group takes the next chain (sequences in `order`, heads within a
// sequence) from a device counter and walks all of its chunk steps: every
// step, each member computes its shard (StepCtx), the members meet at a
// barrier, each reduces a 1/G slice of the G shard partials in a fixed order
// into W_{s+1} (and the checkpoint / final weights / loss), and they meet
// again before the next step reads W_{s+1}.  Barriers are counters in device
// memory with bounded waits (a wait that exceeds spin_limit polls sets *err
// and gives up); a group whose members share one XCD synchronises through
// that XCD's L2 alone.  All members of all groups must be resident at once; the
// host sizes the grid from the occupancy of this kernel.
struct PersistArgs {
  const void* Q;
  const void* K;
  const void* V;
  void* O;
  int64_t stride_tok, stride_head;
  const float* w1_0;   // W1_0 of (sequence b, head) at w1_0 + ((w0_per_seq ? b * H : 0) + head) * D * h
  const float* w2_0;
  int32_t w0_per_seq;
  int32_t H;
  uint32_t flags;
  float eta;
  int32_t G, n_groups, n_chains;
  int32_t xcd_map;      // 1: groups mapped to XCDs (grid a multiple of 8 * G)
  uint32_t spin_limit;
  int64_t M;            // tokens per chunk
  float* partial;       // [n_groups][G][2*D*h]
  float* partial_loss;  // [n_groups][G]
  float* wbuf;          // [n_groups][2][2*D*h] ping-pong weights
  uint32_t* bar;        // [n_groups] barrier counters, zero at launch
  uint32_t* slot;       // [n_groups] chain taken by the group
  uint32_t* next;       // next chain counter, zero at launch
  uint32_t* xcds;       // [n_groups] set of XCDs of the group's members, zero at launch
  uint32_t* err;        // bit 0: a barrier wait gave up
  float* ckpt;          // nullable; chunk c of entry e, head: row ck_row[e] + c of [rows][H][2*D*h]
  float* wT1;           // nullable; [B][H][D][h]
  float* wT2;           // [B][H][h][D]
  float* loss;          // nullable (single sequence): loss[head * loss_stride + c]
  int32_t loss_stride;
  // schedule entry e (chains e*H .. e*H+H-1), longest sequence first:
  int32_t seq_id[MAXS];     // its sequence b (index of W_0 with w0_per_seq, and of W_T)
  int64_t seq_start[MAXS];  // its first token
  int64_t seq_len[MAXS];    // its token count (> 0)
  int64_t ck_row[MAXS];     // its chunk-0 checkpoint row
};

// Reduction of the gradient partials and the fast-weight step W <- W - eta*g.
struct UpdStepArgs {
  const float* w1_src;
  const float* w2_src;
  int64_t w_cstride;
  int32_t w_mod;
  int32_t H, h;
  float eta;
  int32_t G;
  const float* partial;
  const float* partial_loss;
  float* w_dst;      // [chains][2*D*h] next weights
  float* ckpt;       // checkpoint rows: weights before this chunk; nullable
  int64_t ckpt_off[MAXS];  // float offset of active sequence i's row [H][2*D*h] in ckpt
  float* wT1;        // [chains][D][h] final weights, nullable
  float* wT2;        // [chains][h][D]
  float* loss;       // single sequence: loss[head * loss_stride + chunk]; nullable
  int32_t loss_stride, chunk;
  int32_t n_active;
  int32_t seq_id[MAXS];
  int32_t grad_len[MAXS];
  int32_t is_last[MAXS];
  // Global Context Synchronization: when gcs_chunks > 0 the grid covers the
  // H heads of one sequence and each head sums the partials of all
  // gcs_chunks chunk entries (entry e, slot (e*H + head)*G + g); chunk e has
  // gcs_M tokens except the last (gcs_last_len).
  int32_t gcs_chunks, gcs_M, gcs_last_len;
  // Streams with more chunks than partial slots are summed in passes of
  // gcs_chunks chunks each (the first chunk of this pass is gcs_entry0, the
  // index of its loss entry).  gcs_acc (nullable: one pass) is the running
  // sum [H][2*D*h]: a pass that is not the first adds its sum to it, a pass
  // that is not the last stores the total there and takes no step.
  float* gcs_acc;
  int32_t gcs_entry0, gcs_first, gcs_last;
};

// One reverse chunk step of the backward for every head of the active
// sequences: per sequence, the update adjoint of its chunk s and the apply
// adjoint of its chunk s-1.  Work-group slot = (active sequence * H + head)
// * G + shard.
struct BwdStepArgs {
  const void* Q;
  const void* K;
  const void* V;
  const void* dO;
  void* dQ;
  void* dK;
  void* dV;
  int64_t stride_tok, stride_head;
  const void* prep;     // per (active sequence, head) 8 operand matrices of D*h (see ttt_bwd_prep)
  int32_t H;
  uint32_t flags;
  float eta;
  int32_t G;
  float* partial;       // [n_active*H*G][2*D*h]
  float* partial_deta;  // [n_active*H*G]
  int32_t n_active;
  int64_t grad_start[MAXS];
  int32_t grad_len[MAXS];  // chunk s tokens (0: none)
  int64_t app_start[MAXS];
  int32_t app_len[MAXS];   // chunk s-1 tokens (0: none)
};

// Operand preparation for the active sequences of one backward step.
struct BwdPrepArgs {
  const float* w_src[MAXS];   // W_s of active sequence i, [H][2*D*h]
  const float* wh_src[MAXS];  // carried adjoint, [H][2*D*h]; null = 0
  void* prep;                 // [n_active][H][8][D*h] operand type
  int32_t H, h;
};

// Per active sequence i (sequence seq[i]): its adjoint output = its adjoint
// input (0 if wh_src_base is null) + the sum of its G shard partials in fixed
// order; deta (+)= the sum of its dη partials.  Chain (b, head) of the
// adjoint buffers lives at base + (b*H + head) * 2*D*h.
struct BwdReduceArgs {
  const float* wh_src_base;  // null: zero adjoint
  float* wh_dst_base;
  float* fin_base;           // final adjoints of a shared W0 (nullable)
  float* dst1;               // final gradients, split: dW1 + (per_seq ? b : 0)*H*D*h + head*D*h
  float* dst2;
  int32_t dst_per_seq;
  float* deta_base;          // deta of sequence b at deta_base + b*H
  const float* partial;
  const float* partial_deta;
  int32_t n_active, G, H, h;
  int32_t seq[MAXS];
  int32_t flags[MAXS];       // bit 0: final step of this sequence; bit 1: first step (deta starts at 0)
  // Fused operand preparation for the next reverse step (prep_next null =
  // none): active sequence i becomes slot next_slot[i] (< 0: not active next
  // step), whose W_s is checkpoint row ckpt_row[i]; layout as in ttt_bwd_prep.
  void* prep_next;
  int32_t prep_bf16;
  const float* ckpt;
  int32_t next_slot[MAXS];
  int64_t ckpt_row[MAXS];
};

// Shared initial weights over B sequences: dW1/dW2 = sum over b of the
// per-sequence gradients src[b] ([H][2*D*h]), deta[head] = sum over b of
// deta_src[b][head], in sequence order.
struct BwdSumArgs {
  const float* src;
  const float* deta_src;
  float* dW1;
  float* dW2;
  float* deta;
  int32_t B, H, h;
};

}  // namespace ttt
