// Forward kernels of the chunked TTT update/apply (Sec. 4.2 Eq. 8, Sec. 3.2
// Eq. 3-4) for gfx950.
//
// One launch of ttt_fwd_step processes one chunk step for every active chain
// (sequence x head): the gradient of chunk s over a token shard (Eq. 8; the
// shards of a chunk are summed afterwards, Eq. 10) and the apply of chunk s-1
// (Eq. 4), since both use the same weights W_s.  ttt_update then reduces the
// shard partials in a fixed order and steps W_{s+1} = W_s - eta * grad.
//
// Work split inside a work-group: wave w owns hidden units [32w, 32w+32), so
// its slices of W1 (columns) and W2 (rows) stay in registers for the whole
// chunk, and it accumulates its slices of grad W1 / grad W2 in registers over
// every token tile of its shard.  Per 32-token tile:
//   P1  load K, V (or Q) rows, L2-normalise (FP32), stage in LDS
//   P2  Z = K W1 (32x32 matrix-core block per wave), A = SiLU(Z), s'(Z);
//       A is staged to LDS for the contraction over the hidden axis
//   P3  Y = A W2 as 16x16 blocks over the full hidden axis, R = Y - V,
//       E = (2/M) R, loss; (apply tiles: store O = Y)
//   P4  P = E W2^T, D = P * s'(Z), grad W1 += K^T D, grad W2 += A^T E
// Z/A/D keep the token index in registers (32x32 result layout), which is
// exactly the contraction-slot layout the token-sum products need, so only A
// goes through LDS to be contracted over the hidden axis.
#include <hip/hip_runtime.h>

#include "ttt_common.h"
#include "ttt_internal.h"

namespace ttt {

// FP32-operand chunk step.  FP32 tiles need twice the LDS of BF16 ones, so
// the gradient tiles and the apply tiles run in two loops over single-
// buffered LDS tiles (4 barriers per tile); the next tile's rows are
// prefetched into registers while the current tile computes.
template <typename IOT, int NW, bool OPAQUE_TID = false>
__device__ __forceinline__ void fwd_body_f32(const StepCtx& p) {
  constexpr int HH = NW * 32;  // hidden size
  constexpr int NT = NW * 64;
  constexpr int EPT = D * TT / NT;  // row elements per thread when loading
  constexpr int TPR = D / EPT;
  constexpr int XS_LD = D + 4;
  constexpr int VS_LD = D + 4;
  constexpr int AS_LD = HH + 4;
  constexpr int W2T_LD = HH + 4;
  constexpr int DH = D * HH;

  __shared__ __attribute__((aligned(16))) float xs[TT * XS_LD];   // K (or Q) rows, normalised
  __shared__ __attribute__((aligned(16))) float vs[TT * VS_LD];   // V rows, normalised
  __shared__ __attribute__((aligned(16))) float as_[TT * AS_LD];  // A = SiLU(K W1) (or of Q)
  __shared__ __attribute__((aligned(16))) float es[TT * XS_LD];   // E
  __shared__ __attribute__((aligned(16))) float w2t[D * W2T_LD];  // W2^T
  __shared__ float red[NW];

  // in a loop that calls this body (the persistent kernel) the lane index is
  // made opaque to the compiler, so that nothing derived from it is hoisted
  // out of the loop (it would hold registers across the whole loop)
  int tid = threadIdx.x;
  if constexpr (OPAQUE_TID) asm volatile("" : "+v"(tid));
  const int w = tid >> 6, l = tid & 63, l32 = l & 31, hf = l >> 5, l16 = l & 15, g4 = l >> 4;
  const int G = p.G, g = p.g, head = p.head;
  const int hid = w * 32 + l32;
  const float* W1 = p.W1;
  const float* W2 = p.W2;

  // B operand of Y = A W2 over the full hidden axis, from LDS (W2^T).
  for (int idx = tid; idx < DH; idx += NT) {
    const int hh = idx / D, dd = idx % D;
    w2t[dd * W2T_LD + hh] = W2[idx];
  }
  // Register-resident operand slices of this wave's hidden block.
  float w1f[32], w2f[32];
#pragma unroll
  for (int s = 0; s < 32; ++s) {
    w1f[s] = W1[(32 * hf + s) * HH + hid];
    w2f[s] = W2[hid * D + 32 * hf + s];
  }

  const bool norm_q = p.flags & 1u, norm_k = p.flags & 2u, norm_v = p.flags & 4u;
  const int row = tid / TPR, col0 = (tid % TPR) * EPT;
  const int64_t hoff = (int64_t)head * p.stride_head;
  const int gl = p.gl, al = p.al;
  const int64_t gs = p.gs, as0 = p.as0;
  const int n_gt = (gl + TT - 1) / TT, n_at = (al + TT - 1) / TT;
  const int my_g = n_gt > g ? (n_gt - g + G - 1) / G : 0;  // tiles of this work-group
  const int my_a = n_at > g ? (n_at - g + G - 1) / G : 0;
  const float e_scale = gl > 0 ? 2.0f / (float)gl : 0.f;

  // ---- phase helpers
  // raw row fetch (registers) for tile `it` of this work-group; zeros when
  // the row is past the chunk end.
  auto fetch_row = [&](const void* base, int64_t start, int len, int it, float (&x)[EPT]) {
    const int tr = (g + it * G) * TT + row;  // token index within the chunk
    if (tr < len) {
      load_vec<IOT, EPT>(static_cast<const IOT*>(base) + (start + tr) * p.stride_tok + hoff + col0, x);
    } else {
#pragma unroll
      for (int i = 0; i < EPT; ++i) x[i] = 0.f;
    }
  };
  auto normalise = [&](float (&x)[EPT], bool do_norm) {
    if (!do_norm) return;
    float ss = 0.f;
#pragma unroll
    for (int i = 0; i < EPT; ++i) ss = fmaf(x[i], x[i], ss);
    ss = lane_group_sum<TPR>(ss);
    const float inv = 1.0f / fmaxf(sqrtf(ss), NORM_EPS);
#pragma unroll
    for (int i = 0; i < EPT; ++i) x[i] *= inv;
  };
  // Z = X W1 for this wave's hidden block: 32x32 result, rows = tokens.
  auto z_block = [&](const float* X) {
    f32x16 z = {};
#pragma unroll
    for (int s4 = 0; s4 < 8; ++s4) {
      const f32x4 a = *reinterpret_cast<const f32x4*>(&X[l32 * XS_LD + 32 * hf + 4 * s4]);
#pragma unroll
      for (int e = 0; e < 4; ++e) z = mma32(a[e], w1f[4 * s4 + e], z);
    }
    return z;
  };
  // 16x16 block (token block tb, feature block db) of S W2, S staged [tok][h].
  auto y_block = [&](const float* S, int tb, int db) {
    f32x4 y = {};
    const int arow = 16 * tb + l16, dcol = 16 * db + l16;
#pragma unroll
    for (int u = 0; u < HH / 16; ++u) {
      const f32x4 a = *reinterpret_cast<const f32x4*>(&S[arow * AS_LD + (HH / 4) * g4 + 4 * u]);
      const f32x4 b = *reinterpret_cast<const f32x4*>(&w2t[dcol * W2T_LD + (HH / 4) * g4 + 4 * u]);
#pragma unroll
      for (int e = 0; e < 4; ++e) y = mma16(a[e], b[e], y);
    }
    return y;
  };
  // A = SiLU(Z) staged to S; keeps s'(Z) and A (in za) for the gradient.
  auto silu_stage = [&](f32x16& za, float (&s1)[16], float* S) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float zr = za[r];
      const float sg = sigmoid(zr);
      const float av = zr * sg;
      s1[r] = fmaf(av, 1.0f - sg, sg);
      za[r] = av;
      S[c32_row(r, hf) * AS_LD + hid] = av;
    }
  };
  auto silu_stage_apply = [&](const f32x16& za, float* S) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float zr = za[r];
      S[c32_row(r, hf) * AS_LD + hid] = zr * sigmoid(zr);
    }
  };
  // Residual, loss and E for this wave's Y blocks (E staged for the gradient).
  auto residual = [&](float& lacc) {
#pragma unroll
    for (int bi = 0; bi < 8 / NW; ++bi) {
      const int b = w + NW * bi, tb = b & 1, db = b >> 1;
      const f32x4 y = y_block(as_, tb, db);
      const int dcol = 16 * db + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int tok = 16 * tb + 4 * g4 + r;
        const float R = y[r] - vs[tok * VS_LD + dcol];
        lacc = fmaf(R, R, lacc);
        es[tok * XS_LD + dcol] = e_scale * R;
      }
    }
  };
  auto apply_out = [&](int it) {
    IOT* O = static_cast<IOT*>(p.O);
    const int t_base = (g + it * G) * TT;
#pragma unroll
    for (int bi = 0; bi < 8 / NW; ++bi) {
      const int b = w + NW * bi, tb = b & 1, db = b >> 1;
      const f32x4 y = y_block(as_, tb, db);
      const int dcol = 16 * db + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int tok = 16 * tb + 4 * g4 + r;
        if (t_base + tok < al) O[(as0 + t_base + tok) * p.stride_tok + hoff + dcol] = from_f<IOT>(y[r]);
      }
    }
  };
  // P = E W2^T, D = P * s'(Z), grad W1 += K^T D, grad W2 += A^T E.
  auto grad_update = [&](const f32x16& za, const float (&s1)[16], f32x16 (&gw1)[2], f32x16 (&gw2)[2]) {
    f32x16 pz = {};
#pragma unroll
    for (int s4 = 0; s4 < 8; ++s4) {
      const f32x4 a = *reinterpret_cast<const f32x4*>(&es[l32 * XS_LD + 32 * hf + 4 * s4]);
#pragma unroll
      for (int e = 0; e < 4; ++e) pz = mma32(a[e], w2f[4 * s4 + e], pz);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) pz[r] *= s1[r];
#pragma unroll
    for (int db = 0; db < 2; ++db) {
      const int dd = 32 * db + l32;
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const int tk = c32_row(s, hf);
        gw1[db] = mma32(xs[tk * XS_LD + dd], pz[s], gw1[db]);
        gw2[db] = mma32(za[s], es[tk * XS_LD + dd], gw2[db]);
      }
    }
  };
  auto stage_kv = [&](float (&xk)[EPT], float (&xv)[EPT]) {
    normalise(xk, norm_k);
    normalise(xv, norm_v);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      xs[row * XS_LD + col0 + i] = xk[i];
      vs[row * VS_LD + col0 + i] = xv[i];
    }
  };

  f32x16 gw1[2] = {}, gw2[2] = {};
  float lacc = 0.f;
  float rk[EPT], rv[EPT], rq[EPT];

  // gradient tiles
  if (my_g > 0) {
    fetch_row(p.K, gs, gl, 0, rk);
    fetch_row(p.V, gs, gl, 0, rv);
  }
  for (int it = 0; it < my_g; ++it) {
    stage_kv(rk, rv);
    if (it + 1 < my_g) {
      fetch_row(p.K, gs, gl, it + 1, rk);
      fetch_row(p.V, gs, gl, it + 1, rv);
    }
    __syncthreads();
    f32x16 za = z_block(xs);
    float s1[16];
    silu_stage(za, s1, as_);
    __syncthreads();
    residual(lacc);
    __syncthreads();
    grad_update(za, s1, gw1, gw2);
    __syncthreads();
  }
  // apply tiles
  if (my_a > 0) fetch_row(p.Q, as0, al, 0, rq);
  for (int it = 0; it < my_a; ++it) {
    normalise(rq, norm_q);
#pragma unroll
    for (int i = 0; i < EPT; ++i) xs[row * XS_LD + col0 + i] = rq[i];
    if (it + 1 < my_a) fetch_row(p.Q, as0, al, it + 1, rq);
    __syncthreads();
    silu_stage_apply(z_block(xs), as_);
    __syncthreads();
    apply_out(it);
    __syncthreads();
  }

  if (gl > 0) {
    // Shard partials: grad W1 [D][h] then grad W2 [h][D].
    float* part = p.part;
#pragma unroll
    for (int db = 0; db < 2; ++db)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int rr = c32_row(r, hf);
        part[(32 * db + rr) * HH + hid] = gw1[db][r];
        part[DH + (32 * w + rr) * D + 32 * db + l32] = gw2[db][r];
      }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) lacc += __shfl_xor(lacc, m, 64);
    if (l == 0) red[w] = lacc;
    __syncthreads();
    if (tid == 0) {
      float s = 0.f;
      for (int i = 0; i < NW; ++i) s += red[i];
      *p.part_loss = s;
    }
  }
}

// BF16-operand chunk step, software-pipelined over token tiles.  Iteration
// i holds, between two barriers each,
//   phase A: Y_i = A_i W2 -> residual -> E_i (staged), O_i = Aq_i W2 (stored),
//            Z_{i+1} = K_{i+1} W1 -> SiLU, s'(Z) (kept in registers)
//   phase B: P_i = E_i W2^T, D_i = P_i s'(Z_i), grad W1 += K_i^T D_i,
//            grad W2 += A_i^T E_i; A_{i+1} staged from registers;
//            Zq_{i+1}^T = W1^T Q_{i+1}^T -> SiLU -> Aq_{i+1} (staged);
//            rows of tile i+2 normalised into LDS, rows of tile i+3 fetched
// which balances matrix-core products against the transcendental-heavy
// activations in both phases, and lets A, Aq and E live in one LDS buffer
// each (each is written in one phase and read in the next).  Every tile is
// staged row-major only: the token-contraction operands K^T and E^T and the
// residual's V columns are read with the transposing LDS load
// (ds_read_b64_tr_b16), so no tile is ever written transposed.
// -log2(e) is folded into the W1 operand (the exponent comes straight out of
// the product) and -ln(2) into the W2 operand of Y and O; the A-side gradient
// is rescaled once at the end.
//
// Token rows are fetched and O is stored through buffer resources that cover
// exactly the valid rows of the tile, so rows past a chunk's end read as zero
// and their stores are dropped by the hardware range check: the loop body is
// free of branches, and zero rows add nothing to the gradient or the loss
// (K = V = 0 gives Z = 0, A = 0, Y = 0, R = 0).  A block whose shard has both
// gradient and apply tiles runs the fused body; shards with only one kind run
// a body without the other's work.
template <typename IOT, int NW, bool OPAQUE_TID = false>
__device__ __forceinline__ void fwd_body_bf(const StepCtx& p) {
  constexpr int HH = NW * 32;
  constexpr int NT = NW * 64;
  constexpr int EPT = D * TT / NT;
  constexpr int TPR = D / EPT;
  // Row pitches of the LDS tiles (elements).  The token-row tiles are read
  // by 16-byte row fragments, by the transposing read and written by 4-byte
  // and 2-byte stores; among the pitches that keep the 16-byte reads aligned
  // (multiples of 8) the measured pass times on MI355X favour 80, 88 and 104
  // (8-sequence batch, persistent launch: 7.44 / 7.48 / 7.51 ms against
  // 8.26 / 8.67 / 8.31 ms at 72 / 96 / 112); outputs are bit-identical.
  constexpr int XS_LD = D + 24;  // K rows
  constexpr int VS_LD = XS_LD;   // V rows
  constexpr int QS_LD = XS_LD;   // Q rows
  constexpr int ES_LD = XS_LD;   // E rows
  constexpr int AS_LD = HH + 8;
  constexpr int DH = D * HH;
  constexpr float LOG2E = 1.4426950408889634f;
  constexpr float LN2 = 0.6931471805599453f;
  typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));
  typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

  __shared__ __attribute__((aligned(16))) bf16 xs[3][TT * XS_LD];    // K rows
  __shared__ __attribute__((aligned(16))) bf16 vs[2][TT * VS_LD];    // V rows
  __shared__ __attribute__((aligned(16))) bf16 qs[2][TT * QS_LD];    // Q rows
  __shared__ __attribute__((aligned(16))) bf16 as_[TT * AS_LD];      // A' = -log2(e) SiLU(K W1)
  __shared__ __attribute__((aligned(16))) bf16 aqs[TT * AS_LD];      // -log2(e) SiLU(Q W1)
  __shared__ __attribute__((aligned(16))) bf16 es[TT * ES_LD];       // E
  __shared__ float red[NW];

  // in a loop that calls this body (the persistent kernel) the lane index is
  // made opaque to the compiler, so that nothing derived from it is hoisted
  // out of the loop (it would hold registers across the whole loop)
  int tid = threadIdx.x;
  if constexpr (OPAQUE_TID) asm volatile("" : "+v"(tid));
  const int w = tid >> 6, l = tid & 63, l32 = l & 31, hf = l >> 5, l16 = l & 15, g4 = l >> 4;
  const int G = p.G, g = p.g, head = p.head;
  const int hid = w * 32 + l32;
  const float* W1 = p.W1;
  const float* W2 = p.W2;

  // Register-resident operands, packed once; the empty asm pins each packed
  // word so that the compiler keeps it instead of re-deriving it from the
  // source floats inside the token loop.  w1b serves as the B operand of
  // Z = K W1 and, unchanged, as the A operand of Zq^T = W1^T Q^T.
  bf16x8 w1b[4], w2b[4], w2y[8 / NW][HH / 32];
  auto pin8 = [](bf16x8& v) {
    u32x4 u = __builtin_bit_cast(u32x4, v);
    asm volatile("" : "+v"(u));
    v = __builtin_bit_cast(bf16x8, u);
  };
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    uint32_t a[4], b[4];
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      a[e / 2] = pack_bf16x2(-LOG2E * W1[(16 * m + 8 * hf + e) * HH + hid],
                             -LOG2E * W1[(16 * m + 8 * hf + e + 1) * HH + hid]);
      b[e / 2] = pack_bf16x2(W2[hid * D + 16 * m + 8 * hf + e], W2[hid * D + 16 * m + 8 * hf + e + 1]);
    }
    w1b[m] = as_bf16x8(a[0], a[1], a[2], a[3]);
    w2b[m] = as_bf16x8(b[0], b[1], b[2], b[3]);
    pin8(w1b[m]);
    pin8(w2b[m]);
  }
#pragma unroll
  for (int bi = 0; bi < 8 / NW; ++bi) {
    const int dcol = 16 * ((w + NW * bi) >> 1) + l16;
#pragma unroll
    for (int u = 0; u < HH / 32; ++u) {
      uint32_t c[4];
#pragma unroll
      for (int e = 0; e < 8; e += 2)
        c[e / 2] = pack_bf16x2(-LN2 * W2[((HH / 4) * g4 + 8 * u + e) * D + dcol],
                               -LN2 * W2[((HH / 4) * g4 + 8 * u + e + 1) * D + dcol]);
      w2y[bi][u] = as_bf16x8(c[0], c[1], c[2], c[3]);
      pin8(w2y[bi][u]);
    }
  }

  const bool norm_q = p.flags & 1u, norm_k = p.flags & 2u, norm_v = p.flags & 4u;
  const int row = tid / TPR, col0 = (tid % TPR) * EPT;
  const int64_t hoff = (int64_t)head * p.stride_head;
  const int gl = p.gl, al = p.al;
  const int64_t gs = p.gs, as0 = p.as0;
  const int n_gt = (gl + TT - 1) / TT, n_at = (al + TT - 1) / TT;
  const int my_g = n_gt > g ? (n_gt - g + G - 1) / G : 0;
  const int my_a = n_at > g ? (n_at - g + G - 1) / G : 0;
  const int iters = max(my_g, my_a);
  const float e_scale = gl > 0 ? 2.0f / (float)gl : 0.f;

  // Buffer resource over the valid rows of tile `it` of this shard (token
  // rows t0 .. t0+rows-1 of a region of `len` rows starting at `base`);
  // stride_tok * TT * 4 bytes fits 31 bits (checked by the host).
  const int tok_bytes = (int)p.stride_tok * (int)sizeof(IOT);
  auto tile_rsrc = [&](const void* base, int len, int it) {
    const int t0 = (g + it * G) * TT;
    const int rows = min(max(len - t0, 0), TT);
    const int bytes = max(rows * tok_bytes - tok_bytes + D * (int)sizeof(IOT), 0);  // 0 rows: 0 bytes
    IOT* b = const_cast<IOT*>(static_cast<const IOT*>(base)) + (int64_t)t0 * p.stride_tok;
    return __builtin_amdgcn_make_buffer_rsrc(b, (short)0, bytes, 0x00020000);
  };
  const IOT* const Kb = static_cast<const IOT*>(p.K) + gs * p.stride_tok + hoff;
  const IOT* const Vb = static_cast<const IOT*>(p.V) + gs * p.stride_tok + hoff;
  const IOT* const Qb = static_cast<const IOT*>(p.Q) + as0 * p.stride_tok + hoff;
  IOT* const Ob = static_cast<IOT*>(p.O) + as0 * p.stride_tok + hoff;
  const int row_voff = row * tok_bytes + col0 * (int)sizeof(IOT);

  // prefetched raw rows kept in the io type (EPT elements per thread)
  typedef IOT iovec __attribute__((ext_vector_type(EPT)));
  iovec rk = {}, rv = {}, rq = {};
  auto load_rows = [&](__amdgpu_buffer_rsrc_t r) -> iovec {
    constexpr int BYTES = EPT * (int)sizeof(IOT);
    if constexpr (BYTES == 8) {
      return __builtin_bit_cast(iovec, __builtin_amdgcn_raw_buffer_load_b64(r, row_voff, 0, 0));
    } else if constexpr (BYTES == 16) {
      return __builtin_bit_cast(iovec, __builtin_amdgcn_raw_buffer_load_b128(r, row_voff, 0, 0));
    } else {
      static_assert(BYTES == 32, "4 or 8 elements of 2 or 4 bytes");
      typedef uint32_t u32x8 __attribute__((ext_vector_type(8)));
      const u32x4 lo = __builtin_amdgcn_raw_buffer_load_b128(r, row_voff, 0, 0);
      const u32x4 hi = __builtin_amdgcn_raw_buffer_load_b128(r, row_voff + 16, 0, 0);
      return __builtin_bit_cast(iovec, (u32x8){lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]});
    }
  };

  // 1 / max(||x||, eps) = rsq(max(||x||^2, eps^2)); computed whether or not
  // the rows are normalised (a select instead of a branch in the loop body)
  auto normalise = [&](float (&x)[EPT], bool do_norm) {
    float ss = 0.f;
#pragma unroll
    for (int i = 0; i < EPT; ++i) ss = fmaf(x[i], x[i], ss);
    ss = lane_group_sum<TPR>(ss);
    const float inv = do_norm ? __builtin_amdgcn_rsqf(fmaxf(ss, NORM_EPS * NORM_EPS)) : 1.0f;
#pragma unroll
    for (int i = 0; i < EPT; ++i) x[i] *= inv;
  };
  auto z_block = [&](const bf16* X) {  // Z' = X W1' (token rows, hidden columns)
    f32x16 z = {};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(&X[l32 * XS_LD + 16 * m + 8 * hf]);
      z = mma32(a, w1b[m], z);
    }
    return z;
  };
  auto zt_block = [&](const bf16* X) {  // Z'^T = W1'^T X^T (hidden rows, token columns)
    f32x16 z = {};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(&X[l32 * QS_LD + 16 * m + 8 * hf]);
      z = mma32(w1b[m], b, z);
    }
    return z;
  };
  auto y_block = [&](const bf16* S, int tb, int bi) {
    f32x4 y = {};
    const int arow = 16 * tb + l16;
#pragma unroll
    for (int u = 0; u < HH / 32; ++u) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(&S[arow * AS_LD + (HH / 4) * g4 + 8 * u]);
      y = mma16(a, w2y[bi][u], y);
    }
    return y;
  };

  // Transposing read of a row-major bf16 tile T (pitch ld): in each
  // group of 16 lanes, lane j receives T[t0 + q][c0 + j] for q = 0..3.  The
  // instruction hands lane j element j%4 of the 8-byte runs addressed by
  // lanes j/4 + 4q of its group, so lane i points at row t0 + i/4, columns
  // c0 + 4(i%4) .. +3.
  // `off` = this lane's element offset; the per-lane part is computed once
  // below, the rest are immediates of the load.
  typedef __attribute__((address_space(3))) bf16x4 lds_bf16x4;
  auto tr4 = [&](const bf16* T, int off) -> bf16x4 {
    return __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4*)((__attribute__((address_space(3))) bf16*)(T + off)));
  };
  auto tr_lane = [&](int ld) { return (l16 >> 2) * ld + 4 * (l16 & 3); };
  // token-contraction operand of a row-major [token][d] tile: lane (d = 32 db
  // + l32, hf) holds tokens 16m + 4hf + 0..3 and 16m + 8 + 4hf + 0..3, the
  // token slots of result registers 8m .. 8m+7 of a 32x32 block
  auto tok_frag = [&](const bf16* T, int ld, int m, int db) -> bf16x8 {
    const int tok_lane = tr_lane(ld) + 4 * hf * ld + 16 * ((l >> 4) & 1);
    const bf16x4 lo = tr4(T, tok_lane + 16 * m * ld + 32 * db);
    const bf16x4 hi = tr4(T, tok_lane + (16 * m + 8) * ld + 32 * db);
    return (bf16x8){lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  };

  f32x16 gw1[2] = {}, gw2[2] = {};
  float lacc = 0.f;
  uint32_t apk[2][8];     // per tile parity: A' packed in bf16 pairs (token-contraction operand)
  h16x2 s1h[2][8];        // per tile parity: s'(Z) in f16 pairs

  auto run = [&](auto MC) {
    constexpr int MODE = decltype(MC)::value;
    constexpr bool DO_G = (MODE & 1) != 0, DO_A = (MODE & 2) != 0;

    auto fetch = [&](int it) {
      if constexpr (DO_G) {
        rk = load_rows(tile_rsrc(Kb, gl, it));
        rv = load_rows(tile_rsrc(Vb, gl, it));
      }
      if constexpr (DO_A) rq = load_rows(tile_rsrc(Qb, al, it));
    };
    // normalise the fetched rows of tile `it` into LDS
    auto stage_rows = [&](int it) {
      const int b3 = it % 3, b2 = it & 1;
      if constexpr (DO_G) {
        float fk[EPT], fv[EPT];
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
          fk[i] = (float)rk[i];
          fv[i] = (float)rv[i];
        }
        normalise(fk, norm_k);
        normalise(fv, norm_v);
#pragma unroll
        for (int i = 0; i < EPT; i += 2) {
          *reinterpret_cast<uint32_t*>(&xs[b3][row * XS_LD + col0 + i]) = pack_bf16x2(fk[i], fk[i + 1]);
          *reinterpret_cast<uint32_t*>(&vs[b2][row * VS_LD + col0 + i]) = pack_bf16x2(fv[i], fv[i + 1]);
        }
      }
      if constexpr (DO_A) {
        float fq[EPT];
#pragma unroll
        for (int i = 0; i < EPT; ++i) fq[i] = (float)rq[i];
        normalise(fq, norm_q);
#pragma unroll
        for (int i = 0; i < EPT; i += 2)
          *reinterpret_cast<uint32_t*>(&qs[b2][row * QS_LD + col0 + i]) = pack_bf16x2(fq[i], fq[i + 1]);
      }
    };
    // z' = -log2(e) z:  sigma = 1/(1+2^z'),  A' = z' sigma = -log2(e) SiLU(z),
    // s'(z) = sigma + A (1 - sigma) = sigma + A' ln2 (sigma - 1).  Results
    // are packed in pairs: A' as bf16 (token-contraction operand, staged to
    // LDS one phase later), s'(z) as f16.
    auto act_grad = [&](const f32x16& z, uint32_t (&ap)[8], h16x2 (&sh)[8]) {
#pragma unroll
      for (int r = 0; r < 16; r += 2) {
        const float z0 = z[r], z1 = z[r + 1];
        const float s0g = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z0));
        const float s1g = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z1));
        const float a0 = z0 * s0g, a1 = z1 * s1g;
        ap[r >> 1] = pack_bf16x2(a0, a1);
        sh[r >> 1] = __builtin_convertvector((f32x2){fmaf(a0, fmaf(s0g, LN2, -LN2), s0g),
                                                      fmaf(a1, fmaf(s1g, LN2, -LN2), s1g)}, h16x2);
      }
    };
    // A' of one tile from its packed register copy into the [token][hidden] tile
    auto put_a = [&](const uint32_t (&ap)[8]) {
      uint16_t* S16 = reinterpret_cast<uint16_t*>(as_);
#pragma unroll
      for (int r = 0; r < 16; r += 2) {
        S16[c32_row(r, hf) * AS_LD + hid] = (uint16_t)ap[r >> 1];
        S16[c32_row(r + 1, hf) * AS_LD + hid] = (uint16_t)(ap[r >> 1] >> 16);
      }
    };
    // Aq' from Zq'^T: lane (token l32) holds 4 runs of 4 consecutive hidden
    // units, each written as one 8-byte word of the [token][hidden] tile.
    auto act_apply_t = [&](const f32x16& zt) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float z = zt[4 * j + q];
          a[q] = z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z));
        }
        *reinterpret_cast<u32x2*>(&aqs[l32 * AS_LD + 32 * w + 8 * j + 4 * hf]) =
            (u32x2){pack_bf16x2(a[0], a[1]), pack_bf16x2(a[2], a[3])};
      }
    };

    // phase A of iteration `it` (tile parity P = it & 1)
    auto phase_a = [&](int it, auto PC) {
      constexpr int P = decltype(PC)::value;
      // the next tile's product first: its activation (the long VALU part)
      // then overlaps the Y and O products
      f32x16 zn;
      if constexpr (DO_G) zn = z_block(xs[(it + 1) % 3]);
      if constexpr (DO_G) {
#pragma unroll
        for (int bi = 0; bi < 8 / NW; ++bi) {
          const int b = w + NW * bi, tb = b & 1, db = b >> 1;
          const f32x4 y = y_block(as_, tb, bi);
          const int dcol = 16 * db + l16;
          const int tok0 = 16 * tb + 4 * g4;
          const bf16x4 vv = tr4(vs[P], tr_lane(VS_LD) + tok0 * VS_LD + 16 * db);  // V[tok0 + r][dcol]
          float ev[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float R = y[r] - (float)vv[r];
            lacc = fmaf(R, R, lacc);
            ev[r] = e_scale * R;
          }
          const uint32_t e01 = pack_bf16x2(ev[0], ev[1]), e23 = pack_bf16x2(ev[2], ev[3]);
          uint16_t* es16 = reinterpret_cast<uint16_t*>(es);
          es16[(tok0 + 0) * ES_LD + dcol] = (uint16_t)e01;
          es16[(tok0 + 1) * ES_LD + dcol] = (uint16_t)(e01 >> 16);
          es16[(tok0 + 2) * ES_LD + dcol] = (uint16_t)e23;
          es16[(tok0 + 3) * ES_LD + dcol] = (uint16_t)(e23 >> 16);
        }
      }
      if constexpr (DO_A) {
        const auto ro = tile_rsrc(Ob, al, it);
#pragma unroll
        for (int bi = 0; bi < 8 / NW; ++bi) {
          const int b = w + NW * bi, tb = b & 1, db = b >> 1;
          const f32x4 y = y_block(aqs, tb, bi);
          const int voff = (16 * tb + 4 * g4) * tok_bytes + (16 * db + l16) * (int)sizeof(IOT);
          // whole-vector bit cast: this compiler turns a bit cast of one
          // vector element (y[r]) into a read of element 0
          const u32x4 yu = __builtin_bit_cast(u32x4, y);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if constexpr (std::is_same_v<IOT, float>)
              __builtin_amdgcn_raw_buffer_store_b32(yu[r], ro, voff, r * tok_bytes, 0);
            else
              __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, (bf16)y[r]), ro, voff, r * tok_bytes, 0);
          }
        }
      }
      if constexpr (DO_G) act_grad(zn, apk[P ^ 1], s1h[P ^ 1]);
    };
    // phase B of iteration `it`.  The LDS writes that depend only on
    // registers (the rows of tile i+2, A of tile i+1) go first: their buffers
    // are not read in this phase, and issued early their latency overlaps
    // the products instead of delaying the closing barrier.
    auto phase_b = [&](int it, auto PC) {
      constexpr int P = decltype(PC)::value;
      stage_rows(it + 2);
      fetch(it + 3);
      if constexpr (DO_G) put_a(apk[P ^ 1]);
      f32x16 zq;
      if constexpr (DO_A) zq = zt_block(qs[P ^ 1]);
      if constexpr (DO_G) {
        const int b3 = it % 3;
        f32x16 pz = {};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const bf16x8 a = *reinterpret_cast<const bf16x8*>(&es[l32 * ES_LD + 16 * m + 8 * hf]);
          pz = mma32(a, w2b[m], pz);
        }
        const bf16x8 apv[2] = {as_bf16x8(apk[P][0], apk[P][1], apk[P][2], apk[P][3]),
                               as_bf16x8(apk[P][4], apk[P][5], apk[P][6], apk[P][7])};
#pragma unroll
        for (int db = 0; db < 2; ++db)
#pragma unroll
          for (int m = 0; m < 2; ++m) gw2[db] = mma32(apv[m], tok_frag(es, ES_LD, m, db), gw2[db]);
        uint32_t dw[8];
#pragma unroll
        for (int r = 0; r < 16; r += 2) {
          const h16x2 sv = s1h[P][r >> 1];
          dw[r >> 1] = pack_bf16x2(fmaf(pz[r], (float)sv[0], 0.0f), fmaf(pz[r + 1], (float)sv[1], 0.0f));
        }
        const bf16x8 dpk[2] = {as_bf16x8(dw[0], dw[1], dw[2], dw[3]), as_bf16x8(dw[4], dw[5], dw[6], dw[7])};
#pragma unroll
        for (int db = 0; db < 2; ++db)
#pragma unroll
          for (int m = 0; m < 2; ++m) gw1[db] = mma32(tok_frag(xs[b3], XS_LD, m, db), dpk[m], gw1[db]);
      }
      if constexpr (DO_A) act_apply_t(zq);
    };

    // prologue: rows of tiles 0 and 1 staged, activations of tile 0 staged
    fetch(0);
    stage_rows(0);
    fetch(1);
    __syncthreads();
    if constexpr (DO_G) {
      act_grad(z_block(xs[0]), apk[0], s1h[0]);
      put_a(apk[0]);
    }
    if constexpr (DO_A) act_apply_t(zt_block(qs[0]));
    stage_rows(1);
    fetch(2);
    __syncthreads();
    for (int it = 0; it < iters; it += 2) {
      phase_a(it, std::integral_constant<int, 0>{});
      __syncthreads();
      phase_b(it, std::integral_constant<int, 0>{});
      __syncthreads();
      if (it + 1 < iters) {
        phase_a(it + 1, std::integral_constant<int, 1>{});
        __syncthreads();
        phase_b(it + 1, std::integral_constant<int, 1>{});
        __syncthreads();
      }
    }
  };
  if (my_g > 0 && my_a > 0)
    run(std::integral_constant<int, 3>{});
  else if (my_g > 0)
    run(std::integral_constant<int, 1>{});
  else if (my_a > 0)
    run(std::integral_constant<int, 2>{});

  if (gl > 0) {
    float* part = p.part;
#pragma unroll
    for (int db = 0; db < 2; ++db)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int rr = c32_row(r, hf);
        part[(32 * db + rr) * HH + hid] = gw1[db][r];
        part[DH + (32 * w + rr) * D + 32 * db + l32] = -LN2 * gw2[db][r];
      }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) lacc += __shfl_xor(lacc, m, 64);
    if (l == 0) red[w] = lacc;
    __syncthreads();
    if (tid == 0) {
      float s = 0.f;
      for (int i = 0; i < NW; ++i) s += red[i];
      *p.part_loss = s;
    }
  }
}

// Fixed-order reduction of the G shard partials of each active chain and the
// step W_{s+1} = W_s - eta * grad.  Also writes the checkpoint W_s, the final
// weights after a sequence's last chunk, and the chunk's inner loss.
//
// The shard sums of each float4 of the gradient form four streams (shards
// q, q+4, q+8, ..., with the shards past the last multiple of 4 appended to
// stream 0, in order) combined as (s0 + s1) + (s2 + s3).  SPLIT = 1: one lane
// runs the four streams.  SPLIT = 4: lane q of a quad runs stream q and the
// sums are combined through two quad exchanges, so each lane has a quarter
// of the dependent loads in flight; the additions, and the result, are the
// same.  The split pays when few chains leave most of the GPU idle.  A
// chain's float4s are spread over SPLIT x as many work-groups as float4s / 256.
template <int SPLIT>
__global__ __launch_bounds__(256) void ttt_update(UpdStepArgs p) {
  static_assert(SPLIT == 1 || SPLIT == 4, "one lane or a quad per float4");
  const int dh = D * p.h;
  const int n4 = (2 * dh) / 4;
  const int nbpc = SPLIT * ((n4 + 255) / 256);
  const int lin = xcd_linear_block();
  const int slot = lin / nbpc, k = lin % nbpc;
  const bool gcs = p.gcs_chunks > 0;
  const int ai = gcs ? 0 : slot / p.H, head = gcs ? slot : slot % p.H;
  const int gl = gcs ? 1 : p.grad_len[ai];
  if (gl <= 0) return;
  const int chain = gcs ? head : p.seq_id[ai] * p.H + head;
  const int n_ent = gcs ? p.gcs_chunks : 1;
  const int q = SPLIT == 4 ? (threadIdx.x & 3) : 0;
  const int i4 = SPLIT == 4 ? k * 64 + (threadIdx.x >> 2) : k * 256 + threadIdx.x;  // quad-uniform
  if (i4 < n4) {
    // fixed order: entries, then shards
    f32x4 s;
    if constexpr (SPLIT == 4) {
      f32x4 sq = {0.f, 0.f, 0.f, 0.f};  // stream q
      const int g4 = p.G & ~3;
      for (int e = 0; e < n_ent; ++e) {
        const int64_t sl = gcs ? (int64_t)e * p.H + head : slot;
        const f32x4* part = reinterpret_cast<const f32x4*>(p.partial + sl * p.G * 2 * dh) + i4;
        int gg = q;
        for (; gg + 28 < g4; gg += 32) {  // 8 loads in flight, added in shard order
          f32x4 v[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) v[j] = part[(int64_t)(gg + 4 * j) * n4];
#pragma unroll
          for (int j = 0; j < 8; ++j) sq += v[j];
        }
        for (; gg < g4; gg += 4) sq += part[(int64_t)gg * n4];
        if (q == 0)
          for (gg = g4; gg < p.G; ++gg) sq += part[(int64_t)gg * n4];
      }
      f32x4 t;  // lanes 0 and 2: s0 + s1 and s2 + s3
#pragma unroll
      for (int c = 0; c < 4; ++c) t[c] = sq[c] + __shfl_xor(sq[c], 1, 64);
#pragma unroll
      for (int c = 0; c < 4; ++c) s[c] = t[c] + __shfl_xor(t[c], 2, 64);  // lane 0
      if (q != 0) return;
    } else {
      f32x4 s0 = {0.f, 0.f, 0.f, 0.f}, s1 = s0, s2 = s0, s3 = s0;
      for (int e = 0; e < n_ent; ++e) {
        const int64_t sl = gcs ? (int64_t)e * p.H + head : slot;
        const f32x4* part = reinterpret_cast<const f32x4*>(p.partial + sl * p.G * 2 * dh) + i4;
        int gg = 0;
        for (; gg + 4 <= p.G; gg += 4) {
          s0 += part[(int64_t)gg * n4];
          s1 += part[(int64_t)(gg + 1) * n4];
          s2 += part[(int64_t)(gg + 2) * n4];
          s3 += part[(int64_t)(gg + 3) * n4];
        }
        for (; gg < p.G; ++gg) s0 += part[(int64_t)gg * n4];
      }
      s = (s0 + s1) + (s2 + s3);
    }
    const int idx = 4 * i4;
    bool step = true;
    if (gcs && p.gcs_acc) {  // a pass of a multi-pass sum: the running total first, then this pass
      f32x4* acc = reinterpret_cast<f32x4*>(p.gcs_acc + (int64_t)head * 2 * dh + idx);
      if (!p.gcs_first) s = *acc + s;
      if (!p.gcs_last) *acc = s;
      step = p.gcs_last != 0;
    }
    const int64_t wc = (int64_t)(chain % p.w_mod) * p.w_cstride;
    const f32x4 wv = idx < dh ? *reinterpret_cast<const f32x4*>(p.w1_src + wc + idx)
                              : *reinterpret_cast<const f32x4*>(p.w2_src + wc + (idx - dh));
    const f32x4 wn = wv - p.eta * s;
    if (step) *reinterpret_cast<f32x4*>(p.w_dst + (int64_t)chain * 2 * dh + idx) = wn;
    if (p.ckpt) *reinterpret_cast<f32x4*>(p.ckpt + p.ckpt_off[ai] + (int64_t)head * 2 * dh + idx) = wv;
    if (step && (gcs || p.is_last[ai]) && p.wT1) {
      if (idx < dh)
        *reinterpret_cast<f32x4*>(p.wT1 + (int64_t)chain * dh + idx) = wn;
      else
        *reinterpret_cast<f32x4*>(p.wT2 + (int64_t)chain * dh + (idx - dh)) = wn;
    }
  }
  if (k == 0 && threadIdx.x == 0 && p.loss) {
    for (int e = 0; e < n_ent; ++e) {
      const int64_t sl = gcs ? (int64_t)e * p.H + head : slot;
      const int len = gcs ? (e + 1 < n_ent ? p.gcs_M : p.gcs_last_len) : gl;
      float sum = 0.f;
      for (int gg = 0; gg < p.G; ++gg) sum += p.partial_loss[sl * p.G + gg];
      p.loss[(int64_t)head * p.loss_stride + (gcs ? p.gcs_entry0 + e : p.chunk)] = sum / (float)len;
    }
  }
}

// ----------------------------------------------------------------- step kernel
// One chunk step for every active chain of a launch plan (one work-group per
// (chain, token shard)); the partials are reduced by ttt_update.
template <typename IOT, int NW, bool BF>
__global__ __launch_bounds__(NW * 64) void ttt_fwd_step(FwdStepArgs p) {
  constexpr int DH = D * NW * 32;
  const int lin = xcd_linear_block();
  const int slot = lin / p.G, g = lin % p.G;
  const int ai = slot / p.H, head = slot % p.H;
  const int chain = p.seq_id[ai] * p.H + head;
  StepCtx c;
  c.Q = p.Q; c.K = p.K; c.V = p.V; c.O = p.O;
  c.stride_tok = p.stride_tok; c.stride_head = p.stride_head; c.flags = p.flags;
  c.W1 = p.w1_src + (int64_t)(chain % p.w_mod) * p.w_cstride;
  c.W2 = p.w2_src + (int64_t)(chain % p.w_mod) * p.w_cstride;
  c.head = head; c.g = g; c.G = p.G;
  c.gs = p.grad_start[ai]; c.gl = p.grad_len[ai];
  c.as0 = p.app_start[ai]; c.al = p.app_len[ai];
  c.part = p.partial + ((int64_t)slot * p.G + g) * (2 * DH);
  c.part_loss = p.partial_loss + (int64_t)slot * p.G + g;
  if constexpr (BF)
    fwd_body_bf<IOT, NW>(c);
  else
    fwd_body_f32<IOT, NW>(c);
}

// ----------------------------------------------------------------- persistent forward
// Barrier of the G work-groups of a group: every member adds one to the
// group's counter once its earlier stores are complete, and waits until the
// counter reaches `target`.  The wait polls at most spin_limit times; past
// that, or once another wait has given up, it sets bit 0 of *err and returns,
// so that no wave waits forever (the results are then invalid and the error
// word says so).
//
// Two protocols.  LOCAL (every member of the group runs on the same XCD,
// checked at run time): the members share that XCD's L2, and a store is
// visible there once it has completed (the vector L1 is write-through), so a
// member waits for its own stores (vmcnt 0, every wave), increments the
// counter, and after the wait drops its CU's L1 lines (buffer_inv sc0) so
// that its loads read the L2.  AGENT (members on several XCDs, whose L2s are
// not coherent with each other): release / acquire at agent scope, which
// writes the L2 back and invalidates it, several microseconds per barrier.
template <bool LOCAL>
__device__ __forceinline__ void group_barrier(uint32_t* ctr, uint32_t target, uint32_t* err, uint32_t spin_limit) {
  if constexpr (LOCAL) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    if constexpr (LOCAL)
      __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
      __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t n = 0;
    while (__hip_atomic_load(ctr, LOCAL ? __ATOMIC_RELAXED : __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      ++n;
      if (n > spin_limit ||
          ((n & 255u) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)) {
        __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    if constexpr (LOCAL) asm volatile("buffer_inv sc0\n\ts_waitcnt vmcnt(0)" ::: "memory");
  }
  __syncthreads();
}
__device__ __forceinline__ void group_barrier(bool local, uint32_t* ctr, uint32_t target, uint32_t* err,
                                              uint32_t spin_limit) {
  if (local)
    group_barrier<true>(ctr, target, err, spin_limit);
  else
    group_barrier<false>(ctr, target, err, spin_limit);
}

// Slice g of G of the chain's step: W_{s+1} = W_s - eta * (sum of the G shard
// partials, in the fixed order of ttt_update: four streams of shards q, q+4,
// ... combined as (s0 + s1) + (s2 + s3)); also the checkpoint row (W_s), the
// final weights after the last chunk and, by member 0, the chunk's loss.
template <int NT, int DH, typename PA>
__device__ __forceinline__ void group_reduce(const PA& p, int g, const float* part, const float* ploss,
                                             const float* w1s, const float* w2s, float* wdst, float* ck, float* t1,
                                             float* t2, int head, int s, int gl) {
  constexpr int n4 = 2 * DH / 4;
  const int G = p.G;
  const int lo = (int)((int64_t)g * n4 / G), hi = (int)((int64_t)(g + 1) * n4 / G);
  for (int i4 = lo + (int)threadIdx.x; i4 < hi; i4 += NT) {
    const f32x4* pp = reinterpret_cast<const f32x4*>(part) + i4;
    f32x4 s0 = {0.f, 0.f, 0.f, 0.f}, s1 = s0, s2 = s0, s3 = s0;
    int gg = 0;
    for (; gg + 4 <= G; gg += 4) {
      s0 += pp[(int64_t)gg * n4];
      s1 += pp[(int64_t)(gg + 1) * n4];
      s2 += pp[(int64_t)(gg + 2) * n4];
      s3 += pp[(int64_t)(gg + 3) * n4];
    }
    for (; gg < G; ++gg) s0 += pp[(int64_t)gg * n4];
    const f32x4 sum = (s0 + s1) + (s2 + s3);
    const int idx = 4 * i4;
    const f32x4 wv = idx < DH ? *reinterpret_cast<const f32x4*>(w1s + idx)
                              : *reinterpret_cast<const f32x4*>(w2s + (idx - DH));
    const f32x4 wn = wv - p.eta * sum;
    *reinterpret_cast<f32x4*>(wdst + idx) = wn;
    if (ck) *reinterpret_cast<f32x4*>(ck + idx) = wv;
    if (t1) {
      if (idx < DH)
        *reinterpret_cast<f32x4*>(t1 + idx) = wn;
      else
        *reinterpret_cast<f32x4*>(t2 + (idx - DH)) = wn;
    }
  }
  if (g == 0 && threadIdx.x == 0 && p.loss) {
    float sum = 0.f;
    for (int gg = 0; gg < G; ++gg) sum += ploss[gg];
    p.loss[(int64_t)head * p.loss_stride + s] = sum / (float)gl;
  }
}

template <typename IOT, int NW, bool BF>
__global__ __launch_bounds__(NW * 64) void ttt_fwd_persist(PersistArgs p) {
  constexpr int NT = NW * 64;
  constexpr int DH = D * NW * 32;
  // Loop state lives in LDS and is re-read (volatile) after every step body,
  // so that none of it occupies registers while the body runs: the body uses
  // the whole register budget of two waves per SIMD.
  __shared__ int st_[6];  // chain entry, step, barrier count, chunks of the chain, LOCAL protocol, member
  volatile int* st = st_;
  // Inside the loops the arguments are read through a pointer to the kernel
  // argument segment that the compiler cannot see through, so each step
  // re-reads them with scalar loads instead of keeping them in scalar
  // registers across the step body (which spilled them into vector
  // registers).  p (the first argument) starts the segment.
  typedef const __attribute__((address_space(4))) PersistArgs* KP;
  auto kargs = []() -> KP {
    KP k = (KP)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(k));
    return k;
  };
  {
    const int nb = gridDim.x, bid = blockIdx.x;
    const int lin = p.xcd_map ? (bid % 8) * (nb / 8) + bid / 8 : bid;
    if (lin / p.G >= p.n_groups) return;
    if (threadIdx.x == 0) st[5] = lin;
    // every member records its XCD; the first barrier (agent protocol)
    // publishes the group's set, and the LOCAL protocol is used from then on
    // iff it is a single XCD
    if (threadIdx.x == 0) {
      const uint32_t xcc = __builtin_amdgcn_s_getreg((3 << 11) | 20) & 15u;  // HW_REG_XCC_ID[3:0]
      __hip_atomic_fetch_or(p.xcds + lin / p.G, 1u << xcc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      st[2] = 1;
    }
    group_barrier<false>(p.bar + lin / p.G, (uint32_t)p.G, p.err, p.spin_limit);
    if (threadIdx.x == 0) {
      const uint32_t m = __hip_atomic_load(p.xcds + lin / p.G, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      st[4] = (m & (m - 1u)) == 0u ? 1 : 0;
    }
    __syncthreads();
  }
  for (;;) {
    KP q = kargs();
    {
        const int lin = __builtin_amdgcn_readfirstlane(st[5]);
      const int grp = lin / q->G, g = lin % q->G;
      // the group's member 0 takes the next chain; the barrier publishes it
      if (g == 0 && threadIdx.x == 0) {
        const uint32_t c = __hip_atomic_fetch_add(q->next, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(q->slot + grp, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      __syncthreads();
      const uint32_t nbar = (uint32_t)__builtin_amdgcn_readfirstlane(st[2]) + 1u;
      group_barrier(st[4] != 0, q->bar + grp, nbar * (uint32_t)q->G, q->err, q->spin_limit);
      if (threadIdx.x == 0) {
        st[2] = (int)nbar;
        const int c = (int)__hip_atomic_load(q->slot + grp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        st[0] = c;
        st[1] = 0;
        if (c < q->n_chains) {
          const int64_t N = q->seq_len[c / q->H];
          st[3] = (int)((N + q->M - 1) / q->M);
        }
      }
      __syncthreads();
      if (__builtin_amdgcn_readfirstlane(st[0]) >= q->n_chains) break;
    }
    for (;;) {
      KP q = kargs();
        const int c = __builtin_amdgcn_readfirstlane(st[0]), s = __builtin_amdgcn_readfirstlane(st[1]),
                C = __builtin_amdgcn_readfirstlane(st[3]);
      if (s > C) break;
      const int lin = __builtin_amdgcn_readfirstlane(st[5]);
      const int grp = lin / q->G, g = lin % q->G;
      float* const wb = q->wbuf + (int64_t)grp * 2 * (2 * DH);
      float* const part = q->partial + (int64_t)grp * q->G * (2 * DH);
      float* const ploss = q->partial_loss + (int64_t)grp * q->G;
      const int e = c / q->H, head = c % q->H, b = q->seq_id[e];
      const int64_t N = q->seq_len[e], start = q->seq_start[e], M = q->M;
      const int64_t w0 = ((int64_t)(q->w0_per_seq ? b * q->H : 0) + head) * DH;
      const float* w1s = s == 0 ? q->w1_0 + w0 : wb + (s & 1) * (2 * DH);
      const float* w2s = s == 0 ? q->w2_0 + w0 : wb + (s & 1) * (2 * DH) + DH;
      const int gl = s < C ? (int32_t)min(M, N - (int64_t)s * M) : 0;
      {
        StepCtx x;
        x.Q = q->Q; x.K = q->K; x.V = q->V; x.O = q->O;
        x.stride_tok = q->stride_tok; x.stride_head = q->stride_head; x.flags = q->flags;
        x.W1 = w1s; x.W2 = w2s;
        x.head = head; x.g = g; x.G = q->G;
        x.gs = start + (int64_t)s * M;
        x.gl = gl;
        x.as0 = start + (int64_t)(s - 1) * M;
        x.al = s >= 1 ? (int32_t)min(M, N - (int64_t)(s - 1) * M) : 0;
        x.part = part + (int64_t)g * (2 * DH);
        x.part_loss = ploss + g;
        if constexpr (BF)
          fwd_body_bf<IOT, NW, true>(x);
        else
          fwd_body_f32<IOT, NW, true>(x);
      }
      __syncthreads();
      // everything the reduction needs is re-read here, so that nothing
      // computed before the step body stays live through it
      const int ss = __builtin_amdgcn_readfirstlane(st[1]), CC = __builtin_amdgcn_readfirstlane(st[3]);
      if (ss < CC) {
            const int cc = __builtin_amdgcn_readfirstlane(st[0]);
        const uint32_t nbar = (uint32_t)__builtin_amdgcn_readfirstlane(st[2]);
        const int lin = __builtin_amdgcn_readfirstlane(st[5]);
        const int grp = lin / q->G, g = lin % q->G;
        float* const wb = q->wbuf + (int64_t)grp * 2 * (2 * DH);
        float* const part = q->partial + (int64_t)grp * q->G * (2 * DH);
        float* const ploss = q->partial_loss + (int64_t)grp * q->G;
        const int ee = cc / q->H, hh = cc % q->H, bb = q->seq_id[ee];
        const int64_t NN = q->seq_len[ee], MM = q->M;
        const int gll = (int32_t)min(MM, NN - (int64_t)ss * MM);
        const int64_t w00 = ((int64_t)(q->w0_per_seq ? bb * q->H : 0) + hh) * DH;
        const float* w1r = ss == 0 ? q->w1_0 + w00 : wb + (ss & 1) * (2 * DH);
        const float* w2r = ss == 0 ? q->w2_0 + w00 : wb + (ss & 1) * (2 * DH) + DH;
        const bool local = st[4] != 0;
        group_barrier(local, q->bar + grp, (nbar + 1u) * (uint32_t)q->G, q->err, q->spin_limit);
        const bool last = ss == CC - 1;
        const int64_t chain = (int64_t)bb * q->H + hh;
        float* ck = q->ckpt ? q->ckpt + ((q->ck_row[ee] + ss) * q->H + hh) * (2 * DH) : nullptr;
        float* t1 = last && q->wT1 ? q->wT1 + chain * DH : nullptr;
        float* t2 = last && q->wT1 ? q->wT2 + chain * DH : nullptr;
        group_reduce<NT, DH>(p, g, part, ploss, w1r, w2r, wb + ((ss + 1) & 1) * (2 * DH), ck, t1, t2, hh, ss, gll);
        group_barrier(local, q->bar + grp, (nbar + 2u) * (uint32_t)q->G, q->err, q->spin_limit);
        if (threadIdx.x == 0) st[2] = (int)(nbar + 2u);
      }
      if (threadIdx.x == 0) st[1] = ss + 1;
      __syncthreads();
    }
  }
}

// Zero n words (the persistent forward's counters and error word).
__global__ void ttt_zero_words(uint32_t* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// ----------------------------------------------------------------- launchers
template <typename IOT, bool BF, int NW>
static hipError_t launch_fwd_step_t(const FwdStepArgs& a, int n_blocks, hipStream_t st) {
  hipLaunchKernelGGL((ttt_fwd_step<IOT, NW, BF>), dim3(n_blocks), dim3(NW * 64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fwd_step(const FwdStepArgs& a, int n_blocks, int h, bool io_bf16, bool mma_bf16, hipStream_t st) {
  if (h == 128) {
    if (io_bf16) return launch_fwd_step_t<bf16, true, 4>(a, n_blocks, st);
    return mma_bf16 ? launch_fwd_step_t<float, true, 4>(a, n_blocks, st)
                    : launch_fwd_step_t<float, false, 4>(a, n_blocks, st);
  }
  if (io_bf16) return launch_fwd_step_t<bf16, true, 8>(a, n_blocks, st);
  return mma_bf16 ? launch_fwd_step_t<float, true, 8>(a, n_blocks, st)
                  : launch_fwd_step_t<float, false, 8>(a, n_blocks, st);
}

hipError_t launch_update(const UpdStepArgs& a, int n_blocks, hipStream_t st) {
  // n_blocks = active chains x float4s / 256; below one work-group per CU
  // the quad split spreads the reduction over four times as many
  if (n_blocks < 256)
    hipLaunchKernelGGL(ttt_update<4>, dim3(4 * n_blocks), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(ttt_update<1>, dim3(n_blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// Persistent forward: the kernel instance for (h, io type, operand type).
template <typename F>
static auto with_persist_kernel(int h, bool io_bf16, bool mma_bf16, F&& f) {
  if (h == 128) {
    if (io_bf16) return f(ttt_fwd_persist<bf16, 4, true>, 4);
    return mma_bf16 ? f(ttt_fwd_persist<float, 4, true>, 4) : f(ttt_fwd_persist<float, 4, false>, 4);
  }
  if (io_bf16) return f(ttt_fwd_persist<bf16, 8, true>, 8);
  return mma_bf16 ? f(ttt_fwd_persist<float, 8, true>, 8) : f(ttt_fwd_persist<float, 8, false>, 8);
}

hipError_t persist_occupancy(int h, bool io_bf16, bool mma_bf16, int* blocks_per_cu, int* threads) {
  return with_persist_kernel(h, io_bf16, mma_bf16, [&](auto kern, int nw) {
    *threads = nw * 64;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, kern, nw * 64, 0);
  });
}

hipError_t launch_fwd_persist(const PersistArgs& a, int n_blocks, int h, bool io_bf16, bool mma_bf16,
                              hipStream_t st) {
  return with_persist_kernel(h, io_bf16, mma_bf16, [&](auto kern, int nw) {
    hipLaunchKernelGGL(kern, dim3(n_blocks), dim3(nw * 64), 0, st, a);
    return hipGetLastError();
  });
}

hipError_t launch_zero_words(uint32_t* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(ttt_zero_words, dim3(1), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace ttt
