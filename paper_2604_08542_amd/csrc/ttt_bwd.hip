// Backward kernels of the chunked TTT chain: reverse mode through every
// inner update, second-order terms through the inner gradient included, for
// the outer loss sum <O, dO> (the forward is Sec. 4.2 Eq. 8 and Sec. 3.2
// Eq. 3-4).
//
// Chunks are walked backwards.  With Wh the adjoint of W_{s+1} and W = W_s
// recomputed from the checkpoint, one launch of ttt_bwd_step handles, per
// token shard of every head:
//   - the update adjoint of chunk s (recompute Z, A, E, P, D; then
//       deta += -<K Wh1, D> - <A Wh2, E>,  dD = -eta K Wh1,
//       dA = -eta E Wh2^T + dY W2^T,  dE = -eta A Wh2 + dP W2,
//       dP = dD s'(Z),  dZ = dD P s''(Z) + dA s'(Z),  dY = (2/M) dE,
//       dV = -dY,  dK = -eta D Wh1^T + dZ W1^T,
//       token sums  dP^T E + A^T dY  and  K^T dZ),
//   - the apply adjoint of chunk s-1, whose output used W_s
//       (dZq = (dO W2^T) s'(Zq), token sums Aq^T dO and Q^T dZq,
//        dQ = dZq W1^T),
// and ttt_bwd_reduce adds the shard sums, in a fixed order, to Wh, giving the
// adjoint of W_s.  The L2-normalisation adjoint maps dQ, dK, dV to the raw
// inputs.
//
// Layout inside a work-group follows the forward kernel: wave w owns hidden
// units [32w, 32w+32) for the products whose result has a hidden axis
// (32x32 blocks with tokens in registers, which also feed the token-sum
// products directly); products contracting the hidden axis read staged
// [token][hidden] tiles from LDS as 16x16 blocks.  This first backward reads
// its weight operands straight from memory (they are L2-resident per chain)
// instead of keeping four weight matrices on chip.
#include <hip/hip_runtime.h>

#include "ttt_common.h"
#include "ttt_internal.h"

namespace ttt {

// Hides a (wave-uniform) pointer's value from the optimiser so that loads
// through it are not hoisted out of the token loop into registers.
template <typename T>
__device__ __forceinline__ T* opaque(T* ptr) {
  asm volatile("" : "+v"(ptr));
  return ptr;
}

#ifndef BWD_F32_NW256
#define BWD_F32_NW256 8
#endif

template <typename IOT, int NW, int NB>
__global__ __launch_bounds__(NW * 64) void ttt_bwd_step(BwdStepArgs p) {
  constexpr int HH = NW * 32 * NB;  // hidden size: NW waves x NB 32-wide blocks each
  constexpr int NT = NW * 64;
  constexpr int EPT = D * TT / NT;
  constexpr int TPR = D / EPT;
  constexpr int DH = D * HH;
  constexpr int LD = D + 4;  // f32 [token][d] tiles
  using MT = float;  // FP32 operands (BF16 operands: ttt_bwd_step_bf)
  constexpr int AS_LD = HH + 4;

  __shared__ __attribute__((aligned(16))) float xs[TT * LD];    // K or Q rows (normalised)
  __shared__ __attribute__((aligned(16))) float vs[TT * LD];    // V rows (normalised)
  __shared__ __attribute__((aligned(16))) float es[TT * LD];    // E
  __shared__ __attribute__((aligned(16))) float des[TT * LD];   // -eta A Wh2, then dE
  __shared__ __attribute__((aligned(16))) float dys[TT * LD];   // dY, or dO rows for apply tiles
  __shared__ __attribute__((aligned(16))) float dxs[TT * LD];   // dK or dQ before the norm adjoint
  __shared__ __attribute__((aligned(16))) MT sta[TT * AS_LD];   // staged A, then D, or dZq
  __shared__ __attribute__((aligned(16))) MT stb[TT * AS_LD];   // staged dP, then dZ
  __shared__ float ninv[2][TT];   // 1 / max(||x||, eps) of the two staged row sets
  __shared__ int nabove[2][TT];   // ||x|| > eps
  __shared__ float red[NW];

  // Lane-derived indices live in `li`, recomputed from an opaque thread id at
  // the top of every tile iteration: the kernel's LDS exceeds the 64 KiB reach
  // of LDS immediate offsets, and hoisting every per-lane address out of the
  // token loop would otherwise exhaust the register file.
  struct LaneIds {
    int tid, w, l, l32, hf, l16, g4, hid0, row, col0;
  };
  auto lane_ids = [](int t) {
    LaneIds r;
    r.tid = t; r.w = t >> 6; r.l = t & 63; r.l32 = t & 31; r.hf = (t & 63) >> 5; r.l16 = t & 15;
    r.g4 = (t & 63) >> 4; r.hid0 = r.w * 32 * NB + r.l32; r.row = t / TPR; r.col0 = (t % TPR) * EPT;
    return r;
  };
  LaneIds li = lane_ids(threadIdx.x);
  auto refresh = [&]() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    li = lane_ids(t);
  };
  const int lin = xcd_linear_block();
  const int G = p.G;
  const int slot = lin / G, g = lin % G;  // slot = active sequence * H + head
  const int ai = slot / p.H, head = slot % p.H;
  const float eta = p.eta;
  // prepared operand block of this head: 8 matrices of D*h elements
  const MT* prep0 = static_cast<const MT*>(p.prep) + (int64_t)slot * 8 * DH;
  // Operand fragments by buffer loads: one descriptor for the 8 prepared
  // matrices of this head, matrix offsets in scalar registers.
  const __amdgpu_buffer_rsrc_t prsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<MT*>(prep0), (short)0, (int)(8 * DH * sizeof(MT)), 0x00020000);
  auto bload = [&](int voff, int soff) {
    return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(prsrc, voff, soff, 0));
  };
  const int64_t hoff = (int64_t)head * p.stride_head;
  const bool norm_q = p.flags & 1u, norm_k = p.flags & 2u, norm_v = p.flags & 4u;

  // ---- operand helpers
  // The prepared operand copies of W_s and of the carried adjoint (see
  // ttt_bwd_prep) are [hid][d] or [d][hid] matrices in the operand type.
  // 32x32 block C[tok][hid] (hidden block j of this wave) = X[tok][:] F with
  // F(d, hid) = M[hid][d].
  auto th = [&](const float* X, int k, int j) {
    f32x16 c = {};
    const int voff = (int)(((li.hid0 + 32 * j) * D) * sizeof(MT));
#pragma unroll 2
    for (int s4 = 0; s4 < 8; ++s4) {
      const int d0 = 32 * li.hf + 4 * s4;
      const f32x4 x = *reinterpret_cast<const f32x4*>(&X[li.l32 * LD + d0]);
      const f32x4 b = bload(voff + 128 * li.hf, k * DH * 4 + 16 * s4);
#pragma unroll
      for (int e = 0; e < 4; ++e) c = mma32(x[e], b[e], c);
    }
    __builtin_amdgcn_sched_barrier(0);
    return c;
  };
  // 16x16 block C[tok][d] (token block tb, feature block db) = S[tok][:] F,
  // S staged [tok][hidden] in LDS, F(hid, d) = M[d][hid].
  auto td = [&](const MT* S, int tb, int db, int k) {
    f32x4 c = {};
    const int arow = 16 * tb + li.l16, dcol = 16 * db + li.l16;
    const int voff = (int)((dcol * HH + (HH / 4) * li.g4) * sizeof(MT));
#pragma unroll 2
    for (int u = 0; u < HH / 16; ++u) {
      const int k0 = (HH / 4) * li.g4 + 4 * u;
      const f32x4 a = *reinterpret_cast<const f32x4*>(&S[arow * AS_LD + k0]);
      const f32x4 b = bload(voff, k * DH * 4 + 16 * u);
#pragma unroll
      for (int e = 0; e < 4; ++e) c = mma16(a[e], b[e], c);
    }
    __builtin_amdgcn_sched_barrier(0);
    return c;
  };
  // gW1[j][db] (rows d, cols hidden block j) += X[:, d]^T Yw ;
  // gW2[j][db] (rows hidden block j, cols d) += Yw^T X[:, d]
  auto tok_sum_w1 = [&](f32x16 (&acc)[2], const float* X, const f32x16& Yw) {
#pragma unroll
    for (int db = 0; db < 2; ++db) {
      const int dd = 32 * db + li.l32;
#pragma unroll
      for (int s = 0; s < 16; ++s) acc[db] = mma32(X[c32_row(s, li.hf) * LD + dd], Yw[s], acc[db]);
    }
  };
  auto tok_sum_w2 = [&](f32x16 (&acc)[2], const f32x16& Yw, const float* X) {
#pragma unroll
    for (int db = 0; db < 2; ++db) {
      const int dd = 32 * db + li.l32;
#pragma unroll
      for (int s = 0; s < 16; ++s) acc[db] = mma32(Yw[s], X[c32_row(s, li.hf) * LD + dd], acc[db]);
    }
  };
  auto stage = [&](MT* S, const f32x16& Yw, int j) {
#pragma unroll
    for (int r = 0; r < 16; ++r) S[c32_row(r, li.hf) * AS_LD + li.hid0 + 32 * j] = (MT)Yw[r];
  };
  // Load rows of a token tensor for tokens [t0, t0+nv) into an LDS tile,
  // optionally L2-normalised (recording the norm data in set ns).
  auto load_rows = [&](const void* base, int64_t t0, int nv, float* dst, bool do_norm, int ns) {
    float x[EPT];
    const bool valid = li.row < nv;
    if (valid) {
      load_vec<IOT, EPT>(static_cast<const IOT*>(base) + (t0 + li.row) * p.stride_tok + hoff + li.col0, x);
    } else {
#pragma unroll
      for (int i = 0; i < EPT; ++i) x[i] = 0.f;
    }
    if (do_norm) {
      float ss = 0.f;
#pragma unroll
      for (int i = 0; i < EPT; ++i) ss = fmaf(x[i], x[i], ss);
      ss = lane_group_sum<TPR>(ss);
      const float nrm = sqrtf(ss);
      const float inv = 1.0f / fmaxf(nrm, NORM_EPS);
#pragma unroll
      for (int i = 0; i < EPT; ++i) x[i] *= inv;
      if (ns >= 0 && (li.tid % TPR) == 0) {
        ninv[ns][li.row] = inv;
        nabove[ns][li.row] = nrm > NORM_EPS;
      }
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) dst[li.row * LD + li.col0 + i] = x[i];
  };
  // Write dx~ = norm adjoint of dx (rows in LDS) for tokens [t0, t0+nv).
  auto store_grad_rows = [&](void* base, int64_t t0, int nv, const float* dx, const float* xhat, bool did_norm,
                             int ns, float sign) {
    float v[EPT], xh[EPT];
    float dot = 0.f;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      v[i] = sign * dx[li.row * LD + li.col0 + i];
      xh[i] = xhat[li.row * LD + li.col0 + i];
      dot = fmaf(v[i], xh[i], dot);
    }
    if (did_norm) {
      dot = lane_group_sum<TPR>(dot);
      const float inv = ninv[ns][li.row];
      const bool above = nabove[ns][li.row];
#pragma unroll
      for (int i = 0; i < EPT; ++i) v[i] = above ? (v[i] - xh[i] * dot) * inv : v[i] * inv;
    }
    if (li.row < nv) store_vec<IOT, EPT>(static_cast<IOT*>(base) + (t0 + li.row) * p.stride_tok + hoff + li.col0, v);
  };

  f32x16 gw1[NB][2] = {}, gw2[NB][2] = {};
  float deta_acc = 0.f;

  // ------------------------------------------------ update adjoint of chunk s
  const int gl = p.grad_len[ai];
  const int64_t grad_start = p.grad_start[ai];
  const int n_gt = (gl + TT - 1) / TT;
  const float e_scale = gl > 0 ? 2.0f / (float)gl : 0.f;
  for (int t = g; t < n_gt; t += G) {
    const int64_t t0 = grad_start + (int64_t)t * TT;
    const int nv = min(TT, gl - t * TT);
    // prepared operand indices: [hid][d] of W1, W2, Wh1, Wh2, then [d][hid] of the same
    constexpr int W1t = 0, W2n = 1, H1t = 2, H2n = 3, W1n = 4, W2t = 5, H1n = 6, H2t = 7;
    refresh();
    load_rows(p.K, t0, nv, xs, norm_k, 0);
    load_rows(p.V, t0, nv, vs, norm_v, 1);
    __syncthreads();
    // Z = K W1 is kept; A, s'(Z), s''(Z) are recomputed from it where needed.
    f32x16 Z[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      Z[j] = th(xs, W1t, j);
      f32x16 A;
#pragma unroll
      for (int r = 0; r < 16; ++r) A[r] = Z[j][r] * sigmoid(Z[j][r]);
      stage(sta, A, j);
    }
    __syncthreads();
    // Y = A W2 -> E;  A Wh2 -> -eta A Wh2 and its deta term
#pragma unroll
    for (int bi = 0; bi < 8 / NW; ++bi) {
      const int b = li.w + NW * bi, tb = b & 1, db = b >> 1;
      const f32x4 y = td(sta, tb, db, W2t);
      const f32x4 aw = td(sta, tb, db, H2t);
      const int dcol = 16 * db + li.l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int tok = 16 * tb + 4 * li.g4 + r;
        const float E = e_scale * (y[r] - vs[tok * LD + dcol]);
        es[tok * LD + dcol] = E;
        des[tok * LD + dcol] = -eta * aw[r];
        deta_acc -= aw[r] * E;
      }
    }
    __syncthreads();
    // P = E W2^T, D = P s'(Z) (staged), K Wh1 -> dD and its deta term,
    // dP = dD s'(Z) (staged), dZ = dD P s''(Z)
    f32x16 dP[NB], dZ[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const f32x16 P = th(es, W2n, j);
      const f32x16 KW = th(xs, H1t, j);
      f32x16 Dm;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float z = Z[j][r];
        const float sg = sigmoid(z);
        const float a = z * sg;
        const float s1 = fmaf(a, 1.0f - sg, sg);
        const float s2 = sg * (1.0f - sg) * fmaf(z, 1.0f - 2.0f * sg, 2.0f);
        Dm[r] = P[r] * s1;
        deta_acc -= KW[r] * Dm[r];
        const float dD = -eta * KW[r];
        dP[j][r] = dD * s1;
        dZ[j][r] = dD * P[r] * s2;
      }
      stage(sta, Dm, j);
      stage(stb, dP[j], j);
    }
    __syncthreads();
    // dE = -eta A Wh2 + dP W2 ; dY = (2/M) dE
#pragma unroll
    for (int bi = 0; bi < 8 / NW; ++bi) {
      const int b = li.w + NW * bi, tb = b & 1, db = b >> 1;
      const f32x4 de = td(stb, tb, db, W2t);
      const int dcol = 16 * db + li.l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int tok = 16 * tb + 4 * li.g4 + r;
        dys[tok * LD + dcol] = e_scale * (des[tok * LD + dcol] + de[r]);
      }
    }
    __syncthreads();
    // dA = -eta E Wh2^T + dY W2^T ; dZ += dA s'(Z) ; token sums
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const f32x16 dA1 = th(es, H2n, j);
      const f32x16 dA2 = th(dys, W2n, j);
      f32x16 A;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float z = Z[j][r];
        const float sg = sigmoid(z);
        const float a = z * sg;
        A[r] = a;
        dZ[j][r] += (-eta * dA1[r] + dA2[r]) * fmaf(a, 1.0f - sg, sg);
      }
      tok_sum_w2(gw2[j], A, dys);
      tok_sum_w2(gw2[j], dP[j], es);
      tok_sum_w1(gw1[j], xs, dZ[j]);
      stage(stb, dZ[j], j);
    }
    __syncthreads();
    // dK = -eta D Wh1^T + dZ W1^T
#pragma unroll
    for (int bi = 0; bi < 8 / NW; ++bi) {
      const int b = li.w + NW * bi, tb = b & 1, db = b >> 1;
      const f32x4 k1 = td(sta, tb, db, H1n);
      const f32x4 k2 = td(stb, tb, db, W1n);
      const int dcol = 16 * db + li.l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) dxs[(16 * tb + 4 * li.g4 + r) * LD + dcol] = -eta * k1[r] + k2[r];
    }
    __syncthreads();
    store_grad_rows(p.dK, t0, nv, dxs, xs, norm_k, 0, 1.0f);
    store_grad_rows(p.dV, t0, nv, dys, vs, norm_v, 1, -1.0f);
    __syncthreads();
  }

  // ------------------------------------------------ apply adjoint of chunk s-1
  const int al = p.app_len[ai];
  const int64_t app_start = p.app_start[ai];
  const int n_at = (al + TT - 1) / TT;
  for (int t = g; t < n_at; t += G) {
    const int64_t t0 = app_start + (int64_t)t * TT;
    const int nv = min(TT, al - t * TT);
    constexpr int W1t = 0, W2n = 1, W1n = 4;
    refresh();
    load_rows(p.Q, t0, nv, xs, norm_q, 0);
    load_rows(p.dO, t0, nv, dys, false, -1);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      f32x16 Aq = th(xs, W1t, j);
      f32x16 dZq = th(dys, W2n, j);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float z = Aq[r];
        const float sg = sigmoid(z);
        const float a = z * sg;
        dZq[r] *= fmaf(a, 1.0f - sg, sg);
        Aq[r] = a;
      }
      tok_sum_w2(gw2[j], Aq, dys);
      tok_sum_w1(gw1[j], xs, dZq);
      stage(sta, dZq, j);
    }
    __syncthreads();
#pragma unroll
    for (int bi = 0; bi < 8 / NW; ++bi) {
      const int b = li.w + NW * bi, tb = b & 1, db = b >> 1;
      const f32x4 q1 = td(sta, tb, db, W1n);
      const int dcol = 16 * db + li.l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) dxs[(16 * tb + 4 * li.g4 + r) * LD + dcol] = q1[r];
    }
    __syncthreads();
    store_grad_rows(p.dQ, t0, nv, dxs, xs, norm_q, 0, 1.0f);
    __syncthreads();
  }

  // ------------------------------------------------ shard partials
  float* part = p.partial + ((int64_t)slot * G + g) * (2 * DH);
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int db = 0; db < 2; ++db)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int rr = c32_row(r, li.hf);
        part[(32 * db + rr) * HH + li.hid0 + 32 * j] = gw1[j][db][r];
        part[DH + ((li.w * NB + j) * 32 + rr) * D + 32 * db + li.l32] = gw2[j][db][r];
      }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) deta_acc += __shfl_xor(deta_acc, m, 64);
  if (li.l == 0) red[li.w] = deta_acc;
  __syncthreads();
  if (li.tid == 0) {
    float s = 0.f;
    for (int i = 0; i < NW; ++i) s += red[i];
    p.partial_deta[(int64_t)slot * G + g] = s;
  }
}

// Operand copies for one backward step, per (active sequence, head): W_s and
// the carried adjoint Wh (zeros when absent), each of W1 [d][h] and W2 [h][d]
// written in both orientations ([hid][d] and [d][hid]) in the matrix-core
// operand type, so that every operand fragment is one contiguous vector load.
template <typename MT>
__global__ __launch_bounds__(256) void ttt_bwd_prep(BwdPrepArgs p) {
  const int dh = D * p.h;
  const int chain = blockIdx.y;  // active sequence * H + head
  const int ai = chain / p.H, head = chain % p.H;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= dh) return;
  const float* W = p.w_src[ai] + (int64_t)head * 2 * dh;
  const float* Wh = p.wh_src[ai] ? p.wh_src[ai] + (int64_t)head * 2 * dh : nullptr;
  MT* o = static_cast<MT*>(p.prep) + (int64_t)chain * 8 * dh;
  const int h = p.h;
  const int d = idx / h, hh = idx % h;    // idx = d*h + hh: W1 element (d, hh)
  const int hh2 = idx / D, d2 = idx % D;  // idx = hh2*D + d2: W2 element (hh2, d2)
  const float w1 = W[idx], h1 = Wh ? Wh[idx] : 0.f;
  const float w2 = W[dh + idx], h2 = Wh ? Wh[dh + idx] : 0.f;
  o[0 * dh + hh * D + d] = (MT)w1;     // W1 as [hid][d]
  o[1 * dh + idx] = (MT)w2;            // W2 as [hid][d]
  o[2 * dh + hh * D + d] = (MT)h1;
  o[3 * dh + idx] = (MT)h2;
  o[4 * dh + idx] = (MT)w1;            // W1 as [d][hid]
  o[5 * dh + d2 * h + hh2] = (MT)w2;   // W2 as [d][hid]
  o[6 * dh + idx] = (MT)h1;
  o[7 * dh + d2 * h + hh2] = (MT)h2;
}

hipError_t launch_bwd_prep(const BwdPrepArgs& a, int n_active, bool mma_bf16, hipStream_t st) {
  const dim3 grid((D * a.h + 255) / 256, n_active * a.H);
  if (mma_bf16)
    hipLaunchKernelGGL(ttt_bwd_prep<bf16>, grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(ttt_bwd_prep<float>, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

// Four consecutive elements idx..idx+3 of one chain's [W1 | W2] (W) and of
// its adjoint (Wh) into the 8 operand matrices of ttt_bwd_prep.
template <typename MT>
__device__ __forceinline__ void prep_scatter4(MT* o, int idx, int dh, int h, const f32x4& w, const f32x4& wh) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int ie = idx + e;
    if (ie < dh) {
      const int d = ie / h, hh = ie % h;
      o[0 * dh + hh * D + d] = (MT)w[e];
      o[4 * dh + ie] = (MT)w[e];
      o[2 * dh + hh * D + d] = (MT)wh[e];
      o[6 * dh + ie] = (MT)wh[e];
    } else {
      const int i2 = ie - dh, hh2 = i2 / D, d2 = i2 % D;
      o[1 * dh + i2] = (MT)w[e];
      o[5 * dh + d2 * h + hh2] = (MT)w[e];
      o[3 * dh + i2] = (MT)wh[e];
      o[7 * dh + d2 * h + hh2] = (MT)wh[e];
    }
  }
}

// Per (active sequence, head): Wh_dst = Wh_src (0 if null) + the sum of the
// G shard partials, in fixed order; deta[head] (+)= the sum of the dη
// partials.  dst may be split into W1 / W2 destinations (the final dW1_0 /
// dW2_0 of that sequence).
__global__ __launch_bounds__(256) void ttt_bwd_reduce(BwdReduceArgs p) {
  const int dh = D * p.h;
  const int n4 = (2 * dh) / 4;
  const int nbpc = (n4 + 255) / 256;
  const int lin = xcd_linear_block();
  const int chain = lin / nbpc, k = lin % nbpc;
  const int ai = chain / p.H, head = chain % p.H;
  const int b = p.seq[ai];
  const bool final = p.flags[ai] & 1, first = p.flags[ai] & 2;
  const int64_t cw = ((int64_t)b * p.H + head) * 2 * dh;  // this chain in the adjoint buffers
  const int i4 = k * 256 + threadIdx.x;
  if (i4 < n4) {
    const int idx = 4 * i4;
    f32x4 s = {0.f, 0.f, 0.f, 0.f};
    if (p.wh_src_base) s = *reinterpret_cast<const f32x4*>(p.wh_src_base + cw + idx);
    const f32x4* part = reinterpret_cast<const f32x4*>(p.partial + (int64_t)chain * p.G * 2 * dh) + i4;
    s = add_shards(s, part, n4, p.G);
    if (final && !p.fin_base) {
      const int64_t fo = ((int64_t)(p.dst_per_seq ? b : 0) * p.H + head) * dh;
      if (idx < dh)
        *reinterpret_cast<f32x4*>(p.dst1 + fo + idx) = s;
      else
        *reinterpret_cast<f32x4*>(p.dst2 + fo + (idx - dh)) = s;
    } else {
      *reinterpret_cast<f32x4*>((final ? p.fin_base : p.wh_dst_base) + cw + idx) = s;
    }
    if (p.prep_next && p.next_slot[ai] >= 0) {
      const int64_t pc = ((int64_t)p.next_slot[ai] * p.H + head) * 8 * dh;
      const f32x4 wv =
          *reinterpret_cast<const f32x4*>(p.ckpt + (p.ckpt_row[ai] * p.H + head) * 2 * dh + idx);
      if (p.prep_bf16)
        prep_scatter4(static_cast<bf16*>(p.prep_next) + pc, idx, dh, p.h, wv, s);
      else
        prep_scatter4(static_cast<float*>(p.prep_next) + pc, idx, dh, p.h, wv, s);
    }
  }
  if (k == 0 && threadIdx.x == 0) {
    float* dt = p.deta_base + (int64_t)b * p.H + head;
    float sd = first ? 0.f : *dt;
    for (int gg = 0; gg < p.G; ++gg) sd += p.partial_deta[(int64_t)chain * p.G + gg];
    *dt = sd;
  }
}

// Shared initial weights: sum the per-sequence gradients in sequence order
// (src may be null: d(eta) only).
__global__ __launch_bounds__(256) void ttt_bwd_sum(BwdSumArgs p) {
  const int dh = D * p.h;
  const int n4 = (2 * dh) / 4;
  const int i4 = blockIdx.x * 256 + threadIdx.x;
  const int head = blockIdx.y;
  if (p.src && i4 < n4) {
    const int idx = 4 * i4;
    f32x4 s = {0.f, 0.f, 0.f, 0.f};
    for (int b = 0; b < p.B; ++b)
      s += *reinterpret_cast<const f32x4*>(p.src + ((int64_t)b * p.H + head) * 2 * dh + idx);
    if (idx < dh)
      *reinterpret_cast<f32x4*>(p.dW1 + (int64_t)head * dh + idx) = s;
    else
      *reinterpret_cast<f32x4*>(p.dW2 + (int64_t)head * dh + (idx - dh)) = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float sd = 0.f;
    for (int b = 0; b < p.B; ++b) sd += p.deta_src[(int64_t)b * p.H + head];
    p.deta[head] = sd;
  }
}

hipError_t launch_bwd_sum(const BwdSumArgs& a, hipStream_t st) {
  const dim3 grid(((2 * D * a.h) / 4 + 255) / 256, a.H);
  hipLaunchKernelGGL(ttt_bwd_sum, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

// FP32 operands: one wave per 32-wide hidden block (4 waves at h=128, 8 at
// h=256); BF16 operands: ttt_bwd_step_bf.
template <int NW, int NB>
static hipError_t launch_bwd_step_t(const BwdStepArgs& a, int n_blocks, hipStream_t st) {
  hipLaunchKernelGGL((ttt_bwd_step<float, NW, NB>), dim3(n_blocks), dim3(NW * 64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_bwd_step(const BwdStepArgs& a, int n_blocks, int h, bool io_bf16, bool mma_bf16, hipStream_t st) {
  if (mma_bf16 || io_bf16) return launch_bwd_step_bf(a, n_blocks, h, io_bf16, st);
  return h == 128 ? launch_bwd_step_t<4, 1>(a, n_blocks, st) : launch_bwd_step_t<BWD_F32_NW256, 256 / (32 * BWD_F32_NW256)>(a, n_blocks, st);
}

hipError_t launch_bwd_reduce(const BwdReduceArgs& a, int n_blocks, hipStream_t st) {
  hipLaunchKernelGGL(ttt_bwd_reduce, dim3(n_blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace ttt
