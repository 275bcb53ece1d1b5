// The paper's own adaptive memory unit on gfx950: a SwiGLU fast network
// f_W(x) = (SiLU(x W1) * (x W3)) W2 per head (Supp. A), the dot-product inner
// loss with token-wise step sizes, L_c(W) = -sum_i eta_i <f_W(k_i), v_i>
// (Sec. 4.2 Eq. 9 inside the token-wise update of Eq. 8), the step
// W <- W - grad L_c (the step sizes live inside the loss), and the apply
// O = f_W(Q) after the update (Sec. 3.2 Eq. 4).
//
// With E = -eta_i v_i (independent of W) the gradient of a chunk is
//   Z1 = K W1, Z3 = K W3, S = SiLU(Z1), Hd = S * Z3, dH = E W2^T,
//   grad W2 = Hd^T E, grad W3 = K^T (dH * S), grad W1 = K^T (dH * Z3 * s'(Z1)),
// so every product of the update has a hidden axis in its result (32x32
// blocks, tokens in registers, wave w owning hidden units [32w, 32w+32)) and
// the token sums take those registers directly; only the apply contracts the
// hidden axis (O = Hq W2 from a staged [token][hidden] tile).
//
// ttt_amu_step: one chunk step (gradient of chunk s over a token shard, apply
// of chunk s-1); ttt_amu_update: fixed-order sum of the shard partials and the
// step; ttt_amu_prep: operand copies of the weights in the matrix-core type.
#include <hip/hip_runtime.h>

#include "ttt_common.h"
#include "ttt_internal.h"

namespace ttt {

// Token t of a 32-token tile at slot(t) of a [d][token slot] column tile:
// bits 2 and 3 swapped, so the 8 tokens whose values a lane holds in
// registers 8m..8m+7 of a 32x32 result are 8 consecutive slots.
__device__ __forceinline__ constexpr int amu_slot(int t) { return (t & ~12) | ((t & 4) << 1) | ((t & 8) >> 1); }

template <typename IOT, bool BF, int NW>
__global__ __launch_bounds__(NW * 64) void ttt_amu_step(AmuStepArgs p) {
  constexpr int HH = NW * 32;
  constexpr int NT = NW * 64;
  constexpr int EPT = D * TT / NT;
  constexpr int TPR = D / EPT;
  constexpr int DH = D * HH;
  constexpr int LD = D + 4;
  using MT = std::conditional_t<BF, bf16, float>;
  constexpr int AS_LD = HH + (BF ? 8 : 4);

  // FP32 products read the token rows as FP32 tiles; BF16 products read each
  // token operand from two BF16 tiles written once per tile: rows [token][d]
  // (A operand of the 32x32 products, one 16-byte read per fragment) and
  // columns [d][token slot] (operand of the token sums, likewise).
  constexpr int XB = D + 8, XT = TT + 8;
  // The gradient loop alternates between two copies of its token tiles, so
  // one barrier per tile suffices (a tile's tiles are rewritten two tiles
  // later, after every wave has passed the next tile's barrier); the apply
  // uses copy 0.
  __shared__ __attribute__((aligned(16))) float xs[2][BF ? 1 : TT * LD];  // K or Q rows (normalised)
  __shared__ __attribute__((aligned(16))) float es[2][TT * LD];  // E = -eta v rows (FP32 products), or O rows
  __shared__ __attribute__((aligned(16))) MT sta[TT * AS_LD];  // staged Hq
  __shared__ __attribute__((aligned(16))) bf16 xr[2][BF ? TT * XB : 1];
  __shared__ __attribute__((aligned(16))) bf16 xc[2][BF ? D * XT : 1];
  __shared__ __attribute__((aligned(16))) bf16 er[2][BF ? TT * XB : 1];
  __shared__ __attribute__((aligned(16))) bf16 ec[2][BF ? D * XT : 1];

  const int tid = threadIdx.x;
  const int w = tid >> 6, l32 = tid & 31, hf = (tid >> 5) & 1, l16 = tid & 15, g4 = (tid >> 4) & 3;
  const int hid = 32 * w + l32;
  const int row = tid / TPR, col0 = (tid % TPR) * EPT;
  const int lin = xcd_linear_block();
  const int G = p.G;
  const int head = lin / G, g = lin % G;
  const int64_t hoff = (int64_t)head * p.stride_head;
  const bool norm_q = p.flags & 1u, norm_k = p.flags & 2u, norm_v = p.flags & 4u;
  // operand copies of this head: W1, W3, W2 as [hid][d], W2 as [d][hid]
  const MT* W1t = static_cast<const MT*>(p.prep) + (int64_t)head * p.n_prep * DH;
  const MT* W3t = W1t + AMU_W3T * DH;
  const MT* W2n = W1t + AMU_W2N * DH;
  const MT* W2d = W1t + AMU_W2D * DH;

  // BF16 operand fragments of M[hid][:] for this lane (M rows contiguous),
  // loaded before the barrier that precedes their products so that their
  // latency overlaps it.
  struct WF {
    bf16x8 f[4];
  };
  auto wload = [&](const MT* M) {
    WF r;
    if constexpr (BF) {
#pragma unroll
      for (int m = 0; m < 4; ++m) r.f[m] = *reinterpret_cast<const bf16x8*>(M + hid * D + 16 * m + 8 * hf);
    }
    return r;
  };
  // 32x32 block C[token][hid] = X[token][:] M[hid][:]^T (M rows contiguous);
  // FP32 products read the FP32 row tile X and M, BF16 products the BF16 row
  // tile Xb and the fragments wf of M.
  auto th = [&](const float* X, const bf16* Xb, const MT* M, const WF& wf) {
    f32x16 c = {};
    const MT* mrow = M + hid * D;
    if constexpr (BF) {
#pragma unroll
      for (int m = 0; m < 4; ++m)
        c = mma32(*reinterpret_cast<const bf16x8*>(&Xb[l32 * XB + 16 * m + 8 * hf]), wf.f[m], c);
    } else {
#pragma unroll
      for (int s4 = 0; s4 < 8; ++s4) {
        const int d0 = 32 * hf + 4 * s4;
        const f32x4 x = *reinterpret_cast<const f32x4*>(&X[l32 * LD + d0]);
        const f32x4 b = *reinterpret_cast<const f32x4*>(mrow + d0);
#pragma unroll
        for (int e = 0; e < 4; ++e) c = mma32(x[e], b[e], c);
      }
    }
    return c;
  };
  // 16x16 block C[token][d] (token half tb, feature block db) = S[token][:] F,
  // S the staged tile, F(hid, d) = M[d][hid].
  auto td = [&](int tb, int db, const MT* M) {
    f32x4 c = {};
    const int arow = 16 * tb + l16;
    const MT* mrow = M + (16 * db + l16) * HH;
    if constexpr (BF) {
#pragma unroll
      for (int u = 0; u < HH / 32; ++u) {
        const int k0 = (HH / 4) * g4 + 8 * u;
        c = mma16(*reinterpret_cast<const bf16x8*>(&sta[arow * AS_LD + k0]),
                  *reinterpret_cast<const bf16x8*>(mrow + k0), c);
      }
    } else {
#pragma unroll
      for (int u = 0; u < HH / 16; ++u) {
        const int k0 = (HH / 4) * g4 + 4 * u;
        const f32x4 a = *reinterpret_cast<const f32x4*>(&sta[arow * AS_LD + k0]);
        const f32x4 b = *reinterpret_cast<const f32x4*>(mrow + k0);
#pragma unroll
        for (int e = 0; e < 4; ++e) c = mma16(a[e], b[e], c);
      }
    }
    return c;
  };
  // Column fragment (feature dd, register group m) of a [d][token slot] tile.
  auto cfrag = [&](const bf16* Xc, int dd, int m) {
    return *reinterpret_cast<const bf16x8*>(&Xc[dd * XT + 16 * m + 8 * hf]);
  };
  // Registers 8m..8m+7 of a 32x32 result as one BF16 operand fragment.
  auto rfrag = [&](const f32x16& Yw, int m) {
    return as_bf16x8(pack_bf16x2(Yw[8 * m], Yw[8 * m + 1]), pack_bf16x2(Yw[8 * m + 2], Yw[8 * m + 3]),
                     pack_bf16x2(Yw[8 * m + 4], Yw[8 * m + 5]), pack_bf16x2(Yw[8 * m + 6], Yw[8 * m + 7]));
  };
  // acc[db] (rows d = 32db.., cols hid) += X[:, d]^T Yw (BF16: X from its column tile Xc)
  auto tok_sum_dh = [&](f32x16 (&acc)[2], const float* X, const bf16* Xc, const f32x16& Yw) {
#pragma unroll
    for (int db = 0; db < 2; ++db) {
      const int dd = 32 * db + l32;
      if constexpr (BF) {
#pragma unroll
        for (int m = 0; m < 2; ++m) acc[db] = mma32(cfrag(Xc, dd, m), rfrag(Yw, m), acc[db]);
      } else {
#pragma unroll
        for (int s = 0; s < 16; ++s) acc[db] = mma32(X[c32_row(s, hf) * LD + dd], Yw[s], acc[db]);
      }
    }
  };
  // acc[db] (rows hid, cols d = 32db..) += Yw^T X[:, d] (BF16: X from its column tile Xc)
  auto tok_sum_hd = [&](f32x16 (&acc)[2], const f32x16& Yw, const float* X, const bf16* Xc) {
#pragma unroll
    for (int db = 0; db < 2; ++db) {
      const int dd = 32 * db + l32;
      if constexpr (BF) {
#pragma unroll
        for (int m = 0; m < 2; ++m) acc[db] = mma32(rfrag(Yw, m), cfrag(Xc, dd, m), acc[db]);
      } else {
#pragma unroll
        for (int s = 0; s < 16; ++s) acc[db] = mma32(Yw[s], X[c32_row(s, hf) * LD + dd], acc[db]);
      }
    }
  };
  // Rows [t0, t0+nv) of a token tensor into an f32 LDS tile (zeros beyond
  // nv), optionally L2-normalised, optionally scaled by -eta_i: fetched into
  // registers one tile ahead (fetch_rows), written to LDS when the tile
  // starts (stage_rows), so the global-load latency overlaps a tile's work.
  struct RawRows {
    float x[EPT];
    float et;  // eta_i of this thread's row (0 past nv)
  };
  auto fetch_rows = [&](const void* base, int64_t t0, int nv, bool times_eta, RawRows& r) {
    const bool valid = row < nv;
    if (valid) {
      load_vec<IOT, EPT>(static_cast<const IOT*>(base) + (t0 + row) * p.stride_tok + hoff + col0, r.x);
    } else {
#pragma unroll
      for (int i = 0; i < EPT; ++i) r.x[i] = 0.f;
    }
    r.et = (times_eta && valid) ? p.eta_tok[(t0 + row) * p.H + head] : 0.f;
  };
  // FP32 products: into the FP32 row tile dst; BF16 products: into the
  // BF16 row tile rb and column tile cb.
  auto stage_rows = [&](const RawRows& r, float* dst, bf16* rb, bf16* cb, bool do_norm, bool times_eta) {
    float scale = 1.f;
    if (do_norm) {
      float ss = 0.f;
#pragma unroll
      for (int i = 0; i < EPT; ++i) ss = fmaf(r.x[i], r.x[i], ss);
      ss = lane_group_sum<TPR>(ss);
      scale = 1.0f / fmaxf(sqrtf(ss), NORM_EPS);
    }
    if (times_eta) scale *= -r.et;
    if constexpr (BF) {
      uint32_t pk[EPT / 2];
#pragma unroll
      for (int i = 0; i < EPT; i += 2) pk[i / 2] = pack_bf16x2(r.x[i] * scale, r.x[i + 1] * scale);
      uint32_t* rw = reinterpret_cast<uint32_t*>(&rb[row * XB + col0]);
#pragma unroll
      for (int i = 0; i < EPT / 2; ++i) rw[i] = pk[i];
      uint16_t* cw = reinterpret_cast<uint16_t*>(cb) + amu_slot(row);
#pragma unroll
      for (int i = 0; i < EPT; i += 2) {
        cw[(col0 + i) * XT] = (uint16_t)(pk[i / 2] & 0xffffu);
        cw[(col0 + i + 1) * XT] = (uint16_t)(pk[i / 2] >> 16);
      }
    } else {
#pragma unroll
      for (int i = 0; i < EPT; ++i) dst[row * LD + col0 + i] = r.x[i] * scale;
    }
  };

  f32x16 g1[2] = {}, g2[2] = {}, g3[2] = {};

  // ------------------------------------------------ gradient of chunk s
  const int gl = p.grad_len;
  RawRows rk, rv;
  auto fetch_grad = [&](int t) {
    const int64_t t0 = p.grad_start + (int64_t)t * TT;
    const int nv = min(TT, gl - t * TT);
    fetch_rows(p.K, t0, nv, false, rk);
    fetch_rows(p.V, t0, nv, true, rv);
  };
  if (g * TT < gl) fetch_grad(g);
  for (int t = g; t * TT < gl; t += G) {
    const int b = ((t - g) / G) & 1;
    stage_rows(rk, xs[b], xr[b], xc[b], norm_k, false);
    stage_rows(rv, es[b], er[b], ec[b], norm_v, true);
    if ((t + G) * TT < gl) fetch_grad(t + G);
    const WF f1 = wload(W1t), f3 = wload(W3t), f2 = wload(W2n);
    __syncthreads();
    const f32x16 Z1 = th(xs[b], xr[b], W1t, f1);
    const f32x16 Z3 = th(xs[b], xr[b], W3t, f3);
    const f32x16 dH = th(es[b], er[b], W2n, f2);
    f32x16 Hd, dZ1, dZ3;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float z = Z1[r];
      const float sg = sigmoid(z);
      const float s = z * sg;
      Hd[r] = s * Z3[r];
      dZ3[r] = dH[r] * s;
      dZ1[r] = dH[r] * Z3[r] * fmaf(s, 1.0f - sg, sg);
    }
    tok_sum_hd(g2, Hd, es[b], ec[b]);
    tok_sum_dh(g3, xs[b], xc[b], dZ3);
    tok_sum_dh(g1, xs[b], xc[b], dZ1);
  }
  __syncthreads();  // the apply reuses copy 0

  // ------------------------------------------------ apply of chunk s-1
  const int al = p.app_len;
  RawRows rq;
  auto fetch_app = [&](int t) {
    fetch_rows(p.Q, p.app_start + (int64_t)t * TT, min(TT, al - t * TT), false, rq);
  };
  // Pipelined over two copies of the row tiles: tile t+G is staged while the
  // products of tile t are finishing, so the barrier that publishes O rows of
  // tile t also publishes the rows of tile t+G (two barriers per tile).
  if (g * TT < al) {
    fetch_app(g);
    stage_rows(rq, xs[0], xr[0], xc[0], norm_q, false);
    if ((g + G) * TT < al) fetch_app(g + G);
  }
  const WF f1 = wload(W1t), f3 = wload(W3t);
  __syncthreads();
  for (int t = g, i = 0; t * TT < al; t += G, ++i) {
    const int b = i & 1;
    const int64_t t0 = p.app_start + (int64_t)t * TT;
    const int nv = min(TT, al - t * TT);
    {
      const f32x16 Zq1 = th(xs[b], xr[b], W1t, f1);
      const f32x16 Zq3 = th(xs[b], xr[b], W3t, f3);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float z = Zq1[r];
        sta[c32_row(r, hf) * AS_LD + hid] = (MT)(z * sigmoid(z) * Zq3[r]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int bi = 0; bi < 8 / NW; ++bi) {
      const int bk = w + NW * bi, tb = bk & 1, db = bk >> 1;
      const f32x4 o = td(tb, db, W2d);
#pragma unroll
      for (int r = 0; r < 4; ++r) es[0][(16 * tb + 4 * g4 + r) * LD + 16 * db + l16] = o[r];
    }
    if ((t + G) * TT < al) {  // rows of the next tile into the other copy (last read two tiles ago)
      stage_rows(rq, xs[b ^ 1], xr[b ^ 1], xc[b ^ 1], norm_q, false);
      if ((t + 2 * G) * TT < al) fetch_app(t + 2 * G);
    }
    __syncthreads();
    if (row < nv) {
      float v[EPT];
#pragma unroll
      for (int e = 0; e < EPT; ++e) v[e] = es[0][row * LD + col0 + e];
      store_vec<IOT, EPT>(static_cast<IOT*>(p.O) + (t0 + row) * p.stride_tok + hoff + col0, v);
    }
  }

  // ------------------------------------------------ shard partials
  if (gl > 0) {
    float* part = p.partial + ((int64_t)head * G + g) * (3 * DH);
#pragma unroll
    for (int db = 0; db < 2; ++db)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int rr = c32_row(r, hf);
        part[(32 * db + rr) * HH + hid] = g1[db][r];
        part[DH + (32 * w + rr) * D + 32 * db + l32] = g2[db][r];
        part[2 * DH + (32 * db + rr) * HH + hid] = g3[db][r];
      }
  }
}

// W_dst = W_src - (sum of the G shard partials, fixed order), per head; the
// final weights are also written split when asked.
__global__ __launch_bounds__(256) void ttt_amu_update(AmuUpdArgs p) {
  const int dh = D * p.h;
  const int n4 = (3 * dh) / 4;
  const int nbpc = (n4 + 255) / 256;
  const int head = blockIdx.x / nbpc, k = blockIdx.x % nbpc;
  const int i4 = k * 256 + threadIdx.x;
  if (i4 >= n4) return;
  const int idx = 4 * i4;
  f32x4 s = {0.f, 0.f, 0.f, 0.f};
  const f32x4* part = reinterpret_cast<const f32x4*>(p.partial + (int64_t)head * p.G * 3 * dh) + i4;
  s = add_shards(s, part, n4, p.G);
  const int mat = idx / dh, off = idx % dh;
  const float* src = mat == 0 ? p.src.w1 : (mat == 1 ? p.src.w2 : p.src.w3);
  const f32x4 wn = *reinterpret_cast<const f32x4*>(src + (int64_t)head * p.src.stride + off) - s;
  *reinterpret_cast<f32x4*>(p.w_dst + (int64_t)head * 3 * dh + idx) = wn;
  float* fin = mat == 0 ? p.wT1 : (mat == 1 ? p.wT2 : p.wT3);
  if (fin) *reinterpret_cast<f32x4*>(fin + (int64_t)head * dh + off) = wn;
}

// Operand copies per head: W1 and W3 as [hid][d], W2 as [hid][d] and [d][hid],
// and with n_mats = 6 also W1 and W3 as [d][hid] (their own layout).
template <typename MT>
__global__ __launch_bounds__(256) void ttt_amu_prep(AmuPrepArgs p) {
  const int h = p.h, dh = D * h;
  const int head = blockIdx.y;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= dh) return;
  const int64_t hb = (int64_t)head * p.src.stride;
  MT* o = static_cast<MT*>(p.prep) + (int64_t)head * p.n_mats * dh;
  const int d = idx / h, hh = idx % h;    // W1 / W3 element (d, hh)
  const int hh2 = idx / D, d2 = idx % D;  // W2 element (hh2, d2)
  const float w1 = p.src.w1[hb + idx], w3 = p.src.w3[hb + idx];
  o[AMU_W1T * dh + hh * D + d] = (MT)w1;
  o[AMU_W3T * dh + hh * D + d] = (MT)w3;
  const float w2 = p.src.w2[hb + idx];
  o[AMU_W2N * dh + idx] = (MT)w2;
  o[AMU_W2D * dh + d2 * h + hh2] = (MT)w2;
  if (p.n_mats == 6) {
    o[AMU_W1D * dh + idx] = (MT)w1;
    o[AMU_W3D * dh + idx] = (MT)w3;
  }
}

template <typename IOT, bool BF, int NW>
static hipError_t launch_amu_step_t(const AmuStepArgs& a, int n_blocks, hipStream_t st) {
  hipLaunchKernelGGL((ttt_amu_step<IOT, BF, NW>), dim3(n_blocks), dim3(NW * 64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_amu_step(const AmuStepArgs& a, int n_blocks, int h, bool io_bf16, bool mma_bf16, hipStream_t st) {
  if (h == 128) {
    if (io_bf16) return launch_amu_step_t<bf16, true, 4>(a, n_blocks, st);
    return mma_bf16 ? launch_amu_step_t<float, true, 4>(a, n_blocks, st)
                    : launch_amu_step_t<float, false, 4>(a, n_blocks, st);
  }
  if (io_bf16) return launch_amu_step_t<bf16, true, 8>(a, n_blocks, st);
  return mma_bf16 ? launch_amu_step_t<float, true, 8>(a, n_blocks, st)
                  : launch_amu_step_t<float, false, 8>(a, n_blocks, st);
}

hipError_t launch_amu_update(const AmuUpdArgs& a, hipStream_t st) {
  const int nbpc = ((3 * D * a.h) / 4 + 255) / 256;
  hipLaunchKernelGGL(ttt_amu_update, dim3(a.H * nbpc), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_amu_prep(const AmuPrepArgs& a, bool mma_bf16, hipStream_t st) {
  const dim3 grid((D * a.h + 255) / 256, a.H);
  if (mma_bf16)
    hipLaunchKernelGGL(ttt_amu_prep<bf16>, grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(ttt_amu_prep<float>, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace ttt
