// Reverse mode of the paper's memory unit (SwiGLU fast network, dot-product
// inner loss with token-wise step sizes; Supp. A, Sec. 4.2 Eq. 8-10) for the
// outer loss sum <O, dO>, on gfx950.
//
// Apply adjoint (O = f_W(Q) after an update, Sec. 3.2 Eq. 4), per token tile:
//   Zq1 = Q W1, Zq3 = Q W3, S = SiLU(Zq1), Hq = S * Zq3, dHq = dO W2^T,
//   adj W2 += Hq^T dO, adj W1 += Q^T (dHq * Zq3 * s'(Zq1)),
//   adj W3 += Q^T (dHq * S), dQ = (dHq * Zq3 * s') W1^T + (dHq * S) W3^T.
// Update adjoint of W' = W - G(W), G the gradient of L(W) = sum_i <f_W(k_i),
// E_i> with E_i = -eta_i v_i: for every input X, (dG/dX)^T Wh is the gradient
// of phi = d/dt L(W + t Wh) at t = 0 (the derivative of L along the carried
// adjoint Wh), so one tangent pass and its reverse give the second-order
// terms:
//   dot Z1 = K Wh1, dot Z3 = K Wh3, dot S = s'(Z1) dot Z1,
//   dot H = dot S * Z3 + S * dot Z3, dot Y = dot H W2 + Hd Wh2,
//   dH = E W2^T, dHh = E Wh2^T,
//   a(dot S) = dH * Z3, a(Z3) = dH * dot S + dHh * S,
//   a(S) = dH * dot Z3 + dHh * Z3, a(dot Z3) = dH * S,
//   a(dot Z1) = a(dot S) s'(Z1), a(Z1) = a(dot S) s''(Z1) dot Z1 + a(S) s'(Z1),
//   contribution to adj W: -(K^T a(Z1), dot H^T E, K^T a(Z3)),
//   dK = -(a(Z1) W1^T + a(Z3) W3^T + a(dot Z1) Wh1^T + a(dot Z3) Wh3^T),
//   dV_i = eta_i dot Y_i, d eta_i = <v_i, dot Y_i>,
// each followed by the adjoint of the per-token L2 normalisation.
//
// Layout as in the forward kernels: wave w owns hidden units [32w, 32w+32);
// products with a hidden axis in the result are 32x32 blocks with tokens in
// registers, which feed the token sums directly; products contracting the
// hidden axis read a staged [token][hidden] tile (two at a time) against the
// [d][hidden] operand copies.
#include <hip/hip_runtime.h>

#include "ttt_common.h"
#include "ttt_internal.h"

namespace ttt {
namespace {

// Per-kernel tile machinery shared by the two reverse-mode kernels.
template <typename MT, int NW>
struct AmuTiles {
  static constexpr bool BF = std::is_same_v<MT, bf16>;
  static constexpr int HH = NW * 32;
  static constexpr int DH = D * HH;
  static constexpr int LD = D + 4;                 // f32 [token][d] tiles
  static constexpr int AS_LD = HH + (BF ? 8 : 4);  // staged [token][hidden] tiles
  int hid, l32, hf, l16, g4;

  // 32x32 block C[token][hid] = X[token][:] M[hid][:]^T (M rows contiguous).
  __device__ f32x16 th(const float* X, const MT* M) const {
    f32x16 c = {};
    const MT* mrow = M + hid * D;
    if constexpr (BF) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int d0 = 16 * m + 8 * hf;
        const f32x4 x0 = *reinterpret_cast<const f32x4*>(&X[l32 * LD + d0]);
        const f32x4 x1 = *reinterpret_cast<const f32x4*>(&X[l32 * LD + d0 + 4]);
        const bf16x8 a = as_bf16x8(pack_bf16x2(x0[0], x0[1]), pack_bf16x2(x0[2], x0[3]),
                                   pack_bf16x2(x1[0], x1[1]), pack_bf16x2(x1[2], x1[3]));
        c = mma32(a, *reinterpret_cast<const bf16x8*>(mrow + d0), c);
      }
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
  }
  // 16x16 block C[token][d] (token half tb, feature block db) += S[token][:] F,
  // S a staged tile, F(hid, d) = M[d][hid].
  __device__ f32x4 td(const MT* S, int tb, int db, const MT* M, f32x4 c) const {
    const int arow = 16 * tb + l16;
    const MT* mrow = M + (16 * db + l16) * HH;
    if constexpr (BF) {
#pragma unroll
      for (int u = 0; u < HH / 32; ++u) {
        const int k0 = (HH / 4) * g4 + 8 * u;
        c = mma16(*reinterpret_cast<const bf16x8*>(&S[arow * AS_LD + k0]),
                  *reinterpret_cast<const bf16x8*>(mrow + k0), c);
      }
    } else {
#pragma unroll
      for (int u = 0; u < HH / 16; ++u) {
        const int k0 = (HH / 4) * g4 + 4 * u;
        const f32x4 a = *reinterpret_cast<const f32x4*>(&S[arow * AS_LD + k0]);
        const f32x4 b = *reinterpret_cast<const f32x4*>(mrow + k0);
#pragma unroll
        for (int e = 0; e < 4; ++e) c = mma16(a[e], b[e], c);
      }
    }
    return c;
  }
  // acc[db] (rows d = 32db.., cols hid) += X[:, d]^T Yw
  __device__ void tok_sum_dh(f32x16 (&acc)[2], const float* X, const f32x16& Yw) const {
#pragma unroll
    for (int db = 0; db < 2; ++db) {
      const int dd = 32 * db + l32;
      if constexpr (BF) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          uint32_t aw[4], bw[4];
#pragma unroll
          for (int e = 0; e < 8; e += 2) {
            aw[e / 2] = pack_bf16x2(X[c32_row(8 * m + e, hf) * LD + dd], X[c32_row(8 * m + e + 1, hf) * LD + dd]);
            bw[e / 2] = pack_bf16x2(Yw[8 * m + e], Yw[8 * m + e + 1]);
          }
          acc[db] = mma32(as_bf16x8(aw[0], aw[1], aw[2], aw[3]), as_bf16x8(bw[0], bw[1], bw[2], bw[3]), acc[db]);
        }
      } else {
#pragma unroll
        for (int s = 0; s < 16; ++s) acc[db] = mma32(X[c32_row(s, hf) * LD + dd], Yw[s], acc[db]);
      }
    }
  }
  // acc[db] (rows hid, cols d = 32db..) += Yw^T X[:, d]
  __device__ void tok_sum_hd(f32x16 (&acc)[2], const f32x16& Yw, const float* X) const {
#pragma unroll
    for (int db = 0; db < 2; ++db) {
      const int dd = 32 * db + l32;
      if constexpr (BF) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          uint32_t aw[4], bw[4];
#pragma unroll
          for (int e = 0; e < 8; e += 2) {
            aw[e / 2] = pack_bf16x2(Yw[8 * m + e], Yw[8 * m + e + 1]);
            bw[e / 2] = pack_bf16x2(X[c32_row(8 * m + e, hf) * LD + dd], X[c32_row(8 * m + e + 1, hf) * LD + dd]);
          }
          acc[db] = mma32(as_bf16x8(aw[0], aw[1], aw[2], aw[3]), as_bf16x8(bw[0], bw[1], bw[2], bw[3]), acc[db]);
        }
      } else {
#pragma unroll
        for (int s = 0; s < 16; ++s) acc[db] = mma32(Yw[s], X[c32_row(s, hf) * LD + dd], acc[db]);
      }
    }
  }
  // A 32x32 result (token rows in registers) into a staged [token][hidden] tile.
  __device__ void stage(MT* S, const f32x16& v) const {
#pragma unroll
    for (int r = 0; r < 16; ++r) S[c32_row(r, hf) * AS_LD + hid] = (MT)v[r];
  }
  // Shard partials of the three weight adjoints (W1 [d][h], W2 [h][d], W3 [d][h]),
  // each multiplied by `sign`.
  __device__ void write_partial(float* part, const f32x16 (&g1)[2], const f32x16 (&g2)[2], const f32x16 (&g3)[2],
                                int w, float sign) const {
#pragma unroll
    for (int db = 0; db < 2; ++db)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int rr = c32_row(r, hf);
        part[(32 * db + rr) * HH + hid] = sign * g1[db][r];
        part[DH + (32 * w + rr) * D + 32 * db + l32] = sign * g2[db][r];
        part[2 * DH + (32 * db + rr) * HH + hid] = sign * g3[db][r];
      }
  }
};

// Rows [t0, t0+nv) of a token tensor into an f32 LDS tile (zeros beyond nv),
// optionally L2-normalised; the row's 1/max(||x||, eps) and whether the norm
// exceeds eps go to inv[] / above[] (one writer lane per row).
template <typename IOT, int EPT>
__device__ __forceinline__ void load_rows_n(const IOT* base, int64_t t0, int nv, int64_t stride_tok, int64_t hoff,
                                            float* dst, bool do_norm, float* inv, int* above) {
  constexpr int LD = D + 4;
  constexpr int TPR = D / EPT;
  const int row = threadIdx.x / TPR, col0 = (threadIdx.x % TPR) * EPT;
  float x[EPT];
  if (row < nv) {
    load_vec<IOT, EPT>(base + (t0 + row) * stride_tok + hoff + col0, x);
  } else {
#pragma unroll
    for (int i = 0; i < EPT; ++i) x[i] = 0.f;
  }
  float sc = 1.f;
  int ab = 1;
  if (do_norm) {
    float ss = 0.f;
#pragma unroll
    for (int i = 0; i < EPT; ++i) ss = fmaf(x[i], x[i], ss);
    ss = lane_group_sum<TPR>(ss);
    const float nrm = sqrtf(ss);
    sc = 1.0f / fmaxf(nrm, NORM_EPS);
    ab = nrm > NORM_EPS;
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) dst[row * LD + col0 + i] = x[i] * sc;
  if (inv && threadIdx.x % TPR == 0) {
    inv[row] = sc;
    above[row] = ab;
  }
}

// Adjoint of the normalisation for this thread's row part: g is the adjoint
// of the normalised row xh; returns (g - xh (xh . g)) / ||x|| where the norm
// exceeds eps and g / eps otherwise (g unchanged when not normalised).
template <int EPT>
__device__ __forceinline__ void norm_adjoint(float (&g)[EPT], const float (&xh)[EPT], bool did_norm, float inv,
                                             int above) {
  if (!did_norm) return;
  float dot = 0.f;
#pragma unroll
  for (int i = 0; i < EPT; ++i) dot = fmaf(xh[i], g[i], dot);
  dot = lane_group_sum<D / EPT>(dot);
#pragma unroll
  for (int i = 0; i < EPT; ++i) g[i] = above ? (g[i] - xh[i] * dot) * inv : g[i] * inv;
}

}  // namespace

// Apply adjoint over [start, start+len): X = Q, Y = dO, dX = dQ.
template <typename IOT, bool BF, int NW>
__global__ __launch_bounds__(NW * 64) void ttt_amu_bwd_apply(AmuBwdArgs p) {
  using MT = std::conditional_t<BF, bf16, float>;
  using T = AmuTiles<MT, NW>;
  constexpr int DH = T::DH, LD = T::LD, AS_LD = T::AS_LD;
  constexpr int NT = NW * 64;
  constexpr int EPT = D * TT / NT;

  // Two copies of the row tiles: the rows of the next tile are loaded into
  // the other copy before the barrier that publishes this tile's dQ, so that
  // barrier also publishes them (two barriers per tile).
  __shared__ __attribute__((aligned(16))) float xs[2][TT * LD];    // normalised Q rows
  __shared__ __attribute__((aligned(16))) float ys[2][TT * LD];    // dO rows, then dQ before its norm adjoint
  __shared__ __attribute__((aligned(16))) MT sa[TT * AS_LD];
  __shared__ __attribute__((aligned(16))) MT sb[TT * AS_LD];
  __shared__ float ninv[2][TT];
  __shared__ int nabove[2][TT];

  const int tid = threadIdx.x;
  const int w = tid >> 6;
  T t;
  t.l32 = tid & 31; t.hf = (tid >> 5) & 1; t.l16 = tid & 15; t.g4 = (tid >> 4) & 3; t.hid = 32 * w + t.l32;
  const int row = tid / (D / EPT), col0 = (tid % (D / EPT)) * EPT;
  const int lin = xcd_linear_block();
  const int G = p.G;
  const int head = lin / G, g = lin % G;
  const int64_t hoff = (int64_t)head * p.stride_head;
  const bool norm_q = p.flags & 1u;
  const MT* Wb = static_cast<const MT*>(p.prep_w) + (int64_t)head * 6 * DH;

  f32x16 g1[2] = {}, g2[2] = {}, g3[2] = {};
  auto load_tile = [&](int tile, int b) {
    const int64_t t0 = p.start + (int64_t)tile * TT;
    const int nv = min(TT, p.len - tile * TT);
    load_rows_n<IOT, EPT>(static_cast<const IOT*>(p.X), t0, nv, p.stride_tok, hoff, xs[b], norm_q, ninv[b], nabove[b]);
    load_rows_n<IOT, EPT>(static_cast<const IOT*>(p.Y), t0, nv, p.stride_tok, hoff, ys[b], false, nullptr, nullptr);
  };
  if (g * TT < p.len) load_tile(g, 0);
  __syncthreads();
  for (int tile = g, i = 0; tile * TT < p.len; tile += G, ++i) {
    const int b = i & 1;
    const int64_t t0 = p.start + (int64_t)tile * TT;
    const int nv = min(TT, p.len - tile * TT);
    {
      const f32x16 Z1 = t.th(xs[b], Wb + AMU_W1T * DH);
      const f32x16 Z3 = t.th(xs[b], Wb + AMU_W3T * DH);
      const f32x16 dH = t.th(ys[b], Wb + AMU_W2N * DH);
      f32x16 Hq, dZ1, dZ3;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float z = Z1[r];
        const float sg = sigmoid(z);
        const float s = z * sg;
        Hq[r] = s * Z3[r];
        dZ3[r] = dH[r] * s;
        dZ1[r] = dH[r] * Z3[r] * fmaf(s, 1.0f - sg, sg);
      }
      t.tok_sum_hd(g2, Hq, ys[b]);
      t.tok_sum_dh(g1, xs[b], dZ1);
      t.tok_sum_dh(g3, xs[b], dZ3);
      t.stage(sa, dZ1);
      t.stage(sb, dZ3);
    }
    __syncthreads();
#pragma unroll
    for (int bi = 0; bi < 8 / NW; ++bi) {
      const int bk = w + NW * bi, tb = bk & 1, db = bk >> 1;
      f32x4 c = {};
      c = t.td(sa, tb, db, Wb + AMU_W1D * DH, c);
      c = t.td(sb, tb, db, Wb + AMU_W3D * DH, c);
#pragma unroll
      for (int r = 0; r < 4; ++r) ys[b][(16 * tb + 4 * t.g4 + r) * LD + 16 * db + t.l16] = c[r];
    }
    // the other copy was last read by the previous tile's dQ stage, which
    // every wave finished before the barrier above
    if ((tile + G) * TT < p.len) load_tile(tile + G, b ^ 1);
    __syncthreads();
    {
      float gq[EPT], xh[EPT];
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        gq[e] = ys[b][row * LD + col0 + e];
        xh[e] = xs[b][row * LD + col0 + e];
      }
      norm_adjoint<EPT>(gq, xh, norm_q, ninv[b][row], nabove[b][row]);
      if (row < nv) store_vec<IOT, EPT>(static_cast<IOT*>(p.dX) + (t0 + row) * p.stride_tok + hoff + col0, gq);
    }
  }
  if (p.len > 0) t.write_partial(p.partial + ((int64_t)head * G + g) * (3 * DH), g1, g2, g3, w, 1.0f);
}

// Update adjoint over [start, start+len): X = K, Y = V, dX = dK, dY = dV, at
// the weights in prep_w with the carried adjoint in prep_a.
template <typename IOT, bool BF, int NW>
__global__ __launch_bounds__(NW * 64) void ttt_amu_bwd_update(AmuBwdArgs p) {
  using MT = std::conditional_t<BF, bf16, float>;
  using T = AmuTiles<MT, NW>;
  constexpr int DH = T::DH, LD = T::LD, AS_LD = T::AS_LD;
  constexpr int NT = NW * 64;
  constexpr int EPT = D * TT / NT;
  constexpr int TPR = D / EPT;

  __shared__ __attribute__((aligned(16))) float xs[TT * LD];   // normalised K rows
  __shared__ __attribute__((aligned(16))) float vs[TT * LD];   // normalised V rows
  __shared__ __attribute__((aligned(16))) float es[TT * LD];   // E = -eta v, then dot Y
  __shared__ __attribute__((aligned(16))) float ks[TT * LD];   // adjoint of K (before the sign and norm)
  // Staged [token][hidden] pairs: with BF16 products the three pairs of a
  // tile (Hdot, Hd), (aZ1, aZ3), (aZd1, aZd3) get buffers of their own and are
  // staged together behind one barrier; FP32 tiles are twice as large and
  // reuse one pair, with a barrier before and after each restaging.
  constexpr int NS = BF ? 3 : 1;
  __shared__ __attribute__((aligned(16))) MT sa[NS][TT * AS_LD];
  __shared__ __attribute__((aligned(16))) MT sb[NS][TT * AS_LD];
  __shared__ float kinv[TT], vinv[TT], etas[TT];
  __shared__ int kab[TT], vab[TT];

  const int tid = threadIdx.x;
  const int w = tid >> 6;
  T t;
  t.l32 = tid & 31; t.hf = (tid >> 5) & 1; t.l16 = tid & 15; t.g4 = (tid >> 4) & 3; t.hid = 32 * w + t.l32;
  const int row = tid / TPR, col0 = (tid % TPR) * EPT;
  const int lin = xcd_linear_block();
  const int G = p.G;
  const int head = lin / G, g = lin % G;
  const int64_t hoff = (int64_t)head * p.stride_head;
  const bool norm_k = p.flags & 2u, norm_v = p.flags & 4u;
  const MT* Wb = static_cast<const MT*>(p.prep_w) + (int64_t)head * 6 * DH;
  const MT* Ab = static_cast<const MT*>(p.prep_a) + (int64_t)head * 6 * DH;

  f32x16 g1[2] = {}, g2[2] = {}, g3[2] = {};
  for (int tile = g; tile * TT < p.len; tile += G) {
    const int64_t t0 = p.start + (int64_t)tile * TT;
    const int nv = min(TT, p.len - tile * TT);
    load_rows_n<IOT, EPT>(static_cast<const IOT*>(p.X), t0, nv, p.stride_tok, hoff, xs, norm_k, kinv, kab);
    load_rows_n<IOT, EPT>(static_cast<const IOT*>(p.Y), t0, nv, p.stride_tok, hoff, vs, norm_v, vinv, vab);
    {
      const float et = row < nv ? p.eta_tok[(t0 + row) * p.H + head] : 0.f;
      if (tid % TPR == 0) etas[row] = et;
#pragma unroll
      for (int i = 0; i < EPT; ++i) es[row * LD + col0 + i] = -et * vs[row * LD + col0 + i];
    }
    __syncthreads();
    f32x16 aZ1, aZ3, aZd1, aZd3;
    {
      const f32x16 Z1 = t.th(xs, Wb + AMU_W1T * DH);
      const f32x16 Z3 = t.th(xs, Wb + AMU_W3T * DH);
      const f32x16 Zd1 = t.th(xs, Ab + AMU_W1T * DH);
      const f32x16 Zd3 = t.th(xs, Ab + AMU_W3T * DH);
      const f32x16 dH = t.th(es, Wb + AMU_W2N * DH);
      const f32x16 dHh = t.th(es, Ab + AMU_W2N * DH);
      f32x16 Hdot, Hd;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float z = Z1[r];
        const float sg = sigmoid(z);
        const float s = z * sg;
        const float s1 = fmaf(s, 1.0f - sg, sg);                          // s'(z)
        const float s2 = sg * (1.0f - sg) * fmaf(z, 1.0f - 2.0f * sg, 2.0f);  // s''(z)
        const float sd = s1 * Zd1[r];
        Hdot[r] = fmaf(sd, Z3[r], s * Zd3[r]);
        Hd[r] = s * Z3[r];
        const float asd = dH[r] * Z3[r];
        aZ3[r] = fmaf(dH[r], sd, dHh[r] * s);
        const float as = fmaf(dH[r], Zd3[r], dHh[r] * Z3[r]);
        aZd3[r] = dH[r] * s;
        aZd1[r] = asd * s1;
        aZ1[r] = fmaf(asd * s2, Zd1[r], as * s1);
      }
      t.tok_sum_hd(g2, Hdot, es);
      t.tok_sum_dh(g1, xs, aZ1);
      t.tok_sum_dh(g3, xs, aZ3);
      t.stage(sa[0], Hdot);
      t.stage(sb[0], Hd);
      if constexpr (NS == 3) {
        t.stage(sa[1], aZ1);
        t.stage(sb[1], aZ3);
        t.stage(sa[2], aZd1);
        t.stage(sb[2], aZd3);
      }
    }
    __syncthreads();
    constexpr int P1 = NS == 3 ? 1 : 0, P2 = NS == 3 ? 2 : 0;
    f32x4 yd[8 / NW], kb[8 / NW];
#pragma unroll
    for (int bi = 0; bi < 8 / NW; ++bi) {
      const int b = w + NW * bi, tb = b & 1, db = b >> 1;
      f32x4 c = {};
      c = t.td(sa[0], tb, db, Wb + AMU_W2D * DH, c);
      yd[bi] = t.td(sb[0], tb, db, Ab + AMU_W2D * DH, c);
    }
    if constexpr (NS == 1) {
      __syncthreads();
      t.stage(sa[0], aZ1);
      t.stage(sb[0], aZ3);
      __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 8 / NW; ++bi) {
      const int b = w + NW * bi, tb = b & 1, db = b >> 1;
      f32x4 c = {};
      c = t.td(sa[P1], tb, db, Wb + AMU_W1D * DH, c);
      kb[bi] = t.td(sb[P1], tb, db, Wb + AMU_W3D * DH, c);
    }
    if constexpr (NS == 1) {
      __syncthreads();
      t.stage(sa[0], aZd1);
      t.stage(sb[0], aZd3);
      __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 8 / NW; ++bi) {
      const int b = w + NW * bi, tb = b & 1, db = b >> 1;
      f32x4 c = kb[bi];
      c = t.td(sa[P2], tb, db, Ab + AMU_W1D * DH, c);
      c = t.td(sb[P2], tb, db, Ab + AMU_W3D * DH, c);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = (16 * tb + 4 * t.g4 + r) * LD + 16 * db + t.l16;
        ks[o] = c[r];
        es[o] = yd[bi][r];
      }
    }
    __syncthreads();
    {
      float gv[EPT], gk[EPT], xh[EPT], vh[EPT];
      float de = 0.f;
      const float et = etas[row];
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const float yv = es[row * LD + col0 + i];
        vh[i] = vs[row * LD + col0 + i];
        xh[i] = xs[row * LD + col0 + i];
        de = fmaf(vh[i], yv, de);
        gv[i] = et * yv;
        gk[i] = -ks[row * LD + col0 + i];
      }
      de = lane_group_sum<TPR>(de);
      norm_adjoint<EPT>(gv, vh, norm_v, vinv[row], vab[row]);
      norm_adjoint<EPT>(gk, xh, norm_k, kinv[row], kab[row]);
      if (row < nv) {
        store_vec<IOT, EPT>(static_cast<IOT*>(p.dY) + (t0 + row) * p.stride_tok + hoff + col0, gv);
        store_vec<IOT, EPT>(static_cast<IOT*>(p.dX) + (t0 + row) * p.stride_tok + hoff + col0, gk);
        if (tid % TPR == 0) p.deta_tok[(t0 + row) * p.H + head] = de;
      }
    }
    __syncthreads();
  }
  if (p.len > 0) t.write_partial(p.partial + ((int64_t)head * G + g) * (3 * DH), g1, g2, g3, w, -1.0f);
}

// dst = base + sum of the G shard partials (shard order), per head.
__global__ __launch_bounds__(256) void ttt_amu_psum(AmuPsumArgs p) {
  const int dh = D * p.h;
  const int n4 = (3 * dh) / 4;
  const int nbpc = (n4 + 255) / 256;
  const int head = blockIdx.x / nbpc, k = blockIdx.x % nbpc;
  const int i4 = k * 256 + threadIdx.x;
  if (i4 >= n4) return;
  const int idx = 4 * i4;
  const int64_t hb = (int64_t)head * 3 * dh;
  f32x4 s = p.base ? *reinterpret_cast<const f32x4*>(p.base + hb + idx) : (f32x4){0.f, 0.f, 0.f, 0.f};
  const f32x4* part = reinterpret_cast<const f32x4*>(p.partial + (int64_t)head * p.G * 3 * dh) + i4;
  s = add_shards(s, part, n4, p.G);
  if (p.dst) *reinterpret_cast<f32x4*>(p.dst + hb + idx) = s;
  const int mat = idx / dh, off = idx % dh;
  float* out = mat == 0 ? p.out1 : (mat == 1 ? p.out2 : p.out3);
  if (out) *reinterpret_cast<f32x4*>(out + (int64_t)head * dh + off) = s;
}

template <typename IOT, bool BF, int NW>
static hipError_t launch_apply_t(const AmuBwdArgs& a, int n_blocks, hipStream_t st) {
  hipLaunchKernelGGL((ttt_amu_bwd_apply<IOT, BF, NW>), dim3(n_blocks), dim3(NW * 64), 0, st, a);
  return hipGetLastError();
}
template <typename IOT, bool BF, int NW>
static hipError_t launch_update_t(const AmuBwdArgs& a, int n_blocks, hipStream_t st) {
  hipLaunchKernelGGL((ttt_amu_bwd_update<IOT, BF, NW>), dim3(n_blocks), dim3(NW * 64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_amu_bwd_apply(const AmuBwdArgs& a, int n_blocks, int h, bool io_bf16, bool mma_bf16,
                                hipStream_t st) {
  if (h == 128) {
    if (io_bf16) return launch_apply_t<bf16, true, 4>(a, n_blocks, st);
    return mma_bf16 ? launch_apply_t<float, true, 4>(a, n_blocks, st) : launch_apply_t<float, false, 4>(a, n_blocks, st);
  }
  if (io_bf16) return launch_apply_t<bf16, true, 8>(a, n_blocks, st);
  return mma_bf16 ? launch_apply_t<float, true, 8>(a, n_blocks, st) : launch_apply_t<float, false, 8>(a, n_blocks, st);
}

hipError_t launch_amu_bwd_update(const AmuBwdArgs& a, int n_blocks, int h, bool io_bf16, bool mma_bf16,
                                 hipStream_t st) {
  if (h == 128) {
    if (io_bf16) return launch_update_t<bf16, true, 4>(a, n_blocks, st);
    return mma_bf16 ? launch_update_t<float, true, 4>(a, n_blocks, st)
                    : launch_update_t<float, false, 4>(a, n_blocks, st);
  }
  if (io_bf16) return launch_update_t<bf16, true, 8>(a, n_blocks, st);
  return mma_bf16 ? launch_update_t<float, true, 8>(a, n_blocks, st) : launch_update_t<float, false, 8>(a, n_blocks, st);
}

hipError_t launch_amu_psum(const AmuPsumArgs& a, hipStream_t st) {
  const int nbpc = ((3 * D * a.h) / 4 + 255) / 256;
  hipLaunchKernelGGL(ttt_amu_psum, dim3(a.H * nbpc), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace ttt
