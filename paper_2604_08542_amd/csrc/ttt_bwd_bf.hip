// BF16 matrix-core backward step of the chunked TTT chain (h = 128 or 256).
//
// Same mathematics as ttt_bwd_step (reverse mode through the inner update of
// chunk s, second-order terms included, plus the apply adjoint of chunk s-1;
// Sec. 4.2 Eq. 8 and Sec. 3.2 Eq. 3-4), organised for BF16 operands:
//
//  - 4 waves, one per SIMD; wave w owns hidden blocks hb = NB*w .. NB*w+NB-1
//    (32 units each, NB = h/128).  Products whose result has a hidden axis
//    are 32x32 blocks with tokens in registers; they feed the token-sum
//    products (gradients of W) straight from registers as packed BF16 pairs.
//  - Products contracting the hidden axis read [token][hidden] BF16 tiles
//    staged in LDS; wave w computes the 16 feature columns 16w..16w+15 of
//    both 16-token halves, so each weight fragment is loaded once per phase.
//  - Every token-side operand (K, Q, E, dY, dO) is written once to LDS in two
//    BF16 forms: rows [token][d] for the 32x32 products and columns
//    [d][token slot] for the token sums, the slot order matching the
//    register order of a 32x32 result so that one 16-byte read is one
//    operand fragment.
//  - sigma(Z) is computed once per element and kept; the raw rows of the
//    next tile are loaded into registers while the current tile computes.
//
// One update tile runs in 7 LDS phases: rows -> Z, A (stage A) -> Y, A Wh2
// (E, -eta A Wh2) -> P, K Wh1 (stage D, dP) -> dE (dY) -> dA, token sums
// (stage dZ) -> dK -> normalisation adjoint of dK, dV.  An apply tile runs
// rows -> Zq, dZq, token sums (stage dZq) -> dQ -> adjoint of dQ.
#include <hip/hip_runtime.h>

#include "ttt_common.h"
#include "ttt_internal.h"

namespace ttt {
namespace {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// LDS plan (byte offsets).  The BF16 tiles come first so that their
// addresses stay within reach of the 16-bit immediate offsets.
template <int NB>
struct BwdLds {
  static constexpr int HH = 128 * NB;
  static constexpr int XB = D + 8;   // bf16 [token][d]
  static constexpr int XT = TT + 8;  // bf16 [d][token slot]
  static constexpr int SL = HH + 8;  // bf16 [token][hidden]
  static constexpr int FL = D + 4;   // f32 [token][d]
  static constexpr int xb = 0;                   // K or Q rows
  static constexpr int eb = xb + TT * XB * 2;    // E rows
  static constexpr int yb = eb + TT * XB * 2;    // dY or dO rows
  static constexpr int xt = yb + TT * XB * 2;    // K or Q columns
  static constexpr int et = xt + D * XT * 2;     // E columns
  static constexpr int yt = et + D * XT * 2;     // dY or dO columns
  static constexpr int s0 = yt + D * XT * 2;     // staged A, then dP, then dZ (or dZq)
  static constexpr int s1 = s0 + TT * SL * 2;    // staged D
  static constexpr int xf = s1 + TT * SL * 2;    // K or Q rows, f32 (normalisation adjoint)
  static constexpr int vf = xf + TT * FL * 4;    // V rows, f32
  static constexpr int yf = vf + TT * FL * 4;    // dY rows, f32
  static constexpr int df = yf + TT * FL * 4;    // dK or dQ rows, f32
  static constexpr int ninv = df + TT * FL * 4;  // float [2][TT]
  static constexpr int above = ninv + 2 * TT * 4;  // int [2][TT]
  static constexpr int red = above + 2 * TT * 4;   // float [4]
  static constexpr int total = red + 16;
};

// Token t of a 32-token tile sits at slot(t) of the column tiles: bits 2
// and 3 swapped, so that the 8 tokens a lane holds in registers 8m..8m+7 of
// a 32x32 result (rows 8(r/4) + 4*half + r%4) are 8 consecutive slots.
__device__ __forceinline__ constexpr int slot_of(int t) { return (t & ~12) | ((t & 4) << 1) | ((t & 8) >> 1); }

// The 8 io elements a thread loads per row, as loaded (f32 values, or bf16
// pairs in 32-bit words).  FP32 rows are held as float vectors: this
// compiler turns a select over bit-cast elements of an integer vector into a
// splat of element 0, so integer words are used only for the bf16 pairs.
template <typename IOT>
struct RawRow {
  f32x4 a, b;
};
template <>
struct RawRow<bf16> {
  u32x4 a;
};

// Rows are always loaded (masked rows of a ragged tile read the tile's last
// valid row) and zeroed when unpacked, so the loads need no branch.
template <typename IOT>
__device__ __forceinline__ void fetch_row(const IOT* base, uint32_t elem, RawRow<IOT>& r) {
  if constexpr (std::is_same_v<IOT, float>) {
    const f32x4* s = reinterpret_cast<const f32x4*>(base + elem);
    r.a = s[0];
    r.b = s[1];
  } else {
    r.a = *reinterpret_cast<const u32x4*>(base + elem);
  }
}

template <typename IOT>
__device__ __forceinline__ void unpack_row(const RawRow<IOT>& r, bool valid, float (&x)[8]) {
  if constexpr (std::is_same_v<IOT, float>) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      x[i] = valid ? r.a[i] : 0.f;
      x[4 + i] = valid ? r.b[i] : 0.f;
    }
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      x[2 * i] = valid ? __builtin_bit_cast(float, r.a[i] << 16) : 0.f;
      x[2 * i + 1] = valid ? __builtin_bit_cast(float, r.a[i] & 0xffff0000u) : 0.f;
    }
  }
}

}  // namespace

template <typename IOT, int NB>
__global__ __launch_bounds__(256) void ttt_bwd_step_bf(BwdStepArgs p) {
  using L = BwdLds<NB>;
  constexpr int HH = L::HH;
  constexpr int DH = D * HH;
  constexpr int XB = L::XB, XT = L::XT, SL = L::SL, FL = L::FL;
  constexpr int NU = HH / 32;  // 16x16x32 products along the hidden axis

  __shared__ __attribute__((aligned(16))) char smem[L::total];
  auto lds = [&](int off) { return smem + off; };

  const int tid = threadIdx.x;
  const int w = tid >> 6, l32 = tid & 31, hf = (tid >> 5) & 1, l16 = tid & 15, g4 = (tid >> 4) & 3;
  const int row = tid >> 3, col0 = (tid & 7) * 8;  // row mapping: 8 threads x 8 elements per token
  const int lin = xcd_linear_block();
  const int G = p.G;
  const int slot = lin / G, g = lin % G;  // slot = active sequence * H + head
  const int ai = slot / p.H, head = slot % p.H;
  const float eta = p.eta;
  const bf16* prep = static_cast<const bf16*>(p.prep) + (int64_t)slot * 8 * DH;
  const int64_t hoff = (int64_t)head * p.stride_head;
  const bool norm_q = p.flags & 1u, norm_k = p.flags & 2u, norm_v = p.flags & 4u;
  float* ninv = reinterpret_cast<float*>(lds(L::ninv));
  int* above = reinterpret_cast<int*>(lds(L::above));

  // ---------------------------------------------------------------- helpers
  // A fragments of a [token][d] tile for the 32x32 products (token = l32).
  auto xfrag = [&](int off, bf16x8 (&a)[4]) {
#pragma unroll
    for (int m = 0; m < 4; ++m) a[m] = *reinterpret_cast<const bf16x8*>(lds(off + (l32 * XB + 16 * m + 8 * hf) * 2));
  };
  // Weight fragments are loaded one LDS phase before the phase that uses
  // them (the barrier between phases does not wait for global loads), so
  // their L2 latency overlaps the elementwise epilogue of the current phase.
  // Prepared operand k: 0..3 = W1, W2, Wh1, Wh2 as [hid][d]; 4..7 = the same
  // as [d][hid].
  struct ThW {  // B fragments of the 32x32 products for this wave's NB hidden blocks
    bf16x8 f[NB][4];
  };
  struct TdW {  // B fragments of the 16x16 products for this wave's 16 feature columns
    bf16x8 f[NU];
  };
  // Buffer loads: one descriptor for this head's 8 prepared operands, a
  // per-lane byte offset shared by every matrix of a kind, and the matrix /
  // fragment offset in a scalar register (no per-matrix address registers).
  const __amdgpu_buffer_rsrc_t prsrc =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<bf16*>(prep), (short)0, 8 * DH * 2, 0x00020000);
  const int th_off = ((32 * NB * w + l32) * D + 8 * hf) * 2;
  const int td_off = ((16 * w + l16) * HH + (HH / 4) * g4) * 2;
  auto bload = [&](int voff, int soff) {
    return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(prsrc, voff, soff, 0));
  };
  auto load_th = [&](int k) {
    ThW r;
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int m = 0; m < 4; ++m) r.f[j][m] = bload(th_off, k * DH * 2 + j * 32 * D * 2 + 32 * m);
    return r;
  };
  auto load_td = [&](int k) {
    TdW r;
#pragma unroll
    for (int u = 0; u < NU; ++u) r.f[u] = bload(td_off, k * DH * 2 + 16 * u);
    return r;
  };
  // 32x32 block C[token][hid] of hidden block j: X[token][:] M[hid][:]^T.
  auto th = [&](const bf16x8 (&a)[4], const ThW& wt, int j) {
    f32x16 c = {};
#pragma unroll
    for (int m = 0; m < 4; ++m) c = mma32(a[m], wt.f[j][m], c);
    return c;
  };
  // Keeps the scheduler from hoisting a prefetch above the products before it.
  auto fence_sched = [] { __builtin_amdgcn_sched_barrier(0); };
  // A fragment u of the staged [token][hid] tile for token half tb.
  auto sfrag = [&](int soff, int tb, int u) {
    return *reinterpret_cast<const bf16x8*>(lds(soff + ((16 * tb + l16) * SL + (HH / 4) * g4 + 8 * u) * 2));
  };
  // Column fragment (feature block db, register group m) of a [d][slot] tile.
  auto tfrag = [&](int off, int db, int m) {
    return *reinterpret_cast<const bf16x8*>(lds(off + ((32 * db + l32) * XT + 16 * m + 8 * hf) * 2));
  };
  auto pack16 = [&](const f32x16& v, uint32_t (&pk)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) pk[q] = pack_bf16x2(v[2 * q], v[2 * q + 1]);
  };
  auto opnd = [&](const uint32_t (&pk)[8], int m) { return as_bf16x8(pk[4 * m], pk[4 * m + 1], pk[4 * m + 2], pk[4 * m + 3]); };
  // Write a packed 32x32 result column (hidden block hb) into a staged tile.
  auto stage = [&](int soff, const uint32_t (&pk)[8], int hb) {
    uint16_t* col = reinterpret_cast<uint16_t*>(lds(soff)) + 4 * hf * SL + 32 * hb + l32;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int r0 = 2 * q, r1 = 2 * q + 1;
      col[(8 * (r0 >> 2) + (r0 & 3)) * SL] = (uint16_t)(pk[q] & 0xffffu);
      col[(8 * (r1 >> 2) + (r1 & 3)) * SL] = (uint16_t)(pk[q] >> 16);
    }
  };
  // Token-side value v (4 tokens 16tb+4g4+r, feature 16w+l16 of a 16x16
  // result) into a row tile and a column tile.
  auto put_bf = [&](int roff, int coff, int tb, const f32x4& v) {
    const int d = 16 * w + l16;
    uint16_t* rt = reinterpret_cast<uint16_t*>(lds(roff));
    const uint32_t p01 = pack_bf16x2(v[0], v[1]), p23 = pack_bf16x2(v[2], v[3]);
    const int t0 = 16 * tb + 4 * g4;
    rt[(t0 + 0) * XB + d] = (uint16_t)(p01 & 0xffffu);
    rt[(t0 + 1) * XB + d] = (uint16_t)(p01 >> 16);
    rt[(t0 + 2) * XB + d] = (uint16_t)(p23 & 0xffffu);
    rt[(t0 + 3) * XB + d] = (uint16_t)(p23 >> 16);
    *reinterpret_cast<u32x2*>(lds(coff + (d * XT + slot_of(t0)) * 2)) = (u32x2){p01, p23};
  };
  // Normalise a fetched row (optionally) and write it to the f32, bf16 row
  // and bf16 column tiles (any offset < 0 is skipped).
  auto put_row = [&](const RawRow<IOT>& raw, bool valid, bool do_norm, int ns, int foff, int boff, int toff) {
    float x[8];
    unpack_row<IOT>(raw, valid, x);
    if (do_norm) {
      float ss = 0.f;
#pragma unroll
      for (int i = 0; i < 8; ++i) ss = fmaf(x[i], x[i], ss);
      ss = lane_group_sum<8>(ss);
      const float nrm = sqrtf(ss);
      const float inv = 1.0f / fmaxf(nrm, NORM_EPS);
#pragma unroll
      for (int i = 0; i < 8; ++i) x[i] *= inv;
      if ((tid & 7) == 0) {
        ninv[ns * TT + row] = inv;
        above[ns * TT + row] = nrm > NORM_EPS;
      }
    }
    if (foff >= 0) {
      f32x4* f = reinterpret_cast<f32x4*>(lds(foff + (row * FL + col0) * 4));
      f[0] = (f32x4){x[0], x[1], x[2], x[3]};
      f[1] = (f32x4){x[4], x[5], x[6], x[7]};
    }
    uint32_t pk[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) pk[i] = pack_bf16x2(x[2 * i], x[2 * i + 1]);
    if (boff >= 0) *reinterpret_cast<u32x4*>(lds(boff + (row * XB + col0) * 2)) = (u32x4){pk[0], pk[1], pk[2], pk[3]};
    if (toff >= 0) {
      uint16_t* ct = reinterpret_cast<uint16_t*>(lds(toff)) + slot_of(row);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ct[(col0 + 2 * i) * XT] = (uint16_t)(pk[i] & 0xffffu);
        ct[(col0 + 2 * i + 1) * XT] = (uint16_t)(pk[i] >> 16);
      }
    }
  };
  // Normalisation adjoint of the f32 row tile at doff (times sign), stored
  // to the io tensor for tokens [t0, t0+nv).
  auto store_adj = [&](void* base, int64_t t0, int nv, int doff, int xoff, bool did_norm, int ns, float sign) {
    const f32x4* dp = reinterpret_cast<const f32x4*>(lds(doff + (row * FL + col0) * 4));
    const f32x4* xp = reinterpret_cast<const f32x4*>(lds(xoff + (row * FL + col0) * 4));
    float v[8], xh[8];
    float dot = 0.f;
#pragma unroll
    for (int h4 = 0; h4 < 2; ++h4) {
      const f32x4 dv = dp[h4], xv = xp[h4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        v[4 * h4 + i] = sign * dv[i];
        xh[4 * h4 + i] = xv[i];
        dot = fmaf(v[4 * h4 + i], xv[i], dot);
      }
    }
    if (did_norm) {
      dot = lane_group_sum<8>(dot);
      const float inv = ninv[ns * TT + row];
      const bool ab = above[ns * TT + row];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = ab ? (v[i] - xh[i] * dot) * inv : v[i] * inv;
    }
    IOT* tile = static_cast<IOT*>(base) + t0 * p.stride_tok + hoff;  // wave-uniform
    if (row < nv) store_vec<IOT, 8>(tile + (uint32_t)(row * (uint32_t)p.stride_tok + col0), v);
  };

  f32x16 gw1[NB][2] = {}, gw2[NB][2] = {};
  float deta_acc = 0.f;

  const int gl = p.grad_len[ai], al = p.app_len[ai];
  const int64_t grad_start = p.grad_start[ai], app_start = p.app_start[ai];
  const int n_gt = (gl + TT - 1) / TT, n_at = (al + TT - 1) / TT;
  const float e_scale = gl > 0 ? 2.0f / (float)gl : 0.f;
  RawRow<IOT> ra, rb;
  // Row loads: a wave-uniform tile base plus a 32-bit per-lane offset.
  auto fetch_upd = [&](int t) {
    const int64_t tb0 = (grad_start + (int64_t)t * TT) * p.stride_tok + hoff;
    const uint32_t e = (uint32_t)(min(row, gl - t * TT - 1) * (uint32_t)p.stride_tok + col0);
    fetch_row<IOT>(static_cast<const IOT*>(p.K) + tb0, e, ra);
    fetch_row<IOT>(static_cast<const IOT*>(p.V) + tb0, e, rb);
  };
  auto fetch_app = [&](int t) {
    const int64_t tb0 = (app_start + (int64_t)t * TT) * p.stride_tok + hoff;
    const uint32_t e = (uint32_t)(min(row, al - t * TT - 1) * (uint32_t)p.stride_tok + col0);
    fetch_row<IOT>(static_cast<const IOT*>(p.Q) + tb0, e, ra);
    fetch_row<IOT>(static_cast<const IOT*>(p.dO) + tb0, e, rb);
  };
  if (g < n_gt)
    fetch_upd(g);
  else if (g < n_at)
    fetch_app(g);

  ThW wA = load_th(0);  // W1 for the first Z (or Zq) products

  // ------------------------------------------------ update adjoint of chunk s
  for (int t = g; t < n_gt; t += G) {
    const int64_t t0 = grad_start + (int64_t)t * TT;
    const int nv = min(TT, gl - t * TT);
    // phase 0: rows of K and V
    put_row(ra, row < nv, norm_k, 0, L::xf, L::xb, L::xt);
    put_row(rb, row < nv, norm_v, 1, L::vf, -1, -1);
    if (t + G < n_gt)
      fetch_upd(t + G);
    else if (g < n_at)
      fetch_app(g);
    __syncthreads();
    // phase 1: Z = K W1, sigma(Z), A = s(Z) (staged)
    f32x16 Z[NB], Sg[NB];
    uint32_t Apk[NB][8];
    TdW b2, bh;
    {
      bf16x8 xa[4];
      xfrag(L::xb, xa);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        Z[j] = th(xa, wA, j);
        if (j == NB - 1) {
          fence_sched();
          b2 = load_td(5);
          bh = load_td(7);
        }
        f32x16 A;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          Sg[j][r] = sigmoid(Z[j][r]);
          A[r] = Z[j][r] * Sg[j][r];
        }
        pack16(A, Apk[j]);
        stage(L::s0, Apk[j], NB * w + j);
      }
    }
    __syncthreads();
    // phase 2: Y = A W2 -> E;  A Wh2 -> -eta A Wh2 (kept) and its d(eta) term
    f32x4 des[2];
    ThW wP, wK;
    {
      f32x4 y[2] = {}, aw[2] = {};
#pragma unroll
      for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int tb = 0; tb < 2; ++tb) {
          const bf16x8 a = sfrag(L::s0, tb, u);
          y[tb] = mma16(a, b2.f[u], y[tb]);
          aw[tb] = mma16(a, bh.f[u], aw[tb]);
        }
      fence_sched();
      wP = load_th(1);
      wK = load_th(2);
      const float* vf = reinterpret_cast<const float*>(lds(L::vf));
      const int d = 16 * w + l16;
#pragma unroll
      for (int tb = 0; tb < 2; ++tb) {
        f32x4 E;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          E[r] = e_scale * (y[tb][r] - vf[(16 * tb + 4 * g4 + r) * FL + d]);
          deta_acc -= aw[tb][r] * E[r];
          des[tb][r] = -eta * aw[tb][r];
        }
        put_bf(L::eb, L::et, tb, E);
      }
    }
    __syncthreads();
    // phase 3: P = E W2^T, K Wh1; D = P s'(Z) (staged), dP = dD s'(Z)
    // (staged), dZ = dD P s''(Z) with dD = -eta K Wh1
    f32x16 S1[NB], dZ[NB];
    uint32_t dPpk[NB][8];
    TdW b2b;
    {
      bf16x8 ea[4], xa[4];
      xfrag(L::eb, ea);
      xfrag(L::xb, xa);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const f32x16 P = th(ea, wP, j);
        const f32x16 KW = th(xa, wK, j);
        if (j == NB - 1) {
          fence_sched();
          b2b = load_td(5);
        }
        f32x16 Dm, dP;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float z = Z[j][r], sg = Sg[j][r];
          const float a = z * sg;
          const float s1 = fmaf(a, 1.0f - sg, sg);
          const float s2 = sg * (1.0f - sg) * fmaf(z, 1.0f - 2.0f * sg, 2.0f);
          Dm[r] = P[r] * s1;
          deta_acc -= KW[r] * Dm[r];
          const float dD = -eta * KW[r];
          dP[r] = dD * s1;
          dZ[j][r] = dD * P[r] * s2;
          S1[j][r] = s1;
        }
        uint32_t Dpk[8];
        pack16(Dm, Dpk);
        pack16(dP, dPpk[j]);
        stage(L::s1, Dpk, NB * w + j);
        stage(L::s0, dPpk[j], NB * w + j);
      }
    }
    __syncthreads();
    // phase 4: dE = -eta A Wh2 + dP W2;  dY = (2/M) dE
    ThW wH, wW;
    {
      f32x4 de[2] = {};
#pragma unroll
      for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int tb = 0; tb < 2; ++tb) de[tb] = mma16(sfrag(L::s0, tb, u), b2b.f[u], de[tb]);
      fence_sched();
      wH = load_th(3);
      wW = load_th(1);
      float* yf = reinterpret_cast<float*>(lds(L::yf));
      const int d = 16 * w + l16;
#pragma unroll
      for (int tb = 0; tb < 2; ++tb) {
        f32x4 dY;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          dY[r] = e_scale * (des[tb][r] + de[tb][r]);
          yf[(16 * tb + 4 * g4 + r) * FL + d] = dY[r];
        }
        put_bf(L::yb, L::yt, tb, dY);
      }
    }
    __syncthreads();
    // phase 5: dA = -eta E Wh2^T + dY W2^T;  dZ += dA s'(Z);  token sums
    //          dP^T E + A^T dY (W2) and K^T dZ (W1);  stage dZ
    TdW b1, bh1;
    {
      bf16x8 ea[4], ya[4];
      xfrag(L::eb, ea);
      xfrag(L::yb, ya);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const f32x16 dA1 = th(ea, wH, j);
        const f32x16 dA2 = th(ya, wW, j);
        if (j == NB - 1) {
          fence_sched();
          b1 = load_td(4);
          bh1 = load_td(6);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) dZ[j][r] += (-eta * dA1[r] + dA2[r]) * S1[j][r];
        uint32_t dZpk[8];
        pack16(dZ[j], dZpk);
#pragma unroll
        for (int db = 0; db < 2; ++db)
#pragma unroll
          for (int m = 0; m < 2; ++m) {
            gw2[j][db] = mma32(opnd(Apk[j], m), tfrag(L::yt, db, m), gw2[j][db]);
            gw2[j][db] = mma32(opnd(dPpk[j], m), tfrag(L::et, db, m), gw2[j][db]);
            gw1[j][db] = mma32(tfrag(L::xt, db, m), opnd(dZpk, m), gw1[j][db]);
          }
        stage(L::s0, dZpk, NB * w + j);
      }
    }
    __syncthreads();
    // phase 6: dK = -eta D Wh1^T + dZ W1^T
    {
      f32x4 k1[2] = {}, k2[2] = {};
#pragma unroll
      for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int tb = 0; tb < 2; ++tb) {
          k1[tb] = mma16(sfrag(L::s1, tb, u), bh1.f[u], k1[tb]);
          k2[tb] = mma16(sfrag(L::s0, tb, u), b1.f[u], k2[tb]);
        }
      fence_sched();
      wA = load_th(0);
      float* df = reinterpret_cast<float*>(lds(L::df));
      const int d = 16 * w + l16;
#pragma unroll
      for (int tb = 0; tb < 2; ++tb)
#pragma unroll
        for (int r = 0; r < 4; ++r) df[(16 * tb + 4 * g4 + r) * FL + d] = -eta * k1[tb][r] + k2[tb][r];
    }
    __syncthreads();
    // phase 7: normalisation adjoints, dK and dV = -dY.  The next tile's
    // phase 0 writes only this thread's own row positions, so no barrier.
    store_adj(p.dK, t0, nv, L::df, L::xf, norm_k, 0, 1.0f);
    store_adj(p.dV, t0, nv, L::yf, L::vf, norm_v, 1, -1.0f);
  }

  // ------------------------------------------------ apply adjoint of chunk s-1
  ThW wB;
  if (g < n_at) wB = load_th(1);  // W2 for the dO W2^T products
  for (int t = g; t < n_at; t += G) {
    const int64_t t0 = app_start + (int64_t)t * TT;
    const int nv = min(TT, al - t * TT);
    put_row(ra, row < nv, norm_q, 0, L::xf, L::xb, L::xt);
    put_row(rb, row < nv, false, 1, -1, L::yb, L::yt);
    if (t + G < n_at) fetch_app(t + G);
    __syncthreads();
    // Zq = Q W1, dZq = (dO W2^T) s'(Zq); token sums Aq^T dO and Q^T dZq
    TdW b1;
    {
      bf16x8 xa[4], ya[4];
      xfrag(L::xb, xa);
      xfrag(L::yb, ya);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const f32x16 Zq = th(xa, wA, j);
        const f32x16 Gq = th(ya, wB, j);
        if (j == NB - 1) {
          fence_sched();
          b1 = load_td(4);
        }
        f32x16 Aq, dZq;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float z = Zq[r];
          const float sg = sigmoid(z);
          const float a = z * sg;
          Aq[r] = a;
          dZq[r] = Gq[r] * fmaf(a, 1.0f - sg, sg);
        }
        uint32_t Apq[8], dZpk[8];
        pack16(Aq, Apq);
        pack16(dZq, dZpk);
#pragma unroll
        for (int db = 0; db < 2; ++db)
#pragma unroll
          for (int m = 0; m < 2; ++m) {
            gw2[j][db] = mma32(opnd(Apq, m), tfrag(L::yt, db, m), gw2[j][db]);
            gw1[j][db] = mma32(tfrag(L::xt, db, m), opnd(dZpk, m), gw1[j][db]);
          }
        stage(L::s0, dZpk, NB * w + j);
      }
    }
    __syncthreads();
    // dQ = dZq W1^T
    {
      f32x4 q1[2] = {};
#pragma unroll
      for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int tb = 0; tb < 2; ++tb) q1[tb] = mma16(sfrag(L::s0, tb, u), b1.f[u], q1[tb]);
      if (t + G < n_at) {
        fence_sched();
        wA = load_th(0);
        wB = load_th(1);
      }
      float* df = reinterpret_cast<float*>(lds(L::df));
      const int d = 16 * w + l16;
#pragma unroll
      for (int tb = 0; tb < 2; ++tb)
#pragma unroll
        for (int r = 0; r < 4; ++r) df[(16 * tb + 4 * g4 + r) * FL + d] = q1[tb][r];
    }
    __syncthreads();
    store_adj(p.dQ, t0, nv, L::df, L::xf, norm_q, 0, 1.0f);
  }

  // ------------------------------------------------ shard partials
  float* part = p.partial + ((int64_t)slot * G + g) * (2 * DH);
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int hb = NB * w + j;
#pragma unroll
    for (int db = 0; db < 2; ++db)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int rr = c32_row(r, hf);
        part[(32 * db + rr) * HH + 32 * hb + l32] = gw1[j][db][r];
        part[DH + (32 * hb + rr) * D + 32 * db + l32] = gw2[j][db][r];
      }
  }
  float* red = reinterpret_cast<float*>(lds(L::red));
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) deta_acc += __shfl_xor(deta_acc, m, 64);
  __syncthreads();
  if ((tid & 63) == 0) red[w] = deta_acc;
  __syncthreads();
  if (tid == 0) p.partial_deta[(int64_t)slot * G + g] = red[0] + red[1] + red[2] + red[3];
}

template <typename IOT, int NB>
static hipError_t launch_bwd_step_bf_t(const BwdStepArgs& a, int n_blocks, hipStream_t st) {
  hipLaunchKernelGGL((ttt_bwd_step_bf<IOT, NB>), dim3(n_blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_bwd_step_bf(const BwdStepArgs& a, int n_blocks, int h, bool io_bf16, hipStream_t st) {
  if (h == 128)
    return io_bf16 ? launch_bwd_step_bf_t<bf16, 1>(a, n_blocks, st) : launch_bwd_step_bf_t<float, 1>(a, n_blocks, st);
  return io_bf16 ? launch_bwd_step_bf_t<bf16, 2>(a, n_blocks, st) : launch_bwd_step_bf_t<float, 2>(a, n_blocks, st);
}

}  // namespace ttt
