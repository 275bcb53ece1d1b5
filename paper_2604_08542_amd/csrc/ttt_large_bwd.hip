// Reverse mode of the chunk step at large state sizes (the MSE unit of
// Sec. 4.2 Eq. 8 with the apply of Eq. 4, differentiated for an outer loss
// <O, dO>; second-order terms through every inner gradient included).  As in
// the forward at these sizes, every product is a matrix-core GEMM over
// operands streamed from HBM with the elementwise work in its epilogue.
//
// One chunk, walking the chain backwards, with W = W_c, W' = W_{c+1} and the
// carried adjoint Wh of W' (Wh is the adjoint of W_c afterwards):
//   recompute   Z = K W1 -> A, s'(Z), s''(Z);  E = (2/M)(A W2 - V);
//               P = E W2^T -> D = P s'(Z)
//   apply       Zq = Q W1' -> Aq, s'(Zq);  Wh2 += Aq^T dO;
//               dZq = (dO W2'^T) s'(Zq);  Wh1 += Q^T dZq;  dq = dZq W1'^T
//   update      u1 = K Wh1 -> dD = -eta u1, deta -= <u1, D>,
//                             dP = dD s'(Z), dZa = dD P s''(Z)
//               u2 = A Wh2 -> dE = -eta u2, deta -= <u2, E>
//               dY = (2/M)(dE + dP W2), dv = -dY
//               dZ = dZa + (-eta E Wh2^T + dY W2^T) s'(Z)
//               dk = -eta D Wh1^T + dZ W1^T
//               Wh2 += dP^T E + A^T dY;  Wh1 += K^T dZ
//   rows        dQ, dK, dV = the L2-normalisation adjoints of dq, dk, dv
// The apply and update parts can run alone (the GCS form takes the apply
// adjoint of every chunk at W* first, then every chunk's update adjoint at W0
// against that fixed Wh, adding the weight terms to a separate total).
// Every output element is owned by one work-group summing its whole
// contraction in a fixed order; the step-size derivative is summed from
// per-tile partials in a fixed order (runs of consecutive tiles, then the
// run sums in order).  The result is deterministic.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "ttt_common.h"
#include "ttt_gemm.h"
#include "ttt_internal.h"

namespace ttt {
namespace large {
namespace bwd {

// Sum of one value per lane over the work-group, written by thread 0 to
// part[tile] (4 waves).
__device__ __forceinline__ void tile_sum(float v, float* part) {
  __shared__ float red[NTH / 64];
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// The intermediates that the update part of a reverse step writes in one
// product and reads in a later one over the same grid (S1, S2, P, dZa, and
// Sq1 of the apply part) are kept in the tile-native layout; operands of
// later products (A, Aq, D, dP, dZ, dZq) stay row-major.
template <typename T>
union Blk16 {
  T t[16];
  Native16<T> n;
};
// A = s(Z), S1 = s'(Z), S2 = s''(Z) for s = SiLU.
template <typename T>
struct EpAct3 : EpBase {
  T* a;
  T* s1;
  T* s2;
  int ld, rows;
  static constexpr bool TILED = true;
  __device__ __forceinline__ void block(int64_t blk, int row0, int col, const f32x16& z, TIn) {
    const int hf = (threadIdx.x >> 5) & 1;
    Blk16<T> v1, v2;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + c32_row(r, hf);
      float sg;
      const float av = silu_sig(z[r], sg);
      if (row < rows) put(a + (int64_t)row * ld + col, av);
      v1.t[r] = (T)fmaf(av, 1.0f - sg, sg);
      v2.t[r] = (T)(sg * (1.0f - sg) * fmaf(z[r], 1.0f - 2.0f * sg, 2.0f));
    }
    Native16<T>::store(s1, blk, v1.n);
    Native16<T>::store(s2, blk, v2.n);
  }
};
// Aq = s(Zq), Sq1 = s'(Zq).
template <typename T>
struct EpAct2 : EpBase {
  T* a;
  T* s1;
  int ld, rows;
  static constexpr bool TILED = true;
  __device__ __forceinline__ void block(int64_t blk, int row0, int col, const f32x16& z, TIn) {
    const int hf = (threadIdx.x >> 5) & 1;
    Blk16<T> v1;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + c32_row(r, hf);
      float sg;
      const float av = silu_sig(z[r], sg);
      if (row < rows) put(a + (int64_t)row * ld + col, av);
      v1.t[r] = (T)fmaf(av, 1.0f - sg, sg);
    }
    Native16<T>::store(s1, blk, v1.n);
  }
};
// E = scale (Y - V).
template <typename T>
struct EpE : EpBase {
  T* e;
  const float* v;
  int ld, rows;
  float scale;
  typedef float In;
  __device__ __forceinline__ float load(int r, int c) const { return r < rows ? v[(int64_t)r * ld + c] : 0.f; }
  __device__ __forceinline__ void operator()(int r, int c, float y, float vv) {
    if (r >= rows) return;
    put(e + (int64_t)r * ld + c, scale * (y - vv));
  }
};
// P stored, D = P S1.
template <typename T>
struct EpPD : EpBase {
  T* p;
  T* d;
  const T* s1;
  int ld, rows;
  static constexpr bool TILED = true;
  typedef Native16<T> TIn;
  __device__ __forceinline__ TIn tload(int64_t blk) const { return Native16<T>::load(s1, blk); }
  __device__ __forceinline__ void block(int64_t blk, int row0, int col, const f32x16& pv, const TIn& sn) {
    const int hf = (threadIdx.x >> 5) & 1;
    Blk16<T> sv, pp;
    sv.n = sn;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + c32_row(r, hf);
      pp.t[r] = (T)pv[r];
      if (row < rows) put(d + (int64_t)row * ld + col, pv[r] * (float)sv.t[r]);
    }
    Native16<T>::store(p, blk, pp.n);
  }
};
// out = value * fac.
template <typename T>
struct EpMul : EpBase {
  T* out;
  const T* fac;  // tile-native
  int ld, rows;
  static constexpr bool TILED = true;
  typedef Native16<T> TIn;
  __device__ __forceinline__ TIn tload(int64_t blk) const { return Native16<T>::load(fac, blk); }
  __device__ __forceinline__ void block(int64_t, int row0, int col, const f32x16& v, const TIn& fn) {
    const int hf = (threadIdx.x >> 5) & 1;
    Blk16<T> f;
    f.n = fn;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + c32_row(r, hf);
      if (row < rows) put(out + (int64_t)row * ld + col, v[r] * (float)f.t[r]);
    }
  }
};
// FP32 token-side result: out = scale * value (+ out when ADD).
template <bool ADD>
struct EpF32 : EpBase {
  float* out;
  int ld, rows;
  float scale;
  typedef float In;
  __device__ __forceinline__ float load(int r, int c) const {
    return (ADD && r < rows) ? out[(int64_t)r * ld + c] : 0.f;
  }
  __device__ __forceinline__ void operator()(int r, int c, float v, float o) {
    if (r >= rows) return;
    out[(int64_t)r * ld + c] = ADD ? o + scale * v : scale * v;
  }
};
// A product stored in the operand type.
template <typename T>
struct EpPut : EpBase {
  T* out;
  int ld, rows;
  __device__ __forceinline__ void operator()(int r, int c, float v, In) {
    if (r >= rows) return;
    put(out + (int64_t)r * ld + c, v);
  }
};
// Carried adjoint: Wh += G (or -= G) in the FP32 master, then its operand
// copy (nullable: the master only, while further terms are still to be
// added).
template <typename T>
struct EpAcc : EpBase {
  float* w;
  T* wop;
  int ld;
  float sign = 1.0f;  // -1: the term is subtracted
  typedef float In;
  __device__ __forceinline__ float load(int r, int c) const { return w[(int64_t)r * ld + c]; }
  __device__ __forceinline__ void operator()(int r, int c, float g, float wv) {
    const int64_t i = (int64_t)r * ld + c;
    const float wn = fmaf(sign, g, wv);
    w[i] = wn;
    if (wop) put(wop + i, wn);
  }
};
// u1 = K Wh1: dD = -eta u1, dP = dD S1, dZa = dD P S2; -<u1, D> into the
// step-size partials.
template <typename T>
struct EpU1 {
  T* dp;
  T* dza;
  const T* d;
  const T* s1;
  const T* p;
  const T* s2;
  float* part;
  int ld, rows;
  float eta;
  float acc = 0.f;
  // S1, P, S2 and dZa tile-native; D (an operand of a later product) and dP
  // row-major
  static constexpr bool TILED = true;
  struct TIn {
    Native16<T> s1, p, s2;
  };
  __device__ __forceinline__ TIn tload(int64_t blk) const {
    return {Native16<T>::load(s1, blk), Native16<T>::load(p, blk), Native16<T>::load(s2, blk)};
  }
  __device__ __forceinline__ void block(int64_t blk, int row0, int col, const f32x16& u, const TIn& x) {
    const int hf = (threadIdx.x >> 5) & 1;
    Blk16<T> vs1, vp, vs2, vz;
    vs1.n = x.s1;
    vp.n = x.p;
    vs2.n = x.s2;
    T dv[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + c32_row(r, hf);
      dv[r] = row < rows ? d[(int64_t)row * ld + col] : T(0.f);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + c32_row(r, hf);
      const float dd = -eta * u[r];
      vz.t[r] = (T)(dd * (float)vp.t[r] * (float)vs2.t[r]);
      if (row < rows) {
        acc = fmaf(-u[r], (float)dv[r], acc);
        put(dp + (int64_t)row * ld + col, dd * (float)vs1.t[r]);
      }
    }
    Native16<T>::store(dza, blk, vz.n);
  }
  __device__ __forceinline__ void finish() { tile_sum(acc, part); }
};
// u2 = A Wh2: dE = -eta u2 (FP32); -<u2, E> into the step-size partials.
template <typename T>
struct EpU2 {
  float* de;
  const T* e;
  float* part;
  int ld, rows;
  float eta;
  float acc = 0.f;
  typedef T In;
  __device__ __forceinline__ T load(int r, int c) const { return r < rows ? e[(int64_t)r * ld + c] : T(0.f); }
  __device__ __forceinline__ void operator()(int r, int c, float u, T ev) {
    if (r >= rows) return;
    acc = fmaf(-u, (float)ev, acc);
    de[(int64_t)r * ld + c] = -eta * u;
  }
  __device__ __forceinline__ void finish() { tile_sum(acc, part); }
};
// dP W2: dY = scale (dE + dP W2) (operand type), dv = -dY (FP32).
template <typename T>
struct EpDY : EpBase {
  T* dy;
  float* dv;
  const float* de;
  int ld, rows;
  float scale;
  typedef float In;
  __device__ __forceinline__ float load(int r, int c) const { return r < rows ? de[(int64_t)r * ld + c] : 0.f; }
  __device__ __forceinline__ void operator()(int r, int c, float v, float dev) {
    if (r >= rows) return;
    const int64_t i = (int64_t)r * ld + c;
    const float y = scale * (dev + v);
    put(dy + i, y);
    dv[i] = -y;
  }
};
// dY W2^T: dA = -eta EWh + dY W2^T, dZ = dZa + dA S1.
template <typename T>
struct EpDZ : EpBase {
  T* dz;
  const T* ewh;
  const T* dza;
  const T* s1;
  int ld, rows;
  float eta;
  // dZa and S1 tile-native, EWh row-major
  static constexpr bool TILED = true;
  struct TIn {
    Native16<T> dza, s1;
  };
  __device__ __forceinline__ TIn tload(int64_t blk) const {
    return {Native16<T>::load(dza, blk), Native16<T>::load(s1, blk)};
  }
  __device__ __forceinline__ void block(int64_t, int row0, int col, const f32x16& v, const TIn& x) {
    const int hf = (threadIdx.x >> 5) & 1;
    Blk16<T> vz, vs1;
    vz.n = x.dza;
    vs1.n = x.s1;
    T ev[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + c32_row(r, hf);
      ev[r] = row < rows ? ewh[(int64_t)row * ld + col] : T(0.f);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + c32_row(r, hf);
      if (row >= rows) continue;
      const float da = fmaf(-eta, (float)ev[r], v[r]);
      put(dz + (int64_t)row * ld + col, fmaf(da, (float)vs1.t[r], (float)vz.t[r]));
    }
  }
};

// dO rows of the chunk in the operand type ([rows][d]; one wave per row).
template <typename IOT, typename T>
__global__ __launch_bounds__(256) void k_rows(const IOT* src, int64_t stride_tok, T* dst, int rows, int d) {
  typedef IOT iov4 __attribute__((ext_vector_type(4)));
  typedef T opv4 __attribute__((ext_vector_type(4)));
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (row >= rows) return;
  for (int c = 4 * l; c < d; c += 256) {
    const iov4 v = *reinterpret_cast<const iov4*>(src + (int64_t)row * stride_tok + c);
    *reinterpret_cast<opv4*>(dst + (int64_t)row * d + c) = (opv4){(T)(float)v[0], (T)(float)v[1], (T)(float)v[2],
                                                                  (T)(float)v[3]};
  }
}

// Adjoint of the row normalisation x / max(||x||, eps) for the chunk's Q, K, V
// rows: (g - xhat <xhat, g>) / ||x|| where ||x|| > eps, g / eps where the
// floor is active, g itself for a tensor that is not normalised.  One wave per
// token, 4 consecutive elements per lane, at most 16 passes of 256.
template <typename IOT>
__global__ __launch_bounds__(256) void k_norm_bwd(LargeBwdArgs p) {
  typedef IOT iov4 __attribute__((ext_vector_type(4)));
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (row >= p.rows) return;
  const int passes = p.d / 256;
  for (int which = 0; which < 3; ++which) {
    if (which < 2 ? !p.update : !p.apply) continue;
    const IOT* src = static_cast<const IOT*>(which == 0 ? p.K : which == 1 ? p.V : p.Q) +
                     (int64_t)row * p.stride_tok;
    IOT* dst = static_cast<IOT*>(which == 0 ? p.dK : which == 1 ? p.dV : p.dQ) + (int64_t)row * p.stride_tok;
    const float* g = (which == 0 ? p.dk : which == 1 ? p.dv : p.dq) + (int64_t)row * p.d;
    const bool nrm = (p.flags >> (which == 0 ? 1 : which == 1 ? 2 : 0)) & 1u;
    f32x4 x[16], gv[16];
    float ss = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if (i < passes) {
        const iov4 v = *reinterpret_cast<const iov4*>(src + 256 * i + 4 * l);
        x[i] = (f32x4){(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
        gv[i] = *reinterpret_cast<const f32x4*>(g + 256 * i + 4 * l);
#pragma unroll
        for (int e = 0; e < 4; ++e) ss = fmaf(x[i][e], x[i][e], ss);
      }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) ss += __shfl_xor(ss, m, 64);
    const float n = sqrtf(ss);
    const bool above = n > NORM_EPS;
    const float inv = 1.0f / fmaxf(n, NORM_EPS);
    float proj = 0.f;
    if (nrm && above) {
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (i < passes)
#pragma unroll
          for (int e = 0; e < 4; ++e) proj = fmaf(x[i][e] * inv, gv[i][e], proj);
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) proj += __shfl_xor(proj, m, 64);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if (i < passes) {
        f32x4 y = gv[i];
        if (nrm) {
          if (above) {
#pragma unroll
            for (int e = 0; e < 4; ++e) y[e] = (gv[i][e] - x[i][e] * inv * proj) * inv;
          } else {
            y = gv[i] * (1.0f / NORM_EPS);
          }
        }
        *reinterpret_cast<iov4*>(dst + 256 * i + 4 * l) = (iov4){(IOT)y[0], (IOT)y[1], (IOT)y[2], (IOT)y[3]};
      }
    }
  }
}

// *deta += (the n step-size partials, summed in a fixed order); one work-group
__global__ __launch_bounds__(NTH) void k_deta(const float* part, int n, float* deta) {
  const float s = fixed_order_sum(part, n);
  if (threadIdx.x == 0) *deta += s;
}

__global__ void k_add(const float* src, float* dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] += src[i];
}

__global__ void k_zero(float* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

template <typename T, typename IOT>
hipError_t step_t(const LargeBwdArgs& a, hipStream_t st) {
  const int M = a.rows, d = a.d, h = a.h;
  constexpr int BMT = 128, BMW = 128;
  const int mt = (M + BMT - 1) / BMT;
  const float eta = a.eta, scale = 2.0f / (float)M;
  T* Kn = static_cast<T*>(a.Kn);
  T* Qn = static_cast<T*>(a.Qn);
  T* E = static_cast<T*>(a.E);
  T* dOn = static_cast<T*>(a.dOn);
  T* dY = static_cast<T*>(a.dY);
  T* A = static_cast<T*>(a.A);
  T* S1 = static_cast<T*>(a.S1);
  T* S2 = static_cast<T*>(a.S2);
  T* P = static_cast<T*>(a.P);
  T* D = static_cast<T*>(a.D);
  T* Aq = static_cast<T*>(a.Aq);
  T* Sq1 = static_cast<T*>(a.Sq1);
  T* dZq = static_cast<T*>(a.dZq);
  T* dP = static_cast<T*>(a.dP);
  T* dZa = static_cast<T*>(a.dZa);
  T* EWh = static_cast<T*>(a.EWh);
  T* dZ = static_cast<T*>(a.dZ);
  const T* W1 = static_cast<const T*>(a.W1op);
  const T* W2 = static_cast<const T*>(a.W2op);
  const T* W1n = static_cast<const T*>(a.W1nop);
  const T* W2n = static_cast<const T*>(a.W2nop);
  T* Wh1o = static_cast<T*>(a.Wh1op);
  T* Wh2o = static_cast<T*>(a.Wh2op);
  const dim3 gh(h / BN, mt), gd(d / BN, mt), nt(NTH);
  // rows of the chunk
  LargeNormArgs na{a.K, a.V, a.Q, a.stride_tok, a.flags, M, d, a.Kn, a.Vn, a.Qn};
  const hipError_t en = launch_large_norm(na, std::is_same_v<IOT, bf16>, std::is_same_v<T, bf16>, st);
  if (en != hipSuccess) return en;
  if (a.apply)
    hipLaunchKernelGGL((k_rows<IOT, T>), dim3((M + 3) / 4), dim3(256), 0, st, static_cast<const IOT*>(a.dO),
                       a.stride_tok, dOn, M, d);
  if (a.update) {
    // recompute the chunk's gradient terms at W_c
    EpAct3<T> e1{{}, A, S1, S2, h, M};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpAct3<T>>), gh, nt, 0, st, Kn, d, M, W1, h, d, d, e1);
    EpE<T> e2{{}, E, a.Vn, d, M, scale};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpE<T>>), gd, nt, 0, st, A, h, M, W2, d, h, h, e2);
    EpPD<T> e3{{}, P, D, S1, h, M};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, BMT, EpPD<T>>), gh, nt, 0, st, E, d, M, W2, d, h, d, e3);
  }
  if (a.apply) {
    // apply adjoint at W_{c+1}
    EpAct2<T> e4{{}, Aq, Sq1, h, M};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpAct2<T>>), gh, nt, 0, st, Qn, d, M, W1n, h, d, d, e4);
    EpAcc<T> e5{{}, a.Wh2, Wh2o, d};
    hipLaunchKernelGGL((k_gemm<T, MNMAJ, MNMAJ, BMW, EpAcc<T>>), dim3(d / BN, h / BMW), nt, 0, st, Aq, h, M, dOn, d, M,
                       M, e5);
    EpMul<T> e6{{}, dZq, Sq1, h, M};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, BMT, EpMul<T>>), gh, nt, 0, st, dOn, d, M, W2n, d, h, d, e6);
    EpAcc<T> e7{{}, a.Wh1, Wh1o, h};
    hipLaunchKernelGGL((k_gemm<T, MNMAJ, MNMAJ, BMW, EpAcc<T>>), dim3(h / BN, d / BMW), nt, 0, st, Qn, d, M, dZq, h, M,
                       M, e7);
    EpF32<false> e8{{}, a.dq, d, M, 1.0f};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, BMT, EpF32<false>>), gd, nt, 0, st, dZq, h, M, W1n, h, d, h, e8);
  }
  if (a.update) {
    // update adjoint at W_c along Wh
    EpU1<T> e9{dP, dZa, D, S1, P, S2, a.deta_part, h, M, eta};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpU1<T>>), gh, nt, 0, st, Kn, d, M, Wh1o, h, d, d, e9);
    EpU2<T> e10{a.dE, E, a.deta_part + (h / BN) * mt, d, M, eta};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpU2<T>>), gd, nt, 0, st, A, h, M, Wh2o, d, h, h, e10);
    hipLaunchKernelGGL(k_deta, dim3(1), dim3(NTH), 0, st, a.deta_part, (h / BN + d / BN) * mt, a.deta);
    EpDY<T> e11{{}, dY, a.dv, a.dE, d, M, scale};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpDY<T>>), gd, nt, 0, st, dP, h, M, W2, d, h, h, e11);
    EpPut<T> e12{{}, EWh, h, M};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, BMT, EpPut<T>>), gh, nt, 0, st, E, d, M, Wh2o, d, h, d, e12);
    EpDZ<T> e13{{}, dZ, EWh, dZa, S1, h, M, eta};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, BMT, EpDZ<T>>), gh, nt, 0, st, dY, d, M, W2, d, h, d, e13);
    EpF32<false> e14{{}, a.dk, d, M, -eta};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, BMT, EpF32<false>>), gd, nt, 0, st, D, h, M, Wh1o, h, d, h, e14);
    EpF32<true> e15{{}, a.dk, d, M, 1.0f};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, BMT, EpF32<true>>), gd, nt, 0, st, dZ, h, M, W1, h, d, h, e15);
    // the weight terms of the update adjoint (the adjoint of W_c in the chain)
    EpAcc<T> e16{{}, a.Acc2, nullptr, d};
    hipLaunchKernelGGL((k_gemm<T, MNMAJ, MNMAJ, BMW, EpAcc<T>>), dim3(d / BN, h / BMW), nt, 0, st, dP, h, M, E, d, M, M,
                       e16);
    EpAcc<T> e17{{}, a.Acc2, static_cast<T*>(a.Acc2op), d};
    hipLaunchKernelGGL((k_gemm<T, MNMAJ, MNMAJ, BMW, EpAcc<T>>), dim3(d / BN, h / BMW), nt, 0, st, A, h, M, dY, d, M, M,
                       e17);
    EpAcc<T> e18{{}, a.Acc1, static_cast<T*>(a.Acc1op), h};
    hipLaunchKernelGGL((k_gemm<T, MNMAJ, MNMAJ, BMW, EpAcc<T>>), dim3(h / BN, d / BMW), nt, 0, st, Kn, d, M, dZ, h, M,
                       M, e18);
  }
  // gradients of the raw rows
  hipLaunchKernelGGL(k_norm_bwd<IOT>, dim3((M + 3) / 4), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ the paper's unit
// Reverse step of one chunk of the SwiGLU unit with the dot-product loss
// (Supp. A; Sec. 4.2 Eq. 8-10).  With W = W_c, W' = W_{c+1}, the adjoint Wh
// of W' and E_i = -eta_i v_i:
//   apply    Zq3 = Q W3', Zq1 = Q W1' -> Hq = s(Zq1) Zq3;  dHq = dO W2'^T
//            -> dZq1 = dHq Zq3 s'(Zq1), dZq3 = dHq s(Zq1);
//            Wh1 += Q^T dZq1, Wh2 += Hq^T dO, Wh3 += Q^T dZq3;
//            dq = dZq1 W1'^T + dZq3 W3'^T
//   update   the gradient G of L = sum_i <f_W(k_i), E_i> enters W_{c+1} = W - G,
//            so the adjoint of W gains -(dG/dW)^T Wh, the gradient of the
//            derivative of L along Wh (tangents Zd1 = K Wh1, Zd3 = K Wh3,
//            Sd = s'(Z1) Zd1, Hdot = Sd Z3 + s(Z1) Zd3, Ydot = Hdot W2 + Hd Wh2):
//            dH = E W2^T, dHh = E Wh2^T;  aSd = dH Z3, aZ3 = dH Sd + dHh S,
//            aS = dH Zd3 + dHh Z3, aZd3 = dH S, aZd1 = aSd s'(Z1),
//            aZ1 = aSd s''(Z1) Zd1 + aS s'(Z1);
//            W1 -= K^T aZ1, W2 -= Hdot^T E, W3 -= K^T aZ3;
//            dk = -(aZ1 W1^T + aZ3 W3^T + aZd1 Wh1^T + aZd3 Wh3^T);
//            dv_i = eta_i Ydot_i, deta_i = <v_i, Ydot_i>
namespace amu {

// Z1 -> S = s(Z1), S1 = s'(Z1), S2 = s''(Z1), Hd = S Z3 (Z3 loaded).
template <typename T>
struct EpZ1 : EpBase {  // Z3, Sv, S1, S2 tile-native; Hd row-major (an operand)
  const T* z3;
  T* sv;
  T* s1;
  T* s2;
  T* hd;
  int ld, rows;
  static constexpr bool TILED = true;
  __device__ __forceinline__ void block(int64_t blk, int row0, int col, const f32x16& z, TIn) {
    const int hf = (threadIdx.x >> 5) & 1;
    Blk16<T> z3v, vs, v1, v2;
    z3v.n = Native16<T>::load(z3, blk);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + c32_row(r, hf);
      float sg;
      const float a = silu_sig(z[r], sg);
      vs.t[r] = (T)a;
      v1.t[r] = (T)fmaf(a, 1.0f - sg, sg);
      v2.t[r] = (T)(sg * (1.0f - sg) * fmaf(z[r], 1.0f - 2.0f * sg, 2.0f));
      if (row < rows) put(hd + (int64_t)row * ld + col, a * (float)z3v.t[r]);
    }
    Native16<T>::store(sv, blk, vs.n);
    Native16<T>::store(s1, blk, v1.n);
    Native16<T>::store(s2, blk, v2.n);
  }
};
// Zd1 = K Wh1 -> Sd = S1 Zd1, Hdot = Sd Z3 + S Zd3, T2 = S2 Zd1.
template <typename T>
struct EpZd1 : EpBase {  // inputs and Sd, T2 tile-native; Hdot row-major (an operand)
  const T* s1;
  const T* z3;
  const T* sv;
  const T* zd3;
  const T* s2;
  T* sd;
  T* hdot;
  T* t2;
  int ld, rows;
  static constexpr bool TILED = true;
  __device__ __forceinline__ void block(int64_t blk, int row0, int col, const f32x16& zd1, TIn) {
    const int hf = (threadIdx.x >> 5) & 1;
    Blk16<T> x1, xz3, xs, xzd3, x2, osd, ot2;
    x1.n = Native16<T>::load(s1, blk);
    xz3.n = Native16<T>::load(z3, blk);
    xs.n = Native16<T>::load(sv, blk);
    xzd3.n = Native16<T>::load(zd3, blk);
    x2.n = Native16<T>::load(s2, blk);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + c32_row(r, hf);
      const float sdv = (float)x1.t[r] * zd1[r];
      osd.t[r] = (T)sdv;
      ot2.t[r] = (T)((float)x2.t[r] * zd1[r]);
      if (row < rows)
        put(hdot + (int64_t)row * ld + col, fmaf(sdv, (float)xz3.t[r], (float)xs.t[r] * (float)xzd3.t[r]));
    }
    Native16<T>::store(sd, blk, osd.n);
    Native16<T>::store(t2, blk, ot2.n);
  }
};
// dH = E W2^T with dHh = E Wh2^T loaded: the adjoints aZ1, aZ3, aZd1, aZd3.
template <typename T>
struct EpAdj : EpBase {  // inputs tile-native; the four adjoints row-major (operands)
  const T* z3;
  const T* sd;
  const T* sv;
  const T* zd3;
  const T* dhh;
  const T* s1;
  const T* t2;
  T* az1;
  T* az3;
  T* azd1;
  T* azd3;
  int ld, rows;
  static constexpr bool TILED = true;
  __device__ __forceinline__ void block(int64_t blk, int row0, int col, const f32x16& dh, TIn) {
    const int hf = (threadIdx.x >> 5) & 1;
    Blk16<T> xz3, xsd, xs, xzd3, xdhh, x1, xt2;
    xz3.n = Native16<T>::load(z3, blk);
    xsd.n = Native16<T>::load(sd, blk);
    xs.n = Native16<T>::load(sv, blk);
    xzd3.n = Native16<T>::load(zd3, blk);
    xdhh.n = Native16<T>::load(dhh, blk);
    x1.n = Native16<T>::load(s1, blk);
    xt2.n = Native16<T>::load(t2, blk);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + c32_row(r, hf);
      if (row >= rows) continue;
      const int64_t i = (int64_t)row * ld + col;
      const float z3v = (float)xz3.t[r], sdv = (float)xsd.t[r], sa = (float)xs.t[r], zd3v = (float)xzd3.t[r],
                  dhv = (float)xdhh.t[r], s1v = (float)x1.t[r];
      const float asd = dh[r] * z3v;
      const float as = fmaf(dh[r], zd3v, dhv * z3v);
      put(az3 + i, fmaf(dh[r], sdv, dhv * sa));
      put(azd3 + i, dh[r] * sa);
      put(azd1 + i, asd * s1v);
      put(az1 + i, fmaf(asd, (float)xt2.t[r], as * s1v));
    }
  }
};
// Apply: Zq1 -> Hq = s(Zq1) Zq3, F1 = Zq3 s'(Zq1), F3 = s(Zq1) (Zq3 loaded).
template <typename T>
struct EpQ1 : EpBase {  // Zq3 in, F1, F3 out tile-native; Hq row-major (an operand)
  const T* z3;
  T* hq;
  T* f1;
  T* f3;
  int ld, rows;
  static constexpr bool TILED = true;
  typedef Native16<T> TIn;
  __device__ __forceinline__ TIn tload(int64_t blk) const { return Native16<T>::load(z3, blk); }
  __device__ __forceinline__ void block(int64_t blk, int row0, int col, const f32x16& z, const TIn& zn) {
    const int hf = (threadIdx.x >> 5) & 1;
    Blk16<T> z3v, o1, o3;
    z3v.n = zn;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + c32_row(r, hf);
      float sg;
      const float a = silu_sig(z[r], sg);
      const float zz = (float)z3v.t[r];
      o1.t[r] = (T)(zz * fmaf(a, 1.0f - sg, sg));
      o3.t[r] = (T)a;
      if (row < rows) put(hq + (int64_t)row * ld + col, a * zz);
    }
    Native16<T>::store(f1, blk, o1.n);
    Native16<T>::store(f3, blk, o3.n);
  }
};
// dHq = dO W2'^T -> dZq1 = dHq F1, dZq3 = dHq F3.
template <typename T>
struct EpQ2 : EpBase {  // F1, F3 tile-native; dZq1, dZq3 row-major (operands)
  const T* f1;
  const T* f3;
  T* d1;
  T* d3;
  int ld, rows;
  static constexpr bool TILED = true;
  struct TIn {
    Native16<T> a, b;
  };
  __device__ __forceinline__ TIn tload(int64_t blk) const { return {Native16<T>::load(f1, blk), Native16<T>::load(f3, blk)}; }
  __device__ __forceinline__ void block(int64_t, int row0, int col, const f32x16& v, const TIn& f) {
    const int hf = (threadIdx.x >> 5) & 1;
    Blk16<T> a, b;
    a.n = f.a;
    b.n = f.b;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + c32_row(r, hf);
      if (row >= rows) continue;
      const int64_t i = (int64_t)row * ld + col;
      put(d1 + i, v[r] * (float)a.t[r]);
      put(d3 + i, v[r] * (float)b.t[r]);
    }
  }
};

// The product stored in the tile-native layout (Z3, Zd3, dHh of the paper
// unit's reverse step, read by the epilogues above over the same grid).
template <typename T>
struct EpPutTiled : EpBase {
  T* z;
  static constexpr bool TILED = true;
  __device__ __forceinline__ void block(int64_t blk, int, int, const f32x16& v, TIn) {
    Blk16<T> o;
#pragma unroll
    for (int r = 0; r < 16; ++r) o.t[r] = (T)v[r];
    Native16<T>::store(z, blk, o.n);
  }
};

// E = -eta_i Vn_i (operand type) of the chunk's rows.
template <typename T>
__global__ __launch_bounds__(256) void k_e(T* e, const float* vn, const float* eta, int64_t eta_stride, int rows,
                                           int d) {
  const int64_t n = (int64_t)rows * d;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    e[i] = (T)(-eta[(i / d) * eta_stride] * vn[i]);
}

// Per token: dv = eta_i Ydot_i, deta_i = <v_i, Ydot_i> (one wave per token).
__global__ __launch_bounds__(256) void k_ydot(LargeAmuBwdArgs p) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (row >= p.rows) return;
  const float et = p.eta[(int64_t)row * p.eta_stride];
  float s = 0.f;
  for (int c = 4 * l; c < p.d; c += 256) {
    const int64_t i = (int64_t)row * p.d + c;
    const f32x4 y = *reinterpret_cast<const f32x4*>(p.Ydot + i);
    const f32x4 v = *reinterpret_cast<const f32x4*>(p.Vn + i);
#pragma unroll
    for (int e = 0; e < 4; ++e) s = fmaf(v[e], y[e], s);
    *reinterpret_cast<f32x4*>(p.dv + i) = et * y;
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
  if (l == 0) p.deta[(int64_t)row * p.eta_stride] = s;
}

template <typename T, typename IOT>
hipError_t step_t(const LargeAmuBwdArgs& a, hipStream_t st) {
  const int M = a.rows, d = a.d, h = a.h;
  constexpr int BMT = 128, BMW = 128;
  const int mt = (M + BMT - 1) / BMT;
  auto P = [](void* q) { return static_cast<T*>(q); };
  auto C = [](const void* q) { return static_cast<const T*>(q); };
  T* Kn = P(a.Kn);
  T* Qn = P(a.Qn);
  T* E = P(a.E);
  T* dOn = P(a.dOn);
  T *Z3 = P(a.Z3), *Sv = P(a.S), *S1 = P(a.S1), *S2 = P(a.S2), *Hd = P(a.Hd), *Zd3 = P(a.Zd3), *Sd = P(a.Sd),
    *Hdot = P(a.Hdot), *T2 = P(a.T2), *dHh = P(a.dHh), *aZ1 = P(a.aZ1), *aZ3 = P(a.aZ3), *aZd1 = P(a.aZd1),
    *aZd3 = P(a.aZd3);
  const T *W1 = C(a.Wop[0]), *W2 = C(a.Wop[1]), *W3 = C(a.Wop[2]);
  const T *W1n = C(a.Wnop[0]), *W2n = C(a.Wnop[1]), *W3n = C(a.Wnop[2]);
  T *Wh1o = P(a.Whop[0]), *Wh2o = P(a.Whop[1]), *Wh3o = P(a.Whop[2]);
  const dim3 gh(h / BN, mt), gd(d / BN, mt), gwh(h / BN, d / BMW), gwd(d / BN, h / BMW), nt(NTH);
  LargeNormArgs na{a.K, a.V, a.Q, a.stride_tok, a.flags, M, d, a.Kn, a.Vn, a.Qn};
  const hipError_t en = launch_large_norm(na, std::is_same_v<IOT, bf16>, std::is_same_v<T, bf16>, st);
  if (en != hipSuccess) return en;
  if (a.apply) {
    hipLaunchKernelGGL((k_rows<IOT, T>), dim3((M + 3) / 4), dim3(256), 0, st, static_cast<const IOT*>(a.dO),
                       a.stride_tok, dOn, M, d);
    EpPutTiled<T> q3{{}, Z3};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpPutTiled<T>>), gh, nt, 0, st, Qn, d, M, W3n, h, d, d, q3);
    EpQ1<T> q1{{}, Z3, Hd, S1, Sv, h, M};  // Hq, F1, F3
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpQ1<T>>), gh, nt, 0, st, Qn, d, M, W1n, h, d, d, q1);
    EpQ2<T> q2{{}, S1, Sv, aZ1, aZ3, h, M};  // dZq1, dZq3
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, BMT, EpQ2<T>>), gh, nt, 0, st, dOn, d, M, W2n, d, h, d, q2);
    EpAcc<T> w1{{}, a.Wh[0], Wh1o, h};
    hipLaunchKernelGGL((k_gemm<T, MNMAJ, MNMAJ, BMW, EpAcc<T>>), gwh, nt, 0, st, Qn, d, M, aZ1, h, M, M, w1);
    EpAcc<T> w2{{}, a.Wh[1], Wh2o, d};
    hipLaunchKernelGGL((k_gemm<T, MNMAJ, MNMAJ, BMW, EpAcc<T>>), gwd, nt, 0, st, Hd, h, M, dOn, d, M, M, w2);
    EpAcc<T> w3{{}, a.Wh[2], Wh3o, h};
    hipLaunchKernelGGL((k_gemm<T, MNMAJ, MNMAJ, BMW, EpAcc<T>>), gwh, nt, 0, st, Qn, d, M, aZ3, h, M, M, w3);
    EpF32<false> g1{{}, a.dq, d, M, 1.0f};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, BMT, EpF32<false>>), gd, nt, 0, st, aZ1, h, M, W1n, h, d, h, g1);
    EpF32<true> g3{{}, a.dq, d, M, 1.0f};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, BMT, EpF32<true>>), gd, nt, 0, st, aZ3, h, M, W3n, h, d, h, g3);
  }
  if (a.update) {
    EpPutTiled<T> u1{{}, Z3};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpPutTiled<T>>), gh, nt, 0, st, Kn, d, M, W3, h, d, d, u1);
    EpZ1<T> u2{{}, Z3, Sv, S1, S2, Hd, h, M};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpZ1<T>>), gh, nt, 0, st, Kn, d, M, W1, h, d, d, u2);
    EpPutTiled<T> u3{{}, Zd3};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpPutTiled<T>>), gh, nt, 0, st, Kn, d, M, Wh3o, h, d, d, u3);
    EpZd1<T> u4{{}, S1, Z3, Sv, Zd3, S2, Sd, Hdot, T2, h, M};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpZd1<T>>), gh, nt, 0, st, Kn, d, M, Wh1o, h, d, d, u4);
    const int64_t ne = (int64_t)M * d;
    hipLaunchKernelGGL(k_e<T>, dim3((unsigned)std::min<int64_t>((ne + 255) / 256, 4096)), dim3(256), 0, st, E, a.Vn,
                       a.eta, a.eta_stride, M, d);
    EpF32<false> y1{{}, a.Ydot, d, M, 1.0f};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpF32<false>>), gd, nt, 0, st, Hdot, h, M, W2, d, h, h, y1);
    EpF32<true> y2{{}, a.Ydot, d, M, 1.0f};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpF32<true>>), gd, nt, 0, st, Hd, h, M, Wh2o, d, h, h, y2);
    hipLaunchKernelGGL(k_ydot, dim3((M + 3) / 4), dim3(256), 0, st, a);
    EpPutTiled<T> u8{{}, dHh};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, BMT, EpPutTiled<T>>), gh, nt, 0, st, E, d, M, Wh2o, d, h, d, u8);
    EpAdj<T> u9{{}, Z3, Sd, Sv, Zd3, dHh, S1, T2, aZ1, aZ3, aZd1, aZd3, h, M};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, BMT, EpAdj<T>>), gh, nt, 0, st, E, d, M, W2, d, h, d, u9);
    // dk (uses Wh before the weight terms below change it, in the chain)
    EpF32<false> k1{{}, a.dk, d, M, -1.0f};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, BMT, EpF32<false>>), gd, nt, 0, st, aZ1, h, M, W1, h, d, h, k1);
    EpF32<true> k3{{}, a.dk, d, M, -1.0f};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, BMT, EpF32<true>>), gd, nt, 0, st, aZ3, h, M, W3, h, d, h, k3);
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, BMT, EpF32<true>>), gd, nt, 0, st, aZd1, h, M, Wh1o, h, d, h, k3);
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, BMT, EpF32<true>>), gd, nt, 0, st, aZd3, h, M, Wh3o, h, d, h, k3);
    // the weight terms: W1 -= K^T aZ1, W2 -= Hdot^T E, W3 -= K^T aZ3
    EpAcc<T> a1{{}, a.Acc[0], P(a.Accop[0]), h, -1.0f};
    hipLaunchKernelGGL((k_gemm<T, MNMAJ, MNMAJ, BMW, EpAcc<T>>), gwh, nt, 0, st, Kn, d, M, aZ1, h, M, M, a1);
    EpAcc<T> a2{{}, a.Acc[1], P(a.Accop[1]), d, -1.0f};
    hipLaunchKernelGGL((k_gemm<T, MNMAJ, MNMAJ, BMW, EpAcc<T>>), gwd, nt, 0, st, Hdot, h, M, E, d, M, M, a2);
    EpAcc<T> a3{{}, a.Acc[2], P(a.Accop[2]), h, -1.0f};
    hipLaunchKernelGGL((k_gemm<T, MNMAJ, MNMAJ, BMW, EpAcc<T>>), gwh, nt, 0, st, Kn, d, M, aZ3, h, M, M, a3);
  }
  // gradients of the raw rows: only the parts that ran
  LargeBwdArgs nb{};
  nb.K = a.K; nb.V = a.V; nb.Q = a.Q; nb.dQ = a.dQ; nb.dK = a.dK; nb.dV = a.dV;
  nb.stride_tok = a.stride_tok; nb.flags = a.flags; nb.rows = M; nb.d = d;
  nb.dq = a.dq; nb.dk = a.dk; nb.dv = a.dv; nb.apply = a.apply; nb.update = a.update;
  hipLaunchKernelGGL(k_norm_bwd<IOT>, dim3((M + 3) / 4), dim3(256), 0, st, nb);
  return hipGetLastError();
}

}  // namespace amu
}  // namespace bwd
}  // namespace large

hipError_t launch_large_bwd_step(const LargeBwdArgs& a, bool io_bf16, bool mma_bf16, hipStream_t st) {
  using namespace large::bwd;
  if (mma_bf16) return io_bf16 ? step_t<bf16, bf16>(a, st) : step_t<bf16, float>(a, st);
  return step_t<float, float>(a, st);
}

hipError_t launch_large_amu_bwd_step(const LargeAmuBwdArgs& a, bool io_bf16, bool mma_bf16, hipStream_t st) {
  using namespace large::bwd;
  if (mma_bf16) return io_bf16 ? amu::step_t<bf16, bf16>(a, st) : amu::step_t<bf16, float>(a, st);
  return amu::step_t<float, float>(a, st);
}

hipError_t launch_large_zero(float* p, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(large::bwd::k_zero, dim3(1024), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_large_add(const float* src, float* dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(large::bwd::k_add, dim3(1024), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

}  // namespace ttt
