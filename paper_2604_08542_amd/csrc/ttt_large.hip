// Chunk step at the paper's state size (Supp. A: one head of hd = 1024 with
// a hidden width of 4 hd), where the fast weights (W1: [d][h], W2: [h][d],
// 16 MiB each in FP32) cannot stay on chip: every product of the chunk step
// (Sec. 4.2 Eq. 8, Sec. 3.2 Eq. 3-4) is a matrix-core GEMM over operands
// streamed from HBM, with the elementwise work fused into its epilogue.
//
// Per chunk (M_c tokens):
//   norm   K, V, Q rows / max(||row||, eps)                      (FP32)
//   Z      Z = K W1           -> A = SiLU(Z), S1 = SiLU'(Z)
//   Y      Y = A W2           -> R = Y - V, E = (2/M_c) R, loss partials
//   P      P = E W2^T         -> D = P * S1
//   gW1    W1 -= eta K^T D    (FP32 master updated in the epilogue)
//   gW2    W2 -= eta A^T E
//   Zq     Zq = Q W1'         -> Aq = SiLU(Zq)
//   O      O = Aq W2'
// The paper's memory unit (Supp. A: f_W(x) = (SiLU(x W1) * (x W3)) W2, the
// dot-product loss with token-wise step sizes, W <- W - grad) runs the same
// way; E = -eta_i v_i does not depend on W, so its gradient needs no
// contraction over the hidden axis before the hidden adjoint:
//   Z3     Z3 = K W3          (stored)
//   Z1     Z1 = K W1          -> Hd = SiLU(Z1) Z3, G1 = Z3 SiLU'(Z1), G3 = SiLU(Z1)
//   E      E = -eta_i Vn_i
//   dH     dH = E W2^T        -> D1 = dH G1, D3 = dH G3
//   gW     W1 -= K^T D1, W3 -= K^T D3, W2 -= Hd^T E
//   apply  Zq3 = Q W3', Hq = SiLU(Q W1') Zq3, O = Hq W2'
// The masters stay FP32; the matrix-core operands are BF16 copies (or FP32
// with FP32 matrix cores).  Each output element of every product is owned by
// one work-group, which sums its whole contraction in a fixed order, so the
// result is deterministic.
#include <hip/hip_runtime.h>

#include "ttt_common.h"
#include "ttt_gemm.h"
#include "ttt_internal.h"

namespace ttt {
namespace large {

// ------------------------------------------------------------- epilogues
// A = SiLU(Z), S1 = SiLU'(Z) (for the gradient; S1 in the tile-native
// layout, read back by EpD in the same grid) or only A (for the apply).
template <typename T, bool GRAD>
struct EpAct : EpBase {
  T* a;
  T* s1;
  int ld, rows;
  static constexpr bool TILED = GRAD;
  __device__ __forceinline__ void operator()(int r, int c, float z, In) {
    if (r >= rows) return;
    float sg;
    const float av = silu_sig(z, sg);
    put(a + (int64_t)r * ld + c, av);
  }
  __device__ __forceinline__ void block(int64_t blk, int row0, int col, const f32x16& z, TIn) {
    const int hf = (threadIdx.x >> 5) & 1;
    union {
      T t[16];
      Native16<T> n;
    } sv;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + c32_row(r, hf);
      float sg;
      const float av = silu_sig(z[r], sg);
      if (row < rows) put(a + (int64_t)row * ld + col, av);
      sv.t[r] = (T)fmaf(av, 1.0f - sg, sg);
    }
    u32x4* dst = reinterpret_cast<u32x4*>(Native16<T>::at(s1, blk));
#pragma unroll
    for (int i = 0; i < Native16<T>::W; ++i) dst[i] = sv.n.v[i];
  }
};
// R = Y - V, E = scale * R; sum of R^2 of this tile into loss_part[tile].
template <typename T>
struct EpRes {
  T* e;
  const float* v;
  float* loss_part;
  int ld, rows;
  float scale;
  float acc = 0.f;
  typedef float In;
  __device__ __forceinline__ float load(int r, int c) const { return r < rows ? v[(int64_t)r * ld + c] : 0.f; }
  __device__ __forceinline__ void operator()(int r, int c, float y, float vv) {
    if (r >= rows) return;
    const float R = y - vv;
    acc = fmaf(R, R, acc);
    put(e + (int64_t)r * ld + c, scale * R);
  }
  __device__ __forceinline__ void finish() {
    __shared__ float red[NTH / 64];
    float s = acc;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) loss_part[blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
  }
};
// D = P * S1.
template <typename T>
struct EpD : EpBase {
  T* d;
  const T* s1;  // tile-native layout, written by EpAct<T, true> over the same grid
  int ld, rows;
  static constexpr bool TILED = true;
  typedef Native16<T> TIn;
  __device__ __forceinline__ TIn tload(int64_t blk) const {
    TIn r;
    const u32x4* src = reinterpret_cast<const u32x4*>(Native16<T>::at(const_cast<T*>(s1), blk));
#pragma unroll
    for (int i = 0; i < Native16<T>::W; ++i) r.v[i] = src[i];
    return r;
  }
  __device__ __forceinline__ void block(int64_t, int row0, int col, const f32x16& p, const TIn& n) {
    const int hf = (threadIdx.x >> 5) & 1;
    union {
      T t[16];
      Native16<T> n;
    } sv;
    sv.n = n;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + c32_row(r, hf);
      if (row < rows) put(d + (int64_t)row * ld + col, p[r] * (float)sv.t[r]);
    }
  }
};
// W -= eta * G (FP32 master), then the operand copy of the new W (nullable:
// masters only, while a sum of several gradients is being taken).
template <typename T>
struct EpUpd : EpBase {
  float* w;
  T* wop;
  int ld;
  float eta;
  typedef float In;
  __device__ __forceinline__ float load(int r, int c) const { return w[(int64_t)r * ld + c]; }
  __device__ __forceinline__ void operator()(int r, int c, float g, float wv) {
    const int64_t i = (int64_t)r * ld + c;
    const float wn = wv - eta * g;
    w[i] = wn;
    if (wop) put(wop + i, wn);
  }
};
// O rows of the chunk into the strided token tensor.
template <typename IOT>
struct EpOut : EpBase {
  IOT* o;  // first token of the chunk, head offset applied
  int64_t stride_tok;
  int rows;
  __device__ __forceinline__ void operator()(int r, int c, float y, In) {
    if (r >= rows) return;
    o[(int64_t)r * stride_tok + c] = (IOT)y;
  }
};

// A product stored as it is ([rows][ld], operand type).
template <typename T>
struct EpStoreTiled : EpBase {  // the product in the tile-native layout (read by EpSwi over the same grid)
  T* z;
  static constexpr bool TILED = true;
  __device__ __forceinline__ void block(int64_t blk, int, int, const f32x16& v, TIn) {
    union {
      T t[16];
      Native16<T> n;
    } sv;
#pragma unroll
    for (int r = 0; r < 16; ++r) sv.t[r] = (T)v[r];
    u32x4* dst = reinterpret_cast<u32x4*>(Native16<T>::at(z, blk));
#pragma unroll
    for (int i = 0; i < Native16<T>::W; ++i) dst[i] = sv.n.v[i];
  }
};
// Z1 = x W1 of the memory unit with Z3 = x W3 stored: Hd = SiLU(Z1) Z3; for
// the gradient also the factors of the hidden adjoint, G1 = Z3 SiLU'(Z1)
// (towards W1) and G3 = SiLU(Z1) (towards W3).
// Z3, G1 and G3 are in the tile-native layout (written and read by products
// of one chunk step over the same grid); Hd is an operand, row-major.
template <typename T, bool GRAD>
struct EpSwi : EpBase {
  const T* z3;
  T* hd;
  T* g1;
  T* g3;
  int ld, rows;
  static constexpr bool TILED = true;
  typedef Native16<T> TIn;
  __device__ __forceinline__ TIn tload(int64_t blk) const { return Native16<T>::load(z3, blk); }
  __device__ __forceinline__ void block(int64_t blk, int row0, int col, const f32x16& z1, const TIn& z3n) {
    const int hf = (threadIdx.x >> 5) & 1;
    union U {
      T t[16];
      Native16<T> n;
    } z3v, gv1, gv3;
    z3v.n = z3n;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + c32_row(r, hf);
      float sg;
      const float sv = silu_sig(z1[r], sg);
      const float zz = (float)z3v.t[r];
      if (row < rows) put(hd + (int64_t)row * ld + col, sv * zz);
      if constexpr (GRAD) {
        gv1.t[r] = (T)(zz * fmaf(sv, 1.0f - sg, sg));
        gv3.t[r] = (T)sv;
      }
    }
    if constexpr (GRAD) {
      Native16<T>::store(g1, blk, gv1.n);
      Native16<T>::store(g3, blk, gv3.n);
    }
  }
};
// dH = E W2^T: D1 = dH G1, D3 = dH G3.
template <typename T>
struct EpD2 : EpBase {
  const T* g1;  // tile-native, from EpSwi<T, true> over the same grid
  const T* g3;
  T* d1;
  T* d3;
  int ld, rows;
  static constexpr bool TILED = true;
  struct TIn {
    Native16<T> a, b;
  };
  __device__ __forceinline__ TIn tload(int64_t blk) const {
    return {Native16<T>::load(g1, blk), Native16<T>::load(g3, blk)};
  }
  __device__ __forceinline__ void block(int64_t, int row0, int col, const f32x16& dh, const TIn& g) {
    const int hf = (threadIdx.x >> 5) & 1;
    union U {
      T t[16];
      Native16<T> n;
    } a, b;
    a.n = g.a;
    b.n = g.b;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + c32_row(r, hf);
      if (row >= rows) continue;
      const int64_t i = (int64_t)row * ld + col;
      put(d1 + i, dh[r] * (float)a.t[r]);
      put(d3 + i, dh[r] * (float)b.t[r]);
    }
  }
};

// ------------------------------------------------------------- kernels
// Row normalisation of the chunk's K, V, Q rows (one wave per token; each
// lane holds runs of 4 consecutive elements, 256 elements per wave pass, at
// most 16 passes): Kn, Qn in the operand type, Vn in FP32 (the residual is
// formed in FP32).
template <typename IOT, typename T>
__global__ __launch_bounds__(256) void k_norm(LargeNormArgs p) {
  typedef IOT iov4 __attribute__((ext_vector_type(4)));
  typedef T opv4 __attribute__((ext_vector_type(4)));
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (row >= p.rows) return;
  const int passes = p.d / 256;
  for (int which = 0; which < 3; ++which) {
    const IOT* src = static_cast<const IOT*>(which == 0 ? p.K : which == 1 ? p.V : p.Q) +
                     (int64_t)row * p.stride_tok;
    const bool nrm = (p.flags >> (which == 0 ? 1 : which == 1 ? 2 : 0)) & 1u;
    f32x4 x[16];
    float ss = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if (i < passes) {
        const iov4 v = *reinterpret_cast<const iov4*>(src + 256 * i + 4 * l);
        x[i] = (f32x4){(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
#pragma unroll
        for (int e = 0; e < 4; ++e) ss = fmaf(x[i][e], x[i][e], ss);
      }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) ss += __shfl_xor(ss, m, 64);
    const float inv = nrm ? 1.0f / fmaxf(sqrtf(ss), NORM_EPS) : 1.0f;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if (i < passes) {
        const f32x4 y = x[i] * inv;
        const int64_t o = (int64_t)row * p.d + 256 * i + 4 * l;
        if (which == 1)
          *reinterpret_cast<f32x4*>(p.Vn + o) = y;
        else
          *reinterpret_cast<opv4*>(static_cast<T*>(which == 0 ? p.Kn : p.Qn) + o) = (opv4){(T)y[0], (T)y[1], (T)y[2], (T)y[3]};
      }
    }
  }
}

// FP32 masters and operand copies from the initial weights.
template <typename T>
__global__ void k_init_w(const float* w1, const float* w2, float* m1, float* m2, T* o1, T* o2, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float a = w1[i], b = w2[i];
    m1[i] = a;
    m2[i] = b;
    o1[i] = (T)a;
    o2[i] = (T)b;
  }
}

// E = -eta_i Vn_i of the memory unit's chunk, in the operand type.
template <typename T>
__global__ __launch_bounds__(256) void k_amu_e(T* e, const float* vn, const float* eta, int64_t eta_stride, int rows,
                                               int d) {
  const int64_t n = (int64_t)rows * d;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    e[i] = (T)(-eta[(i / d) * eta_stride] * vn[i]);
}

template <typename T>
__global__ void k_cast(const float* src, T* dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (T)src[i];
}

// loss[c] = (sum of the tile partials, in a fixed order) / M_c; one work-group
__global__ __launch_bounds__(NTH) void k_loss(const float* part, int n, float inv_m, float* out) {
  const float s = fixed_order_sum(part, n);
  if (threadIdx.x == 0) *out = s * inv_m;
}

template <typename T, typename IOT>
hipError_t step_t(const LargeStepArgs& a, hipStream_t st) {
  const int M = a.rows, d = a.d, h = a.h;
  // tile rows: 128 for the products over the chunk's tokens (two waves per
  // SIMD fit, which a 256-row tile with its 128 accumulator registers per lane
  // does not) and for the weight updates too, although their d x h outputs
  // give only 256 tiles of 128 x 128, one per CU: with the contraction loop
  // free of waits on the next slice's loads, 64-row tiles (twice the
  // work-groups) are slower for these 10,992-token contractions
  constexpr int BMT = 128, BMW = 128;
  const int mt = (M + BMT - 1) / BMT;
  T* Kn = static_cast<T*>(a.Kn);
  T* Qn = static_cast<T*>(a.Qn);
  T* E = static_cast<T*>(a.E);
  T* Aa = static_cast<T*>(a.A);
  T* Dd = static_cast<T*>(a.D);
  T* Aq = static_cast<T*>(a.Aq);
  T* W1o = static_cast<T*>(a.W1op);
  T* W2o = static_cast<T*>(a.W2op);
  LargeNormArgs na{a.K, a.V, a.Q, a.stride_tok, a.flags, M, d, a.Kn, a.Vn, a.Qn};
  hipLaunchKernelGGL((k_norm<IOT, T>), dim3((M + 3) / 4), dim3(256), 0, st, na);
  if (a.grad) {
    // Z = Kn W1 -> A, S1
    EpAct<T, true> e1{{}, Aa, static_cast<T*>(a.S1), h, M};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpAct<T, true>>), dim3(h / BN, mt), dim3(NTH), 0, st, Kn, d, M,
                       W1o, h, d, d, e1);
    // Y = A W2 -> E, loss partials
    EpRes<T> e2{E, a.Vn, a.loss_part, d, M, 2.0f / (float)M};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpRes<T>>), dim3(d / BN, mt), dim3(NTH), 0, st, Aa, h, M, W2o, d,
                       h, h, e2);
    if (a.loss) hipLaunchKernelGGL(k_loss, dim3(1), dim3(NTH), 0, st, a.loss_part, (d / BN) * mt, 1.0f / (float)M,
                                   a.loss);
    // P = E W2^T -> D
    EpD<T> e3{{}, Dd, static_cast<const T*>(a.S1), h, M};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, BMT, EpD<T>>), dim3(h / BN, mt), dim3(NTH), 0, st, E, d, M, W2o, d, h, d,
                       e3);
    // W1 -= eta Kn^T D ; W2 -= eta A^T E (contractions over the chunk's tokens)
    EpUpd<T> e4{{}, a.W1, a.masters_only ? nullptr : W1o, h, a.eta};
    hipLaunchKernelGGL((k_gemm<T, MNMAJ, MNMAJ, BMW, EpUpd<T>>), dim3(h / BN, d / BMW), dim3(NTH), 0, st, Kn, d, M, Dd,
                       h, M, M, e4);
    EpUpd<T> e5{{}, a.W2, a.masters_only ? nullptr : W2o, d, a.eta};
    hipLaunchKernelGGL((k_gemm<T, MNMAJ, MNMAJ, BMW, EpUpd<T>>), dim3(d / BN, h / BMW), dim3(NTH), 0, st, Aa, h, M, E, d,
                       M, M, e5);
  }
  if (a.O) {
    EpAct<T, false> e6{{}, Aq, nullptr, h, M};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpAct<T, false>>), dim3(h / BN, mt), dim3(NTH), 0, st, Qn, d, M, W1o,
                       h, d, d, e6);
    EpOut<IOT> e7{{}, static_cast<IOT*>(a.O), a.stride_tok, M};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpOut<IOT>>), dim3(d / BN, mt), dim3(NTH), 0, st, Aq, h, M, W2o, d,
                       h, h, e7);
  }
  return hipGetLastError();
}

template <typename T, typename IOT>
hipError_t amu_step_t(const LargeAmuArgs& a, hipStream_t st) {
  const int M = a.rows, d = a.d, h = a.h;
  constexpr int BMT = 128, BMW = 128;  // as in step_t
  const int mt = (M + BMT - 1) / BMT;
  T* Kn = static_cast<T*>(a.Kn);
  T* Qn = static_cast<T*>(a.Qn);
  T* E = static_cast<T*>(a.E);
  T* Z3 = static_cast<T*>(a.Z3);
  T* Hd = static_cast<T*>(a.Hd);
  T* G1 = static_cast<T*>(a.G1);
  T* G3 = static_cast<T*>(a.G3);
  T* D1 = static_cast<T*>(a.D1);
  T* D3 = static_cast<T*>(a.D3);
  T* W1o = static_cast<T*>(a.W1op);
  T* W2o = static_cast<T*>(a.W2op);
  T* W3o = static_cast<T*>(a.W3op);
  LargeNormArgs na{a.K, a.V, a.Q, a.stride_tok, a.flags, M, d, a.Kn, a.Vn, a.Qn};
  hipLaunchKernelGGL((k_norm<IOT, T>), dim3((M + 3) / 4), dim3(256), 0, st, na);
  if (a.grad) {
    EpStoreTiled<T> e1{{}, Z3};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpStoreTiled<T>>), dim3(h / BN, mt), dim3(NTH), 0, st, Kn, d, M, W3o,
                       h, d, d, e1);
    EpSwi<T, true> e2{{}, Z3, Hd, G1, G3, h, M};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpSwi<T, true>>), dim3(h / BN, mt), dim3(NTH), 0, st, Kn, d, M,
                       W1o, h, d, d, e2);
    const int64_t ne = (int64_t)M * d;
    hipLaunchKernelGGL(k_amu_e<T>, dim3((unsigned)std::min<int64_t>((ne + 255) / 256, 4096)), dim3(256), 0, st, E,
                       a.Vn, a.eta, a.eta_stride, M, d);
    EpD2<T> e3{{}, G1, G3, D1, D3, h, M};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, BMT, EpD2<T>>), dim3(h / BN, mt), dim3(NTH), 0, st, E, d, M, W2o, d, h,
                       d, e3);
    // the step sizes are inside the loss: W <- W - grad
    EpUpd<T> u1{{}, a.W1, a.write_op ? W1o : nullptr, h, 1.0f};
    hipLaunchKernelGGL((k_gemm<T, MNMAJ, MNMAJ, BMW, EpUpd<T>>), dim3(h / BN, d / BMW), dim3(NTH), 0, st, Kn, d, M, D1,
                       h, M, M, u1);
    EpUpd<T> u3{{}, a.W3, a.write_op ? W3o : nullptr, h, 1.0f};
    hipLaunchKernelGGL((k_gemm<T, MNMAJ, MNMAJ, BMW, EpUpd<T>>), dim3(h / BN, d / BMW), dim3(NTH), 0, st, Kn, d, M, D3,
                       h, M, M, u3);
    EpUpd<T> u2{{}, a.W2, a.write_op ? W2o : nullptr, d, 1.0f};
    hipLaunchKernelGGL((k_gemm<T, MNMAJ, MNMAJ, BMW, EpUpd<T>>), dim3(d / BN, h / BMW), dim3(NTH), 0, st, Hd, h, M, E,
                       d, M, M, u2);
  }
  if (a.O) {
    EpStoreTiled<T> e6{{}, Z3};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpStoreTiled<T>>), dim3(h / BN, mt), dim3(NTH), 0, st, Qn, d, M, W3o,
                       h, d, d, e6);
    EpSwi<T, false> e7{{}, Z3, Hd, nullptr, nullptr, h, M};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpSwi<T, false>>), dim3(h / BN, mt), dim3(NTH), 0, st, Qn, d, M,
                       W1o, h, d, d, e7);
    EpOut<IOT> e8{{}, static_cast<IOT*>(a.O), a.stride_tok, M};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, BMT, EpOut<IOT>>), dim3(d / BN, mt), dim3(NTH), 0, st, Hd, h, M, W2o, d,
                       h, h, e8);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t init_t(const float* w1, const float* w2, float* m1, float* m2, void* o1, void* o2, int64_t n,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_init_w<T>, dim3(1024), dim3(256), 0, st, w1, w2, m1, m2, static_cast<T*>(o1),
                     static_cast<T*>(o2), n);
  return hipGetLastError();
}

}  // namespace large

hipError_t launch_large_step(const LargeStepArgs& a, bool io_bf16, bool mma_bf16, hipStream_t st) {
  using namespace large;
  if (mma_bf16) return io_bf16 ? step_t<bf16, bf16>(a, st) : step_t<bf16, float>(a, st);
  return step_t<float, float>(a, st);
}

hipError_t launch_large_norm(const LargeNormArgs& a, bool io_bf16, bool mma_bf16, hipStream_t st) {
  using namespace large;
  const dim3 grid((a.rows + 3) / 4);
  if (mma_bf16) {
    if (io_bf16)
      hipLaunchKernelGGL((k_norm<bf16, bf16>), grid, dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL((k_norm<float, bf16>), grid, dim3(256), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_norm<float, float>), grid, dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_large_amu_step(const LargeAmuArgs& a, bool io_bf16, bool mma_bf16, hipStream_t st) {
  using namespace large;
  if (mma_bf16) return io_bf16 ? amu_step_t<bf16, bf16>(a, st) : amu_step_t<bf16, float>(a, st);
  return amu_step_t<float, float>(a, st);
}

hipError_t launch_large_cast(const float* src, void* dst, int64_t n, bool mma_bf16, hipStream_t st) {
  using namespace large;
  if (mma_bf16)
    hipLaunchKernelGGL(k_cast<bf16>, dim3(1024), dim3(256), 0, st, src, static_cast<bf16*>(dst), n);
  else
    hipLaunchKernelGGL(k_cast<float>, dim3(1024), dim3(256), 0, st, src, static_cast<float*>(dst), n);
  return hipGetLastError();
}

hipError_t launch_large_init(const float* w1, const float* w2, float* m1, float* m2, void* o1, void* o2, int64_t n,
                             bool mma_bf16, hipStream_t st) {
  using namespace large;
  return mma_bf16 ? init_t<bf16>(w1, w2, m1, m2, o1, o2, n, st) : init_t<float>(w1, w2, m1, m2, o1, o2, n, st);
}

}  // namespace ttt
