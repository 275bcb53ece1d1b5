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

__device__ __forceinline__ float silu_sig(float z, float& sg) {
  sg = sigmoid(z);
  return z * sg;
}

template <typename T>
__device__ __forceinline__ void put(T* p, float v) {
  *p = (T)v;
}

// ------------------------------------------------------------- epilogues
// A = SiLU(Z), S1 = SiLU'(Z) (for the gradient) or only A (for the apply).
template <typename T, bool GRAD>
struct EpAct : EpBase {
  T* a;
  T* s1;
  int ld, rows;
  __device__ __forceinline__ void operator()(int r, int c, float z) {
    if (r >= rows) return;
    float sg;
    const float av = silu_sig(z, sg);
    put(a + (int64_t)r * ld + c, av);
    if constexpr (GRAD) put(s1 + (int64_t)r * ld + c, fmaf(av, 1.0f - sg, sg));
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
  __device__ __forceinline__ void operator()(int r, int c, float y) {
    if (r >= rows) return;
    const float R = y - v[(int64_t)r * ld + c];
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
  const T* s1;
  int ld, rows;
  __device__ __forceinline__ void operator()(int r, int c, float p) {
    if (r >= rows) return;
    put(d + (int64_t)r * ld + c, p * (float)s1[(int64_t)r * ld + c]);
  }
};
// W -= eta * G (FP32 master), then the operand copy of the new W.
template <typename T>
struct EpUpd : EpBase {
  float* w;
  T* wop;
  int ld;
  float eta;
  __device__ __forceinline__ void operator()(int r, int c, float g) {
    const int64_t i = (int64_t)r * ld + c;
    const float wn = w[i] - eta * g;
    w[i] = wn;
    put(wop + i, wn);
  }
};
// O rows of the chunk into the strided token tensor.
template <typename IOT>
struct EpOut : EpBase {
  IOT* o;  // first token of the chunk, head offset applied
  int64_t stride_tok;
  int rows;
  __device__ __forceinline__ void operator()(int r, int c, float y) {
    if (r >= rows) return;
    o[(int64_t)r * stride_tok + c] = (IOT)y;
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

// loss[c] = (sum of the tile partials, in tile order) / M_c
__global__ void k_loss(const float* part, int n, float inv_m, float* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = s * inv_m;
  }
}

template <typename T, typename IOT>
hipError_t step_t(const LargeStepArgs& a, hipStream_t st) {
  const int M = a.rows, d = a.d, h = a.h;
  // tile rows (128 everywhere: two waves per SIMD fit, which a 256-row tile
  // with its 128 accumulator registers per lane does not)
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
    if (a.loss) hipLaunchKernelGGL(k_loss, dim3(1), dim3(64), 0, st, a.loss_part, (d / BN) * mt, 1.0f / (float)M,
                                   a.loss);
    // P = E W2^T -> D
    EpD<T> e3{{}, Dd, static_cast<const T*>(a.S1), h, M};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, BMT, EpD<T>>), dim3(h / BN, mt), dim3(NTH), 0, st, E, d, M, W2o, d, h, d,
                       e3);
    // W1 -= eta Kn^T D ; W2 -= eta A^T E (contractions over the chunk's tokens)
    EpUpd<T> e4{{}, a.W1, W1o, h, a.eta};
    hipLaunchKernelGGL((k_gemm<T, MNMAJ, MNMAJ, BMW, EpUpd<T>>), dim3(h / BN, d / BMW), dim3(NTH), 0, st, Kn, d, M, Dd,
                       h, M, M, e4);
    EpUpd<T> e5{{}, a.W2, W2o, d, a.eta};
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

hipError_t launch_large_init(const float* w1, const float* w2, float* m1, float* m2, void* o1, void* o2, int64_t n,
                             bool mma_bf16, hipStream_t st) {
  using namespace large;
  return mma_bf16 ? init_t<bf16>(w1, w2, m1, m2, o1, o2, n, st) : init_t<float>(w1, w2, m1, m2, o1, o2, n, st);
}

}  // namespace ttt
