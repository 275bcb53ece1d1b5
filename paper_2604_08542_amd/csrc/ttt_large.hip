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
#include "ttt_internal.h"

namespace ttt {
namespace large {

constexpr int BN = 128;   // work-group tile width
constexpr int NTH = 256;  // 4 waves, each a (BM/2) x 64 quarter of the BM x 128 tile
// contraction slice per LDS stage: 64 BF16 or 32 FP32 elements (128 bytes)
template <typename T>
constexpr int bk() {
  return sizeof(T) == 2 ? 64 : 32;
}

// Operand layouts of C[m][n] = sum_k A(m, k) B(k, n):
//   KMAJ  the operand is stored [m or n][k] (k contiguous), pitch ld
//   MNMAJ the operand is stored [k][m or n] (m or n contiguous), pitch ld
enum { KMAJ = 0, MNMAJ = 1 };

// LDS tile of ROWS rows (m or n) by BK (contraction).  BF16 operands feed
// 32x32x16 products: a lane's 8 contraction slots hold, for lane half hf and
// product step j, k = 16j + 4hf + {0..3} and 16j + 8 + 4hf + {0..3}; both
// operands use this order (the order of the transposing LDS read), so a
// k-major and an mn-major operand can be mixed.  FP32 operands feed 32x32x2
// products, lane (l32, hf) holding k = 2j + hf.
//
// Pitches (in 4-byte LDS banks): a k-major BF16 row is 34 banks, so the
// 8-byte reads of 16 lanes from 16 consecutive rows cover the 32 banks once;
// an mn-major BF16 row is 72 banks (8 mod 32), so the four rows of 32 bytes
// that a 16-lane group of the transposing read touches fall on disjoint
// banks.  FP32: 33 banks (k-major, 4-byte reads down a column), 132 (mn-major,
// consecutive lanes on consecutive banks).
template <typename T, int ROWS>
struct Tile {
  static constexpr int BK = bk<T>();
  static constexpr int KLD = sizeof(T) == 2 ? BK + 4 : BK + 1;       // pitch of a k-major tile [ROWS][BK]
  static constexpr int MLD = sizeof(T) == 2 ? ROWS + 16 : ROWS + 4;  // pitch of an mn-major tile [BK][ROWS]
  static constexpr int ELEMS = ROWS * KLD > BK * MLD ? ROWS * KLD : BK * MLD;
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Global -> registers -> LDS staging of one operand tile (rows mn0 .. +ROWS
// of the m/n axis, k0 .. k0+BK of the contraction).  Loads go through a
// buffer resource that covers exactly the valid part of the operand, so rows
// past its end (ragged token counts) read as zero.
template <typename T, int LAYOUT, int ROWS>
struct Stage {
  static constexpr int BK = bk<T>();
  static constexpr int BYTES = ROWS * BK * (int)sizeof(T);
  static constexpr int PER = BYTES / NTH / 16;  // 16-byte loads per thread
  static constexpr int EPC = 16 / (int)sizeof(T);  // elements per 16-byte chunk
  u32x4 r[PER];
  __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, int ld, int mn0, int k0) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int c = tid + i * NTH;  // 16-byte chunk index within the tile
      int row, col;
      if constexpr (LAYOUT == KMAJ) {  // [ROWS][BK]
        constexpr int CPR = BK / EPC;
        row = mn0 + c / CPR;
        col = k0 + (c % CPR) * EPC;
      } else {  // [BK][ROWS]
        constexpr int CPR = ROWS / EPC;
        row = k0 + c / CPR;
        col = mn0 + (c % CPR) * EPC;
      }
      r[i] = __builtin_amdgcn_raw_buffer_load_b128(rs, (row * ld + col) * (int)sizeof(T), 0, 0);
    }
  }
  __device__ __forceinline__ void store(T* lds) const {
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int c = tid + i * NTH;
      int off;
      if constexpr (LAYOUT == KMAJ) {
        constexpr int CPR = BK / EPC;
        off = (c / CPR) * Tile<T, ROWS>::KLD + (c % CPR) * EPC;
      } else {
        constexpr int CPR = ROWS / EPC;
        off = (c / CPR) * Tile<T, ROWS>::MLD + (c % CPR) * EPC;
      }
      if constexpr (LAYOUT == MNMAJ) {
        *reinterpret_cast<u32x4*>(lds + off) = r[i];
      } else if constexpr (sizeof(T) == 2) {  // k-major BF16 rows are 8-byte aligned: two 8-byte stores
        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
        const u32x4 v = r[i];
        reinterpret_cast<u32x2*>(lds + off)[0] = (u32x2){v[0], v[1]};
        reinterpret_cast<u32x2*>(lds + off)[1] = (u32x2){v[2], v[3]};
      } else {  // FP32 k-major rows have an odd pitch: four 4-byte stores
        const u32x4 v = r[i];
#pragma unroll
        for (int e = 0; e < 4; ++e) reinterpret_cast<uint32_t*>(lds + off)[e] = v[e];
      }
    }
  }
};

// Operand fragment of product step j for the 32-wide block starting at mn
// (tile-local) of a staged tile.
template <typename T, int LAYOUT, int ROWS>
__device__ __forceinline__ auto frag(const T* t, int mn, int j) {
  const int l = threadIdx.x & 63, l32 = l & 31, hf = l >> 5;
  using TL = Tile<T, ROWS>;
  if constexpr (sizeof(T) == 2) {
    typedef __attribute__((address_space(3))) bf16x4 lds_bf16x4;
    if constexpr (LAYOUT == KMAJ) {
      const bf16* row = t + (mn + l32) * TL::KLD + 16 * j + 4 * hf;
      const bf16x4 lo = *reinterpret_cast<const bf16x4*>(row);
      const bf16x4 hi = *reinterpret_cast<const bf16x4*>(row + 8);
      return (bf16x8){lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    } else {
      // transposing read: in each 16-lane group lane i addresses row
      // t0 + i/4, columns c0 + 4(i%4)..+3 and receives T[t0 + q][c0 + i], q < 4
      const int l16 = l & 15;
      const int off = (4 * hf + (l16 >> 2)) * TL::MLD + mn + 16 * ((l >> 4) & 1) + 4 * (l16 & 3);
      const bf16* p0 = t + off + 16 * j * TL::MLD;
      const bf16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4bf16(
          (lds_bf16x4*)((__attribute__((address_space(3))) bf16*)(p0)));
      const bf16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4bf16(
          (lds_bf16x4*)((__attribute__((address_space(3))) bf16*)(p0 + 8 * TL::MLD)));
      return (bf16x8){lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    }
  } else {
    if constexpr (LAYOUT == KMAJ)
      return t[(mn + l32) * TL::KLD + 2 * j + hf];
    else
      return t[(2 * j + hf) * TL::MLD + mn + l32];
  }
}

// Product steps per contraction slice.
template <typename T>
constexpr int ksteps() {
  return sizeof(T) == 2 ? bk<T>() / 16 : bk<T>() / 2;
}

// C tile (this work-group's BM x 128) accumulated over the whole
// contraction, then handed to the epilogue element by element:
// ep(row, col, value); rows past the operand's end are the epilogue's to skip.
template <typename T, int LA, int LB, int BM, typename EP>
__device__ __forceinline__ void gemm_tile(const T* A, int lda, int a_rows, const T* B, int ldb, int b_rows, int K,
                                          int m0, int n0, EP& ep) {
  constexpr int MB = BM / 64;  // 32-row blocks per wave (each wave: BM/2 rows x 64 columns)
  __shared__ __attribute__((aligned(16))) T sa[2][Tile<T, BM>::ELEMS];
  __shared__ __attribute__((aligned(16))) T sb[2][Tile<T, BN>::ELEMS];
  const int w = threadIdx.x >> 6, wm = (w >> 1) * (BM / 2), wn = (w & 1) * 64;
  // buffer resources over the valid rows of each operand
  auto rsrc = [](const T* p, int rows, int ld) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p), (short)0, rows * ld * (int)sizeof(T), 0x00020000);
  };
  const auto ra = rsrc(A, a_rows, lda), rb = rsrc(B, b_rows, ldb);
  // Three-stage pipeline: while slice kt is multiplied out of one LDS
  // buffer, slice kt+1 waits in the other and slice kt+2 is in flight from
  // HBM into registers (two register stages, alternating), so a global load
  // has two slices of products to arrive before it is needed.
  Stage<T, LA, BM> ga[2];
  Stage<T, LB, BN> gb[2];
  constexpr int BK = bk<T>();
  const int nk = (K + BK - 1) / BK;
  f32x16 acc[MB][2] = {};
  ga[0].load(ra, lda, m0, 0);
  gb[0].load(rb, ldb, n0, 0);
  if (nk > 1) {
    ga[1].load(ra, lda, m0, BK);
    gb[1].load(rb, ldb, n0, BK);
  }
  ga[0].store(sa[0]);
  gb[0].store(sb[0]);
  __syncthreads();
  auto body = [&](int kt, auto PC) {
    constexpr int P = decltype(PC)::value;  // kt & 1
    if (kt + 2 < nk) {  // slice kt+2 into register stage P (free: slice kt left it last iteration)
      ga[P].load(ra, lda, m0, (kt + 2) * BK);
      gb[P].load(rb, ldb, n0, (kt + 2) * BK);
    }
#pragma unroll
    for (int j = 0; j < ksteps<T>(); ++j) {
      const auto b0 = frag<T, LB, BN>(sb[P], wn, j), b1 = frag<T, LB, BN>(sb[P], wn + 32, j);
#pragma unroll
      for (int bm = 0; bm < MB; ++bm) {
        const auto a = frag<T, LA, BM>(sa[P], wm + 32 * bm, j);
        acc[bm][0] = mma32(a, b0, acc[bm][0]);
        acc[bm][1] = mma32(a, b1, acc[bm][1]);
      }
    }
    if (kt + 1 < nk) {  // slice kt+1 (register stage P^1) into the other LDS buffer
      ga[P ^ 1].store(sa[P ^ 1]);
      gb[P ^ 1].store(sb[P ^ 1]);
    }
    __syncthreads();
  };
  for (int kt = 0; kt < nk; kt += 2) {
    body(kt, std::integral_constant<int, 0>{});
    if (kt + 1 < nk) body(kt + 1, std::integral_constant<int, 1>{});
  }
  const int l = threadIdx.x & 63, l32 = l & 31, hf = l >> 5;
#pragma unroll
  for (int bm = 0; bm < MB; ++bm)
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm + 32 * bm + c32_row(r, hf), col = n0 + wn + 32 * bn + l32;
        ep(row, col, acc[bm][bn][r]);
      }
  ep.finish();
}

__device__ __forceinline__ float silu_sig(float z, float& sg) {
  sg = sigmoid(z);
  return z * sg;
}

template <typename T>
__device__ __forceinline__ void put(T* p, float v) {
  *p = (T)v;
}

// ------------------------------------------------------------- epilogues
struct EpBase {
  __device__ __forceinline__ void finish() {}
};
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
// One launch of one product; grid (N / 128, ceil(M / 128)).
template <typename T, int LA, int LB, int BM, typename EP>
__global__ __launch_bounds__(NTH) void k_gemm(const T* A, int lda, int a_rows, const T* B, int ldb, int b_rows,
                                                int K, EP ep) {
  gemm_tile<T, LA, LB, BM>(A, lda, a_rows, B, ldb, b_rows, K, blockIdx.y * BM, blockIdx.x * BN, ep);
}

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
