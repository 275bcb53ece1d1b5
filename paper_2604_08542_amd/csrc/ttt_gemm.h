// Matrix-core GEMM tiles for gfx950 shared by the large-state chunk step and
// the surrounding layer's projections: C[m][n] = sum_k A(m, k) B(k, n) over
// BF16 (32x32x16 products) or FP32 (32x32x2) operands in their natural
// layouts, a work-group owning one BM x 128 tile of C and its whole
// contraction (fixed order, deterministic), the elementwise work of the
// caller fused into an epilogue functor.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "ttt_common.h"

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

// Epilogues derive from this.  An epilogue that reads an input per element
// (a factor, a residual target, the FP32 master) defines In and load(r, c);
// the tile calls load for 16 elements (BF16 tiles with a small input: for all
// of its elements) before it calls operator() for any of them, so those
// reads are in flight together instead of each waiting behind the previous
// element's store.  finish() runs once per work-group after its last element.
//
// An epilogue with TILED = true instead takes each 32x32 block whole:
// tload(blk) for every block of the wave first, then block(blk, row0, col,
// acc, tin), where the lane owns rows row0 + c32_row(r, hf) of column col.
// blk numbers the 32x32 blocks of the launch, so that an intermediate one
// product writes and a later product of the same grid reads can be kept in
// a tile-native layout (the 16 values of a lane contiguous, two 16-byte
// accesses per block, 1,024 elements per block).
struct EpBase {
  struct In {};
  __device__ __forceinline__ In load(int, int) const { return {}; }
  __device__ __forceinline__ void finish() {}
  static constexpr bool TILED = false;
  struct TIn {};
  __device__ __forceinline__ TIn tload(int64_t) const { return {}; }
};

// whether an epilogue takes whole blocks (TILED = true; epilogues that do
// not derive from EpBase have no TILED member)
template <typename E, typename = void>
struct is_tiled : std::false_type {};
template <typename E>
struct is_tiled<E, std::void_t<decltype(E::TILED)>> : std::bool_constant<E::TILED> {};

constexpr int BN = 128;   // work-group tile width
constexpr int NTH = 256;  // 4 waves, each a (BM/2) x 64 quarter of the BM x 128 tile
// contraction slice per LDS stage: 64 BF16 or 32 FP32 elements (128 bytes)
template <typename T>
constexpr int bk() {
  return sizeof(T) == 2 ? 64 : 32;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// A lane's 16 values of one 32x32 block in the tile-native layout (see
// EpBase): 16 * sizeof(T) contiguous bytes at base + blk * 1024 + lane * 16.
template <typename T>
struct Native16 {
  static constexpr int W = (int)sizeof(T);  // 16-byte words per lane and block
  u32x4 v[W];
  __device__ __forceinline__ static T* at(T* base, int64_t blk) {
    return base + blk * 1024 + (threadIdx.x & 63) * 16;
  }
  __device__ __forceinline__ static Native16 load(const T* base, int64_t blk) {
    Native16 r;
    const u32x4* src = reinterpret_cast<const u32x4*>(at(const_cast<T*>(base), blk));
#pragma unroll
    for (int i = 0; i < W; ++i) r.v[i] = src[i];
    return r;
  }
  __device__ __forceinline__ static void store(T* base, int64_t blk, const Native16& n) {
    u32x4* dst = reinterpret_cast<u32x4*>(at(base, blk));
#pragma unroll
    for (int i = 0; i < W; ++i) dst[i] = n.v[i];
  }
};
// Operand layouts of C[m][n] = sum_k A(m, k) B(k, n):
//   KMAJ  the operand is stored [m or n][k] (k contiguous), pitch ld
//   MNMAJ the operand is stored [k][m or n] (m or n contiguous), pitch ld
enum { KMAJ = 0, MNMAJ = 1 };

// LDS tile of ROWS rows (m or n) by BK (contraction).  BF16 operands feed
// 32x32x16 products: a lane's 8 contraction slots hold, for lane half hf and
// product step j, k = 16j + 8hf + {0..7}, so a k-major fragment is one
// 16-byte LDS read and an mn-major one two transposing reads of four rows
// each; both operands use this order, so a k-major and an mn-major operand
// can be mixed.  FP32 operands feed 32x32x2 products, lane (l32, hf) holding
// k = 2j + hf.
//
// Pitches (in 4-byte LDS banks): a k-major BF16 row is 36 banks (16-byte
// aligned), so the 16-byte reads of 8 lanes from 8 consecutive rows start 4
// banks apart mod 32 and cover the banks once; an mn-major BF16 row is 72
// banks (8 mod 32), so the four rows of 32 bytes that a 16-lane group of the
// transposing read touches fall on disjoint banks.  FP32: 33 banks (k-major,
// 4-byte reads down a column), 132 (mn-major, consecutive lanes on
// consecutive banks).
template <typename T, int ROWS>
struct Tile {
  static constexpr int BK = bk<T>();
  static constexpr int KLD = sizeof(T) == 2 ? BK + 8 : BK + 1;       // pitch of a k-major tile [ROWS][BK]
  static constexpr int MLD = sizeof(T) == 2 ? ROWS + 16 : ROWS + 4;  // pitch of an mn-major tile [BK][ROWS]
  static constexpr int ELEMS = ROWS * KLD > BK * MLD ? ROWS * KLD : BK * MLD;
};


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
  // This thread's byte offsets of its chunks for the slice at k0 = 0; a
  // slice at k0 adds the uniform kbytes(ld) * k0.
  __device__ __forceinline__ static void offsets(int ld, int mn0, int (&vo)[PER]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int c = tid + i * NTH;  // 16-byte chunk index within the tile
      int row, col;
      if constexpr (LAYOUT == KMAJ) {  // [ROWS][BK]
        constexpr int CPR = BK / EPC;
        row = mn0 + c / CPR;
        col = (c % CPR) * EPC;
      } else {  // [BK][ROWS]
        constexpr int CPR = ROWS / EPC;
        row = c / CPR;
        col = mn0 + (c % CPR) * EPC;
      }
      vo[i] = (row * ld + col) * (int)sizeof(T);
    }
  }
  __device__ __forceinline__ static int kbytes(int ld) {
    return LAYOUT == KMAJ ? (int)sizeof(T) : ld * (int)sizeof(T);
  }
  __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, const int (&vo)[PER], int kofs) {
#pragma unroll
    for (int i = 0; i < PER; ++i) r[i] = __builtin_amdgcn_raw_buffer_load_b128(rs, vo[i] + kofs, 0, 0);
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
      } else if constexpr (sizeof(T) == 2) {  // k-major BF16 rows are 16-byte aligned
        *reinterpret_cast<u32x4*>(lds + off) = r[i];
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
      return *reinterpret_cast<const bf16x8*>(t + (mn + l32) * TL::KLD + 16 * j + 8 * hf);
    } else {
      // transposing read: in each 16-lane group lane i addresses row
      // t0 + i/4, columns c0 + 4(i%4)..+3 and receives T[t0 + q][c0 + i], q < 4;
      // rows 8hf..8hf+3, then 8hf+4..8hf+7
      const int l16 = l & 15;
      const int off = (8 * hf + (l16 >> 2)) * TL::MLD + mn + 16 * ((l >> 4) & 1) + 4 * (l16 & 3);
      const bf16* p0 = t + off + 16 * j * TL::MLD;
      const bf16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4bf16(
          (lds_bf16x4*)((__attribute__((address_space(3))) bf16*)(p0)));
      const bf16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4bf16(
          (lds_bf16x4*)((__attribute__((address_space(3))) bf16*)(p0 + 4 * TL::MLD)));
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
// ep(row, col, value, ep.load(row, col)); rows past the operand's end are the
// epilogue's to skip (in load as well).
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
  using SA = Stage<T, LA, BM>;
  using SB = Stage<T, LB, BN>;
  SA ga[2];
  SB gb[2];
  int voa[SA::PER], vob[SB::PER];
  SA::offsets(lda, m0, voa);
  SB::offsets(ldb, n0, vob);
  const int ka = SA::kbytes(lda) * bk<T>(), kb = SB::kbytes(ldb) * bk<T>();  // bytes per slice
  constexpr int BK = bk<T>();
  const int nk = (K + BK - 1) / BK;
  f32x16 acc[MB][2] = {};
  // Every load and LDS store below is unconditional (a slice past the end
  // reloads slice 0, which nothing reads), and the loop runs the two
  // register stages in pairs with a separate last slice: with a branch around
  // the loads, the compiler's load counters merge conservatively and each
  // slice waited for the loads issued for the next one.
  ga[0].load(ra, voa, 0);
  gb[0].load(rb, vob, 0);
  ga[1].load(ra, voa, nk > 1 ? ka : 0);
  gb[1].load(rb, vob, nk > 1 ? kb : 0);
  ga[0].store(sa[0]);
  gb[0].store(sb[0]);
  __syncthreads();
  auto body = [&](int kt, auto PC) {
    constexpr int P = decltype(PC)::value;  // kt & 1
    {  // slice kt+2 into register stage P (free: slice kt left it last iteration)
      const bool more = kt + 2 < nk;
      ga[P].load(ra, voa, more ? (kt + 2) * ka : 0);
      gb[P].load(rb, vob, more ? (kt + 2) * kb : 0);
    }
    // every operand fragment of the slice is read before the products, so
    // the LDS latency is paid once per slice, not once per product step
    using FT = decltype(frag<T, LB, BN>(sb[P], wn, 0));
    FT fb[ksteps<T>()][2], fa[ksteps<T>()][MB];
#pragma unroll
    for (int j = 0; j < ksteps<T>(); ++j) {
      fb[j][0] = frag<T, LB, BN>(sb[P], wn, j);
      fb[j][1] = frag<T, LB, BN>(sb[P], wn + 32, j);
#pragma unroll
      for (int bm = 0; bm < MB; ++bm) fa[j][bm] = frag<T, LA, BM>(sa[P], wm + 32 * bm, j);
    }
#pragma unroll
    for (int j = 0; j < ksteps<T>(); ++j) {
#pragma unroll
      for (int bm = 0; bm < MB; ++bm) {
        acc[bm][0] = mma32(fa[j][bm], fb[j][0], acc[bm][0]);
        acc[bm][1] = mma32(fa[j][bm], fb[j][1], acc[bm][1]);
      }
    }
    // slice kt+1 (register stage P^1) into the other LDS buffer
    ga[P ^ 1].store(sa[P ^ 1]);
    gb[P ^ 1].store(sb[P ^ 1]);
    __syncthreads();
  };
  int kt = 0;
  for (; kt + 1 < nk; kt += 2) {
    body(kt, std::integral_constant<int, 0>{});
    body(kt + 1, std::integral_constant<int, 1>{});
  }
  if (kt < nk) body(kt, std::integral_constant<int, 0>{});
  const int l = threadIdx.x & 63, l32 = l & 31, hf = l >> 5;
  if constexpr (is_tiled<EP>::value) {
    const int64_t blk0 = ((int64_t)(blockIdx.y * gridDim.x + blockIdx.x) * 4 + (threadIdx.x >> 6)) * (MB * 2);
    typename EP::TIn tin[MB][2];
#pragma unroll
    for (int bm = 0; bm < MB; ++bm)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn) tin[bm][bn] = ep.tload(blk0 + 2 * bm + bn);
#pragma unroll
    for (int bm = 0; bm < MB; ++bm)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn)
        ep.block(blk0 + 2 * bm + bn, m0 + wm + 32 * bm, n0 + wn + 32 * bn + l32, acc[bm][bn], tin[bm][bn]);
  } else if constexpr (sizeof(T) == 2 && sizeof(typename EP::In) <= 4) {
    // BF16 tiles with at most one 4-byte input per element request every
    // input of the tile before the first element is stored (one load latency
    // per tile, not one per 32x32 block); the registers fit beside the
    // accumulators at two waves per SIMD
    typename EP::In in[MB][2][16];
#pragma unroll
    for (int bm = 0; bm < MB; ++bm)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn)
#pragma unroll
        for (int r = 0; r < 16; ++r) in[bm][bn][r] = ep.load(m0 + wm + 32 * bm + c32_row(r, hf), n0 + wn + 32 * bn + l32);
#pragma unroll
    for (int bm = 0; bm < MB; ++bm)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          ep(m0 + wm + 32 * bm + c32_row(r, hf), n0 + wn + 32 * bn + l32, acc[bm][bn][r], in[bm][bn][r]);
  } else {
#pragma unroll
    for (int bm = 0; bm < MB; ++bm)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn) {
        const int col = n0 + wn + 32 * bn + l32;
        typename EP::In in[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) in[r] = ep.load(m0 + wm + 32 * bm + c32_row(r, hf), col);
#pragma unroll
        for (int r = 0; r < 16; ++r) ep(m0 + wm + 32 * bm + c32_row(r, hf), col, acc[bm][bn][r], in[r]);
      }
  }
  ep.finish();
}

// Sum of part[0..n) by one work-group of NTH threads in a fixed order:
// thread t adds the run part[t c .. t c + c) in index order (c = ceil(n /
// NTH)), then thread 0 adds the NTH run sums in thread order.  The result is
// valid in thread 0 only.
__device__ __forceinline__ float fixed_order_sum(const float* part, int n) {
  __shared__ float run[NTH];
  const int t = threadIdx.x, c = (n + NTH - 1) / NTH;
  const int i0 = t * c, i1 = i0 + c < n ? i0 + c : n;
  float s = 0.f;
  for (int i = i0; i < i1; ++i) s += part[i];
  run[t] = s;
  __syncthreads();
  float tot = 0.f;
  if (t == 0)
    for (int i = 0; i < NTH; ++i) tot += run[i];
  return tot;
}

// One launch of one product; grid (N / 128, ceil(M / 128)).
template <typename T, int LA, int LB, int BM, typename EP>
__global__ __launch_bounds__(NTH) void k_gemm(const T* A, int lda, int a_rows, const T* B, int ldb, int b_rows,
                                                int K, EP ep) {
  gemm_tile<T, LA, LB, BM>(A, lda, a_rows, B, ldb, b_rows, K, blockIdx.y * BM, blockIdx.x * BN, ep);
}

}  // namespace large
}  // namespace ttt
