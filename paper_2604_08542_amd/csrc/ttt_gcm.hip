// The layer around the memory unit (Sec. 4.2: a query-key-value projection,
// the memory unit, an output projection; Sec. 4.1 Eq. 5: the gate
// alpha * GCM(X) + X with a learnable per-feature vector alpha).  The two
// projections are matrix-core GEMMs over the token rows, with their
// elementwise work fused into the epilogue:
//   projection  [Q | K | V] = X Wqkv (+ bqkv), each third stored as its own
//               [N][H*d] token tensor (head h = features h*d .. h*d+d-1)
//   output      Y = alpha * (O Wo (+ bo)) + X
// The memory unit between them is the chunked forward of this library.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ttt_common.h"
#include "ttt_gemm.h"
#include "ttt_internal.h"

namespace ttt {
namespace large {

// Column c of the projection goes to tensor c / D, feature c % D.
template <typename T>
struct EpProj : EpBase {
  T* q;
  T* k;
  T* v;
  const float* bias;  // nullable
  int D, rows;
  __device__ __forceinline__ void operator()(int r, int c, float x, In) {
    if (r >= rows) return;
    const float y = bias ? x + bias[c] : x;
    // a 128-column tile never straddles two of the thirds (D % 128 == 0),
    // so the selection is uniform over the tile; comparisons, no division
    T* dst = c < D ? q : c < 2 * D ? k : v;
    const int f = c < D ? c : c < 2 * D ? c - D : c - 2 * D;
    dst[(int64_t)r * D + f] = (T)y;
  }
};

// Y = alpha * (O Wo + bo) + X, all [N][D].
template <typename T>
struct EpGate : EpBase {
  T* y;
  const T* x;
  const float* bias;  // nullable
  const float* alpha;
  int D, rows;
  __device__ __forceinline__ void operator()(int r, int c, float g, In) {
    if (r >= rows) return;
    const int64_t i = (int64_t)r * D + c;
    const float gg = bias ? g + bias[c] : g;
    y[i] = (T)fmaf(alpha[c], gg, (float)x[i]);
  }
};

// The rows of one launch are limited so that an operand slab stays within
// the 32-bit byte range of a buffer resource; larger token counts run as
// several launches over consecutive row slabs.
template <typename T>
hipError_t gcm_t(const GcmGemmArgs& a, hipStream_t st) {
  const int D = a.D;
  const int64_t slab = std::max<int64_t>(128, ((int64_t(1) << 31) - 1) / ((int64_t)D * (int64_t)sizeof(T)) / 128 * 128);
  for (int64_t r0 = 0; r0 < a.rows; r0 += slab) {
    const int rows = (int)std::min<int64_t>(slab, a.rows - r0);
    const int64_t off = r0 * D;
    const dim3 grid_p(3 * D / BN, (rows + 127) / 128), grid_o(D / BN, (rows + 127) / 128);
    if (a.kind == 0) {
      EpProj<T> ep{{}, static_cast<T*>(a.q) + off, static_cast<T*>(a.k) + off, static_cast<T*>(a.v) + off, a.bias, D,
                   rows};
      hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, 128, EpProj<T>>), grid_p, dim3(NTH), 0, st,
                         static_cast<const T*>(a.x) + off, D, rows, static_cast<const T*>(a.w), 3 * D, D, D, ep);
    } else {
      EpGate<T> ep{{}, static_cast<T*>(a.y) + off, static_cast<const T*>(a.x) + off, a.bias, a.alpha, D, rows};
      hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, 128, EpGate<T>>), grid_o, dim3(NTH), 0, st,
                         static_cast<const T*>(a.o) + off, D, rows, static_cast<const T*>(a.w), D, D, D, ep);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ------------------------------------------------------------------ reverse mode
// A product stored with a bias per column (nullable) and a row pitch.
template <typename T>
struct EpBiasT : EpBase {
  T* out;
  const float* bias;
  int64_t ld;
  int rows;
  __device__ __forceinline__ void operator()(int r, int c, float v, In) {
    if (r >= rows) return;
    out[(int64_t)r * ld + c] = (T)(bias ? v + bias[c] : v);
  }
};
// A product stored in FP32 with a bias per column (nullable).
struct EpBiasF : EpBase {
  float* out;
  const float* bias;
  int64_t ld;
  int rows;
  __device__ __forceinline__ void operator()(int r, int c, float v, In) {
    if (r >= rows) return;
    out[(int64_t)r * ld + c] = bias ? v + bias[c] : v;
  }
};
// out = add + product (io type), both [rows][ld].
template <typename T>
struct EpAddT : EpBase {
  T* out;
  const T* add;
  int64_t ld;
  int rows;
  typedef T In;
  __device__ __forceinline__ T load(int r, int c) const { return r < rows ? add[(int64_t)r * ld + c] : T(0.f); }
  __device__ __forceinline__ void operator()(int r, int c, float v, T a) {
    if (r >= rows) return;
    out[(int64_t)r * ld + c] = (T)((float)a + v);
  }
};

constexpr int SLAB = 256;  // rows per column-sum partial

// Gate adjoint over a slab of rows, one thread per column: dG = alpha dY, and
// the slab's sums of G dY (part[slab][c]) and of dG (part[slab][D + c]).
template <typename T>
__global__ __launch_bounds__(256) void k_gate_bwd(const float* G, const T* dY, const float* alpha, int64_t rows,
                                                  int D, T* dG, float* part) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= D) return;
  const int64_t r0 = (int64_t)blockIdx.y * SLAB, r1 = r0 + SLAB < rows ? r0 + SLAB : rows;
  const float a = alpha[c];
  float sa = 0.f, sb = 0.f;
  for (int64_t r = r0; r < r1; ++r) {
    const int64_t i = r * D + c;
    const float dy = (float)dY[i];
    const float dg = a * dy;
    sa = fmaf(G[i], dy, sa);
    sb += dg;
    dG[i] = (T)dg;
  }
  part[(int64_t)blockIdx.y * 2 * D + c] = sa;
  part[(int64_t)blockIdx.y * 2 * D + D + c] = sb;
}
// Column sums of a slab of rows of a [rows][ld] tensor: part[slab][c].
template <typename T>
__global__ __launch_bounds__(256) void k_colsum(const T* a, int64_t ld, int64_t rows, int cols, float* part) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  const int64_t r0 = (int64_t)blockIdx.y * SLAB, r1 = r0 + SLAB < rows ? r0 + SLAB : rows;
  float s = 0.f;
  for (int64_t r = r0; r < r1; ++r) s += (float)a[r * ld + c];
  part[(int64_t)blockIdx.y * cols + c] = s;
}
// out[c] = the slabs' partials of column c, summed in slab order.
__global__ __launch_bounds__(256) void k_slabs(const float* part, int nslab, int64_t pitch, int cols, float* out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int i = 0; i < nslab; ++i) s += part[(int64_t)i * pitch + c];
  out[c] = s;
}

template <typename T>
hipError_t gcm_bwd_t(const GcmBwdArgs& a, hipStream_t st) {
  const int D = a.D, rows = (int)a.rows;
  const int64_t D3 = 3 * (int64_t)D;
  const int mt = (rows + 127) / 128, nslab = (rows + SLAB - 1) / SLAB;
  const dim3 nt(NTH);
  if (a.phase == 0) {
    EpBiasT<T> ep{{}, static_cast<T*>(a.P), a.bqkv, D3, rows};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, 128, EpBiasT<T>>), dim3(3 * D / BN, mt), nt, 0, st,
                       static_cast<const T*>(a.X), D, rows, static_cast<const T*>(a.Wqkv), (int)D3, D, D, ep);
  } else if (a.phase == 1) {
    const T* O = static_cast<const T*>(a.O);
    EpBiasF eg{{}, a.G, a.bo, D, rows};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, MNMAJ, 128, EpBiasF>), dim3(D / BN, mt), nt, 0, st, O, (int)D3, rows,
                       static_cast<const T*>(a.Wo), D, D, D, eg);
    hipLaunchKernelGGL(k_gate_bwd<T>, dim3((D + 255) / 256, nslab), dim3(256), 0, st, a.G,
                       static_cast<const T*>(a.dY), a.alpha, a.rows, D, static_cast<T*>(a.dG), a.part);
    hipLaunchKernelGGL(k_slabs, dim3((D + 255) / 256), dim3(256), 0, st, a.part, nslab, 2 * (int64_t)D, D, a.dalpha);
    if (a.dbo)
      hipLaunchKernelGGL(k_slabs, dim3((D + 255) / 256), dim3(256), 0, st, a.part + D, nslab, 2 * (int64_t)D, D,
                         a.dbo);
    EpBiasF ew{{}, a.dWo, nullptr, D, D};
    hipLaunchKernelGGL((k_gemm<T, MNMAJ, MNMAJ, 128, EpBiasF>), dim3(D / BN, D / 128), nt, 0, st, O, (int)D3, rows,
                       static_cast<const T*>(a.dG), D, rows, rows, ew);
    EpBiasT<T> eo{{}, static_cast<T*>(a.dO), nullptr, D3, rows};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, 128, EpBiasT<T>>), dim3(D / BN, mt), nt, 0, st,
                       static_cast<const T*>(a.dG), D, rows, static_cast<const T*>(a.Wo), D, D, D, eo);
  } else {
    const T* dP = static_cast<const T*>(a.dP);
    EpBiasF ew{{}, a.dWqkv, nullptr, D3, D};
    hipLaunchKernelGGL((k_gemm<T, MNMAJ, MNMAJ, 128, EpBiasF>), dim3(3 * D / BN, D / 128), nt, 0, st,
                       static_cast<const T*>(a.X), D, rows, dP, (int)D3, rows, rows, ew);
    if (a.dbqkv) {
      hipLaunchKernelGGL(k_colsum<T>, dim3((3 * D + 255) / 256, nslab), dim3(256), 0, st, dP, D3, a.rows, 3 * D,
                         a.part);
      hipLaunchKernelGGL(k_slabs, dim3((3 * D + 255) / 256), dim3(256), 0, st, a.part, nslab, D3, 3 * D, a.dbqkv);
    }
    EpAddT<T> ex{{}, static_cast<T*>(a.dX), static_cast<const T*>(a.dY), D, rows};
    hipLaunchKernelGGL((k_gemm<T, KMAJ, KMAJ, 128, EpAddT<T>>), dim3(D / BN, mt), nt, 0, st, dP, (int)D3, rows,
                       static_cast<const T*>(a.Wqkv), (int)D3, D, (int)D3, ex);
  }
  return hipGetLastError();
}

}  // namespace large

hipError_t launch_gcm_gemm(const GcmGemmArgs& a, bool io_bf16, hipStream_t st) {
  return io_bf16 ? large::gcm_t<bf16>(a, st) : large::gcm_t<float>(a, st);
}

hipError_t launch_gcm_bwd(const GcmBwdArgs& a, bool io_bf16, hipStream_t st) {
  return io_bf16 ? large::gcm_bwd_t<bf16>(a, st) : large::gcm_bwd_t<float>(a, st);
}

}  // namespace ttt
