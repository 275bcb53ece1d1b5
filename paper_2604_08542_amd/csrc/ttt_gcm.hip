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

}  // namespace large

hipError_t launch_gcm_gemm(const GcmGemmArgs& a, bool io_bf16, hipStream_t st) {
  return io_bf16 ? large::gcm_t<bf16>(a, st) : large::gcm_t<float>(a, st);
}

}  // namespace ttt
