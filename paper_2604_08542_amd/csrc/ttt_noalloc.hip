// ttt_chunk_fwd_noalloc: the chunked forward for callers that cannot
// allocate device memory or pass a workspace (code under HIP graph capture,
// tight serving loops).  Its scratch (shard partials, ping-pong weights,
// counters) is one file-scope device array of fixed size, which every GPU
// the library runs on holds until the process ends.  The array's address on
// a device is looked up once per device (hipGetSymbolAddress) and kept; host
// code never passes the array's own name to a kernel.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ttt.h"
#include "ttt_internal.h"

namespace {

constexpr size_t SCRATCH_BYTES = size_t(40) << 20;  // TTT_NOALLOC_SCRATCH_BYTES in include/ttt.h
static_assert(SCRATCH_BYTES == TTT_NOALLOC_SCRATCH_BYTES, "header and library agree on the scratch size");

__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;

struct ScratchPtrs {
  std::mutex mu;
  void* ptr[MAX_DEVICES] = {};
};

ScratchPtrs& scratch_ptrs() {
  static ScratchPtrs s;
  return s;
}

// The device address of `scratch` on the current device (looked up on the
// first call for that device), or null if the lookup failed.
void* scratch_on_current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  ScratchPtrs& s = scratch_ptrs();
  std::lock_guard<std::mutex> g(s.mu);
  if (!s.ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    s.ptr[dev] = p;
  }
  return s.ptr[dev];
}

}  // namespace

extern "C" ttt_status_t ttt_chunk_fwd_noalloc(const ttt_problem_t* p, const void* Q, const void* K, const void* V,
                                              const float* W1_0, const float* W2_0, void* O, float* W1_T,
                                              float* W2_T, float* ckpt, float* loss, void* hip_stream) {
  try {
    return ttt::chunk_fwd_impl(p, Q, K, V, W1_0, W2_0, O, W1_T, W2_T, ckpt, loss, nullptr, SCRATCH_BYTES,
                               scratch_on_current_device, static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return TTT_EINVAL;
  }
}
