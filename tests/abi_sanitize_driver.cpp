// Host-side driver for the sanitizer check of the C ABI layer: linked against
// an AddressSanitizer + UndefinedBehaviorSanitizer (host) build of
// ttt_abi.cpp and the library's kernel objects.  Every call below is
// rejected, or is a no-op, before the library reaches a HIP call, so no GPU
// is needed; the sanitizers watch the validation and workspace-sizing code on
// the way.  Exits non-zero if any call returns an unexpected status.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>

#include "../include/ttt.h"

namespace {

int failures = 0;

void expect(int line, ttt_status_t got, ttt_status_t want) {
  if (got != want) {
    std::fprintf(stderr, "line %d: status %d (%s), expected %d\n", line, (int)got, ttt_status_string(got), (int)want);
    ++failures;
  }
}
#define EXPECT(call, want) expect(__LINE__, (call), (want))

ttt_problem_t prob() {
  ttt_problem_t p;
  std::memset(&p, 0, sizeof p);
  p.n_heads = 16;
  p.d_head = 64;
  p.d_hidden = 256;
  p.n_tokens = 87936;
  p.chunk_tokens = 10992;
  p.eta = 0.05f;
  p.flags = TTT_NORM_Q | TTT_NORM_K | TTT_NORM_V;
  p.io_dtype = TTT_F32;
  return p;
}

// A stand-in device address: never dereferenced, validation fails first.
void* const FAKE = reinterpret_cast<void*>(uintptr_t(1) << 20);
float* const FF = static_cast<float*>(FAKE);
const size_t BIG = size_t(1) << 40;

ttt_status_t fwd(const ttt_problem_t& p, const void* Q = FAKE, void* ws = FAKE, size_t nws = BIG,
                 float* ckpt = nullptr, float* loss = nullptr, float* W1T = nullptr) {
  return ttt_chunk_fwd(&p, Q, FAKE, FAKE, FF, FF, FAKE, W1T, nullptr, ckpt, loss, ws, nws, nullptr);
}

}  // namespace

int main() {
  // workspace sizing over many shapes (and the invalid ones)
  {
    ttt_problem_t p = prob();
    const size_t n1 = ttt_workspace_bytes(&p, 1), n8 = ttt_workspace_bytes(&p, 8);
    if (n1 == 0 || n8 < n1) ++failures;
    const int hs[] = {128, 256};
    for (int h : hs)
      for (int H = 1; H <= 64; H *= 2)
        for (int64_t M = 1; M <= 20000; M = M * 7 + 3) {
          ttt_problem_t q = prob();
          q.d_hidden = h;
          q.n_heads = H;
          q.chunk_tokens = M;
          for (int B = 1; B <= 128; B *= 4)
            if (ttt_workspace_bytes(&q, B) == 0) ++failures;
        }
    const int big[][2] = {{256, 512}, {1024, 4096}, {4096, 16384}, {512, 128}};
    for (auto& dh : big) {
      ttt_problem_t q = prob();
      q.n_heads = 1;
      q.d_head = dh[0];
      q.d_hidden = dh[1];
      q.chunk_tokens = 2748;
      if (ttt_workspace_bytes(&q, 1) == 0) ++failures;
    }
    ttt_problem_t bad[8];
    for (auto& b : bad) b = prob();
    bad[0].d_head = 32;
    bad[1].d_hidden = 192;
    bad[2].chunk_tokens = 0;
    bad[3].n_heads = 0;
    const int32_t seven = 7;  // a dtype code outside the enumeration, as a C caller could store it
    std::memcpy(&bad[4].io_dtype, &seven, sizeof seven);
    bad[5].flags = 1u << 20;
    bad[6].stride_tok = 3;
    bad[7].eta = std::numeric_limits<float>::infinity();
    for (auto& b : bad)
      if (ttt_workspace_bytes(&b, 1) != 0) ++failures;
    if (ttt_workspace_bytes(&p, 0) != 0 || ttt_workspace_bytes(nullptr, 1) != 0) ++failures;
    if (ttt_amu_workspace_bytes(&p) == 0 || ttt_amu_bwd_workspace_bytes(&p, TTT_SYNC_CHAIN) == 0 ||
        ttt_amu_bwd_workspace_bytes(&p, 5) != 0)
      ++failures;
  }
  // forward validation
  {
    ttt_problem_t p = prob();
    ttt_problem_t q = p;
    q.d_head = 32;
    EXPECT(fwd(q), TTT_ESHAPE);
    q = p;
    q.d_hidden = 64;
    EXPECT(fwd(q), TTT_ESHAPE);
    q = p;
    q.eta = std::nanf("");
    EXPECT(fwd(q), TTT_EINVAL);
    EXPECT(fwd(p, nullptr), TTT_EINVAL);
    EXPECT(fwd(p, FAKE, FAKE, BIG, nullptr, nullptr, FF), TTT_EINVAL);  // W1_T without W2_T
    q = p;
    q.flags |= TTT_SAVE_CKPT;
    EXPECT(fwd(q), TTT_EINVAL);
    EXPECT(fwd(p, FAKE, FAKE, BIG, FF), TTT_EINVAL);
    q = p;
    q.flags |= TTT_EMIT_LOSS;
    EXPECT(fwd(q), TTT_EINVAL);
    EXPECT(fwd(p, static_cast<char*>(FAKE) + 4), TTT_EINVAL);  // misaligned
    EXPECT(fwd(p, FAKE, nullptr), TTT_EWORKSPACE);
    EXPECT(fwd(p, FAKE, FAKE, 16), TTT_EWORKSPACE);
    q = p;
    q.stride_tok = (int64_t(1) << 22) + 64;
    EXPECT(fwd(q), TTT_ESHAPE);
    q = p;
    q.n_tokens = 0;
    EXPECT(fwd(q), TTT_OK);
    EXPECT(ttt_chunk_fwd(&q, nullptr, nullptr, nullptr, FF, FF, nullptr, nullptr, nullptr, nullptr, nullptr, FAKE,
                         BIG, nullptr),
           TTT_OK);  // empty stream: null token pointers accepted
    // large state: the forward validates the GEMM operand limit
    q = p;
    q.n_heads = 1;
    q.d_head = 4096;
    q.d_hidden = 16384;
    q.chunk_tokens = q.n_tokens = 1 << 20;
    EXPECT(fwd(q), TTT_ESHAPE);
    q.chunk_tokens = 2748;
    EXPECT(fwd(q, FAKE, nullptr), TTT_EWORKSPACE);
  }
  // backward, GCS, batched
  {
    ttt_problem_t p = prob();
    EXPECT(ttt_chunk_bwd(&p, FAKE, FAKE, FAKE, FF, FF, nullptr, FAKE, FAKE, FAKE, FAKE, FF, FF, FF, FAKE, BIG,
                         nullptr),
           TTT_EINVAL);  // no checkpoints
    EXPECT(ttt_chunk_bwd(&p, FAKE, FAKE, FAKE, FF, FF, FF, FAKE, FAKE, FAKE, FAKE, FF, FF, FF, nullptr, BIG, nullptr),
           TTT_EWORKSPACE);
    EXPECT(ttt_gcs_fwd(&p, FAKE, FAKE, FAKE, FF, FF, FAKE, nullptr, nullptr, nullptr, nullptr, BIG, nullptr),
           TTT_EWORKSPACE);
    ttt_problem_t q = p;
    q.flags |= TTT_SAVE_CKPT;
    EXPECT(ttt_gcs_fwd(&q, FAKE, FAKE, FAKE, FF, FF, FAKE, nullptr, nullptr, nullptr, FAKE, BIG, nullptr),
           TTT_EINVAL);
    EXPECT(ttt_gcs_bwd(&p, FAKE, FAKE, FAKE, FF, FF, FAKE, FAKE, FAKE, FAKE, FF, FF, nullptr, FAKE, BIG, nullptr),
           TTT_EINVAL);  // no deta
    const int64_t bad_cu[4] = {0, 10, 5, 20}, cu0[2] = {5, 10}, empty[3] = {0, 0, 0}, good[3] = {0, 10, 30};
    q = p;
    q.n_tokens = 0;
    auto bat = [&](int n, const int64_t* cu, int w0, const ttt_tile_cfg_t* cfg, void* ws) {
      return ttt_batched_fwd(&q, n, cu, FAKE, FAKE, FAKE, FF, FF, w0, FAKE, nullptr, nullptr, cfg, ws, BIG, nullptr);
    };
    EXPECT(bat(3, bad_cu, 0, nullptr, FAKE), TTT_EINVAL);
    EXPECT(bat(1, cu0, 0, nullptr, FAKE), TTT_EINVAL);
    EXPECT(bat(0, empty, 0, nullptr, FAKE), TTT_EINVAL);
    EXPECT(bat(2, empty, 2, nullptr, FAKE), TTT_EINVAL);
    EXPECT(bat(2, empty, 0, nullptr, FAKE), TTT_OK);
    ttt_tile_cfg_t cfg{-1, 0, 0, 0};
    EXPECT(bat(2, good, 0, &cfg, FAKE), TTT_EINVAL);
    EXPECT(bat(2, good, 0, nullptr, nullptr), TTT_EWORKSPACE);
    q.flags |= TTT_SAVE_CKPT;
    EXPECT(ttt_batched_fwd_ckpt(&q, 2, bad_cu, FAKE, FAKE, FAKE, FF, FF, 0, FAKE, nullptr, nullptr, FF, nullptr,
                                FAKE, BIG, nullptr),
           TTT_EINVAL);
    EXPECT(ttt_batched_bwd(&q, 2, good, FAKE, FAKE, FAKE, FF, FF, 3, FF, FAKE, FAKE, FAKE, FAKE, FF, FF, FF, nullptr,
                           FAKE, BIG, nullptr),
           TTT_EINVAL);
  }
  // the paper's memory unit
  {
    ttt_problem_t p = prob();
    p.n_tokens = 1000;
    p.chunk_tokens = 100;
    EXPECT(ttt_amu_fwd(&p, 2, FAKE, FAKE, FAKE, FF, FF, FF, FF, FAKE, nullptr, nullptr, nullptr, FAKE, BIG, nullptr),
           TTT_EINVAL);
    EXPECT(ttt_amu_fwd(&p, 0, FAKE, FAKE, FAKE, nullptr, FF, FF, FF, FAKE, nullptr, nullptr, nullptr, FAKE, BIG,
                       nullptr),
           TTT_EINVAL);
    EXPECT(ttt_amu_fwd(&p, 0, FAKE, FAKE, FAKE, FF, FF, FF, FF, FAKE, nullptr, nullptr, nullptr, nullptr, BIG,
                       nullptr),
           TTT_EWORKSPACE);
    EXPECT(ttt_amu_bwd(&p, 0, FAKE, FAKE, FAKE, FF, FF, FF, FF, nullptr, FAKE, FAKE, FAKE, FF, FF, FF, FF, FAKE, BIG,
                       nullptr),
           TTT_EINVAL);
  }
  // the layer around the memory unit
  {
    ttt_problem_t p = prob();
    p.n_tokens = 5000;
    p.chunk_tokens = 1000;
    if (ttt_gcm_workspace_bytes(&p) == 0) ++failures;
    ttt_problem_t q = p;
    q.n_heads = 1;  // D = 64: not a multiple of 128
    if (ttt_gcm_workspace_bytes(&q) != 0) ++failures;
    q = p;
    q.stride_tok = 2048;  // the layer's tensors are packed
    if (ttt_gcm_workspace_bytes(&q) != 0) ++failures;
    auto gcm = [&](const ttt_problem_t& pp, const float* alpha, void* ws, size_t nws) {
      return ttt_gcm_fwd(&pp, FAKE, FAKE, nullptr, FAKE, nullptr, alpha, FF, FF, FAKE, nullptr, nullptr, ws, nws,
                         nullptr);
    };
    EXPECT(gcm(p, nullptr, FAKE, BIG), TTT_EINVAL);
    EXPECT(gcm(p, FF, nullptr, BIG), TTT_EWORKSPACE);
    EXPECT(gcm(p, FF, FAKE, 64), TTT_EWORKSPACE);
    q = p;
    q.flags |= TTT_SAVE_CKPT;
    EXPECT(gcm(q, FF, FAKE, BIG), TTT_ENOTSUP);
    q = p;
    q.n_heads = 1;
    EXPECT(gcm(q, FF, FAKE, BIG), TTT_ESHAPE);
  }
  // status strings
  for (int s = 0; s < 6; ++s)
    if (ttt_status_string((ttt_status_t)s) == nullptr) ++failures;
  if (ttt_version() < 100) ++failures;
  std::printf("sanitizer driver: %d failure(s)\n", failures);
  return failures == 0 ? 0 : 1;
}
