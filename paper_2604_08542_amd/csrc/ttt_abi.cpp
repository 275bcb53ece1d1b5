// C ABI of the chunked TTT library: argument validation, workspace layout,
// launch planning (work-groups per chain, active-sequence lists per chunk
// step) and the stream-ordered launch sequence.  No device memory is
// allocated here and the stream is never synchronised.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>
#include <vector>

#include "../../include/ttt.h"
#include "ttt_internal.h"
#include "ttt_tuned.h"

namespace {

using namespace ttt;

constexpr uint32_t KNOWN_FLAGS = TTT_NORM_Q | TTT_NORM_K | TTT_NORM_V | TTT_SAVE_CKPT | TTT_EMIT_LOSS | TTT_MMA_BF16;
constexpr int64_t SLOT_CAP_MIN = 1024;  // shard-partial slots available per chunk step
constexpr int64_t MAX_STRIDE_TOK = int64_t(1) << 22;  // elements; token tiles are addressed with 32-bit offsets
constexpr size_t ALIGN = 256;

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

struct Shape {
  int H, d, h;
  int64_t M, stride_tok, stride_head;
  bool io_bf16, mma_bf16;
  bool large;  // d >= 256: the streamed-weight (GEMM) chunk step
  int64_t Mrows;
  int64_t dh() const { return (int64_t)d * h; }
};

// Large state sizes (the paper's one head of 1024 with hidden 4096 and
// similar): d a multiple of 256 up to 4096, h a multiple of 128 up to 16384.
bool large_shape(int d, int h) {
  return d >= 256 && d <= 4096 && d % 256 == 0 && h >= 128 && h <= 16384 && h % 128 == 0;
}

ttt_status_t check_problem(const ttt_problem_t* p, Shape* s) {
  if (!p) return TTT_EINVAL;
  if (p->n_heads < 1 || p->chunk_tokens < 1 || p->n_tokens < 0) return TTT_EINVAL;
  if (!std::isfinite(p->eta)) return TTT_EINVAL;
  if (p->flags & ~KNOWN_FLAGS) return TTT_EINVAL;
  // the dtype field is read as an integer: a C caller may store any value
  // there, and loading one outside the enumeration as the enum type is
  // undefined in C++
  int32_t io_dtype;
  static_assert(sizeof(io_dtype) == sizeof(p->io_dtype), "ttt_dtype_t is a 32-bit enum");
  std::memcpy(&io_dtype, &p->io_dtype, sizeof io_dtype);
  if (io_dtype != TTT_F32 && io_dtype != TTT_BF16) return TTT_EINVAL;
  const bool large = large_shape(p->d_head, p->d_hidden);
  if (!large && (p->d_head != 64 || (p->d_hidden != 128 && p->d_hidden != 256))) return TTT_ESHAPE;
  const int64_t st = p->stride_tok ? p->stride_tok : (int64_t)p->n_heads * p->d_head;
  const int64_t sh = p->stride_head ? p->stride_head : p->d_head;
  if (st <= 0 || sh <= 0 || (st % 8) || (sh % 8)) return TTT_ESHAPE;
  if (st > MAX_STRIDE_TOK) return TTT_ESHAPE;  // a 32-token tile spans < 2^31 bytes
  s->H = p->n_heads;
  s->d = p->d_head;
  s->h = p->d_hidden;
  s->M = p->chunk_tokens;
  s->stride_tok = st;
  s->stride_head = sh;
  s->io_bf16 = io_dtype == TTT_BF16;
  s->mma_bf16 = s->io_bf16 || (p->flags & TTT_MMA_BF16);
  s->large = large;
  // rows of one chunk as the large-state step buffers them: the chunk size,
  // or the whole stream when it is shorter (single-sequence calls)
  s->Mrows = p->n_tokens > 0 ? std::min<int64_t>(s->M, p->n_tokens) : s->M;
  if (large) {
    // the GEMM operand buffers are addressed with 32-bit byte offsets
    const int64_t op = s->mma_bf16 ? 2 : 4;
    if (s->Mrows * std::max(s->d, s->h) * op >= (int64_t(1) << 31)) return TTT_ESHAPE;
  }
  return TTT_OK;
}

// Workspace of the large-state chunk step (one chunk of one head at a time):
// the chunk's normalised rows and intermediate products, the FP32 masters and
// their operand copies, the loss partials.
struct LargeLayout {
  size_t sync, Kn, Qn, E, A, D, Aq, Vn, S1, W1, W2, W1op, W2op, loss_part, total;
};
LargeLayout large_layout(const Shape& s) {
  LargeLayout L{};
  const size_t op = s.mma_bf16 ? 2 : 4;
  const size_t M = (size_t)s.Mrows, d = (size_t)s.d, h = (size_t)s.h;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) / 256 * 256;
    return o;
  };
  L.sync = take(256);  // word 0: the device error word (no barrier here; kept clear)
  L.Kn = take(M * d * op);
  L.Qn = take(M * d * op);
  L.E = take(M * d * op);
  L.A = take(M * h * op);
  L.D = take(M * h * op);
  L.Aq = take(M * h * op);
  L.Vn = take(M * d * 4);
  L.S1 = take((M + 127) / 128 * 128 * h * op);  // tile-native: whole 128-row tiles
  L.W1 = take(d * h * 4);
  L.W2 = take(d * h * 4);
  L.W1op = take(d * h * op);
  L.W2op = take(d * h * op);
  L.loss_part = take((d / 128) * ((M + 127) / 128) * 4);
  L.total = off;
  return L;
}

// Workspace of the reverse mode at large state sizes: the forward's layout
// (its step recomputes the weights after the last chunk) followed by the
// reverse step's buffers.
struct LargeBwdLayout {
  LargeLayout f;
  size_t dOn, dY, dq, dk, dv, dE, S2, P, Sq1, dZq, dP, dZa, EWh, dZ, W1nop, W2nop, Wh1, Wh2, Wh1op, Wh2op, tot1, tot2,
      deta_part, deta, total;
};
LargeBwdLayout large_bwd_layout(const Shape& s) {
  LargeBwdLayout L{};
  L.f = large_layout(s);
  const size_t op = s.mma_bf16 ? 2 : 4;
  const size_t M = (size_t)s.Mrows, d = (size_t)s.d, h = (size_t)s.h;
  size_t off = L.f.total;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) / 256 * 256;
    return o;
  };
  L.dOn = take(M * d * op);
  L.dY = take(M * d * op);
  L.dq = take(M * d * 4);
  L.dk = take(M * d * 4);
  L.dv = take(M * d * 4);
  L.dE = take(M * d * 4);
  L.S2 = take((M + 127) / 128 * 128 * h * op);  // tile-native
  L.P = take((M + 127) / 128 * 128 * h * op);  // tile-native
  L.Sq1 = take((M + 127) / 128 * 128 * h * op);  // tile-native
  L.dZq = take(M * h * op);
  L.dP = take(M * h * op);
  L.dZa = take((M + 127) / 128 * 128 * h * op);  // tile-native
  L.EWh = take(M * h * op);
  L.dZ = take(M * h * op);
  L.W1nop = take(d * h * op);
  L.W2nop = take(d * h * op);
  L.Wh1 = take(d * h * 4);
  L.Wh2 = take(d * h * 4);
  L.Wh1op = take(d * h * op);
  L.Wh2op = take(d * h * op);
  L.tot1 = take(d * h * 4);  // GCS: the adjoint of W0 (the apply adjoint plus every chunk's update terms)
  L.tot2 = take(d * h * 4);
  L.deta_part = take((d / 128 + h / 128) * ((M + 127) / 128) * 4);
  L.deta = take(4);
  L.total = off;
  return L;
}

// Workspace of the memory unit's large-state chunk step: the chunk's
// normalised rows, E, the [rows][h] intermediates, three FP32 masters and
// their operand copies.
struct LargeAmuLayout {
  size_t sync, Kn, Qn, E, Vn, Z3, Hd, G1, G3, D1, D3, W1, W2, W3, W1op, W2op, W3op, total;
};
LargeAmuLayout large_amu_layout(const Shape& s) {
  LargeAmuLayout L{};
  const size_t op = s.mma_bf16 ? 2 : 4;
  const size_t M = (size_t)s.Mrows, d = (size_t)s.d, h = (size_t)s.h;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) / 256 * 256;
    return o;
  };
  L.sync = take(256);
  L.Kn = take(M * d * op);
  L.Qn = take(M * d * op);
  L.E = take(M * d * op);
  L.Vn = take(M * d * 4);
  const size_t Mt = (M + 127) / 128 * 128;  // Z3, G1, G3 tile-native in the forward step: whole 128-row tiles
  L.Z3 = take(Mt * h * op);
  L.Hd = take(M * h * op);
  L.G1 = take(Mt * h * op);
  L.G3 = take(Mt * h * op);
  L.D1 = take(M * h * op);
  L.D3 = take(M * h * op);
  L.W1 = take(d * h * 4);
  L.W2 = take(d * h * 4);
  L.W3 = take(d * h * 4);
  L.W1op = take(d * h * op);
  L.W2op = take(d * h * op);
  L.W3op = take(d * h * op);
  L.total = off;
  return L;
}

// Workspace of the paper's unit's reverse mode at large state sizes: the
// forward step's layout (it recomputes the weights), the reverse step's
// buffers, and for the chain the weights before every chunk and after the
// last ([C+1][3][d h] FP32).
struct LargeAmuBwdLayout {
  LargeAmuLayout f;
  size_t dOn, Ydot, dq, dk, dv, S, S1, S2, Zd3, Sd, Hdot, T2, dHh, aZ1, aZ3, aZd1, aZd3, Wnop[3], Wh[3], Whop[3],
      tot[3], wlist, total;
};
LargeAmuBwdLayout large_amu_bwd_layout(const Shape& s, int64_t n_tokens, int sync) {
  LargeAmuBwdLayout L{};
  L.f = large_amu_layout(s);
  const size_t op = s.mma_bf16 ? 2 : 4;
  const size_t M = (size_t)s.Mrows, d = (size_t)s.d, h = (size_t)s.h;
  size_t off = L.f.total;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) / 256 * 256;
    return o;
  };
  L.dOn = take(M * d * op);
  L.Ydot = take(M * d * 4);
  L.dq = take(M * d * 4);
  L.dk = take(M * d * 4);
  L.dv = take(M * d * 4);
  // whole 128-row tiles: S, S1, S2, Zd3, Sd, T2, dHh are tile-native in the reverse step
  for (size_t* b : {&L.S, &L.S1, &L.S2, &L.Zd3, &L.Sd, &L.Hdot, &L.T2, &L.dHh, &L.aZ1, &L.aZ3, &L.aZd1, &L.aZd3})
    *b = take((M + 127) / 128 * 128 * h * op);
  for (int m = 0; m < 3; ++m) {
    L.Wnop[m] = take(d * h * op);
    L.Wh[m] = take(d * h * 4);
    L.Whop[m] = take(d * h * op);
    L.tot[m] = take(d * h * 4);
  }
  const int64_t C = (n_tokens + s.M - 1) / s.M;
  L.wlist = take(sync == TTT_SYNC_CHAIN ? (size_t)(C + 1) * 3 * d * h * 4 : 0);
  L.total = off;
  return L;
}

struct WsLayout {
  size_t sync, partial, partial_loss, pp, adj, wlast, prep, fin, deta_seq, total;
  int64_t slot_cap;
};

// Words at the start of every workspace: the device error word (word 0, read
// by ttt_workspace_status), the persistent forward's chain counter (word 1),
// its group barrier counters, group chain slots and group XCD sets.
constexpr int SYNC_ERR = 0, SYNC_NEXT = 1, SYNC_BAR = 4;
constexpr int MAX_GROUPS = 2048;
constexpr size_t SYNC_BYTES = (size_t)(SYNC_BAR + 3 * MAX_GROUPS) * sizeof(uint32_t);

// n_chains = sequences x heads of the call.
WsLayout ws_layout(const Shape& s, int64_t n_chains) {
  WsLayout L{};
  L.slot_cap = std::max<int64_t>(n_chains, SLOT_CAP_MIN);
  const size_t wbytes = (size_t)2 * s.dh() * sizeof(float);  // one chain's [W1 | W2]
  size_t off = 0;
  L.sync = off;
  off = align_up(off + SYNC_BYTES);
  L.partial = off;
  off = align_up(off + (size_t)L.slot_cap * wbytes);
  L.partial_loss = off;
  off = align_up(off + (size_t)L.slot_cap * sizeof(float));
  L.pp = off;  // forward: ping-pong weights per chain
  off = align_up(off + 2 * (size_t)n_chains * wbytes);
  // backward: two adjoint buffers per chain, the recomputed last weights,
  // operand copies (8 matrices per chain of one launch, float-sized slots),
  // per-sequence final adjoints and d(eta) sums (shared initial weights)
  L.adj = off;
  off = align_up(off + 2 * (size_t)n_chains * wbytes);
  L.wlast = off;
  off = align_up(off + (size_t)n_chains * wbytes);
  L.prep = off;
  off = align_up(off + (size_t)std::min<int64_t>(n_chains, (int64_t)MAXS * s.H) * 8 * s.dh() * sizeof(float));
  L.fin = off;
  off = align_up(off + (size_t)n_chains * wbytes);
  L.deta_seq = off;
  off = align_up(off + (size_t)n_chains * sizeof(float));
  L.total = off;
  return L;
}

// A forward-only layout inside `capacity` bytes (the fixed scratch of
// ttt_chunk_fwd_noalloc): the error word and counters, as many shard-partial
// slots as fit, and the ping-pong weights of every chain.  slot_cap < n_chains
// means the problem does not fit (not even one work-group per chain).
WsLayout fwd_layout_in(const Shape& s, int64_t n_chains, size_t capacity) {
  WsLayout L{};
  const size_t wbytes = (size_t)2 * s.dh() * sizeof(float);
  const size_t fixed = align_up(SYNC_BYTES) + align_up(2 * (size_t)n_chains * wbytes) + 2 * ALIGN;
  const int64_t slots = capacity > fixed ? (int64_t)((capacity - fixed) / (wbytes + sizeof(float))) : 0;
  L.slot_cap = slots;
  size_t off = 0;
  L.sync = off;
  off = align_up(off + SYNC_BYTES);
  L.partial = off;
  off = align_up(off + (size_t)slots * wbytes);
  L.partial_loss = off;
  off = align_up(off + (size_t)slots * sizeof(float));
  L.pp = off;
  off = align_up(off + 2 * (size_t)n_chains * wbytes);
  L.adj = L.wlast = L.prep = L.fin = L.deta_seq = off;  // not used by the forward
  L.total = off;
  return L;
}

int default_target_wgs(const Shape& s) { return s.h == 256 ? 256 : 512; }

// The launch shape of a call: the caller's, else the autotuner's recorded
// shape for this (h, operand path, chunk size, chains, direction), else the
// built-in heuristic (stepwise schedule, automatic sizes).
ttt_tile_cfg_t resolve_cfg(const ttt_tile_cfg_t* given, const Shape& S, int64_t n_chains, bool bwd) {
  if (given) return *given;
  const bool f32_ops = !S.io_bf16 && !S.mma_bf16;
  for (const TunedShape& t : kTuned) {
    if (t.h == S.h && t.chunk_tokens == S.M && t.chains == n_chains && (t.bwd != 0) == bwd &&
        ((t.bf16 != 0) == S.io_bf16) && (S.io_bf16 || f32_ops))
      return t.cfg;
  }
  ttt_tile_cfg_t c{};
  c.schedule = TTT_SCHED_STEPWISE;
  return c;
}

// A launch helper: true when the launch was accepted.
template <typename F>
bool launched(F&& f) {
  return f() == hipSuccess;
}

template <typename T> T* at(void* base, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(base) + off); }

// Sequences without tokens take no chunk step: their final weights (when
// asked for) are their initial weights.
// Also clears the workspace's error word when there are tokens: every
// forward call starts here (a call without tokens enqueues nothing else).
ttt_status_t copy_w0_to_final(const Shape& S, int B, const int64_t* cu, const float* W1_0, const float* W2_0,
                              int w0_per_seq, float* W1_T, float* W2_T, void* ws, size_t ws_bytes, hipStream_t st,
                              const WsLayout* layout = nullptr) {
  const WsLayout L = layout ? *layout : ws_layout(S, (int64_t)B * S.H);
  if (!ws || ws_bytes < L.total) return TTT_EWORKSPACE;
  if (cu[B] > 0 &&
      !launched([&] { return launch_zero_words(at<uint32_t>(ws, L.sync) + SYNC_ERR, 1, st); }))
    return TTT_EHIP;
  if (!W1_T) return TTT_OK;
  const int64_t dh = S.dh();
  for (int b = 0; b < B; ++b) {
    if (cu[b + 1] > cu[b]) continue;
    const int64_t src = (int64_t)(w0_per_seq ? b : 0) * S.H * dh, dst = (int64_t)b * S.H * dh;
    if (hipMemcpyAsync(W1_T + dst, W1_0 + src, S.H * dh * sizeof(float), hipMemcpyDeviceToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(W2_T + dst, W2_0 + src, S.H * dh * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess)
      return TTT_EHIP;
  }
  return TTT_OK;
}

// ---------------------------------------------------------------- persistent forward
// Launch shape of the persistent forward: groups of G work-groups, each group
// walking whole chains.  Every work-group of the grid must be resident at
// once (the groups wait for each other at barriers), so the grid is sized
// from this kernel's occupancy; with 8 XCDs the groups are laid out so that
// each group's members share one XCD (and its L2).
struct PersistPlan {
  int G = 0, n_groups = 0, grid = 0;
  bool xcd = false;
};

ttt_status_t plan_persist(const Shape& S, const std::vector<int64_t>& nb, int64_t M, const ttt_tile_cfg_t* cfg,
                          int64_t slot_cap, PersistPlan* out) {
  int bpc = 0, threads = 0, dev = 0, n_cu = 0;
  if (persist_occupancy(S.h, S.io_bf16, S.mma_bf16, &bpc, &threads) != hipSuccess || bpc < 1) return TTT_EHIP;
  if (hipGetDevice(&dev) != hipSuccess) return TTT_EHIP;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1)
    return TTT_EHIP;
  const int64_t resident = (int64_t)bpc * n_cu;
  int64_t T = resident;
  if (cfg && cfg->target_wgs > 0) T = std::min<int64_t>(cfg->target_wgs, resident);
  int64_t n_chains = 0, L = 0, W = 0, tiles_max = 1;
  for (int64_t n : nb) {
    if (n <= 0) continue;
    const int64_t steps = (n + M - 1) / M + 1;
    n_chains += S.H;
    L = std::max(L, steps);
    W += steps * S.H;
    tiles_max = std::max(tiles_max, (std::min(n, M) + TT - 1) / TT);
  }
  if (n_chains == 0) return TTT_OK;
  int64_t G;
  if (cfg && cfg->wg_per_chain > 0) {
    G = cfg->wg_per_chain;
  } else {
    // enough members that the longest chain is not the critical path of a
    // longest-first list schedule, and enough to fill T when chains are few
    const int64_t g_lpt = (T * L + W - 1) / W;
    const int64_t g_fill = std::max<int64_t>(1, T / n_chains);
    G = 1;
    while (G < std::max(g_lpt, g_fill)) G *= 2;
  }
  // members past a chunk's tile count would have no tokens; the stepwise
  // schedule clamps its shards the same way, so both give the same partition
  G = std::max<int64_t>(1, std::min<int64_t>({G, tiles_max, resident}));
  int64_t n_groups = std::max<int64_t>(1, std::min<int64_t>(n_chains, T / G));
  if (n_groups >= 8) n_groups -= n_groups % 8;
  n_groups = std::min<int64_t>({n_groups, (int64_t)MAX_GROUPS, slot_cap / G});
  if (n_groups < 1) return TTT_EINVAL;
  const bool xcd = n_cu % 8 == 0 && G <= resident / 8;
  if (xcd) {
    const int64_t per_xcd = resident / 8;
    int64_t gpx = (n_groups + 7) / 8;
    while (gpx * G > per_xcd) --gpx;
    n_groups = std::min<int64_t>(n_groups, gpx * 8);
    out->grid = (int)(8 * gpx * G);
  } else {
    n_groups = std::min<int64_t>(n_groups, resident / G);
    out->grid = (int)(n_groups * G);
  }
  out->G = (int)G;
  out->n_groups = (int)n_groups;
  out->xcd = xcd;
  return TTT_OK;
}

constexpr uint32_t DEFAULT_SPIN_LIMIT = 1u << 22;  // polls of a barrier wait (about a second or more)

// The whole forward of B sequences in one persistent launch per MAXS
// sequences (non-empty sequences longest first).
ttt_status_t run_forward_persist(const ttt_problem_t* p, const Shape& S, int B, const int64_t* cu, const void* Q,
                                 const void* K, const void* V, const float* W1_0, const float* W2_0, int w0_per_seq,
                                 void* O, float* W1_T, float* W2_T, float* ckpt, float* loss,
                                 const ttt_tile_cfg_t* cfg, void* ws, size_t ws_bytes, hipStream_t st) {
  const int64_t nch_total = (int64_t)B * S.H;
  const WsLayout Lw = ws_layout(S, nch_total);
  if (!ws || ws_bytes < Lw.total) return TTT_EWORKSPACE;
  const int64_t M = S.M;
  std::vector<int64_t> nb(B), ckrow(B, 0);
  for (int b = 0; b < B; ++b) {
    nb[b] = cu[b + 1] - cu[b];
    if (b > 0) ckrow[b] = ckrow[b - 1] + (nb[b - 1] + M - 1) / M;
  }
  const ttt_status_t e0 = copy_w0_to_final(S, B, cu, W1_0, W2_0, w0_per_seq, W1_T, W2_T, ws, ws_bytes, st);
  if (e0 != TTT_OK || cu[B] == 0) return e0;
  PersistPlan plan;
  ttt_status_t e = plan_persist(S, nb, M, cfg, Lw.slot_cap, &plan);
  if (e != TTT_OK) return e;
  uint32_t* sync = at<uint32_t>(ws, Lw.sync);
  constexpr int SYNC_WORDS = SYNC_BAR + 3 * MAX_GROUPS;
  std::vector<int> order;
  for (int b = 0; b < B; ++b)
    if (nb[b] > 0) order.push_back(b);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return nb[x] > nb[y]; });
  for (size_t base = 0; base < order.size(); base += MAXS) {
    const int na = (int)std::min<size_t>(MAXS, order.size() - base);
    PersistArgs a{};
    a.Q = Q; a.K = K; a.V = V; a.O = O;
    a.stride_tok = S.stride_tok; a.stride_head = S.stride_head;
    a.w1_0 = W1_0; a.w2_0 = W2_0; a.w0_per_seq = w0_per_seq;
    a.H = S.H; a.flags = p->flags; a.eta = p->eta;
    a.G = plan.G; a.n_groups = plan.n_groups; a.n_chains = na * S.H; a.xcd_map = plan.xcd ? 1 : 0;
    a.spin_limit = (cfg && cfg->spin_limit > 0) ? (uint32_t)cfg->spin_limit : DEFAULT_SPIN_LIMIT;
    a.M = M;
    a.partial = at<float>(ws, Lw.partial);
    a.partial_loss = at<float>(ws, Lw.partial_loss);
    a.wbuf = at<float>(ws, Lw.pp);
    a.err = sync + SYNC_ERR;
    a.next = sync + SYNC_NEXT;
    a.bar = sync + SYNC_BAR;
    a.slot = sync + SYNC_BAR + MAX_GROUPS;
    a.xcds = sync + SYNC_BAR + 2 * MAX_GROUPS;
    a.ckpt = ckpt; a.wT1 = W1_T; a.wT2 = W2_T;
    a.loss = loss; a.loss_stride = (int32_t)((nb[0] + M - 1) / M);
    // schedule entry i (longest first) is sequence order[base + i]
    for (int i = 0; i < na; ++i) {
      const int b = order[base + i];
      a.seq_id[i] = b;
      a.seq_start[i] = cu[b];
      a.seq_len[i] = nb[b];
      a.ck_row[i] = ckrow[b];
    }
    // counters of this launch (and, for the call's first launch, the error word)
    const int z0 = base == 0 ? SYNC_ERR : SYNC_NEXT;
    if (!launched([&] { return launch_zero_words(sync + z0, SYNC_WORDS - z0, st); })) return TTT_EHIP;
    if (!launched([&] { return launch_fwd_persist(a, plan.grid, S.h, S.io_bf16, S.mma_bf16, st); }))
      return TTT_EHIP;
  }
  return TTT_OK;
}

// The whole forward: for s = 0..C_max, one fwd-step launch (gradient of chunk
// s, apply of chunk s-1) and, while any chunk s exists, one update launch.
ttt_status_t run_forward(const ttt_problem_t* p, const Shape& S, int B, const int64_t* cu, const void* Q,
                         const void* K, const void* V, const float* W1_0, const float* W2_0, int w0_per_seq,
                         void* O, float* W1_T, float* W2_T, float* ckpt, float* loss, const ttt_tile_cfg_t* cfg,
                         void* ws, size_t ws_bytes, hipStream_t st, const WsLayout* layout = nullptr) {
  const int64_t nch_total = (int64_t)B * S.H;
  const WsLayout L = layout ? *layout : ws_layout(S, nch_total);
  if (!ws || ws_bytes < L.total) return TTT_EWORKSPACE;
  const int64_t M = S.M;
  std::vector<int64_t> nb(B), cb(B);
  int64_t cmax = 0, nmax = 0;
  for (int b = 0; b < B; ++b) {
    nb[b] = cu[b + 1] - cu[b];
    cb[b] = (nb[b] + M - 1) / M;
    cmax = std::max(cmax, cb[b]);
    nmax = std::max(nmax, nb[b]);
  }
  if (cmax == 0) return TTT_OK;
  const int64_t dh = S.dh();
  std::vector<int64_t> ckoff(B, 0);  // checkpoint row of each sequence's chunk 0
  for (int b = 1; b < B; ++b) ckoff[b] = ckoff[b - 1] + cb[b - 1];
  float* partial = at<float>(ws, L.partial);
  float* partial_loss = at<float>(ws, L.partial_loss);
  float* pp[2] = {at<float>(ws, L.pp), at<float>(ws, L.pp) + nch_total * 2 * dh};
  const int64_t tiles_per_chunk = (std::min(M, nmax) + TT - 1) / TT;
  const int target = (cfg && cfg->target_wgs > 0) ? cfg->target_wgs : default_target_wgs(S);
  const int nbpc = (int)((2 * dh / 4 + 255) / 256);

  for (int64_t s = 0; s <= cmax; ++s) {
    std::vector<int> act;
    for (int b = 0; b < B; ++b)
      if (nb[b] > 0 && s <= cb[b]) act.push_back(b);
    if (act.empty()) continue;
    const int64_t n_chains = (int64_t)act.size() * S.H;
    int64_t G = (cfg && cfg->wg_per_chain > 0) ? cfg->wg_per_chain : (target + n_chains - 1) / n_chains;
    G = std::max<int64_t>(1, std::min<int64_t>({G, tiles_per_chunk, L.slot_cap / n_chains}));
    bool any_grad = false;
    for (size_t base = 0; base < act.size(); base += MAXS) {
      const int na = (int)std::min<size_t>(MAXS, act.size() - base);
      FwdStepArgs a{};
      a.Q = Q; a.K = K; a.V = V; a.O = O;
      a.stride_tok = S.stride_tok; a.stride_head = S.stride_head;
      if (s == 0) {
        a.w1_src = W1_0; a.w2_src = W2_0; a.w_cstride = dh;
        a.w_mod = w0_per_seq ? (int32_t)nch_total : S.H;
      } else {
        a.w1_src = pp[s % 2]; a.w2_src = pp[s % 2] + dh; a.w_cstride = 2 * dh;
        a.w_mod = (int32_t)nch_total;
      }
      a.H = S.H; a.flags = p->flags; a.G = (int32_t)G;
      const int64_t slot0 = (int64_t)base * S.H * G;
      a.partial = partial + slot0 * 2 * dh;
      a.partial_loss = partial_loss + slot0;
      a.n_active = na;
      UpdStepArgs u{};
      bool grad_here = false;
      for (int i = 0; i < na; ++i) {
        const int b = act[base + i];
        a.seq_id[i] = b;
        a.grad_start[i] = cu[b] + s * M;
        a.grad_len[i] = s < cb[b] ? (int32_t)std::min<int64_t>(M, nb[b] - s * M) : 0;
        a.app_start[i] = cu[b] + (s - 1) * M;
        a.app_len[i] = s >= 1 ? (int32_t)std::min<int64_t>(M, nb[b] - (s - 1) * M) : 0;
        u.seq_id[i] = b;
        u.ckpt_off[i] = (ckoff[b] + s) * S.H * 2 * dh;
        u.grad_len[i] = a.grad_len[i];
        u.is_last[i] = (s == cb[b] - 1);
        grad_here |= a.grad_len[i] > 0;
      }
      const int n_blocks = (int)(na * S.H * G);
      if (!launched([&] { return launch_fwd_step(a, n_blocks, S.h, S.io_bf16, S.mma_bf16, st); }))
        return TTT_EHIP;
      if (grad_here) {
        any_grad = true;
        u.w1_src = a.w1_src; u.w2_src = a.w2_src; u.w_cstride = a.w_cstride; u.w_mod = a.w_mod;
        u.H = S.H; u.h = S.h; u.eta = p->eta; u.G = (int32_t)G;
        u.partial = a.partial; u.partial_loss = a.partial_loss;
        u.w_dst = pp[(s + 1) % 2];
        u.ckpt = ckpt;
        u.wT1 = W1_T; u.wT2 = W2_T;
        u.loss = loss; u.loss_stride = (int32_t)cmax; u.chunk = (int32_t)s;
        u.n_active = na;
        if (!launched([&] { return launch_update(u, na * S.H * nbpc, st); })) return TTT_EHIP;
      }
    }
    (void)any_grad;
  }
  return TTT_OK;
}

// Backward over B sequences (B = 1 for ttt_chunk_bwd).  Every sequence's
// W_C is recomputed from its last checkpoint; then reverse step r = 0..C_max
// handles, for every sequence b with C_b >= r, its chunk s = C_b - r: one
// operand-preparation launch, one bwd-step launch (update adjoint of chunk
// s, apply adjoint of chunk s-1) and one reduction launch for all of them.
// Sequences are aligned at their last chunk, so a sequence's gradient is
// final (s = 0) at step C_b.
ttt_status_t run_backward(const ttt_problem_t* p, const Shape& S, int B, const int64_t* cu, int w0_per_seq,
                          const float* ckpt, const void* Q, const void* K, const void* V, const void* dO, void* dQ,
                          void* dK, void* dV, float* dW1_0, float* dW2_0, float* deta, const ttt_tile_cfg_t* cfg,
                          void* ws, size_t ws_bytes, hipStream_t st) {
  const int64_t H = S.H;
  const WsLayout L = ws_layout(S, (int64_t)B * H);
  if (!ws || ws_bytes < L.total) return TTT_EWORKSPACE;
  const int64_t M = S.M, dh = S.dh(), wsz = 2 * dh;
  std::vector<int64_t> nb(B), cb(B), ckoff(B, 0);
  int64_t cmax = 0, nmax = 0;
  for (int b = 0; b < B; ++b) {
    nb[b] = cu[b + 1] - cu[b];
    cb[b] = (nb[b] + M - 1) / M;
    if (b > 0) ckoff[b] = ckoff[b - 1] + cb[b - 1];
    cmax = std::max(cmax, cb[b]);
    nmax = std::max(nmax, nb[b]);
  }
  float* partial = at<float>(ws, L.partial);
  float* pdeta = at<float>(ws, L.partial_loss);
  float* adj[2] = {at<float>(ws, L.adj), at<float>(ws, L.adj) + B * H * wsz};
  float* wlast = at<float>(ws, L.wlast);
  void* prep = at<char>(ws, L.prep);
  float* fin = at<float>(ws, L.fin);
  float* deta_seq = B == 1 ? deta : at<float>(ws, L.deta_seq);
  const bool shared_w0 = B > 1 && !w0_per_seq;
  const ttt_tile_cfg_t rc = resolve_cfg(cfg, S, (int64_t)B * H, true);
  cfg = &rc;
  const int target = cfg->target_wgs > 0 ? cfg->target_wgs : default_target_wgs(S);
  const int nbpc = (int)((2 * dh / 4 + 255) / 256);
  const int64_t tiles = std::max<int64_t>((std::min(M, nmax) + TT - 1) / TT, 1);
  auto mlen = [&](int b, int64_t c) { return (int32_t)std::min<int64_t>(M, nb[b] - c * M); };

  // W_{C_b} = W_{C_b - 1} - eta * grad L_{C_b - 1}(W_{C_b - 1}) per sequence
  for (int b = 0; b < B; ++b) {
    if (cb[b] == 0) continue;
    const int64_t G = std::max<int64_t>(1, std::min<int64_t>({(target + H - 1) / H, tiles, L.slot_cap / H}));
    FwdStepArgs a{};
    a.Q = Q; a.K = K; a.V = V; a.O = nullptr;
    a.stride_tok = S.stride_tok; a.stride_head = S.stride_head;
    a.w1_src = ckpt + (ckoff[b] + cb[b] - 1) * H * wsz; a.w2_src = a.w1_src + dh; a.w_cstride = wsz;
    a.w_mod = (int32_t)H; a.H = (int32_t)H; a.flags = p->flags; a.G = (int32_t)G;
    a.partial = partial; a.partial_loss = pdeta; a.n_active = 1;
    a.seq_id[0] = 0; a.grad_start[0] = cu[b] + (cb[b] - 1) * M; a.grad_len[0] = mlen(b, cb[b] - 1);
    a.app_start[0] = 0; a.app_len[0] = 0;
    if (!launched([&] { return launch_fwd_step(a, (int)(H * G), S.h, S.io_bf16, S.mma_bf16, st); }))
      return TTT_EHIP;
    UpdStepArgs u{};
    u.w1_src = a.w1_src; u.w2_src = a.w2_src; u.w_cstride = a.w_cstride; u.w_mod = a.w_mod;
    u.H = (int32_t)H; u.h = S.h; u.eta = p->eta; u.G = (int32_t)G;
    u.partial = partial; u.partial_loss = pdeta; u.w_dst = wlast + b * H * wsz;
    u.n_active = 1; u.seq_id[0] = 0; u.grad_len[0] = a.grad_len[0]; u.is_last[0] = 0;
    if (!launched([&] { return launch_update(u, (int)(H * nbpc), st); })) return TTT_EHIP;
  }

  // With one launch group per step, each reduction also writes the operand
  // copies of the next step (its adjoint output is the next step's input).
  bool prep_ready = false;
  for (int64_t r = 0; r <= cmax; ++r) {
    std::vector<int> act;
    for (int b = 0; b < B; ++b)
      if (r <= cb[b]) act.push_back(b);
    std::vector<int> next_slot(B, -1);
    int n_next = 0;
    for (int b = 0; b < B; ++b)
      if (r + 1 <= cb[b]) next_slot[b] = n_next++;
    const bool fuse = r < cmax && (int64_t)act.size() <= MAXS && n_next <= MAXS;
    for (size_t base = 0; base < act.size(); base += MAXS) {
      const int na = (int)std::min<size_t>(MAXS, act.size() - base);
      const int64_t n_chains = (int64_t)na * H;
      int64_t G = (cfg && cfg->wg_per_chain > 0) ? cfg->wg_per_chain : (target + n_chains - 1) / n_chains;
      G = std::max<int64_t>(1, std::min<int64_t>({G, tiles, L.slot_cap / n_chains}));
      BwdPrepArgs pa{};
      pa.prep = prep; pa.H = (int32_t)H; pa.h = S.h;
      BwdStepArgs bs{};
      bs.Q = Q; bs.K = K; bs.V = V; bs.dO = dO; bs.dQ = dQ; bs.dK = dK; bs.dV = dV;
      bs.stride_tok = S.stride_tok; bs.stride_head = S.stride_head;
      bs.prep = prep; bs.H = (int32_t)H; bs.flags = p->flags; bs.eta = p->eta; bs.G = (int32_t)G;
      bs.partial = partial; bs.partial_deta = pdeta; bs.n_active = na;
      BwdReduceArgs rd{};
      rd.partial = partial; rd.partial_deta = pdeta; rd.n_active = na; rd.G = (int32_t)G;
      rd.H = (int32_t)H; rd.h = S.h;
      rd.wh_src_base = r == 0 ? nullptr : adj[(r + 1) % 2];
      rd.wh_dst_base = adj[r % 2];
      rd.fin_base = shared_w0 ? fin : nullptr;
      rd.dst1 = dW1_0; rd.dst2 = dW2_0; rd.dst_per_seq = w0_per_seq ? 1 : 0;
      rd.deta_base = deta_seq;
      if (fuse) {
        rd.prep_next = prep;
        rd.prep_bf16 = S.mma_bf16 ? 1 : 0;
        rd.ckpt = ckpt;
      }
      for (int i = 0; i < na; ++i) {
        const int b = act[base + i];
        const int64_t s = cb[b] - r;
        const float* whs = r == 0 ? nullptr : adj[(r + 1) % 2] + b * H * wsz;
        pa.w_src[i] = s < cb[b] ? ckpt + (ckoff[b] + s) * H * wsz : wlast + b * H * wsz;
        pa.wh_src[i] = whs;
        bs.grad_start[i] = cu[b] + s * M;
        bs.grad_len[i] = s < cb[b] ? mlen(b, s) : 0;
        bs.app_start[i] = cu[b] + (s - 1) * M;
        bs.app_len[i] = s >= 1 ? mlen(b, s - 1) : 0;
        rd.seq[i] = B == 1 ? 0 : b;
        rd.flags[i] = (s == 0 ? 1 : 0) | (r == 0 ? 2 : 0);
        rd.next_slot[i] = fuse ? next_slot[b] : -1;
        rd.ckpt_row[i] = ckoff[b] + s - 1;  // this sequence's W at step r + 1 (read only when next_slot >= 0)
      }
      if (!prep_ready && !launched([&] { return launch_bwd_prep(pa, na, S.mma_bf16, st); }))
        return TTT_EHIP;
      if (!launched([&] { return launch_bwd_step(bs, (int)(n_chains * G), S.h, S.io_bf16, S.mma_bf16, st); }))
        return TTT_EHIP;
      if (!launched([&] { return launch_bwd_reduce(rd, (int)(n_chains * nbpc), st); })) return TTT_EHIP;
    }
    prep_ready = fuse;
  }
  if (B > 1) {  // d(eta) over sequences, and the shared initial weights' gradient
    BwdSumArgs sm{};
    sm.src = shared_w0 ? fin : nullptr;
    sm.deta_src = deta_seq; sm.dW1 = dW1_0; sm.dW2 = dW2_0; sm.deta = deta;
    sm.B = B; sm.H = (int32_t)H; sm.h = S.h;
    if (!launched([&] { return launch_bwd_sum(sm, st); })) return TTT_EHIP;
  }
  return TTT_OK;
}

// GCS forward: gradient launches over all chunks at W0 (entries = chunks),
// one summing update into W*, one apply launch over all tokens.  A stream
// with more chunks x heads than shard-partial slots is summed in passes of
// as many chunks as the slots hold: each pass adds its chunks' sum onto a
// running total (fixed order: pass by pass, chunks in order within a pass),
// the last one takes the step.
ttt_status_t run_gcs_forward(const ttt_problem_t* p, const Shape& S, const void* Q, const void* K, const void* V,
                             const float* W1_0, const float* W2_0, void* O, float* W1_T, float* W2_T, float* loss,
                             void* ws, size_t ws_bytes, hipStream_t st, float* wstar_out) {
  const int64_t H = S.H;
  const WsLayout L = ws_layout(S, H);
  if (!ws || ws_bytes < L.total) return TTT_EWORKSPACE;
  const int64_t N = p->n_tokens, M = S.M, dh = S.dh();
  const int64_t C = (N + M - 1) / M;
  float* partial = at<float>(ws, L.partial);
  float* partial_loss = at<float>(ws, L.partial_loss);
  float* wstar = wstar_out ? wstar_out : at<float>(ws, L.pp);
  float* acc = at<float>(ws, L.fin);  // [H][2dh] running sum of a multi-pass stream
  const int nbpc = (int)((2 * dh / 4 + 255) / 256);
  const int64_t per_pass = std::min<int64_t>(C, L.slot_cap / H);  // >= 1: slot_cap >= H
  const int64_t n_chains = per_pass * H;
  const int64_t tiles = (std::min(M, N) + TT - 1) / TT;
  int64_t G = (default_target_wgs(S) + n_chains - 1) / n_chains;
  G = std::max<int64_t>(1, std::min<int64_t>({G, tiles, L.slot_cap / n_chains}));
  const bool passes = per_pass < C;
  for (int64_t c0 = 0; c0 < C; c0 += per_pass) {
    const int64_t cp = std::min<int64_t>(per_pass, C - c0);
    for (int64_t base = 0; base < cp; base += MAXS) {
      const int na = (int)std::min<int64_t>(MAXS, cp - base);
      FwdStepArgs a{};
      a.Q = Q; a.K = K; a.V = V; a.O = O;
      a.stride_tok = S.stride_tok; a.stride_head = S.stride_head;
      a.w1_src = W1_0; a.w2_src = W2_0; a.w_cstride = dh; a.w_mod = (int32_t)H;
      a.H = (int32_t)H; a.flags = p->flags; a.G = (int32_t)G;
      const int64_t slot0 = base * H * G;
      a.partial = partial + slot0 * 2 * dh;
      a.partial_loss = partial_loss + slot0;
      a.n_active = na;
      for (int i = 0; i < na; ++i) {
        const int64_t c = c0 + base + i;
        a.seq_id[i] = 0;
        a.grad_start[i] = c * M;
        a.grad_len[i] = (int32_t)std::min<int64_t>(M, N - c * M);
        a.app_start[i] = 0;
        a.app_len[i] = 0;
      }
      if (!launched([&] { return launch_fwd_step(a, (int)(na * H * G), S.h, S.io_bf16, S.mma_bf16, st); }))
        return TTT_EHIP;
    }
    const bool last = c0 + cp == C;
    UpdStepArgs u{};
    u.w1_src = W1_0; u.w2_src = W2_0; u.w_cstride = dh; u.w_mod = (int32_t)H;
    u.H = (int32_t)H; u.h = S.h; u.eta = p->eta; u.G = (int32_t)G;
    u.partial = partial; u.partial_loss = partial_loss; u.w_dst = wstar;
    u.wT1 = W1_T; u.wT2 = W2_T; u.loss = loss; u.loss_stride = (int32_t)C; u.chunk = 0;
    u.gcs_chunks = (int32_t)cp; u.gcs_M = (int32_t)M;
    u.gcs_last_len = (int32_t)(last ? N - (C - 1) * M : M);
    u.gcs_acc = passes ? acc : nullptr;
    u.gcs_entry0 = (int32_t)c0; u.gcs_first = c0 == 0; u.gcs_last = last;
    if (!launched([&] { return launch_update(u, (int)(H * nbpc), st); })) return TTT_EHIP;
  }
  if (O) {
    FwdStepArgs a{};
    a.Q = Q; a.K = K; a.V = V; a.O = O;
    a.stride_tok = S.stride_tok; a.stride_head = S.stride_head;
    a.w1_src = wstar; a.w2_src = wstar + dh; a.w_cstride = 2 * dh; a.w_mod = (int32_t)H;
    a.H = (int32_t)H; a.flags = p->flags;
    const int64_t atiles = (N + TT - 1) / TT;
    int64_t Ga = std::max<int64_t>(1, std::min<int64_t>((default_target_wgs(S) + H - 1) / H, atiles));
    a.G = (int32_t)Ga;
    a.partial = partial; a.partial_loss = partial_loss;
    a.n_active = 1; a.seq_id[0] = 0;
    a.grad_start[0] = 0; a.grad_len[0] = 0; a.app_start[0] = 0; a.app_len[0] = (int32_t)N;
    if (!launched([&] { return launch_fwd_step(a, (int)(H * Ga), S.h, S.io_bf16, S.mma_bf16, st); }))
      return TTT_EHIP;
  }
  return TTT_OK;
}

// GCS backward: W* recomputed; apply adjoint over all tokens at W* -> Wh;
// then per chunk the update adjoint at W0 against the fixed Wh, accumulated.
ttt_status_t run_gcs_backward(const ttt_problem_t* p, const Shape& S, const void* Q, const void* K, const void* V,
                              const float* W1_0, const float* W2_0, const void* dO, void* dQ, void* dK, void* dV,
                              float* dW1_0, float* dW2_0, float* deta, void* ws, size_t ws_bytes, hipStream_t st) {
  const int64_t H = S.H;
  const WsLayout L = ws_layout(S, H);
  if (!ws || ws_bytes < L.total) return TTT_EWORKSPACE;
  const int64_t N = p->n_tokens, M = S.M, dh = S.dh();
  const int64_t C = (N + M - 1) / M;
  float* partial = at<float>(ws, L.partial);
  float* pdeta = at<float>(ws, L.partial_loss);
  float* wstar = at<float>(ws, L.wlast);
  float* wh = at<float>(ws, L.adj);                      // adjoint of W* (fixed)
  float* acc[2] = {at<float>(ws, L.pp), at<float>(ws, L.pp) + H * 2 * dh};  // running dW0
  float* w0 = at<float>(ws, L.adj) + H * 2 * dh;         // W0 packed [W1 | W2] per head
  void* prep = at<char>(ws, L.prep);
  const int nbpc = (int)((2 * dh / 4 + 255) / 256);
  // single sequence: chain (0, head) of an adjoint buffer is at base + head * 2dh
  auto reduce_args = [&](const float* src, float* dst, bool final, int first, int64_t G) {
    BwdReduceArgs r{};
    r.wh_src_base = src; r.wh_dst_base = dst; r.dst1 = dW1_0; r.dst2 = dW2_0; r.deta_base = deta;
    r.partial = partial; r.partial_deta = pdeta; r.n_active = 1; r.G = (int32_t)G; r.H = (int32_t)H; r.h = S.h;
    r.seq[0] = 0; r.flags[0] = (final ? 1 : 0) | (first ? 2 : 0); r.next_slot[0] = -1;
    return r;
  };
  auto prep_args = [&](const float* w, const float* whs) {
    BwdPrepArgs a{};
    a.w_src[0] = w; a.wh_src[0] = whs; a.prep = prep; a.H = (int32_t)H; a.h = S.h;
    return a;
  };
  auto step_args = [&](int64_t G, int64_t gs, int32_t gl, int64_t as, int32_t al) {
    BwdStepArgs b{};
    b.Q = Q; b.K = K; b.V = V; b.dO = dO; b.dQ = dQ; b.dK = dK; b.dV = dV;
    b.stride_tok = S.stride_tok; b.stride_head = S.stride_head;
    b.prep = prep; b.H = (int32_t)H; b.flags = p->flags; b.eta = p->eta;
    b.G = (int32_t)G; b.partial = partial; b.partial_deta = pdeta; b.n_active = 1;
    b.grad_start[0] = gs; b.grad_len[0] = gl; b.app_start[0] = as; b.app_len[0] = al;
    return b;
  };
  if (C == 0) {  // no tokens: zero gradients
    const BwdReduceArgs r = reduce_args(nullptr, nullptr, true, 1, 0);
    return launched([&] { return launch_bwd_reduce(r, (int)(H * nbpc), st); }) ? TTT_OK : TTT_EHIP;
  }
  // W* (no outputs)
  ttt_status_t e = run_gcs_forward(p, S, Q, K, V, W1_0, W2_0, nullptr, nullptr, nullptr, nullptr, ws, ws_bytes, st,
                                   wstar);
  if (e != TTT_OK) return e;
  // W0 packed like a checkpoint: an update with zero partials copies it
  {
    UpdStepArgs u{};
    u.w1_src = W1_0; u.w2_src = W2_0; u.w_cstride = dh; u.w_mod = (int32_t)H;
    u.H = (int32_t)H; u.h = S.h; u.eta = 0.f; u.G = 0;
    u.partial = partial; u.partial_loss = pdeta; u.w_dst = w0;
    u.gcs_chunks = 1; u.gcs_M = 1; u.gcs_last_len = 1;
    if (!launched([&] { return launch_update(u, (int)(H * nbpc), st); })) return TTT_EHIP;
  }
  const int target = default_target_wgs(S);
  auto grid_g = [&](int64_t len) {
    const int64_t tiles = (len + TT - 1) / TT;
    return std::max<int64_t>(1, std::min<int64_t>({(target + H - 1) / H, std::max<int64_t>(tiles, 1),
                                                   L.slot_cap / H}));
  };
  // apply adjoint of all tokens at W*  ->  Wh (and dQ), deta starts at 0
  {
    const BwdPrepArgs pa = prep_args(wstar, nullptr);
    if (!launched([&] { return launch_bwd_prep(pa, 1, S.mma_bf16, st); })) return TTT_EHIP;
    const int64_t G = grid_g(N);
    const BwdStepArgs b = step_args(G, 0, 0, 0, (int32_t)N);
    if (!launched([&] { return launch_bwd_step(b, (int)(H * G), S.h, S.io_bf16, S.mma_bf16, st); }))
      return TTT_EHIP;
    const BwdReduceArgs r = reduce_args(nullptr, wh, false, 1, G);
    if (!launched([&] { return launch_bwd_reduce(r, (int)(H * nbpc), st); })) return TTT_EHIP;
  }
  // update adjoint of each chunk at W0 against Wh, accumulated on top of Wh
  {
    const BwdPrepArgs pa = prep_args(w0, wh);
    if (!launched([&] { return launch_bwd_prep(pa, 1, S.mma_bf16, st); })) return TTT_EHIP;
  }
  const float* prev = wh;
  for (int64_t c = 0; c < C; ++c) {
    const int32_t len = (int32_t)std::min<int64_t>(M, N - c * M);
    const int64_t G = grid_g(len);
    const BwdStepArgs b = step_args(G, c * M, len, 0, 0);
    if (!launched([&] { return launch_bwd_step(b, (int)(H * G), S.h, S.io_bf16, S.mma_bf16, st); }))
      return TTT_EHIP;
    const BwdReduceArgs r = reduce_args(prev, acc[c % 2], c == C - 1, 0, G);
    if (!launched([&] { return launch_bwd_reduce(r, (int)(H * nbpc), st); })) return TTT_EHIP;
    prev = acc[c % 2];
  }
  return TTT_OK;
}

// The forward at large state sizes: per sequence and head, the chunks in
// order, each one normalisation launch and seven GEMM launches (gradient,
// update, apply of the updated weights); the FP32 masters live in the
// workspace between chunks.
ttt_status_t run_forward_large(const ttt_problem_t* p, const Shape& S, int B, const int64_t* cu, const void* Q,
                               const void* K, const void* V, const float* W1_0, const float* W2_0, int w0_per_seq,
                               void* O, float* W1_T, float* W2_T, float* ckpt, float* loss, void* ws, size_t ws_bytes,
                               hipStream_t st) {
  const LargeLayout L = large_layout(S);
  if (!ws || ws_bytes < L.total) return TTT_EWORKSPACE;
  const int64_t dh = S.dh(), M = S.M;
  const size_t iob = S.io_bf16 ? 2 : 4;
  // the error word reads 0 after a call (nothing here can give up)
  if (cu[B] > 0 && !launched([&] { return launch_zero_words(at<uint32_t>(ws, L.sync) + SYNC_ERR, 1, st); }))
    return TTT_EHIP;
  float* W1 = at<float>(ws, L.W1);
  float* W2 = at<float>(ws, L.W2);
  int64_t ckrow = 0;
  for (int b = 0; b < B; ++b) {
    const int64_t n = cu[b + 1] - cu[b];
    const int64_t C = (n + M - 1) / M;
    for (int hd = 0; hd < S.H; ++hd) {
      const int64_t w0 = ((int64_t)(w0_per_seq ? b * S.H : 0) + hd) * dh;
      if (!launched([&] {
            return launch_large_init(W1_0 + w0, W2_0 + w0, W1, W2, at<char>(ws, L.W1op), at<char>(ws, L.W2op), dh,
                                     S.mma_bf16, st);
          }))
        return TTT_EHIP;
      for (int64_t c = 0; c < C; ++c) {
        const int64_t t0 = cu[b] + c * M;
        const int32_t rows = (int32_t)std::min<int64_t>(M, n - c * M);
        if (ckpt) {
          float* row = ckpt + ((ckrow + c) * S.H + hd) * 2 * dh;
          if (hipMemcpyAsync(row, W1, dh * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess ||
              hipMemcpyAsync(row + dh, W2, dh * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess)
            return TTT_EHIP;
        }
        const int64_t off = (t0 * S.stride_tok + (int64_t)hd * S.stride_head) * (int64_t)iob;
        LargeStepArgs a{};
        a.K = static_cast<const char*>(K) + off;
        a.V = static_cast<const char*>(V) + off;
        a.Q = static_cast<const char*>(Q) + off;
        a.O = static_cast<char*>(O) + off;
        a.stride_tok = S.stride_tok;
        a.flags = p->flags;
        a.rows = rows; a.d = S.d; a.h = S.h;
        a.grad = 1; a.eta = p->eta;
        a.Kn = at<char>(ws, L.Kn); a.Qn = at<char>(ws, L.Qn); a.E = at<char>(ws, L.E);
        a.A = at<char>(ws, L.A); a.D = at<char>(ws, L.D); a.Aq = at<char>(ws, L.Aq);
        a.Vn = at<float>(ws, L.Vn); a.S1 = at<char>(ws, L.S1);
        a.W1 = W1; a.W2 = W2; a.W1op = at<char>(ws, L.W1op); a.W2op = at<char>(ws, L.W2op);
        a.loss_part = at<float>(ws, L.loss_part);
        a.loss = loss ? loss + (int64_t)hd * C + c : nullptr;
        if (!launched([&] { return launch_large_step(a, S.io_bf16, S.mma_bf16, st); })) return TTT_EHIP;
      }
      if (W1_T) {
        const int64_t o = ((int64_t)b * S.H + hd) * dh;
        if (hipMemcpyAsync(W1_T + o, C > 0 ? W1 : W1_0 + w0, dh * sizeof(float), hipMemcpyDeviceToDevice, st) !=
                hipSuccess ||
            hipMemcpyAsync(W2_T + o, C > 0 ? W2 : W2_0 + w0, dh * sizeof(float), hipMemcpyDeviceToDevice, st) !=
                hipSuccess)
          return TTT_EHIP;
      }
    }
    ckrow += C;
  }
  return TTT_OK;
}

// GCS at large state sizes (Eq. 10), per head: every chunk's gradient at W0
// (its own 1/M_c, its loss at W0) stepped into the FP32 masters in chunk
// order while the operand copies keep W0, then the operand copies of W*, then
// every chunk's apply.
ttt_status_t run_gcs_forward_large(const ttt_problem_t* p, const Shape& S, const void* Q, const void* K,
                                   const void* V, const float* W1_0, const float* W2_0, void* O, float* W1_T,
                                   float* W2_T, float* loss, void* ws, size_t ws_bytes, hipStream_t st) {
  const LargeLayout L = large_layout(S);
  if (!ws || ws_bytes < L.total) return TTT_EWORKSPACE;
  const int64_t N = p->n_tokens, M = S.M, dh = S.dh();
  const int64_t C = (N + M - 1) / M;
  const size_t iob = S.io_bf16 ? 2 : 4;
  if (!launched([&] { return launch_zero_words(at<uint32_t>(ws, L.sync) + SYNC_ERR, 1, st); })) return TTT_EHIP;
  float* W1 = at<float>(ws, L.W1);
  float* W2 = at<float>(ws, L.W2);
  for (int hd = 0; hd < S.H; ++hd) {
    const int64_t w0 = (int64_t)hd * dh;
    if (!launched([&] {
          return launch_large_init(W1_0 + w0, W2_0 + w0, W1, W2, at<char>(ws, L.W1op), at<char>(ws, L.W2op), dh,
                                   S.mma_bf16, st);
        }))
      return TTT_EHIP;
    auto step = [&](int64_t c, bool grad) {
      const int64_t t0 = c * M;
      const int64_t off = (t0 * S.stride_tok + (int64_t)hd * S.stride_head) * (int64_t)iob;
      LargeStepArgs a{};
      a.K = static_cast<const char*>(K) + off;
      a.V = static_cast<const char*>(V) + off;
      a.Q = static_cast<const char*>(Q) + off;
      a.O = grad ? nullptr : static_cast<char*>(O) + off;
      a.stride_tok = S.stride_tok;
      a.flags = p->flags;
      a.rows = (int32_t)std::min<int64_t>(M, N - t0); a.d = S.d; a.h = S.h;
      a.grad = grad ? 1 : 0; a.masters_only = 1; a.eta = p->eta;
      a.Kn = at<char>(ws, L.Kn); a.Qn = at<char>(ws, L.Qn); a.E = at<char>(ws, L.E);
      a.A = at<char>(ws, L.A); a.D = at<char>(ws, L.D); a.Aq = at<char>(ws, L.Aq);
      a.Vn = at<float>(ws, L.Vn); a.S1 = at<char>(ws, L.S1);
      a.W1 = W1; a.W2 = W2; a.W1op = at<char>(ws, L.W1op); a.W2op = at<char>(ws, L.W2op);
      a.loss_part = at<float>(ws, L.loss_part);
      a.loss = grad && loss ? loss + (int64_t)hd * C + c : nullptr;
      return launched([&] { return launch_large_step(a, S.io_bf16, S.mma_bf16, st); });
    };
    for (int64_t c = 0; c < C; ++c)
      if (!step(c, true)) return TTT_EHIP;
    if (!launched([&] { return launch_large_cast(W1, at<char>(ws, L.W1op), dh, S.mma_bf16, st); }) ||
        !launched([&] { return launch_large_cast(W2, at<char>(ws, L.W2op), dh, S.mma_bf16, st); }))
      return TTT_EHIP;
    for (int64_t c = 0; c < C; ++c)
      if (!step(c, false)) return TTT_EHIP;
    if (W1_T && (hipMemcpyAsync(W1_T + w0, W1, dh * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess ||
                 hipMemcpyAsync(W2_T + w0, W2, dh * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess))
      return TTT_EHIP;
  }
  return TTT_OK;
}

// Arguments of a large-state reverse step over the chunk at byte offset off
// of the token tensors, its buffers in the workspace (W_c in the forward
// layout's operand copies, W_{c+1} in W1nop / W2nop, the carried adjoint in
// Wh1 / Wh2); the caller sets the parts to run, where the weight terms go and
// the step-size output.
LargeBwdArgs large_bwd_args(const ttt_problem_t* p, const Shape& S, const LargeBwdLayout& L, void* ws, int64_t off,
                            int32_t rows, const void* Q, const void* K, const void* V, const void* dO, void* dQ,
                            void* dK, void* dV) {
  LargeBwdArgs b{};
  b.K = static_cast<const char*>(K) + off;
  b.V = static_cast<const char*>(V) + off;
  b.Q = static_cast<const char*>(Q) + off;
  b.dO = static_cast<const char*>(dO) + off;
  b.dQ = static_cast<char*>(dQ) + off;
  b.dK = static_cast<char*>(dK) + off;
  b.dV = static_cast<char*>(dV) + off;
  b.stride_tok = S.stride_tok;
  b.flags = p->flags;
  b.rows = rows; b.d = S.d; b.h = S.h;
  b.eta = p->eta;
  b.Kn = at<char>(ws, L.f.Kn); b.Qn = at<char>(ws, L.f.Qn); b.E = at<char>(ws, L.f.E);
  b.dOn = at<char>(ws, L.dOn); b.dY = at<char>(ws, L.dY);
  b.Vn = at<float>(ws, L.f.Vn); b.dq = at<float>(ws, L.dq); b.dk = at<float>(ws, L.dk);
  b.dv = at<float>(ws, L.dv); b.dE = at<float>(ws, L.dE);
  b.A = at<char>(ws, L.f.A); b.S1 = at<char>(ws, L.f.S1); b.S2 = at<char>(ws, L.S2); b.P = at<char>(ws, L.P);
  b.D = at<char>(ws, L.f.D); b.Aq = at<char>(ws, L.f.Aq); b.Sq1 = at<char>(ws, L.Sq1);
  b.dZq = at<char>(ws, L.dZq); b.dP = at<char>(ws, L.dP); b.dZa = at<char>(ws, L.dZa);
  b.EWh = at<char>(ws, L.EWh); b.dZ = at<char>(ws, L.dZ);
  b.W1op = at<char>(ws, L.f.W1op); b.W2op = at<char>(ws, L.f.W2op);
  b.W1nop = at<char>(ws, L.W1nop); b.W2nop = at<char>(ws, L.W2nop);
  b.Wh1 = at<float>(ws, L.Wh1); b.Wh2 = at<float>(ws, L.Wh2);
  b.Wh1op = at<char>(ws, L.Wh1op); b.Wh2op = at<char>(ws, L.Wh2op);
  b.deta_part = at<float>(ws, L.deta_part);
  return b;
}

// Reverse mode at large state sizes for one sequence (tokens t0 .. t0+N-1,
// its checkpoints from ckpt on), per head: the weights after the last chunk
// recomputed from its checkpoint with one forward step, then for c = C-1 .. 0
// the reverse step of chunk c with W_c (checkpoint c) and W_{c+1} (checkpoint
// c+1, or the recomputed weights), carrying the adjoint of the weights from
// chunk to chunk; at the end it is the adjoint of W_0, written to dW1_0 /
// dW2_0 (added to them with add_w0) and added to deta (or written, without
// add_eta).
ttt_status_t backward_large_seq(const ttt_problem_t* p, const Shape& S, const LargeBwdLayout& L, int64_t t0,
                                int64_t N, const float* ckpt, const void* Q, const void* K, const void* V,
                                const void* dO, void* dQ, void* dK, void* dV, float* dW1_0, float* dW2_0, float* deta,
                                bool add_w0, bool add_eta, void* ws, hipStream_t st) {
  const int64_t M = S.M, dh = S.dh();
  const int64_t C = (N + M - 1) / M;
  const size_t iob = S.io_bf16 ? 2 : 4;
  float* Wh1 = at<float>(ws, L.Wh1);
  float* Wh2 = at<float>(ws, L.Wh2);
  float* dt = at<float>(ws, L.deta);
  auto cast = [&](const float* src, size_t off) {
    return launched([&] { return launch_large_cast(src, at<char>(ws, off), dh, S.mma_bf16, st); });
  };
  auto zero = [&](float* q, int64_t n) { return launched([&] { return launch_large_zero(q, n, st); }); };
  for (int hd = 0; hd < S.H; ++hd) {
    if (!zero(Wh1, dh) || !zero(Wh2, dh) || !zero(dt, 1) || !cast(Wh1, L.Wh1op) || !cast(Wh2, L.Wh2op))
      return TTT_EHIP;
    auto row = [&](int64_t c) { return ckpt + (c * S.H + hd) * 2 * dh; };
    auto chunk_off = [&](int64_t c) {
      return ((t0 + c * M) * S.stride_tok + (int64_t)hd * S.stride_head) * (int64_t)iob;
    };
    if (C > 0) {
      // W_C: one forward step of the last chunk from its checkpoint
      const int64_t c = C - 1;
      float* W1 = at<float>(ws, L.f.W1);
      float* W2 = at<float>(ws, L.f.W2);
      if (!launched([&] {
            return launch_large_init(row(c), row(c) + dh, W1, W2, at<char>(ws, L.f.W1op), at<char>(ws, L.f.W2op), dh,
                                     S.mma_bf16, st);
          }))
        return TTT_EHIP;
      LargeStepArgs a{};
      a.K = static_cast<const char*>(K) + chunk_off(c);
      a.V = static_cast<const char*>(V) + chunk_off(c);
      a.Q = static_cast<const char*>(Q) + chunk_off(c);
      a.O = nullptr;
      a.stride_tok = S.stride_tok;
      a.flags = p->flags;
      a.rows = (int32_t)(N - c * M); a.d = S.d; a.h = S.h;
      a.grad = 1; a.eta = p->eta;
      a.Kn = at<char>(ws, L.f.Kn); a.Qn = at<char>(ws, L.f.Qn); a.E = at<char>(ws, L.f.E);
      a.A = at<char>(ws, L.f.A); a.D = at<char>(ws, L.f.D); a.Aq = at<char>(ws, L.f.Aq);
      a.Vn = at<float>(ws, L.f.Vn); a.S1 = at<char>(ws, L.f.S1);
      a.W1 = W1; a.W2 = W2; a.W1op = at<char>(ws, L.f.W1op); a.W2op = at<char>(ws, L.f.W2op);
      a.loss_part = at<float>(ws, L.f.loss_part);
      if (!launched([&] { return launch_large_step(a, S.io_bf16, S.mma_bf16, st); })) return TTT_EHIP;
      if (!cast(W1, L.W1nop) || !cast(W2, L.W2nop)) return TTT_EHIP;
    }
    for (int64_t c = C - 1; c >= 0; --c) {
      if (c + 1 < C && (!cast(row(c + 1), L.W1nop) || !cast(row(c + 1) + dh, L.W2nop))) return TTT_EHIP;
      if (!cast(row(c), L.f.W1op) || !cast(row(c) + dh, L.f.W2op)) return TTT_EHIP;
      LargeBwdArgs b = large_bwd_args(p, S, L, ws, chunk_off(c), (int32_t)std::min<int64_t>(M, N - c * M), Q, K, V,
                                      dO, dQ, dK, dV);
      b.Acc1 = Wh1; b.Acc2 = Wh2; b.Acc1op = b.Wh1op; b.Acc2op = b.Wh2op;
      b.apply = 1; b.update = 1;
      b.deta = dt;
      if (!launched([&] { return launch_large_bwd_step(b, S.io_bf16, S.mma_bf16, st); })) return TTT_EHIP;
    }
    if (add_w0) {
      if (!launched([&] { return launch_large_add(Wh1, dW1_0 + hd * dh, dh, st); }) ||
          !launched([&] { return launch_large_add(Wh2, dW2_0 + hd * dh, dh, st); }))
        return TTT_EHIP;
    } else if (hipMemcpyAsync(dW1_0 + hd * dh, Wh1, dh * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess ||
               hipMemcpyAsync(dW2_0 + hd * dh, Wh2, dh * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess) {
      return TTT_EHIP;
    }
    if (add_eta) {
      if (!launched([&] { return launch_large_add(dt, deta + hd, 1, st); })) return TTT_EHIP;
    } else if (hipMemcpyAsync(deta + hd, dt, sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess) {
      return TTT_EHIP;
    }
  }
  return TTT_OK;
}

// Reverse mode at large state sizes over B sequences (B = 1: the chain call),
// one sequence after another.  Shared W0 (w0_per_seq = 0): its adjoint is the
// sum over sequences in sequence order; deta always is.
ttt_status_t run_backward_large(const ttt_problem_t* p, const Shape& S, int B, const int64_t* cu, int w0_per_seq,
                                const float* ckpt, const void* Q, const void* K, const void* V, const void* dO,
                                void* dQ, void* dK, void* dV, float* dW1_0, float* dW2_0, float* deta, void* ws,
                                size_t ws_bytes, hipStream_t st) {
  const LargeBwdLayout L = large_bwd_layout(S);
  if (!ws || ws_bytes < L.total) return TTT_EWORKSPACE;
  if (!launched([&] { return launch_zero_words(at<uint32_t>(ws, L.f.sync) + SYNC_ERR, 1, st); })) return TTT_EHIP;
  const int64_t dh = S.dh();
  int64_t ckrow = 0;
  for (int b = 0; b < B; ++b) {
    const int64_t n = cu[b + 1] - cu[b];
    const int64_t o = w0_per_seq ? (int64_t)b * S.H * dh : 0;
    const ttt_status_t e =
        backward_large_seq(p, S, L, cu[b], n, ckpt ? ckpt + ckrow * S.H * 2 * dh : nullptr, Q, K, V, dO, dQ, dK, dV,
                           dW1_0 + o, dW2_0 + o, deta, !w0_per_seq && b > 0, b > 0, ws, st);
    if (e != TTT_OK) return e;
    ckrow += (n + S.M - 1) / S.M;
  }
  return TTT_OK;
}

// Reverse mode of the GCS form at large state sizes (Eq. 10), per head: W*
// recomputed as in the forward; the apply adjoint of every chunk at W*
// accumulated into Wh (dQ written); then every chunk's update adjoint at W0
// against that fixed Wh, its weight terms added to a total that starts at Wh
// (dK, dV and d/d eta written); the total is the adjoint of W0.
ttt_status_t run_gcs_backward_large(const ttt_problem_t* p, const Shape& S, const void* Q, const void* K,
                                    const void* V, const float* W1_0, const float* W2_0, const void* dO, void* dQ,
                                    void* dK, void* dV, float* dW1_0, float* dW2_0, float* deta, void* ws,
                                    size_t ws_bytes, hipStream_t st) {
  const LargeBwdLayout L = large_bwd_layout(S);
  if (!ws || ws_bytes < L.total) return TTT_EWORKSPACE;
  const int64_t N = p->n_tokens, M = S.M, dh = S.dh();
  const int64_t C = (N + M - 1) / M;
  const size_t iob = S.io_bf16 ? 2 : 4;
  if (!launched([&] { return launch_zero_words(at<uint32_t>(ws, L.f.sync) + SYNC_ERR, 1, st); })) return TTT_EHIP;
  float* W1 = at<float>(ws, L.f.W1);
  float* W2 = at<float>(ws, L.f.W2);
  float* Wh1 = at<float>(ws, L.Wh1);
  float* Wh2 = at<float>(ws, L.Wh2);
  float* tot1 = at<float>(ws, L.tot1);
  float* tot2 = at<float>(ws, L.tot2);
  float* dt = at<float>(ws, L.deta);
  auto cast = [&](const float* src, size_t off) {
    return launched([&] { return launch_large_cast(src, at<char>(ws, off), dh, S.mma_bf16, st); });
  };
  auto zero = [&](float* q, int64_t n) { return launched([&] { return launch_large_zero(q, n, st); }); };
  auto copy = [&](float* dst, const float* src, int64_t n) {
    return hipMemcpyAsync(dst, src, n * sizeof(float), hipMemcpyDeviceToDevice, st) == hipSuccess;
  };
  for (int hd = 0; hd < S.H; ++hd) {
    const int64_t w0 = (int64_t)hd * dh;
    auto chunk_off = [&](int64_t c) {
      return (c * M * S.stride_tok + (int64_t)hd * S.stride_head) * (int64_t)iob;
    };
    auto rows = [&](int64_t c) { return (int32_t)std::min<int64_t>(M, N - c * M); };
    if (!zero(Wh1, dh) || !zero(Wh2, dh) || !zero(dt, 1) || !cast(Wh1, L.Wh1op) || !cast(Wh2, L.Wh2op))
      return TTT_EHIP;
    // W* = W0 - eta * sum_c grad L_c(W0), as the forward takes it
    if (!launched([&] {
          return launch_large_init(W1_0 + w0, W2_0 + w0, W1, W2, at<char>(ws, L.f.W1op), at<char>(ws, L.f.W2op), dh,
                                   S.mma_bf16, st);
        }))
      return TTT_EHIP;
    for (int64_t c = 0; c < C; ++c) {
      LargeStepArgs a{};
      a.K = static_cast<const char*>(K) + chunk_off(c);
      a.V = static_cast<const char*>(V) + chunk_off(c);
      a.Q = static_cast<const char*>(Q) + chunk_off(c);
      a.stride_tok = S.stride_tok;
      a.flags = p->flags;
      a.rows = rows(c); a.d = S.d; a.h = S.h;
      a.grad = 1; a.masters_only = 1; a.eta = p->eta;
      a.Kn = at<char>(ws, L.f.Kn); a.Qn = at<char>(ws, L.f.Qn); a.E = at<char>(ws, L.f.E);
      a.A = at<char>(ws, L.f.A); a.D = at<char>(ws, L.f.D); a.Aq = at<char>(ws, L.f.Aq);
      a.Vn = at<float>(ws, L.f.Vn); a.S1 = at<char>(ws, L.f.S1);
      a.W1 = W1; a.W2 = W2; a.W1op = at<char>(ws, L.f.W1op); a.W2op = at<char>(ws, L.f.W2op);
      a.loss_part = at<float>(ws, L.f.loss_part);
      if (!launched([&] { return launch_large_step(a, S.io_bf16, S.mma_bf16, st); })) return TTT_EHIP;
    }
    if (!cast(W1, L.W1nop) || !cast(W2, L.W2nop)) return TTT_EHIP;
    // the apply adjoint of every chunk at W*
    for (int64_t c = 0; c < C; ++c) {
      LargeBwdArgs b = large_bwd_args(p, S, L, ws, chunk_off(c), rows(c), Q, K, V, dO, dQ, dK, dV);
      b.apply = 1; b.update = 0;
      b.deta = dt;
      if (!launched([&] { return launch_large_bwd_step(b, S.io_bf16, S.mma_bf16, st); })) return TTT_EHIP;
    }
    // every chunk's update adjoint at W0 against the fixed Wh
    if (!copy(tot1, Wh1, dh) || !copy(tot2, Wh2, dh) || !cast(W1_0 + w0, L.f.W1op) || !cast(W2_0 + w0, L.f.W2op))
      return TTT_EHIP;
    for (int64_t c = 0; c < C; ++c) {
      LargeBwdArgs b = large_bwd_args(p, S, L, ws, chunk_off(c), rows(c), Q, K, V, dO, dQ, dK, dV);
      b.apply = 0; b.update = 1;
      b.Acc1 = tot1; b.Acc2 = tot2;  // operand copies not needed
      b.deta = dt;
      if (!launched([&] { return launch_large_bwd_step(b, S.io_bf16, S.mma_bf16, st); })) return TTT_EHIP;
    }
    if (!copy(dW1_0 + w0, C > 0 ? tot1 : Wh1, dh) || !copy(dW2_0 + w0, C > 0 ? tot2 : Wh2, dh) ||
        !copy(deta + hd, dt, 1))
      return TTT_EHIP;
  }
  return TTT_OK;
}

ttt_status_t check_batch(const ttt_problem_t* p, int32_t n_seqs, const int64_t* cu, int32_t w0_per_seq,
                         const ttt_tile_cfg_t* tile_cfg) {
  if (n_seqs < 1 || !cu) return TTT_EINVAL;
  if (w0_per_seq != 0 && w0_per_seq != 1) return TTT_EINVAL;
  if (cu[0] != 0) return TTT_EINVAL;
  for (int b = 0; b < n_seqs; ++b)
    if (cu[b + 1] < cu[b]) return TTT_EINVAL;
  if (tile_cfg && (tile_cfg->wg_per_chain < 0 || tile_cfg->target_wgs < 0 || tile_cfg->spin_limit < 0))
    return TTT_EINVAL;
  (void)p;
  return TTT_OK;
}

ttt_status_t batched_fwd_impl(const ttt_problem_t* p, int32_t n_seqs, const int64_t* cu_seqlens_host, const void* Q,
                              const void* K, const void* V, const float* W1_0, const float* W2_0, int32_t w0_per_seq,
                              void* O, float* W1_T, float* W2_T, float* ckpt, const ttt_tile_cfg_t* tile_cfg,
                              void* ws, size_t ws_bytes, void* hip_stream) {
  Shape S{};
  ttt_status_t e = check_problem(p, &S);
  if (e != TTT_OK) return e;
  if ((e = check_batch(p, n_seqs, cu_seqlens_host, w0_per_seq, tile_cfg)) != TTT_OK) return e;
  if (!W1_0 || !W2_0) return TTT_EINVAL;
  const bool any = cu_seqlens_host[n_seqs] > 0;
  // token tensors and checkpoints may be empty (null) when there are no tokens
  if (any && (!Q || !K || !V || !O)) return TTT_EINVAL;
  if ((W1_T == nullptr) != (W2_T == nullptr)) return TTT_EINVAL;
  if (any && ((p->flags & TTT_SAVE_CKPT) != 0) != (ckpt != nullptr)) return TTT_EINVAL;
  if (p->flags & TTT_EMIT_LOSS) return TTT_ENOTSUP;
  if (tile_cfg && tile_cfg->schedule != TTT_SCHED_PERSISTENT && tile_cfg->schedule != TTT_SCHED_STEPWISE)
    return TTT_EINVAL;
  for (const void* q : {Q, K, V, (const void*)W1_0, (const void*)W2_0, (const void*)O, (const void*)W1_T,
                        (const void*)W2_T, (const void*)ckpt})
    if (q && !aligned16(q)) return TTT_EINVAL;
  const hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (S.large)
    return run_forward_large(p, S, n_seqs, cu_seqlens_host, Q, K, V, W1_0, W2_0, w0_per_seq, O, W1_T, W2_T, ckpt,
                             nullptr, ws, ws_bytes, st);
  const ttt_tile_cfg_t cfg = resolve_cfg(tile_cfg, S, (int64_t)n_seqs * S.H, false);
  if (cfg.schedule == TTT_SCHED_STEPWISE) {
    // sequences without tokens take no chunk step: their final weights are W_0
    const ttt_status_t e0 = copy_w0_to_final(S, n_seqs, cu_seqlens_host, W1_0, W2_0, w0_per_seq, W1_T, W2_T, ws,
                                             ws_bytes, st);
    if (e0 != TTT_OK || !any) return e0;
    return run_forward(p, S, n_seqs, cu_seqlens_host, Q, K, V, W1_0, W2_0, w0_per_seq, O, W1_T, W2_T, ckpt, nullptr,
                       &cfg, ws, ws_bytes, st);
  }
  return run_forward_persist(p, S, n_seqs, cu_seqlens_host, Q, K, V, W1_0, W2_0, w0_per_seq, O, W1_T, W2_T, ckpt,
                             nullptr, &cfg, ws, ws_bytes, st);
}
// ---------------------------------------------------------------- paper AMU
struct AmuWs {
  size_t partial, pp, prep, total;
  int64_t slot_cap;
};

AmuWs amu_ws_layout(const Shape& s) {
  AmuWs L{};
  L.slot_cap = std::max<int64_t>(s.H, SLOT_CAP_MIN);
  const size_t wbytes = (size_t)3 * s.dh() * sizeof(float);
  size_t off = 0;
  L.partial = off;
  off = align_up(off + (size_t)L.slot_cap * wbytes);
  L.pp = off;  // ping-pong packed weights per head
  off = align_up(off + 2 * (size_t)s.H * wbytes);
  L.prep = off;  // 4 operand matrices per head (float-sized slots)
  off = align_up(off + (size_t)s.H * 4 * s.dh() * sizeof(float));
  L.total = off;
  return L;
}

// Chain: for s = 0..C one operand-preparation launch (W_s), one step launch
// (gradient of chunk s, apply of chunk s-1) and, while chunk s exists, one
// update launch.  GCS: the gradients of all chunks at W0 are one
// shard-parallel gradient over every token (the dot-product loss has no
// per-chunk normalisation, so the sum over chunks is the sum over tokens),
// one update, then one apply over every token.
ttt_status_t run_amu(const ttt_problem_t* p, const Shape& S, int sync, const void* Q, const void* K, const void* V,
                     const float* eta_tok, const float* W1_0, const float* W2_0, const float* W3_0, void* O,
                     float* W1_T, float* W2_T, float* W3_T, void* ws, size_t ws_bytes, hipStream_t st) {
  const AmuWs L = amu_ws_layout(S);
  if (!ws || ws_bytes < L.total) return TTT_EWORKSPACE;
  const int64_t H = S.H, N = p->n_tokens, M = S.M, dh = S.dh();
  const int64_t C = (N + M - 1) / M;
  float* partial = at<float>(ws, L.partial);
  float* pp[2] = {at<float>(ws, L.pp), at<float>(ws, L.pp) + H * 3 * dh};
  void* prep = at<char>(ws, L.prep);
  const int target = default_target_wgs(S);
  auto grid_g = [&](int64_t len) {
    const int64_t tiles = std::max<int64_t>((len + TT - 1) / TT, 1);
    return std::max<int64_t>(1, std::min<int64_t>({(target + H - 1) / H, tiles, L.slot_cap / H}));
  };
  const AmuWeights w0{W1_0, W2_0, W3_0, dh};
  auto packed = [&](const float* b) { return AmuWeights{b, b + dh, b + 2 * dh, 3 * dh}; };
  auto do_prep = [&](const AmuWeights& w) {
    AmuPrepArgs a{};
    a.src = w; a.prep = prep; a.n_mats = 4; a.H = (int32_t)H; a.h = S.h;
    return launched([&] { return launch_amu_prep(a, S.mma_bf16, st); });
  };
  auto do_step = [&](int64_t G, int64_t gs, int64_t gl, int64_t as, int64_t al) {
    AmuStepArgs a{};
    a.Q = Q; a.K = K; a.V = V; a.O = O; a.eta_tok = eta_tok;
    a.stride_tok = S.stride_tok; a.stride_head = S.stride_head;
    a.H = (int32_t)H; a.flags = p->flags; a.G = (int32_t)G; a.prep = prep; a.n_prep = 4; a.partial = partial;
    a.grad_start = gs; a.grad_len = (int32_t)gl; a.app_start = as; a.app_len = (int32_t)al;
    return launched([&] { return launch_amu_step(a, (int)(H * G), S.h, S.io_bf16, S.mma_bf16, st); });
  };
  auto do_update = [&](const AmuWeights& src, int64_t G, float* dst, bool last) {
    AmuUpdArgs u{};
    u.src = src; u.partial = partial; u.G = (int32_t)G; u.H = (int32_t)H; u.h = S.h; u.w_dst = dst;
    u.wT1 = last ? W1_T : nullptr; u.wT2 = last ? W2_T : nullptr; u.wT3 = last ? W3_T : nullptr;
    return launched([&] { return launch_amu_update(u, st); });
  };
  if (C == 0) {  // no tokens: W_T = W_0
    if (W1_T && !do_update(w0, 0, pp[0], true)) return TTT_EHIP;
    return TTT_OK;
  }
  auto mlen = [&](int64_t c) { return std::min<int64_t>(M, N - c * M); };
  if (sync == TTT_SYNC_CHAIN) {
    AmuWeights cur = w0;
    for (int64_t s = 0; s <= C; ++s) {
      const int64_t gl = s < C ? mlen(s) : 0, al = s >= 1 ? mlen(s - 1) : 0;
      const int64_t G = grid_g(std::max(gl, al));
      if (!do_prep(cur)) return TTT_EHIP;
      if (!do_step(G, s * M, gl, (s - 1) * M, al)) return TTT_EHIP;
      if (s < C) {
        if (!do_update(cur, G, pp[s % 2], s == C - 1)) return TTT_EHIP;
        cur = packed(pp[s % 2]);
      }
    }
    return TTT_OK;
  }
  const int64_t G = grid_g(N);
  if (!do_prep(w0)) return TTT_EHIP;
  if (!do_step(G, 0, N, 0, 0)) return TTT_EHIP;
  if (!do_update(w0, G, pp[0], true)) return TTT_EHIP;
  if (!do_prep(packed(pp[0]))) return TTT_EHIP;
  if (!do_step(G, 0, 0, 0, N)) return TTT_EHIP;
  return TTT_OK;
}


// The memory unit at large state sizes, per head: the FP32 masters and their
// operand copies from W0, then chain: per chunk in order, its gradient, the
// update (masters and operand copies) and the apply of its queries; GCS:
// every chunk's gradient at W0 subtracted from the masters in chunk order
// (the operand copies keep W0), the operand copies of W*, then every
// chunk's apply.
ttt_status_t run_amu_large(const ttt_problem_t* p, const Shape& S, int sync, const void* Q, const void* K,
                           const void* V, const float* eta_tok, const float* W1_0, const float* W2_0,
                           const float* W3_0, void* O, float* W1_T, float* W2_T, float* W3_T, void* ws,
                           size_t ws_bytes, hipStream_t st) {
  const LargeAmuLayout L = large_amu_layout(S);
  if (!ws || ws_bytes < L.total) return TTT_EWORKSPACE;
  const int64_t N = p->n_tokens, M = S.M, dh = S.dh(), H = S.H;
  const int64_t C = (N + M - 1) / M;
  const size_t iob = S.io_bf16 ? 2 : 4;
  if (N > 0 && !launched([&] { return launch_zero_words(at<uint32_t>(ws, L.sync) + SYNC_ERR, 1, st); }))
    return TTT_EHIP;
  float* Wm[3] = {at<float>(ws, L.W1), at<float>(ws, L.W2), at<float>(ws, L.W3)};
  void* Wo[3] = {at<char>(ws, L.W1op), at<char>(ws, L.W2op), at<char>(ws, L.W3op)};
  const float* W0[3] = {W1_0, W2_0, W3_0};
  float* WT[3] = {W1_T, W2_T, W3_T};
  auto copy = [&](float* dst, const float* src) {
    return hipMemcpyAsync(dst, src, dh * sizeof(float), hipMemcpyDeviceToDevice, st) == hipSuccess;
  };
  auto cast_all = [&]() {
    for (int m = 0; m < 3; ++m)
      if (!launched([&] { return launch_large_cast(Wm[m], Wo[m], dh, S.mma_bf16, st); })) return false;
    return true;
  };
  for (int64_t hd = 0; hd < H; ++hd) {
    if (C > 0) {
      for (int m = 0; m < 3; ++m)
        if (!copy(Wm[m], W0[m] + hd * dh)) return TTT_EHIP;
      if (!cast_all()) return TTT_EHIP;
      auto step = [&](int64_t c, bool grad, bool write_op, bool apply) {
        const int64_t t0 = c * M;
        const int64_t off = (t0 * S.stride_tok + hd * S.stride_head) * (int64_t)iob;
        LargeAmuArgs a{};
        a.K = static_cast<const char*>(K) + off;
        a.V = static_cast<const char*>(V) + off;
        a.Q = static_cast<const char*>(Q) + off;
        a.O = apply ? static_cast<char*>(O) + off : nullptr;
        a.stride_tok = S.stride_tok;
        a.eta = eta_tok + t0 * H + hd;
        a.eta_stride = H;
        a.flags = p->flags;
        a.rows = (int32_t)std::min<int64_t>(M, N - t0); a.d = S.d; a.h = S.h;
        a.grad = grad ? 1 : 0; a.write_op = write_op ? 1 : 0;
        a.Kn = at<char>(ws, L.Kn); a.Qn = at<char>(ws, L.Qn); a.E = at<char>(ws, L.E); a.Vn = at<float>(ws, L.Vn);
        a.Z3 = at<char>(ws, L.Z3); a.Hd = at<char>(ws, L.Hd); a.G1 = at<char>(ws, L.G1); a.G3 = at<char>(ws, L.G3);
        a.D1 = at<char>(ws, L.D1); a.D3 = at<char>(ws, L.D3);
        a.W1 = Wm[0]; a.W2 = Wm[1]; a.W3 = Wm[2];
        a.W1op = Wo[0]; a.W2op = Wo[1]; a.W3op = Wo[2];
        return launched([&] { return launch_large_amu_step(a, S.io_bf16, S.mma_bf16, st); });
      };
      if (sync == TTT_SYNC_CHAIN) {
        for (int64_t c = 0; c < C; ++c)
          if (!step(c, true, true, true)) return TTT_EHIP;
      } else {
        for (int64_t c = 0; c < C; ++c)
          if (!step(c, true, false, false)) return TTT_EHIP;
        if (!cast_all()) return TTT_EHIP;
        for (int64_t c = 0; c < C; ++c)
          if (!step(c, false, false, true)) return TTT_EHIP;
      }
    }
    if (W1_T)
      for (int m = 0; m < 3; ++m)
        if (!copy(WT[m] + hd * dh, C > 0 ? Wm[m] : W0[m] + hd * dh)) return TTT_EHIP;
  }
  return TTT_OK;
}

// The paper's unit in reverse at large state sizes, per head.  Chain: the
// weights before every chunk recomputed with forward steps (W_0 .. W_C), then
// for c = C-1 .. 0 the apply adjoint of chunk c at W_{c+1} and its update
// adjoint at W_c, carrying the adjoint of the weights.  GCS: W* recomputed,
// the apply adjoint of every chunk at W*, then every chunk's update adjoint
// at W0 against that fixed adjoint, the weight terms added to a total that
// starts at it.
ttt_status_t run_amu_bwd_large(const ttt_problem_t* p, const Shape& S, int sync, const void* Q, const void* K,
                               const void* V, const float* eta_tok, const float* W1_0, const float* W2_0,
                               const float* W3_0, const void* dO, void* dQ, void* dK, void* dV, float* deta_tok,
                               float* dW1_0, float* dW2_0, float* dW3_0, void* ws, size_t ws_bytes, hipStream_t st) {
  const int64_t N = p->n_tokens, M = S.M, dh = S.dh(), H = S.H;
  const LargeAmuBwdLayout L = large_amu_bwd_layout(S, N, sync);
  if (!ws || ws_bytes < L.total) return TTT_EWORKSPACE;
  const int64_t C = (N + M - 1) / M;
  const size_t iob = S.io_bf16 ? 2 : 4;
  if (!launched([&] { return launch_zero_words(at<uint32_t>(ws, L.f.sync) + SYNC_ERR, 1, st); })) return TTT_EHIP;
  float* Wm[3] = {at<float>(ws, L.f.W1), at<float>(ws, L.f.W2), at<float>(ws, L.f.W3)};
  const size_t Wo[3] = {L.f.W1op, L.f.W2op, L.f.W3op};
  const float* W0[3] = {W1_0, W2_0, W3_0};
  float* dW0[3] = {dW1_0, dW2_0, dW3_0};
  float* wl = at<float>(ws, L.wlist);
  auto cast = [&](const float* src, size_t off) {
    return launched([&] { return launch_large_cast(src, at<char>(ws, off), dh, S.mma_bf16, st); });
  };
  auto copy = [&](float* dst, const float* src) {
    return hipMemcpyAsync(dst, src, dh * sizeof(float), hipMemcpyDeviceToDevice, st) == hipSuccess;
  };
  for (int64_t hd = 0; hd < H; ++hd) {
    auto chunk_off = [&](int64_t c) { return (c * M * S.stride_tok + hd * S.stride_head) * (int64_t)iob; };
    auto rows = [&](int64_t c) { return (int32_t)std::min<int64_t>(M, N - c * M); };
    // a forward step of chunk c (the gradient and the update, no apply)
    auto fwd_step = [&](int64_t c, bool write_op) {
      LargeAmuArgs a{};
      a.K = static_cast<const char*>(K) + chunk_off(c);
      a.V = static_cast<const char*>(V) + chunk_off(c);
      a.Q = static_cast<const char*>(Q) + chunk_off(c);
      a.O = nullptr;
      a.stride_tok = S.stride_tok;
      a.eta = eta_tok + c * M * H + hd;
      a.eta_stride = H;
      a.flags = p->flags;
      a.rows = rows(c); a.d = S.d; a.h = S.h;
      a.grad = 1; a.write_op = write_op ? 1 : 0;
      a.Kn = at<char>(ws, L.f.Kn); a.Qn = at<char>(ws, L.f.Qn); a.E = at<char>(ws, L.f.E); a.Vn = at<float>(ws, L.f.Vn);
      a.Z3 = at<char>(ws, L.f.Z3); a.Hd = at<char>(ws, L.f.Hd); a.G1 = at<char>(ws, L.f.G1); a.G3 = at<char>(ws, L.f.G3);
      a.D1 = at<char>(ws, L.f.D1); a.D3 = at<char>(ws, L.f.D3);
      a.W1 = Wm[0]; a.W2 = Wm[1]; a.W3 = Wm[2];
      a.W1op = at<char>(ws, Wo[0]); a.W2op = at<char>(ws, Wo[1]); a.W3op = at<char>(ws, Wo[2]);
      return launched([&] { return launch_large_amu_step(a, S.io_bf16, S.mma_bf16, st); });
    };
    // the reverse step of chunk c with W (operand copies in Wo) and W' (in Wnop)
    auto bwd_step = [&](int64_t c, bool apply, bool update, float* const* acc, bool acc_op) {
      const int64_t off = chunk_off(c);
      LargeAmuBwdArgs b{};
      b.K = static_cast<const char*>(K) + off;
      b.V = static_cast<const char*>(V) + off;
      b.Q = static_cast<const char*>(Q) + off;
      b.dO = static_cast<const char*>(dO) + off;
      b.dQ = static_cast<char*>(dQ) + off;
      b.dK = static_cast<char*>(dK) + off;
      b.dV = static_cast<char*>(dV) + off;
      b.stride_tok = S.stride_tok;
      b.eta = eta_tok + c * M * H + hd;
      b.deta = deta_tok + c * M * H + hd;
      b.eta_stride = H;
      b.flags = p->flags;
      b.rows = rows(c); b.d = S.d; b.h = S.h;
      b.apply = apply ? 1 : 0; b.update = update ? 1 : 0;
      b.Kn = at<char>(ws, L.f.Kn); b.Qn = at<char>(ws, L.f.Qn); b.E = at<char>(ws, L.f.E);
      b.dOn = at<char>(ws, L.dOn);
      b.Vn = at<float>(ws, L.f.Vn); b.Ydot = at<float>(ws, L.Ydot);
      b.dq = at<float>(ws, L.dq); b.dk = at<float>(ws, L.dk); b.dv = at<float>(ws, L.dv);
      b.Z3 = at<char>(ws, L.f.Z3); b.Hd = at<char>(ws, L.f.Hd);
      b.S = at<char>(ws, L.S); b.S1 = at<char>(ws, L.S1); b.S2 = at<char>(ws, L.S2); b.Zd3 = at<char>(ws, L.Zd3);
      b.Sd = at<char>(ws, L.Sd); b.Hdot = at<char>(ws, L.Hdot); b.T2 = at<char>(ws, L.T2); b.dHh = at<char>(ws, L.dHh);
      b.aZ1 = at<char>(ws, L.aZ1); b.aZ3 = at<char>(ws, L.aZ3); b.aZd1 = at<char>(ws, L.aZd1);
      b.aZd3 = at<char>(ws, L.aZd3);
      for (int m = 0; m < 3; ++m) {
        b.Wop[m] = at<char>(ws, Wo[m]);
        b.Wnop[m] = at<char>(ws, L.Wnop[m]);
        b.Wh[m] = at<float>(ws, L.Wh[m]);
        b.Whop[m] = at<char>(ws, L.Whop[m]);
        b.Acc[m] = acc[m];
        b.Accop[m] = acc_op ? at<char>(ws, L.Whop[m]) : nullptr;
      }
      return launched([&] { return launch_large_amu_bwd_step(b, S.io_bf16, S.mma_bf16, st); });
    };
    float* Wh[3] = {at<float>(ws, L.Wh[0]), at<float>(ws, L.Wh[1]), at<float>(ws, L.Wh[2])};
    float* tot[3] = {at<float>(ws, L.tot[0]), at<float>(ws, L.tot[1]), at<float>(ws, L.tot[2])};
    for (int m = 0; m < 3; ++m)
      if (!launched([&] { return launch_large_zero(Wh[m], dh, st); }) || !cast(Wh[m], L.Whop[m])) return TTT_EHIP;
    for (int m = 0; m < 3; ++m)
      if (!copy(Wm[m], W0[m] + hd * dh) || !cast(Wm[m], Wo[m])) return TTT_EHIP;
    float* const* result = Wh;
    if (sync == TTT_SYNC_CHAIN) {
      auto wl_at = [&](int64_t c, int m) { return wl + (c * 3 + m) * dh; };
      for (int m = 0; m < 3; ++m)
        if (!copy(wl_at(0, m), Wm[m])) return TTT_EHIP;
      for (int64_t c = 0; c < C; ++c) {
        if (!fwd_step(c, true)) return TTT_EHIP;
        for (int m = 0; m < 3; ++m)
          if (!copy(wl_at(c + 1, m), Wm[m])) return TTT_EHIP;
      }
      for (int64_t c = C - 1; c >= 0; --c) {
        for (int m = 0; m < 3; ++m)
          if (!cast(wl_at(c + 1, m), L.Wnop[m]) || !cast(wl_at(c, m), Wo[m])) return TTT_EHIP;
        if (!bwd_step(c, true, true, Wh, true)) return TTT_EHIP;
      }
    } else {
      for (int64_t c = 0; c < C; ++c)
        if (!fwd_step(c, false)) return TTT_EHIP;
      for (int m = 0; m < 3; ++m)
        if (!cast(Wm[m], L.Wnop[m])) return TTT_EHIP;
      for (int64_t c = 0; c < C; ++c)
        if (!bwd_step(c, true, false, tot, false)) return TTT_EHIP;
      for (int m = 0; m < 3; ++m)
        if (!copy(tot[m], Wh[m]) || !cast(W0[m] + hd * dh, Wo[m])) return TTT_EHIP;
      for (int64_t c = 0; c < C; ++c)
        if (!bwd_step(c, false, true, tot, false)) return TTT_EHIP;
      if (C > 0) result = tot;
    }
    for (int m = 0; m < 3; ++m)
      if (!copy(dW0[m] + hd * dh, result[m])) return TTT_EHIP;
  }
  return TTT_OK;
}

// Reverse mode of the paper's memory unit.  Workspace: shard partials, the
// carried adjoint Wh [H][3dh], the weights the backward needs ([C+1][H][3dh]
// for the chain: every W_c, recomputed; [1][H][3dh] for GCS: W*), and three
// sets of six operand copies per head (weights at the update, weights at the
// apply, Wh).
struct AmuBwdWs {
  size_t partial, wh, wlist, prep_u, prep_a, prep_h, total;
  int64_t slot_cap;
};

AmuBwdWs amu_bwd_ws_layout(const Shape& s, int64_t n_tokens, int sync) {
  AmuBwdWs L{};
  L.slot_cap = std::max<int64_t>(s.H, SLOT_CAP_MIN);
  const size_t wbytes = (size_t)3 * s.dh() * sizeof(float);
  const int64_t C = (n_tokens + s.M - 1) / s.M;
  const int64_t n_w = sync == TTT_SYNC_CHAIN ? C + 1 : 1;
  const size_t pbytes = (size_t)s.H * 6 * s.dh() * sizeof(float);
  size_t off = 0;
  L.partial = off;
  off = align_up(off + (size_t)L.slot_cap * wbytes);
  L.wh = off;
  off = align_up(off + (size_t)s.H * wbytes);
  L.wlist = off;
  off = align_up(off + (size_t)n_w * s.H * wbytes);
  L.prep_u = off;
  off = align_up(off + pbytes);
  L.prep_a = off;
  off = align_up(off + pbytes);
  L.prep_h = off;
  off = align_up(off + pbytes);
  L.total = off;
  return L;
}

// chain: recompute W_1..W_C (one gradient launch and one update per chunk),
// then for c = C-1..0: Wh += apply adjoint of chunk c at W_{c+1}; Wh += update
// adjoint of chunk c at W_c along Wh.  gcs: W* = W0 - (gradient over all
// tokens); Wh = apply adjoint over all tokens at W*; dW0 = Wh + update
// adjoint over all tokens at W0 along Wh (the chunks' update adjoints at W0
// with the same Wh sum to one pass over the tokens: no per-chunk
// normalisation in this loss).
ttt_status_t run_amu_bwd(const ttt_problem_t* p, const Shape& S, int sync, const void* Q, const void* K,
                         const void* V, const float* eta_tok, const float* W1_0, const float* W2_0,
                         const float* W3_0, const void* dO, void* dQ, void* dK, void* dV, float* deta_tok,
                         float* dW1_0, float* dW2_0, float* dW3_0, void* ws, size_t ws_bytes, hipStream_t st) {
  const int64_t H = S.H, N = p->n_tokens, M = S.M, dh = S.dh();
  const AmuBwdWs L = amu_bwd_ws_layout(S, N, sync);
  if (!ws || ws_bytes < L.total) return TTT_EWORKSPACE;
  const int64_t C = (N + M - 1) / M;
  float* partial = at<float>(ws, L.partial);
  float* wh = at<float>(ws, L.wh);
  float* wlist = at<float>(ws, L.wlist);
  void* prep_u = at<char>(ws, L.prep_u);
  void* prep_a = at<char>(ws, L.prep_a);
  void* prep_h = at<char>(ws, L.prep_h);
  const int target = default_target_wgs(S);
  auto grid_g = [&](int64_t len) {
    const int64_t tiles = std::max<int64_t>((len + TT - 1) / TT, 1);
    return std::max<int64_t>(1, std::min<int64_t>({(target + H - 1) / H, tiles, L.slot_cap / H}));
  };
  const AmuWeights w0{W1_0, W2_0, W3_0, dh};
  auto packed = [&](const float* b) { return AmuWeights{b, b + dh, b + 2 * dh, 3 * dh}; };
  auto do_prep = [&](const AmuWeights& w, void* dst) {
    AmuPrepArgs a{};
    a.src = w; a.prep = dst; a.n_mats = 6; a.H = (int32_t)H; a.h = S.h;
    return launched([&] { return launch_amu_prep(a, S.mma_bf16, st); });
  };
  auto do_grad = [&](int64_t start, int64_t len) {  // gradient partials at the weights in prep_u
    AmuStepArgs a{};
    a.Q = Q; a.K = K; a.V = V; a.O = nullptr; a.eta_tok = eta_tok;
    a.stride_tok = S.stride_tok; a.stride_head = S.stride_head;
    const int64_t G = grid_g(len);
    a.H = (int32_t)H; a.flags = p->flags; a.G = (int32_t)G; a.prep = prep_u; a.n_prep = 6; a.partial = partial;
    a.grad_start = start; a.grad_len = (int32_t)len; a.app_start = 0; a.app_len = 0;
    if (!launched([&] { return launch_amu_step(a, (int)(H * G), S.h, S.io_bf16, S.mma_bf16, st); }))
      return int64_t(-1);
    return G;
  };
  auto do_update = [&](const AmuWeights& src, int64_t G, float* dst) {
    AmuUpdArgs u{};
    u.src = src; u.partial = partial; u.G = (int32_t)G; u.H = (int32_t)H; u.h = S.h; u.w_dst = dst;
    return launched([&] { return launch_amu_update(u, st); });
  };
  auto bwd_args = [&](int64_t start, int64_t len, int64_t G) {
    AmuBwdArgs a{};
    a.stride_tok = S.stride_tok; a.stride_head = S.stride_head;
    a.H = (int32_t)H; a.flags = p->flags; a.G = (int32_t)G; a.partial = partial;
    a.start = start; a.len = (int32_t)len;
    return a;
  };
  auto do_apply_adj = [&](int64_t start, int64_t len) {  // at the weights in prep_a
    const int64_t G = grid_g(len);
    AmuBwdArgs a = bwd_args(start, len, G);
    a.X = Q; a.Y = dO; a.dX = dQ; a.prep_w = prep_a;
    if (!launched([&] { return launch_amu_bwd_apply(a, (int)(H * G), S.h, S.io_bf16, S.mma_bf16, st); }))
      return int64_t(-1);
    return G;
  };
  auto do_update_adj = [&](int64_t start, int64_t len) {  // at prep_u along prep_h
    const int64_t G = grid_g(len);
    AmuBwdArgs a = bwd_args(start, len, G);
    a.X = K; a.Y = V; a.dX = dK; a.dY = dV; a.eta_tok = eta_tok; a.deta_tok = deta_tok;
    a.prep_w = prep_u; a.prep_a = prep_h;
    if (!launched([&] { return launch_amu_bwd_update(a, (int)(H * G), S.h, S.io_bf16, S.mma_bf16, st); }))
      return int64_t(-1);
    return G;
  };
  auto do_psum = [&](int64_t G, const float* base, float* dst, bool final) {
    AmuPsumArgs a{};
    a.partial = partial; a.G = (int32_t)G; a.H = (int32_t)H; a.h = S.h; a.base = base; a.dst = dst;
    if (final) { a.out1 = dW1_0; a.out2 = dW2_0; a.out3 = dW3_0; }
    return launched([&] { return launch_amu_psum(a, st); });
  };

  if (C == 0) {  // no tokens: O is empty, every adjoint is zero
    return do_psum(0, nullptr, wh, true) ? TTT_OK : TTT_EHIP;
  }
  if (sync == TTT_SYNC_GCS) {
    float* wstar = wlist;
    if (!do_prep(w0, prep_u)) return TTT_EHIP;
    const int64_t Gg = do_grad(0, N);
    if (Gg < 0 || !do_update(w0, Gg, wstar)) return TTT_EHIP;
    if (!do_prep(packed(wstar), prep_a)) return TTT_EHIP;
    const int64_t Ga = do_apply_adj(0, N);
    if (Ga < 0 || !do_psum(Ga, nullptr, wh, false)) return TTT_EHIP;
    if (!do_prep(packed(wh), prep_h)) return TTT_EHIP;
    const int64_t Gu = do_update_adj(0, N);
    if (Gu < 0 || !do_psum(Gu, wh, wh, true)) return TTT_EHIP;
    return TTT_OK;
  }
  // chain: W_c at wlist + c * H * 3dh (c >= 1); W_0 is the caller's
  auto wc = [&](int64_t c) { return c == 0 ? w0 : packed(wlist + c * H * 3 * dh); };
  auto mlen = [&](int64_t c) { return std::min<int64_t>(M, N - c * M); };
  for (int64_t c = 0; c < C; ++c) {
    if (!do_prep(wc(c), prep_u)) return TTT_EHIP;
    const int64_t G = do_grad(c * M, mlen(c));
    if (G < 0 || !do_update(wc(c), G, wlist + (c + 1) * H * 3 * dh)) return TTT_EHIP;
  }
  for (int64_t c = C - 1; c >= 0; --c) {
    if (!do_prep(wc(c + 1), prep_a)) return TTT_EHIP;
    const int64_t Ga = do_apply_adj(c * M, mlen(c));
    if (Ga < 0 || !do_psum(Ga, c == C - 1 ? nullptr : wh, wh, false)) return TTT_EHIP;
    if (!do_prep(wc(c), prep_u) || !do_prep(packed(wh), prep_h)) return TTT_EHIP;
    const int64_t Gu = do_update_adj(c * M, mlen(c));
    if (Gu < 0 || !do_psum(Gu, wh, wh, c == 0)) return TTT_EHIP;
  }
  return TTT_OK;
}

}  // namespace

namespace ttt {
// ttt_chunk_fwd, on a caller workspace (fixed_scratch null) or on a fixed
// scratch of ws_bytes whose device address fixed_scratch() returns after the
// arguments are validated (forward-only compact layout, stepwise schedule,
// work-groups per chain limited by the slots that fit).
ttt_status_t chunk_fwd_impl(const ttt_problem_t* p, const void* Q, const void* K, const void* V, const float* W1_0,
                            const float* W2_0, void* O, float* W1_T, float* W2_T, float* ckpt, float* loss, void* ws,
                            size_t ws_bytes, void* (*fixed_scratch)(), hipStream_t st) {
  Shape S{};
  const ttt_status_t e = check_problem(p, &S);
  if (e != TTT_OK) return e;
  if (!W1_0 || !W2_0) return TTT_EINVAL;
  // token tensors may be empty (null) when there are no tokens
  if (p->n_tokens > 0 && (!Q || !K || !V || !O)) return TTT_EINVAL;
  if ((W1_T == nullptr) != (W2_T == nullptr)) return TTT_EINVAL;
  if (p->n_tokens > 0 && ((p->flags & TTT_SAVE_CKPT) != 0) != (ckpt != nullptr)) return TTT_EINVAL;
  if (p->n_tokens > 0 && ((p->flags & TTT_EMIT_LOSS) != 0) != (loss != nullptr)) return TTT_EINVAL;
  for (const void* q : {Q, K, V, (const void*)W1_0, (const void*)W2_0, (const void*)O, (const void*)W1_T,
                        (const void*)W2_T, (const void*)ckpt})
    if (q && !aligned16(q)) return TTT_EINVAL;
  const int64_t cu[2] = {0, p->n_tokens};
  if (S.large) {
    if (fixed_scratch) return TTT_ENOTSUP;  // the fixed scratch holds the small-state layout only
    return run_forward_large(p, S, 1, cu, Q, K, V, W1_0, W2_0, 0, O, W1_T, W2_T, ckpt, loss, ws, ws_bytes, st);
  }
  ttt_tile_cfg_t cfg = resolve_cfg(nullptr, S, S.H, false);
  WsLayout fixed{};
  const WsLayout* layout = nullptr;
  if (fixed_scratch) {
    fixed = fwd_layout_in(S, S.H, ws_bytes);
    if (fixed.slot_cap < S.H) return TTT_EWORKSPACE;  // more chains than the scratch holds
    layout = &fixed;
    cfg.schedule = TTT_SCHED_STEPWISE;
    ws = fixed_scratch();  // after validation: the only HIP calls before enqueueing
    if (!ws) return TTT_EHIP;
  }
  if (cfg.schedule == TTT_SCHED_STEPWISE) {
    const ttt_status_t e0 = copy_w0_to_final(S, 1, cu, W1_0, W2_0, 0, W1_T, W2_T, ws, ws_bytes, st, layout);
    if (e0 != TTT_OK || p->n_tokens == 0) return e0;
    return run_forward(p, S, 1, cu, Q, K, V, W1_0, W2_0, 0, O, W1_T, W2_T, ckpt, loss, &cfg, ws, ws_bytes, st,
                       layout);
  }
  return run_forward_persist(p, S, 1, cu, Q, K, V, W1_0, W2_0, 0, O, W1_T, W2_T, ckpt, loss, &cfg, ws, ws_bytes, st);
}
}  // namespace ttt

extern "C" {

size_t ttt_workspace_bytes(const ttt_problem_t* p, int32_t n_seqs) {
  Shape S{};
  if (check_problem(p, &S) != TTT_OK || n_seqs < 1) return 0;
  if (S.large) return large_bwd_layout(S).total;  // the reverse mode's layout contains the forward's
  return ws_layout(S, (int64_t)n_seqs * S.H).total;
}

ttt_status_t ttt_chunk_fwd(const ttt_problem_t* p, const void* Q, const void* K, const void* V, const float* W1_0,
                           const float* W2_0, void* O, float* W1_T, float* W2_T, float* ckpt, float* loss, void* ws,
                           size_t ws_bytes, void* hip_stream) {
  try {
    return ttt::chunk_fwd_impl(p, Q, K, V, W1_0, W2_0, O, W1_T, W2_T, ckpt, loss, ws, ws_bytes, nullptr,
                               static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return TTT_EINVAL;
  }
}

ttt_status_t ttt_batched_fwd(const ttt_problem_t* p, int32_t n_seqs, const int64_t* cu_seqlens_host, const void* Q,
                             const void* K, const void* V, const float* W1_0, const float* W2_0, int32_t w0_per_seq,
                             void* O, float* W1_T, float* W2_T, const ttt_tile_cfg_t* tile_cfg, void* ws,
                             size_t ws_bytes, void* hip_stream) {
  try {
    if (p && (p->flags & TTT_SAVE_CKPT)) return TTT_EINVAL;  // checkpoints: ttt_batched_fwd_ckpt
    return batched_fwd_impl(p, n_seqs, cu_seqlens_host, Q, K, V, W1_0, W2_0, w0_per_seq, O, W1_T, W2_T, nullptr,
                            tile_cfg, ws, ws_bytes, hip_stream);
  } catch (...) {
    return TTT_EINVAL;
  }
}

ttt_status_t ttt_batched_fwd_ckpt(const ttt_problem_t* p, int32_t n_seqs, const int64_t* cu_seqlens_host,
                                  const void* Q, const void* K, const void* V, const float* W1_0, const float* W2_0,
                                  int32_t w0_per_seq, void* O, float* W1_T, float* W2_T, float* ckpt,
                                  const ttt_tile_cfg_t* tile_cfg, void* ws, size_t ws_bytes, void* hip_stream) {
  try {
    return batched_fwd_impl(p, n_seqs, cu_seqlens_host, Q, K, V, W1_0, W2_0, w0_per_seq, O, W1_T, W2_T, ckpt,
                            tile_cfg, ws, ws_bytes, hip_stream);
  } catch (...) {
    return TTT_EINVAL;
  }
}

ttt_status_t ttt_batched_bwd(const ttt_problem_t* p, int32_t n_seqs, const int64_t* cu_seqlens_host, const void* Q,
                             const void* K, const void* V, const float* W1_0, const float* W2_0, int32_t w0_per_seq,
                             const float* ckpt, const void* dO, void* dQ, void* dK, void* dV, float* dW1_0,
                             float* dW2_0, float* deta, const ttt_tile_cfg_t* tile_cfg, void* ws, size_t ws_bytes,
                             void* hip_stream) {
  try {
    Shape S{};
    ttt_status_t e = check_problem(p, &S);
    if (e != TTT_OK) return e;
    if ((e = check_batch(p, n_seqs, cu_seqlens_host, w0_per_seq, tile_cfg)) != TTT_OK) return e;
    if (!dW1_0 || !dW2_0 || !deta) return TTT_EINVAL;
    const bool any = cu_seqlens_host[n_seqs] > 0;
    if (any && (!Q || !K || !V || !ckpt || !dO || !dQ || !dK || !dV)) return TTT_EINVAL;
    (void)W1_0; (void)W2_0;  // each sequence's chunk-0 checkpoint holds its W_0
    for (const void* q : {Q, K, V, dO, (const void*)dQ, (const void*)dK, (const void*)dV, (const void*)ckpt,
                          (const void*)dW1_0, (const void*)dW2_0})
      if (q && !aligned16(q)) return TTT_EINVAL;
    if (S.large)
      return run_backward_large(p, S, n_seqs, cu_seqlens_host, w0_per_seq, ckpt, Q, K, V, dO, dQ, dK, dV, dW1_0,
                                dW2_0, deta, ws, ws_bytes, static_cast<hipStream_t>(hip_stream));
    return run_backward(p, S, n_seqs, cu_seqlens_host, w0_per_seq, ckpt, Q, K, V, dO, dQ, dK, dV, dW1_0, dW2_0,
                        deta, tile_cfg, ws, ws_bytes, static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return TTT_EINVAL;
  }
}

ttt_status_t ttt_chunk_bwd(const ttt_problem_t* p, const void* Q, const void* K, const void* V, const float* W1_0,
                           const float* W2_0, const float* ckpt, const void* dO, void* dQ, void* dK, void* dV,
                           float* dW1_0, float* dW2_0, float* deta, void* ws, size_t ws_bytes, void* hip_stream) {
  try {
    Shape S{};
    const ttt_status_t e = check_problem(p, &S);
    if (e != TTT_OK) return e;
    if (!dW1_0 || !dW2_0 || !deta) return TTT_EINVAL;
    if (p->n_tokens > 0 && (!Q || !K || !V || !ckpt || !dO || !dQ || !dK || !dV)) return TTT_EINVAL;
    (void)W1_0; (void)W2_0;  // the checkpoint of chunk 0 holds W_0
    for (const void* q : {Q, K, V, dO, (const void*)dQ, (const void*)dK, (const void*)dV, (const void*)ckpt,
                          (const void*)dW1_0, (const void*)dW2_0})
      if (q && !aligned16(q)) return TTT_EINVAL;
    const int64_t cu[2] = {0, p->n_tokens};
    if (S.large)
      return run_backward_large(p, S, 1, cu, 0, ckpt, Q, K, V, dO, dQ, dK, dV, dW1_0, dW2_0, deta, ws, ws_bytes,
                                static_cast<hipStream_t>(hip_stream));
    return run_backward(p, S, 1, cu, 0, ckpt, Q, K, V, dO, dQ, dK, dV, dW1_0, dW2_0, deta, nullptr, ws, ws_bytes,
                        static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return TTT_EINVAL;
  }
}

ttt_status_t ttt_gcs_fwd(const ttt_problem_t* p, const void* Q, const void* K, const void* V, const float* W1_0,
                         const float* W2_0, void* O, float* W1_T, float* W2_T, float* loss, void* ws, size_t ws_bytes,
                         void* hip_stream) {
  try {
    Shape S{};
    const ttt_status_t e = check_problem(p, &S);
    if (e != TTT_OK) return e;
    if (!W1_0 || !W2_0) return TTT_EINVAL;
    if (p->n_tokens > 0 && (!Q || !K || !V || !O)) return TTT_EINVAL;
    if ((W1_T == nullptr) != (W2_T == nullptr)) return TTT_EINVAL;
    if (p->flags & TTT_SAVE_CKPT) return TTT_EINVAL;
    if (p->n_tokens > 0 && ((p->flags & TTT_EMIT_LOSS) != 0) != (loss != nullptr)) return TTT_EINVAL;
    for (const void* q : {Q, K, V, (const void*)W1_0, (const void*)W2_0, (const void*)O, (const void*)W1_T,
                          (const void*)W2_T})
      if (q && !aligned16(q)) return TTT_EINVAL;
    if (p->n_tokens == 0) {  // no chunks: W* = W0
      if (!W1_T) return TTT_OK;
      const hipStream_t st = static_cast<hipStream_t>(hip_stream);
      const size_t bytes = (size_t)S.H * S.dh() * sizeof(float);
      if (hipMemcpyAsync(W1_T, W1_0, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
          hipMemcpyAsync(W2_T, W2_0, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return TTT_EHIP;
      return TTT_OK;
    }
    if (S.large)
      return run_gcs_forward_large(p, S, Q, K, V, W1_0, W2_0, O, W1_T, W2_T, loss, ws, ws_bytes,
                                   static_cast<hipStream_t>(hip_stream));
    return run_gcs_forward(p, S, Q, K, V, W1_0, W2_0, O, W1_T, W2_T, loss, ws, ws_bytes,
                           static_cast<hipStream_t>(hip_stream), nullptr);
  } catch (...) {
    return TTT_EINVAL;
  }
}

ttt_status_t ttt_gcs_bwd(const ttt_problem_t* p, const void* Q, const void* K, const void* V, const float* W1_0,
                         const float* W2_0, const void* dO, void* dQ, void* dK, void* dV, float* dW1_0, float* dW2_0,
                         float* deta, void* ws, size_t ws_bytes, void* hip_stream) {
  try {
    Shape S{};
    const ttt_status_t e = check_problem(p, &S);
    if (e != TTT_OK) return e;
    if (!W1_0 || !W2_0 || !dW1_0 || !dW2_0 || !deta) return TTT_EINVAL;
    if (p->n_tokens > 0 && (!Q || !K || !V || !dO || !dQ || !dK || !dV)) return TTT_EINVAL;
    if (p->flags & (TTT_SAVE_CKPT | TTT_EMIT_LOSS)) return TTT_EINVAL;
    for (const void* q : {Q, K, V, dO, (const void*)dQ, (const void*)dK, (const void*)dV, (const void*)W1_0,
                          (const void*)W2_0, (const void*)dW1_0, (const void*)dW2_0})
      if (q && !aligned16(q)) return TTT_EINVAL;
    if (S.large)
      return run_gcs_backward_large(p, S, Q, K, V, W1_0, W2_0, dO, dQ, dK, dV, dW1_0, dW2_0, deta, ws, ws_bytes,
                                    static_cast<hipStream_t>(hip_stream));
    return run_gcs_backward(p, S, Q, K, V, W1_0, W2_0, dO, dQ, dK, dV, dW1_0, dW2_0, deta, ws, ws_bytes,
                            static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return TTT_EINVAL;
  }
}

size_t ttt_amu_workspace_bytes(const ttt_problem_t* p) {
  Shape S{};
  if (check_problem(p, &S) != TTT_OK) return 0;
  if (S.large) return large_amu_layout(S).total;
  return amu_ws_layout(S).total;
}

ttt_status_t ttt_amu_fwd(const ttt_problem_t* p, int32_t sync, const void* Q, const void* K, const void* V,
                         const float* eta_tok, const float* W1_0, const float* W2_0, const float* W3_0, void* O,
                         float* W1_T, float* W2_T, float* W3_T, void* ws, size_t ws_bytes, void* hip_stream) {
  try {
    Shape S{};
    const ttt_status_t e = check_problem(p, &S);
    if (e != TTT_OK) return e;
    if (sync != TTT_SYNC_CHAIN && sync != TTT_SYNC_GCS) return TTT_EINVAL;
    if (p->flags & (TTT_SAVE_CKPT | TTT_EMIT_LOSS)) return TTT_ENOTSUP;
    if (!W1_0 || !W2_0 || !W3_0) return TTT_EINVAL;
    if ((W1_T == nullptr) != (W2_T == nullptr) || (W1_T == nullptr) != (W3_T == nullptr)) return TTT_EINVAL;
    if (p->n_tokens > 0 && (!Q || !K || !V || !eta_tok || !O)) return TTT_EINVAL;
    for (const void* q : {Q, K, V, (const void*)W1_0, (const void*)W2_0, (const void*)W3_0, (const void*)O,
                          (const void*)W1_T, (const void*)W2_T, (const void*)W3_T})
      if (q && !aligned16(q)) return TTT_EINVAL;
    if (p->n_tokens == 0 && !W1_T) return TTT_OK;
    if (S.large)
      return run_amu_large(p, S, sync, Q, K, V, eta_tok, W1_0, W2_0, W3_0, O, W1_T, W2_T, W3_T, ws, ws_bytes,
                           static_cast<hipStream_t>(hip_stream));
    return run_amu(p, S, sync, Q, K, V, eta_tok, W1_0, W2_0, W3_0, O, W1_T, W2_T, W3_T, ws, ws_bytes,
                   static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return TTT_EINVAL;
  }
}

size_t ttt_amu_bwd_workspace_bytes(const ttt_problem_t* p, int32_t sync) {
  Shape S{};
  if (check_problem(p, &S) != TTT_OK || (sync != TTT_SYNC_CHAIN && sync != TTT_SYNC_GCS)) return 0;
  if (S.large) return large_amu_bwd_layout(S, p->n_tokens, sync).total;
  return amu_bwd_ws_layout(S, p->n_tokens, sync).total;
}

ttt_status_t ttt_amu_bwd(const ttt_problem_t* p, int32_t sync, const void* Q, const void* K, const void* V,
                         const float* eta_tok, const float* W1_0, const float* W2_0, const float* W3_0,
                         const void* dO, void* dQ, void* dK, void* dV, float* deta_tok, float* dW1_0, float* dW2_0,
                         float* dW3_0, void* ws, size_t ws_bytes, void* hip_stream) {
  try {
    Shape S{};
    const ttt_status_t e = check_problem(p, &S);
    if (e != TTT_OK) return e;
    if (sync != TTT_SYNC_CHAIN && sync != TTT_SYNC_GCS) return TTT_EINVAL;
    if (p->flags & (TTT_SAVE_CKPT | TTT_EMIT_LOSS)) return TTT_ENOTSUP;
    if (!W1_0 || !W2_0 || !W3_0 || !dW1_0 || !dW2_0 || !dW3_0) return TTT_EINVAL;
    if (p->n_tokens > 0 && (!Q || !K || !V || !eta_tok || !dO || !dQ || !dK || !dV || !deta_tok))
      return TTT_EINVAL;
    for (const void* q : {Q, K, V, dO, (const void*)dQ, (const void*)dK, (const void*)dV, (const void*)W1_0,
                          (const void*)W2_0, (const void*)W3_0, (const void*)dW1_0, (const void*)dW2_0,
                          (const void*)dW3_0})
      if (q && !aligned16(q)) return TTT_EINVAL;
    if (S.large)
      return run_amu_bwd_large(p, S, sync, Q, K, V, eta_tok, W1_0, W2_0, W3_0, dO, dQ, dK, dV, deta_tok, dW1_0,
                               dW2_0, dW3_0, ws, ws_bytes, static_cast<hipStream_t>(hip_stream));
    return run_amu_bwd(p, S, sync, Q, K, V, eta_tok, W1_0, W2_0, W3_0, dO, dQ, dK, dV, deta_tok, dW1_0, dW2_0,
                       dW3_0, ws, ws_bytes, static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return TTT_EINVAL;
  }
}

// The layer around the memory unit: token buffers Q, K, V, O of [N][D] in
// the io type, then the memory unit's own workspace.
static ttt_status_t gcm_check(const ttt_problem_t* p, Shape* S, size_t* tok_bytes, size_t* ttt_bytes) {
  const ttt_status_t e = check_problem(p, S);
  if (e != TTT_OK) return e;
  if (p->stride_tok != 0 || p->stride_head != 0) return TTT_EINVAL;  // the layer's tensors are packed
  if (p->flags & (TTT_SAVE_CKPT | TTT_EMIT_LOSS)) return TTT_ENOTSUP;
  const int64_t D = (int64_t)S->H * S->d;
  if (D % 128 != 0 || D > 16384) return TTT_ESHAPE;
  *tok_bytes = align_up((size_t)p->n_tokens * (size_t)D * (S->io_bf16 ? 2 : 4));
  *ttt_bytes = ttt_workspace_bytes(p, 1);
  return *ttt_bytes ? TTT_OK : TTT_EINVAL;
}

size_t ttt_gcm_workspace_bytes(const ttt_problem_t* p) {
  try {
    Shape S{};
    size_t tb = 0, wb = 0;
    if (gcm_check(p, &S, &tb, &wb) != TTT_OK) return 0;
    return 4 * tb + wb;
  } catch (...) {
    return 0;
  }
}

ttt_status_t ttt_gcm_fwd(const ttt_problem_t* p, const void* X, const void* Wqkv, const float* bqkv, const void* Wo,
                         const float* bo, const float* alpha, const float* W1_0, const float* W2_0, void* Y,
                         float* W1_T, float* W2_T, void* ws, size_t ws_bytes, void* hip_stream) {
  try {
    Shape S{};
    size_t tb = 0, wb = 0;
    const ttt_status_t e = gcm_check(p, &S, &tb, &wb);
    if (e != TTT_OK) return e;
    if (!Wqkv || !Wo || !alpha || !W1_0 || !W2_0) return TTT_EINVAL;
    if (p->n_tokens > 0 && (!X || !Y)) return TTT_EINVAL;
    if ((W1_T == nullptr) != (W2_T == nullptr)) return TTT_EINVAL;
    for (const void* q : {X, Wqkv, Wo, (const void*)Y, (const void*)W1_0, (const void*)W2_0, (const void*)W1_T,
                          (const void*)W2_T})
      if (q && !aligned16(q)) return TTT_EINVAL;
    if (!ws || ws_bytes < 4 * tb + wb) return TTT_EWORKSPACE;
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    char* base = static_cast<char*>(ws);
    void* q = base;
    void* k = base + tb;
    void* v = base + 2 * tb;
    void* o = base + 3 * tb;
    if (p->n_tokens > 0) {
      GcmGemmArgs a{};
      a.kind = 0; a.D = S.H * S.d; a.rows = p->n_tokens;
      a.x = X; a.w = Wqkv; a.bias = bqkv; a.q = q; a.k = k; a.v = v;
      if (launch_gcm_gemm(a, S.io_bf16, st) != hipSuccess) return TTT_EHIP;
    }
    const ttt_status_t et = ttt_chunk_fwd(p, q, k, v, W1_0, W2_0, o, W1_T, W2_T, nullptr, nullptr, base + 4 * tb, wb,
                                          hip_stream);
    if (et != TTT_OK || p->n_tokens == 0) return et;
    GcmGemmArgs g{};
    g.kind = 1; g.D = S.H * S.d; g.rows = p->n_tokens;
    g.x = X; g.w = Wo; g.bias = bo; g.alpha = alpha; g.o = o; g.y = Y;
    return launch_gcm_gemm(g, S.io_bf16, st) == hipSuccess ? TTT_OK : TTT_EHIP;
  } catch (...) {
    return TTT_EINVAL;
  }
}

// Reverse mode of the layer: workspace regions.  The unit runs on views of
// the projection P [N][3D] (Q, K, V at column offsets 0, D, 2D, token pitch
// 3D), so its problem is the layer's with that pitch.
struct GcmBwdLayout {
  size_t P, O, dO, dP, dG, G, part, ckpt, unit, total;
  ttt_problem_t pu;
};
static ttt_status_t gcm_bwd_layout(const ttt_problem_t* p, GcmBwdLayout* L) {
  Shape S{};
  size_t tb = 0, wb = 0;
  const ttt_status_t e = gcm_check(p, &S, &tb, &wb);
  if (e != TTT_OK) return e;
  const int64_t N = p->n_tokens, D = (int64_t)S.H * S.d;
  const size_t io = S.io_bf16 ? 2 : 4;
  // the [N][3D] operands are addressed with 32-bit byte offsets
  if ((size_t)N * 3 * D * io >= ((size_t)1 << 31)) return TTT_ESHAPE;
  L->pu = *p;
  L->pu.stride_tok = 3 * D;
  L->pu.stride_head = S.d;
  Shape Su{};
  if (check_problem(&L->pu, &Su) != TTT_OK) return TTT_ESHAPE;
  const size_t ub = ttt_workspace_bytes(&L->pu, 1);
  if (!ub) return TTT_EINVAL;
  const int64_t C = (N + S.M - 1) / S.M;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L->P = take((size_t)N * 3 * D * io);
  L->O = take((size_t)N * 3 * D * io);
  L->dO = take((size_t)N * 3 * D * io);
  L->dP = take((size_t)N * 3 * D * io);
  L->dG = take((size_t)N * D * io);
  L->G = take((size_t)N * D * 4);
  L->part = take((size_t)((N + 255) / 256) * 3 * D * 4);
  L->ckpt = take((size_t)C * S.H * 2 * S.dh() * 4);
  L->unit = take(ub);
  L->total = off;
  return TTT_OK;
}

size_t ttt_gcm_bwd_workspace_bytes(const ttt_problem_t* p) {
  try {
    GcmBwdLayout L{};
    return gcm_bwd_layout(p, &L) == TTT_OK ? L.total : 0;
  } catch (...) {
    return 0;
  }
}

ttt_status_t ttt_gcm_bwd(const ttt_problem_t* p, const void* X, const void* Wqkv, const float* bqkv, const void* Wo,
                         const float* bo, const float* alpha, const float* W1_0, const float* W2_0, const void* dY,
                         void* dX, float* dWqkv, float* dbqkv, float* dWo, float* dbo, float* dalpha, float* dW1_0,
                         float* dW2_0, float* deta, void* ws, size_t ws_bytes, void* hip_stream) {
  try {
    GcmBwdLayout L{};
    const ttt_status_t e = gcm_bwd_layout(p, &L);
    if (e != TTT_OK) return e;
    Shape S{};
    check_problem(p, &S);
    if (!Wqkv || !Wo || !alpha || !W1_0 || !W2_0 || !dWqkv || !dWo || !dalpha || !dW1_0 || !dW2_0 || !deta)
      return TTT_EINVAL;
    if ((bqkv == nullptr) != (dbqkv == nullptr) || (bo == nullptr) != (dbo == nullptr)) return TTT_EINVAL;
    if (p->n_tokens > 0 && (!X || !dY || !dX)) return TTT_EINVAL;
    for (const void* q : {X, Wqkv, Wo, dY, (const void*)dX, (const void*)W1_0, (const void*)W2_0, (const void*)dWqkv,
                          (const void*)dWo, (const void*)dW1_0, (const void*)dW2_0})
      if (q && !aligned16(q)) return TTT_EINVAL;
    if (!ws || ws_bytes < L.total) return TTT_EWORKSPACE;
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int64_t N = p->n_tokens, D = (int64_t)S.H * S.d;
    const size_t io = S.io_bf16 ? 2 : 4;
    if (N == 0) {  // no tokens: every gradient is zero, dW of the unit too
      for (const std::pair<float*, int64_t>& z :
           {std::pair<float*, int64_t>{dWqkv, 3 * D * D}, {dWo, D * D}, {dalpha, D}, {dbqkv, dbqkv ? 3 * D : 0},
            {dbo, dbo ? D : 0}, {dW1_0, S.H * S.dh()}, {dW2_0, S.H * S.dh()}, {deta, S.H}})
        if (z.second > 0 && !launched([&] { return launch_large_zero(z.first, z.second, st); })) return TTT_EHIP;
      return TTT_OK;
    }
    char* b = static_cast<char*>(ws);
    GcmBwdArgs a{};
    a.D = (int32_t)D; a.rows = N;
    a.X = X; a.Wqkv = Wqkv; a.bqkv = bqkv; a.Wo = Wo; a.bo = bo; a.alpha = alpha; a.dY = dY;
    a.P = b + L.P; a.O = b + L.O; a.G = reinterpret_cast<float*>(b + L.G); a.dG = b + L.dG; a.dO = b + L.dO;
    a.dP = b + L.dP; a.part = reinterpret_cast<float*>(b + L.part);
    a.dX = dX; a.dWqkv = dWqkv; a.dbqkv = dbqkv; a.dWo = dWo; a.dbo = dbo; a.dalpha = dalpha;
    // the projection, then the unit's forward with its checkpoints
    a.phase = 0;
    if (launch_gcm_bwd(a, S.io_bf16, st) != hipSuccess) return TTT_EHIP;
    char* P = b + L.P;
    char* dP = b + L.dP;
    float* ckpt = reinterpret_cast<float*>(b + L.ckpt);
    ttt_problem_t pf = L.pu;
    pf.flags = (p->flags & ~(uint32_t)TTT_EMIT_LOSS) | TTT_SAVE_CKPT;
    ttt_status_t eu = ttt_chunk_fwd(&pf, P, P + D * io, P + 2 * D * io, W1_0, W2_0, b + L.O, nullptr, nullptr, ckpt,
                                    nullptr, b + L.unit, ws_bytes - L.unit, hip_stream);
    if (eu != TTT_OK) return eu;
    // the gate and the output projection
    a.phase = 1;
    if (launch_gcm_bwd(a, S.io_bf16, st) != hipSuccess) return TTT_EHIP;
    // the unit's reverse mode, its adjoints of Q, K, V into dP
    ttt_problem_t pb = L.pu;
    pb.flags = p->flags & ~(uint32_t)(TTT_EMIT_LOSS | TTT_SAVE_CKPT);
    eu = ttt_chunk_bwd(&pb, P, P + D * io, P + 2 * D * io, W1_0, W2_0, ckpt, b + L.dO, dP, dP + D * io,
                       dP + 2 * D * io, dW1_0, dW2_0, deta, b + L.unit, ws_bytes - L.unit, hip_stream);
    if (eu != TTT_OK) return eu;
    // the query-key-value projection
    a.phase = 2;
    return launch_gcm_bwd(a, S.io_bf16, st) == hipSuccess ? TTT_OK : TTT_EHIP;
  } catch (...) {
    return TTT_EINVAL;
  }
}

ttt_status_t ttt_workspace_status(const void* ws, size_t ws_bytes, uint32_t* flags_host, void* hip_stream) {
  if (!ws || !flags_host || ws_bytes < SYNC_BYTES) return TTT_EINVAL;
  const hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (hipMemcpyAsync(flags_host, static_cast<const uint32_t*>(ws) + SYNC_ERR, sizeof(uint32_t),
                     hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return TTT_EHIP;
  return TTT_OK;
}

const char* ttt_status_string(ttt_status_t s) {
  switch (s) {
    case TTT_OK: return "TTT_OK";
    case TTT_EINVAL: return "TTT_EINVAL: invalid argument";
    case TTT_ESHAPE: return "TTT_ESHAPE: unsupported shape or stride";
    case TTT_EWORKSPACE: return "TTT_EWORKSPACE: workspace missing or too small";
    case TTT_EHIP: return "TTT_EHIP: HIP launch failed";
    case TTT_ENOTSUP: return "TTT_ENOTSUP: not supported";
  }
  return "unknown status";
}

int32_t ttt_version(void) { return 200; }

}  // extern "C"
