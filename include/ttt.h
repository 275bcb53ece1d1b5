/*
 * ttt.h - C ABI of the MI355X (gfx950) chunked test-time-training library.
 *
 * The operation (Scal3R, Sec. 3.2 Eq. 3-4 and Sec. 4.2 Eq. 8): per sequence
 * and head there is a fast MLP f_W(x) = SiLU(x W1) W2 with W1: [d][h] and
 * W2: [h][d] (the per-head matrices of Supp. A, row-vector convention).  The
 * token stream is cut into chunks of `chunk_tokens` tokens (the last one may
 * be shorter).  For chunk c with M_c tokens, in sequence order:
 *
 *     L_c(W)  = (1/M_c) * sum_i || f_W(k_i) - v_i ||^2      (inner loss)
 *     W      <- W - eta * grad_W L_c(W)                      (update, Eq. 3/8)
 *     O_c     = f_W(Q_c)   with the updated W                (apply, Eq. 4)
 *
 * Q, K, V are optionally L2-normalised per token and head first,
 * x / max(||x||_2, 1e-12), inside the differentiated function.
 *
 * Conventions shared by every entry point
 *   - Token tensors (Q, K, V, O, dO, dQ, dK, dV) are [N][H][d] with d
 *     contiguous; element (t, h, j) lives at t*stride_tok + h*stride_head + j
 *     (defaults stride_tok = H*d, stride_head = d).  Their element type is
 *     io_dtype (float32 or bfloat16).
 *   - Fast weights and everything derived from them (W1_0, W2_0, W1_T, W2_T,
 *     checkpoints, dW1_0, dW2_0, deta, loss) are float32, dense, row-major:
 *     W1 [H][d][h], W2 [H][h][d].
 *   - All pointers except *_host ones are device pointers.  The caller owns
 *     every buffer, including the workspace; the library allocates no device
 *     memory and keeps no device state between calls.  Inputs are never
 *     modified; outputs are fully overwritten (never accumulated into).
 *   - Work is enqueued on `hip_stream` (a hipStream_t; NULL = default
 *     stream) and is asynchronous; the library never synchronises.
 *   - Validation happens before anything is enqueued: on any error status
 *     nothing has been launched.  Launch failures return TTT_EHIP.  No C++
 *     exception crosses this boundary.  Calls from different host threads
 *     are safe; calls that share a workspace must be stream-ordered.
 *   - Supported shapes: d = 64 with h in {128, 256} (fast weights held on
 *     chip by every entry point), and large states for ttt_chunk_fwd,
 *     ttt_chunk_bwd, ttt_batched_fwd, ttt_batched_fwd_ckpt, ttt_batched_bwd,
 *     ttt_gcs_fwd, ttt_gcs_bwd, ttt_amu_fwd, ttt_amu_bwd and ttt_gcm_fwd: d a multiple of 256 up to 4096 and h a
 *     multiple of 128 up to 16384 (the paper's single head of 1024 with
 *     hidden 4096), where every product of a chunk step is a GEMM over
 *     weights streamed from HBM and a chunk's rows times max(d, h) elements
 *     must stay below 2^31 bytes.  Other sizes return TTT_ESHAPE; the other
 *     entry points return TTT_ENOTSUP for large states.  n_tokens may be 0:
 *     token pointers may then be NULL, the final weights (if asked for) are
 *     the initial ones and nothing else is written.
 */
#ifndef TTT_H_
#define TTT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TTT_OK = 0,
  TTT_EINVAL = 1,      /* null pointer, bad flag, non-monotone cu_seqlens, ... */
  TTT_ESHAPE = 2,      /* unsupported d / h / strides */
  TTT_EWORKSPACE = 3,  /* workspace missing or smaller than ttt_workspace_bytes */
  TTT_EHIP = 4,        /* a HIP launch failed */
  TTT_ENOTSUP = 5      /* valid request this library does not implement */
} ttt_status_t;

typedef enum { TTT_F32 = 0, TTT_BF16 = 1 } ttt_dtype_t;

enum {
  TTT_NORM_Q = 1u,     /* L2-normalise Q rows */
  TTT_NORM_K = 2u,     /* L2-normalise K rows */
  TTT_NORM_V = 4u,     /* L2-normalise V rows */
  TTT_SAVE_CKPT = 8u,  /* write the weights before every chunk to `ckpt` */
  TTT_EMIT_LOSS = 16u, /* write the inner loss of every chunk to `loss` */
  TTT_MMA_BF16 = 32u   /* with io_dtype F32: round operands to bfloat16 for
                          the matrix cores (always on for io_dtype BF16) */
};

typedef struct {
  int32_t n_heads;      /* H >= 1 */
  int32_t d_head;       /* d: 64, or a large state (see above) */
  int32_t d_hidden;     /* h: 128 or 256 with d = 64, else a large state */
  int64_t n_tokens;     /* N for single-sequence calls (ignored by ttt_batched_fwd) */
  int64_t chunk_tokens; /* tokens per update chunk, >= 1 */
  int64_t stride_tok;   /* elements between consecutive tokens; 0 = H*d; at most 2^22 */
  int64_t stride_head;  /* elements between consecutive heads; 0 = d */
  float eta;            /* inner step size (one scalar for all heads and chunks) */
  uint32_t flags;       /* TTT_* bits */
  ttt_dtype_t io_dtype; /* element type of the token tensors */
} ttt_problem_t;

/* Optional launch shape; pass NULL for the built-in heuristic or the tuned
 * table.
 *   wg_per_chain  work-groups that share the chunks of one chain (0 =
 *                 automatic): each takes every wg_per_chain-th 32-token tile.
 *   target_wgs    total work-groups aimed for (0 = automatic: every
 *                 work-group the GPU can hold at once for the persistent
 *                 schedule, a per-step target for the stepwise one).
 *   schedule      TTT_SCHED_PERSISTENT (0): one launch walks every chunk of
 *                 every chain; the work-groups of a chain meet at barriers
 *                 between chunks and are sized so that all are resident.
 *                 TTT_SCHED_STEPWISE (1): one step launch and one update
 *                 launch per chunk step (the stream orders the steps).
 *   spin_limit    persistent schedule: polls a barrier wait may take before
 *                 it gives up and flags the workspace (see
 *                 ttt_workspace_status); 0 = default (about a second or
 *                 more).  Only meant to test that path. */
enum { TTT_SCHED_PERSISTENT = 0, TTT_SCHED_STEPWISE = 1 };
typedef struct {
  int32_t wg_per_chain;
  int32_t target_wgs;
  int32_t schedule;
  int32_t spin_limit;
} ttt_tile_cfg_t;

/* Bytes of device workspace needed by any call on `p` with `n_seqs`
 * sequences (1 for the chunk calls).  Returns 0 for an invalid problem. */
size_t ttt_workspace_bytes(const ttt_problem_t* p, int32_t n_seqs);

/* Forward over one sequence (Sec. 4.2, Eq. 8 then Eq. 4 per chunk).
 *   Q, K, V   [N][H][d] io_dtype, read only.
 *   W1_0      [H][d][h] f32; W2_0 [H][h][d] f32: initial fast weights.
 *   O         [N][H][d] io_dtype: O_c = f_{W_{c+1}}(Q_c).
 *   W1_T,W2_T final fast weights (same shapes as W1_0/W2_0), nullable.
 *   ckpt      [C][H][d*h + h*d] f32, required iff TTT_SAVE_CKPT: the weights
 *             before chunk c (W1 block then W2 block per head).
 *   loss      [H][C] f32, required iff TTT_EMIT_LOSS: L_c at the weights
 *             before chunk c's step.
 *   ws        device workspace of ws_bytes >= ttt_workspace_bytes(p, 1). */
ttt_status_t ttt_chunk_fwd(const ttt_problem_t* p, const void* Q, const void* K, const void* V,
                           const float* W1_0, const float* W2_0, void* O, float* W1_T, float* W2_T,
                           float* ckpt, float* loss, void* ws, size_t ws_bytes, void* hip_stream);

/* Backward of ttt_chunk_fwd for the outer loss sum <O, dO>, second-order
 * terms through every inner gradient included; recomputes each chunk from
 * its checkpoint.
 *   ckpt          the checkpoints written by ttt_chunk_fwd with TTT_SAVE_CKPT
 *                 on the same inputs.
 *   dO            [N][H][d] io_dtype.
 *   dQ, dK, dV    [N][H][d] io_dtype, gradients w.r.t. the *raw* Q, K, V.
 *   dW1_0, dW2_0  gradients w.r.t. the initial fast weights, f32.
 *   deta          [H] f32, per-head contribution to d/d eta (sum = total).
 * At large state sizes every product of the reverse step is a GEMM over
 * weights streamed from HBM, one head and one chunk at a time (the weights
 * after the last chunk are recomputed from its checkpoint first). */
ttt_status_t ttt_chunk_bwd(const ttt_problem_t* p, const void* Q, const void* K, const void* V,
                           const float* W1_0, const float* W2_0, const float* ckpt, const void* dO,
                           void* dQ, void* dK, void* dV, float* dW1_0, float* dW2_0, float* deta,
                           void* ws, size_t ws_bytes, void* hip_stream);

/* Forward over B sequences packed along the token axis ([sum N_b][H][d]),
 * each an independent chain.  cu_seqlens_host [B+1] is a HOST array of
 * monotone token offsets with cu_seqlens_host[0] = 0.  w0_per_seq = 0: all
 * sequences start from W1_0 [H][d][h] / W2_0 [H][h][d]; 1: per-sequence
 * [B][H][..].  W1_T, W2_T are [B][H][..] (nullable).  tile_cfg nullable.
 * Every chunk step of every sequence runs in the same stream-ordered
 * schedule; a sequence's ragged last chunk is normalised by its own size. */
ttt_status_t ttt_batched_fwd(const ttt_problem_t* p, int32_t n_seqs, const int64_t* cu_seqlens_host,
                             const void* Q, const void* K, const void* V, const float* W1_0,
                             const float* W2_0, int32_t w0_per_seq, void* O, float* W1_T, float* W2_T,
                             const ttt_tile_cfg_t* tile_cfg, void* ws, size_t ws_bytes, void* hip_stream);
/* ttt_batched_fwd that also writes the per-chunk checkpoints needed by
 * ttt_batched_bwd (TTT_SAVE_CKPT must be set, and only here: ttt_batched_fwd
 * rejects it with TTT_EINVAL; TTT_EMIT_LOSS is TTT_ENOTSUP for batches).
 *   ckpt  [sum_b C_b][H][d*h + h*d] f32, C_b = ceil(N_b / chunk_tokens):
 *         sequence b's rows follow those of sequences 0..b-1; row j of
 *         sequence b holds the weights before its chunk j. */
ttt_status_t ttt_batched_fwd_ckpt(const ttt_problem_t* p, int32_t n_seqs, const int64_t* cu_seqlens_host,
                                  const void* Q, const void* K, const void* V, const float* W1_0,
                                  const float* W2_0, int32_t w0_per_seq, void* O, float* W1_T, float* W2_T,
                                  float* ckpt, const ttt_tile_cfg_t* tile_cfg, void* ws, size_t ws_bytes,
                                  void* hip_stream);
/* Backward of ttt_batched_fwd_ckpt for the outer loss sum <O, dO> over all
 * sequences (each sequence's chain differentiated as in ttt_chunk_bwd).
 * The reverse chunk walks of all sequences run in one stream-ordered
 * schedule, aligned at each sequence's last chunk.
 *   ckpt          checkpoints of ttt_batched_fwd_ckpt on the same inputs.
 *   dO            [sum N_b][H][d] io_dtype; dQ, dK, dV likewise (raw inputs).
 *   dW1_0, dW2_0  w0_per_seq = 1: per-sequence gradients [B][H][..];
 *                 w0_per_seq = 0: gradient of the shared W_0, [H][..]
 *                 (the sum over sequences, in sequence order).
 *   deta          [H] f32: per-head d/d eta summed over sequences.
 *   tile_cfg      as in ttt_batched_fwd (nullable; not used at large state
 *                 sizes, where the sequences run one after another).
 *   ws            ws_bytes >= ttt_workspace_bytes(p, n_seqs). */
ttt_status_t ttt_batched_bwd(const ttt_problem_t* p, int32_t n_seqs, const int64_t* cu_seqlens_host,
                             const void* Q, const void* K, const void* V, const float* W1_0,
                             const float* W2_0, int32_t w0_per_seq, const float* ckpt, const void* dO,
                             void* dQ, void* dK, void* dV, float* dW1_0, float* dW2_0, float* deta,
                             const ttt_tile_cfg_t* tile_cfg, void* ws, size_t ws_bytes, void* hip_stream);

/* Global Context Synchronization form over one sequence (Sec. 4.2, Eq. 10):
 * every chunk's gradient is taken at the same initial weights W0 (chunk c
 * normalised by its own M_c), the gradients are summed over chunks, one step
 * W* = W0 - eta * sum_c grad L_c(W0) is applied, and every token's query is
 * mapped with W*: O = f_{W*}(Q).  Equal to ttt_chunk_fwd when there is one
 * chunk.  Buffers as in ttt_chunk_fwd; W1_T/W2_T receive W* (nullable);
 * loss [H][C] (iff TTT_EMIT_LOSS) holds each chunk's loss at W0.
 * TTT_SAVE_CKPT is not used (the only weights are W0 and W*).  The chunks'
 * shard partials share the workspace's max(H, 1024) partial slots: a stream
 * with more chunks x heads than that is summed in passes of as many chunks
 * as fit (each pass's sum added onto the running total in pass order), so
 * any chunk count runs in the workspace of ttt_workspace_bytes(p, 1).  At
 * large state sizes the chunks' steps -eta * grad L_c(W0) are subtracted
 * from the FP32 weights one chunk after another (in chunk order), one head
 * at a time, before the apply. */
ttt_status_t ttt_gcs_fwd(const ttt_problem_t* p, const void* Q, const void* K, const void* V,
                         const float* W1_0, const float* W2_0, void* O, float* W1_T, float* W2_T,
                         float* loss, void* ws, size_t ws_bytes, void* hip_stream);

/* Backward of ttt_gcs_fwd for sum <O, dO>: the adjoint of W* collects the
 * apply adjoint of every token, each chunk's update adjoint is taken at W0
 * against it, and dW0 = adjoint of W* + the sum of the chunks' terms.
 * Outputs as in ttt_chunk_bwd; W* is recomputed (as ttt_gcs_fwd, in passes
 * when the chunks x heads exceed the partial slots), no checkpoint is
 * needed. */
ttt_status_t ttt_gcs_bwd(const ttt_problem_t* p, const void* Q, const void* K, const void* V,
                         const float* W1_0, const float* W2_0, const void* dO, void* dQ, void* dK,
                         void* dV, float* dW1_0, float* dW2_0, float* deta, void* ws, size_t ws_bytes,
                         void* hip_stream);

/* The paper's adaptive memory unit (Supp. A; Sec. 4.2 Eq. 8-10) over one
 * sequence: per head a SwiGLU fast network
 *     f_W(x) = (SiLU(x W1) * (x W3)) W2,   W1, W3: [d][h], W2: [h][d],
 * the dot-product inner loss with token-wise step sizes,
 *     L_c(W) = - sum_{i in chunk c} eta_i <f_W(k_i), v_i>,
 * the step W <- W - grad_W L_c(W) (the step sizes are inside the loss, so
 * p->eta is not used), and the apply O_c = f_W(Q_c) after the update.
 *   sync      TTT_SYNC_CHAIN: chunks in sequence order, each updates then maps
 *             its queries; TTT_SYNC_GCS: every chunk's gradient at W_0 is
 *             summed, one update W*, every query mapped with W* (Eq. 10).
 *   eta_tok   [N][H] f32 token-wise step sizes (predicted by the model in the
 *             paper; an input here).
 *   W3_0      [H][d][h] f32; W3_T likewise (W1_T, W2_T, W3_T all or none).
 *   ws        ws_bytes >= ttt_amu_workspace_bytes(p).
 * Q, K, V, O, normalisation flags, TTT_MMA_BF16 and strides as in
 * ttt_chunk_fwd; TTT_SAVE_CKPT / TTT_EMIT_LOSS return TTT_ENOTSUP.  At
 * large state sizes (the paper's d = 1024, h = 4096) every product is a GEMM
 * over weights streamed from HBM, one head and one chunk at a time; the GCS
 * form then subtracts the chunks' gradients at W0 from the FP32 weights one
 * chunk after another (in chunk order) before the apply. */
enum { TTT_SYNC_CHAIN = 0, TTT_SYNC_GCS = 1 };
size_t ttt_amu_workspace_bytes(const ttt_problem_t* p);
ttt_status_t ttt_amu_fwd(const ttt_problem_t* p, int32_t sync, const void* Q, const void* K, const void* V,
                         const float* eta_tok, const float* W1_0, const float* W2_0, const float* W3_0,
                         void* O, float* W1_T, float* W2_T, float* W3_T, void* ws, size_t ws_bytes,
                         void* hip_stream);

/* Reverse mode of ttt_amu_fwd (same sync, same inputs) for the outer loss
 * sum <O, dO>, second-order terms through every inner update included:
 *   dQ, dK, dV  [N][H][d] in the io dtype (through the L2 normalisation);
 *   deta_tok    [N][H] f32, the derivative along each token's step size;
 *   dW1_0, dW3_0 [H][d][h], dW2_0 [H][h][d] f32.
 * The update of one chunk is W' = W - G(W) with G the gradient of
 * L(W) = sum_i <f_W(k_i), E_i>, E_i = -eta_i v_i; its adjoint needs
 * (dG/dX)^T Wh for the carried adjoint Wh of W', which is the gradient with
 * respect to X of the derivative of L along Wh (Supp. A network, Eq. 8-10).
 * TTT_SYNC_CHAIN recomputes W_1..W_C (no checkpoint argument) and walks the
 * chunks in reverse; TTT_SYNC_GCS recomputes W* and needs one apply-adjoint
 * and one update-adjoint pass over all tokens.  Every output is overwritten;
 * with n_tokens = 0 the weight adjoints are zero.  ws_bytes >=
 * ttt_amu_bwd_workspace_bytes(p, sync) (it grows with the chunk count for the
 * chain).  Errors as ttt_amu_fwd.  At large state sizes every product is a
 * GEMM over weights streamed from HBM, one head and one chunk at a time. */
size_t ttt_amu_bwd_workspace_bytes(const ttt_problem_t* p, int32_t sync);
ttt_status_t ttt_amu_bwd(const ttt_problem_t* p, int32_t sync, const void* Q, const void* K, const void* V,
                         const float* eta_tok, const float* W1_0, const float* W2_0, const float* W3_0,
                         const void* dO, void* dQ, void* dK, void* dV, float* deta_tok, float* dW1_0,
                         float* dW2_0, float* dW3_0, void* ws, size_t ws_bytes, void* hip_stream);

/* ttt_chunk_fwd without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, results and errors as ttt_chunk_fwd,
 * minus ws / ws_bytes: the scratch (shard partials, per-head ping-pong
 * weights, counters) is one fixed device array of
 * TTT_NOALLOC_SCRATCH_BYTES inside the library, present on every GPU the
 * library runs on until the process ends; the call allocates nothing.
 * Each head needs three fast-weight-sized FP32 blocks (2*d*h floats each:
 * two ping-pong copies and at least one shard partial), so problems with
 * more than 106 heads at h = 256 (213 at h = 128) return TTT_EWORKSPACE
 * with nothing enqueued; the work-groups per head are limited to the shard
 * partials that fit.  Every call on one GPU
 * uses that GPU's one array: calls that overlap on a GPU (other streams,
 * other host threads) race and must not be issued; calls ordered on one
 * stream are fine.  Always the stepwise schedule. */
#define TTT_NOALLOC_SCRATCH_BYTES (40u << 20)
ttt_status_t ttt_chunk_fwd_noalloc(const ttt_problem_t* p, const void* Q, const void* K, const void* V,
                                   const float* W1_0, const float* W2_0, void* O, float* W1_T, float* W2_T,
                                   float* ckpt, float* loss, void* hip_stream);

/* The layer around the memory unit over one sequence (Sec. 4.2: a
 * query-key-value projection, the memory unit, an output projection; Sec. 4.1
 * Eq. 5: the gate alpha * GCM(X) + X), for N tokens of width D = H * d:
 *     [Q | K | V] = X Wqkv (+ bqkv)     head h = features h*d .. h*d+d-1
 *     O = ttt_chunk_fwd(p, Q, K, V, W1_0, W2_0)
 *     Y = alpha * (O Wo (+ bo)) + X     alpha a per-feature gate vector
 *   p       the memory unit's problem; its strides must be 0 (the layer's
 *           token tensors are packed [N][D]); TTT_SAVE_CKPT / TTT_EMIT_LOSS
 *           are TTT_ENOTSUP.  D must be a multiple of 128 (TTT_ESHAPE).
 *   X, Y    [N][D] io_dtype (Y may not alias X).
 *   Wqkv    [D][3D] io_dtype, row-vector convention (x W): columns 0..D-1
 *           give Q, D..2D-1 K, 2D..3D-1 V.  bqkv [3D] f32, nullable.
 *   Wo      [D][D] io_dtype; bo [D] f32, nullable; alpha [D] f32.
 *   W1_0, W2_0, W1_T, W2_T  as ttt_chunk_fwd.
 *   ws      ws_bytes >= ttt_gcm_workspace_bytes(p): the projected Q, K, V
 *           and the unit's output O ([N][D] each, io_dtype) and the unit's
 *           own workspace.
 * The projections are matrix-core GEMMs in the io type (BF16 or FP32
 * operands, FP32 accumulation), each output element summed in a fixed
 * order.  Returns 0 bytes / TTT_EINVAL etc. as ttt_chunk_fwd. */
size_t ttt_gcm_workspace_bytes(const ttt_problem_t* p);
ttt_status_t ttt_gcm_fwd(const ttt_problem_t* p, const void* X, const void* Wqkv, const float* bqkv,
                         const void* Wo, const float* bo, const float* alpha, const float* W1_0,
                         const float* W2_0, void* Y, float* W1_T, float* W2_T, void* ws, size_t ws_bytes,
                         void* hip_stream);

/* Reverse mode of ttt_gcm_fwd for the outer loss sum <Y, dY> (Sec. 4.1
 * Eq. 5 and the projections of Sec. 4.2 taken back, with the memory unit's
 * reverse mode of ttt_chunk_bwd in between):
 *   dG = alpha * dY, dalpha = sum_n G * dY, dbo = sum_n dG, dWo = O^T dG,
 *   dO = dG Wo^T -> the unit's reverse mode -> dQ, dK, dV, dW1_0, dW2_0, deta,
 *   dP = [dQ | dK | dV], dWqkv = X^T dP, dbqkv = sum_n dP, dX = dY + dP Wqkv^T
 * with G = O Wo (+ bo) and O the unit's output, both recomputed.
 *   dY, dX     [N][D] io_dtype.
 *   dWqkv      [D][3D] f32; dbqkv [3D] f32 (given iff bqkv is).
 *   dWo        [D][D] f32; dbo [D] f32 (given iff bo is); dalpha [D] f32.
 *   dW1_0, dW2_0, deta  as ttt_chunk_bwd.
 *   ws         ws_bytes >= ttt_gcm_bwd_workspace_bytes(p): the projection,
 *              the unit's output and adjoints ([N][3D] each, io_dtype), G
 *              (FP32), the unit's checkpoints and its own workspace.
 * Column sums (dalpha, dbo, dbqkv) add slabs of 256 rows, then the slabs in
 * order; every product is a matrix-core GEMM summing its whole contraction
 * in a fixed order, so the result is deterministic.  The [N][3D] tensors
 * must stay below 2^31 bytes (TTT_ESHAPE).  Other errors as ttt_gcm_fwd. */
size_t ttt_gcm_bwd_workspace_bytes(const ttt_problem_t* p);
ttt_status_t ttt_gcm_bwd(const ttt_problem_t* p, const void* X, const void* Wqkv, const float* bqkv,
                         const void* Wo, const float* bo, const float* alpha, const float* W1_0,
                         const float* W2_0, const void* dY, void* dX, float* dWqkv, float* dbqkv, float* dWo,
                         float* dbo, float* dalpha, float* dW1_0, float* dW2_0, float* deta, void* ws,
                         size_t ws_bytes, void* hip_stream);

/* Device-side status of the last call that used workspace `ws`: copies the
 * workspace's error word to *flags_host (bit 0: a barrier wait of the
 * persistent forward gave up, so that call's outputs are invalid; 0: no
 * error).  The word is cleared by every forward call that has tokens
 * (ttt_chunk_fwd, ttt_batched_fwd, ttt_batched_fwd_ckpt).  This is the one
 * entry point that synchronises: it waits for `hip_stream`. */
ttt_status_t ttt_workspace_status(const void* ws, size_t ws_bytes, uint32_t* flags_host, void* hip_stream);

/* Human-readable name of a status code (static storage). */
const char* ttt_status_string(ttt_status_t s);

/* Library version as an integer (major*10000 + minor*100 + patch). */
int32_t ttt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TTT_H_ */
