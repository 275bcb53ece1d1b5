"""torch-facing wrappers of the C ABI (include/ttt.h).

Only argument marshalling happens here: shapes and dtypes are checked, output
and workspace tensors are allocated with torch (device memory plumbing), and
the library call is enqueued on torch's current stream.  Every step of the
computation runs in the HIP kernels of libttt_hip.so.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _lib as L

_DT = {torch.float32: L.TTT_F32, torch.bfloat16: L.TTT_BF16}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(dev: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _flags(norm, save_ckpt=False, emit_loss=False, mma_bf16=False):
    nq, nk, nv = (norm, norm, norm) if isinstance(norm, bool) else norm
    f = (L.TTT_NORM_Q if nq else 0) | (L.TTT_NORM_K if nk else 0) | (L.TTT_NORM_V if nv else 0)
    f |= (L.TTT_SAVE_CKPT if save_ckpt else 0) | (L.TTT_EMIT_LOSS if emit_loss else 0)
    f |= L.TTT_MMA_BF16 if mma_bf16 else 0
    return f


def _check_tokens(Q, K, V):
    for t in (Q, K, V):
        if not t.is_cuda:
            raise ValueError("token tensors must be on the GPU")
        if t.dim() != 3 or (t.numel() > 0 and t.stride(-1) != 1):
            raise ValueError("token tensors must be [N][H][d] with d contiguous")
        if t.dtype not in _DT:
            raise ValueError(f"unsupported dtype {t.dtype}")
    if not (Q.shape == K.shape == V.shape and Q.dtype == K.dtype == V.dtype):
        raise ValueError("Q, K, V must share shape and dtype")
    if Q.numel() > 0 and not (Q.stride() == K.stride() == V.stride()):
        raise ValueError("Q, K, V must share strides")


def _like_tokens(Q, out):
    """Output token tensor with exactly Q's strides (the ABI addresses every
    token tensor with one (stride_tok, stride_head) pair)."""
    if out is None:
        return torch.empty_strided(Q.size(), Q.stride(), dtype=Q.dtype, device=Q.device)
    if out.shape != Q.shape or out.stride() != Q.stride() or out.dtype != Q.dtype or out.device != Q.device:
        raise ValueError("output token tensor must match Q's shape, strides, dtype and device")
    return out


def _check_w(W1, W2, H, lead=()):
    if W1.dtype != torch.float32 or W2.dtype != torch.float32:
        raise ValueError("fast weights are float32")
    if not (W1.is_contiguous() and W2.is_contiguous()):
        raise ValueError("fast weights must be contiguous")
    d, h = W1.shape[-2], W1.shape[-1]
    if tuple(W1.shape) != tuple(lead) + (H, d, h) or tuple(W2.shape) != tuple(lead) + (H, h, d):
        raise ValueError(f"bad fast-weight shapes {tuple(W1.shape)} {tuple(W2.shape)}")
    return d, h


def problem(Q, h, n_tokens, chunk_tokens, eta, flags):
    N, H, d = Q.shape
    # an empty tensor's strides carry no layout: the defaults apply (0)
    st_tok, st_head = (Q.stride(0), Q.stride(1)) if Q.numel() > 0 else (0, 0)
    return L.Problem(n_heads=H, d_head=d, d_hidden=h, n_tokens=n_tokens, chunk_tokens=int(chunk_tokens),
                     stride_tok=st_tok, stride_head=st_head, eta=float(eta), flags=flags, io_dtype=_DT[Q.dtype])


def workspace(prob, n_seqs, device):
    lib = L.load()
    nbytes = lib.ttt_workspace_bytes(ctypes.byref(prob), n_seqs)
    if nbytes == 0:
        raise L.TTTError(L.TTT_ESHAPE, lib, "ttt_workspace_bytes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def workspace_status(ws) -> int:
    """Error word of the last call on workspace `ws` (bit 0: a barrier wait of
    the persistent forward gave up).  Waits for the current stream."""
    lib = L.load()
    out = ctypes.c_uint32(0)
    L.check(lib.ttt_workspace_status(_ptr(ws), ws.numel(), ctypes.byref(out), _stream(ws.device)),
            "ttt_workspace_status")
    return int(out.value)


def n_chunks(n_tokens: int, chunk_tokens: int) -> int:
    return (n_tokens + chunk_tokens - 1) // chunk_tokens


def chunk_fwd(Q, K, V, W1, W2, eta, chunk_tokens, *, norm=True, save_ckpt=False, emit_loss=False,
              mma_bf16=False, want_final=True, out=None, ws=None):
    """Chunked TTT forward over one sequence.  Returns a dict with O and,
    as requested, W1_T, W2_T, ckpt [C][H][2dh], loss [H][C]."""
    lib = L.load()
    _check_tokens(Q, K, V)
    N, H, d = Q.shape
    _, h = _check_w(W1, W2, H)
    prob = problem(Q, h, N, chunk_tokens, eta, _flags(norm, save_ckpt, emit_loss, mma_bf16))
    C = n_chunks(N, chunk_tokens)
    dev = Q.device
    O = _like_tokens(Q, out)
    W1_T = torch.empty_like(W1) if want_final else None
    W2_T = torch.empty_like(W2) if want_final else None
    ckpt = torch.empty((C, H, 2 * d * h), dtype=torch.float32, device=dev) if save_ckpt else None
    loss = torch.empty((H, C), dtype=torch.float32, device=dev) if emit_loss else None
    if ws is None:
        ws = workspace(prob, 1, dev)
    st = lib.ttt_chunk_fwd(ctypes.byref(prob), _ptr(Q), _ptr(K), _ptr(V), _ptr(W1), _ptr(W2), _ptr(O),
                           _ptr(W1_T), _ptr(W2_T), _ptr(ckpt), _ptr(loss), _ptr(ws), ws.numel(), _stream(dev))
    L.check(st, "ttt_chunk_fwd")
    return dict(O=O, W1_T=W1_T, W2_T=W2_T, ckpt=ckpt, loss=loss)


def _gcm_problem(X, Wqkv, Wo, alpha, W1, W2, eta, chunk_tokens, bqkv, bo, norm):
    if X.dim() != 2 or not X.is_contiguous():
        raise ValueError("X must be a contiguous [N][D] tensor")
    N, D = X.shape
    H = W1.shape[0]
    if D % H:
        raise ValueError("D must be a multiple of the head count")
    d = D // H
    _, h = _check_w(W1, W2, H)
    if W1.shape[1] != d:
        raise ValueError(f"fast weights of head size {W1.shape[1]} for features {D} / {H} heads")
    for t, shp in ((Wqkv, (D, 3 * D)), (Wo, (D, D))):
        if tuple(t.shape) != shp or t.dtype != X.dtype or not t.is_contiguous():
            raise ValueError(f"projection weight must be contiguous {shp} in {X.dtype}")
    for t, n in ((alpha, D), (bqkv, 3 * D), (bo, D)):
        if t is not None and (t.dtype != torch.float32 or t.numel() != n or not t.is_contiguous()):
            raise ValueError("alpha and the biases are contiguous float32 vectors")
    return L.Problem(n_heads=H, d_head=d, d_hidden=h, n_tokens=N, chunk_tokens=int(chunk_tokens), stride_tok=0,
                     stride_head=0, eta=float(eta), flags=_flags(norm), io_dtype=_DT[X.dtype])


def gcm_fwd(X, Wqkv, Wo, alpha, W1, W2, eta, chunk_tokens, *, bqkv=None, bo=None, norm=True, want_final=True,
            out=None, ws=None):
    """The layer around the memory unit over one sequence: [Q|K|V] = X Wqkv
    (+ bqkv), O = chunked TTT forward of Q, K, V with H = W1.shape[0] heads,
    Y = alpha * (O Wo (+ bo)) + X.  X: [N][D] (float32 or bfloat16), Wqkv
    [D][3D] and Wo [D][D] in X's dtype, biases and alpha float32.  Returns
    dict(Y, W1_T, W2_T)."""
    lib = L.load()
    prob = _gcm_problem(X, Wqkv, Wo, alpha, W1, W2, eta, chunk_tokens, bqkv, bo, norm)
    Y = torch.empty_like(X) if out is None else out
    W1_T = torch.empty_like(W1) if want_final else None
    W2_T = torch.empty_like(W2) if want_final else None
    if ws is None:
        nbytes = lib.ttt_gcm_workspace_bytes(ctypes.byref(prob))
        if nbytes == 0:
            raise L.TTTError(L.TTT_ESHAPE, lib, "ttt_gcm_workspace_bytes")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=X.device)
    st = lib.ttt_gcm_fwd(ctypes.byref(prob), _ptr(X), _ptr(Wqkv), _ptr(bqkv), _ptr(Wo), _ptr(bo), _ptr(alpha),
                         _ptr(W1), _ptr(W2), _ptr(Y), _ptr(W1_T), _ptr(W2_T), _ptr(ws), ws.numel(), _stream(X.device))
    L.check(st, "ttt_gcm_fwd")
    return dict(Y=Y, W1_T=W1_T, W2_T=W2_T)


def gcm_bwd(X, Wqkv, Wo, alpha, W1, W2, eta, chunk_tokens, dY, *, bqkv=None, bo=None, norm=True, ws=None):
    """Reverse mode of gcm_fwd for sum <Y, dY> (same inputs): returns dX (X's
    dtype) and float32 dWqkv, dbqkv, dWo, dbo (None where the bias is),
    dalpha, dW1_0, dW2_0, deta [H]."""
    lib = L.load()
    prob = _gcm_problem(X, Wqkv, Wo, alpha, W1, W2, eta, chunk_tokens, bqkv, bo, norm)
    if dY.shape != X.shape or dY.dtype != X.dtype or not dY.is_contiguous():
        raise ValueError("dY must be a contiguous tensor like X")
    D = X.shape[1]
    dev = X.device
    f32 = dict(dtype=torch.float32, device=dev)
    dX = torch.empty_like(X)
    g = dict(dWqkv=torch.empty((D, 3 * D), **f32), dbqkv=torch.empty(3 * D, **f32) if bqkv is not None else None,
             dWo=torch.empty((D, D), **f32), dbo=torch.empty(D, **f32) if bo is not None else None,
             dalpha=torch.empty(D, **f32), dW1_0=torch.empty_like(W1), dW2_0=torch.empty_like(W2),
             deta=torch.empty(W1.shape[0], **f32))
    if ws is None:
        nbytes = lib.ttt_gcm_bwd_workspace_bytes(ctypes.byref(prob))
        if nbytes == 0:
            raise L.TTTError(L.TTT_ESHAPE, lib, "ttt_gcm_bwd_workspace_bytes")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    st = lib.ttt_gcm_bwd(ctypes.byref(prob), _ptr(X), _ptr(Wqkv), _ptr(bqkv), _ptr(Wo), _ptr(bo), _ptr(alpha),
                         _ptr(W1), _ptr(W2), _ptr(dY), _ptr(dX), _ptr(g["dWqkv"]), _ptr(g["dbqkv"]), _ptr(g["dWo"]),
                         _ptr(g["dbo"]), _ptr(g["dalpha"]), _ptr(g["dW1_0"]), _ptr(g["dW2_0"]), _ptr(g["deta"]),
                         _ptr(ws), ws.numel(), _stream(dev))
    L.check(st, "ttt_gcm_bwd")
    return dict(dX=dX, **g)


def chunk_fwd_noalloc(Q, K, V, W1, W2, eta, chunk_tokens, *, norm=True, save_ckpt=False, emit_loss=False,
                      mma_bf16=False, out=None, W1_T=None, W2_T=None, ckpt=None, loss=None):
    """chunk_fwd through the allocation-free entry point: the library uses its
    fixed device scratch instead of a workspace.  Output tensors may be
    passed in (then nothing at all is allocated here)."""
    lib = L.load()
    _check_tokens(Q, K, V)
    N, H, d = Q.shape
    _, h = _check_w(W1, W2, H)
    prob = problem(Q, h, N, chunk_tokens, eta, _flags(norm, save_ckpt, emit_loss, mma_bf16))
    C = n_chunks(N, chunk_tokens)
    dev = Q.device
    O = _like_tokens(Q, out)
    W1_T = torch.empty_like(W1) if W1_T is None else W1_T
    W2_T = torch.empty_like(W2) if W2_T is None else W2_T
    if save_ckpt and ckpt is None:
        ckpt = torch.empty((C, H, 2 * d * h), dtype=torch.float32, device=dev)
    if emit_loss and loss is None:
        loss = torch.empty((H, C), dtype=torch.float32, device=dev)
    st = lib.ttt_chunk_fwd_noalloc(ctypes.byref(prob), _ptr(Q), _ptr(K), _ptr(V), _ptr(W1), _ptr(W2), _ptr(O),
                                   _ptr(W1_T), _ptr(W2_T), _ptr(ckpt if save_ckpt else None),
                                   _ptr(loss if emit_loss else None), _stream(dev))
    L.check(st, "ttt_chunk_fwd_noalloc")
    return dict(O=O, W1_T=W1_T, W2_T=W2_T, ckpt=ckpt, loss=loss)


def _tile_cfg(tile_cfg, Q, h, chunk_tokens, n_chains, kind="fwd"):
    """An explicit launch shape (dict), or None: the library then uses the
    autotuner's recorded shape for the problem (compiled in), else its
    heuristic."""
    if tile_cfg is None:
        return None
    sched = {"persistent": L.TTT_SCHED_PERSISTENT, "stepwise": L.TTT_SCHED_STEPWISE}[tile_cfg.get("schedule",
                                                                                                  "persistent")]
    return L.TileCfg(int(tile_cfg.get("wg_per_chain", 0)), int(tile_cfg.get("target_wgs", 0)), sched,
                     int(tile_cfg.get("spin_limit", 0)))


def batch_chunks(cu_seqlens: Sequence[int], chunk_tokens: int):
    """Chunks per sequence and the first checkpoint row of each sequence."""
    cu = [int(x) for x in cu_seqlens]
    cb = [n_chunks(cu[b + 1] - cu[b], chunk_tokens) for b in range(len(cu) - 1)]
    rows = [0]
    for c in cb:
        rows.append(rows[-1] + c)
    return cb, rows


def batched_fwd(Q, K, V, cu_seqlens: Sequence[int], W1, W2, eta, chunk_tokens, *, norm=True, w0_per_seq=False,
                mma_bf16=False, want_final=True, save_ckpt=False, tile_cfg=None, out=None, ws=None):
    """Many sequences packed along the token axis ([sum N_b][H][d]) with host
    offsets cu_seqlens [B+1]; one independent chain per sequence and head.
    With save_ckpt, also returns ckpt [sum_b C_b][H][2dh] (sequence b's rows
    start at batch_chunks(cu_seqlens, chunk_tokens)[1][b])."""
    lib = L.load()
    _check_tokens(Q, K, V)
    N, H, d = Q.shape
    cu = [int(x) for x in cu_seqlens]
    B = len(cu) - 1
    _, h = _check_w(W1, W2, H, (B,) if w0_per_seq else ())
    if cu[-1] != N:
        raise ValueError("cu_seqlens[-1] must equal the packed token count")
    prob = problem(Q, h, 0, chunk_tokens, eta, _flags(norm, save_ckpt=save_ckpt, mma_bf16=mma_bf16))
    dev = Q.device
    O = _like_tokens(Q, out)
    W1_T = torch.empty((B, H, d, h), dtype=torch.float32, device=dev) if want_final else None
    W2_T = torch.empty((B, H, h, d), dtype=torch.float32, device=dev) if want_final else None
    cu_arr = (ctypes.c_int64 * (B + 1))(*cu)
    cfg = _tile_cfg(tile_cfg, Q, h, chunk_tokens, B * H)
    if ws is None:
        ws = workspace(prob, B, dev)
    args = [ctypes.byref(prob), B, cu_arr, _ptr(Q), _ptr(K), _ptr(V), _ptr(W1), _ptr(W2), 1 if w0_per_seq else 0,
            _ptr(O), _ptr(W1_T), _ptr(W2_T)]
    tail = [ctypes.byref(cfg) if cfg is not None else None, _ptr(ws), ws.numel(), _stream(dev)]
    ckpt = None
    if save_ckpt:
        rows = batch_chunks(cu, chunk_tokens)[1][-1]
        ckpt = torch.empty((rows, H, 2 * d * h), dtype=torch.float32, device=dev)
        st = lib.ttt_batched_fwd_ckpt(*args, _ptr(ckpt), *tail)
        L.check(st, "ttt_batched_fwd_ckpt")
    else:
        st = lib.ttt_batched_fwd(*args, *tail)
        L.check(st, "ttt_batched_fwd")
    return dict(O=O, W1_T=W1_T, W2_T=W2_T, ckpt=ckpt)


def batched_bwd(Q, K, V, cu_seqlens: Sequence[int], W1, W2, eta, chunk_tokens, ckpt, dO, *, norm=True,
                w0_per_seq=False, mma_bf16=False, tile_cfg=None, ws=None):
    """Backward of batched_fwd(save_ckpt=True) for sum <O, dO>.  dW1_0/dW2_0
    are per sequence [B][H][..] with w0_per_seq, else the shared W0's
    gradient [H][..]; deta [H] is summed over sequences."""
    lib = L.load()
    _check_tokens(Q, K, V)
    _check_tokens(Q, dO, dO)
    N, H, d = Q.shape
    cu = [int(x) for x in cu_seqlens]
    B = len(cu) - 1
    _, h = _check_w(W1, W2, H, (B,) if w0_per_seq else ())
    if cu[-1] != N:
        raise ValueError("cu_seqlens[-1] must equal the packed token count")
    if dO.stride() != Q.stride():
        raise ValueError("dO must share Q's strides")
    prob = problem(Q, h, 0, chunk_tokens, eta, _flags(norm, mma_bf16=mma_bf16))
    dev = Q.device
    dQ, dK, dV = (_like_tokens(Q, None) for _ in range(3))
    dW1 = torch.empty_like(W1)
    dW2 = torch.empty_like(W2)
    deta = torch.empty((H,), dtype=torch.float32, device=dev)
    cu_arr = (ctypes.c_int64 * (B + 1))(*cu)
    cfg = _tile_cfg(tile_cfg, Q, h, chunk_tokens, B * H, "bwd")
    if ws is None:
        ws = workspace(prob, B, dev)
    st = lib.ttt_batched_bwd(ctypes.byref(prob), B, cu_arr, _ptr(Q), _ptr(K), _ptr(V), _ptr(W1), _ptr(W2),
                             1 if w0_per_seq else 0, _ptr(ckpt), _ptr(dO), _ptr(dQ), _ptr(dK), _ptr(dV), _ptr(dW1),
                             _ptr(dW2), _ptr(deta), ctypes.byref(cfg) if cfg is not None else None, _ptr(ws),
                             ws.numel(), _stream(dev))
    L.check(st, "ttt_batched_bwd")
    return dict(dQ=dQ, dK=dK, dV=dV, dW1_0=dW1, dW2_0=dW2, deta=deta)


def chunk_bwd(Q, K, V, W1, W2, eta, chunk_tokens, ckpt, dO, *, norm=True, mma_bf16=False, ws=None):
    """Backward of chunk_fwd for the outer loss sum <O, dO>.  `ckpt` is the
    [C][H][2dh] checkpoint tensor of the forward (save_ckpt=True).  Returns
    dQ, dK, dV (raw-input gradients, io dtype), dW1_0, dW2_0 and deta [H]."""
    lib = L.load()
    _check_tokens(Q, K, V)
    _check_tokens(Q, dO, dO)
    N, H, d = Q.shape
    _, h = _check_w(W1, W2, H)
    if dO.stride() != Q.stride():
        raise ValueError("dO must share Q's strides")
    prob = problem(Q, h, N, chunk_tokens, eta, _flags(norm, mma_bf16=mma_bf16))
    dev = Q.device
    dQ, dK, dV = (_like_tokens(Q, None) for _ in range(3))
    dW1 = torch.empty_like(W1)
    dW2 = torch.empty_like(W2)
    deta = torch.empty((H,), dtype=torch.float32, device=dev)
    if ws is None:
        ws = workspace(prob, 1, dev)
    st = lib.ttt_chunk_bwd(ctypes.byref(prob), _ptr(Q), _ptr(K), _ptr(V), _ptr(W1), _ptr(W2), _ptr(ckpt), _ptr(dO),
                           _ptr(dQ), _ptr(dK), _ptr(dV), _ptr(dW1), _ptr(dW2), _ptr(deta), _ptr(ws), ws.numel(),
                           _stream(dev))
    L.check(st, "ttt_chunk_bwd")
    return dict(dQ=dQ, dK=dK, dV=dV, dW1_0=dW1, dW2_0=dW2, deta=deta)


class TTTChunk(torch.autograd.Function):
    """O = chunked TTT forward over one sequence, differentiable in
    (Q, K, V, W1_0, W2_0, eta).  The forward saves the per-chunk weight
    checkpoints; the backward recomputes each chunk from them in the HIP
    backward kernels."""

    @staticmethod
    def forward(ctx, Q, K, V, W1, W2, eta, chunk_tokens, norm=True, mma_bf16=False):
        # eta is a Python number or a one-element tensor (read on the host:
        # the step size is a launch argument; a GPU tensor costs one sync)
        if isinstance(eta, torch.Tensor) and eta.numel() != 1:
            raise ValueError("eta must be a scalar or a one-element tensor")
        eta_f = float(eta)
        need = any(ctx.needs_input_grad[:6])
        r = chunk_fwd(Q, K, V, W1, W2, eta_f, chunk_tokens, norm=norm, save_ckpt=need, mma_bf16=mma_bf16,
                      want_final=False)
        ctx.chunk_tokens, ctx.norm, ctx.mma_bf16, ctx.eta = chunk_tokens, norm, mma_bf16, eta_f
        ctx.eta_is_tensor = isinstance(eta, torch.Tensor)
        ctx.eta_shape = tuple(eta.shape) if ctx.eta_is_tensor else ()
        if need:
            ctx.save_for_backward(Q, K, V, W1, W2, r["ckpt"])
        return r["O"]

    @staticmethod
    def backward(ctx, dO):
        Q, K, V, W1, W2, ckpt = ctx.saved_tensors
        dO = dO.contiguous() if dO.stride() != Q.stride() else dO
        if dO.stride() != Q.stride():
            dO = torch.empty_strided(Q.size(), Q.stride(), dtype=Q.dtype, device=Q.device).copy_(dO)
        g = chunk_bwd(Q, K, V, W1, W2, ctx.eta, ctx.chunk_tokens, ckpt, dO.to(Q.dtype), norm=ctx.norm,
                      mma_bf16=ctx.mma_bf16)
        deta = g["deta"].sum().reshape(ctx.eta_shape) if ctx.eta_is_tensor else None
        return g["dQ"], g["dK"], g["dV"], g["dW1_0"], g["dW2_0"], deta, None, None, None


def ttt_chunk(Q, K, V, W1, W2, eta, chunk_tokens, norm=True, mma_bf16=False):
    """Differentiable chunked TTT forward (see TTTChunk)."""
    return TTTChunk.apply(Q, K, V, W1, W2, eta, chunk_tokens, norm, mma_bf16)


def gcs_fwd(Q, K, V, W1, W2, eta, chunk_tokens, *, norm=True, emit_loss=False, mma_bf16=False, want_final=True,
            out=None, ws=None):
    """Global Context Synchronization forward over one sequence: the chunks'
    gradients at W0 are summed, one step gives W*, O = f_{W*}(Q)."""
    lib = L.load()
    _check_tokens(Q, K, V)
    N, H, d = Q.shape
    _, h = _check_w(W1, W2, H)
    prob = problem(Q, h, N, chunk_tokens, eta, _flags(norm, emit_loss=emit_loss, mma_bf16=mma_bf16))
    dev = Q.device
    O = _like_tokens(Q, out)
    W1_T = torch.empty_like(W1) if want_final else None
    W2_T = torch.empty_like(W2) if want_final else None
    loss = torch.empty((H, n_chunks(N, chunk_tokens)), dtype=torch.float32, device=dev) if emit_loss else None
    if ws is None:
        ws = workspace(prob, 1, dev)
    st = lib.ttt_gcs_fwd(ctypes.byref(prob), _ptr(Q), _ptr(K), _ptr(V), _ptr(W1), _ptr(W2), _ptr(O), _ptr(W1_T),
                         _ptr(W2_T), _ptr(loss), _ptr(ws), ws.numel(), _stream(dev))
    L.check(st, "ttt_gcs_fwd")
    return dict(O=O, W1_T=W1_T, W2_T=W2_T, loss=loss)


def gcs_bwd(Q, K, V, W1, W2, eta, chunk_tokens, dO, *, norm=True, mma_bf16=False, ws=None):
    """Backward of gcs_fwd for sum <O, dO>."""
    lib = L.load()
    _check_tokens(Q, K, V)
    _check_tokens(Q, dO, dO)
    N, H, d = Q.shape
    _, h = _check_w(W1, W2, H)
    if dO.stride() != Q.stride():
        raise ValueError("dO must share Q's strides")
    prob = problem(Q, h, N, chunk_tokens, eta, _flags(norm, mma_bf16=mma_bf16))
    dev = Q.device
    dQ, dK, dV = (_like_tokens(Q, None) for _ in range(3))
    dW1 = torch.empty_like(W1)
    dW2 = torch.empty_like(W2)
    deta = torch.empty((H,), dtype=torch.float32, device=dev)
    if ws is None:
        ws = workspace(prob, 1, dev)
    st = lib.ttt_gcs_bwd(ctypes.byref(prob), _ptr(Q), _ptr(K), _ptr(V), _ptr(W1), _ptr(W2), _ptr(dO), _ptr(dQ),
                         _ptr(dK), _ptr(dV), _ptr(dW1), _ptr(dW2), _ptr(deta), _ptr(ws), ws.numel(), _stream(dev))
    L.check(st, "ttt_gcs_bwd")
    return dict(dQ=dQ, dK=dK, dV=dV, dW1_0=dW1, dW2_0=dW2, deta=deta)


def amu_fwd(Q, K, V, eta_tok, W1, W2, W3, chunk_tokens, *, sync="chain", norm=True, mma_bf16=False,
            want_final=True, out=None, ws=None):
    """The paper's adaptive memory unit over one sequence: SwiGLU fast network
    (W1, W3: [H][d][h], W2: [H][h][d]), dot-product inner loss with the
    token-wise step sizes eta_tok [N][H] (float32), chain or GCS ("gcs")
    synchronisation.  Returns O and, if want_final, W1_T, W2_T, W3_T."""
    lib = L.load()
    _check_tokens(Q, K, V)
    N, H, d = Q.shape
    _, h = _check_w(W1, W2, H)
    if W3.shape != W1.shape or W3.dtype != torch.float32 or not W3.is_contiguous():
        raise ValueError("W3 must be a contiguous float32 tensor shaped like W1")
    if eta_tok.shape != (N, H) or eta_tok.dtype != torch.float32 or not eta_tok.is_contiguous():
        raise ValueError("eta_tok must be a contiguous float32 [N][H] tensor")
    sync_id = {"chain": L.TTT_SYNC_CHAIN, "gcs": L.TTT_SYNC_GCS}[sync]
    prob = problem(Q, h, N, chunk_tokens, 0.0, _flags(norm, mma_bf16=mma_bf16))
    dev = Q.device
    O = _like_tokens(Q, out)
    fin = [torch.empty_like(W) if want_final else None for W in (W1, W2, W3)]
    if ws is None:
        nbytes = lib.ttt_amu_workspace_bytes(ctypes.byref(prob))
        if nbytes == 0:
            raise L.TTTError(L.TTT_ESHAPE, lib, "ttt_amu_workspace_bytes")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    st = lib.ttt_amu_fwd(ctypes.byref(prob), sync_id, _ptr(Q), _ptr(K), _ptr(V), _ptr(eta_tok), _ptr(W1), _ptr(W2),
                         _ptr(W3), _ptr(O), _ptr(fin[0]), _ptr(fin[1]), _ptr(fin[2]), _ptr(ws), ws.numel(),
                         _stream(dev))
    L.check(st, "ttt_amu_fwd")
    return dict(O=O, W1_T=fin[0], W2_T=fin[1], W3_T=fin[2])


def amu_bwd(Q, K, V, eta_tok, W1, W2, W3, chunk_tokens, dO, *, sync="chain", norm=True, mma_bf16=False, ws=None):
    """Reverse mode of amu_fwd for sum <O, dO> (same inputs and sync): returns
    dQ, dK, dV (io dtype), deta_tok [N][H] and dW1_0, dW2_0, dW3_0 (float32)."""
    lib = L.load()
    _check_tokens(Q, K, V)
    N, H, d = Q.shape
    _, h = _check_w(W1, W2, H)
    if W3.shape != W1.shape or W3.dtype != torch.float32 or not W3.is_contiguous():
        raise ValueError("W3 must be a contiguous float32 tensor shaped like W1")
    if eta_tok.shape != (N, H) or eta_tok.dtype != torch.float32 or not eta_tok.is_contiguous():
        raise ValueError("eta_tok must be a contiguous float32 [N][H] tensor")
    sync_id = {"chain": L.TTT_SYNC_CHAIN, "gcs": L.TTT_SYNC_GCS}[sync]
    prob = problem(Q, h, N, chunk_tokens, 0.0, _flags(norm, mma_bf16=mma_bf16))
    dev = Q.device
    dQ, dK, dV = (_like_tokens(Q, None) for _ in range(3))
    if dO.shape != Q.shape or dO.stride() != Q.stride() or dO.dtype != Q.dtype:
        raise ValueError("dO must match Q's shape, strides and dtype")
    deta = torch.empty_like(eta_tok)
    dW = [torch.empty_like(W) for W in (W1, W2, W3)]
    if ws is None:
        nbytes = lib.ttt_amu_bwd_workspace_bytes(ctypes.byref(prob), sync_id)
        if nbytes == 0:
            raise L.TTTError(L.TTT_ESHAPE, lib, "ttt_amu_bwd_workspace_bytes")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    st = lib.ttt_amu_bwd(ctypes.byref(prob), sync_id, _ptr(Q), _ptr(K), _ptr(V), _ptr(eta_tok), _ptr(W1), _ptr(W2),
                         _ptr(W3), _ptr(dO), _ptr(dQ), _ptr(dK), _ptr(dV), _ptr(deta), _ptr(dW[0]), _ptr(dW[1]),
                         _ptr(dW[2]), _ptr(ws), ws.numel(), _stream(dev))
    L.check(st, "ttt_amu_bwd")
    return dict(dQ=dQ, dK=dK, dV=dV, deta_tok=deta, dW1_0=dW[0], dW2_0=dW[1], dW3_0=dW[2])


class AMUChunk(torch.autograd.Function):
    """O = the paper's memory unit (SwiGLU fast network, dot-product inner
    loss with token-wise step sizes, chain or GCS) over one sequence,
    differentiable in (Q, K, V, eta_tok, W1_0, W2_0, W3_0).  The backward
    recomputes the weights it needs in the HIP reverse-mode kernels (nothing
    beyond the inputs is saved)."""

    @staticmethod
    def forward(ctx, Q, K, V, eta_tok, W1, W2, W3, chunk_tokens, sync="chain", norm=True, mma_bf16=False):
        r = amu_fwd(Q, K, V, eta_tok, W1, W2, W3, chunk_tokens, sync=sync, norm=norm, mma_bf16=mma_bf16,
                    want_final=False)
        ctx.chunk_tokens, ctx.sync, ctx.norm, ctx.mma_bf16 = chunk_tokens, sync, norm, mma_bf16
        ctx.save_for_backward(Q, K, V, eta_tok, W1, W2, W3)
        return r["O"]

    @staticmethod
    def backward(ctx, dO):
        Q, K, V, eta_tok, W1, W2, W3 = ctx.saved_tensors
        if dO.stride() != Q.stride() or dO.dtype != Q.dtype:
            dO = torch.empty_strided(Q.size(), Q.stride(), dtype=Q.dtype, device=Q.device).copy_(dO)
        g = amu_bwd(Q, K, V, eta_tok, W1, W2, W3, ctx.chunk_tokens, dO, sync=ctx.sync, norm=ctx.norm,
                    mma_bf16=ctx.mma_bf16)
        return (g["dQ"], g["dK"], g["dV"], g["deta_tok"], g["dW1_0"], g["dW2_0"], g["dW3_0"], None, None, None,
                None)


def amu_chunk(Q, K, V, eta_tok, W1, W2, W3, chunk_tokens, sync="chain", norm=True, mma_bf16=False):
    """Differentiable paper memory unit (see AMUChunk)."""
    return AMUChunk.apply(Q, K, V, eta_tok, W1, W2, W3, chunk_tokens, sync, norm, mma_bf16)
