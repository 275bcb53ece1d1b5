"""Seeded synthetic inputs shaped like VGGT token streams.

This module only draws random numbers and rounds them to the storage dtype.
It holds none of the method's arithmetic, so both the FP64 oracle's tests and
the HIP path's tests and benchmark can use it.

Recipe (stands in for VGGT features of real video frames, which are not
available here): a frame is 37*37 patch tokens + 5 special tokens = 1374
tokens; per head the raw Q, K, V ~ N(0, 1) i.i.d. with layout [N][H][d]
(d contiguous); W1 ~ N(0, 1/d) [H][d][h]; W2 ~ N(0, 1/h) [H][h][d];
dO ~ N(0, 1) [N][H][d].  Draw order Q, K, V, W1, W2, dO from one PCG64
stream seeded with `seed`.  Q, K, V (and dO) are rounded to the storage dtype
(round-to-nearest-even); the fast weights stay float32.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

TOKENS_PER_FRAME = 37 * 37 + 5  # 1374


@dataclass(frozen=True)
class Workload:
    name: str
    n_heads: int
    d_head: int
    d_hidden: int
    frames: tuple            # frames per sequence (one entry per sequence)
    chunk_frames: int
    eta: float
    io_dtype: str            # "f32" or "bf16"
    description: str = ""

    @property
    def chunk_tokens(self) -> int:
        return self.chunk_frames * TOKENS_PER_FRAME

    @property
    def seq_tokens(self) -> List[int]:
        return [f * TOKENS_PER_FRAME for f in self.frames]

    @property
    def n_tokens(self) -> int:
        return sum(self.seq_tokens)

    def cu_seqlens(self) -> List[int]:
        cu = [0]
        for n in self.seq_tokens:
            cu.append(cu[-1] + n)
        return cu


WORKLOADS = {
    "single_head_4x1374": Workload(
        "single_head_4x1374", 1, 64, 128, (4,), 1, 0.1, "f32",
        "1 head x 64, hidden 128, 4 chunks of one 1374-token frame, eta 0.1, FP32"),
    "layer16_64f_chunk8f": Workload(
        "layer16_64f_chunk8f", 16, 64, 256, (64,), 8, 0.05, "f32",
        "16 heads x 64, hidden 256, 64 frames, chunk 8 frames (10992 tokens), eta 0.05"),
    "single_head_256x1374_bf16": Workload(
        "single_head_256x1374_bf16", 1, 64, 128, (256,), 1, 0.1, "bf16",
        "1 head x 64, hidden 128, 256 chunks of one frame, BF16 operands"),
    "layer16_32f_chunk4f_bwd": Workload(
        "layer16_32f_chunk4f_bwd", 16, 64, 256, (32,), 4, 0.05, "f32",
        "16 heads x 64, hidden 256, 32 frames, chunk 4 frames, forward+backward"),
    "paper_state_64f_chunk8f_bf16": Workload(
        "paper_state_64f_chunk8f_bf16", 1, 1024, 4096, (64,), 8, 0.5, "bf16",
        "the paper's state: 1 head x 1024, hidden 4096, 64 frames, chunk 8 frames, BF16 operands"),
    "batch8_uneven_chunk8f_bf16": Workload(
        "batch8_uneven_chunk8f_bf16", 16, 64, 256, (12, 24, 40, 64, 96, 128, 200, 300), 8, 0.05, "bf16",
        "8 sequences of uneven frame counts, 16 heads x 64, hidden 256, chunk 8 frames"),
}


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (via float32, round-to-nearest-even); returns float32
    values that are exactly representable in bfloat16."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    return np.where(nan, np.float32(np.nan), out)


def round_io(x: np.ndarray, io_dtype: str) -> np.ndarray:
    if io_dtype == "f32":
        return np.asarray(x, dtype=np.float32)
    if io_dtype == "bf16":
        return round_bf16(x)
    raise ValueError(io_dtype)


def make_inputs(n_tokens: int, n_heads: int, d: int, h: int, seed: int = 0,
                io_dtype: str = "f32", with_dO: bool = False, n_w0: int = 1):
    """Draw raw (Q, K, V, W1, W2[, dO]) as float32 numpy arrays whose values
    are exactly representable in `io_dtype` (W1/W2 always float32).
    n_w0 > 1 draws that many independent initial-weight sets ([n_w0][H]...)."""
    rng = np.random.default_rng(seed)
    shape = (n_tokens, n_heads, d)
    Q = round_io(rng.standard_normal(shape), io_dtype)
    K = round_io(rng.standard_normal(shape), io_dtype)
    V = round_io(rng.standard_normal(shape), io_dtype)
    wshape1 = (n_heads, d, h) if n_w0 == 1 else (n_w0, n_heads, d, h)
    wshape2 = (n_heads, h, d) if n_w0 == 1 else (n_w0, n_heads, h, d)
    W1 = (rng.standard_normal(wshape1) / np.sqrt(d)).astype(np.float32)
    W2 = (rng.standard_normal(wshape2) / np.sqrt(h)).astype(np.float32)
    out = dict(Q=Q, K=K, V=V, W1=W1, W2=W2)
    if with_dO:
        out["dO"] = round_io(rng.standard_normal(shape), io_dtype)
    return out


def make_inputs_torch(n_tokens: int, n_heads: int, d: int, h: int, seed: int = 0,
                      io_dtype: str = "f32", device="cuda", with_dO: bool = False):
    """Same recipe drawn with torch's generator directly in device memory (for
    sizes too large to draw on the host).  The stream differs from
    make_inputs; values for a slice can be copied back to the host for
    sampled checks."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    tdt = torch.float32 if io_dtype == "f32" else torch.bfloat16
    shape = (n_tokens, n_heads, d)
    out = {}
    for name in ("Q", "K", "V"):
        out[name] = torch.randn(shape, generator=g, device=device, dtype=torch.float32).to(tdt)
    out["W1"] = torch.randn((n_heads, d, h), generator=g, device=device) / float(np.sqrt(d))
    out["W2"] = torch.randn((n_heads, h, d), generator=g, device=device) / float(np.sqrt(h))
    if with_dO:
        out["dO"] = torch.randn(shape, generator=g, device=device, dtype=torch.float32).to(tdt)
    return out


def make_eta_tok(n_tokens: int, n_heads: int, chunk_tokens: int, eta: float, seed: int = 0):
    """Token-wise step sizes for the paper's memory unit, [N][H] float32:
    uniform in [0.5, 1.5] x eta / chunk_tokens (the unit's loss is a plain sum
    over the chunk, so this keeps a chunk's step comparable to a mean-loss
    step of size eta)."""
    rng = np.random.default_rng(seed + 7919)
    return (rng.uniform(0.5, 1.5, (n_tokens, n_heads)) * (eta / chunk_tokens)).astype(np.float32)


def make_layer_inputs(n_tokens: int, n_heads: int, d: int, h: int, seed: int = 0, io_dtype: str = "f32",
                      bias: bool = True):
    """Inputs of the layer around the memory unit (features D = n_heads * d):
    tokens X ~ N(0, 1) [N][D]; projections Wqkv ~ N(0, 1/D) [D][3D] and
    Wo ~ N(0, 4d/D) [D][D] (X and the projections exactly representable in
    `io_dtype`); biases ~ N(0, 0.02^2) float32 (None without `bias`); the gate
    alpha ~ U(0.5, 1.5) [D] float32; fast weights W1 ~ N(0, 1/d) [H][d][h],
    W2 ~ N(0, 1/h) [H][h][d] float32.  With these fast weights the unit's
    outputs have an rms of about 1/(2 sqrt(d)), so the scale of Wo makes the
    gated term alpha * (O Wo) of the same order as X."""
    rng = np.random.default_rng(seed + 104729)
    D = n_heads * d
    X = round_io(rng.standard_normal((n_tokens, D)), io_dtype)
    Wqkv = round_io(rng.standard_normal((D, 3 * D)) / np.sqrt(D), io_dtype)
    Wo = round_io(rng.standard_normal((D, D)) * np.sqrt(4.0 * d / D), io_dtype)
    bqkv = (0.02 * rng.standard_normal(3 * D)).astype(np.float32) if bias else None
    bo = (0.02 * rng.standard_normal(D)).astype(np.float32) if bias else None
    alpha = rng.uniform(0.5, 1.5, D).astype(np.float32)
    W1 = (rng.standard_normal((n_heads, d, h)) / np.sqrt(d)).astype(np.float32)
    W2 = (rng.standard_normal((n_heads, h, d)) / np.sqrt(h)).astype(np.float32)
    return dict(X=X, Wqkv=Wqkv, Wo=Wo, bqkv=bqkv, bo=bo, alpha=alpha, W1=W1, W2=W2)
