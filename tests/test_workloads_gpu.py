"""Parity at the workloads' full sizes, in the launch configuration the
benchmark uses: the whole problem runs on the GPU, and sampled heads /
sequences are recomputed by the FP64 oracle one by one."""
import numpy as np
import pytest
import torch

import oracle as orc
from gpu_util import TOL, apply_consistency, check, rel, storage_floor
from workloads import WORKLOADS, make_inputs_torch

pytestmark = pytest.mark.gpu


def ops():
    from paper_2604_08542_amd import ops
    return ops


def host_heads(dev, heads, sl=slice(None)):
    return {k: dev[k][sl][:, heads].double().cpu().numpy() for k in ("Q", "K", "V", "dO") if k in dev}


@pytest.mark.parametrize("name,io", [("layer16_64f_chunk8f", "f32"), ("layer16_64f_chunk8f", "bf16"),
                                     ("single_head_4x1374", "f32")])
def test_forward_full_size(gpu, name, io):
    w = WORKLOADS[name]
    dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype=io)
    r = ops().batched_fwd(dev["Q"], dev["K"], dev["V"], w.cu_seqlens(), dev["W1"], dev["W2"], w.eta, w.chunk_tokens,
                          save_ckpt=True)
    torch.cuda.synchronize()
    heads = [0, w.n_heads - 1]
    x = host_heads(dev, heads)
    W1 = dev["W1"][heads].cpu().numpy(); W2 = dev["W2"][heads].cpu().numpy()
    ref = orc.ttt_forward(x["Q"], x["K"], x["V"], W1, W2, w.eta, w.chunk_tokens)
    tol = TOL[io]
    print(f"{name} {io}, heads {heads}:")
    check("O", r["O"][:, heads].double().cpu().numpy(), ref["O"], tol)
    check("W2_T", r["W2_T"][0][heads].cpu().numpy(), ref["W2_T"], tol)
    check("dW1", r["W1_T"][0][heads].cpu().numpy() - W1, ref["W1_T"] - W1, tol, floor=storage_floor(ref["W1_T"], W1))
    check("dW2", r["W2_T"][0][heads].cpu().numpy() - W2, ref["W2_T"] - W2, tol, floor=storage_floor(ref["W2_T"], W2))
    # the apply of every chunk uses the updated weights (all heads)
    worst = apply_consistency(ops().chunk_fwd, dev["Q"], dev["K"], dev["V"], r["ckpt"], r["W1_T"][0], r["W2_T"][0],
                              r["O"], w.chunk_tokens, False)
    print(f"  apply with W_(c+1) vs chain O: worst chunk rel {worst:.2e}")
    assert worst <= 1e-6


def test_precision_form_long_chain(gpu):
    """256 chunks of one frame, BF16 operands: error vs FP64 per output."""
    w = WORKLOADS["single_head_256x1374_bf16"]
    dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype="bf16")
    r = ops().chunk_fwd(dev["Q"], dev["K"], dev["V"], dev["W1"], dev["W2"], w.eta, w.chunk_tokens, emit_loss=True,
                        save_ckpt=True)
    torch.cuda.synchronize()
    x = host_heads(dev, [0])
    W1 = dev["W1"].cpu().numpy(); W2 = dev["W2"].cpu().numpy()
    ref = orc.ttt_forward(x["Q"], x["K"], x["V"], W1, W2, w.eta, w.chunk_tokens)
    tol = TOL["bf16"]
    print("precision form, 256 chunks:")
    check("O", r["O"].double().cpu().numpy(), ref["O"], tol)
    check("W1_T", r["W1_T"].cpu().numpy(), ref["W1_T"], tol)
    check("dW1", r["W1_T"].cpu().numpy() - W1, ref["W1_T"] - W1, tol, floor=storage_floor(ref["W1_T"], W1))
    check("dW2", r["W2_T"].cpu().numpy() - W2, ref["W2_T"] - W2, tol, floor=storage_floor(ref["W2_T"], W2))
    check("loss", r["loss"].cpu().numpy(), ref["loss"], tol)
    worst = apply_consistency(ops().chunk_fwd, dev["Q"], dev["K"], dev["V"], r["ckpt"], r["W1_T"], r["W2_T"], r["O"],
                              w.chunk_tokens, False, chunks=[0, 1, 127, 254, 255])
    print(f"  apply with W_(c+1) vs chain O: worst chunk rel {worst:.2e}")
    assert worst <= 1e-6


def test_batching_form_full_size(gpu):
    """8 uneven sequences (12..300 frames) x 16 heads in one schedule; every
    sequence is checked against the oracle on one head (a different head
    per sequence), the longest also on a second head."""
    w = WORKLOADS["batch8_uneven_chunk8f_bf16"]
    dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype="bf16")
    cu = w.cu_seqlens()
    M = w.chunk_tokens
    r = ops().batched_fwd(dev["Q"], dev["K"], dev["V"], cu, dev["W1"], dev["W2"], w.eta, M, save_ckpt=True)
    torch.cuda.synchronize()
    tol = TOL["bf16"]
    _, rows = ops().batch_chunks(cu, M)
    for b in range(len(cu) - 1):
        heads = [(5 * b + 3) % w.n_heads] + ([0] if b == len(cu) - 2 else [])
        sl = slice(cu[b], cu[b + 1])
        x = host_heads(dev, heads, sl)
        W1 = dev["W1"][heads].cpu().numpy(); W2 = dev["W2"][heads].cpu().numpy()
        ref = orc.ttt_forward(x["Q"], x["K"], x["V"], W1, W2, w.eta, M)
        print(f"batching seq {b} ({cu[b + 1] - cu[b]} tokens) heads {heads}:")
        check("O", r["O"][sl][:, heads].double().cpu().numpy(), ref["O"], tol)
        check("dW1", r["W1_T"][b][heads].cpu().numpy() - W1, ref["W1_T"] - W1, tol)
        check("dW2", r["W2_T"][b][heads].cpu().numpy() - W2, ref["W2_T"] - W2, tol)
        # first, middle and last chunk: applied with the updated weights
        C = rows[b + 1] - rows[b]
        ck = r["ckpt"][rows[b]:rows[b + 1]]
        worst = apply_consistency(ops().chunk_fwd, dev["Q"][sl], dev["K"][sl], dev["V"][sl], ck, r["W1_T"][b],
                                  r["W2_T"][b], r["O"][sl], M, False, chunks=sorted({0, C // 2, C - 1}))
        print(f"  apply with W_(c+1) vs chain O: worst chunk rel {worst:.2e}")
        assert worst <= 1e-6


@pytest.mark.parametrize("io", ["f32", "bf16"])
def test_differentiation_form_full_size(gpu, io):
    """16 heads x 64, h 256, 32 frames, chunk 4 frames: the full backward on
    the GPU, two heads recomputed by the oracle's backward."""
    w = WORKLOADS["layer16_32f_chunk4f_bwd"]
    dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype=io, with_dO=True)
    f = ops().chunk_fwd(dev["Q"], dev["K"], dev["V"], dev["W1"], dev["W2"], w.eta, w.chunk_tokens, save_ckpt=True)
    g = ops().chunk_bwd(dev["Q"], dev["K"], dev["V"], dev["W1"], dev["W2"], w.eta, w.chunk_tokens, f["ckpt"], dev["dO"])
    torch.cuda.synchronize()
    heads = [0, 9]
    x = host_heads(dev, heads)
    W1 = dev["W1"][heads].cpu().numpy(); W2 = dev["W2"][heads].cpu().numpy()
    ref = orc.ttt_backward(x["Q"], x["K"], x["V"], W1, W2, w.eta, w.chunk_tokens, x["dO"])
    errs = {k: rel(g[k][:, heads].double().cpu().numpy() if k in ("dQ", "dK", "dV") else g[k][heads].cpu().numpy(),
                   ref[k]) for k in ("dQ", "dK", "dV", "dW1_0", "dW2_0", "deta")}
    print(f"differentiation {io}:", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= TOL[io], (k, v)
