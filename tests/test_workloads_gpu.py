"""Parity at the workloads' full sizes, in the launch configuration the
benchmark uses: the whole problem runs on the GPU, and sampled heads /
sequences are recomputed by the FP64 oracle one by one."""
import numpy as np
import pytest
import torch

import oracle as orc
from gpu_util import TOL, rel
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
    r = ops().batched_fwd(dev["Q"], dev["K"], dev["V"], w.cu_seqlens(), dev["W1"], dev["W2"], w.eta, w.chunk_tokens)
    torch.cuda.synchronize()
    heads = [0, w.n_heads - 1]
    x = host_heads(dev, heads)
    W1 = dev["W1"][heads].cpu().numpy(); W2 = dev["W2"][heads].cpu().numpy()
    ref = orc.ttt_forward(x["Q"], x["K"], x["V"], W1, W2, w.eta, w.chunk_tokens)
    O = r["O"][:, heads].double().cpu().numpy()
    e_o = rel(O, ref["O"])
    e_w = rel(r["W2_T"][0][heads].cpu().numpy(), ref["W2_T"])
    e_dw = rel(r["W1_T"][0][heads].cpu().numpy() - W1, ref["W1_T"] - W1)
    print(f"{name} {io}: O {e_o:.2e} W2_T {e_w:.2e} dW1 {e_dw:.2e}")
    tol = TOL[io]
    assert e_o <= tol and e_w <= tol and e_dw <= tol


def test_precision_form_long_chain(gpu):
    """256 chunks of one frame, BF16 operands: error vs FP64 per output."""
    w = WORKLOADS["single_head_256x1374_bf16"]
    dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype="bf16")
    r = ops().chunk_fwd(dev["Q"], dev["K"], dev["V"], dev["W1"], dev["W2"], w.eta, w.chunk_tokens, emit_loss=True)
    torch.cuda.synchronize()
    x = host_heads(dev, [0])
    W1 = dev["W1"].cpu().numpy(); W2 = dev["W2"].cpu().numpy()
    ref = orc.ttt_forward(x["Q"], x["K"], x["V"], W1, W2, w.eta, w.chunk_tokens)
    errs = dict(O=rel(r["O"].double().cpu().numpy(), ref["O"]),
                W1_T=rel(r["W1_T"].cpu().numpy(), ref["W1_T"]),
                dW2=rel(r["W2_T"].cpu().numpy() - W2, ref["W2_T"] - W2),
                loss=rel(r["loss"].cpu().numpy(), ref["loss"]))
    print("precision form:", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= TOL["bf16"], (k, v)


def test_batching_form_full_size(gpu):
    """8 uneven sequences (12..300 frames) x 16 heads in one schedule; the
    shortest and the longest sequence are checked for sampled heads."""
    w = WORKLOADS["batch8_uneven_chunk8f_bf16"]
    dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype="bf16")
    cu = w.cu_seqlens()
    r = ops().batched_fwd(dev["Q"], dev["K"], dev["V"], cu, dev["W1"], dev["W2"], w.eta, w.chunk_tokens)
    torch.cuda.synchronize()
    for b, heads in ((0, [3]), (7, [0, 15])):
        sl = slice(cu[b], cu[b + 1])
        x = host_heads(dev, heads, sl)
        W1 = dev["W1"][heads].cpu().numpy(); W2 = dev["W2"][heads].cpu().numpy()
        ref = orc.ttt_forward(x["Q"], x["K"], x["V"], W1, W2, w.eta, w.chunk_tokens)
        e_o = rel(r["O"][sl][:, heads].double().cpu().numpy(), ref["O"])
        e_dw = rel(r["W2_T"][b][heads].cpu().numpy() - W2, ref["W2_T"] - W2)
        print(f"batching seq {b} heads {heads}: O {e_o:.2e} dW2 {e_dw:.2e}")
        assert e_o <= TOL["bf16"] and e_dw <= TOL["bf16"]


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
