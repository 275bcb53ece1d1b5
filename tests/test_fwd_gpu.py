"""GPU parity of the forward (chunk update + apply) against the FP64 oracle,
through the C ABI.  FP32 path: normwise relative error <= 1e-4 per output;
BF16 operands with FP32 accumulation: <= 2e-2."""
import numpy as np
import pytest
import torch

import oracle as orc
from gpu_util import TOL, host, inputs, rel

pytestmark = pytest.mark.gpu


def ops():
    from paper_2604_08542_amd import ops
    return ops


CASES = [
    # N, H, h, M, eta, io, mma_bf16
    (5496, 1, 128, 1374, 0.1, "f32", False),   # single head, 4 one-frame chunks
    (2500, 2, 256, 1000, 0.05, "f32", False),  # ragged last chunk, ragged tiles
    (700, 3, 128, 64, 0.3, "f32", False),      # many small chunks
    (1000, 2, 256, 333, 0.05, "bf16", True),
    (5496, 1, 128, 1374, 0.1, "bf16", True),
    (1500, 2, 256, 500, 0.05, "f32", True),    # f32 io, bf16 matrix-core operands
]


@pytest.mark.parametrize("N,H,h,M,eta,io,mma", CASES)
def test_forward_matches_oracle(gpu, N, H, h, M, eta, io, mma):
    x, d = inputs(N, H, h, seed=N + H, io=io)
    r = ops().chunk_fwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], eta, M, save_ckpt=True, emit_loss=True,
                        mma_bf16=mma)
    torch.cuda.synchronize()
    ref = orc.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], eta, M)
    tol = TOL["bf16" if mma or io == "bf16" else "f32"]
    errs = dict(
        O=rel(host(r["O"]), ref["O"]),
        W1_T=rel(host(r["W1_T"]), ref["W1_T"]),
        W2_T=rel(host(r["W2_T"]), ref["W2_T"]),
        dW1=rel(host(r["W1_T"]) - x["W1"], ref["W1_T"] - x["W1"]),
        dW2=rel(host(r["W2_T"]) - x["W2"], ref["W2_T"] - x["W2"]),
        loss=rel(host(r["loss"]), ref["loss"]),
        ckpt1=rel(host(r["ckpt"])[:, :, :64 * h].reshape(ref["ckpt1"].shape), ref["ckpt1"]),
    )
    print(f"N={N} H={H} h={h} M={M} io={io} mma_bf16={mma}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= tol, (k, v)
    if tol == TOL["f32"]:
        r0 = ops().chunk_fwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], 0.0, M)
        dO_gpu = host(r["O"]) - host(r0["O"])
        O0 = orc.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.0, M)["O"]
        e = rel(dO_gpu, ref["O"] - O0)
        print(f"  delta-O rel err {e:.2e}")
        assert e <= tol


def test_eta_zero_is_plain_mlp(gpu):
    x, d = inputs(1000, 2, 256, seed=3, io="f32")
    r = ops().chunk_fwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], 0.0, 300)
    ref = orc.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.0, 300)
    assert rel(host(r["O"]), ref["O"]) <= 1e-5
    assert torch.equal(r["W1_T"], d["W1"]) and torch.equal(r["W2_T"], d["W2"])


def test_deterministic(gpu):
    x, d = inputs(3000, 2, 256, seed=4, io="bf16")
    a = ops().chunk_fwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], 0.05, 1000)
    b = ops().chunk_fwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], 0.05, 1000)
    assert torch.equal(a["O"], b["O"]) and torch.equal(a["W1_T"], b["W1_T"])


@pytest.mark.parametrize("G", [1, 2, 5, 16])
def test_shard_count_invariance(gpu, G):
    """Token-shard additivity (Eq. 10) on the GPU: any number of work-groups
    per chain gives the same result up to rounding."""
    x, d = inputs(2000, 2, 128, seed=5, io="f32")
    r = ops().batched_fwd(d["Q"], d["K"], d["V"], [0, 2000], d["W1"], d["W2"], 0.1, 700,
                          tile_cfg=dict(wg_per_chain=G))
    ref = orc.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.1, 700)
    assert rel(host(r["O"]), ref["O"]) <= 1e-4
    assert rel(host(r["W1_T"][0]), ref["W1_T"]) <= 1e-4


def test_batched_equals_per_sequence(gpu):
    x, d = inputs(2600, 2, 256, seed=6, io="bf16")
    cu = [0, 300, 301, 1500, 1500, 2600]   # includes an empty and a 1-token sequence
    cfg = dict(wg_per_chain=3)
    r = ops().batched_fwd(d["Q"], d["K"], d["V"], cu, d["W1"], d["W2"], 0.05, 512, tile_cfg=cfg)
    for b in range(len(cu) - 1):
        s, e = cu[b], cu[b + 1]
        if e == s:
            continue
        rb = ops().batched_fwd(d["Q"][s:e], d["K"][s:e], d["V"][s:e], [0, e - s], d["W1"], d["W2"], 0.05, 512,
                               tile_cfg=cfg)
        assert torch.equal(r["O"][s:e], rb["O"]), b
        assert torch.equal(r["W1_T"][b], rb["W1_T"][0]), b
    ref = orc.ttt_forward_batched(x["Q"], x["K"], x["V"], cu, x["W1"], x["W2"], 0.05, 512)
    assert rel(host(r["O"]), ref["O"]) <= 2e-2


def test_per_sequence_initial_weights(gpu):
    from workloads import make_inputs
    x = make_inputs(900, 2, 64, 128, seed=7, n_w0=3)
    cu = [0, 200, 650, 900]
    d = {k: torch.from_numpy(v).cuda() for k, v in x.items()}
    r = ops().batched_fwd(d["Q"], d["K"], d["V"], cu, d["W1"], d["W2"], 0.1, 128, w0_per_seq=True)
    ref = orc.ttt_forward_batched(x["Q"], x["K"], x["V"], cu, x["W1"], x["W2"], 0.1, 128, w0_per_seq=True)
    assert rel(host(r["O"]), ref["O"]) <= 1e-4
    assert rel(host(r["W2_T"]), ref["W2_T"]) <= 1e-4


def test_strided_heads(gpu):
    """Q/K/V as views with padded token stride (e.g. slices of a fused QKV)."""
    x, _ = inputs(800, 2, 128, seed=8, io="f32")
    big = torch.zeros((800, 3, 2, 64), device="cuda")
    big[:, 0] = torch.from_numpy(x["Q"]).cuda()
    big[:, 1] = torch.from_numpy(x["K"]).cuda()
    big[:, 2] = torch.from_numpy(x["V"]).cuda()
    Q, K, V = big[:, 0], big[:, 1], big[:, 2]
    W1 = torch.from_numpy(x["W1"]).cuda(); W2 = torch.from_numpy(x["W2"]).cuda()
    r = ops().chunk_fwd(Q, K, V, W1, W2, 0.1, 256)
    ref = orc.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.1, 256)
    assert rel(host(r["O"]), ref["O"]) <= 1e-4
