"""GPU parity of the backward (through every inner update, second-order terms
included) against the FP64 oracle's hand-derived reverse mode, through the C
ABI and the autograd wrapper.  FP32: normwise relative error <= 1e-4 per
gradient; BF16 operands: <= 2e-2."""
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
    (700, 2, 128, 256, 0.3, "f32", False),    # ragged last chunk (188 tokens)
    (1100, 2, 256, 500, 0.05, "f32", False),  # ragged, h=256
    (96, 1, 128, 40, 0.5, "f32", False),      # tiny chunks, ragged tiles
    (1000, 2, 256, 333, 0.05, "bf16", True),
    (800, 2, 128, 300, 0.1, "f32", True),
    (700, 2, 128, 256, 0.3, "bf16", True),    # ragged, h=128, bf16 io
    (96, 1, 256, 40, 0.5, "bf16", True),      # tiny chunks, ragged tiles, h=256
]


@pytest.mark.parametrize("N,H,h,M,eta,io,mma", CASES)
def test_backward_matches_oracle(gpu, N, H, h, M, eta, io, mma):
    x, d = inputs(N, H, h, seed=100 + N, io=io, with_dO=True)
    f = ops().chunk_fwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], eta, M, save_ckpt=True, mma_bf16=mma)
    g = ops().chunk_bwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], eta, M, f["ckpt"], d["dO"], mma_bf16=mma)
    torch.cuda.synchronize()
    ref = orc.ttt_backward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], eta, M, x["dO"])
    tol = TOL["bf16" if mma or io == "bf16" else "f32"]
    errs = {k: rel(host(g[k]), ref[k]) for k in ("dQ", "dK", "dV", "dW1_0", "dW2_0", "deta")}
    print(f"N={N} H={H} h={h} M={M} io={io} mma_bf16={mma}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= tol, (k, v)


def test_backward_eta_zero(gpu):
    """eta = 0: dK = dV = 0 and dQ, dW0 are the plain MLP's gradients."""
    x, d = inputs(500, 2, 128, seed=7, io="f32", with_dO=True)
    f = ops().chunk_fwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], 0.0, 200, save_ckpt=True)
    g = ops().chunk_bwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], 0.0, 200, f["ckpt"], d["dO"])
    ref = orc.ttt_backward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.0, 200, x["dO"])
    assert float(g["dK"].abs().max()) == 0.0 and float(g["dV"].abs().max()) == 0.0
    assert rel(host(g["dQ"]), ref["dQ"]) <= 1e-4
    assert rel(host(g["dW1_0"]), ref["dW1_0"]) <= 1e-4


def test_autograd_function(gpu):
    x, d = inputs(600, 2, 128, seed=8, io="f32", with_dO=True)
    t = {k: d[k].clone().requires_grad_() for k in ("Q", "K", "V", "W1", "W2")}
    eta = torch.tensor(0.2, device="cuda", requires_grad=True)
    O = ops().ttt_chunk(t["Q"], t["K"], t["V"], t["W1"], t["W2"], eta, 250)
    (O * d["dO"]).sum().backward()
    ref = orc.ttt_backward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.2, 250, x["dO"])
    for k, rk in dict(Q="dQ", K="dK", V="dV", W1="dW1_0", W2="dW2_0").items():
        assert rel(host(t[k].grad), ref[rk]) <= 1e-4, k
    assert abs(eta.grad.item() - ref["deta"].sum()) <= 1e-4 * max(1.0, abs(ref["deta"].sum()))


def test_backward_deterministic(gpu):
    x, d = inputs(900, 2, 256, seed=9, io="bf16", with_dO=True)
    f = ops().chunk_fwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], 0.05, 300, save_ckpt=True)
    a = ops().chunk_bwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], 0.05, 300, f["ckpt"], d["dO"])
    b = ops().chunk_bwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], 0.05, 300, f["ckpt"], d["dO"])
    for k in a:
        assert torch.equal(a[k], b[k]), k
