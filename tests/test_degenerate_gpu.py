"""GPU parity against the FP64 oracle at the degenerate chunk sizes of the
chunk-wise update (Sec. 4.2): one token per chunk (every token its own update
unit, the token-wise limit of Eq. 8), chunks smaller than one 32-token tile
with a ragged last chunk, and a stream shorter than one chunk.  Forward,
reverse mode and the GCS form, FP32 (1e-4) and BF16 operands (2e-2)."""
import pytest
import torch

import oracle as orc
from gpu_util import TOL, host, inputs, rel

pytestmark = pytest.mark.gpu


def ops():
    from paper_2604_08542_amd import ops
    return ops


FWD_CASES = [
    # N, H, h, M, eta, io
    (40, 2, 128, 1, 0.05, "f32"),    # one token per chunk: 40 chunks
    (40, 2, 256, 1, 0.05, "bf16"),
    (50, 2, 256, 7, 0.1, "f32"),     # sub-tile chunks, last chunk of 1 token
    (50, 1, 128, 7, 0.1, "bf16"),
    (20, 3, 256, 1000, 0.1, "f32"),  # stream shorter than one chunk
    (20, 1, 128, 1000, 0.1, "bf16"),
]


@pytest.mark.parametrize("N,H,h,M,eta,io", FWD_CASES)
def test_forward_degenerate_chunks(gpu, N, H, h, M, eta, io):
    x, d = inputs(N, H, h, seed=7 * N + M, io=io)
    mma = io == "bf16"
    r = ops().chunk_fwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], eta, M, save_ckpt=True, emit_loss=True,
                        mma_bf16=mma)
    torch.cuda.synchronize()
    ref = orc.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], eta, M)
    tol = TOL[io]
    errs = dict(O=rel(host(r["O"]), ref["O"]), W1_T=rel(host(r["W1_T"]), ref["W1_T"]),
                W2_T=rel(host(r["W2_T"]), ref["W2_T"]), loss=rel(host(r["loss"]), ref["loss"]),
                dW1=rel(host(r["W1_T"]) - x["W1"], ref["W1_T"] - x["W1"]))
    print(f"N={N} H={H} h={h} M={M} io={io}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    assert host(r["loss"]).shape == (H, -(-N // M))
    for k, v in errs.items():
        assert v <= tol, (k, v)


BWD_CASES = [
    (24, 2, 128, 1, 0.05, "f32"),
    (30, 1, 256, 7, 0.1, "f32"),
    (24, 2, 256, 1, 0.05, "bf16"),
    (20, 2, 128, 1000, 0.1, "bf16"),
]


@pytest.mark.parametrize("N,H,h,M,eta,io", BWD_CASES)
def test_backward_degenerate_chunks(gpu, N, H, h, M, eta, io):
    x, d = inputs(N, H, h, seed=11 * N + M, io=io, with_dO=True)
    mma = io == "bf16"
    f = ops().chunk_fwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], eta, M, save_ckpt=True, mma_bf16=mma)
    g = ops().chunk_bwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], eta, M, f["ckpt"], d["dO"], mma_bf16=mma)
    torch.cuda.synchronize()
    ref = orc.ttt_backward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], eta, M, x["dO"])
    errs = {k: rel(host(g[k]), ref[k]) for k in ("dQ", "dK", "dV", "dW1_0", "dW2_0", "deta")}
    print(f"N={N} H={H} h={h} M={M} io={io}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= TOL[io], (k, v)


@pytest.mark.parametrize("N,H,h,M,eta,io", [(30, 2, 128, 1, 0.02, "f32"), (50, 2, 256, 7, 0.05, "f32"),
                                            (50, 1, 256, 7, 0.05, "bf16")])
def test_gcs_degenerate_chunks(gpu, N, H, h, M, eta, io):
    x, d = inputs(N, H, h, seed=13 * N + M, io=io)
    r = ops().gcs_fwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], eta, M, mma_bf16=io == "bf16")
    torch.cuda.synchronize()
    ref = orc.ttt_forward_gcs(x["Q"], x["K"], x["V"], x["W1"], x["W2"], eta, M)
    errs = dict(O=rel(host(r["O"]), ref["O"]), W1_T=rel(host(r["W1_T"]), ref["W1_T"]),
                W2_T=rel(host(r["W2_T"]), ref["W2_T"]))
    print(f"GCS N={N} H={H} h={h} M={M} io={io}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= TOL[io], (k, v)
