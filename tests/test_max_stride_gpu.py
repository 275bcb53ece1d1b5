"""GPU parity at the largest token stride the ABI accepts (2^22 elements:
a 32-token tile then spans just under 2^31 bytes, the reach of the 32-bit
tile offsets).  Token tensors are views into one buffer of that row pitch,
as slices of a wide fused projection would be."""
import pytest
import torch

import oracle as orc
from gpu_util import TOL, host, inputs, rel

pytestmark = pytest.mark.gpu

STRIDE = 1 << 22


def ops():
    from paper_2604_08542_amd import ops
    return ops


def wide_views(x, names, io):
    """[N][H][d] views with token stride STRIDE into one zero buffer."""
    N, H, d = x[names[0]].shape
    dt = torch.float32 if io == "f32" else torch.bfloat16
    big = torch.zeros((N, STRIDE), dtype=dt, device="cuda")
    out = []
    for i, n in enumerate(names):
        v = big[:, i * H * d:(i + 1) * H * d].view(N, H, d)
        v.copy_(torch.from_numpy(x[n]).to(dt))
        out.append(v)
    return big, out


@pytest.mark.parametrize("N,H,h,M,eta,io", [(40, 2, 128, 16, 0.1, "f32"), (40, 2, 256, 16, 0.05, "bf16")])
def test_forward_max_stride(gpu, N, H, h, M, eta, io):
    x, d = inputs(N, H, h, seed=17 + N, io=io)
    big, (Q, K, V) = wide_views(x, ("Q", "K", "V"), io)
    assert Q.stride(0) == STRIDE
    r = ops().chunk_fwd(Q, K, V, d["W1"], d["W2"], eta, M, mma_bf16=io == "bf16")
    torch.cuda.synchronize()
    assert r["O"].stride(0) == STRIDE
    ref = orc.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], eta, M)
    errs = dict(O=rel(host(r["O"]), ref["O"]), W1_T=rel(host(r["W1_T"]), ref["W1_T"]))
    print(f"stride 2^22 N={N} H={H} h={h} M={M} io={io}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= TOL[io], (k, v)
    del big


def test_backward_max_stride(gpu):
    N, H, h, M, eta = 40, 2, 128, 16, 0.1
    x, d = inputs(N, H, h, seed=23, io="f32", with_dO=True)
    big, (Q, K, V, dO) = wide_views(x, ("Q", "K", "V", "dO"), "f32")
    f = ops().chunk_fwd(Q, K, V, d["W1"], d["W2"], eta, M, save_ckpt=True)
    g = ops().chunk_bwd(Q, K, V, d["W1"], d["W2"], eta, M, f["ckpt"], dO)
    torch.cuda.synchronize()
    assert g["dQ"].stride(0) == STRIDE
    ref = orc.ttt_backward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], eta, M, x["dO"])
    errs = {k: rel(host(g[k]), ref[k]) for k in ("dQ", "dK", "dV", "dW1_0", "dW2_0", "deta")}
    print("stride 2^22 backward: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= TOL["f32"], (k, v)
    del big
