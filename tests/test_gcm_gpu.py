"""GPU parity of the layer around the memory unit (Sec. 4.2 projections and
memory unit, Sec. 4.1 Eq. 5 gate) against the FP64 oracle, through the C
ABI: the 16-head layer shape (d = 64, h = 256) and the paper's state (one
head of 1024 with hidden 4096), FP32 and BF16 token paths."""
import numpy as np
import pytest
import torch

import oracle as orc
from gpu_util import TOL, check, host, rel, storage_floor
from workloads import make_layer_inputs

pytestmark = pytest.mark.gpu


def ops():
    from paper_2604_08542_amd import ops
    return ops


def dev_inputs(x, io):
    dt = torch.float32 if io == "f32" else torch.bfloat16
    out = {}
    for k, v in x.items():
        if v is None:
            out[k] = None
        elif k in ("X", "Wqkv", "Wo"):
            out[k] = torch.from_numpy(v).cuda().to(dt)
        else:
            out[k] = torch.from_numpy(v).cuda()
    return out


def run(x, io, eta, M, **kw):
    g = dev_inputs(x, io)
    r = ops().gcm_fwd(g["X"], g["Wqkv"], g["Wo"], g["alpha"], g["W1"], g["W2"], eta, M, bqkv=g["bqkv"], bo=g["bo"],
                      **kw)
    torch.cuda.synchronize()
    return r


@pytest.mark.parametrize("N,H,d,h,M,eta,io,bias", [
    (2500, 16, 64, 256, 600, 0.05, "f32", True),
    (2500, 16, 64, 256, 600, 0.05, "bf16", True),
    (1374 * 2, 1, 1024, 4096, 1374, 0.05, "f32", False),
    (1374 * 2, 1, 1024, 4096, 1374, 0.05, "bf16", True),
])
def test_layer_matches_oracle(gpu, N, H, d, h, M, eta, io, bias):
    x = make_layer_inputs(N, H, d, h, seed=N + H + int(bias), io_dtype=io, bias=bias)
    r = run(x, io, eta, M)
    ref = orc.gcm_layer_forward(x["X"], x["Wqkv"], x["Wo"], x["alpha"], x["W1"], x["W2"], eta, M, bqkv=x["bqkv"],
                                bo=x["bo"])
    X = x["X"].astype(np.float64)
    Y = host(r["Y"])
    tol = TOL[io]
    print(f"gcm layer N={N} H={H} d={d} h={h} {io}:")
    check("Y", Y, ref["Y"], tol)
    check("gated part Y - X", Y - X, ref["Y"] - X, tol)
    check("W1_T", host(r["W1_T"]), ref["W1_T"], tol)
    # each of the chain's C updates rounds the weights to FP32, so the
    # change W_T - W_0 carries up to C times the storage floor of W_T
    C = -(-N // M)
    check("dW1", host(r["W1_T"]) - x["W1"], ref["W1_T"] - x["W1"], tol,
          floor=C * storage_floor(ref["W1_T"], x["W1"]))
    check("dW2", host(r["W2_T"]) - x["W2"], ref["W2_T"] - x["W2"], tol,
          floor=C * storage_floor(ref["W2_T"], x["W2"]))


def test_layer_update_reaches_the_output(gpu):
    """FP32: the memory unit's update changes Y, and that change matches the
    oracle's (Y(eta) - Y(0) gated on its own)."""
    N, H, d, h, M = 1500, 16, 64, 256, 500
    x = make_layer_inputs(N, H, d, h, seed=7, io_dtype="f32")
    y1, y0 = host(run(x, "f32", 0.1, M)["Y"]), host(run(x, "f32", 0.0, M)["Y"])
    r1 = orc.gcm_layer_forward(x["X"], x["Wqkv"], x["Wo"], x["alpha"], x["W1"], x["W2"], 0.1, M, bqkv=x["bqkv"],
                               bo=x["bo"])["Y"]
    r0 = orc.gcm_layer_forward(x["X"], x["Wqkv"], x["Wo"], x["alpha"], x["W1"], x["W2"], 0.0, M, bqkv=x["bqkv"],
                               bo=x["bo"])["Y"]
    e = rel(y1 - y0, r1 - r0)
    print(f"gcm layer delta-Y rel {e:.2e}, |dY|/|Y| {np.linalg.norm(r1 - r0) / np.linalg.norm(r1):.2e}")
    assert e <= 1e-3


def test_layer_empty_and_validation(gpu):
    x = make_layer_inputs(0, 16, 64, 256, seed=1)
    r = run(x, "f32", 0.05, 100)
    assert r["Y"].shape == (0, 1024)
    assert torch.equal(r["W1_T"].cpu(), torch.from_numpy(x["W1"]))
    from paper_2604_08542_amd import _lib as L
    x = make_layer_inputs(10, 1, 64, 128, seed=1)  # D = 64: not a multiple of 128
    with pytest.raises(L.TTTError):
        run(x, "f32", 0.05, 100)


@pytest.mark.parametrize("N,H,d,h,M,eta,io,bias", [
    (2500, 16, 64, 256, 600, 0.05, "f32", True),
    (2500, 16, 64, 256, 600, 0.05, "bf16", True),
    (1374 * 2, 1, 1024, 4096, 1374, 0.05, "bf16", False),
])
def test_layer_backward_matches_oracle(gpu, N, H, d, h, M, eta, io, bias):
    # reverse mode of the whole layer for <Y, dY>: gate, output projection,
    # the unit's reverse mode, query-key-value projection
    x = make_layer_inputs(N, H, d, h, seed=N + H + 3, io_dtype=io, bias=bias)
    dY = np.random.default_rng(N + 7).standard_normal((N, H * d)).astype(np.float32)
    if io == "bf16":
        dY = torch.from_numpy(dY).to(torch.bfloat16).float().numpy()
    g = dev_inputs(x, io)
    dYd = torch.from_numpy(dY).cuda().to(g["X"].dtype)
    r = ops().gcm_bwd(g["X"], g["Wqkv"], g["Wo"], g["alpha"], g["W1"], g["W2"], eta, M, dYd, bqkv=g["bqkv"],
                      bo=g["bo"])
    torch.cuda.synchronize()
    ref = orc.gcm_layer_backward(x["X"], x["Wqkv"], x["Wo"], x["alpha"], x["W1"], x["W2"], eta, M, dY, bqkv=x["bqkv"],
                                 bo=x["bo"])
    tol = TOL[io]
    print(f"gcm layer backward N={N} H={H} d={d} h={h} {io} bias={bias}:")
    keys = ["dX", "dWqkv", "dWo", "dalpha", "dW1_0", "dW2_0"] + (["dbqkv", "dbo"] if bias else [])
    for k in keys:
        check(k, host(r[k]), ref[k], tol)
    # dX - dY is the part that went through the layer (dY itself passes
    # straight through the residual)
    check("dX - dY", host(r["dX"]) - dY, ref["dX"] - dY, tol)
    e = rel(host(r["deta"]), ref["deta"])
    print(f"  deta rel {e:.2e}")
    assert e <= tol
    if not bias:
        assert r["dbqkv"] is None and r["dbo"] is None


def test_layer_backward_empty_stream(gpu):
    x = make_layer_inputs(0, 16, 64, 256, seed=1)
    g = dev_inputs(x, "f32")
    r = ops().gcm_bwd(g["X"], g["Wqkv"], g["Wo"], g["alpha"], g["W1"], g["W2"], 0.05, 100, torch.zeros_like(g["X"]),
                      bqkv=g["bqkv"], bo=g["bo"])
    torch.cuda.synchronize()
    for k in ("dWqkv", "dbqkv", "dWo", "dbo", "dalpha", "dW1_0", "dW2_0", "deta"):
        assert not torch.any(r[k]), k
