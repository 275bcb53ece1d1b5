"""The HIP reverse mode against central finite differences of the HIP forward
itself, at the differentiation workload's shape (64-dim heads, hidden 256,
chunks of 4 frames = 5496 tokens) on a 2-chunk subset, FP32.  Outer
objective J = sum <O, dO>, accumulated in float64 on the host.  Each input
is perturbed along its own gradient direction u = g/|g|, where the
directional derivative is |g|; a gradient with a wrong direction, sign or
scale changes <g_true, u> by far more than the tolerance.  The steps are
sized for the FP32 forward: u is a unit vector over ~1.4M token elements
(65K weight elements), so a step of 1 (0.1 for the weights) moves each
element by ~1e-3 of its scale, where the FP32 rounding of J (~1e-5
absolute) is ~1e-4 of the smallest gradient (dK) and the O(step^2)
truncation is far below it.  (The step-1e-3 central differences on the same
subset pin the FP64 oracle, whose reverse mode the HIP path also matches.)"""
import pytest
import torch

from gpu_util import inputs
from workloads import WORKLOADS

pytestmark = pytest.mark.gpu

STEP = dict(Q=1.0, K=1.0, V=1.0, W1=0.1, W2=0.1)
ETA_STEP = 1e-3


def ops():
    from paper_2604_08542_amd import ops
    return ops


def test_backward_matches_fd_of_gpu_forward(gpu):
    w = WORKLOADS["layer16_32f_chunk4f_bwd"]
    M = w.chunk_tokens
    N, H, h, eta = 2 * M, 2, w.d_hidden, w.eta
    _, d = inputs(N, H, h, seed=0, io="f32", with_dO=True)
    base = dict(Q=d["Q"], K=d["K"], V=d["V"], W1=d["W1"], W2=d["W2"])
    dO = d["dO"].double()

    def J(eta_=eta, **repl):
        a = {k: repl.get(k, v) for k, v in base.items()}
        r = ops().chunk_fwd(a["Q"], a["K"], a["V"], a["W1"], a["W2"], eta_, M, want_final=False)
        torch.cuda.synchronize()
        return float((r["O"].double() * dO).sum())

    f = ops().chunk_fwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], eta, M, save_ckpt=True)
    g = ops().chunk_bwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], eta, M, f["ckpt"], d["dO"])
    torch.cuda.synchronize()
    grads = dict(Q=g["dQ"], K=g["dK"], V=g["dV"], W1=g["dW1_0"], W2=g["dW2_0"])
    for name, gt in grads.items():
        gn = float(gt.double().norm())
        u = (gt.double() / gn).float()
        t = STEP[name]
        fd = (J(**{name: base[name] + t * u}) - J(**{name: base[name] - t * u})) / (2 * t)
        print(f"{name}: |g| {gn:.6e}  fd {fd:.6e}  rel {abs(fd - gn) / gn:.2e}")
        assert abs(fd - gn) <= 2e-3 * gn, (name, fd, gn)
    de = float(g["deta"].double().sum())
    fde = (J(eta_=eta + ETA_STEP) - J(eta_=eta - ETA_STEP)) / (2 * ETA_STEP)
    print(f"eta: deta {de:.6e}  fd {fde:.6e}")
    assert abs(fde - de) <= 2e-3 * max(abs(de), 1.0), (fde, de)
