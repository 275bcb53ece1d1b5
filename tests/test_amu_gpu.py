"""The paper's adaptive memory unit on the GPU (SwiGLU fast network,
dot-product inner loss, token-wise step sizes; chain and synchronised forms)
against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle as orc
from gpu_util import TOL, host, inputs, rel
from workloads import WORKLOADS, make_eta_tok, make_inputs_torch

pytestmark = pytest.mark.gpu


def ops():
    from paper_2604_08542_amd import ops
    return ops


def w3_like(W1, seed):
    return (np.random.default_rng(seed).standard_normal(W1.shape) / np.sqrt(W1.shape[-2])).astype(np.float32)


def run_case(N, H, h, M, eta, io, sync, seed, mma=False):
    x, dev = inputs(N, H, h, seed=seed, io=io)
    W3 = w3_like(x["W1"], seed + 1)
    et = make_eta_tok(N, H, M, eta, seed)
    r = ops().amu_fwd(dev["Q"], dev["K"], dev["V"], torch.from_numpy(et).cuda(), dev["W1"], dev["W2"],
                      torch.from_numpy(W3).cuda(), M, sync=sync, mma_bf16=mma)
    torch.cuda.synchronize()
    ref = orc.ttt_forward_swiglu(x["Q"], x["K"], x["V"], x["W1"], x["W2"], W3, et, M, sync=sync)
    W0 = dict(W1_T=x["W1"], W2_T=x["W2"], W3_T=W3)
    errs = {"O": rel(host(r["O"]), ref["O"])}
    for k in ("W1_T", "W2_T", "W3_T"):
        errs["d" + k] = rel(host(r[k]) - W0[k], ref[k] - W0[k])
    return errs, r, ref


# The unit's loss is a plain sum with the step sizes inside, so the size of
# an update is set by eta_i alone; these cases take eta_i ~ 20 / M, which
# moves W by ~1% over the chain.  (At eta_i ~ 0.3 / M the change of W is
# ~1e-4 of W, and merely storing the exact W_T in FP32 already perturbs
# W_T - W_0 by ~2.5e-4 relative, above the FP32 gate.)
AMU_ETA = 20.0
CASES = [
    (1100, 2, 256, 400, 20.0, "f32", "chain"),
    (700, 2, 128, 256, 20.0, "f32", "gcs"),
    (96, 1, 128, 40, 20.0, "f32", "chain"),
    (1000, 2, 256, 333, 20.0, "bf16", "chain"),
    (2748, 1, 128, 1374, 20.0, "bf16", "gcs"),
    (1100, 2, 256, 400, 20.0, "f32", "gcs"),
    (1000, 2, 256, 500, 20.0, "bf16", "gcs"),
]


@pytest.mark.parametrize("N,H,h,M,eta,io,sync", CASES)
def test_amu_matches_oracle(gpu, N, H, h, M, eta, io, sync):
    errs, _, _ = run_case(N, H, h, M, eta, io, sync, seed=700 + N)
    print(f"amu N={N} H={H} h={h} M={M} {io} {sync}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= TOL[io], (k, v)


@pytest.mark.parametrize("sync", ["chain", "gcs"])
def test_amu_bf16_operands_f32_tokens(gpu, sync):
    # FP32 token tensors with BF16 matrix-core operands (FP32 accumulation)
    errs, _, _ = run_case(1000, 2, 256, 333, AMU_ETA, "f32", sync, seed=901, mma=True)
    print(f"amu f32 io, bf16 operands, {sync}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= TOL["bf16"], (k, v)


def test_amu_one_chunk_chain_equals_gcs(gpu):
    x, dev = inputs(500, 2, 128, seed=720, io="f32")
    W3 = torch.from_numpy(w3_like(x["W1"], 721)).cuda()
    et = torch.from_numpy(make_eta_tok(500, 2, 500, 20.0, 720)).cuda()
    a = ops().amu_fwd(dev["Q"], dev["K"], dev["V"], et, dev["W1"], dev["W2"], W3, 500, sync="chain")
    b = ops().amu_fwd(dev["Q"], dev["K"], dev["V"], et, dev["W1"], dev["W2"], W3, 500, sync="gcs")
    torch.cuda.synchronize()
    assert rel(host(a["O"]), host(b["O"])) <= 1e-6
    assert rel(host(a["W3_T"]), host(b["W3_T"])) <= 1e-6


def test_amu_zero_step_is_plain_swiglu(gpu):
    """eta_i = 0: no update, O = f_W0(Q) exactly as the oracle's SwiGLU map."""
    x, dev = inputs(300, 2, 256, seed=730, io="f32")
    W3 = w3_like(x["W1"], 731)
    et = np.zeros((300, 2), np.float32)
    r = ops().amu_fwd(dev["Q"], dev["K"], dev["V"], torch.from_numpy(et).cuda(), dev["W1"], dev["W2"],
                      torch.from_numpy(W3).cuda(), 128)
    torch.cuda.synchronize()
    assert torch.equal(r["W1_T"], dev["W1"]) and torch.equal(r["W3_T"], torch.from_numpy(W3).cuda())
    for hd in range(2):
        q = orc.l2norm_rows(x["Q"][:, hd].astype(np.float64))[0]
        ref = orc.swiglu_forward(q, x["W1"][hd], x["W2"][hd], W3[hd])
        assert rel(host(r["O"][:, hd]), ref) <= TOL["f32"]


@pytest.mark.parametrize("sync", ["chain", "gcs"])
def test_amu_full_layer(gpu, sync):
    """16 heads x 64, h 256, 87,936 tokens, chunks of 10,992 (the layer
    workload), BF16: two heads recomputed by the oracle."""
    w = WORKLOADS["layer16_64f_chunk8f"]
    dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype="bf16")
    g = torch.Generator(device="cuda"); g.manual_seed(1)
    W3 = torch.randn(dev["W1"].shape, generator=g, device="cuda") / float(np.sqrt(w.d_head))
    et = torch.from_numpy(make_eta_tok(w.n_tokens, w.n_heads, w.chunk_tokens, AMU_ETA, 0)).cuda()
    r = ops().amu_fwd(dev["Q"], dev["K"], dev["V"], et, dev["W1"], dev["W2"], W3, w.chunk_tokens, sync=sync)
    torch.cuda.synchronize()
    heads = [0, 11]
    x = {k: dev[k][:, heads].double().cpu().numpy() for k in ("Q", "K", "V")}
    W1 = dev["W1"][heads].cpu().numpy(); W2 = dev["W2"][heads].cpu().numpy(); W3h = W3[heads].cpu().numpy()
    ref = orc.ttt_forward_swiglu(x["Q"], x["K"], x["V"], W1, W2, W3h, et[:, heads].cpu().numpy(), w.chunk_tokens,
                                 sync=sync)
    errs = dict(O=rel(r["O"][:, heads].double().cpu().numpy(), ref["O"]),
                dW2=rel(r["W2_T"][heads].cpu().numpy() - W2, ref["W2_T"] - W2),
                dW3=rel(r["W3_T"][heads].cpu().numpy() - W3h, ref["W3_T"] - W3h))
    print(f"amu full layer {sync}:", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= TOL["bf16"], (k, v)
