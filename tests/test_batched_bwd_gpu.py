"""Batched backward (packed sequences of uneven length, one reverse schedule
aligned at each sequence's last chunk) against the FP64 oracle, and at full
size against the single-sequence backward of each sequence."""
import numpy as np
import pytest
import torch

import oracle as orc
from gpu_util import TOL, host, inputs, rel
from workloads import WORKLOADS, make_inputs_torch

pytestmark = pytest.mark.gpu


def ops():
    from paper_2604_08542_amd import ops
    return ops


def per_seq_w0(x, dev, B, seed):
    rng = np.random.default_rng(seed)
    W1 = np.stack([x["W1"] * (1.0 + 0.2 * rng.standard_normal()) for _ in range(B)]).astype(np.float32)
    W2 = np.stack([x["W2"] * (1.0 + 0.2 * rng.standard_normal()) for _ in range(B)]).astype(np.float32)
    x = dict(x, W1=W1, W2=W2)
    dev = dict(dev, W1=torch.from_numpy(W1).cuda(), W2=torch.from_numpy(W2).cuda())
    return x, dev


CASES = [
    # lengths, H, h, M, eta, io, w0_per_seq
    ([300, 0, 700, 130], 2, 128, 256, 0.3, "f32", False),
    ([520, 90, 333], 2, 256, 200, 0.05, "f32", True),
    ([400, 1000, 65], 2, 256, 333, 0.05, "bf16", False),
    ([700, 0, 256], 1, 128, 256, 0.1, "bf16", True),
]


@pytest.mark.parametrize("lens,H,h,M,eta,io,w0ps", CASES)
def test_batched_backward_matches_oracle(gpu, lens, H, h, M, eta, io, w0ps):
    cu = np.concatenate([[0], np.cumsum(lens)]).tolist()
    x, dev = inputs(cu[-1], H, h, seed=500 + cu[-1], io=io, with_dO=True)
    if w0ps:
        x, dev = per_seq_w0(x, dev, len(lens), 501)
    f = ops().batched_fwd(dev["Q"], dev["K"], dev["V"], cu, dev["W1"], dev["W2"], eta, M, w0_per_seq=w0ps,
                          save_ckpt=True, want_final=False)
    g = ops().batched_bwd(dev["Q"], dev["K"], dev["V"], cu, dev["W1"], dev["W2"], eta, M, f["ckpt"], dev["dO"],
                          w0_per_seq=w0ps)
    torch.cuda.synchronize()
    ref = orc.ttt_backward_batched(x["Q"], x["K"], x["V"], cu, x["W1"], x["W2"], eta, M, x["dO"], w0_per_seq=w0ps)
    errs = {k: rel(host(g[k]), ref[k]) for k in ("dQ", "dK", "dV", "dW1_0", "dW2_0", "deta")}
    print(f"batched bwd lens={lens} H={H} h={h} M={M} {io} w0_per_seq={w0ps}: " +
          " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= TOL[io], (k, v)
    if w0ps and 0 in lens:
        b = lens.index(0)
        assert not torch.any(g["dW1_0"][b]) and not torch.any(g["dW2_0"][b])


def test_batched_checkpoints_match_single_sequence(gpu):
    """Checkpoint rows of sequence b in the batched layout equal those of the
    single-sequence forward of b."""
    lens, H, h, M, eta = [300, 0, 700], 2, 128, 256, 0.2
    cu = np.concatenate([[0], np.cumsum(lens)]).tolist()
    _, dev = inputs(cu[-1], H, h, seed=510, io="f32")
    f = ops().batched_fwd(dev["Q"], dev["K"], dev["V"], cu, dev["W1"], dev["W2"], eta, M, save_ckpt=True)
    _, rows = ops().batch_chunks(cu, M)
    for b in (0, 2):
        sl = slice(cu[b], cu[b + 1])
        s = ops().chunk_fwd(dev["Q"][sl], dev["K"][sl], dev["V"][sl], dev["W1"], dev["W2"], eta, M, save_ckpt=True)
        torch.cuda.synchronize()
        assert rel(host(f["ckpt"][rows[b]:rows[b + 1]]), host(s["ckpt"])) <= 1e-6


def test_batching_form_backward_full_size(gpu):
    """8 uneven sequences (12..300 frames) x 16 heads, BF16: the batched
    backward equals each sequence's own chunk backward (shard counts differ,
    so only rounding order differs), and the summed d(eta) matches."""
    w = WORKLOADS["batch8_uneven_chunk8f_bf16"]
    dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype="bf16", with_dO=True)
    cu = w.cu_seqlens()
    f = ops().batched_fwd(dev["Q"], dev["K"], dev["V"], cu, dev["W1"], dev["W2"], w.eta, w.chunk_tokens,
                          save_ckpt=True, want_final=False)
    g = ops().batched_bwd(dev["Q"], dev["K"], dev["V"], cu, dev["W1"], dev["W2"], w.eta, w.chunk_tokens, f["ckpt"],
                          dev["dO"])
    torch.cuda.synchronize()
    _, rows = ops().batch_chunks(cu, w.chunk_tokens)
    deta = torch.zeros_like(g["deta"])
    dW1 = torch.zeros_like(g["dW1_0"])
    for b in range(len(cu) - 1):
        sl = slice(cu[b], cu[b + 1])
        s = ops().chunk_bwd(dev["Q"][sl], dev["K"][sl], dev["V"][sl], dev["W1"], dev["W2"], w.eta, w.chunk_tokens,
                            f["ckpt"][rows[b]:rows[b + 1]], dev["dO"][sl])
        torch.cuda.synchronize()
        for k in ("dQ", "dK", "dV"):
            e = rel(host(g[k][sl]), host(s[k]))
            assert e <= 1e-2, (b, k, e)
        deta += s["deta"]
        dW1 += s["dW1_0"]
    e_eta = rel(host(g["deta"]), host(deta))
    e_w = rel(host(g["dW1_0"]), host(dW1))
    print(f"batching-form backward: deta {e_eta:.2e} dW1 {e_w:.2e}")
    assert e_eta <= 1e-3 and e_w <= 1e-3
    # sampled oracle check: shortest sequence, one head
    b, heads = 0, [5]
    sl = slice(cu[b], cu[b + 1])
    x = {k: dev[k][sl][:, heads].double().cpu().numpy() for k in ("Q", "K", "V", "dO")}
    W1 = dev["W1"][heads].cpu().numpy(); W2 = dev["W2"][heads].cpu().numpy()
    ref = orc.ttt_backward(x["Q"], x["K"], x["V"], W1, W2, w.eta, w.chunk_tokens, x["dO"])
    for k in ("dQ", "dK", "dV"):
        e = rel(g[k][sl][:, heads].double().cpu().numpy(), ref[k])
        print(f"batching-form backward seq {b} head {heads[0]} {k}: {e:.2e}")
        assert e <= TOL["bf16"], (k, e)
