"""The persistent schedule of the forward (one launch walks every chunk of
every chain; the work-groups of a chain meet at device-memory barriers
between chunks) against the stepwise schedule (two launches per chunk step,
ordered by the stream) and against the FP64 oracle; its bounded waits; the
empty-stream and NaN edge cases."""
import numpy as np
import pytest
import torch

import oracle as orc
from gpu_util import TOL, check, host, inputs, rel

pytestmark = pytest.mark.gpu


def ops():
    from paper_2604_08542_amd import ops
    return ops


@pytest.mark.parametrize("io,h,G", [("f32", 256, 4), ("bf16", 256, 8), ("f32", 128, 3), ("bf16", 128, 16),
                                    ("bf16", 128, 24), ("bf16", 256, 12)])
def test_persistent_equals_stepwise(gpu, io, h, G):
    """Same shards, same fixed-order reductions: both schedules give the same
    bits; the batch mixes a long, a ragged and a one-token sequence."""
    x, d = inputs(4100, 3, h, seed=40 + h, io=io)
    cu = [0, 2500, 2501, 3000, 4100]
    kw = dict(save_ckpt=True)
    rp = ops().batched_fwd(d["Q"], d["K"], d["V"], cu, d["W1"], d["W2"], 0.1, 600, tile_cfg=dict(wg_per_chain=G), **kw)
    rs = ops().batched_fwd(d["Q"], d["K"], d["V"], cu, d["W1"], d["W2"], 0.1, 600,
                           tile_cfg=dict(wg_per_chain=G, schedule="stepwise"), **kw)
    torch.cuda.synchronize()
    for k in ("O", "W1_T", "W2_T", "ckpt"):
        assert torch.equal(rp[k], rs[k]), k
    ref = orc.ttt_forward_batched(x["Q"], x["K"], x["V"], cu, x["W1"], x["W2"], 0.1, 600)
    check("O", host(rp["O"]), ref["O"], TOL[io])
    check("W1_T", host(rp["W1_T"]), ref["W1_T"], TOL[io])


@pytest.mark.parametrize("target", [8, 24, 64])
def test_more_chains_than_groups(gpu, target):
    """Few groups, many chains: each group takes chain after chain from the
    device counter (longest sequence first); the result does not depend on
    which group ran which chain."""
    x, d = inputs(3000, 4, 128, seed=41, io="f32")
    cu = [0, 100, 1100, 1200, 2900, 3000]
    r = ops().batched_fwd(d["Q"], d["K"], d["V"], cu, d["W1"], d["W2"], 0.1, 256,
                          tile_cfg=dict(wg_per_chain=4, target_wgs=target))
    r1 = ops().batched_fwd(d["Q"], d["K"], d["V"], cu, d["W1"], d["W2"], 0.1, 256, tile_cfg=dict(wg_per_chain=4))
    torch.cuda.synchronize()
    assert torch.equal(r["O"], r1["O"]) and torch.equal(r["W2_T"], r1["W2_T"])
    ref = orc.ttt_forward_batched(x["Q"], x["K"], x["V"], cu, x["W1"], x["W2"], 0.1, 256)
    check("O", host(r["O"]), ref["O"], TOL["f32"])


def test_many_sequences_split_over_launches(gpu):
    """More sequences than one launch descriptor holds (64): consecutive
    persistent launches."""
    rng = np.random.default_rng(42)
    lens = rng.integers(0, 90, size=70)
    cu = np.concatenate([[0], np.cumsum(lens)]).tolist()
    x, d = inputs(cu[-1], 2, 128, seed=43, io="f32")
    r = ops().batched_fwd(d["Q"], d["K"], d["V"], cu, d["W1"], d["W2"], 0.1, 32)
    torch.cuda.synchronize()
    ref = orc.ttt_forward_batched(x["Q"], x["K"], x["V"], cu, x["W1"], x["W2"], 0.1, 32)
    check("O", host(r["O"]), ref["O"], TOL["f32"])
    check("W1_T", host(r["W1_T"]), ref["W1_T"], TOL["f32"])


def test_workspace_status_clear_after_a_normal_call(gpu):
    x, d = inputs(2000, 2, 256, seed=44, io="bf16")
    from paper_2604_08542_amd.ops import problem, workspace, _flags
    prob = problem(d["Q"], 256, 0, 500, 0.1, _flags(True))
    ws = workspace(prob, 1, d["Q"].device)
    ops().batched_fwd(d["Q"], d["K"], d["V"], [0, 2000], d["W1"], d["W2"], 0.1, 500, ws=ws)
    assert ops().workspace_status(ws) == 0


def test_bounded_wait_gives_up_and_flags(gpu):
    """A barrier wait limited to one poll gives up instead of waiting: the
    call still completes (no wave waits forever) and the workspace's error
    word reports it.  The outputs of such a call are not meaningful."""
    x, d = inputs(6000, 2, 256, seed=45, io="bf16")
    from paper_2604_08542_amd.ops import problem, workspace, _flags
    prob = problem(d["Q"], 256, 0, 1000, 0.1, _flags(True))
    ws = workspace(prob, 1, d["Q"].device)
    ops().batched_fwd(d["Q"], d["K"], d["V"], [0, 6000], d["W1"], d["W2"], 0.1, 1000, ws=ws,
                      tile_cfg=dict(wg_per_chain=16, spin_limit=1))
    assert ops().workspace_status(ws) & 1 == 1
    # the next call on the same workspace clears the word and is correct
    r = ops().batched_fwd(d["Q"], d["K"], d["V"], [0, 6000], d["W1"], d["W2"], 0.1, 1000, ws=ws)
    assert ops().workspace_status(ws) == 0
    ref = orc.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.1, 1000)
    check("O", host(r["O"]), ref["O"], TOL["bf16"])


def test_empty_stream(gpu):
    """No tokens: nothing but the final weights (= initial weights) is written;
    empty token tensors pass null pointers."""
    x, d = inputs(0, 2, 128, seed=46, io="f32")
    r = ops().chunk_fwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], 0.1, 100, save_ckpt=True, emit_loss=True)
    assert r["O"].numel() == 0
    assert torch.equal(r["W1_T"], d["W1"]) and torch.equal(r["W2_T"], d["W2"])
    rb = ops().batched_fwd(d["Q"], d["K"], d["V"], [0, 0, 0], d["W1"], d["W2"], 0.1, 100)
    assert torch.equal(rb["W1_T"][1], d["W1"]) and torch.equal(rb["W2_T"][0], d["W2"])
    rg = ops().gcs_fwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], 0.1, 100)
    assert torch.equal(rg["W1_T"], d["W1"])


def test_nan_input_propagates(gpu):
    """A NaN in one key of chunk 0 reaches that chunk's gradient, so every
    later weight and every output from chunk 0 on is NaN; the call ends
    normally (no wave waits on data)."""
    x, d = inputs(3000, 2, 256, seed=47, io="bf16")
    K = d["K"].clone()
    K[17, 1, 5] = float("nan")
    r = ops().chunk_fwd(d["Q"], K, d["V"], d["W1"], d["W2"], 0.1, 1000)
    torch.cuda.synchronize()
    assert torch.isnan(r["O"][:, 1]).all()
    assert torch.isnan(r["W1_T"][1]).all()
    # head 0 never sees the NaN
    assert not torch.isnan(r["O"][:, 0]).any() and not torch.isnan(r["W1_T"][0]).any()
