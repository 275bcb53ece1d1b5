"""The allocation-free forward entry point (ttt_chunk_fwd_noalloc, fixed
device scratch inside the library) against ttt_chunk_fwd (caller
workspace) through the C ABI: two calls in a row on the same GPU, the second
with a smaller input, each matching the workspace entry point to the
parity tolerance; and the size limit of the fixed scratch."""
import pytest
import torch

from gpu_util import TOL, check, host, inputs

pytestmark = pytest.mark.gpu


def ops():
    from paper_2604_08542_amd import ops
    return ops


@pytest.mark.parametrize("io,h", [("f32", 256), ("bf16", 256), ("bf16", 128)])
def test_noalloc_matches_workspace_entry_point(gpu, io, h):
    tol = TOL[io]
    for (N, H, M, seed) in ((6000, 8, 1374, 60), (1100, 2, 300, 61)):   # second call smaller
        x, d = inputs(N, H, h, seed=seed, io=io)
        ref = ops().chunk_fwd(d["Q"], d["K"], d["V"], d["W1"], d["W2"], 0.1, M, save_ckpt=True, emit_loss=True)
        r = ops().chunk_fwd_noalloc(d["Q"], d["K"], d["V"], d["W1"], d["W2"], 0.1, M, save_ckpt=True,
                                    emit_loss=True)
        torch.cuda.synchronize()
        print(f"N={N} H={H} h={h} M={M} io={io}: bit-exact O {torch.equal(r['O'], ref['O'])}")
        for k in ("O", "W1_T", "W2_T", "ckpt", "loss"):
            check(k, host(r[k]), host(ref[k]), tol)


def test_noalloc_rejects_problems_beyond_the_scratch(gpu):
    from paper_2604_08542_amd import _lib
    # 107 heads at h = 256 need 3 x 107 x 128 KiB > 40 MiB of scratch
    x, d = inputs(64, 107, 256, seed=62, io="bf16")
    with pytest.raises(_lib.TTTError) as e:
        ops().chunk_fwd_noalloc(d["Q"], d["K"], d["V"], d["W1"], d["W2"], 0.1, 32)
    assert e.value.status == _lib.TTT_EWORKSPACE
    # 100 heads fit
    r = ops().chunk_fwd_noalloc(d["Q"][:, :100].contiguous(), d["K"][:, :100].contiguous(),
                                d["V"][:, :100].contiguous(), d["W1"][:100].contiguous(), d["W2"][:100].contiguous(),
                                0.1, 32)
    torch.cuda.synchronize()
    assert torch.isfinite(r["O"].float()).all()
