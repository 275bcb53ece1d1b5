"""The chunk step at large state sizes (d >= 128; the paper's single head of
hd = 1024 with hidden 4096): every product is a matrix-core GEMM over
operands streamed from HBM.  GPU parity against the FP64 oracle (the same
oracle as the small-state path: it is written for any d and h), through the
C ABI."""
import numpy as np
import pytest
import torch

import oracle as orc
from gpu_util import TOL, apply_consistency, check, err_report, fmt, host, rel, storage_floor, to_dev
from workloads import make_inputs

pytestmark = pytest.mark.gpu


def ops():
    from paper_2604_08542_amd import ops
    return ops


def dev_inputs(N, H, d, h, seed, io):
    x = make_inputs(N, H, d, h, seed=seed, io_dtype=io)
    dev = {k: to_dev(x[k], io) for k in ("Q", "K", "V")}
    dev["W1"] = torch.from_numpy(x["W1"]).cuda()
    dev["W2"] = torch.from_numpy(x["W2"]).cuda()
    return x, dev


CASES = [
    # N, H, d, h, M, eta, io, mma_bf16
    (700, 2, 256, 512, 300, 0.5, "f32", False),    # ragged last chunk (100 tokens), two heads
    (700, 2, 256, 512, 300, 0.5, "bf16", True),
    (700, 2, 256, 512, 300, 0.5, "f32", True),     # FP32 tokens, BF16 matrix-core operands
    (700, 2, 256, 512, 300, 16.0, "bf16", True),   # large step: the update moves O well past the tolerance
    (620, 2, 256, 512, 300, 0.5, "f32", False),    # last chunk of 20 tokens: one contraction slice (FP32)
    (640, 2, 256, 512, 300, 0.5, "bf16", True),    # last chunk of 40 tokens: one contraction slice (BF16)
    (5496, 1, 1024, 4096, 2748, 0.5, "f32", False),  # the paper's state: 2 chunks of 2 frames
    (5496, 1, 1024, 4096, 2748, 0.5, "bf16", True),
]


@pytest.mark.parametrize("N,H,d,h,M,eta,io,mma", CASES)
def test_large_forward_matches_oracle(gpu, N, H, d, h, M, eta, io, mma):
    x, dv = dev_inputs(N, H, d, h, seed=N + d, io=io)
    r = ops().chunk_fwd(dv["Q"], dv["K"], dv["V"], dv["W1"], dv["W2"], eta, M, save_ckpt=True, emit_loss=True,
                        mma_bf16=mma)
    torch.cuda.synchronize()
    ref = orc.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], eta, M)
    ref0 = orc.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.0, M)
    tol = TOL["bf16" if mma or io == "bf16" else "f32"]
    print(f"N={N} H={H} d={d} h={h} M={M} eta={eta} io={io} mma_bf16={mma}")
    O = host(r["O"])
    check("O", O, ref["O"], tol)
    check("W1_T", host(r["W1_T"]), ref["W1_T"], tol)
    check("W2_T", host(r["W2_T"]), ref["W2_T"], tol)
    check("dW1", host(r["W1_T"]) - x["W1"], ref["W1_T"] - x["W1"], tol, floor=storage_floor(ref["W1_T"], x["W1"]))
    check("dW2", host(r["W2_T"]) - x["W2"], ref["W2_T"] - x["W2"], tol, floor=storage_floor(ref["W2_T"], x["W2"]))
    check("loss", host(r["loss"]), ref["loss"], tol)
    C = (N + M - 1) // M
    ck = host(r["ckpt"]).reshape(C, H, 2, -1)
    assert np.array_equal(ck[0, :, 0].reshape(x["W1"].shape), x["W1"])
    for c in range(1, C):
        check(f"dW1 ckpt {c}", ck[c, :, 0].reshape(x["W1"].shape) - x["W1"], ref["ckpt1"][c] - x["W1"], tol,
              floor=storage_floor(ref["ckpt1"][c], x["W1"]))
    e_eta, e_0 = rel(O, ref["O"]), rel(O, ref0["O"])
    print(f"  |O - O_ref(eta)| {e_eta:.2e} < |O - O_ref(0)| {e_0:.2e}")
    assert e_eta < e_0
    dref = ref["O"] - ref0["O"]
    effect = np.linalg.norm(dref) / np.linalg.norm(ref["O"])
    r0 = ops().chunk_fwd(dv["Q"], dv["K"], dv["V"], dv["W1"], dv["W2"], 0.0, M, mma_bf16=mma)
    O0 = host(r0["O"])
    rep = err_report(O - O0, dref)
    # delta-O is the difference of two outputs: their own errors bound how
    # well it can be resolved (|err O(eta)| + |err O(0)|, relative to |dO|)
    floor = (np.linalg.norm(O - ref["O"]) + np.linalg.norm(O0 - ref0["O"])) / np.linalg.norm(dref)
    print(f"  delta-O (|dO_ref|/|O_ref| = {effect:.2e}, resolution floor {floor:.2e}): " + fmt("", rep))
    if tol == TOL["f32"] or effect >= 0.25:
        assert rep["norm"] <= tol + floor, rep
    worst = apply_consistency(ops().chunk_fwd, dv["Q"], dv["K"], dv["V"], r["ckpt"], r["W1_T"], r["W2_T"], r["O"], M,
                              mma)
    print(f"  apply with W_(c+1) (eta=0 rerun) vs chain O: worst chunk rel {worst:.2e}")
    assert worst <= 1e-6


def test_large_batched_and_strided(gpu):
    """Two sequences (one of them shorter than a chunk) packed along the token
    axis, Q/K/V as strided views of one fused tensor; equal to the
    sequences run one by one and to the oracle."""
    N, H, d, h, M, eta = 900, 2, 256, 384, 256, 0.5
    x = make_inputs(N, H, d, h, seed=71)
    big = torch.zeros((N, 3, H, d), device="cuda")
    for i, k in enumerate(("Q", "K", "V")):
        big[:, i] = torch.from_numpy(x[k]).cuda()
    Q, K, V = big[:, 0], big[:, 1], big[:, 2]
    W1 = torch.from_numpy(x["W1"]).cuda(); W2 = torch.from_numpy(x["W2"]).cuda()
    cu = [0, 700, 900]
    r = ops().batched_fwd(Q, K, V, cu, W1, W2, eta, M)
    ref = orc.ttt_forward_batched(x["Q"], x["K"], x["V"], cu, x["W1"], x["W2"], eta, M)
    check("O", host(r["O"]), ref["O"], TOL["f32"])
    check("W2_T", host(r["W2_T"]), ref["W2_T"], TOL["f32"])
    for b in range(2):
        s, e = cu[b], cu[b + 1]
        rb = ops().chunk_fwd(Q[s:e], K[s:e], V[s:e], W1, W2, eta, M)
        assert torch.equal(rb["O"], r["O"][s:e]) and torch.equal(rb["W1_T"], r["W1_T"][b])


GCS_CASES = [
    # N, H, d, h, M, eta, io, mma_bf16
    (700, 2, 256, 512, 300, 4.0, "f32", False),   # ragged last chunk, two heads
    (700, 2, 256, 512, 300, 4.0, "bf16", True),   # the step moves O well past the BF16 tolerance
    (5496, 1, 1024, 4096, 2748, 2.0, "bf16", True),  # the paper's state
]


@pytest.mark.parametrize("N,H,d,h,M,eta,io,mma", GCS_CASES)
def test_large_gcs_matches_oracle(gpu, N, H, d, h, M, eta, io, mma):
    # Eq. 10 at large state sizes: every chunk's gradient at W0, one step, all
    # queries mapped with W*
    x, dv = dev_inputs(N, H, d, h, seed=N + d + 1, io=io)
    r = ops().gcs_fwd(dv["Q"], dv["K"], dv["V"], dv["W1"], dv["W2"], eta, M, emit_loss=True, mma_bf16=mma)
    torch.cuda.synchronize()
    ref = orc.ttt_forward_gcs(x["Q"], x["K"], x["V"], x["W1"], x["W2"], eta, M)
    ref0 = orc.ttt_forward_gcs(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.0, M)
    tol = TOL["bf16" if mma or io == "bf16" else "f32"]
    print(f"gcs N={N} H={H} d={d} h={h} M={M} eta={eta} io={io} mma_bf16={mma}")
    O = host(r["O"])
    check("O", O, ref["O"], tol)
    check("dW1", host(r["W1_T"]) - x["W1"], ref["W1_T"] - x["W1"], tol, floor=storage_floor(ref["W1_T"], x["W1"]))
    check("dW2", host(r["W2_T"]) - x["W2"], ref["W2_T"] - x["W2"], tol, floor=storage_floor(ref["W2_T"], x["W2"]))
    check("loss", host(r["loss"]), ref["loss"], tol)
    e_eta, e_0 = rel(O, ref["O"]), rel(O, ref0["O"])
    print(f"  |O - O_ref(eta)| {e_eta:.2e} < |O - O_ref(0)| {e_0:.2e}")
    assert e_eta < e_0


def test_large_gcs_one_chunk_equals_chain(gpu):
    x, dv = dev_inputs(300, 2, 256, 512, seed=73, io="bf16")
    a = ops().gcs_fwd(dv["Q"], dv["K"], dv["V"], dv["W1"], dv["W2"], 4.0, 300)
    b = ops().chunk_fwd(dv["Q"], dv["K"], dv["V"], dv["W1"], dv["W2"], 4.0, 300)
    for k in ("O", "W1_T", "W2_T"):
        assert torch.equal(a[k], b[k]), k


BWD_CASES = [
    # N, H, d, h, M, eta, io, mma_bf16
    (700, 2, 256, 512, 300, 0.5, "f32", False),   # ragged last chunk, two heads
    (700, 2, 256, 512, 300, 0.5, "bf16", True),
    (700, 1, 256, 512, 300, 0.5, "f32", True),    # FP32 tokens, BF16 matrix-core operands
    (2748, 1, 1024, 4096, 1374, 0.5, "bf16", True),  # the paper's state: 2 chunks of one frame
]


@pytest.mark.parametrize("N,H,d,h,M,eta,io,mma", BWD_CASES)
def test_large_backward_matches_oracle(gpu, N, H, d, h, M, eta, io, mma):
    # reverse mode through every inner update (Sec. 4.2 Eq. 8 differentiated)
    x = make_inputs(N, H, d, h, seed=N + d + 2, io_dtype=io, with_dO=True)
    dv = {k: to_dev(x[k], io) for k in ("Q", "K", "V", "dO")}
    W1, W2 = torch.from_numpy(x["W1"]).cuda(), torch.from_numpy(x["W2"]).cuda()
    f = ops().chunk_fwd(dv["Q"], dv["K"], dv["V"], W1, W2, eta, M, save_ckpt=True, mma_bf16=mma)
    g = ops().chunk_bwd(dv["Q"], dv["K"], dv["V"], W1, W2, eta, M, f["ckpt"], dv["dO"], mma_bf16=mma)
    torch.cuda.synchronize()
    ref = orc.ttt_backward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], eta, M, x["dO"])
    tol = TOL["bf16" if mma or io == "bf16" else "f32"]
    print(f"bwd N={N} H={H} d={d} h={h} M={M} eta={eta} io={io} mma_bf16={mma}")
    for k in ("dQ", "dK", "dV", "dW1_0", "dW2_0"):
        check(k, host(g[k]), ref[k], tol)
    e = rel(host(g["deta"]), ref["deta"])
    print(f"  deta {host(g['deta'])} ref {ref['deta']} rel {e:.2e}")
    assert e <= tol


@pytest.mark.parametrize("io,w0_per_seq", [("f32", False), ("bf16", True), ("bf16", False)])
def test_large_batched_backward_matches_oracle(gpu, io, w0_per_seq):
    # uneven sequences (3 chunks with a ragged last one, an empty one, one
    # chunk), each an independent chain; a shared W0 collects their sum
    d, h, M, eta = 256, 512, 300, 0.5
    cu = [0, 700, 700, 1000]
    B = len(cu) - 1
    x = make_inputs(1000, 2, d, h, seed=75, io_dtype=io, with_dO=True, n_w0=B if w0_per_seq else 1)
    dv = {k: to_dev(x[k], io) for k in ("Q", "K", "V", "dO")}
    W1, W2 = torch.from_numpy(x["W1"]).cuda(), torch.from_numpy(x["W2"]).cuda()
    mma = io == "bf16"
    f = ops().batched_fwd(dv["Q"], dv["K"], dv["V"], cu, W1, W2, eta, M, w0_per_seq=w0_per_seq, save_ckpt=True,
                          mma_bf16=mma)
    g = ops().batched_bwd(dv["Q"], dv["K"], dv["V"], cu, W1, W2, eta, M, f["ckpt"], dv["dO"], w0_per_seq=w0_per_seq,
                          mma_bf16=mma)
    torch.cuda.synchronize()
    ref = orc.ttt_backward_batched(x["Q"], x["K"], x["V"], cu, x["W1"], x["W2"], eta, M, x["dO"],
                                   w0_per_seq=w0_per_seq)
    tol = TOL[io]
    print(f"batched bwd {io} w0_per_seq={w0_per_seq}")
    for k in ("dQ", "dK", "dV", "dW1_0", "dW2_0"):
        check(k, host(g[k]), ref[k], tol)
    e = rel(host(g["deta"]), ref["deta"])
    print(f"  deta rel {e:.2e}")
    assert e <= tol


@pytest.mark.parametrize("N,H,d,h,M,eta,io,mma", [
    (700, 2, 256, 512, 300, 0.5, "f32", False),
    (700, 2, 256, 512, 300, 0.5, "bf16", True),
    (5496, 1, 1024, 4096, 2748, 0.5, "bf16", True),  # the paper's state: 2 chunks of 2 frames
])
def test_large_gcs_backward_matches_oracle(gpu, N, H, d, h, M, eta, io, mma):
    # reverse mode of Eq. 10: the apply adjoint of every token at W*, every
    # chunk's update adjoint at W0 against it
    x = make_inputs(N, H, d, h, seed=N + d + 3, io_dtype=io, with_dO=True)
    dv = {k: to_dev(x[k], io) for k in ("Q", "K", "V", "dO")}
    W1, W2 = torch.from_numpy(x["W1"]).cuda(), torch.from_numpy(x["W2"]).cuda()
    g = ops().gcs_bwd(dv["Q"], dv["K"], dv["V"], W1, W2, eta, M, dv["dO"], mma_bf16=mma)
    torch.cuda.synchronize()
    ref = orc.ttt_backward_gcs(x["Q"], x["K"], x["V"], x["W1"], x["W2"], eta, M, x["dO"])
    tol = TOL["bf16" if mma or io == "bf16" else "f32"]
    print(f"gcs bwd N={N} H={H} d={d} h={h} M={M} eta={eta} io={io} mma_bf16={mma}")
    for k in ("dQ", "dK", "dV", "dW1_0", "dW2_0"):
        check(k, host(g[k]), ref[k], tol)
    e = rel(host(g["deta"]), ref["deta"])
    print(f"  deta rel {e:.2e}")
    assert e <= tol


def test_large_backward_deterministic(gpu):
    x = make_inputs(700, 1, 256, 512, seed=74, io_dtype="bf16", with_dO=True)
    dv = {k: to_dev(x[k], "bf16") for k in ("Q", "K", "V", "dO")}
    W1, W2 = torch.from_numpy(x["W1"]).cuda(), torch.from_numpy(x["W2"]).cuda()
    f = ops().chunk_fwd(dv["Q"], dv["K"], dv["V"], W1, W2, 0.5, 300, save_ckpt=True)
    a = ops().chunk_bwd(dv["Q"], dv["K"], dv["V"], W1, W2, 0.5, 300, f["ckpt"], dv["dO"])
    b = ops().chunk_bwd(dv["Q"], dv["K"], dv["V"], W1, W2, 0.5, 300, f["ckpt"], dv["dO"])
    for k in ("dQ", "dK", "dV", "dW1_0", "dW2_0", "deta"):
        assert torch.equal(a[k], b[k]), k


def test_large_shapes_rejected_where_not_built(gpu):
    from paper_2604_08542_amd import _lib
    x, dv = dev_inputs(64, 1, 256, 512, seed=72, io="f32")
    for fn in (lambda: ops().chunk_fwd_noalloc(dv["Q"], dv["K"], dv["V"], dv["W1"], dv["W2"], 0.1, 32),):
        with pytest.raises(_lib.TTTError) as e:
            fn()
        assert e.value.status == _lib.TTT_ENOTSUP
