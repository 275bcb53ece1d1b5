"""The paper's memory unit (Supp. A: SwiGLU fast network, dot-product inner
loss with token-wise step sizes; Sec. 4.2 Eq. 8-10, chain and GCS forms) at
large state sizes, up to the paper's single head of hd = 1024 with hidden
4096: every product of a chunk step is a matrix-core GEMM over weights
streamed from HBM.  GPU parity against the FP64 oracle through the C ABI."""
import numpy as np
import pytest
import torch

import oracle as orc
from gpu_util import TOL, check, err_report, fmt, host, rel, storage_floor, to_dev
from workloads import make_eta_tok, make_inputs

pytestmark = pytest.mark.gpu


def ops():
    from paper_2604_08542_amd import ops
    return ops


def dev_inputs(N, H, d, h, M, eta, seed, io):
    x = make_inputs(N, H, d, h, seed=seed, io_dtype=io)
    x["W3"] = (np.random.default_rng(seed + 1).standard_normal(x["W1"].shape) / np.sqrt(d)).astype(np.float32)
    x["eta"] = make_eta_tok(N, H, M, eta, seed)
    dev = {k: to_dev(x[k], io) for k in ("Q", "K", "V")}
    for k in ("W1", "W2", "W3", "eta"):
        dev[k] = torch.from_numpy(x[k]).cuda()
    return x, dev


def run(dev, M, sync, mma, scale=1.0):
    r = ops().amu_fwd(dev["Q"], dev["K"], dev["V"], dev["eta"] * scale, dev["W1"], dev["W2"], dev["W3"], M,
                      sync=sync, mma_bf16=mma)
    torch.cuda.synchronize()
    return r


# eta_i ~ eta / M: at d = 256 an eta of 100 moves O by ~2.7% (above the BF16
# gate, so an apply with stale weights fails it); at the paper's state it
# moves W by ~0.1-0.4% and O by ~0.4%
CASES = [
    # N, H, d, h, M, eta, io, mma_bf16, sync
    (700, 2, 256, 512, 300, 100.0, "f32", False, "chain"),  # ragged last chunk (100 tokens), two heads
    (700, 2, 256, 512, 300, 100.0, "f32", False, "gcs"),
    (700, 2, 256, 512, 300, 100.0, "bf16", True, "chain"),
    (700, 2, 256, 512, 300, 100.0, "bf16", True, "gcs"),
    (700, 2, 256, 512, 300, 100.0, "f32", True, "chain"),   # FP32 tokens, BF16 matrix-core operands
    (2748, 1, 1024, 4096, 1374, 100.0, "f32", False, "chain"),  # the paper's state: 2 chunks of one frame
    (2748, 1, 1024, 4096, 1374, 100.0, "bf16", True, "chain"),
    (2748, 1, 1024, 4096, 1374, 100.0, "bf16", True, "gcs"),
]


@pytest.mark.parametrize("N,H,d,h,M,eta,io,mma,sync", CASES)
def test_large_amu_matches_oracle(gpu, N, H, d, h, M, eta, io, mma, sync):
    x, dev = dev_inputs(N, H, d, h, M, eta, seed=N + d + (sync == "gcs"), io=io)
    r = run(dev, M, sync, mma)
    ref = orc.ttt_forward_swiglu(x["Q"], x["K"], x["V"], x["W1"], x["W2"], x["W3"], x["eta"], M, sync=sync)
    ref0 = orc.ttt_forward_swiglu(x["Q"], x["K"], x["V"], x["W1"], x["W2"], x["W3"], 0.0 * x["eta"], M, sync=sync)
    tol = TOL["bf16" if mma or io == "bf16" else "f32"]
    print(f"amu N={N} H={H} d={d} h={h} M={M} eta={eta} io={io} mma_bf16={mma} {sync}")
    O = host(r["O"])
    check("O", O, ref["O"], tol)
    for k, w in (("W1_T", "W1"), ("W2_T", "W2"), ("W3_T", "W3")):
        check("d" + w, host(r[k]) - x[w], ref[k] - x[w], tol, floor=storage_floor(ref[k], x[w]))
    # the output is closer to the updated model than to the initial one
    e_eta, e_0 = rel(O, ref["O"]), rel(O, ref0["O"])
    print(f"  |O - O_ref(eta)| {e_eta:.2e} < |O - O_ref(0)| {e_0:.2e}")
    assert e_eta < e_0
    # delta-O = O(eta) - O(0) from the same path, against the oracle's
    O0 = host(run(dev, M, sync, mma, scale=0.0)["O"])
    dref = ref["O"] - ref0["O"]
    effect = np.linalg.norm(dref) / np.linalg.norm(ref["O"])
    rep = err_report(O - O0, dref)
    floor = (np.linalg.norm(O - ref["O"]) + np.linalg.norm(O0 - ref0["O"])) / np.linalg.norm(dref)
    print(f"  delta-O (|dO_ref|/|O_ref| = {effect:.2e}, resolution floor {floor:.2e}): " + fmt("", rep))
    if tol == TOL["f32"]:
        assert rep["norm"] <= tol + floor, rep


def test_large_amu_one_chunk_chain_equals_gcs(gpu):
    # with one chunk both forms take the same gradient at W0 and the same step
    _, dev = dev_inputs(300, 2, 256, 512, 300, 100.0, seed=5, io="bf16")
    a = run(dev, 300, "chain", True)
    b = run(dev, 300, "gcs", True)
    for k in ("O", "W1_T", "W2_T", "W3_T"):
        assert torch.equal(a[k], b[k]), k


def test_large_amu_deterministic(gpu):
    _, dev = dev_inputs(700, 1, 256, 512, 300, 100.0, seed=6, io="bf16")
    a = run(dev, 300, "chain", True)
    b = run(dev, 300, "chain", True)
    for k in ("O", "W1_T", "W2_T", "W3_T"):
        assert torch.equal(a[k], b[k]), k


def test_large_amu_empty_stream(gpu):
    x, dev = dev_inputs(0, 1, 256, 512, 300, 100.0, seed=7, io="f32")
    r = run(dev, 300, "chain", False)
    assert r["O"].shape == (0, 1, 256)
    for k, w in (("W1_T", "W1"), ("W2_T", "W2"), ("W3_T", "W3")):
        assert torch.equal(r[k], dev[w]), k


BWD_CASES = [
    # N, H, d, h, M, eta, io, mma_bf16, sync
    (700, 2, 256, 512, 300, 100.0, "f32", False, "chain"),
    (700, 2, 256, 512, 300, 100.0, "f32", False, "gcs"),
    (700, 2, 256, 512, 300, 100.0, "bf16", True, "chain"),
    (700, 2, 256, 512, 300, 100.0, "bf16", True, "gcs"),
    (2748, 1, 1024, 4096, 1374, 100.0, "bf16", True, "chain"),  # the paper's state
    (2748, 1, 1024, 4096, 1374, 100.0, "bf16", True, "gcs"),
]


@pytest.mark.parametrize("N,H,d,h,M,eta,io,mma,sync", BWD_CASES)
def test_large_amu_backward_matches_oracle(gpu, N, H, d, h, M, eta, io, mma, sync):
    # reverse mode through every inner update of the paper's unit, with the
    # per-token step-size derivative
    x, dev = dev_inputs(N, H, d, h, M, eta, seed=N + d + 11 + (sync == "gcs"), io=io)
    dO = np.random.default_rng(N + 5).standard_normal((N, H, d)).astype(np.float32)
    if io == "bf16":
        dO = torch.from_numpy(dO).to(torch.bfloat16).float().numpy()
    g = ops().amu_bwd(dev["Q"], dev["K"], dev["V"], dev["eta"], dev["W1"], dev["W2"], dev["W3"], M,
                      to_dev(dO, io), sync=sync, mma_bf16=mma)
    torch.cuda.synchronize()
    ref = orc.ttt_backward_swiglu(x["Q"], x["K"], x["V"], x["W1"], x["W2"], x["W3"], x["eta"], M, dO, sync=sync)
    tol = TOL["bf16" if mma or io == "bf16" else "f32"]
    print(f"amu bwd N={N} H={H} d={d} h={h} M={M} eta={eta} io={io} mma_bf16={mma} {sync}")
    for k in ("dQ", "dK", "dV", "dW1_0", "dW2_0", "dW3_0"):
        check(k, host(g[k]), ref[k], tol)
    # per-token step-size derivatives: normwise over the tokens of each head
    check("deta_tok", host(g["deta_tok"]).T, ref["deta_tok"].T, tol, row_mult=1.0)
