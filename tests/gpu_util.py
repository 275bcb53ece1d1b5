"""Helpers for GPU parity tests: run the HIP path and the FP64 oracle on the
same seeded inputs and compare per output."""
import numpy as np
import torch

import oracle as orc
from workloads import make_inputs

TOL = {"f32": 1e-4, "bf16": 2e-2}
# The worst single row (a token's output vector, a row of a weight matrix)
# may be this many times the normwise tolerance off.  Rows are short
# (64 or h elements), so their relative error scatters above the normwise
# figure; a localised fault (one wrong tile, one wrong token) shows up here
# long before it moves the normwise error of a whole tensor.
ROW_MULT = 5.0


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def err_report(a, b):
    """Normwise relative error, max-abs error, max-abs / max|ref| and the
    worst per-row relative error (rows along the last axis) of a vs ref b."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    diff = a - b
    maxabs = float(np.max(np.abs(diff))) if diff.size else 0.0
    maxref = float(np.max(np.abs(b))) if b.size else 0.0
    rb = np.linalg.norm(b.reshape(-1, b.shape[-1]), axis=1)
    rd = np.linalg.norm(diff.reshape(-1, b.shape[-1]), axis=1)
    ok = rb > 0
    row = float(np.max(rd[ok] / rb[ok])) if ok.any() else 0.0
    return dict(norm=rel(a, b), maxabs=maxabs, maxabs_rel=maxabs / maxref if maxref > 0 else maxabs, row=row)


def fmt(name, r):
    return (f"{name}: norm {r['norm']:.2e} maxabs {r['maxabs']:.2e} "
            f"maxabs/max|ref| {r['maxabs_rel']:.2e} worst-row {r['row']:.2e}")


def check(name, a, b, tol, row_mult=ROW_MULT, floor=0.0):
    """Gate normwise error at tol + floor and the worst row at
    row_mult * (tol + floor); prints the whole report.  `floor` is the
    error that even the exactly rounded result has (see storage_floor)."""
    r = err_report(a, b)
    print("  " + fmt(name, r) + (f" (storage floor {floor:.2e})" if floor else ""))
    assert r["norm"] <= tol + floor, (name, "normwise", r)
    assert r["row"] <= row_mult * (tol + floor), (name, "worst row", r)
    return r


def storage_floor(w_ref, w0):
    """A weight change W - W0 read from FP32-stored weights: even the exactly
    rounded FP32 value of W carries this normwise relative error in the
    change (the FP32 spacing of W against the size of the change)."""
    w_ref = np.asarray(w_ref, np.float64)
    dw = w_ref - np.asarray(w0, np.float64)
    nd = np.linalg.norm(dw)
    return float(np.linalg.norm(w_ref.astype(np.float32).astype(np.float64) - w_ref) / nd) if nd > 0 else 0.0


def to_dev(x, io):
    dt = torch.float32 if io == "f32" else torch.bfloat16
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda").to(dt)


def inputs(N, H, h, seed, io, with_dO=False):
    x = make_inputs(N, H, 64, h, seed=seed, io_dtype=io, with_dO=with_dO)
    dev = {k: to_dev(v, io) for k, v in x.items() if k in ("Q", "K", "V", "dO")}
    dev["W1"] = torch.from_numpy(x["W1"]).cuda()
    dev["W2"] = torch.from_numpy(x["W2"]).cuda()
    return x, dev


def host(t):
    return t.detach().float().cpu().numpy().astype(np.float64)


def apply_consistency(chunk_fwd, Q, K, V, ckpt, W1_T, W2_T, O, M, mma_bf16, chunks=None):
    """The apply of chunk c must use the weights after chunk c's update
    (W_{c+1}; Sec. 4.2 and Eq. 4).  Re-run the same GPU path on chunk c alone
    with eta = 0 and initial weights W_{c+1} (checkpoint c+1, or W_T for the
    last chunk): its output must equal the chain's O_c up to rounding.  This
    pins the apply to the updated weights even where the whole effect of the
    update on O is below the BF16 tolerance.  Returns the worst relative
    difference over the checked chunks."""
    N, H, d = Q.shape
    h = W1_T.shape[-1]
    C = (N + M - 1) // M
    worst = 0.0
    for c in (range(C) if chunks is None else chunks):
        s, e = c * M, min((c + 1) * M, N)
        if c + 1 < C:
            w = ckpt[c + 1].view(H, 2, d * h)
            w1 = w[:, 0].reshape(H, d, h).contiguous()
            w2 = w[:, 1].reshape(H, h, d).contiguous()
        else:
            w1, w2 = W1_T, W2_T
        r = chunk_fwd(Q[s:e], K[s:e], V[s:e], w1, w2, 0.0, M, mma_bf16=mma_bf16)
        worst = max(worst, rel(host(r["O"]), host(O[s:e])))
    return worst
