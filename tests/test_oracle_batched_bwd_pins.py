"""Pins of the oracle's batched backward (packed sequences of uneven length,
an empty one included): central finite differences of the summed outer
objective sum_b <O_b, dO_b> computed from the batched forward, for a shared
W0 and for per-sequence W0, eta included.  The forward is the only code the
finite differences share with the backward."""
import numpy as np
import pytest

import oracle as orc
from workloads import make_inputs

CU = [0, 5, 5, 14]  # lengths 5, 0, 9 with chunks of 4: ragged last chunks


def rel(a, b):
    a = np.asarray(a, np.float64); b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def setup(w0_per_seq):
    x = {k: v.astype(np.float64) for k, v in make_inputs(CU[-1], 2, 3, 5, seed=40, with_dO=True).items()}
    if w0_per_seq:
        rng = np.random.default_rng(41)
        x["W1"] = np.stack([x["W1"] + 0.1 * rng.standard_normal(x["W1"].shape) for _ in range(3)])
        x["W2"] = np.stack([x["W2"] + 0.1 * rng.standard_normal(x["W2"].shape) for _ in range(3)])
    return x


def objective(x, eta0, M, w0_per_seq, **over):
    a = {n: over.get(n, x[n]) for n in ("Q", "K", "V", "W1", "W2")}
    O = orc.ttt_forward_batched(a["Q"], a["K"], a["V"], CU, a["W1"], a["W2"], over.get("eta", eta0), M,
                                w0_per_seq=w0_per_seq)["O"]
    return float(np.sum(O * x["dO"]))


@pytest.mark.parametrize("w0_per_seq", [False, True])
def test_batched_backward_matches_fd(w0_per_seq):
    x = setup(w0_per_seq)
    eta, M, h = 0.35, 4, 1e-6
    g = orc.ttt_backward_batched(x["Q"], x["K"], x["V"], CU, x["W1"], x["W2"], eta, M, x["dO"],
                                 w0_per_seq=w0_per_seq)
    gmap = dict(Q="dQ", K="dK", V="dV", W1="dW1_0", W2="dW2_0")
    for n, gk in gmap.items():
        fd = np.zeros_like(x[n])
        for idx in np.ndindex(x[n].shape):
            e = np.zeros_like(x[n]); e[idx] = h
            fd[idx] = (objective(x, eta, M, w0_per_seq, **{n: x[n] + e}) -
                       objective(x, eta, M, w0_per_seq, **{n: x[n] - e})) / (2 * h)
        assert rel(g[gk], fd) < 1e-6, n
    fde = (objective(x, eta, M, w0_per_seq, eta=eta + h) - objective(x, eta, M, w0_per_seq, eta=eta - h)) / (2 * h)
    assert abs(g["deta"].sum() - fde) < 1e-6 * max(1.0, abs(fde))
    # the empty sequence contributes nothing; with per-sequence W0 its gradient is exactly zero
    if w0_per_seq:
        assert not np.any(g["dW1_0"][1]) and not np.any(g["dW2_0"][1])


def test_single_sequence_batch_equals_chain_backward():
    x = setup(False)
    eta, M = 0.35, 4
    a = orc.ttt_backward_batched(x["Q"], x["K"], x["V"], [0, CU[-1]], x["W1"], x["W2"], eta, M, x["dO"])
    b = orc.ttt_backward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], eta, M, x["dO"])
    for k in ("dQ", "dK", "dV", "dW1_0", "dW2_0", "deta"):
        assert np.array_equal(a[k], b[k]), k
