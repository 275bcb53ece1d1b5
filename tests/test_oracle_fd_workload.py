"""The oracle's backward at the differentiation workload's shape (16 x 64,
hidden 256, chunks of 4 frames = 5496 tokens) on a 2-chunk subset, checked
by central finite differences with step 1e-3 along random directions (one
head: heads are independent)."""
import numpy as np
import pytest

import oracle as orc
from workloads import WORKLOADS, make_inputs


@pytest.mark.slow
def test_backward_fd_two_chunk_subset():
    w = WORKLOADS["layer16_32f_chunk4f_bwd"]
    N = 2 * w.chunk_tokens
    x = {k: v.astype(np.float64) for k, v in make_inputs(N, 1, w.d_head, w.d_hidden, seed=0, with_dO=True).items()}
    g = orc.ttt_backward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], w.eta, w.chunk_tokens, x["dO"])
    rng = np.random.default_rng(1)
    h = 1e-3

    def obj(**o):
        a = {k: o.get(k, x[k]) for k in ("Q", "K", "V", "W1", "W2")}
        return orc.outer_objective(a["Q"], a["K"], a["V"], a["W1"], a["W2"], o.get("eta", w.eta), w.chunk_tokens,
                                   x["dO"])
    for name, gname in (("K", "dK"), ("V", "dV"), ("W1", "dW1_0"), ("W2", "dW2_0"), ("Q", "dQ")):
        u = rng.standard_normal(x[name].shape)
        u /= np.linalg.norm(u)
        fd = (obj(**{name: x[name] + h * u}) - obj(**{name: x[name] - h * u})) / (2 * h)
        an = float(np.sum(g[gname] * u))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-9, (name, fd, an)
    fd = (obj(eta=w.eta + h) - obj(eta=w.eta - h)) / (2 * h)
    assert abs(fd - g["deta"].sum()) <= 1e-6 * max(1.0, abs(fd))
