"""Pins of the oracle's Global Context Synchronization form (Sec. 4.2,
Eq. 10): the synchronised gradient is the sum of per-chunk gradients at the
shared weights, one step is applied, every chunk is mapped with the result."""
import numpy as np
import torch

import oracle as orc
from workloads import make_inputs
from test_oracle_backward_pins import f64, rel


def test_one_chunk_equals_chain():
    x = f64(make_inputs(9, 2, 4, 6, seed=40))
    a = orc.ttt_forward_gcs(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.3, 9)
    b = orc.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.3, 9)
    assert rel(a["O"], b["O"]) < 1e-14 and rel(a["W2_T"], b["W2_T"]) < 1e-14


def test_synchronised_gradient_is_fd_of_summed_loss():
    """W* = W0 - eta * grad(sum_c L_c)(W0), the gradient by FD of the summed
    chunk losses (ragged last chunk with its own 1/M_c)."""
    x = f64(make_inputs(11, 1, 3, 4, seed=41))
    eta, M = 0.2, 4
    r = orc.ttt_forward_gcs(x["Q"], x["K"], x["V"], x["W1"], x["W2"], eta, M)
    k = torch.nn.functional.normalize(torch.from_numpy(x["K"][:, 0]), dim=-1).numpy()
    v = torch.nn.functional.normalize(torch.from_numpy(x["V"][:, 0]), dim=-1).numpy()

    def total(W1, W2):
        return sum(orc.inner_loss(k[s:e], v[s:e], W1, W2) for s, e in orc.chunk_bounds(11, M))
    for W, which in ((x["W1"][0], 1), (x["W2"][0], 2)):
        g = np.zeros_like(W)
        for idx in np.ndindex(W.shape):
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += 1e-6
            Wm[idx] -= 1e-6
            if which == 1:
                g[idx] = (total(Wp, x["W2"][0]) - total(Wm, x["W2"][0])) / 2e-6
            else:
                g[idx] = (total(x["W1"][0], Wp) - total(x["W1"][0], Wm)) / 2e-6
        got = r["W1_T"][0] if which == 1 else r["W2_T"][0]
        assert rel(got, W - eta * g) < 1e-8


def test_chunk_order_does_not_matter():
    x = f64(make_inputs(12, 1, 4, 6, seed=42))
    perm = np.concatenate([np.arange(8, 12), np.arange(0, 4), np.arange(4, 8)])
    a = orc.ttt_forward_gcs(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.2, 4)
    b = orc.ttt_forward_gcs(x["Q"][perm], x["K"][perm], x["V"][perm], x["W1"], x["W2"], 0.2, 4)
    assert rel(b["W1_T"], a["W1_T"]) < 1e-13
    assert rel(b["O"], a["O"][perm]) < 1e-13


def test_gcs_backward_matches_fd_and_autograd():
    x = f64(make_inputs(10, 2, 3, 5, seed=43, with_dO=True))
    eta, M = 0.4, 4
    g = orc.ttt_backward_gcs(x["Q"], x["K"], x["V"], x["W1"], x["W2"], eta, M, x["dO"])
    t = {n: torch.from_numpy(x[n]).requires_grad_() for n in ["Q", "K", "V", "W1", "W2"]}
    te = torch.tensor(eta, dtype=torch.float64, requires_grad=True)
    outs = []
    for hd in range(2):
        q, k, v = (torch.nn.functional.normalize(t[n][:, hd], dim=-1) for n in "QKV")
        w1, w2 = t["W1"][hd], t["W2"][hd]
        L = sum(((torch.nn.functional.silu(k[s:e] @ w1) @ w2 - v[s:e]) ** 2).sum(1).mean()
                for s, e in orc.chunk_bounds(10, M))
        g1, g2 = torch.autograd.grad(L, (w1, w2), create_graph=True)
        outs.append(torch.nn.functional.silu(q @ (w1 - te * g1)) @ (w2 - te * g2))
    O = torch.stack(outs, 1)
    assert rel(g["fwd"]["O"], O.detach().numpy()) < 1e-13
    (O * torch.from_numpy(x["dO"])).sum().backward()
    for n, gn in dict(Q="dQ", K="dK", V="dV", W1="dW1_0", W2="dW2_0").items():
        assert rel(g[gn], t[n].grad.numpy()) < 1e-11, n
    assert abs(g["deta"].sum() - te.grad.item()) < 1e-11 * max(1.0, abs(te.grad.item()))
