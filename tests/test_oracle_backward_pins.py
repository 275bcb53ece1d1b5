"""Pins of the oracle's hand-derived backward through the chain of inner
updates: central finite differences of the outer objective, and torch
float64 autograd through an unrolled chain whose inner gradient is itself
taken by autograd (create_graph=True), so no hand-derived derivative is
shared with the oracle."""
import numpy as np
import pytest
import torch

import oracle as orc
from workloads import make_inputs


def rel(a, b):
    a = np.asarray(a, np.float64); b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def f64(x):
    return {k: v.astype(np.float64) for k, v in x.items()}


def fd_directional(fun, x, direction, step=1e-5):
    return (fun(x + step * direction) - fun(x - step * direction)) / (2 * step)


@pytest.mark.parametrize("norm", [(True, True, True), (False, False, False)])
def test_backward_matches_fd_ragged(norm):
    """Ragged 3-chunk case (N=11, M=4): directional and coordinate FD of
    sum <O, dO> for every input, eta included."""
    x = f64(make_inputs(11, 2, 3, 5, seed=20, with_dO=True))
    eta, M = 0.4, 4
    g = orc.ttt_backward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], eta, M, x["dO"], norm)
    names = ["Q", "K", "V", "W1", "W2"]
    rng = np.random.default_rng(21)

    def obj(**over):
        a = {n: over.get(n, x[n]) for n in names}
        return orc.outer_objective(a["Q"], a["K"], a["V"], a["W1"], a["W2"], over.get("eta", eta), M, x["dO"], norm)

    gmap = dict(Q="dQ", K="dK", V="dV", W1="dW1_0", W2="dW2_0")
    for n in names:
        # every coordinate
        fd = np.zeros_like(x[n])
        for idx in np.ndindex(x[n].shape):
            e = np.zeros_like(x[n]); e[idx] = 1.0
            fd[idx] = fd_directional(lambda t: obj(**{n: t}), x[n], e, 1e-6)
        assert rel(g[gmap[n]], fd) < 1e-6, n
        # a random direction
        dirn = rng.standard_normal(x[n].shape)
        fdd = fd_directional(lambda t: obj(**{n: t}), x[n], dirn, 1e-6)
        assert abs(np.sum(g[gmap[n]] * dirn) - fdd) < 1e-6 * max(1.0, abs(fdd))
    fde = (obj(eta=eta + 1e-6) - obj(eta=eta - 1e-6)) / 2e-6
    assert abs(g["deta"].sum() - fde) < 1e-6 * max(1.0, abs(fde))


def torch_chain(Q, K, V, W1, W2, eta, M, norm=True):
    """Unrolled chain in torch; the inner gradient is taken by autograd."""
    N, H, d = K.shape
    outs = []
    for hd in range(H):
        q, k, v = Q[:, hd], K[:, hd], V[:, hd]
        if norm:
            q, k, v = (torch.nn.functional.normalize(t, dim=-1, eps=1e-12) for t in (q, k, v))
        w1, w2 = W1[hd], W2[hd]
        o = []
        for s in range(0, N, M):
            e = min(s + M, N)
            L = ((torch.nn.functional.silu(k[s:e] @ w1) @ w2 - v[s:e]) ** 2).sum(dim=1).mean()
            g1, g2 = torch.autograd.grad(L, (w1, w2), create_graph=True)
            w1 = w1 - eta * g1
            w2 = w2 - eta * g2
            o.append(torch.nn.functional.silu(q[s:e] @ w1) @ w2)
        outs.append(torch.cat(o, 0))
    return torch.stack(outs, 1)


def test_backward_matches_torch_double_autograd():
    x = f64(make_inputs(26, 2, 4, 6, seed=22, with_dO=True))
    eta, M = 0.3, 7
    g = orc.ttt_backward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], eta, M, x["dO"])
    t = {n: torch.from_numpy(x[n]).requires_grad_() for n in ["Q", "K", "V", "W1", "W2"]}
    te = torch.tensor(eta, dtype=torch.float64, requires_grad=True)
    O = torch_chain(t["Q"], t["K"], t["V"], t["W1"], t["W2"], te, M)
    assert rel(g["fwd"]["O"], O.detach().numpy()) < 1e-13
    (O * torch.from_numpy(x["dO"])).sum().backward()
    for n, gn in dict(Q="dQ", K="dK", V="dV", W1="dW1_0", W2="dW2_0").items():
        assert rel(g[gn], t[n].grad.numpy()) < 1e-11, n
    assert abs(g["deta"].sum() - te.grad.item()) < 1e-11 * max(1, abs(te.grad.item()))


def test_backward_at_eta_zero():
    """eta = 0: K and V do not influence O (dK = dV = 0 exactly) and dQ, dW0
    are the plain MLP's gradients."""
    x = f64(make_inputs(9, 1, 4, 6, seed=23, with_dO=True))
    g = orc.ttt_backward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.0, 4, x["dO"])
    assert not np.any(g["dK"]) and not np.any(g["dV"])
    tq = torch.from_numpy(x["Q"][:, 0]).requires_grad_()
    t1 = torch.from_numpy(x["W1"][0]).requires_grad_()
    t2 = torch.from_numpy(x["W2"][0]).requires_grad_()
    O = torch.nn.functional.silu(torch.nn.functional.normalize(tq, dim=-1) @ t1) @ t2
    (O * torch.from_numpy(x["dO"][:, 0])).sum().backward()
    assert rel(g["dQ"][:, 0], tq.grad.numpy()) < 1e-13
    assert rel(g["dW1_0"][0], t1.grad.numpy()) < 1e-13
    assert rel(g["dW2_0"][0], t2.grad.numpy()) < 1e-13
