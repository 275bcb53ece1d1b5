"""Pins of the oracle's layer around the memory unit (Sec. 4.2 projections,
Sec. 4.1 Eq. 5 gate), each against something other than the oracle itself:
exact identities of the gate, the invariance that the per-head L2
normalisation implies, and independent torch float64 implementations (plain
MLP at eta = 0; one chunk with the inner gradient taken by autograd)."""
import numpy as np
import torch
import torch.nn.functional as F

import oracle as orc
from workloads import make_layer_inputs

N, H, d, h, M, ETA = 37, 2, 8, 12, 16, 0.3


def layer(x, **kw):
    a = dict(X=x["X"], Wqkv=x["Wqkv"], Wo=x["Wo"], alpha=x["alpha"], W1_0=x["W1"], W2_0=x["W2"], eta=ETA,
             chunk_tokens=M, bqkv=x["bqkv"], bo=x["bo"])
    a.update(kw)
    return orc.gcm_layer_forward(**a)


def test_gate_off_returns_the_input():
    x = make_layer_inputs(N, H, d, h, seed=1)
    X = x["X"].astype(np.float64)
    assert np.array_equal(layer(x, alpha=np.zeros(H * d))["Y"], X)
    assert np.array_equal(layer(x, Wo=np.zeros((H * d, H * d)), bo=None)["Y"], X)


def test_per_head_scaling_of_the_projections_is_invisible():
    # Q, K and V are normalised per token and head, so scaling any head's
    # columns of any of the three blocks (and its bias) by a positive factor
    # changes nothing
    x = make_layer_inputs(N, H, d, h, seed=2)
    D = H * d
    s = np.ones(3 * D)
    rng = np.random.default_rng(0)
    for blk in range(3):
        for hd in range(H):
            s[blk * D + hd * d: blk * D + (hd + 1) * d] = rng.uniform(0.1, 5.0)
    ref = layer(x)["Y"]
    got = layer(x, Wqkv=x["Wqkv"] * s, bqkv=x["bqkv"] * s)["Y"]
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    # a scaling shared by the two heads' features of one block is invisible
    # too, but scaling a single feature is not (the normalisation is per head
    # and token, not per feature)
    s1 = np.ones(3 * D)
    s1[D + 3] = 4.0
    assert np.max(np.abs(layer(x, Wqkv=x["Wqkv"] * s1, bqkv=x["bqkv"] * s1)["Y"] - ref)) > 1e-6


def _torch_layer_eta0(x):
    X = torch.tensor(x["X"], dtype=torch.float64)
    D = H * d
    P = X @ torch.tensor(x["Wqkv"], dtype=torch.float64) + torch.tensor(x["bqkv"], dtype=torch.float64)
    Q = F.normalize(P[:, :D].reshape(N, H, d), dim=-1, eps=1e-12)
    O = torch.empty(N, H, d, dtype=torch.float64)
    for hd in range(H):
        W1 = torch.tensor(x["W1"][hd], dtype=torch.float64)
        W2 = torch.tensor(x["W2"][hd], dtype=torch.float64)
        O[:, hd] = F.silu(Q[:, hd] @ W1) @ W2
    G = O.reshape(N, D) @ torch.tensor(x["Wo"], dtype=torch.float64) + torch.tensor(x["bo"], dtype=torch.float64)
    return (torch.tensor(x["alpha"], dtype=torch.float64) * G + X).numpy()


def test_eta_zero_is_the_plain_layer():
    x = make_layer_inputs(N, H, d, h, seed=3)
    got = layer(x, eta=0.0)["Y"]
    ref = _torch_layer_eta0(x)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_one_chunk_against_autograd_inner_step():
    # one chunk: W1 = W0 - eta grad of the mean squared error of f_W(K) - V
    # (the inner gradient by torch autograd), then O = f_W1(Q) and the gate
    x = make_layer_inputs(N, H, d, h, seed=4)
    X = torch.tensor(x["X"], dtype=torch.float64)
    D = H * d
    P = X @ torch.tensor(x["Wqkv"], dtype=torch.float64) + torch.tensor(x["bqkv"], dtype=torch.float64)
    nq, nk, nv = (F.normalize(P[:, i * D:(i + 1) * D].reshape(N, H, d), dim=-1, eps=1e-12) for i in range(3))
    O = torch.empty(N, H, d, dtype=torch.float64)
    for hd in range(H):
        W1 = torch.tensor(x["W1"][hd], dtype=torch.float64, requires_grad=True)
        W2 = torch.tensor(x["W2"][hd], dtype=torch.float64, requires_grad=True)
        loss = ((F.silu(nk[:, hd] @ W1) @ W2 - nv[:, hd]) ** 2).sum(-1).mean()
        g1, g2 = torch.autograd.grad(loss, (W1, W2))
        with torch.no_grad():
            O[:, hd] = F.silu(nq[:, hd] @ (W1 - ETA * g1)) @ (W2 - ETA * g2)
    G = O.reshape(N, D) @ torch.tensor(x["Wo"], dtype=torch.float64) + torch.tensor(x["bo"], dtype=torch.float64)
    ref = (torch.tensor(x["alpha"], dtype=torch.float64) * G + X).numpy()
    got = layer(x, chunk_tokens=N)["Y"]
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))
    # the same with the key and value blocks exchanged differs: the roles of
    # the three blocks are pinned
    Wsw = x["Wqkv"].copy()
    Wsw[:, D:2 * D], Wsw[:, 2 * D:] = x["Wqkv"][:, 2 * D:], x["Wqkv"][:, D:2 * D]
    bsw = x["bqkv"].copy()
    bsw[D:2 * D], bsw[2 * D:] = x["bqkv"][2 * D:], x["bqkv"][D:2 * D]
    assert np.max(np.abs(layer(x, chunk_tokens=N, Wqkv=Wsw, bqkv=bsw)["Y"] - ref)) > 1e-6


def test_layer_backward_against_central_differences():
    # the directional derivative of <Y, dY> along a random direction in every
    # input at once, by central differences of the forward, against the
    # inner product of that direction with the reverse mode's gradients
    x = make_layer_inputs(N, H, d, h, seed=5)
    D = H * d
    rng = np.random.default_rng(6)
    dY = rng.standard_normal((N, D))
    names = ("X", "Wqkv", "Wo", "alpha", "W1", "W2", "bqkv", "bo")
    base = {k: x[k].astype(np.float64) for k in names}
    base["eta"] = ETA
    dirs = {k: rng.standard_normal(np.shape(base[k])) for k in names}
    dirs["eta"] = 0.7

    def objective(t):
        a = {k: base[k] + t * dirs[k] for k in base}
        y = orc.gcm_layer_forward(a["X"], a["Wqkv"], a["Wo"], a["alpha"], a["W1"], a["W2"], a["eta"], M,
                                  bqkv=a["bqkv"], bo=a["bo"])["Y"]
        return float(np.sum(y * dY))

    eps = 1e-5
    fd = (objective(eps) - objective(-eps)) / (2 * eps)
    g = orc.gcm_layer_backward(base["X"], base["Wqkv"], base["Wo"], base["alpha"], base["W1"], base["W2"], ETA, M,
                               dY, bqkv=base["bqkv"], bo=base["bo"])
    pairs = (("dX", "X"), ("dWqkv", "Wqkv"), ("dWo", "Wo"), ("dalpha", "alpha"), ("dW1_0", "W1"), ("dW2_0", "W2"),
             ("dbqkv", "bqkv"), ("dbo", "bo"))
    an = sum(float(np.sum(g[gk] * dirs[k])) for gk, k in pairs) + float(np.sum(g["deta"])) * dirs["eta"]
    assert abs(fd - an) <= 1e-7 * max(1.0, abs(fd)), (fd, an)
    # and each input's share on its own (a dropped or misplaced term would
    # cancel in the sum only by accident)
    for gk, k in pairs:
        one = {kk: (dirs[kk] if kk == k else np.zeros_like(np.asarray(dirs[kk], dtype=np.float64))) for kk in dirs}
        one["eta"] = 0.0

        def obj1(t):
            a = {kk: base[kk] + t * one[kk] for kk in base}
            y = orc.gcm_layer_forward(a["X"], a["Wqkv"], a["Wo"], a["alpha"], a["W1"], a["W2"], a["eta"], M,
                                      bqkv=a["bqkv"], bo=a["bo"])["Y"]
            return float(np.sum(y * dY))
        fd1 = (obj1(eps) - obj1(-eps)) / (2 * eps)
        an1 = float(np.sum(g[gk] * dirs[k]))
        assert abs(fd1 - an1) <= 1e-7 * max(1.0, abs(fd1)), (gk, fd1, an1)


def test_layer_backward_gate_off():
    # alpha = 0: Y = X, so dX = dY and nothing else but dalpha is non-zero
    x = make_layer_inputs(N, H, d, h, seed=8)
    dY = np.random.default_rng(9).standard_normal((N, H * d))
    g = orc.gcm_layer_backward(x["X"], x["Wqkv"], x["Wo"], np.zeros(H * d), x["W1"], x["W2"], ETA, M, dY,
                               bqkv=x["bqkv"], bo=x["bo"])
    assert np.array_equal(g["dX"], dY)
    for k in ("dWqkv", "dbqkv", "dWo", "dbo", "dW1_0", "dW2_0", "deta"):
        assert not np.any(g[k]), k
    G = orc.gcm_layer_forward(x["X"], x["Wqkv"], x["Wo"], np.ones(H * d), x["W1"], x["W2"], ETA, M, bqkv=x["bqkv"],
                              bo=x["bo"])["Y"] - x["X"]
    assert np.allclose(g["dalpha"], np.sum(G * dY, axis=0), rtol=1e-12, atol=0)
