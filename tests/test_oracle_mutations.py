"""The pins must catch plausible mistakes: plant each one in the oracle (on the
CPU, by monkeypatching) and check that an independent reference disagrees."""
import numpy as np
import torch

import oracle as orc
import oracle.ttt_oracle as T
from workloads import make_inputs
from test_oracle_backward_pins import torch_chain, f64, rel


def _bwd_error():
    x = f64(make_inputs(14, 1, 4, 6, seed=30, with_dO=True))
    g = orc.ttt_backward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.3, 5, x["dO"])
    t = {n: torch.from_numpy(x[n]).requires_grad_() for n in ["Q", "K", "V", "W1", "W2"]}
    O = torch_chain(t["Q"], t["K"], t["V"], t["W1"], t["W2"], 0.3, 5)
    (O * torch.from_numpy(x["dO"])).sum().backward()
    return max(rel(g[gn], t[n].grad.numpy()) for n, gn in
               dict(Q="dQ", K="dK", V="dV", W1="dW1_0", W2="dW2_0").items())


def _inner_grad_error():
    rng = np.random.default_rng(31)
    k = rng.standard_normal((6, 3)); v = rng.standard_normal((6, 3))
    W1 = rng.standard_normal((3, 4)); W2 = rng.standard_normal((4, 3))
    G1, G2, _, _ = orc.inner_grad(k, v, W1, W2)
    tk = torch.from_numpy(k); t1 = torch.from_numpy(W1).requires_grad_(); t2 = torch.from_numpy(W2).requires_grad_()
    L = ((torch.nn.functional.silu(tk @ t1) @ t2 - torch.from_numpy(v)) ** 2).sum(1).mean()
    g1, g2 = torch.autograd.grad(L, (t1, t2))
    return max(rel(G1, g1.numpy()), rel(G2, g2.numpy()))


def test_unmutated_baseline():
    assert _bwd_error() < 1e-10 and _inner_grad_error() < 1e-12


def test_wrong_second_derivative_is_caught(monkeypatch):
    good = T._silu_parts

    def bad(z):
        s, d1, d2 = good(z)
        return s, d1, -d2
    monkeypatch.setitem(T.ACTIVATIONS, "silu", bad)
    assert _bwd_error() > 1e-4


def test_dropped_first_derivative_term_is_caught(monkeypatch):
    good = T._silu_parts

    def bad(z):
        s, d1, d2 = good(z)
        from scipy.special import expit
        return s, expit(z), d2
    monkeypatch.setitem(T.ACTIVATIONS, "silu", bad)
    assert _inner_grad_error() > 1e-3


def test_dropped_factor_two_is_caught(monkeypatch):
    good = T.inner_grad

    def bad(k, v, W1, W2, act="silu"):
        G1, G2, l, c = good(k, v, W1, W2, act)
        return G1 / 2, G2 / 2, l, c
    monkeypatch.setattr(T, "inner_grad", bad)
    monkeypatch.setattr(orc, "inner_grad", bad)
    assert _inner_grad_error() > 0.1
    assert _bwd_error() > 1e-3


def test_wrong_norm_adjoint_is_caught(monkeypatch):
    def bad(x, dxhat, eps=T.NORM_EPS):
        xhat, den = T.l2norm_rows(x, eps)
        return dxhat / den          # projection term dropped
    monkeypatch.setattr(T, "l2norm_rows_bwd", bad)
    assert _bwd_error() > 1e-3


def test_apply_before_update_is_caught(monkeypatch):
    """If the apply used the pre-update weights, O would equal f_{W_c}(Q_c);
    the single-chunk pin (apply with W0 - eta grad) must then fail."""
    good_fast = T.fast_forward
    state = {}

    def stale_forward(x, W1, W2, act="silu"):
        if "prev" in state:
            W1, W2 = state.pop("prev")
        return good_fast(x, W1, W2, act)

    good_grad = T.inner_grad

    def spy_grad(k, v, W1, W2, act="silu"):
        state["prev"] = (W1, W2)
        return good_grad(k, v, W1, W2, act)
    monkeypatch.setattr(T, "fast_forward", stale_forward)
    monkeypatch.setattr(T, "inner_grad", spy_grad)
    x = f64(make_inputs(6, 1, 3, 4, seed=32))
    r = orc.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.5, 6)
    q = torch.nn.functional.normalize(torch.from_numpy(x["Q"][:, 0]), dim=-1).numpy()
    ref = torch.nn.functional.silu(torch.from_numpy(q @ r["W1_T"][0])).numpy() @ r["W2_T"][0]
    assert rel(r["O"][:, 0], ref) > 1e-3


def test_floor_branch_with_projection_is_caught(monkeypatch):
    """A norm adjoint that keeps the projection term (and divides by the
    true norm) on rows below the floor is caught by the floor-branch pin."""
    import test_oracle_pins as P

    def bad(x, dxhat, eps=T.NORM_EPS):
        xhat, den = T.l2norm_rows(x, eps)
        n = np.sqrt(np.sum(np.asarray(x, np.float64) ** 2, axis=-1, keepdims=True))
        proj = np.sum(xhat * dxhat, axis=-1, keepdims=True)
        return (dxhat - xhat * proj) / np.maximum(n, 1e-300)
    monkeypatch.setattr(T, "l2norm_rows_bwd", bad)
    monkeypatch.setattr(orc, "l2norm_rows_bwd", bad)
    try:
        P.test_l2norm_adjoint_floor_branch()
    except AssertionError:
        return
    raise AssertionError("the floor-branch pin did not catch the planted mistake")
