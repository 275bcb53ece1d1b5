"""Pins of the oracle's reverse mode of the paper-AMU form (SwiGLU fast
network, dot-product inner loss with token-wise step sizes; Supp. A, Eq. 8-10):
central finite differences of the outer loss sum <O, dO> for every input,
torch float64 autograd of an independent forward, and the eta = 0 case."""
import numpy as np
import pytest
import torch

import oracle as orc
from test_oracle_backward_pins import rel


def problem(seed, N=10, H=2, d=4, h=5, scale=0.6):
    r = np.random.default_rng(seed)
    Q, K, V, dO = (r.standard_normal((N, H, d)) for _ in range(4))
    W1, W3 = r.standard_normal((H, d, h)) * scale, r.standard_normal((H, d, h)) * scale
    W2 = r.standard_normal((H, h, d)) * scale
    et = r.uniform(0.2, 0.9, (N, H))
    return Q, K, V, W1, W2, W3, et, dO


def objective(Q, K, V, W1, W2, W3, et, M, dO, sync):
    return float(np.sum(orc.ttt_forward_swiglu(Q, K, V, W1, W2, W3, et, M, sync=sync)["O"] * dO))


@pytest.mark.parametrize("sync", ["chain", "gcs"])
def test_backward_matches_central_differences(sync):
    """Every input's gradient against central differences (step 1e-6) of the
    outer loss; chunks of 4 over 10 tokens (the last one ragged)."""
    Q, K, V, W1, W2, W3, et, dO = problem(70)
    M = 4
    g = orc.ttt_backward_swiglu(Q, K, V, W1, W2, W3, et, M, dO, sync=sync)
    args = dict(Q=Q, K=K, V=V, W1=W1, W2=W2, W3=W3, et=et)
    names = dict(Q="dQ", K="dK", V="dV", W1="dW1_0", W2="dW2_0", W3="dW3_0", et="deta_tok")
    for name, key in names.items():
        x = args[name]
        fd = np.zeros_like(x)
        for idx in np.ndindex(x.shape):
            p = {k: v.copy() for k, v in args.items()}
            m = {k: v.copy() for k, v in args.items()}
            p[name][idx] += 1e-6
            m[name][idx] -= 1e-6
            fd[idx] = (objective(p["Q"], p["K"], p["V"], p["W1"], p["W2"], p["W3"], p["et"], M, dO, sync)
                       - objective(m["Q"], m["K"], m["V"], m["W1"], m["W2"], m["W3"], m["et"], M, dO, sync)) / 2e-6
        assert rel(g[key], fd) < 1e-7, (sync, name, rel(g[key], fd))


def torch_forward(Q, K, V, W1, W2, W3, et, M, sync):
    """The same forward written independently in torch (float64), rows
    normalised, chunks of M: the reference for autograd."""
    nrm = lambda x: x / torch.clamp(torch.linalg.norm(x, dim=-1, keepdim=True), min=1e-12)
    q, k, v = nrm(Q), nrm(K), nrm(V)
    N, H, _ = Q.shape
    outs = []
    for hd in range(H):
        w = [W1[hd], W2[hd], W3[hd]]

        def f(x, w):
            return (torch.nn.functional.silu(x @ w[0]) * (x @ w[2])) @ w[1]

        def grad(kc, vc, ec, w):
            L = -(ec[:, None] * f(kc, w) * vc).sum()
            return torch.autograd.grad(L, w, create_graph=True)

        o = []
        if sync == "chain":
            for s in range(0, N, M):
                e = min(s + M, N)
                g = grad(k[s:e, hd], v[s:e, hd], et[s:e, hd], w)
                w = [w[i] - g[i] for i in range(3)]
                o.append(f(q[s:e, hd], w))
        else:
            tot = None
            for s in range(0, N, M):
                e = min(s + M, N)
                g = grad(k[s:e, hd], v[s:e, hd], et[s:e, hd], w)
                tot = list(g) if tot is None else [tot[i] + g[i] for i in range(3)]
            w = [w[i] - tot[i] for i in range(3)]
            o.append(f(q[:, hd], w))
        outs.append(torch.cat(o, 0))
    return torch.stack(outs, 1)


@pytest.mark.parametrize("sync", ["chain", "gcs"])
def test_backward_matches_torch_autograd(sync):
    """Second-order reverse mode through every inner update against torch's
    double-backward of an independently written forward (float64)."""
    Q, K, V, W1, W2, W3, et, dO = problem(71, N=23, H=2, d=8, h=12, scale=0.4)
    M = 6
    g = orc.ttt_backward_swiglu(Q, K, V, W1, W2, W3, et, M, dO, sync=sync)
    t = [torch.from_numpy(x).requires_grad_() for x in (Q, K, V, W1, W2, W3, et)]
    O = torch_forward(*t, M, sync)
    ref = torch.autograd.grad((O * torch.from_numpy(dO)).sum(), t)
    for key, r in zip(("dQ", "dK", "dV", "dW1_0", "dW2_0", "dW3_0", "deta_tok"), ref):
        assert rel(g[key], r.numpy()) < 1e-10, (sync, key, rel(g[key], r.numpy()))


def test_zero_steps():
    """With every eta_i = 0 the weights never move: dK = dV = 0, dW0 is the
    plain apply adjoint at W0 over all tokens, and deta_i is the derivative
    along each token's step size (non-zero)."""
    Q, K, V, W1, W2, W3, et, dO = problem(72, N=9, H=1, d=5, h=7)
    et = np.zeros_like(et)
    for sync in ("chain", "gcs"):
        g = orc.ttt_backward_swiglu(Q, K, V, W1, W2, W3, et, 3, dO, sync=sync)
        assert np.abs(g["dK"]).max() == 0.0 and np.abs(g["dV"]).max() == 0.0
        q = orc.l2norm_rows(Q[:, 0])[0]
        ga, dq = orc.swiglu_apply_adjoint(q, dO[:, 0], W1[0], W2[0], W3[0])
        assert rel(g["dW1_0"][0], ga[0]) < 1e-13 and rel(g["dW2_0"][0], ga[1]) < 1e-13
        assert rel(g["dW3_0"][0], ga[2]) < 1e-13
        assert np.abs(g["deta_tok"]).min() > 0.0


def _swiglu_bwd_error(sync="chain"):
    Q, K, V, W1, W2, W3, et, dO = problem(73, N=11, H=1, d=5, h=6, scale=0.5)
    g = orc.ttt_backward_swiglu(Q, K, V, W1, W2, W3, et, 4, dO, sync=sync)
    t = [torch.from_numpy(x).requires_grad_() for x in (Q, K, V, W1, W2, W3, et)]
    ref = torch.autograd.grad((torch_forward(*t, 4, sync) * torch.from_numpy(dO)).sum(), t)
    return max(rel(g[k], r.numpy()) for k, r in zip(("dQ", "dK", "dV", "dW1_0", "dW2_0", "dW3_0", "deta_tok"), ref))


def test_planted_mistakes_are_caught(monkeypatch):
    """A dropped second-derivative term, a dropped W-direction term of the
    tangent output and a dropped step-size factor each break the autograd
    agreement (mistakes planted in the oracle by monkeypatching)."""
    import oracle.ttt_oracle as T
    assert _swiglu_bwd_error() < 1e-10
    good_parts = T._silu_parts

    def no_second(z):
        s, d1, _ = good_parts(z)
        return s, d1, np.zeros_like(z)
    monkeypatch.setitem(T.ACTIVATIONS, "silu", no_second)
    assert _swiglu_bwd_error() > 1e-4
    monkeypatch.setitem(T.ACTIVATIONS, "silu", good_parts)
    good_upd = T.swiglu_update_adjoint

    def no_dv_eta(k, v, et, *w):
        gw, dk, dv, de = good_upd(k, v, et, *w)
        return gw, dk, dv / np.maximum(et[:, None], 1e-30), de
    monkeypatch.setattr(T, "swiglu_update_adjoint", no_dv_eta)
    assert _swiglu_bwd_error("gcs") > 1e-4
    monkeypatch.setattr(T, "swiglu_update_adjoint", good_upd)

    def no_wh2(k, v, et, W1, W2, W3, Wh1, Wh2, Wh3):
        return good_upd(k, v, et, W1, W2, W3, Wh1, np.zeros_like(Wh2), Wh3)
    monkeypatch.setattr(T, "swiglu_update_adjoint", no_wh2)
    assert _swiglu_bwd_error() > 1e-4
