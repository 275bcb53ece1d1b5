"""Pins of the oracle's paper-AMU form: SwiGLU fast network (Supp. A),
dot-product inner loss (Eq. 9), token-wise step sizes inside the update
(Eq. 8), chain and synchronised (Eq. 10) semantics."""
import numpy as np
import torch

import oracle as orc
from test_oracle_backward_pins import rel


def rnd(seed, N=9, d=3, h=5):
    r = np.random.default_rng(seed)
    return (r.standard_normal((N, d)), r.standard_normal((N, d)), r.uniform(0.01, 0.2, N),
            r.standard_normal((d, h)) * 0.5, r.standard_normal((h, d)) * 0.5, r.standard_normal((d, h)) * 0.5)


def test_grad_matches_fd():
    k, v, et, W1, W2, W3 = rnd(50)
    G = orc.swiglu_dot_grad(k, v, et, W1, W2, W3)
    Ws = [W1, W2, W3]
    for i in range(3):
        fd = np.zeros_like(Ws[i])
        for idx in np.ndindex(Ws[i].shape):
            p = [w.copy() for w in Ws]
            m = [w.copy() for w in Ws]
            p[i][idx] += 1e-6
            m[i][idx] -= 1e-6
            fd[idx] = (orc.swiglu_dot_loss(k, v, et, *p) - orc.swiglu_dot_loss(k, v, et, *m)) / 2e-6
        assert rel(G[i], fd) < 1e-8, i


def test_grad_matches_torch_autograd():
    k, v, et, W1, W2, W3 = rnd(51, N=13, d=8, h=16)
    G = orc.swiglu_dot_grad(k, v, et, W1, W2, W3)
    t = [torch.from_numpy(w).requires_grad_() for w in (W1, W2, W3)]
    tk = torch.from_numpy(k)
    y = (torch.nn.functional.silu(tk @ t[0]) * (tk @ t[2])) @ t[1]
    L = -(torch.from_numpy(et)[:, None] * y * torch.from_numpy(v)).sum()
    g = torch.autograd.grad(L, t)
    for i in range(3):
        assert rel(G[i], g[i].numpy()) < 1e-12


def test_value_gradient_is_weight_free():
    """With the dot-product loss the output-side error E = -eta_i v_i does not
    depend on W, so grad W2 is linear in V: doubling V doubles every
    gradient."""
    k, v, et, W1, W2, W3 = rnd(52)
    a = orc.swiglu_dot_grad(k, v, et, W1, W2, W3)
    b = orc.swiglu_dot_grad(k, 2 * v, et, W1, W2, W3)
    for i in range(3):
        assert rel(b[i], 2 * a[i]) < 1e-14


def test_chain_one_chunk_equals_gcs_and_zero_eta():
    r = np.random.default_rng(53)
    N, H, d, h = 10, 2, 4, 6
    Q, K, V = (r.standard_normal((N, H, d)) for _ in range(3))
    W1, W3 = r.standard_normal((H, d, h)) / 2, r.standard_normal((H, d, h)) / 2
    W2 = r.standard_normal((H, h, d)) / 2
    et = r.uniform(0.0, 0.1, (N, H))
    a = orc.ttt_forward_swiglu(Q, K, V, W1, W2, W3, et, N, "chain")
    b = orc.ttt_forward_swiglu(Q, K, V, W1, W2, W3, et, N, "gcs")
    assert rel(a["O"], b["O"]) < 1e-14
    z = orc.ttt_forward_swiglu(Q, K, V, W1, W2, W3, np.zeros((N, H)), 4, "chain")
    q = torch.nn.functional.normalize(torch.from_numpy(Q[:, 0]), dim=-1)
    ref = (torch.nn.functional.silu(q @ torch.from_numpy(W1[0])) * (q @ torch.from_numpy(W3[0]))) @ torch.from_numpy(W2[0])
    assert rel(z["O"][:, 0], ref.numpy()) < 1e-13


def test_chain_steps_compose():
    """Chain form: the weights after chunk c are the FD-verified gradient step
    of chunk c applied to the weights after chunk c-1 (token-wise eta)."""
    r = np.random.default_rng(54)
    N, d, h = 11, 3, 4
    Q, K, V = (r.standard_normal((N, 1, d)) for _ in range(3))
    W = [r.standard_normal((1, d, h)) / 2, r.standard_normal((1, h, d)) / 2, r.standard_normal((1, d, h)) / 2]
    et = r.uniform(0.0, 0.3, (N, 1))
    res = orc.ttt_forward_swiglu(Q, K, V, W[0], W[1], W[2], et, 4, "chain")
    k = torch.nn.functional.normalize(torch.from_numpy(K[:, 0]), dim=-1).numpy()
    v = torch.nn.functional.normalize(torch.from_numpy(V[:, 0]), dim=-1).numpy()
    Wc = [w[0].copy() for w in W]
    for s, e in orc.chunk_bounds(N, 4):
        G = []
        for i in range(3):
            fd = np.zeros_like(Wc[i])
            for idx in np.ndindex(Wc[i].shape):
                p = [w.copy() for w in Wc]
                m = [w.copy() for w in Wc]
                p[i][idx] += 1e-6
                m[i][idx] -= 1e-6
                fd[idx] = (orc.swiglu_dot_loss(k[s:e], v[s:e], et[s:e, 0], *p)
                           - orc.swiglu_dot_loss(k[s:e], v[s:e], et[s:e, 0], *m)) / 2e-6
            G.append(fd)
        Wc = [Wc[i] - G[i] for i in range(3)]
    assert rel(res["W1_T"][0], Wc[0]) < 1e-7 and rel(res["W3_T"][0], Wc[2]) < 1e-7
