"""Pins of the FP64 oracle against facts fixed by mathematics, not by itself.

Every check here is independent of the oracle's own formulas: finite
differences, torch float64 autograd (a library's derivatives), closed forms
of special cases, and invariants of the method (Sec. 3.2 Eq. 3-4, Sec. 4.2
Eq. 8 and Eq. 10).  The paper prints no worked numerical example, so no
golden value comes from it."""
import numpy as np
import pytest
import torch

import oracle as orc
from workloads import make_inputs


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def tiny(N=11, H=1, d=3, h=5, seed=0):
    x = make_inputs(N, H, d, h, seed=seed)
    return {k: v.astype(np.float64) for k, v in x.items()}


# ---------------------------------------------------------------- inner step

def test_inner_grad_matches_central_fd():
    """Eq. 8 gradient of the chunk loss, every entry, brute-force FD."""
    rng = np.random.default_rng(1)
    k = rng.standard_normal((7, 3))
    v = rng.standard_normal((7, 3))
    W1 = rng.standard_normal((3, 5)) * 0.6
    W2 = rng.standard_normal((5, 3)) * 0.6
    G1, G2, _, _ = orc.inner_grad(k, v, W1, W2)
    step = 1e-6
    for W, G, which in ((W1, G1, 1), (W2, G2, 2)):
        fd = np.zeros_like(W)
        for idx in np.ndindex(W.shape):
            Wp = W.copy(); Wp[idx] += step
            Wm = W.copy(); Wm[idx] -= step
            args_p = (k, v, Wp, W2) if which == 1 else (k, v, W1, Wp)
            args_m = (k, v, Wm, W2) if which == 1 else (k, v, W1, Wm)
            fd[idx] = (orc.inner_loss(*args_p) - orc.inner_loss(*args_m)) / (2 * step)
        assert rel(G, fd) < 1e-8


def test_inner_grad_matches_torch_autograd():
    rng = np.random.default_rng(2)
    k = rng.standard_normal((13, 8))
    v = rng.standard_normal((13, 8))
    W1 = rng.standard_normal((8, 16)) / np.sqrt(8)
    W2 = rng.standard_normal((16, 8)) / 4
    G1, G2, loss, _ = orc.inner_grad(k, v, W1, W2)
    tk, tv = torch.from_numpy(k), torch.from_numpy(v)
    t1 = torch.from_numpy(W1).requires_grad_()
    t2 = torch.from_numpy(W2).requires_grad_()
    L = ((torch.nn.functional.silu(tk @ t1) @ t2 - tv) ** 2).sum(dim=1).mean()
    g1, g2 = torch.autograd.grad(L, (t1, t2))
    assert abs(L.item() - loss) < 1e-12
    assert rel(G1, g1.numpy()) < 1e-12
    assert rel(G2, g2.numpy()) < 1e-12


def test_identity_activation_closed_form():
    """With s = identity, f(x) = x W1 W2 and the gradient has the closed form
    grad W1 = (2/M) K^T R W2^T, grad W2 = (2/M) (K W1)^T R."""
    rng = np.random.default_rng(3)
    M = 9
    k = rng.standard_normal((M, 4)); v = rng.standard_normal((M, 4))
    W1 = rng.standard_normal((4, 6)); W2 = rng.standard_normal((6, 4))
    G1, G2, _, _ = orc.inner_grad(k, v, W1, W2, act="identity")
    R = k @ W1 @ W2 - v
    assert rel(G1, (2.0 / M) * k.T @ R @ W2.T) < 1e-13
    assert rel(G2, (2.0 / M) * (k @ W1).T @ R) < 1e-13


def test_silu_derivatives_match_fd():
    z = np.linspace(-8, 8, 101)
    s, d1, d2 = orc.activation(z)
    step = 1e-5
    sp, d1p, _ = orc.activation(z + step)
    sm, d1m, _ = orc.activation(z - step)
    assert np.max(np.abs((sp - sm) / (2 * step) - d1)) < 1e-9
    assert np.max(np.abs((d1p - d1m) / (2 * step) - d2)) < 1e-9
    assert np.allclose(s, torch.nn.functional.silu(torch.from_numpy(z)).numpy(), rtol=0, atol=1e-15)


# ---------------------------------------------------------------- forward chain

def test_eta_zero_is_plain_mlp():
    x = tiny(N=23, H=2, d=6, h=10)
    r = orc.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.0, 5)
    for hd in range(2):
        q = torch.nn.functional.normalize(torch.from_numpy(x["Q"][:, hd]), dim=-1, eps=1e-12)
        ref = torch.nn.functional.silu(q @ torch.from_numpy(x["W1"][hd])) @ torch.from_numpy(x["W2"][hd])
        assert rel(r["O"][:, hd], ref.numpy()) < 1e-13
    assert np.array_equal(r["W1_T"], x["W1"]) and np.array_equal(r["W2_T"], x["W2"])
    assert np.array_equal(r["ckpt1"][-1], x["W1"])


def fd_grad_fn(k, v, W1, W2, step=1e-6):
    G = []
    for which, W in ((1, W1), (2, W2)):
        g = np.zeros_like(W)
        for idx in np.ndindex(W.shape):
            Wp = W.copy(); Wp[idx] += step
            Wm = W.copy(); Wm[idx] -= step
            a = orc.inner_loss(k, v, Wp, W2) if which == 1 else orc.inner_loss(k, v, W1, Wp)
            b = orc.inner_loss(k, v, Wm, W2) if which == 1 else orc.inner_loss(k, v, W1, Wm)
            g[idx] = (a - b) / (2 * step)
        G.append(g)
    return G


@pytest.mark.parametrize("eta", [1e-3, 0.1, 0.7])
def test_single_chunk_step_and_apply_after_update(eta):
    """One chunk (C = 1): W_T = W0 - eta * grad L(W0) with the gradient by FD,
    and O = f_{W_T}(Q) (apply after the update)."""
    x = tiny(N=6, H=1, d=3, h=4, seed=4)
    r = orc.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], eta, 6)
    q, k, v = (torch.nn.functional.normalize(torch.from_numpy(x[n][:, 0]), dim=-1).numpy() for n in "QKV")
    g1, g2 = fd_grad_fn(k, v, x["W1"][0], x["W2"][0])
    W1 = x["W1"][0] - eta * g1
    W2 = x["W2"][0] - eta * g2
    assert rel(r["W1_T"][0], W1) < 1e-8 and rel(r["W2_T"][0], W2) < 1e-8
    ref = torch.nn.functional.silu(torch.from_numpy(q @ W1)).numpy() @ W2
    assert rel(r["O"][:, 0], ref) < 1e-8


def test_ragged_chain_composes_fd_steps():
    """Three chunks (4, 4, 3 tokens): each chunk's weights come from the
    previous by an FD-gradient step normalised by that chunk's own size."""
    x = tiny(N=11, H=1, d=3, h=4, seed=5)
    eta = 0.3
    r = orc.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], eta, 4)
    q, k, v = (torch.nn.functional.normalize(torch.from_numpy(x[n][:, 0]), dim=-1).numpy() for n in "QKV")
    W1, W2 = x["W1"][0].copy(), x["W2"][0].copy()
    for c, (s, e) in enumerate([(0, 4), (4, 8), (8, 11)]):
        assert rel(r["ckpt1"][c, 0], W1) < 1e-8
        g1, g2 = fd_grad_fn(k[s:e], v[s:e], W1, W2)
        W1, W2 = W1 - eta * g1, W2 - eta * g2
        ref = torch.nn.functional.silu(torch.from_numpy(q[s:e] @ W1)).numpy() @ W2
        assert rel(r["O"][s:e, 0], ref) < 1e-7
    assert rel(r["W1_T"][0], W1) < 1e-8


def test_loss_non_increasing_small_eta():
    """For a small step the chunk's own loss does not increase."""
    x = make_inputs(1374, 1, 64, 128, seed=0)
    k = orc.l2norm_rows(x["K"][:, 0])[0]
    v = orc.l2norm_rows(x["V"][:, 0])[0]
    W1 = x["W1"][0].astype(np.float64); W2 = x["W2"][0].astype(np.float64)
    for eta in (1e-3, 1e-2, 0.1):
        G1, G2, l0, _ = orc.inner_grad(k, v, W1, W2)
        l1 = orc.inner_loss(k, v, W1 - eta * G1, W2 - eta * G2)
        assert l1 <= l0


def test_token_shard_additivity():
    """Eq. 10: the gradient of a chunk is the sum of shard gradients taken with
    the chunk's own 1/M (shard gradients with 1/M_s weighted by M_s/M)."""
    rng = np.random.default_rng(6)
    M = 29
    k = rng.standard_normal((M, 5)); v = rng.standard_normal((M, 5))
    W1 = rng.standard_normal((5, 7)) * 0.5; W2 = rng.standard_normal((7, 5)) * 0.5
    G1, G2, _, _ = orc.inner_grad(k, v, W1, W2)
    S1 = np.zeros_like(G1); S2 = np.zeros_like(G2)
    for s, e in [(0, 8), (8, 9), (9, 20), (20, 29)]:
        g1, g2, _, _ = orc.inner_grad(k[s:e], v[s:e], W1, W2)
        S1 += (e - s) / M * g1; S2 += (e - s) / M * g2
    assert rel(G1, S1) < 1e-13 and rel(G2, S2) < 1e-13


def test_permutation_within_chunk():
    x = tiny(N=12, H=1, d=4, h=6, seed=7)
    r = orc.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.2, 4)
    perm = np.concatenate([np.random.default_rng(8).permutation(4) + 4 * c for c in range(3)])
    rp = orc.ttt_forward(x["Q"][perm], x["K"][perm], x["V"][perm], x["W1"], x["W2"], 0.2, 4)
    assert rel(rp["O"], r["O"][perm]) < 1e-13
    assert rel(rp["W1_T"], r["W1_T"]) < 1e-13


def test_heads_independent():
    x = tiny(N=10, H=3, d=4, h=6, seed=9)
    r = orc.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.2, 3)
    r1 = orc.ttt_forward(x["Q"][:, 1:2], x["K"][:, 1:2], x["V"][:, 1:2], x["W1"][1:2], x["W2"][1:2], 0.2, 3)
    assert np.array_equal(r["O"][:, 1:2], r1["O"]) and np.array_equal(r["W2_T"][1:2], r1["W2_T"])


def test_split_call_resume():
    x = tiny(N=14, H=2, d=4, h=6, seed=10)
    full = orc.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.2, 4)
    a = orc.ttt_forward(x["Q"][:8], x["K"][:8], x["V"][:8], x["W1"], x["W2"], 0.2, 4)
    b = orc.ttt_forward(x["Q"][8:], x["K"][8:], x["V"][8:], a["W1_T"], a["W2_T"], 0.2, 4)
    assert np.array_equal(np.concatenate([a["O"], b["O"]]), full["O"])
    assert np.array_equal(b["W1_T"], full["W1_T"])


def test_batched_is_per_sequence():
    x = tiny(N=17, H=2, d=4, h=6, seed=11)
    cu = [0, 5, 6, 17]
    r = orc.ttt_forward_batched(x["Q"], x["K"], x["V"], cu, x["W1"], x["W2"], 0.2, 4)
    for b in range(3):
        s, e = cu[b], cu[b + 1]
        rb = orc.ttt_forward(x["Q"][s:e], x["K"][s:e], x["V"][s:e], x["W1"], x["W2"], 0.2, 4)
        assert np.array_equal(r["O"][s:e], rb["O"])


def test_l2norm_and_adjoint():
    rng = np.random.default_rng(12)
    x = rng.standard_normal((5, 7))
    xh, _ = orc.l2norm_rows(x)
    assert np.allclose(xh, torch.nn.functional.normalize(torch.from_numpy(x), dim=-1).numpy(), atol=1e-15)
    dxh = rng.standard_normal((5, 7))
    dx = orc.l2norm_rows_bwd(x, dxh)
    tx = torch.from_numpy(x).requires_grad_()
    (torch.nn.functional.normalize(tx, dim=-1) * torch.from_numpy(dxh)).sum().backward()
    assert rel(dx, tx.grad.numpy()) < 1e-13
    z = np.zeros((1, 3))
    assert np.array_equal(orc.l2norm_rows(z)[0], z)


def test_l2norm_adjoint_floor_branch():
    """Rows whose norm is below the floor eps = 1e-12 are divided by the
    constant eps, so their adjoint is dxhat / eps with no projection term.
    Pinned against torch autograd of F.normalize (which clamps the norm
    from below at the same eps) on rows above, at and below the floor."""
    rng = np.random.default_rng(13)
    x = rng.standard_normal((6, 5))
    x[1] *= 1e-14   # norm ~2e-14: floor active
    x[2] *= 3e-13   # norm ~6e-13: floor active
    x[3] = 0.0      # zero row: floor active, xhat = 0
    x[4] *= 1e-11   # norm ~2e-11: above the floor
    dxh = rng.standard_normal((6, 5))
    dx = orc.l2norm_rows_bwd(x, dxh)
    tx = torch.from_numpy(x).requires_grad_()
    (torch.nn.functional.normalize(tx, dim=-1, eps=orc.NORM_EPS) * torch.from_numpy(dxh)).sum().backward()
    g = tx.grad.numpy()
    for i in range(6):
        assert rel(dx[i], g[i]) < 1e-12, i
    # the floor rows carry no projection term: exactly dxhat / eps
    assert np.allclose(dx[1], dxh[1] / orc.NORM_EPS, rtol=1e-15, atol=0)
    assert np.allclose(dx[3], dxh[3] / orc.NORM_EPS, rtol=1e-15, atol=0)
