"""FP64 CPU oracle for chunked test-time training (TTT) of a 2-layer fast MLP.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the smoke check
and the benchmark's CPU-baseline leg may import this module.  It shares no
code with the HIP path and never imports it.

What is computed (per sequence and head, heads independent):

* the fast network is ``f_W(x) = SiLU(x W1) W2`` with ``W1: [d][h]`` and
  ``W2: [h][d]`` (row-vector convention of the per-head matrices in Supp. A);
* the token stream is walked chunk by chunk; all tokens of a chunk form one
  update unit (Sec. 4.2, chunk-wise update, Eq. 8);
* the inner loss of chunk c is the mean over its M_c tokens of the squared
  error ``||f_W(k_i) - v_i||^2`` (readings: mean over tokens, sum over the
  feature axis, no 1/2 factor);
* the step is ``W <- W - eta * grad_W L_c`` (TTT update, Sec. 3.2 Eq. 3);
* after the step the chunk's queries are mapped, ``O_c = f_W(Q_c)`` (TTT
  apply, Sec. 3.2 Eq. 4; "after the update" in Sec. 4.2).

Q, K and V are L2-normalised per token and head, ``x / max(||x||, 1e-12)``,
inside the differentiated function (an input-preparation reading; the paper
does not mention it).

The backward pass is the hand-derived reverse mode of the whole chain of inner
updates, second-order terms through the inner gradient included, for the
outer loss ``sum <O, dO>``.

Every formula is plain numpy in float64; the loops follow the paper's order
(chunks in sequence order).  Nothing here is blocked, fused or reordered.

Parity pins (tests/test_oracle_*.py): central finite differences, torch
float64 autograd, the identity-activation closed form, eta=0, first-step
linearity in eta, loss decrease, token-shard additivity (Eq. 10),
permutation within a chunk, head independence, split-call resume.
"""
from __future__ import annotations

import numpy as np
from scipy.special import expit

NORM_EPS = 1e-12


# --------------------------------------------------------------------------
# activations: SiLU (the fast MLP's non-linearity) and identity (a pinning aid)
# --------------------------------------------------------------------------

def _silu_parts(z):
    """Return (s(z), s'(z), s''(z)) for s(z) = z * sigmoid(z)."""
    sg = expit(z)
    s = z * sg
    d1 = sg * (1.0 + z * (1.0 - sg))
    d2 = sg * (1.0 - sg) * (2.0 + z * (1.0 - 2.0 * sg))
    return s, d1, d2


def _identity_parts(z):
    return z.copy(), np.ones_like(z), np.zeros_like(z)


ACTIVATIONS = {"silu": _silu_parts, "identity": _identity_parts}


def activation(z, act="silu"):
    return ACTIVATIONS[act](np.asarray(z, dtype=np.float64))


# --------------------------------------------------------------------------
# per-token L2 normalisation and its adjoint
# --------------------------------------------------------------------------

def l2norm_rows(x, eps=NORM_EPS):
    """x / max(||x||_2, eps) along the last axis; returns (xhat, denom)."""
    x = np.asarray(x, dtype=np.float64)
    n = np.sqrt(np.sum(x * x, axis=-1, keepdims=True))
    den = np.maximum(n, eps)
    return x / den, den


def l2norm_rows_bwd(x, dxhat, eps=NORM_EPS):
    """Adjoint of l2norm_rows: (dxhat - xhat (xhat . dxhat)) / ||x|| where
    ||x|| > eps, and dxhat / eps where the floor is active."""
    xhat, den = l2norm_rows(x, eps)
    n = np.sqrt(np.sum(np.asarray(x, np.float64) ** 2, axis=-1, keepdims=True))
    proj = np.sum(xhat * dxhat, axis=-1, keepdims=True)
    above = (dxhat - xhat * proj) / den
    floor = dxhat / eps
    return np.where(n > eps, above, floor)


# --------------------------------------------------------------------------
# chunking
# --------------------------------------------------------------------------

def chunk_bounds(n_tokens, chunk_tokens):
    """Non-overlapping token ranges [c*M, min((c+1)*M, N)); the last chunk may
    be ragged.  N = 0 gives no chunks."""
    if chunk_tokens < 1:
        raise ValueError("chunk_tokens must be >= 1")
    return [(s, min(s + chunk_tokens, n_tokens)) for s in range(0, n_tokens, chunk_tokens)]


# --------------------------------------------------------------------------
# the inner problem of one chunk (Eq. 8 with the MSE loss)
# --------------------------------------------------------------------------

def fast_forward(x, W1, W2, act="silu"):
    """f_W(x) = s(x W1) W2 for rows x."""
    s, _, _ = activation(x @ W1, act)
    return s @ W2


def inner_loss(k, v, W1, W2, act="silu"):
    """L_c(W) = (1/M_c) * sum_i ||f_W(k_i) - v_i||^2."""
    r = fast_forward(k, W1, W2, act) - v
    return float(np.sum(r * r) / k.shape[0])


def inner_grad(k, v, W1, W2, act="silu"):
    """Hand-derived gradient of inner_loss with respect to (W1, W2).

    Z = k W1, A = s(Z), R = A W2 - v, E = (2/M) R, P = E W2^T, D = P * s'(Z),
    grad W1 = k^T D, grad W2 = A^T E.  Returns (G1, G2, loss, cache)."""
    m = k.shape[0]
    Z = k @ W1
    A, S1, S2 = activation(Z, act)
    R = A @ W2 - v
    loss = float(np.sum(R * R) / m)
    E = (2.0 / m) * R
    P = E @ W2.T
    D = P * S1
    G1 = k.T @ D
    G2 = A.T @ E
    cache = dict(Z=Z, A=A, S1=S1, S2=S2, E=E, P=P, D=D)
    return G1, G2, loss, cache


# --------------------------------------------------------------------------
# forward chain
# --------------------------------------------------------------------------

def _as_f64(*xs):
    return [np.asarray(x, dtype=np.float64) for x in xs]


def _prep(x, do_norm):
    if do_norm:
        return l2norm_rows(x)[0]
    return np.asarray(x, dtype=np.float64)


def ttt_forward(Q, K, V, W1_0, W2_0, eta, chunk_tokens, norm=(True, True, True), act="silu"):
    """Chunked TTT forward for one sequence.

    Q, K, V: [N][H][d] raw tokens; W1_0: [H][d][h]; W2_0: [H][h][d].
    Returns dict with O [N][H][d], W1_T, W2_T (final fast weights),
    ckpt1 [C][H][d][h], ckpt2 [C][H][h][d] (weights *before* chunk c) and
    loss [H][C] (inner loss of chunk c at the weights before its step)."""
    Q, K, V, W1_0, W2_0 = _as_f64(Q, K, V, W1_0, W2_0)
    N, H, d = K.shape
    h = W1_0.shape[-1]
    bounds = chunk_bounds(N, chunk_tokens)
    C = len(bounds)
    O = np.zeros((N, H, d))
    ckpt1 = np.zeros((C, H, d, h))
    ckpt2 = np.zeros((C, H, h, d))
    loss = np.zeros((H, C))
    W1_T = W1_0.copy()
    W2_T = W2_0.copy()
    for hd in range(H):
        q = _prep(Q[:, hd, :], norm[0])
        k = _prep(K[:, hd, :], norm[1])
        v = _prep(V[:, hd, :], norm[2])
        W1 = W1_0[hd].copy()
        W2 = W2_0[hd].copy()
        for c, (s, e) in enumerate(bounds):
            ckpt1[c, hd] = W1
            ckpt2[c, hd] = W2
            G1, G2, l, _ = inner_grad(k[s:e], v[s:e], W1, W2, act)
            loss[hd, c] = l
            W1 = W1 - eta * G1
            W2 = W2 - eta * G2
            O[s:e, hd, :] = fast_forward(q[s:e], W1, W2, act)
        W1_T[hd] = W1
        W2_T[hd] = W2
    return dict(O=O, W1_T=W1_T, W2_T=W2_T, ckpt1=ckpt1, ckpt2=ckpt2, loss=loss)


def ttt_forward_batched(Q, K, V, cu_seqlens, W1_0, W2_0, eta, chunk_tokens,
                        w0_per_seq=False, norm=(True, True, True), act="silu"):
    """Many sequences packed along the token axis, [sum N_b][H][d], with
    boundaries cu_seqlens [B+1].  Each sequence runs its own chain from its
    initial weights (shared [H][..] or per sequence [B][H][..])."""
    cu = [int(x) for x in cu_seqlens]
    Q, K, V, W1_0, W2_0 = _as_f64(Q, K, V, W1_0, W2_0)
    B = len(cu) - 1
    O = np.zeros_like(Q)
    W1_T = np.zeros((B,) + W1_0.shape[-3:])
    W2_T = np.zeros((B,) + W2_0.shape[-3:])
    for b in range(B):
        s, e = cu[b], cu[b + 1]
        w1 = W1_0[b] if w0_per_seq else W1_0
        w2 = W2_0[b] if w0_per_seq else W2_0
        r = ttt_forward(Q[s:e], K[s:e], V[s:e], w1, w2, eta, chunk_tokens, norm, act)
        O[s:e] = r["O"]
        W1_T[b] = r["W1_T"]
        W2_T[b] = r["W2_T"]
    return dict(O=O, W1_T=W1_T, W2_T=W2_T)


# --------------------------------------------------------------------------
# backward through the whole chain (second-order terms included)
# --------------------------------------------------------------------------

def ttt_backward(Q, K, V, W1_0, W2_0, eta, chunk_tokens, dO, norm=(True, True, True), act="silu"):
    """Reverse mode of ttt_forward for the outer loss sum <O, dO>.

    Walks chunks backwards carrying the adjoints (Wh1, Wh2) of the weights
    *after* chunk c.  Per chunk, with W = W_c recomputed from the forward:

    apply adjoint (O_c = s(q W1') W2' with W' = W_{c+1}):
        Wh2 += Aq^T dO,  dZq = (dO W2'^T) * s'(Zq),  Wh1 += q^T dZq,
        dq = dZq W1'^T
    update adjoint (W' = W - eta * grad):
        deta += -<k Wh1, D> - <A Wh2, E>
        dD = -eta k Wh1,  dk = -eta D Wh1^T,  dA = -eta E Wh2^T,  dE = -eta A Wh2
        dP = dD * s'(Z),  dZ = dD * P * s''(Z)
        dE += dP W2,  dW2 = Wh2 + dP^T E
        dY = (2/M) dE,  dv = -dY
        dA += dY W2^T,  dW2 += A^T dY
        dZ += dA * s'(Z),  dk += dZ W1^T,  dW1 = Wh1 + k^T dZ
    then (Wh1, Wh2) <- (dW1, dW2).  Finally the L2-norm adjoint maps
    dq, dk, dv to the raw inputs.

    Returns dict dQ, dK, dV [N][H][d], dW1_0 [H][d][h], dW2_0 [H][h][d],
    deta [H] (per head; the scalar eta's gradient is their sum)."""
    Q, K, V, W1_0, W2_0, dO = _as_f64(Q, K, V, W1_0, W2_0, dO)
    N, H, d = K.shape
    bounds = chunk_bounds(N, chunk_tokens)
    fwd = ttt_forward(Q, K, V, W1_0, W2_0, eta, chunk_tokens, norm, act)
    dQ = np.zeros_like(Q)
    dK = np.zeros_like(K)
    dV = np.zeros_like(V)
    dW1_0 = np.zeros_like(W1_0)
    dW2_0 = np.zeros_like(W2_0)
    deta = np.zeros(H)
    C = len(bounds)
    for hd in range(H):
        q = _prep(Q[:, hd, :], norm[0])
        k = _prep(K[:, hd, :], norm[1])
        v = _prep(V[:, hd, :], norm[2])
        dq = np.zeros_like(q)
        dk = np.zeros_like(k)
        dv = np.zeros_like(v)
        Wh1 = np.zeros_like(W1_0[hd])
        Wh2 = np.zeros_like(W2_0[hd])
        for c in range(C - 1, -1, -1):
            s, e = bounds[c]
            m = e - s
            W1 = fwd["ckpt1"][c, hd]
            W2 = fwd["ckpt2"][c, hd]
            kc, vc, qc, dOc = k[s:e], v[s:e], q[s:e], dO[s:e, hd, :]
            G1, G2, _, cc = inner_grad(kc, vc, W1, W2, act)
            W1n = W1 - eta * G1
            W2n = W2 - eta * G2
            # apply adjoint
            Zq = qc @ W1n
            Aq, Sq1, _ = activation(Zq, act)
            Wh2 = Wh2 + Aq.T @ dOc
            dZq = (dOc @ W2n.T) * Sq1
            Wh1 = Wh1 + qc.T @ dZq
            dq[s:e] += dZq @ W1n.T
            # update adjoint
            A, S1, S2 = cc["A"], cc["S1"], cc["S2"]
            E, P, D = cc["E"], cc["P"], cc["D"]
            kWh1 = kc @ Wh1
            AWh2 = A @ Wh2
            deta[hd] += -np.sum(kWh1 * D) - np.sum(AWh2 * E)
            dD = -eta * kWh1
            dkc = -eta * (D @ Wh1.T)
            dA = -eta * (E @ Wh2.T)
            dE = -eta * AWh2
            dP = dD * S1
            dZ = dD * P * S2
            dE = dE + dP @ W2
            dW2 = Wh2 + dP.T @ E
            dY = (2.0 / m) * dE
            dv[s:e] += -dY
            dA = dA + dY @ W2.T
            dW2 = dW2 + A.T @ dY
            dZ = dZ + dA * S1
            dkc = dkc + dZ @ W1.T
            dW1 = Wh1 + kc.T @ dZ
            dk[s:e] += dkc
            Wh1, Wh2 = dW1, dW2
        dW1_0[hd] = Wh1
        dW2_0[hd] = Wh2
        dQ[:, hd, :] = l2norm_rows_bwd(Q[:, hd, :], dq) if norm[0] else dq
        dK[:, hd, :] = l2norm_rows_bwd(K[:, hd, :], dk) if norm[1] else dk
        dV[:, hd, :] = l2norm_rows_bwd(V[:, hd, :], dv) if norm[2] else dv
    return dict(dQ=dQ, dK=dK, dV=dV, dW1_0=dW1_0, dW2_0=dW2_0, deta=deta, fwd=fwd)


def ttt_backward_batched(Q, K, V, cu_seqlens, W1_0, W2_0, eta, chunk_tokens, dO,
                         w0_per_seq=False, norm=(True, True, True), act="silu"):
    """Reverse mode of ttt_forward_batched for sum <O, dO> over all
    sequences.  Sequences are independent chains, so each one is ttt_backward
    on its own token range; a shared W0 (and the shared eta) receives the sum
    of the sequences' gradients."""
    cu = [int(x) for x in cu_seqlens]
    Q, K, V, W1_0, W2_0, dO = _as_f64(Q, K, V, W1_0, W2_0, dO)
    B = len(cu) - 1
    dQ, dK, dV = np.zeros_like(Q), np.zeros_like(K), np.zeros_like(V)
    dW1 = np.zeros_like(W1_0)
    dW2 = np.zeros_like(W2_0)
    deta = np.zeros(Q.shape[1])
    for b in range(B):
        s, e = cu[b], cu[b + 1]
        w1 = W1_0[b] if w0_per_seq else W1_0
        w2 = W2_0[b] if w0_per_seq else W2_0
        if e == s:
            continue
        r = ttt_backward(Q[s:e], K[s:e], V[s:e], w1, w2, eta, chunk_tokens, dO[s:e], norm, act)
        dQ[s:e], dK[s:e], dV[s:e] = r["dQ"], r["dK"], r["dV"]
        if w0_per_seq:
            dW1[b], dW2[b] = r["dW1_0"], r["dW2_0"]
        else:
            dW1 += r["dW1_0"]
            dW2 += r["dW2_0"]
        deta += r["deta"]
    return dict(dQ=dQ, dK=dK, dV=dV, dW1_0=dW1, dW2_0=dW2, deta=deta)


def outer_objective(Q, K, V, W1_0, W2_0, eta, chunk_tokens, dO, norm=(True, True, True), act="silu"):
    """sum <O, dO>: the scalar whose gradient ttt_backward returns."""
    O = ttt_forward(Q, K, V, W1_0, W2_0, eta, chunk_tokens, norm, act)["O"]
    return float(np.sum(O * np.asarray(dO, np.float64)))


# --------------------------------------------------------------------------
# Global Context Synchronization form (Sec. 4.2, Eq. 10)
# --------------------------------------------------------------------------

def ttt_forward_gcs(Q, K, V, W1_0, W2_0, eta, chunk_tokens, norm=(True, True, True), act="silu"):
    """GCS semantics for one sequence: every chunk's gradient is taken at the
    same initial weights, the gradients are summed over chunks (Eq. 10: the
    synchronised gradient is the sum of the per-chunk gradients), one step
    W* = W0 - eta * g is applied, and every chunk's queries are mapped with
    W*.  With one chunk this is the chain form.  Returns O, W1_T, W2_T (= W*)
    and loss [H][C] (each chunk's loss at W0)."""
    Q, K, V, W1_0, W2_0 = _as_f64(Q, K, V, W1_0, W2_0)
    N, H, d = K.shape
    bounds = chunk_bounds(N, chunk_tokens)
    O = np.zeros((N, H, d))
    W1_T = W1_0.copy()
    W2_T = W2_0.copy()
    loss = np.zeros((H, len(bounds)))
    for hd in range(H):
        q = _prep(Q[:, hd, :], norm[0])
        k = _prep(K[:, hd, :], norm[1])
        v = _prep(V[:, hd, :], norm[2])
        g1 = np.zeros_like(W1_0[hd])
        g2 = np.zeros_like(W2_0[hd])
        for c, (s, e) in enumerate(bounds):
            G1, G2, l, _ = inner_grad(k[s:e], v[s:e], W1_0[hd], W2_0[hd], act)
            g1 += G1
            g2 += G2
            loss[hd, c] = l
        W1_T[hd] = W1_0[hd] - eta * g1
        W2_T[hd] = W2_0[hd] - eta * g2
        O[:, hd, :] = fast_forward(q, W1_T[hd], W2_T[hd], act)
    return dict(O=O, W1_T=W1_T, W2_T=W2_T, loss=loss)


def ttt_backward_gcs(Q, K, V, W1_0, W2_0, eta, chunk_tokens, dO, norm=(True, True, True), act="silu"):
    """Reverse mode of ttt_forward_gcs for sum <O, dO>.  The adjoint of W*
    collects the apply adjoint of every token; each chunk's update adjoint is
    then taken at W0 with that same adjoint (the per-chunk formulas of
    ttt_backward with W = W0), and dW0 = adjoint of W* + the sum over chunks
    of their token sums."""
    Q, K, V, W1_0, W2_0, dO = _as_f64(Q, K, V, W1_0, W2_0, dO)
    N, H, d = K.shape
    bounds = chunk_bounds(N, chunk_tokens)
    fwd = ttt_forward_gcs(Q, K, V, W1_0, W2_0, eta, chunk_tokens, norm, act)
    dQ = np.zeros_like(Q)
    dK = np.zeros_like(K)
    dV = np.zeros_like(V)
    dW1_0 = np.zeros_like(W1_0)
    dW2_0 = np.zeros_like(W2_0)
    deta = np.zeros(H)
    for hd in range(H):
        q = _prep(Q[:, hd, :], norm[0])
        k = _prep(K[:, hd, :], norm[1])
        v = _prep(V[:, hd, :], norm[2])
        W1, W2 = W1_0[hd], W2_0[hd]
        W1s, W2s = fwd["W1_T"][hd], fwd["W2_T"][hd]
        # apply adjoint over all tokens (O = s(q W1*) W2*)
        Zq = q @ W1s
        Aq, Sq1, _ = activation(Zq, act)
        Wh2 = Aq.T @ dO[:, hd, :]
        dZq = (dO[:, hd, :] @ W2s.T) * Sq1
        Wh1 = q.T @ dZq
        dq = dZq @ W1s.T
        dk = np.zeros_like(k)
        dv = np.zeros_like(v)
        tot1, tot2 = Wh1.copy(), Wh2.copy()
        for (s, e) in bounds:
            m = e - s
            kc, vc = k[s:e], v[s:e]
            _, _, _, cc = inner_grad(kc, vc, W1, W2, act)
            A, S1, S2 = cc["A"], cc["S1"], cc["S2"]
            E, P, D = cc["E"], cc["P"], cc["D"]
            kWh1 = kc @ Wh1
            AWh2 = A @ Wh2
            deta[hd] += -np.sum(kWh1 * D) - np.sum(AWh2 * E)
            dD = -eta * kWh1
            dkc = -eta * (D @ Wh1.T)
            dA = -eta * (E @ Wh2.T)
            dE = -eta * AWh2
            dP = dD * S1
            dZ = dD * P * S2
            dE = dE + dP @ W2
            tot2 = tot2 + dP.T @ E
            dY = (2.0 / m) * dE
            dv[s:e] += -dY
            dA = dA + dY @ W2.T
            tot2 = tot2 + A.T @ dY
            dZ = dZ + dA * S1
            dkc = dkc + dZ @ W1.T
            tot1 = tot1 + kc.T @ dZ
            dk[s:e] += dkc
        dW1_0[hd] = tot1
        dW2_0[hd] = tot2
        dQ[:, hd, :] = l2norm_rows_bwd(Q[:, hd, :], dq) if norm[0] else dq
        dK[:, hd, :] = l2norm_rows_bwd(K[:, hd, :], dk) if norm[1] else dk
        dV[:, hd, :] = l2norm_rows_bwd(V[:, hd, :], dv) if norm[2] else dv
    return dict(dQ=dQ, dK=dK, dV=dV, dW1_0=dW1_0, dW2_0=dW2_0, deta=deta, fwd=fwd)


# --------------------------------------------------------------------------
# The paper's own adaptive memory unit: SwiGLU fast network (Supp. A),
# dot-product inner loss (Sec. 4.2, Eq. 9), token-wise step sizes (Eq. 8)
# --------------------------------------------------------------------------

def swiglu_forward(x, W1, W2, W3):
    """f_W(x) = (SiLU(x W1) * (x W3)) W2 for rows x (W1, W3: [d][h], W2: [h][d])."""
    s, _, _ = activation(x @ W1)
    return (s * (x @ W3)) @ W2


def swiglu_dot_loss(k, v, eta_tok, W1, W2, W3):
    """sum_i eta_i * ( - f_W(k_i)^T v_i ): the chunk's weighted dot-product
    loss whose gradient is the update of Eq. 8 (the step size lives inside)."""
    y = swiglu_forward(k, W1, W2, W3)
    return float(-np.sum(eta_tok[:, None] * y * v))


def swiglu_dot_grad(k, v, eta_tok, W1, W2, W3):
    """Hand-derived gradient of swiglu_dot_loss w.r.t. (W1, W2, W3).

    Z1 = k W1, Z3 = k W3, S = SiLU(Z1), Hd = S * Z3, E = -eta_i v_i (does not
    depend on W), grad W2 = Hd^T E, dHd = E W2^T, dZ3 = dHd * S,
    dZ1 = dHd * Z3 * s'(Z1), grad W1 = k^T dZ1, grad W3 = k^T dZ3."""
    Z1 = k @ W1
    Z3 = k @ W3
    S, S1, _ = activation(Z1)
    Hd = S * Z3
    E = -eta_tok[:, None] * v
    G2 = Hd.T @ E
    dH = E @ W2.T
    G3 = k.T @ (dH * S)
    G1 = k.T @ (dH * Z3 * S1)
    return G1, G2, G3


def ttt_forward_swiglu(Q, K, V, W1_0, W2_0, W3_0, eta_tok, chunk_tokens, sync="chain", norm=(True, True, True)):
    """The paper's AMU over one sequence.  eta_tok [N][H] are the token-wise
    step sizes (predicted from the tokens in the paper; an input here).
    sync="chain": each chunk updates W then maps its queries (Eq. 8 then
    Eq. 4, chunks in sequence order); sync="gcs": all chunks' gradients at W0
    are summed, one update, all queries mapped with the result (Eq. 10).
    Returns O, W1_T, W2_T, W3_T."""
    Q, K, V, W1_0, W2_0, W3_0, eta_tok = _as_f64(Q, K, V, W1_0, W2_0, W3_0, eta_tok)
    N, H, d = K.shape
    bounds = chunk_bounds(N, chunk_tokens)
    O = np.zeros((N, H, d))
    WT = [W1_0.copy(), W2_0.copy(), W3_0.copy()]
    for hd in range(H):
        q = _prep(Q[:, hd, :], norm[0])
        k = _prep(K[:, hd, :], norm[1])
        v = _prep(V[:, hd, :], norm[2])
        W = [W1_0[hd].copy(), W2_0[hd].copy(), W3_0[hd].copy()]
        if sync == "chain":
            for (s, e) in bounds:
                G = swiglu_dot_grad(k[s:e], v[s:e], eta_tok[s:e, hd], *W)
                W = [W[i] - G[i] for i in range(3)]
                O[s:e, hd, :] = swiglu_forward(q[s:e], *W)
        elif sync == "gcs":
            tot = [np.zeros_like(x) for x in W]
            for (s, e) in bounds:
                G = swiglu_dot_grad(k[s:e], v[s:e], eta_tok[s:e, hd], *W)
                tot = [tot[i] + G[i] for i in range(3)]
            W = [W[i] - tot[i] for i in range(3)]
            O[:, hd, :] = swiglu_forward(q, *W)
        else:
            raise ValueError(sync)
        for i in range(3):
            WT[i][hd] = W[i]
    return dict(O=O, W1_T=WT[0], W2_T=WT[1], W3_T=WT[2])


def swiglu_apply_adjoint(q, dO, W1, W2, W3):
    """Reverse mode of O = f_W(q) for the outer loss sum <O, dO>: returns the
    adjoints (dW1, dW2, dW3) and dq.

    Zq1 = q W1, Zq3 = q W3, S = SiLU(Zq1), Hq = S * Zq3, O = Hq W2;
    dW2 = Hq^T dO, dHq = dO W2^T, dZq3 = dHq * S, dZq1 = dHq * Zq3 * s'(Zq1),
    dW1 = q^T dZq1, dW3 = q^T dZq3, dq = dZq1 W1^T + dZq3 W3^T."""
    Z1 = q @ W1
    Z3 = q @ W3
    S, S1, _ = activation(Z1)
    Hq = S * Z3
    dH = dO @ W2.T
    dZ3 = dH * S
    dZ1 = dH * Z3 * S1
    return (q.T @ dZ1, Hq.T @ dO, q.T @ dZ3), dZ1 @ W1.T + dZ3 @ W3.T


def swiglu_update_adjoint(k, v, eta_tok, W1, W2, W3, Wh1, Wh2, Wh3):
    """Reverse mode of one update W' = W - G(W), G = swiglu_dot_grad, given the
    adjoint Wh of W'.  Returns (the contribution -dG/dW^T Wh to the adjoint of
    W as three matrices, dk, dv, deta_tok); the identity part of W' = W - ...
    (adjoint Wh passed through) is left to the caller.

    G is the gradient of L(W) = sum_i <f_W(k_i), E_i> with E_i = -eta_i v_i,
    so for any input X the needed product (dG/dX)^T Wh is the gradient with
    respect to X of phi = <G, Wh> = d/dt L(W + t Wh) at t = 0, the derivative
    of L along Wh:
      dot Z1 = k Wh1, dot Z3 = k Wh3, dot S = s'(Z1) dot Z1,
      dot H = dot S * Z3 + S * dot Z3, dot Y = dot H W2 + H Wh2,
      phi = sum_i <dot Y_i, E_i>.
    Its reverse mode, line by line:
      dH = E W2^T, dHh = E Wh2^T        (adjoints of dot H and H)
      grad_W2 phi = dot H^T E,  grad_E phi = dot Y
      dot S: dH * Z3;  Z3: dH * dot S + dHh * S;  S: dH * dot Z3 + dHh * Z3
      dot Z3: dH * S;  dot Z1: (dH * Z3) s'(Z1)
      Z1: (dH * Z3) s''(Z1) dot Z1 + (adjoint of S) s'(Z1)
      grad_W1 phi = k^T (adjoint of Z1), grad_W3 phi = k^T (adjoint of Z3)
      grad_k phi = adj(Z1) W1^T + adj(Z3) W3^T + adj(dot Z1) Wh1^T + adj(dot Z3) Wh3^T.
    The update subtracts G, so the contributions are minus these; through
    E_i = -eta_i v_i: dv_i = eta_i dot Y_i and deta_i = <v_i, dot Y_i>."""
    Z1 = k @ W1
    Z3 = k @ W3
    S, S1, S2 = activation(Z1)
    Hd = S * Z3
    E = -eta_tok[:, None] * v
    Zd1 = k @ Wh1
    Zd3 = k @ Wh3
    Sd = S1 * Zd1
    Hdot = Sd * Z3 + S * Zd3
    Ydot = Hdot @ W2 + Hd @ Wh2
    dH = E @ W2.T
    dHh = E @ Wh2.T
    aSd = dH * Z3
    aZ3 = dH * Sd + dHh * S
    aS = dH * Zd3 + dHh * Z3
    aZd3 = dH * S
    aZd1 = aSd * S1
    aZ1 = aSd * S2 * Zd1 + aS * S1
    gW = (k.T @ aZ1, Hdot.T @ E, k.T @ aZ3)
    gk = aZ1 @ W1.T + aZ3 @ W3.T + aZd1 @ Wh1.T + aZd3 @ Wh3.T
    return tuple(-g for g in gW), -gk, eta_tok[:, None] * Ydot, np.sum(v * Ydot, axis=1)


def ttt_backward_swiglu(Q, K, V, W1_0, W2_0, W3_0, eta_tok, chunk_tokens, dO, sync="chain", norm=(True, True, True)):
    """Reverse mode of ttt_forward_swiglu for the outer loss sum <O, dO>:
    dQ, dK, dV, deta_tok [N][H] and dW1_0, dW2_0, dW3_0.

    chain: for c = C-1 .. 0 the adjoint of W_{c+1} collects chunk c's apply
    adjoint (at W_{c+1}), then the update adjoint of chunk c (at W_c) gives
    the adjoint of W_c.  gcs: the adjoint of W* collects every token's apply
    adjoint; each chunk's update adjoint is taken at W0 with that adjoint, and
    dW0 = adjoint of W* + the sum of the chunks' contributions."""
    Q, K, V, W1_0, W2_0, W3_0, eta_tok, dO = _as_f64(Q, K, V, W1_0, W2_0, W3_0, eta_tok, dO)
    N, H, d = K.shape
    bounds = chunk_bounds(N, chunk_tokens)
    dQ, dK, dV = np.zeros_like(Q), np.zeros_like(K), np.zeros_like(V)
    deta = np.zeros_like(eta_tok)
    dW = [np.zeros_like(W1_0), np.zeros_like(W2_0), np.zeros_like(W3_0)]
    for hd in range(H):
        q = _prep(Q[:, hd, :], norm[0])
        k = _prep(K[:, hd, :], norm[1])
        v = _prep(V[:, hd, :], norm[2])
        et = eta_tok[:, hd]
        do = dO[:, hd, :]
        dq, dk, dv = np.zeros_like(q), np.zeros_like(k), np.zeros_like(v)
        W0 = [W1_0[hd], W2_0[hd], W3_0[hd]]
        if sync == "chain":
            Ws = [W0]
            for (s, e) in bounds:
                G = swiglu_dot_grad(k[s:e], v[s:e], et[s:e], *Ws[-1])
                Ws.append([Ws[-1][i] - G[i] for i in range(3)])
            Wh = [np.zeros_like(x) for x in W0]
            for c in range(len(bounds) - 1, -1, -1):
                s, e = bounds[c]
                ga, dq[s:e] = swiglu_apply_adjoint(q[s:e], do[s:e], *Ws[c + 1])
                Wh = [Wh[i] + ga[i] for i in range(3)]
                gu, dk[s:e], dv[s:e], deta[s:e, hd] = swiglu_update_adjoint(k[s:e], v[s:e], et[s:e], *Ws[c], *Wh)
                Wh = [Wh[i] + gu[i] for i in range(3)]
        elif sync == "gcs":
            tot = [np.zeros_like(x) for x in W0]
            for (s, e) in bounds:
                G = swiglu_dot_grad(k[s:e], v[s:e], et[s:e], *W0)
                tot = [tot[i] + G[i] for i in range(3)]
            Wstar = [W0[i] - tot[i] for i in range(3)]
            ga, dq = swiglu_apply_adjoint(q, do, *Wstar)
            Wh = list(ga)
            acc = [x.copy() for x in ga]
            for (s, e) in bounds:
                gu, dk[s:e], dv[s:e], deta[s:e, hd] = swiglu_update_adjoint(k[s:e], v[s:e], et[s:e], *W0, *Wh)
                acc = [acc[i] + gu[i] for i in range(3)]
            Wh = acc
        else:
            raise ValueError(sync)
        for i in range(3):
            dW[i][hd] = Wh[i]
        dQ[:, hd, :] = l2norm_rows_bwd(Q[:, hd, :], dq) if norm[0] else dq
        dK[:, hd, :] = l2norm_rows_bwd(K[:, hd, :], dk) if norm[1] else dk
        dV[:, hd, :] = l2norm_rows_bwd(V[:, hd, :], dv) if norm[2] else dv
    return dict(dQ=dQ, dK=dK, dV=dV, deta_tok=deta, dW1_0=dW[0], dW2_0=dW[1], dW3_0=dW[2])


# --------------------------------------------------------------------------
# the layer around the memory unit (Sec. 4.2; gate of Sec. 4.1 Eq. 5)
# --------------------------------------------------------------------------

def gcm_layer_forward(X, Wqkv, Wo, alpha, W1_0, W2_0, eta, chunk_tokens, bqkv=None, bo=None,
                      norm=(True, True, True), act="silu"):
    """The memory unit's layer for one sequence.

    X: [N][D] input tokens, D = H * d with H = W1_0.shape[0].  The
    query-key-value projection is one linear map, P = X Wqkv (+ bqkv) with
    Wqkv [D][3D]: P's first D columns are the queries, the next D the keys,
    the last D the values, and head h owns features h*d .. h*d+d-1 of each
    (the multi-head split of Supp. A).  The memory unit maps them
    (ttt_forward above), the output projection gives G = O Wo (+ bo), and the
    gate of Sec. 4.1 Eq. 5 returns alpha * G + X with the per-feature vector
    alpha.  Returns dict(Y, O, W1_T, W2_T)."""
    X, Wqkv, Wo, alpha = _as_f64(X, Wqkv, Wo, alpha)
    N, D = X.shape
    H = W1_0.shape[0]
    d = D // H
    P = X @ Wqkv
    if bqkv is not None:
        P = P + np.asarray(bqkv, dtype=np.float64)
    Q = P[:, :D].reshape(N, H, d)
    K = P[:, D:2 * D].reshape(N, H, d)
    V = P[:, 2 * D:].reshape(N, H, d)
    r = ttt_forward(Q, K, V, W1_0, W2_0, eta, chunk_tokens, norm, act)
    O = r["O"].reshape(N, D)
    G = O @ Wo
    if bo is not None:
        G = G + np.asarray(bo, dtype=np.float64)
    return dict(Y=alpha * G + X, O=O, W1_T=r["W1_T"], W2_T=r["W2_T"])


def gcm_layer_backward(X, Wqkv, Wo, alpha, W1_0, W2_0, eta, chunk_tokens, dY, bqkv=None, bo=None,
                       norm=(True, True, True), act="silu"):
    """Reverse mode of gcm_layer_forward for the outer loss sum <Y, dY>.

    Taken back through Y = alpha * G + X, G = O Wo (+ bo), the memory unit
    (ttt_backward above, with the adjoint dO of its output) and the
    projection P = X Wqkv (+ bqkv):
      dG = alpha * dY,  dalpha = sum_n G * dY,  dbo = sum_n dG,
      dWo = O^T dG,  dO = dG Wo^T,
      (dQ, dK, dV, dW1_0, dW2_0, deta) = the unit's reverse mode,
      dP = [dQ | dK | dV],  dWqkv = X^T dP,  dbqkv = sum_n dP,
      dX = dY + dP Wqkv^T.
    Returns dict(dX, dWqkv, dbqkv, dWo, dbo, dalpha, dW1_0, dW2_0, deta); the
    bias gradients are None where the bias is."""
    X, Wqkv, Wo, alpha, dY = _as_f64(X, Wqkv, Wo, alpha, dY)
    N, D = X.shape
    H = W1_0.shape[0]
    d = D // H
    P = X @ Wqkv
    if bqkv is not None:
        P = P + np.asarray(bqkv, dtype=np.float64)
    Q = P[:, :D].reshape(N, H, d)
    K = P[:, D:2 * D].reshape(N, H, d)
    V = P[:, 2 * D:].reshape(N, H, d)
    r = ttt_forward(Q, K, V, W1_0, W2_0, eta, chunk_tokens, norm, act)
    O = r["O"].reshape(N, D)
    G = O @ Wo
    if bo is not None:
        G = G + np.asarray(bo, dtype=np.float64)
    dG = alpha * dY
    dO = (dG @ Wo.T).reshape(N, H, d)
    u = ttt_backward(Q, K, V, W1_0, W2_0, eta, chunk_tokens, dO, norm, act)
    dP = np.concatenate([u["dQ"].reshape(N, D), u["dK"].reshape(N, D), u["dV"].reshape(N, D)], axis=1)
    return dict(dX=dY + dP @ Wqkv.T, dWqkv=X.T @ dP, dbqkv=dP.sum(axis=0) if bqkv is not None else None,
                dWo=O.T @ dG, dbo=dG.sum(axis=0) if bo is not None else None, dalpha=(G * dY).sum(axis=0),
                dW1_0=u["dW1_0"], dW2_0=u["dW2_0"], deta=u["deta"])
