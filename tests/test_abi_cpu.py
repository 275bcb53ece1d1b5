"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/ttt.h, sizes workspaces, and rejects invalid arguments
before anything is enqueued (no compute call is made here)."""
import ctypes
import os
import re

import pytest

from paper_2604_08542_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return L.load()


def header_functions():
    src = open(os.path.join(ROOT, "include", "ttt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ttt_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert set(L.EXPORTED) <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def prob(**kw):
    base = dict(n_heads=16, d_head=64, d_hidden=256, n_tokens=87936, chunk_tokens=10992, stride_tok=0,
                stride_head=0, eta=0.05, flags=7, io_dtype=L.TTT_F32)
    base.update(kw)
    return L.Problem(**base)


def test_workspace_bytes(lib):
    p = prob()
    n1 = lib.ttt_workspace_bytes(ctypes.byref(p), 1)
    n8 = lib.ttt_workspace_bytes(ctypes.byref(p), 8)
    assert n1 > 0 and n8 >= n1
    assert n1 >= 1024 * 2 * 64 * 256 * 4   # shard-partial slots
    for bad in (dict(d_head=32), dict(d_hidden=192), dict(chunk_tokens=0), dict(n_heads=0),
                dict(io_dtype=7), dict(flags=1 << 20), dict(stride_tok=3)):
        assert lib.ttt_workspace_bytes(ctypes.byref(prob(**bad)), 1) == 0, bad
    assert lib.ttt_workspace_bytes(ctypes.byref(p), 0) == 0
    assert lib.ttt_workspace_bytes(None, 1) == 0


FAKE = ctypes.c_void_p(1 << 20)  # never dereferenced: validation fails first


def fwd(lib, p, **ptrs):
    a = dict(Q=FAKE, K=FAKE, V=FAKE, W1=FAKE, W2=FAKE, O=FAKE, W1T=None, W2T=None, ckpt=None, loss=None,
             ws=FAKE, nws=1 << 40)
    a.update(ptrs)
    return lib.ttt_chunk_fwd(ctypes.byref(p), a["Q"], a["K"], a["V"], a["W1"], a["W2"], a["O"], a["W1T"],
                             a["W2T"], a["ckpt"], a["loss"], a["ws"], a["nws"], None)


def test_fwd_validation(lib):
    assert fwd(lib, prob(d_head=32)) == L.TTT_ESHAPE
    assert fwd(lib, prob(d_hidden=64)) == L.TTT_ESHAPE
    assert fwd(lib, prob(chunk_tokens=0)) == L.TTT_EINVAL
    assert fwd(lib, prob(eta=float("nan"))) == L.TTT_EINVAL
    assert fwd(lib, prob(), Q=None) == L.TTT_EINVAL
    assert fwd(lib, prob(), W1T=FAKE) == L.TTT_EINVAL             # W1_T without W2_T
    assert fwd(lib, prob(flags=7 | L.TTT_SAVE_CKPT)) == L.TTT_EINVAL  # ckpt flag without buffer
    assert fwd(lib, prob(flags=7), ckpt=FAKE) == L.TTT_EINVAL      # buffer without flag
    assert fwd(lib, prob(flags=7 | L.TTT_EMIT_LOSS)) == L.TTT_EINVAL
    assert fwd(lib, prob(), Q=ctypes.c_void_p((1 << 20) + 4)) == L.TTT_EINVAL  # misaligned
    assert fwd(lib, prob(), ws=None) == L.TTT_EWORKSPACE
    assert fwd(lib, prob(stride_tok=(1 << 22) + 64)) == L.TTT_ESHAPE   # just past the 32-bit tile addressing
    assert fwd(lib, prob(stride_tok=1 << 22), ws=None) == L.TTT_EWORKSPACE  # the largest stride is accepted
    assert fwd(lib, prob(), nws=16) == L.TTT_EWORKSPACE
    assert fwd(lib, prob(n_tokens=0)) == L.TTT_OK                  # nothing to do, nothing enqueued


def test_batched_validation(lib):
    p = prob(n_tokens=0)
    cu = (ctypes.c_int64 * 4)(0, 10, 5, 20)  # non-monotone

    def call(n, cu_arr, w0=0, cfg=None, **kw):
        a = dict(Q=FAKE, ws=FAKE, nws=1 << 40)
        a.update(kw)
        return lib.ttt_batched_fwd(ctypes.byref(p), n, cu_arr, a["Q"], FAKE, FAKE, FAKE, FAKE, w0, FAKE, None,
                                   None, cfg, a["ws"], a["nws"], None)
    assert call(3, cu) == L.TTT_EINVAL
    cu0 = (ctypes.c_int64 * 2)(5, 10)
    assert call(1, cu0) == L.TTT_EINVAL                      # cu[0] != 0
    ok = (ctypes.c_int64 * 3)(0, 0, 0)
    assert call(0, ok) == L.TTT_EINVAL                       # no sequences
    assert call(2, ok, w0=2) == L.TTT_EINVAL
    assert call(2, ok) == L.TTT_OK                           # all empty: nothing enqueued
    cfg = L.TileCfg(-1, 0)
    good = (ctypes.c_int64 * 3)(0, 10, 30)
    assert call(2, good, cfg=ctypes.byref(cfg)) == L.TTT_EINVAL
    assert call(2, good, ws=None) == L.TTT_EWORKSPACE


def test_batched_ckpt_and_bwd_validation(lib):
    good = (ctypes.c_int64 * 3)(0, 10, 30)
    bad = (ctypes.c_int64 * 3)(0, 10, 5)

    def fwdc(p, cu, ckpt=FAKE, n=2):
        return lib.ttt_batched_fwd_ckpt(ctypes.byref(p), n, cu, FAKE, FAKE, FAKE, FAKE, FAKE, 0, FAKE, None, None,
                                        ckpt, None, FAKE, 1 << 40, None)
    ck = prob(n_tokens=0, flags=7 | L.TTT_SAVE_CKPT)
    assert fwdc(ck, bad) == L.TTT_EINVAL
    assert fwdc(ck, good, ckpt=None) == L.TTT_EINVAL                  # flag without buffer
    assert fwdc(prob(n_tokens=0), good) == L.TTT_EINVAL               # buffer without flag
    assert fwdc(prob(n_tokens=0, flags=7 | L.TTT_SAVE_CKPT | L.TTT_EMIT_LOSS), good) == L.TTT_ENOTSUP
    # plain batched forward rejects the checkpoint flag (no buffer to write)
    assert lib.ttt_batched_fwd(ctypes.byref(ck), 2, good, FAKE, FAKE, FAKE, FAKE, FAKE, 0, FAKE, None, None,
                               None, FAKE, 1 << 40, None) == L.TTT_EINVAL

    def bwd(cu, n=2, w0=0, **kw):
        a = dict(ckpt=FAKE, dO=FAKE, dW1=FAKE, deta=FAKE, ws=FAKE, nws=1 << 40, Q=FAKE)
        a.update(kw)
        p = prob(n_tokens=0)
        return lib.ttt_batched_bwd(ctypes.byref(p), n, cu, a["Q"], FAKE, FAKE, FAKE, FAKE, w0, a["ckpt"], a["dO"],
                                   FAKE, FAKE, FAKE, a["dW1"], FAKE, a["deta"], None, a["ws"], a["nws"], None)
    assert bwd(bad) == L.TTT_EINVAL
    assert bwd(good, n=0) == L.TTT_EINVAL
    assert bwd(good, w0=3) == L.TTT_EINVAL
    assert bwd(good, ckpt=None) == L.TTT_EINVAL
    assert bwd(good, dO=None) == L.TTT_EINVAL
    assert bwd(good, dW1=None) == L.TTT_EINVAL
    assert bwd(good, deta=None) == L.TTT_EINVAL
    assert bwd(good, Q=ctypes.c_void_p((1 << 20) + 8)) == L.TTT_EINVAL  # misaligned
    assert bwd(good, ws=None) == L.TTT_EWORKSPACE
    assert bwd(good, nws=64) == L.TTT_EWORKSPACE


def test_amu_validation(lib):
    def call(p, sync=0, **kw):
        a = dict(Q=FAKE, eta=FAKE, W3=FAKE, W1T=None, W2T=None, W3T=None, ws=FAKE, nws=1 << 40)
        a.update(kw)
        return lib.ttt_amu_fwd(ctypes.byref(p), sync, a["Q"], FAKE, FAKE, a["eta"], FAKE, FAKE, a["W3"], FAKE,
                               a["W1T"], a["W2T"], a["W3T"], a["ws"], a["nws"], None)
    p = prob(n_tokens=1000, chunk_tokens=100)
    assert lib.ttt_amu_workspace_bytes(ctypes.byref(p)) >= 1024 * 3 * 64 * 256 * 4
    assert lib.ttt_amu_workspace_bytes(ctypes.byref(prob(d_hidden=96))) == 0
    # the paper's state (one head of 1024, hidden 4096): the forward takes a
    # workspace of the chunk's intermediates and three weight sets; the
    # reverse mode's chain form also keeps the weights before every chunk, so
    # it grows with the chunk count, and its GCS form does not
    big = prob(n_heads=1, d_head=1024, d_hidden=4096, n_tokens=2748, chunk_tokens=1374)
    longer = prob(n_heads=1, d_head=1024, d_hidden=4096, n_tokens=4 * 2748, chunk_tokens=1374)
    fwd = lib.ttt_amu_workspace_bytes(ctypes.byref(big))
    assert fwd >= 6 * 1374 * 4096 * 4 + 3 * 1024 * 4096 * 4
    chain, gcs = (lib.ttt_amu_bwd_workspace_bytes(ctypes.byref(big), s) for s in (0, 1))
    assert gcs > fwd and chain >= gcs + 3 * 3 * 1024 * 4096 * 4
    assert lib.ttt_amu_bwd_workspace_bytes(ctypes.byref(longer), 0) - chain == 6 * 3 * 1024 * 4096 * 4
    assert lib.ttt_amu_bwd_workspace_bytes(ctypes.byref(longer), 1) == gcs
    assert call(p, sync=2) == L.TTT_EINVAL
    assert call(p, eta=None) == L.TTT_EINVAL
    assert call(p, W3=None) == L.TTT_EINVAL
    assert call(p, W1T=FAKE, W2T=FAKE) == L.TTT_EINVAL          # W3_T missing
    assert call(prob(n_tokens=1000, flags=7 | L.TTT_SAVE_CKPT)) == L.TTT_ENOTSUP
    assert call(prob(d_head=32)) == L.TTT_ESHAPE
    assert call(p, Q=ctypes.c_void_p((1 << 20) + 4)) == L.TTT_EINVAL
    assert call(p, ws=None) == L.TTT_EWORKSPACE
    assert call(prob(n_tokens=0)) == L.TTT_OK                     # nothing to do, nothing enqueued


def test_amu_bwd_validation(lib):
    """Argument checks of the memory unit's reverse mode (all rejected before
    anything is enqueued, so no GPU is needed)."""
    def call(p, sync=0, **kw):
        a = dict(Q=FAKE, eta=FAKE, dO=FAKE, dW3=FAKE, ws=FAKE, nws=1 << 40)
        a.update(kw)
        return lib.ttt_amu_bwd(ctypes.byref(p), sync, a["Q"], FAKE, FAKE, a["eta"], FAKE, FAKE, FAKE, a["dO"], FAKE,
                               FAKE, FAKE, FAKE, FAKE, FAKE, a["dW3"], a["ws"], a["nws"], None)
    p = prob(n_tokens=1000, chunk_tokens=100)
    chain = lib.ttt_amu_bwd_workspace_bytes(ctypes.byref(p), L.TTT_SYNC_CHAIN)
    gcs = lib.ttt_amu_bwd_workspace_bytes(ctypes.byref(p), L.TTT_SYNC_GCS)
    assert chain > gcs >= 1024 * 3 * 64 * 256 * 4           # the chain keeps every W_c (10 chunks)
    assert lib.ttt_amu_bwd_workspace_bytes(ctypes.byref(p), 5) == 0
    assert call(p, sync=2) == L.TTT_EINVAL
    assert call(p, eta=None) == L.TTT_EINVAL
    assert call(p, dO=None) == L.TTT_EINVAL
    assert call(p, dW3=None) == L.TTT_EINVAL
    assert call(prob(n_tokens=1000, flags=7 | L.TTT_EMIT_LOSS)) == L.TTT_ENOTSUP
    assert call(prob(d_hidden=192)) == L.TTT_ESHAPE
    assert call(prob(stride_tok=1 << 23)) == L.TTT_ESHAPE
    assert call(p, Q=ctypes.c_void_p((1 << 20) + 4)) == L.TTT_EINVAL
    assert call(p, ws=None) == L.TTT_EWORKSPACE
    assert call(p, nws=gcs) == L.TTT_EWORKSPACE                # chain needs more than GCS


def test_status_strings(lib):
    for s in range(6):
        assert lib.ttt_status_string(s).startswith(b"TTT_")
    assert lib.ttt_version() >= 100


def test_missing_library_fails_loudly(tmp_path):
    # a fresh interpreter: the loader raises instead of falling back to anything else
    import subprocess
    import sys
    code = ("from paper_2604_08542_amd import _lib\n"
            f"_lib.load({str(tmp_path / 'absent' / 'libttt_hip.so')!r})\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "not built" in r.stderr


def test_product_never_touches_the_oracle():
    # the oracle is test infrastructure: nothing in the package or the C ABI refers to it
    pkg = os.path.join(ROOT, "paper_2604_08542_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\boracle\b", src), os.path.join(dirpath, f)
    assert not re.search(r"\boracle\b", open(os.path.join(ROOT, "include", "ttt.h")).read())
