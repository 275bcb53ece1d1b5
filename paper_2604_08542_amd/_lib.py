"""ctypes binding of the C ABI declared in include/ttt.h (argument marshalling
only; all computation happens in the HIP library)."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libttt_hip.so")

TTT_OK, TTT_EINVAL, TTT_ESHAPE, TTT_EWORKSPACE, TTT_EHIP, TTT_ENOTSUP = range(6)
TTT_F32, TTT_BF16 = 0, 1
TTT_NORM_Q, TTT_NORM_K, TTT_NORM_V = 1, 2, 4
TTT_SAVE_CKPT, TTT_EMIT_LOSS, TTT_MMA_BF16 = 8, 16, 32
TTT_SYNC_CHAIN, TTT_SYNC_GCS = 0, 1

EXPORTED = ("ttt_workspace_bytes", "ttt_chunk_fwd", "ttt_chunk_bwd", "ttt_batched_fwd", "ttt_batched_fwd_ckpt",
            "ttt_batched_bwd", "ttt_gcs_fwd", "ttt_gcs_bwd", "ttt_amu_workspace_bytes", "ttt_amu_fwd",
            "ttt_amu_bwd_workspace_bytes", "ttt_amu_bwd",
            "ttt_chunk_fwd_noalloc", "ttt_workspace_status", "ttt_gcm_workspace_bytes", "ttt_gcm_fwd",
            "ttt_gcm_bwd_workspace_bytes", "ttt_gcm_bwd",
            "ttt_status_string", "ttt_version")


class Problem(ctypes.Structure):
    _fields_ = [
        ("n_heads", ctypes.c_int32),
        ("d_head", ctypes.c_int32),
        ("d_hidden", ctypes.c_int32),
        ("n_tokens", ctypes.c_int64),
        ("chunk_tokens", ctypes.c_int64),
        ("stride_tok", ctypes.c_int64),
        ("stride_head", ctypes.c_int64),
        ("eta", ctypes.c_float),
        ("flags", ctypes.c_uint32),
        ("io_dtype", ctypes.c_int),
    ]


TTT_SCHED_PERSISTENT, TTT_SCHED_STEPWISE = 0, 1


class TileCfg(ctypes.Structure):
    _fields_ = [("wg_per_chain", ctypes.c_int32), ("target_wgs", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("spin_limit", ctypes.c_int32)]


class TTTError(RuntimeError):
    def __init__(self, status: int, lib=None, where: str = ""):
        msg = lib.ttt_status_string(status).decode() if lib is not None else str(status)
        super().__init__(f"{where}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (built by paper_2604_08542_amd.build).  Raises if
    it has not been built: there is no fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not built; run `python -m paper_2604_08542_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER(Problem)
    vp, fp, sz, st = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
    lib.ttt_workspace_bytes.argtypes = [P, ctypes.c_int32]
    lib.ttt_workspace_bytes.restype = sz
    lib.ttt_chunk_fwd.argtypes = [P, vp, vp, vp, fp, fp, vp, fp, fp, fp, fp, vp, sz, vp]
    lib.ttt_chunk_fwd.restype = st
    lib.ttt_chunk_fwd_noalloc.argtypes = [P, vp, vp, vp, fp, fp, vp, fp, fp, fp, fp, vp]
    lib.ttt_chunk_fwd_noalloc.restype = st
    lib.ttt_chunk_bwd.argtypes = [P, vp, vp, vp, fp, fp, fp, vp, vp, vp, vp, fp, fp, fp, vp, sz, vp]
    lib.ttt_chunk_bwd.restype = st
    lib.ttt_batched_fwd.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), vp, vp, vp, fp, fp,
                                    ctypes.c_int32, vp, fp, fp, ctypes.POINTER(TileCfg), vp, sz, vp]
    lib.ttt_batched_fwd.restype = st
    lib.ttt_batched_fwd_ckpt.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), vp, vp, vp, fp, fp,
                                         ctypes.c_int32, vp, fp, fp, fp, ctypes.POINTER(TileCfg), vp, sz, vp]
    lib.ttt_batched_fwd_ckpt.restype = st
    lib.ttt_batched_bwd.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), vp, vp, vp, fp, fp,
                                    ctypes.c_int32, fp, vp, vp, vp, vp, fp, fp, fp, ctypes.POINTER(TileCfg), vp, sz,
                                    vp]
    lib.ttt_batched_bwd.restype = st
    lib.ttt_status_string.argtypes = [st]
    lib.ttt_status_string.restype = ctypes.c_char_p
    lib.ttt_gcs_fwd.argtypes = [P, vp, vp, vp, fp, fp, vp, fp, fp, fp, vp, sz, vp]
    lib.ttt_gcs_fwd.restype = st
    lib.ttt_gcs_bwd.argtypes = [P, vp, vp, vp, fp, fp, vp, vp, vp, vp, fp, fp, fp, vp, sz, vp]
    lib.ttt_gcs_bwd.restype = st
    lib.ttt_amu_workspace_bytes.argtypes = [P]
    lib.ttt_amu_workspace_bytes.restype = sz
    lib.ttt_amu_fwd.argtypes = [P, ctypes.c_int32, vp, vp, vp, fp, fp, fp, fp, vp, fp, fp, fp, vp, sz, vp]
    lib.ttt_amu_fwd.restype = st
    lib.ttt_amu_bwd_workspace_bytes.argtypes = [P, ctypes.c_int32]
    lib.ttt_amu_bwd_workspace_bytes.restype = sz
    lib.ttt_amu_bwd.argtypes = [P, ctypes.c_int32, vp, vp, vp, fp, fp, fp, fp, vp, vp, vp, vp, fp, fp, fp, fp, vp, sz,
                                vp]
    lib.ttt_amu_bwd.restype = st
    lib.ttt_gcm_workspace_bytes.argtypes = [P]
    lib.ttt_gcm_workspace_bytes.restype = sz
    lib.ttt_gcm_fwd.argtypes = [P, vp, vp, fp, vp, fp, fp, fp, fp, vp, fp, fp, vp, sz, vp]
    lib.ttt_gcm_fwd.restype = st
    lib.ttt_gcm_bwd_workspace_bytes.argtypes = [P]
    lib.ttt_gcm_bwd_workspace_bytes.restype = sz
    lib.ttt_gcm_bwd.argtypes = [P, vp, vp, fp, vp, fp, fp, fp, fp, vp, vp, fp, fp, fp, fp, fp, fp, fp, fp, vp, sz, vp]
    lib.ttt_gcm_bwd.restype = st
    lib.ttt_workspace_status.argtypes = [vp, sz, ctypes.POINTER(ctypes.c_uint32), vp]
    lib.ttt_workspace_status.restype = st
    lib.ttt_version.argtypes = []
    lib.ttt_version.restype = ctypes.c_int32
    _lib = lib
    return lib


def check(status: int, where: str):
    if status != TTT_OK:
        raise TTTError(status, _lib, where)
