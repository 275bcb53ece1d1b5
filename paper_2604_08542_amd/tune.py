"""Launch-shape autotuner for the chunked TTT forward and backward.

    python -m paper_2604_08542_amd.tune --workload batch8_uneven_chunk8f_bf16 [--backward]

For one workload it times the batched forward (or, with --backward, the
batched backward) for each candidate launch shape: the schedule (one
persistent launch, or one step launch and one update launch per chunk step)
and the work-groups per chain (or the total work-groups aimed for), keeps
the fastest, and records it in tuned_tiles.json under a key made of (hidden
size, io dtype, chunk tokens, chains, and "_bwd" for the backward).  The
table is also written as csrc/ttt_tuned.h, which the library compiles in:
every caller of the C ABI that passes no launch shape gets the recorded one
(rebuild after tuning).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_tiles.json")


def key(h: int, io: str, chunk_tokens: int, n_chains: int, kind: str = "fwd") -> str:
    return f"h{h}_{io}_m{chunk_tokens}_c{n_chains}" + ("_bwd" if kind == "bwd" else "")


def load_table(path: str = TABLE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def lookup(h: int, io: str, chunk_tokens: int, n_chains: int, kind: str = "fwd", table=None):
    t = load_table() if table is None else table
    return t.get(key(h, io, chunk_tokens, n_chains, kind), {}).get("tile_cfg")


CANDIDATES = [dict(schedule="stepwise", target_wgs=t) for t in (128, 256, 384, 512, 768, 1024)] + \
             [dict(schedule="stepwise", wg_per_chain=g) for g in (1, 2, 4, 8, 16, 32)] + \
             [dict(schedule="persistent")] + \
             [dict(schedule="persistent", wg_per_chain=g) for g in (4, 8, 12, 16, 20, 24, 32)]
BWD_CANDIDATES = [dict(target_wgs=t) for t in (128, 256, 512, 1024)] + \
                 [dict(wg_per_chain=g) for g in (2, 4, 8, 16, 32)]
HEADER = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "ttt_tuned.h")


def write_header(table: dict, path: str = HEADER):
    """The tuned launch shapes as a C++ table compiled into the library."""
    import re
    rows = []
    for k in sorted(table):
        m = re.fullmatch(r"h(\d+)_(f32|bf16)_m(\d+)_c(\d+)(_bwd)?", k)
        if not m:
            continue
        c = table[k]["tile_cfg"]
        sched = 0 if c.get("schedule", "stepwise") == "persistent" else 1
        rows.append(f"    {{{m.group(1)}, {1 if m.group(2) == 'bf16' else 0}, {m.group(3)}, {m.group(4)}, "
                    f"{1 if m.group(5) else 0}, {{{int(c.get('wg_per_chain', 0))}, {int(c.get('target_wgs', 0))}, "
                    f"{sched}, 0}}}},  // {table[k].get('workload', '')}: {table[k]['ms']:.3f} ms")
    text = ("// Launch shapes recorded by the autotuner (paper_2604_08542_amd/tune.py) on MI355X; generated from\n"
            "// tuned_tiles.json, do not edit.  Key: hidden size, BF16 operands, chunk tokens, chains, backward.\n"
            "#pragma once\n#include <stdint.h>\n\n#include \"../../include/ttt.h\"\n\nnamespace ttt {\n"
            "struct TunedShape {\n  int32_t h, bf16;\n  int64_t chunk_tokens, chains;\n  int32_t bwd;\n"
            "  ttt_tile_cfg_t cfg;\n};\ninline constexpr TunedShape kTuned[] = {\n" + "\n".join(rows) +
            "\n};\n}  // namespace ttt\n")
    with open(path, "w") as f:
        f.write(text)


def tune(workload: str, io: str = None, reps: int = 5, seed: int = 0, write: bool = True, backward: bool = False):
    import torch

    from . import ops
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from workloads import WORKLOADS, make_inputs_torch
    w = WORKLOADS[workload]
    io = io or w.io_dtype
    dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=seed, io_dtype=io, with_dO=backward)
    cu = w.cu_seqlens()
    O = torch.empty_like(dev["Q"])
    prob = ops.problem(dev["Q"], w.d_hidden, 0, w.chunk_tokens, w.eta, ops._flags(True))
    ws = ops.workspace(prob, len(cu) - 1, dev["Q"].device)
    ckpt = None
    if backward:  # the backward needs the forward's checkpoints (default shape)
        ckpt = ops.batched_fwd(dev["Q"], dev["K"], dev["V"], cu, dev["W1"], dev["W2"], w.eta, w.chunk_tokens,
                               save_ckpt=True, want_final=False)["ckpt"]
    results = []
    for cfg in (BWD_CANDIDATES if backward else CANDIDATES):
        def run():
            if backward:
                ops.batched_bwd(dev["Q"], dev["K"], dev["V"], cu, dev["W1"], dev["W2"], w.eta, w.chunk_tokens, ckpt,
                                dev["dO"], tile_cfg=cfg)
            else:
                ops.batched_fwd(dev["Q"], dev["K"], dev["V"], cu, dev["W1"], dev["W2"], w.eta, w.chunk_tokens,
                                tile_cfg=cfg, out=O, ws=ws, want_final=False)
        run()
        torch.cuda.synchronize()
        st, en = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        st.record()
        for _ in range(reps):
            run()
        en.record()
        torch.cuda.synchronize()
        ms = st.elapsed_time(en) / reps
        results.append((ms, cfg))
        print(f"  {cfg}: {ms:.3f} ms", flush=True)
    results.sort(key=lambda r: r[0])
    best_ms, best = results[0]
    k = key(w.d_hidden, io, w.chunk_tokens, w.n_heads * len(w.frames), "bwd" if backward else "fwd")
    entry = dict(tile_cfg=best, ms=best_ms, workload=workload, tuned_at=time.strftime("%Y-%m-%d"),
                 candidates={json.dumps(c): m for m, c in results})
    if write:
        t = load_table()
        t[k] = entry
        with open(TABLE, "w") as f:
            json.dump(t, f, indent=1, sort_keys=True)
        write_header(t)
    print(f"best {best} {best_ms:.3f} ms -> {k}")
    return entry


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", action="append", default=[])
    ap.add_argument("--io", default=None)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--backward", action="store_true", help="tune the batched backward instead of the forward")
    ap.add_argument("--header-only", action="store_true", help="rewrite csrc/ttt_tuned.h from the table and exit")
    a = ap.parse_args()
    if a.header_only:
        write_header(load_table())
        sys.exit(0)
    for wl in a.workload:
        tune(wl, a.io, a.reps, backward=a.backward)
