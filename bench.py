"""Benchmark of the chunked TTT hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]

A step is one whole forward (every chunk update and apply of every head of
every sequence) over the headline workload: 8 sequences of uneven length
(12, 24, 40, 64, 96, 128, 200, 300 frames x 1374 tokens, 1,187,136 tokens),
16 heads x 64, fast-MLP hidden 256, chunks of 8 frames (10,992 tokens, each
sequence's last chunk ragged where its length is not a multiple), eta 0.05,
BF16 operands with FP32 accumulation and FP32 fast weights.  Inputs are
synthetic and resident in HBM before the timed region.  The FP32 path on the
same workload, the other forms (single-sequence layer, single-head chains,
forward + backward, GCS, the paper's memory unit, the layer around the unit
with its projections and gate, the length sweep) and the
FP64 oracle timed on the host cores are reported beside it.  Prints one JSON
line.

Every time is taken with HIP events on the stream the library launches on
(torch's current stream), around whole library calls, after warm-up.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TTT fwd / fwd+bwd tokens/s, BF16 vs FP32 at stated error vs FP64 oracle"
PEAK = {"f32": 157.3, "bf16": 2516.6}   # dense matrix-core TFLOP/s (MI355X)
HEADLINE = "batch8_uneven_chunk8f_bf16"
PERSISTENT = dict(schedule="persistent", wg_per_chain=8)
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "ttt_fwd_persist_batch8_uneven_hbm_counters.md")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline only (no other forms, no oracle timings)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 512 MiB device copy (the reference kernel for HBM byte counters)")
    ap.add_argument("--forms", default="layer,paper_state,single_head,fwd_bwd,batched_fwd_bwd,gcs,amu,"
                                       "gcm,length_sweep",
                    help="comma list of the other forms to time")
    return ap.parse_args()


def fwd_flops(d, h, tokens, heads):
    # 10 d h per token-head for the update chain (K W1, A W2, E W2^T and the
    # two token sums) + 4 d h for the apply (Q W1, A W2)
    return 14.0 * d * h * tokens * heads


def timed(fn, steps, warmup):
    """Milliseconds per call: HIP events on the current stream around `steps`
    calls after `warmup` calls, bracketed by device synchronisation."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st, en = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    st.record()
    for _ in range(steps):
        fn()
    en.record()
    torch.cuda.synchronize()
    return st.elapsed_time(en) / steps


def sources_hash():
    h = hashlib.sha256()
    for f in ("ttt_fwd.hip", "ttt_common.h"):
        with open(os.path.join(ROOT, "paper_2604_08542_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(io):
    """HBM bytes per launch of the persistent forward kernel on the headline
    workload, from the committed rocprofv3 counter summary (FETCH_SIZE +
    WRITE_SIZE scaled by the copy-kernel calibration), or None when that
    summary was taken for other kernel sources."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return None
    text = open(TRAFFIC_PROFILE).read()
    if f"ttt_fwd.hip+ttt_common.h: {sources_hash()}" not in text:
        return None
    for line in text.splitlines():
        if line.startswith(f"traffic_per_launch_bytes {io} = "):
            return float(line.split("=")[1])
    return None


def forward_form(w, io, steps, warmup, cfg=None, dev=None):
    """Batched forward of workload w on the io path; returns timing, roofline
    and the output tensor."""
    import torch

    from paper_2604_08542_amd import ops
    from workloads import make_inputs_torch
    if dev is None:
        dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype=io)
    cu = w.cu_seqlens()
    O = torch.empty_like(dev["Q"])
    prob = ops.problem(dev["Q"], w.d_hidden, 0, w.chunk_tokens, w.eta, ops._flags(True))
    ws = ops.workspace(prob, len(cu) - 1, dev["Q"].device)

    def step():
        ops.batched_fwd(dev["Q"], dev["K"], dev["V"], cu, dev["W1"], dev["W2"], w.eta, w.chunk_tokens, out=O, ws=ws,
                        want_final=False, tile_cfg=cfg)
    ms = timed(step, steps, warmup)
    status = ops.workspace_status(ws)
    ach = fwd_flops(w.d_head, w.d_hidden, w.n_tokens, w.n_heads) / (ms * 1e-3) / 1e12
    return dict(workload=w.name, io=io, ms_per_step=ms, tokens_per_s=w.n_tokens / (ms * 1e-3),
                device_error_word=status,
                roofline=dict(bound="mfma", achieved=ach, peak=PEAK[io], unit="TFLOP/s", frac=ach / PEAK[io])), O, dev


def other_forms(forms, steps, warmup):
    import torch

    from paper_2604_08542_amd import ops
    from workloads import WORKLOADS, make_eta_tok, make_inputs_torch
    res = {}
    few = max(2, steps // 4)
    if "layer" in forms:  # one sequence of 64 frames: the BF16 / FP32 speed-up
        w = WORKLOADS["layer16_64f_chunk8f"]
        for io in ("f32", "bf16"):
            r, _, _ = forward_form(w, io, steps, warmup)
            res[f"layer16_64f_{io}"] = r
        res["layer16_64f_speedup_bf16_over_f32"] = (res["layer16_64f_f32"]["ms_per_step"] /
                                                    res["layer16_64f_bf16"]["ms_per_step"])
    if "paper_state" in forms:  # the paper's state size: streamed-weight GEMM chunk step
        w = WORKLOADS["paper_state_64f_chunk8f_bf16"]
        for io in ("bf16", "f32"):
            r, _, _ = forward_form(w, io, few if io == "bf16" else 2, 1)
            res[f"paper_state_{io}"] = r
            torch.cuda.empty_cache()
        # GCS form (Eq. 10) at the paper's state, BF16
        dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype="bf16")
        O = torch.empty_like(dev["Q"])
        ws = ops.workspace(ops.problem(dev["Q"], w.d_hidden, w.n_tokens, w.chunk_tokens, w.eta, ops._flags(True)), 1,
                           dev["Q"].device)
        ms = timed(lambda: ops.gcs_fwd(dev["Q"], dev["K"], dev["V"], dev["W1"], dev["W2"], w.eta, w.chunk_tokens,
                                       want_final=False, out=O, ws=ws), few, 1)
        ach = fwd_flops(w.d_head, w.d_hidden, w.n_tokens, w.n_heads) / (ms * 1e-3) / 1e12
        res["paper_state_gcs_bf16"] = dict(workload=w.name, ms_per_step=ms, tokens_per_s=w.n_tokens / (ms * 1e-3),
                                           roofline=dict(bound="mfma", achieved=ach, peak=PEAK["bf16"],
                                                         unit="TFLOP/s", frac=ach / PEAK["bf16"]))
        del dev, O, ws
        torch.cuda.empty_cache()
        # forward with checkpoints + reverse mode at the paper's state, BF16
        dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype="bf16", with_dO=True)
        ws = ops.workspace(ops.problem(dev["Q"], w.d_hidden, w.n_tokens, w.chunk_tokens, w.eta, ops._flags(True)), 1,
                           dev["Q"].device)

        def fb():
            f = ops.chunk_fwd(dev["Q"], dev["K"], dev["V"], dev["W1"], dev["W2"], w.eta, w.chunk_tokens,
                              save_ckpt=True, want_final=False, ws=ws)
            ops.chunk_bwd(dev["Q"], dev["K"], dev["V"], dev["W1"], dev["W2"], w.eta, w.chunk_tokens, f["ckpt"],
                          dev["dO"], ws=ws)
        ms = timed(fb, 2, 1)
        # forward 14 d h per token-head; reverse step 36 d h (3 recomputed products, 5 of the apply
        # adjoint, 10 of the update adjoint)
        ach = 50.0 * w.d_head * w.d_hidden * w.n_tokens * w.n_heads / (ms * 1e-3) / 1e12
        res["paper_state_fwd_bwd_bf16"] = dict(workload=w.name, ms_per_step=ms, tokens_per_s=w.n_tokens / (ms * 1e-3),
                                               pass_roofline=dict(bound="mfma", achieved=ach, peak=PEAK["bf16"],
                                                                  unit="TFLOP/s (50 d h per token-head, whole pass)",
                                                                  frac=ach / PEAK["bf16"]))
        del dev, ws
        torch.cuda.empty_cache()
    if "single_head" in forms:  # single-head chains: latency-bound
        for name, io in (("single_head_4x1374", "f32"), ("single_head_256x1374_bf16", "bf16")):
            w = WORKLOADS[name]
            r, _, _ = forward_form(w, io, steps, warmup)
            r["roofline"]["bound"] = "latency (one chain, serial in its chunks)"
            res[f"{name}_{io}" if not name.endswith(io) else name] = r
    if "fwd_bwd" in forms:  # forward with checkpoints + backward through every inner update
        w = WORKLOADS["layer16_32f_chunk4f_bwd"]
        for io in ("f32", "bf16"):
            dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype=io, with_dO=True)

            def fb():
                f = ops.chunk_fwd(dev["Q"], dev["K"], dev["V"], dev["W1"], dev["W2"], w.eta, w.chunk_tokens,
                                  save_ckpt=True, want_final=False)
                ops.chunk_bwd(dev["Q"], dev["K"], dev["V"], dev["W1"], dev["W2"], w.eta, w.chunk_tokens, f["ckpt"],
                              dev["dO"])
            ms = timed(fb, few, 1)
            ach = 3.0 * fwd_flops(w.d_head, w.d_hidden, w.n_tokens, w.n_heads) / (ms * 1e-3) / 1e12
            res[f"fwd_bwd_{io}"] = dict(workload=w.name, ms_per_step=ms, tokens_per_s=w.n_tokens / (ms * 1e-3),
                                        pass_roofline=dict(bound="mfma", achieved=ach, peak=PEAK[io],
                                                           unit="TFLOP/s (42 d h per token-head, whole pass)",
                                                           frac=ach / PEAK[io]))
            del dev
    if "batched_fwd_bwd" in forms:
        w = WORKLOADS[HEADLINE]
        cu = w.cu_seqlens()
        dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype="bf16", with_dO=True)

        def bfb():
            f = ops.batched_fwd(dev["Q"], dev["K"], dev["V"], cu, dev["W1"], dev["W2"], w.eta, w.chunk_tokens,
                                save_ckpt=True, want_final=False)
            ops.batched_bwd(dev["Q"], dev["K"], dev["V"], cu, dev["W1"], dev["W2"], w.eta, w.chunk_tokens, f["ckpt"],
                            dev["dO"])
        ms = timed(bfb, 2, 1)
        ach = 3.0 * fwd_flops(w.d_head, w.d_hidden, w.n_tokens, w.n_heads) / (ms * 1e-3) / 1e12
        res["batched_fwd_bwd_bf16"] = dict(workload=w.name, ms_per_step=ms, tokens_per_s=w.n_tokens / (ms * 1e-3),
                                           pass_roofline=dict(bound="mfma", achieved=ach, peak=PEAK["bf16"],
                                                              unit="TFLOP/s (42 d h per token-head, whole pass)",
                                                              frac=ach / PEAK["bf16"]))
        del dev
    w = WORKLOADS["layer16_64f_chunk8f"]
    if "gcs" in forms:  # Global Context Synchronization form
        for io in ("f32", "bf16"):
            dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype=io)
            ms = timed(lambda: ops.gcs_fwd(dev["Q"], dev["K"], dev["V"], dev["W1"], dev["W2"], w.eta, w.chunk_tokens,
                                           want_final=False), steps, warmup)
            ach = fwd_flops(w.d_head, w.d_hidden, w.n_tokens, w.n_heads) / (ms * 1e-3) / 1e12
            res[f"gcs_fwd_{io}"] = dict(workload=w.name, ms_per_step=ms, tokens_per_s=w.n_tokens / (ms * 1e-3),
                                        roofline=dict(bound="mfma", achieved=ach, peak=PEAK[io], unit="TFLOP/s",
                                                      frac=ach / PEAK[io]))
            del dev
    if "amu" in forms:  # the paper's memory unit: SwiGLU, dot-product loss, token-wise steps
        for io in ("f32", "bf16"):
            dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype=io, with_dO=True)
            g = torch.Generator(device="cuda")
            g.manual_seed(1)
            W3 = torch.randn(dev["W1"].shape, generator=g, device="cuda") / float(w.d_head) ** 0.5
            et = torch.from_numpy(make_eta_tok(w.n_tokens, w.n_heads, w.chunk_tokens, 20.0, 0)).cuda()
            O = torch.empty_like(dev["Q"])
            for sync in ("chain", "gcs"):
                ms = timed(lambda: ops.amu_fwd(dev["Q"], dev["K"], dev["V"], et, dev["W1"], dev["W2"], W3,
                                               w.chunk_tokens, sync=sync, want_final=False, out=O), steps, warmup)
                # 12 d h per token-head for the update (K W1, K W3, E W2^T, three token sums) + 6 d h apply
                ach = 18.0 * w.d_head * w.d_hidden * w.n_tokens * w.n_heads / (ms * 1e-3) / 1e12
                res[f"amu_{sync}_{io}"] = dict(workload=w.name, ms_per_step=ms, tokens_per_s=w.n_tokens / (ms * 1e-3),
                                               roofline=dict(bound="mfma", achieved=ach, peak=PEAK[io],
                                                             unit="TFLOP/s", frac=ach / PEAK[io]))

                def fb():
                    ops.amu_fwd(dev["Q"], dev["K"], dev["V"], et, dev["W1"], dev["W2"], W3, w.chunk_tokens, sync=sync,
                                want_final=False, out=O)
                    ops.amu_bwd(dev["Q"], dev["K"], dev["V"], et, dev["W1"], dev["W2"], W3, w.chunk_tokens,
                                dev["dO"], sync=sync)
                ms = timed(fb, few, 1)
                res[f"amu_fwd_bwd_{sync}_{io}"] = dict(workload=w.name, ms_per_step=ms,
                                                       tokens_per_s=w.n_tokens / (ms * 1e-3))
            del dev, O, W3, et
        # the paper's own regime: one head of 1024, hidden 4096 (streamed-weight GEMM chunk step)
        wp = WORKLOADS["paper_state_64f_chunk8f_bf16"]
        for io in ("bf16", "f32"):
            dev = make_inputs_torch(wp.n_tokens, wp.n_heads, wp.d_head, wp.d_hidden, seed=0, io_dtype=io)
            g = torch.Generator(device="cuda")
            g.manual_seed(1)
            W3 = torch.randn(dev["W1"].shape, generator=g, device="cuda") / float(wp.d_head) ** 0.5
            et = torch.from_numpy(make_eta_tok(wp.n_tokens, wp.n_heads, wp.chunk_tokens, 100.0, 0)).cuda()
            O = torch.empty_like(dev["Q"])
            ws = torch.empty(ops.L.load().ttt_amu_workspace_bytes(ctypes.byref(
                ops.problem(dev["Q"], wp.d_hidden, wp.n_tokens, wp.chunk_tokens, 0.0, ops._flags(True)))),
                dtype=torch.uint8, device="cuda")
            for sync in ("chain", "gcs"):
                ms = timed(lambda: ops.amu_fwd(dev["Q"], dev["K"], dev["V"], et, dev["W1"], dev["W2"], W3,
                                               wp.chunk_tokens, sync=sync, want_final=False, out=O, ws=ws),
                           few if io == "bf16" else 2, 1)
                ach = 18.0 * wp.d_head * wp.d_hidden * wp.n_tokens * wp.n_heads / (ms * 1e-3) / 1e12
                res[f"amu_paper_state_{sync}_{io}"] = dict(
                    workload=wp.name.replace("_bf16", ""), ms_per_step=ms, tokens_per_s=wp.n_tokens / (ms * 1e-3),
                    roofline=dict(bound="mfma", achieved=ach, peak=PEAK[io], unit="TFLOP/s", frac=ach / PEAK[io]))
                if io == "bf16":  # forward + reverse mode
                    dOp = torch.randn(dev["Q"].shape, generator=g, device="cuda").to(dev["Q"].dtype)
                    bws = torch.empty(ops.L.load().ttt_amu_bwd_workspace_bytes(ctypes.byref(
                        ops.problem(dev["Q"], wp.d_hidden, wp.n_tokens, wp.chunk_tokens, 0.0, ops._flags(True))),
                        {"chain": 0, "gcs": 1}[sync]), dtype=torch.uint8, device="cuda")

                    def fbp():
                        ops.amu_fwd(dev["Q"], dev["K"], dev["V"], et, dev["W1"], dev["W2"], W3, wp.chunk_tokens,
                                    sync=sync, want_final=False, out=O, ws=ws)
                        ops.amu_bwd(dev["Q"], dev["K"], dev["V"], et, dev["W1"], dev["W2"], W3, wp.chunk_tokens, dOp,
                                    sync=sync, ws=bws)
                    ms = timed(fbp, 2, 1)
                    # forward 18 d h per token-head; reverse step 46 d h (8 products of the apply adjoint,
                    # 15 of the update adjoint); the chain's recomputed forward steps are not counted
                    ach = 64.0 * wp.d_head * wp.d_hidden * wp.n_tokens * wp.n_heads / (ms * 1e-3) / 1e12
                    res[f"amu_paper_state_fwd_bwd_{sync}_bf16"] = dict(
                        workload=wp.name.replace("_bf16", ""), ms_per_step=ms, tokens_per_s=wp.n_tokens / (ms * 1e-3),
                        pass_roofline=dict(bound="mfma", achieved=ach, peak=PEAK["bf16"],
                                           unit="TFLOP/s (64 d h per token-head, whole pass)",
                                           frac=ach / PEAK["bf16"]))
                    del dOp, bws
            del dev, O, W3, et, ws
            torch.cuda.empty_cache()
    if "gcm" in forms:  # the layer around the memory unit: projections, unit, output projection, gate
        for name, H, d, h, frames in (("gcm_layer16_64f", 16, 64, 256, 64), ("gcm_paper_state_64f", 1, 1024, 4096, 64)):
            N, D, M = frames * 1374, H * d, 8 * 1374
            for io in ("bf16", "f32"):
                dt = torch.bfloat16 if io == "bf16" else torch.float32
                g = torch.Generator(device="cuda")
                g.manual_seed(3)
                X = torch.randn((N, D), generator=g, device="cuda").to(dt)
                Wqkv = (torch.randn((D, 3 * D), generator=g, device="cuda") / D ** 0.5).to(dt)
                Wo = (torch.randn((D, D), generator=g, device="cuda") * (4.0 * d / D) ** 0.5).to(dt)
                alpha = torch.rand(D, generator=g, device="cuda") + 0.5
                W1 = torch.randn((H, d, h), generator=g, device="cuda") / d ** 0.5
                W2 = torch.randn((H, h, d), generator=g, device="cuda") / h ** 0.5
                Y = torch.empty_like(X)
                n = few if (io == "bf16" and H > 1) else 2
                ms = timed(lambda: ops.gcm_fwd(X, Wqkv, Wo, alpha, W1, W2, 0.05, M, out=Y, want_final=False), n, 1)
                flops = fwd_flops(d, h, N, H) + 8.0 * N * D * D  # unit + the two projections (3 D^2 + D^2 per token)
                ach = flops / (ms * 1e-3) / 1e12
                res[f"{name}_{io}"] = dict(workload=f"{name}: {H}x{d}, h{h}, {N} tokens, chunk {M}, D {D}",
                                           ms_per_step=ms, tokens_per_s=N / (ms * 1e-3),
                                           roofline=dict(bound="mfma", achieved=ach, peak=PEAK[io], unit="TFLOP/s",
                                                         frac=ach / PEAK[io],
                                                         note="unit 14 d h per token-head + projections 8 D^2 per "
                                                              "token"))
                if io == "bf16":  # forward + reverse mode of the layer
                    dY = torch.randn((N, D), generator=g, device="cuda").to(dt)

                    def fbl():
                        ops.gcm_fwd(X, Wqkv, Wo, alpha, W1, W2, 0.05, M, out=Y, want_final=False)
                        ops.gcm_bwd(X, Wqkv, Wo, alpha, W1, W2, 0.05, M, dY)
                    ms = timed(fbl, 2, 1)
                    res[f"{name}_fwd_bwd_{io}"] = dict(workload=f"{name}: {H}x{d}, h{h}, {N} tokens, chunk {M}, D {D}",
                                                       ms_per_step=ms, tokens_per_s=N / (ms * 1e-3))
                    del dY
                del X, Wqkv, Wo, Y
                torch.cuda.empty_cache()
    if "length_sweep" in forms:  # one sequence of F frames (the shape of the paper's length table)
        from workloads import Workload
        rows = {}
        for f in (150, 270, 510, 990):
            wl = Workload(f"len{f}", 16, 64, 256, (f,), 8, 0.05, "bf16")
            r, _, _ = forward_form(wl, "bf16", few, 1)
            rows[str(f)] = dict(tokens=wl.n_tokens, ms_per_step=r["ms_per_step"], tokens_per_s=r["tokens_per_s"],
                                frac_bf16_peak=r["roofline"]["frac"])
            torch.cuda.empty_cache()
        tps = [r["tokens_per_s"] for r in rows.values()]
        res["length_sweep_bf16"] = dict(workload="one sequence, 16x64, h256, chunk 8 frames, bf16", frames=rows,
                                        tokens_per_s_max_over_min=max(tps) / min(tps))
    torch.cuda.empty_cache()
    return res


def _median_time(fn, reps=3):
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts), out


def cpu_baselines(w, dev, O_gpu, full):
    """The FP64 oracle on the host cores.  Headline: one head of every
    sequence of the batch (head (5b+3) mod 16 of sequence b: 1,187,136
    token-heads, 1/16 of the workload), one warm-up on the shortest
    sequence, median of 3, scaled to all heads.  With `full`, the other
    workloads' oracle timings on bounded samples as well."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import oracle
    from workloads import WORKLOADS, make_inputs
    cu = w.cu_seqlens()
    heads = [(5 * b + 3) % w.n_heads for b in range(len(cu) - 1)]
    xs = []
    for b, hd in enumerate(heads):
        sl = slice(cu[b], cu[b + 1])
        xs.append({k: dev[k][sl, hd:hd + 1].float().cpu().numpy() for k in ("Q", "K", "V")})
    W1 = dev["W1"].cpu().numpy()
    W2 = dev["W2"].cpu().numpy()

    def run_sample():
        return [oracle.ttt_forward(x["Q"], x["K"], x["V"], W1[hd:hd + 1], W2[hd:hd + 1], w.eta, w.chunk_tokens)
                for x, hd in zip(xs, heads)]
    oracle.ttt_forward(xs[0]["Q"], xs[0]["K"], xs[0]["V"], W1[:1], W2[:1], w.eta, w.chunk_tokens)  # warm-up
    dt, refs = _median_time(run_sample)
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    # error of the GPU output on the sampled heads, per output row and overall
    errs = []
    num = den = 0.0
    worst_row = 0.0
    maxabs = maxref = 0.0
    for b, (hd, ref) in enumerate(zip(heads, refs)):
        o = O_gpu[cu[b]:cu[b + 1], hd].float().cpu().numpy().astype(np.float64)
        r = ref["O"][:, 0]
        num += float(np.sum((o - r) ** 2))
        den += float(np.sum(r * r))
        worst_row = max(worst_row, float(np.max(np.linalg.norm(o - r, axis=1) / np.linalg.norm(r, axis=1))))
        maxabs = max(maxabs, float(np.max(np.abs(o - r))))
        maxref = max(maxref, float(np.max(np.abs(r))))
        errs.append(float(np.linalg.norm(o - r) / np.linalg.norm(r)))
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    base = dict(value=w.n_tokens / w.n_heads / dt, unit="tokens/s", cores=threads, kind="oracle",
                sample=f"FP64 numpy oracle forward of one head of each of the 8 sequences ({w.n_tokens} "
                       f"token-heads = 1/{w.n_heads} of the workload), median of 3 ({dt:.1f} s), scaled to all "
                       f"{w.n_heads} heads", seconds=dt, host_cpus=os.cpu_count(), cpu_model=model)
    accuracy = dict(O_rel_norm=(num / den) ** 0.5, O_worst_row_rel=worst_row, O_maxabs=maxabs,
                    O_maxabs_over_max_ref=maxabs / maxref, per_sequence_rel=errs,
                    note="GPU BF16 path vs FP64 oracle on the same BF16-rounded inputs, sampled heads")
    if not full:
        return base, accuracy
    # the other workloads' oracle timings on bounded samples (median of 3 each)
    other = {}
    for name, n_heads_s, kind in (("single_head_4x1374", 1, "fwd"), ("single_head_256x1374_bf16", 1, "fwd"),
                                  ("layer16_64f_chunk8f", 1, "fwd"), ("layer16_32f_chunk4f_bwd", 1, "fwd+bwd")):
        wl = WORKLOADS[name]
        x = make_inputs(wl.n_tokens, n_heads_s, wl.d_head, wl.d_hidden, seed=0, with_dO=kind != "fwd")
        if kind == "fwd":
            f = lambda: oracle.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], wl.eta, wl.chunk_tokens)
        else:
            def f():
                oracle.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], wl.eta, wl.chunk_tokens)
                return oracle.ttt_backward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], wl.eta, wl.chunk_tokens,
                                           x["dO"])
        t, _ = _median_time(f)
        other[name] = dict(pass_=kind, tokens_per_s=wl.n_tokens * n_heads_s / wl.n_heads / t,
                           gflop_per_s=(42.0 if kind != "fwd" else 14.0) * wl.d_head * wl.d_hidden * wl.n_tokens *
                           n_heads_s / t / 1e9,
                           sample=f"{n_heads_s} of {wl.n_heads} heads, all {wl.n_tokens} tokens, median of 3 "
                                  f"({t:.2f} s), scaled to all heads")
    base["other_workloads"] = other
    return base, accuracy


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}): chains shard over GPUs by "
              f"(sequence, head), but no multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2604_08542_amd as P
    from workloads import WORKLOADS
    P.load()
    w = WORKLOADS[HEADLINE]
    # the batching form as one persistent launch per pass (the dominant and
    # only kernel of the call besides a counter reset), so the events around
    # the call time that kernel's launches
    head, O, dev = forward_form(w, "bf16", a.steps, a.warmup, cfg=PERSISTENT)
    head["roofline"]["traffic"] = measured_traffic("bf16")
    head["roofline"]["traffic_unit"] = "HBM bytes per launch"
    print(f"# headline {HEADLINE} bf16: {head['ms_per_step']:.3f} ms/step, {head['tokens_per_s']:.4g} tokens/s, "
          f"{head['roofline']['achieved']:.1f} TFLOP/s", file=sys.stderr, flush=True)
    if a.copy_calib:
        src = torch.empty(128 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cpu = acc = None
    if not a.no_cpu_baseline:
        cpu, acc = cpu_baselines(w, dev, O, full=not a.quick)
        print(f"# oracle: {cpu['value']:.4g} tokens/s on {cpu['cores']} threads", file=sys.stderr, flush=True)
    del dev, O
    torch.cuda.empty_cache()
    # the other schedule on the same workload: one step launch and one update
    # launch per chunk step (the persistent launch is the tuned one here)
    stepwise, _, _ = forward_form(w, "bf16", a.steps, a.warmup, cfg=dict(schedule="stepwise", wg_per_chain=16))
    print(f"# {HEADLINE} bf16, stepwise schedule: {stepwise['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    f32, _, _ = forward_form(w, "f32", max(2, a.steps // 4), 2, cfg=PERSISTENT)
    f32["roofline"]["traffic"] = measured_traffic("f32")
    print(f"# {HEADLINE} f32: {f32['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    torch.cuda.empty_cache()
    extra = {} if a.quick else other_forms(tuple(f for f in a.forms.split(",") if f), a.steps, a.warmup)
    for k, v in extra.items():
        if isinstance(v, dict) and "ms_per_step" in v:
            print(f"# {k}: {v['ms_per_step']:.3f} ms/step, {v['tokens_per_s']:.4g} tokens/s", file=sys.stderr,
                  flush=True)
    line = {
        "metric": METRIC,
        "value": head["tokens_per_s"],
        "unit": "tokens/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": HEADLINE, "sequences_frames": list(w.frames), "tokens": w.n_tokens,
                   "heads": w.n_heads, "d_head": w.d_head, "d_hidden": w.d_hidden, "chunk_tokens": w.chunk_tokens,
                   "eta": w.eta, "pass": "forward", "arithmetic": "BF16 operands, FP32 accumulate / weights / norms",
                   "schedule": "persistent: one launch per pass, groups of 8 work-groups per chain"},
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "accuracy_vs_oracle": acc,
        "device_error_word": head["device_error_word"],
        "variants": {"f32": f32, "bf16": {k: v for k, v in head.items() if k != "roofline"},
                     "bf16_stepwise_schedule": stepwise},
        "speedup_bf16_over_f32": f32["ms_per_step"] / head["ms_per_step"],
        "other_forms": extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
