"""Benchmark of the chunked TTT hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one whole forward (every chunk update and apply of every head) over
the workload's synthetic token stream, inputs resident in HBM.  The default
workload is 16 heads x 64, fast-MLP hidden 256, 64 frames x 1374 tokens,
chunks of 8 frames, eta 0.05, FP32 (the plain path); the BF16-operand path on
the same workload is timed beside it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TTT fwd / fwd+bwd tokens/s, BF16 vs FP32 at stated error vs FP64 oracle"
PEAK = {"f32": 157.3, "bf16": 2516.6}   # dense matrix-core TFLOP/s (MI355X)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="layer16_64f_chunk8f")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-heads", type=int, default=16)
    ap.add_argument("--variants", default="f32,bf16", help="comma list of operand paths to time")
    ap.add_argument("--no-extra", action="store_true", help="skip the GCS / fwd+bwd / batched forms")
    ap.add_argument("--forms", default="gcs,fwd_bwd,batched_fwd,batched_fwd_bwd,amu,single_head,length_sweep",
                    help="comma list of the other forms to time (gcs, fwd_bwd, batched_fwd, batched_fwd_bwd, amu, "
                         "single_head, length_sweep)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 512 MiB device copy (reference kernel for HBM counters)")
    return ap.parse_args()


def alg_flops(w):
    # forward: 10*d*h per token-head for the update chain + 4*d*h for the apply
    return 14.0 * w.d_head * w.d_hidden * w.n_tokens * w.n_heads


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "ttt_fwd_step_layer16_64f_hbm_counters.md")


def measured_traffic(io, workload):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    summary (FETCH_SIZE / WRITE_SIZE scaled by the copy-kernel calibration),
    or None when that summary is for other kernel sources or another
    workload."""
    import hashlib
    if workload != "layer16_64f_chunk8f" or not os.path.exists(TRAFFIC_PROFILE):
        return None
    h = hashlib.sha256()
    for f in ("ttt_fwd.hip", "ttt_common.h"):
        with open(os.path.join(ROOT, "paper_2604_08542_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    text = open(TRAFFIC_PROFILE).read()
    if f"ttt_fwd.hip+ttt_common.h: {h.hexdigest()[:16]}" not in text:
        return None
    for line in text.splitlines():
        if line.startswith(f"traffic_per_launch_bytes {io} = "):
            return float(line.split("=")[1])
    return None


def run_variant(w, dev_inputs, io, steps, warmup, lib):
    import ctypes

    import torch

    from paper_2604_08542_amd import ops
    dt = torch.float32 if io == "f32" else torch.bfloat16
    Q, K, V = (dev_inputs[n].to(dt) for n in ("Q", "K", "V"))
    W1, W2 = dev_inputs["W1"], dev_inputs["W2"]
    cu = w.cu_seqlens()
    O = torch.empty_like(Q)
    prob = ops.problem(Q, w.d_hidden, 0, w.chunk_tokens, w.eta, ops._flags(True))
    ws = ops.workspace(prob, len(cu) - 1, Q.device)

    def step():
        return ops.batched_fwd(Q, K, V, cu, W1, W2, w.eta, w.chunk_tokens, out=O, ws=ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    lib.ttt_profile_enable(2)  # events around the chunk-step kernels only (the roofline kernel)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (ctypes.c_double * 4)()
    n = (ctypes.c_int64 * 4)()
    lib.ttt_profile_read(4, ms, n)
    lib.ttt_profile_enable(0)
    ms_step = (t1 - t0) * 1e3 / steps
    kern_ms_per_pass = ms[0] / steps
    achieved = alg_flops(w) / (kern_ms_per_pass * 1e-3) / 1e12
    return dict(
        io=io, ms_per_step=ms_step, tokens_per_s=w.n_tokens / (ms_step * 1e-3),
        step_kernel=dict(launches_per_pass=n[0] / steps, avg_launch_us=ms[0] / max(n[0], 1) * 1e3,
                         ms_per_pass=kern_ms_per_pass),
        roofline=dict(bound="mfma", achieved=achieved, peak=PEAK[io], unit="TFLOP/s",
                      frac=achieved / PEAK[io], traffic=measured_traffic(io, w.name),
                      traffic_unit="HBM bytes per step-kernel launch"),
        out=r,
    )


def time_fn(fn, steps, warmup, lib):
    """Wall time per call (synchronised, no instrumentation: the events the
    library records around every launch cost host time that would inflate
    launch-heavy forms), then per-kind kernel times from the library's event
    instrumentation over a separate, shorter run of calls."""
    import ctypes

    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k = max(2, steps // 4)
    lib.ttt_profile_enable(1)
    for _ in range(k):
        fn()
    torch.cuda.synchronize()
    ms = (ctypes.c_double * 5)()
    n = (ctypes.c_int64 * 5)()
    lib.ttt_profile_read(5, ms, n)
    lib.ttt_profile_enable(0)
    kinds = ["fwd_step", "update", "bwd_step", "bwd_reduce", "bwd_prep"]
    per = {kd: dict(ms_per_call=ms[i] / k, launches_per_call=n[i] / k,
                    avg_launch_us=ms[i] / max(n[i], 1) * 1e3) for i, kd in enumerate(kinds) if n[i]}
    return (t1 - t0) * 1e3 / steps, per, out


def length_sweep(steps, warmup, lib, frames=(150, 270, 510, 990)):
    """One sequence of F frames x 1374 tokens, 16 heads x 64, h = 256,
    chunks of 8 frames, BF16 operands, for F in `frames` (the layer shape at
    growing sequence length): with every chunk step filling the chip,
    tokens/s should not depend on the length."""
    import torch

    from paper_2604_08542_amd import ops
    from workloads import make_inputs_torch
    H, d, h, M, eta = 16, 64, 256, 8 * 1374, 0.05
    rows = {}
    for f in frames:
        n = f * 1374
        dev = make_inputs_torch(n, H, d, h, seed=0, io_dtype="bf16")
        O = torch.empty_like(dev["Q"])
        ms, per, _ = time_fn(lambda: ops.chunk_fwd(dev["Q"], dev["K"], dev["V"], dev["W1"], dev["W2"], eta, M, out=O,
                                                   want_final=False), max(2, steps // 4), max(1, warmup // 2), lib)
        kms = per["fwd_step"]["ms_per_call"]
        ach = 14.0 * d * h * n * H / (kms * 1e-3) / 1e12
        rows[str(f)] = dict(tokens=n, chunks=-(-n // M), ms_per_step=ms, tokens_per_s=n / (ms * 1e-3),
                            step_kernel_tflops=ach, frac_bf16_peak=ach / PEAK["bf16"])
        del dev, O
        torch.cuda.empty_cache()
    tps = [r["tokens_per_s"] for r in rows.values()]
    return dict(workload="one sequence, 16x64, h256, chunk 8 frames, bf16", frames=rows,
                tokens_per_s_max_over_min=max(tps) / min(tps))


def extra_variants(steps, warmup, lib, forms=("gcs", "fwd_bwd", "batched_fwd", "batched_fwd_bwd", "amu",
                                             "single_head", "length_sweep")):
    """The other forms on their own workloads: GCS forward (same layer
    workload), forward+backward (differentiation workload), batched forward
    (8 uneven sequences)."""
    import torch

    from paper_2604_08542_amd import ops
    from workloads import WORKLOADS, make_inputs_torch
    res = {}
    if "length_sweep" in forms:
        res["length_sweep_bf16"] = length_sweep(steps, warmup, lib)
    # GCS forward on the layer workload, BF16 and FP32 operands
    w = WORKLOADS["layer16_64f_chunk8f"]
    for io in (("bf16", "f32") if "gcs" in forms else ()):
        dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype=io)
        ms, per, _ = time_fn(lambda: ops.gcs_fwd(dev["Q"], dev["K"], dev["V"], dev["W1"], dev["W2"], w.eta,
                                                 w.chunk_tokens), steps, warmup, lib)
        kms = per["fwd_step"]["ms_per_call"]
        ach = alg_flops(w) / (kms * 1e-3) / 1e12
        res[f"gcs_fwd_{io}"] = dict(workload=w.name, ms_per_step=ms, tokens_per_s=w.n_tokens / (ms * 1e-3),
                                    kernels=per, roofline=dict(bound="mfma", achieved=ach, peak=PEAK[io],
                                                               unit="TFLOP/s", frac=ach / PEAK[io]))
        del dev
    # the paper's memory unit (SwiGLU, dot-product loss, token-wise steps) on the layer workload
    for io in (("bf16", "f32") if "amu" in forms else ()):
        from workloads import make_eta_tok
        dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype=io)
        g = torch.Generator(device="cuda")
        g.manual_seed(1)
        W3 = torch.randn(dev["W1"].shape, generator=g, device="cuda") / float(w.d_head) ** 0.5
        et = torch.from_numpy(make_eta_tok(w.n_tokens, w.n_heads, w.chunk_tokens, 20.0, 0)).cuda()
        O = torch.empty_like(dev["Q"])
        for sync in ("chain", "gcs"):
            ms, per, _ = time_fn(lambda: ops.amu_fwd(dev["Q"], dev["K"], dev["V"], et, dev["W1"], dev["W2"], W3,
                                                     w.chunk_tokens, sync=sync, want_final=False, out=O),
                                 steps, warmup, lib)
            kms = per["fwd_step"]["ms_per_call"]
            # 12 d h per token-head for the update (K W1, K W3, E W2^T, three token sums) + 6 d h apply
            ach = 18.0 * w.d_head * w.d_hidden * w.n_tokens * w.n_heads / (kms * 1e-3) / 1e12
            res[f"amu_{sync}_{io}"] = dict(workload=w.name, ms_per_step=ms, tokens_per_s=w.n_tokens / (ms * 1e-3),
                                           kernels=per, roofline=dict(bound="mfma", achieved=ach, peak=PEAK[io],
                                                                      unit="TFLOP/s", frac=ach / PEAK[io]))
            # forward + reverse mode (the backward recomputes the weights it needs)
            dO = torch.randn(dev["Q"].shape, generator=g, device="cuda").to(dev["Q"].dtype)

            def fb():
                ops.amu_fwd(dev["Q"], dev["K"], dev["V"], et, dev["W1"], dev["W2"], W3, w.chunk_tokens, sync=sync,
                            want_final=False, out=O)
                return ops.amu_bwd(dev["Q"], dev["K"], dev["V"], et, dev["W1"], dev["W2"], W3, w.chunk_tokens, dO,
                                   sync=sync)
            ms, per, _ = time_fn(fb, max(2, steps // 2), 1, lib)
            bk = per["bwd_step"]
            res[f"amu_fwd_bwd_{sync}_{io}"] = dict(workload=w.name, ms_per_step=ms,
                                                   tokens_per_s=w.n_tokens / (ms * 1e-3), kernels=per,
                                                   bwd_kernels_ms=bk["ms_per_call"])
            del dO
        del dev, O, W3, et
    # single-head chains: 4 chunks x 1374 tokens (FP32) and 256 chunks x 1374 tokens (BF16, precision form)
    for name, io in ((("single_head_4x1374", "f32"), ("single_head_256x1374_bf16", "bf16"))
                     if "single_head" in forms else ()):
        ws_ = WORKLOADS[name]
        dev = make_inputs_torch(ws_.n_tokens, ws_.n_heads, ws_.d_head, ws_.d_hidden, seed=0, io_dtype=io)
        O = torch.empty_like(dev["Q"])
        ms, per, _ = time_fn(lambda: ops.chunk_fwd(dev["Q"], dev["K"], dev["V"], dev["W1"], dev["W2"], ws_.eta,
                                                   ws_.chunk_tokens, out=O, want_final=False), steps, warmup, lib)
        kms = per["fwd_step"]["ms_per_call"]
        ach = alg_flops(ws_) / (kms * 1e-3) / 1e12
        key = name if name.endswith(io) else f"{name}_{io}"
        res[key] = dict(workload=name, ms_per_step=ms, tokens_per_s=ws_.n_tokens / (ms * 1e-3),
                                   kernels=per, roofline=dict(bound="latency (one chain)", achieved=ach,
                                                              peak=PEAK[io], unit="TFLOP/s", frac=ach / PEAK[io]))
        # the same pass replayed from a captured HIP graph (no host launch cost per chunk step)
        prob = ops.problem(dev["Q"], ws_.d_hidden, ws_.n_tokens, ws_.chunk_tokens, ws_.eta, ops._flags(True))
        wsb = ops.workspace(prob, 1, dev["Q"].device)

        def one():
            ops.chunk_fwd(dev["Q"], dev["K"], dev["V"], dev["W1"], dev["W2"], ws_.eta, ws_.chunk_tokens, out=O,
                          want_final=False, ws=wsb)
        one()
        torch.cuda.synchronize()
        ref = O.clone()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            one()
        torch.cuda.synchronize()
        O.zero_()
        graph.replay()
        torch.cuda.synchronize()
        same = bool(torch.equal(O, ref))
        for _ in range(warmup):
            graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            graph.replay()
        torch.cuda.synchronize()
        gms = (time.perf_counter() - t0) * 1e3 / steps
        res[key].update(graph_ms_per_step=gms, graph_tokens_per_s=ws_.n_tokens / (gms * 1e-3),
                                   graph_replay_matches_eager=same)
        del dev, O, graph, wsb
    # forward + backward on the differentiation workload
    w = WORKLOADS["layer16_32f_chunk4f_bwd"]
    for io in (("bf16", "f32") if "fwd_bwd" in forms else ()):
        dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype=io, with_dO=True)

        def fb():
            f = ops.chunk_fwd(dev["Q"], dev["K"], dev["V"], dev["W1"], dev["W2"], w.eta, w.chunk_tokens,
                              save_ckpt=True, want_final=False)
            return ops.chunk_bwd(dev["Q"], dev["K"], dev["V"], dev["W1"], dev["W2"], w.eta, w.chunk_tokens,
                                 f["ckpt"], dev["dO"])
        ms, per, _ = time_fn(fb, max(2, steps // 2), 1, lib)
        # algorithmic: forward 14 d h + backward 28 d h per token-head
        fl = 42.0 * w.d_head * w.d_hidden * w.n_tokens * w.n_heads
        bms = per["bwd_step"]["ms_per_call"]
        bach = 28.0 * w.d_head * w.d_hidden * w.n_tokens * w.n_heads / (bms * 1e-3) / 1e12
        res[f"fwd_bwd_{io}"] = dict(workload=w.name, ms_per_step=ms, tokens_per_s=w.n_tokens / (ms * 1e-3),
                                    alg_tflops_per_s=fl / (ms * 1e-3) / 1e12, kernels=per,
                                    bwd_step_roofline=dict(bound="mfma", achieved=bach, peak=PEAK[io],
                                                           unit="TFLOP/s", frac=bach / PEAK[io]))
        del dev
    # batched forward: 8 uneven sequences, BF16
    w = WORKLOADS["batch8_uneven_chunk8f_bf16"]
    cu = w.cu_seqlens()
    if "batched_fwd" not in forms and "batched_fwd_bwd" not in forms:
        return res
    if "batched_fwd" in forms:
        dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype="bf16")
        O = torch.empty_like(dev["Q"])
        ms, per, _ = time_fn(lambda: ops.batched_fwd(dev["Q"], dev["K"], dev["V"], cu, dev["W1"], dev["W2"], w.eta,
                                                     w.chunk_tokens, out=O, want_final=False), steps, warmup, lib)
        kms = per["fwd_step"]["ms_per_call"]
        ach = alg_flops(w) / (kms * 1e-3) / 1e12
        res["batched_fwd_bf16"] = dict(workload=w.name, ms_per_step=ms, tokens_per_s=w.n_tokens / (ms * 1e-3),
                                       kernels=per, roofline=dict(bound="mfma", achieved=ach, peak=PEAK["bf16"],
                                                                  unit="TFLOP/s", frac=ach / PEAK["bf16"]))
        del dev, O
    if "batched_fwd_bwd" not in forms:
        torch.cuda.empty_cache()
        return res
    # batched forward (with checkpoints) + batched backward: 8 uneven sequences, BF16
    dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype="bf16", with_dO=True)

    def bfb():
        f = ops.batched_fwd(dev["Q"], dev["K"], dev["V"], cu, dev["W1"], dev["W2"], w.eta, w.chunk_tokens,
                            save_ckpt=True, want_final=False)
        return ops.batched_bwd(dev["Q"], dev["K"], dev["V"], cu, dev["W1"], dev["W2"], w.eta, w.chunk_tokens,
                               f["ckpt"], dev["dO"])
    ms, per, _ = time_fn(bfb, max(2, steps // 4), 1, lib)
    bms = per["bwd_step"]["ms_per_call"]
    bach = 28.0 * w.d_head * w.d_hidden * w.n_tokens * w.n_heads / (bms * 1e-3) / 1e12
    res["batched_fwd_bwd_bf16"] = dict(workload=w.name, ms_per_step=ms, tokens_per_s=w.n_tokens / (ms * 1e-3),
                                       kernels=per,
                                       bwd_step_roofline=dict(bound="mfma", achieved=bach, peak=PEAK["bf16"],
                                                              unit="TFLOP/s", frac=bach / PEAK["bf16"]))
    del dev
    torch.cuda.empty_cache()
    return res


def cpu_baseline(w, host_inputs, gpu_out, n_heads):
    """Time the FP64 oracle on the host for `n_heads` heads of the same
    inputs (a bounded sample of the workload) and compare those heads."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import oracle
    sl = slice(0, n_heads)
    x = {k: host_inputs[k][:, sl] for k in ("Q", "K", "V")}
    W1, W2 = host_inputs["W1"][sl], host_inputs["W2"][sl]
    cu = w.cu_seqlens()
    t0 = time.perf_counter()
    ref = oracle.ttt_forward_batched(x["Q"], x["K"], x["V"], cu, W1, W2, w.eta, w.chunk_tokens)
    dt = time.perf_counter() - t0
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    tok_s = w.n_tokens * (n_heads / w.n_heads) / dt
    # the same oracle on one thread, one head
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        oracle.ttt_forward_batched(x["Q"][:, :1], x["K"][:, :1], x["V"][:, :1], cu, W1[:1], W2[:1], w.eta,
                                   w.chunk_tokens)
        dt1 = time.perf_counter() - t1
    one = dict(value=w.n_tokens / w.n_heads / dt1, unit="tokens/s", cores=1,
               sample=f"1 of {w.n_heads} heads over all {w.n_tokens} tokens ({dt1:.1f} s), scaled to all heads")
    errs = {}
    for io, out in gpu_out.items():
        O = out["O"][:, sl].float().cpu().numpy().astype(np.float64)
        errs[io] = float(np.linalg.norm(O - ref["O"]) / np.linalg.norm(ref["O"]))
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=tok_s, unit="tokens/s", cores=threads, kind="oracle",
                sample=f"FP64 numpy oracle forward on {n_heads} of {w.n_heads} heads over all "
                       f"{w.n_tokens} tokens ({dt:.1f} s), scaled to all heads",
                seconds=dt, single_thread=one, host_cpus=os.cpu_count(), cpu_model=model), errs


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); chains shard over GPUs by "
              f"(sequence, head) but no multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2604_08542_amd as P
    from workloads import WORKLOADS, make_inputs_torch
    lib = P.load()
    w = WORKLOADS[a.workload]
    dev = make_inputs_torch(w.n_tokens, w.n_heads, w.d_head, w.d_hidden, seed=0, io_dtype=w.io_dtype)
    variants = {}
    for io in a.variants.split(","):
        variants[io] = run_variant(w, dev, io, a.steps, a.warmup, lib)
        print(f"# {io}: {variants[io]['ms_per_step']:.3f} ms/step, "
              f"{variants[io]['tokens_per_s']:.4g} tokens/s, step-kernel "
              f"{variants[io]['roofline']['achieved']:.1f} TFLOP/s", file=sys.stderr, flush=True)
    extra = {}
    if not a.no_extra:
        extra = extra_variants(a.steps, a.warmup, lib, tuple(f for f in a.forms.split(",") if f))
        for k, v in extra.items():
            if "frames" in v:
                for f, r in v["frames"].items():
                    print(f"# {k} {f} frames: {r['ms_per_step']:.3f} ms/step, {r['tokens_per_s']:.4g} tokens/s",
                          file=sys.stderr, flush=True)
                continue
            print(f"# {k}: {v['ms_per_step']:.3f} ms/step, {v['tokens_per_s']:.4g} tokens/s", file=sys.stderr,
                  flush=True)
    if a.copy_calib:
        src = torch.empty(128 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    main_io = w.io_dtype if w.io_dtype in variants else next(iter(variants))
    m = variants[main_io]
    cpu = None
    errs = {}
    if not a.no_cpu_baseline:
        host = {k: dev[k][:, : a.cpu_heads].float().cpu().numpy() for k in ("Q", "K", "V")}
        host["W1"] = dev["W1"].cpu().numpy()
        host["W2"] = dev["W2"].cpu().numpy()
        cpu, errs = cpu_baseline(w, host, {io: variants[io]["out"] for io in variants}, a.cpu_heads)
        if main_io == "f32":
            # the BF16 variant's inputs were rounded from these FP32 values
            errs["bf16_incl_input_rounding"] = errs.pop("bf16")
    line = {
        "metric": METRIC,
        "value": m["tokens_per_s"],
        "unit": "tokens/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_io,
        "data": "synthetic",
        "config": {"workload": w.name, "heads": w.n_heads, "d_head": w.d_head, "d_hidden": w.d_hidden,
                   "frames": list(w.frames), "tokens": w.n_tokens, "chunk_tokens": w.chunk_tokens,
                   "eta": w.eta, "pass": "forward"},
        "roofline": m["roofline"],
        "cpu_baseline": cpu,
        "variants": {io: {k: v for k, v in var.items() if k != "out"} for io, var in variants.items()},
        "speedup_bf16_over_f32": (variants["f32"]["ms_per_step"] / variants["bf16"]["ms_per_step"]
                                  if "f32" in variants and "bf16" in variants else None),
        "rel_err_vs_oracle_sampled_heads": errs,
        "other_forms": extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
