"""Helpers for GPU parity tests: run the HIP path and the FP64 oracle on the
same seeded inputs and compare per output."""
import numpy as np
import torch

import oracle as orc
from workloads import make_inputs

TOL = {"f32": 1e-4, "bf16": 2e-2}


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def to_dev(x, io):
    dt = torch.float32 if io == "f32" else torch.bfloat16
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda").to(dt)


def inputs(N, H, h, seed, io, with_dO=False):
    x = make_inputs(N, H, 64, h, seed=seed, io_dtype=io, with_dO=with_dO)
    dev = {k: to_dev(v, io) for k, v in x.items() if k in ("Q", "K", "V", "dO")}
    dev["W1"] = torch.from_numpy(x["W1"]).cuda()
    dev["W2"] = torch.from_numpy(x["W2"]).cuda()
    return x, dev


def host(t):
    return t.detach().float().cpu().numpy().astype(np.float64)
