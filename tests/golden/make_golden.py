"""Writes the regression fixtures in this folder from the FP64 oracle alone
(no HIP code): a tiny ragged chain (N=11, H=2, d=3, h=5, chunks of 4) of the
main path (forward outputs and the backward of sum <O, dO>) and of the paper
memory unit (chain and GCS).  The values are the oracle's, pinned elsewhere
against finite differences and closed forms; these files only make any later
change of the oracle's arithmetic visible.

    python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as orc  # noqa: E402
from workloads import make_inputs  # noqa: E402


def tiny():
    x = {k: v.astype(np.float64) for k, v in make_inputs(11, 2, 3, 5, seed=90, with_dO=True).items()}
    W3 = np.random.default_rng(91).standard_normal((2, 3, 5)) / np.sqrt(3)
    et = np.random.default_rng(92).uniform(0.05, 0.3, (11, 2))
    return x, W3, et


def compute():
    x, W3, et = tiny()
    out = {}
    f = orc.ttt_forward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.4, 4)
    b = orc.ttt_backward(x["Q"], x["K"], x["V"], x["W1"], x["W2"], 0.4, 4, x["dO"])
    for k in ("O", "W1_T", "W2_T", "loss"):
        out["chain_" + k] = f[k]
    for k in ("dQ", "dK", "dV", "dW1_0", "dW2_0", "deta"):
        out["chain_" + k] = b[k]
    for sync in ("chain", "gcs"):
        a = orc.ttt_forward_swiglu(x["Q"], x["K"], x["V"], x["W1"], x["W2"], W3, et, 4, sync=sync)
        for k in ("O", "W1_T", "W2_T", "W3_T"):
            out[f"amu_{sync}_{k}"] = a[k]
    return out


def main():
    with open(os.path.join(HERE, "tiny_ragged_chain.txt"), "w") as fh:
        fh.write("# FP64 oracle outputs, tiny ragged case (see make_golden.py); name shape then values\n")
        for k, v in compute().items():
            v = np.asarray(v, np.float64)
            fh.write(f"{k} {' '.join(str(s) for s in v.shape)}\n")
            fh.write(" ".join(repr(float(t)) for t in v.ravel()) + "\n")


if __name__ == "__main__":
    main()
