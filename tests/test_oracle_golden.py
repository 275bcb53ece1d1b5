"""The oracle still reproduces the fixtures in tests/golden/ (written by
tests/golden/make_golden.py from the oracle alone): a guard against silent
changes of its arithmetic."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

from make_golden import compute  # noqa: E402


def load():
    out = {}
    with open(os.path.join(HERE, "golden", "tiny_ragged_chain.txt")) as fh:
        lines = [ln for ln in fh.read().splitlines() if not ln.startswith("#")]
    for head, vals in zip(lines[0::2], lines[1::2]):
        name, *shape = head.split()
        out[name] = np.array([float(t) for t in vals.split()]).reshape([int(s) for s in shape])
    return out


def test_oracle_matches_golden():
    ref = load()
    now = compute()
    assert set(ref) == set(now)
    for k in ref:
        np.testing.assert_allclose(now[k], ref[k], rtol=1e-12, atol=1e-14, err_msg=k)
