"""The oracle against hand-worked examples stored under tests/golden/.

Each fixture holds the inputs, the values worked out by hand from the
definitions it cites, and the derivation; none comes from running code.
"""
import json
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle import dls  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def test_rank1_block():
    g = load("rank1_block_2x2.json")
    x = np.array(g["inputs"]["x"])
    e = g["expected"]
    c = dls.encode_block(x, g["inputs"]["eps"], g["inputs"]["rcap"], np.float64)
    assert np.allclose(c.lam, e["lam"], rtol=0, atol=1e-12)
    assert c.r == e["rank"]
    assert c.qV[:, 0].tolist() == e["qV"]
    assert c.qA[:, 0].tolist() == e["qA"]
    assert (c.qV @ c.qA.T).tolist() == e["S"]
    assert dls.unzigzag8(c.codes).tolist() == e["q"]
    assert c.codes.tolist() == e["codes"]
    assert c.esc_values.size == e["escapes"]
    assert np.abs(c.out - x).max() <= e["max_abs_error_below"]


def test_escape_threshold():
    g = load("escape_threshold_2x2.json")
    eps, rcap = g["inputs"]["eps"], g["inputs"]["rcap"]
    e = g["expected"]
    for v, code, esc in zip(g["inputs"]["v"], e["code_11"], e["escaped"]):
        x = np.array([[100.0, 0.0], [0.0, v]])
        c = dls.encode_block(x, eps, rcap, np.float64)
        assert c.qA[:, 0].tolist() == e["qA"]
        assert int(c.codes[1, 1]) == code
        assert (c.esc_values.size == 1) == esc
        assert np.abs(c.out - x).max() <= eps


def spike_field(g):
    i = g["inputs"]
    f = np.zeros((1, 2, 1, i["ny"], i["nx"]))
    x, y, val = i["spike"]
    f[0, 0, 0, y, x] = val
    return f


def test_quadtree_spike():
    g = load("quadtree_spike_8x8.json")
    i, e = g["inputs"], g["expected"]
    f = spike_field(g)
    p = dls.Params(nx=i["nx"], ny=i["ny"], nz=1, nt=2, nvars=1, dtype="f64", px=i["px"], py=i["px"], pz=1,
                   window=2, eps=[0.1], pmin=i["pmin"], adaptive=True)
    assert dls.percentile80(dls.gradient_magnitude(f[0, 0])) == e["p80"]
    leaves, bits = dls.adaptive_leaves(f[0, 0], p)
    assert list(bits) == e["bits"]
    assert [[L[0], L[1], L[6]] for L in leaves] == e["leaves"]
    assert all(L[3] == L[6] and L[4] == L[6] and L[5] == 1 for L in leaves)
