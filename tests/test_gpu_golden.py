"""The HIP path against the hand-worked examples under tests/golden/ (the
same fixtures the oracle is pinned to), through the C ABI: the stream the
library writes is parsed with the format reader of the test side and its
ranks, quantized basis and coefficients, residual codes and escapes are
compared with the values worked out by hand; the adaptive plan's split bits
and leaves likewise."""
import json
import os
import sys

import numpy as np
import pytest
import torch

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import gpu_helpers as H  # noqa: E402
import paper_2601_20113_amd as dls  # noqa: E402
from oracle import container, dls as odls  # noqa: E402

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def one_block_field(x):
    """Field (1 var, W steps, 1 x 1 x M) whose single block is X (W x M)."""
    w, m = x.shape
    return np.ascontiguousarray(x.reshape(1, w, 1, 1, m))


def encode_one_block(x, eps, rcap):
    w, m = x.shape
    p = odls.Params(nx=m, ny=1, nz=1, nt=w, nvars=1, dtype="f64", px=m, py=1, pz=1, window=w, eps=[eps],
                    r_max=rcap)
    g = H.GpuRun(one_block_field(x), p)
    dec = container.unpack(g.stream)
    assert len(dec.codes) == 1
    out = dls.decompress(g.stream).cpu().numpy().reshape(w, m)
    return dec.codes[0], out


def test_rank1_block():
    print("golden rank1_block_2x2", flush=True)
    g = load("rank1_block_2x2.json")
    x = np.array(g["inputs"]["x"])
    e = g["expected"]
    c, out = encode_one_block(x, g["inputs"]["eps"], g["inputs"]["rcap"])
    assert c.r == e["rank"]
    assert c.qV[:, 0].tolist() == e["qV"]
    assert c.qA[:, 0].tolist() == e["qA"]
    assert c.codes.tolist() == e["codes"]
    assert c.esc_values.size == e["escapes"]
    S = np.array(e["S"], dtype=np.float64)
    assert np.array_equal(out, S * (g["inputs"]["eps"] / 65536.0))
    assert np.abs(out - x).max() <= e["max_abs_error_below"]


def test_escape_threshold():
    print("golden escape_threshold_2x2", flush=True)
    g = load("escape_threshold_2x2.json")
    eps, rcap = g["inputs"]["eps"], g["inputs"]["rcap"]
    e = g["expected"]
    for v, code, esc in zip(g["inputs"]["v"], e["code_11"], e["escaped"]):
        x = np.array([[100.0, 0.0], [0.0, v]])
        c, out = encode_one_block(x, eps, rcap)
        assert c.qA[:, 0].tolist() == e["qA"]
        assert int(c.codes[1, 1]) == code
        assert (c.esc_values.size == 1) == esc
        if esc:
            assert out[1, 1] == v
        assert np.abs(out - x).max() <= eps


def test_quadtree_spike():
    print("golden quadtree_spike_8x8", flush=True)
    g = load("quadtree_spike_8x8.json")
    i, e = g["inputs"], g["expected"]
    f = np.zeros((1, 2, 1, i["ny"], i["nx"]))
    x, y, val = i["spike"]
    f[0, 0, 0, y, x] = val
    p = odls.Params(nx=i["nx"], ny=i["ny"], nz=1, nt=2, nvars=1, dtype="f64", px=i["px"], py=i["px"], pz=1,
                    window=2, eps=[0.1], pmin=i["pmin"], adaptive=True)
    run = H.GpuRun(f, p)
    _, bits, nb, _, _ = container.parse_header(run.stream)
    assert list(bits[0]) == e["bits"]
    desc = dls.d2h(run.enc.info().d_desc, nb * 32).view(np.int32).reshape(nb, 8)
    got = [[int(d[0]), int(d[1]), int(d[4]) & 255] for d in desc]
    assert got == e["leaves"]
