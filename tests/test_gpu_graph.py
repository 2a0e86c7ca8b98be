"""The device-driven encode (DLS_PERSISTENT on plans of up to 65536 slices)
replayed from a captured hipGraph, through the C ABI.

* After one eager call the context captures the sequence (Gram, eigensolve
  or learned warm start, scans, classes, encode); later calls with the same
  field, problem, buffers and model replay it.  Every replay's stream equals
  the eager context's (graphs off) byte for byte, over several calls with
  eager host work and synchronizations between them.
* A change the graph bakes in forces a new capture and still gives the
  eager stream: a different field tensor, new model weights (same model
  object), a field that needs larger payload buffers (the call falls back to
  the host-driven launch, then captures again).
* The replay is reported (stage times collapse into the encode stage) and is
  not slower than the eager launches on the 64 x 64 x 32 FP64 workload.
"""
import os
import sys
import time

import numpy as np
import pytest
import torch

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import gpu_helpers as H  # noqa: E402
import paper_2601_20113_amd as dls  # noqa: E402
import synth  # noqa: E402
from oracle import dls as odls  # noqa: E402

pytestmark = pytest.mark.gpu


def _c1(seed=1):
    f = synth.blobs2d(nx=64, ny=64, nt=32, seed=seed)
    e = [1e-3 * synth.range_of(f)[0]]
    p = odls.Params(nx=64, ny=64, nz=1, nt=32, nvars=1, dtype="f64", px=8, py=8, pz=1, window=16, eps=e)
    return f, p


def _model(rhat):
    P = np.zeros(dls.NPARAM, np.float32)
    off_b3 = 80 * 128 + 128 + 128 * 128 + 128 + 128 * 272
    P[off_b3 + rhat - 1] = 10.0
    for k in range(16):
        P[off_b3 + 16 + k * 16 + k] = 1.0
    return P, np.concatenate([np.zeros(16), np.ones(16)]).astype(np.float32)


@pytest.mark.parametrize("learned", [False, True])
def test_replay_equals_eager(learned):
    print("graph replay, learned", learned, flush=True)
    f, p = _c1()
    lp = H.to_lib_params(p)
    lp.persistent = True
    lp.learned = learned
    m = None
    if learned:
        m = dls.Model()
        m.set(*_model(3))
    t = torch.from_numpy(f).cuda()
    eager = dls.Encoder()
    eager.set_graphs(False)
    if learned:
        eager.set_model(m, 2, margin=0)
    eager.encode(t, lp)
    ref = eager.finalize()
    g = dls.Encoder()
    if learned:
        g.set_model(m, 2, margin=0)
    for call in range(4):
        g.encode(t, lp)
        inf = g.info()
        # the first call of a context grows its payload buffers (host-driven)
        assert inf.launch_mode == (0 if call == 0 else 1)
        got = g.finalize()
        assert got == ref, call
        # eager host work and a synchronization between replays
        _ = (t * 2.0).sum().item()
        torch.cuda.synchronize()
    # a different tensor with the same contents: captured again, same stream
    t2 = t.clone()
    g.encode(t2, lp)
    assert g.finalize() == ref
    g.encode(t2, lp)
    assert g.finalize() == ref
    if learned:
        # new weights on the same model object: the replay must see them
        m.set(*_model(5))
        eager.encode(t, lp)
        ref5 = eager.finalize()
        g.encode(t, lp)
        assert g.finalize() == ref5
        g.encode(t, lp)
        assert g.finalize() == ref5


def test_replay_after_growth_and_timing():
    """A field that needs more payload room than the captured buffers: the
    call grows them and encodes host-driven, the next calls capture and
    replay again; replays are not slower than eager calls."""
    print("graph replay after growth", flush=True)
    f, p = _c1(1)
    lp = H.to_lib_params(p)
    lp.persistent = True
    g = dls.Encoder()
    e = dls.Encoder()
    e.set_graphs(False)
    t = torch.from_numpy(f).cuda()
    for _ in range(3):
        g.encode(t, lp)
    noisy = f + np.random.default_rng(3).normal(0, 1e-2, f.shape)
    tn = torch.from_numpy(noisy).cuda()
    for _ in range(3):
        g.encode(tn, lp)
        e.encode(tn, lp)
        assert g.finalize() == e.finalize()
    # timing: median wall time of 20 calls each, after warmup
    def wall(enc):
        for _ in range(3):
            enc.encode(t, lp)
        torch.cuda.synchronize()
        ts = []
        for _ in range(20):
            t0 = time.perf_counter()
            enc.encode(t, lp)
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)) * 1e3
    ms_g, ms_e = wall(g), wall(e)
    print("median encode: replay %.3f ms, eager %.3f ms" % (ms_g, ms_e), flush=True)
    assert ms_g <= ms_e * 1.05
