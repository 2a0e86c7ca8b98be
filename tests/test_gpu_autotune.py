"""The launch-strategy autotuner (paper_2601_20113_amd.autotune) and the
dls_ctx_set_launch knob, through the C ABI: every candidate writes the same
stream (the tuner checks it), the choice is cached per workload signature
and read back without timing, and a negative limit is refused."""
import json
import os
import sys

import numpy as np
import pytest
import torch

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import gpu_helpers as H  # noqa: E402
import paper_2601_20113_amd as dls  # noqa: E402
import synth  # noqa: E402
from oracle import dls as odls  # noqa: E402
from paper_2601_20113_amd import autotune  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", ["c1", "quadtree"])
def test_tuner_streams_equal_and_cache(case, tmp_path):
    print("autotune", case, flush=True)
    if case == "c1":
        f = synth.blobs2d(nx=64, ny=64, nt=32, seed=1)
        p = odls.Params(nx=64, ny=64, nz=1, nt=32, nvars=1, dtype="f64", px=8, py=8, pz=1, window=16,
                        eps=[1e-3 * synth.range_of(f)[0]])
    else:
        f = synth.blobs2d(nx=512, ny=256, nt=20, seed=5, nblobs=64, dtype=np.float32)
        p = odls.Params(nx=512, ny=256, nz=1, nt=20, nvars=1, dtype="f32", px=32, py=32, pz=1, window=16, pmin=4,
                        adaptive=True, eps=[1e-3 * synth.range_of(f)[0]])
    lp = H.to_lib_params(p, "bf16")
    lp.persistent = True
    t = torch.from_numpy(f).cuda()
    cache = str(tmp_path / "tune.json")
    enc = dls.Encoder()
    choice = autotune.tune(t, lp, enc, reps=3, cache=cache)
    print(choice, flush=True)
    assert set(choice["candidates"]) == {"%d/%d" % (l, g) for l in autotune.LIMITS for g in (0, 1)}
    tab = json.load(open(cache))
    assert tab[autotune.signature(lp)]["device_driven_max_items"] == choice["device_driven_max_items"]
    # cached: returned without timing, applied to a fresh encoder
    again = autotune.tune(t, lp, dls.Encoder(), cache=cache)
    assert again == tab[autotune.signature(lp)]
    # the tuned encoder writes the host-driven stream
    enc.encode(t, lp)
    ref = dls.Encoder()
    ref.set_launch(0)
    ref.encode(t, lp)
    assert enc.finalize() == ref.finalize()
    with pytest.raises(dls.DlsError):
        enc.set_launch(-1)
