"""The L2 / NRMSE-bounded mode (DLS_L2) through the C ABI, against the FP64
oracle (oracle.l2) on the same seeded fields:

* every variable's NRMSE of the decoded GPU stream is within its target, and
  every block's exact squared error within its budget e2 (computed from the
  oracle's budget, to 1e-12 relative);
* the oracle's decoder and the library's decoder give bit-identical fields
  from the GPU stream, and so does the device decode of the context;
* final ranks equal the oracle's on >= 99 % of blocks (both Grams are FP64;
  a different summation order can move a tail that sits on 0.36 e2 to the
  other side, and the exact check settles it), raw blocks exactly where the
  oracle has them on non-finite input and on a target below the basis
  grid's resolution;
* the compression ratio within 1 % of the oracle's; dls_stats agrees with
  the stream's ranks;
* the precision parameter has no effect: bf16 gives the fp32 stream.
Cases: FP64 2D blobs, FP32 drifting spectrum (2 variables, W = 16 and
W = 32), an adaptive quadtree; targets 1e-2 .. 1e-4.
"""
import os
import sys

import numpy as np
import pytest
import torch

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import gpu_helpers as H  # noqa: E402
import paper_2601_20113_amd as dls  # noqa: E402
import synth  # noqa: E402
from oracle import container, dls as odls, l2  # noqa: E402

pytestmark = pytest.mark.gpu


def _case(name, target):
    if name == "blobs_f64_64x64x32":
        f = synth.blobs2d(nx=64, ny=64, nt=32, seed=1)
        kw = dict(nx=64, ny=64, nz=1, nt=32, nvars=1, dtype="f64", px=8, py=8, pz=1, window=16)
    elif name == "spec_f32_w16_2var":
        f = np.concatenate([synth.spectrum(40, 36, 20, 24, nmodes=16, seed=s, drift=True) for s in (11, 12)])
        kw = dict(nx=40, ny=36, nz=20, nt=24, nvars=2, dtype="f32", px=16, py=16, pz=16, window=16)
    elif name == "spec_f32_w32":
        f = synth.spectrum(24, 20, 16, 40, nmodes=12, seed=13, drift=True)
        kw = dict(nx=24, ny=20, nz=16, nt=40, nvars=1, dtype="f32", px=8, py=8, pz=8, window=32)
    elif name == "adaptive_quad_f32":
        f = synth.blobs2d(nx=96, ny=80, nt=20, seed=6, nblobs=12, dtype=np.float32)
        kw = dict(nx=96, ny=80, nz=1, nt=20, nvars=1, dtype="f32", px=32, py=32, pz=1, window=16, pmin=4,
                  adaptive=True)
    else:
        raise KeyError(name)
    return f, odls.Params(eps=[target] * kw["nvars"], **kw)


def _lib(p, precision="fp32"):
    lp = H.to_lib_params(p, precision)
    lp.l2 = True
    return lp


def _check(f, p, precision="fp32", rank_share=0.99):
    enc_or = l2.encode(f, p)
    ref = container.pack_l2(enc_or)
    e = dls.Encoder()
    t = torch.from_numpy(f).cuda()
    e.encode(t, _lib(p, precision))
    inf = e.info()
    stream = e.finalize()
    out = dls.decompress(stream).cpu().numpy()
    # the oracle's decoder on the GPU stream, and the device decode
    assert np.array_equal(l2.decompress(stream).view(np.uint8), out.view(np.uint8))
    dev = torch.full_like(t, float("nan"))
    e.decode(dev)
    torch.cuda.synchronize()
    assert np.array_equal(dev.cpu().numpy().view(np.uint8), out.view(np.uint8))
    gpu = container.unpack_l2(stream)
    nrm = [l2.nrmse_fraction(f[v], out[v]) for v in range(p.nvars)]
    c = l2.variable_budgets(f, p.eps)
    worst = 0.0
    for b, cd in zip(gpu.blocks, gpu.codes):
        xb = odls.gather(f, b).astype(np.float64)
        ob = odls.gather(out, b).astype(np.float64)
        fin = np.isfinite(xb)
        err = float(np.sum(np.where(fin, xb - ob, 0.0) ** 2))
        e2 = l2.block_budget(c[b.var], b)
        worst = max(worst, err / e2 if e2 > 0 else 0.0)
        assert err <= e2 * (1 + 1e-12), (b, err, e2)
    r_or = np.array([cd.r for cd in enc_or.codes])
    r_gpu = np.array([cd.r for cd in gpu.codes])
    same = float(np.mean(r_or == r_gpu))
    cr_g, cr_o = f.nbytes / len(stream), f.nbytes / len(ref)
    st = dls.stats(stream)
    print("targets %s: NRMSE %s, worst block err/e2 %.3f, ranks equal %.4f, raw %d/%d, CR gpu %.3f oracle %.3f, "
          "passes %d" % (p.eps, ["%.3g" % x for x in nrm], worst, same, int(np.sum(r_gpu == l2.RAW)),
                         int(np.sum(r_or == l2.RAW)), cr_g, cr_o, inf.l2_passes), flush=True)
    for v in range(p.nvars):
        assert nrm[v] <= p.eps[v]
    assert same >= rank_share
    assert np.array_equal(r_gpu == l2.RAW, r_or == l2.RAW)
    assert abs(cr_g / cr_o - 1.0) <= 0.01
    assert st["nraw"] == int(np.sum(r_gpu == l2.RAW)) == inf.nraw
    assert sum(st["rank_hist"]) + st["nraw"] == len(gpu.blocks)
    return e, stream


CASES = [(n, t) for n in ("blobs_f64_64x64x32", "spec_f32_w16_2var", "spec_f32_w32", "adaptive_quad_f32")
         for t in (1e-2, 1e-3, 1e-4)]


@pytest.mark.parametrize("name,target", CASES, ids=["%s-%g" % c for c in CASES])
def test_l2_parity(name, target):
    print("case", name, target, flush=True)
    f, p = _case(name, target)
    _check(f, p)


@pytest.mark.parametrize("name", ["blobs_f64_64x64x32", "spec_f32_w16_2var"])
def test_l2_precision_without_effect(name):
    print("case bf16", name, flush=True)
    f, p = _case(name, 1e-3)
    _, a = _check(f, p, "bf16")
    _, b = _check(f, p, "fp32")
    assert a == b


def test_l2_raw_blocks_and_rank_zero():
    """A NaN makes its block raw; a zero region takes rank 0; a target below
    the basis grid's resolution makes every block raw; the bound holds."""
    f = synth.blobs2d(nx=32, ny=16, nt=16, seed=7, nblobs=4)
    f[0, :, 0, :, 16:24] = 0.0
    f[0, 3, 0, 2, 1] = np.nan
    p = odls.Params(nx=32, ny=16, nz=1, nt=16, nvars=1, dtype="f64", px=8, py=8, pz=1, window=16, eps=[1e-2])
    _check(f, p)
    g = synth.blobs2d(nx=16, ny=16, nt=16, seed=8, nblobs=2) + 10.0
    q = odls.Params(nx=16, ny=16, nz=1, nt=16, nvars=1, dtype="f64", px=8, py=8, pz=1, window=16, eps=[1e-12])
    e, _ = _check(g, q)
    assert e.info().nraw == 4


def test_l2_learned_refused():
    f, p = _case("blobs_f64_64x64x32", 1e-2)
    lp = _lib(p)
    lp.learned = True
    with pytest.raises(dls.DlsError):
        dls.Encoder().encode(torch.from_numpy(f).cuda(), lp)
