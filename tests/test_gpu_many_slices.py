"""Fields with more slices than one dispatch of one-workgroup-per-slice
kernels takes (2^23 workgroups): the launches are split, and every slice is
still encoded and decoded.

A 2D FP32 field of 8192 x 8192 x 48 steps (12.9 GB) in 4 x 4 patches and
16-step windows has 12.6 M blocks of one slice each.
* absolute bound (plain form): the device decode and the stream decoder
  (dls_decompress, one workgroup per slice) write every value (a NaN-filled
  output keeps none), agree bit for bit, and hold |x - x_hat| <= eps at
  every point;
* L2 mode (its Gram, encode and decode take one workgroup per slice): every
  value written and the NRMSE within the target.
"""
import os
import sys

import pytest
import torch

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import paper_2601_20113_amd as dls  # noqa: E402

pytestmark = pytest.mark.gpu

NX, NY, NT = 8192, 8192, 48


@pytest.fixture(scope="module")
def field():
    from synth import gpu as sg
    f = torch.empty((1, NT, 1, NY, NX), dtype=torch.float32, device="cuda")
    sg.blobs_into(f[0], nblobs=16384, seed=51)
    torch.cuda.synchronize()
    yield f
    del f
    torch.cuda.empty_cache()


def _params(eps, **kw):
    return dls.Params(nx=NX, ny=NY, nz=1, nt=NT, nvars=1, dtype="f32", px=4, py=4, pz=1, window=16,
                      eps=eps, **kw)


def test_abs_bound_many_slices(field):
    print("case 8192 x 8192 x 48 FP32, 4 x 4 patches, absolute bound", flush=True)
    lo, hi = dls.value_range(field)
    eps = 1e-3 * (hi[0] - lo[0])
    enc = dls.Encoder()
    enc.encode(field, _params([eps]))
    assert enc.info().nblocks == 3 * (NX // 4) * (NY // 4) > (1 << 23)
    out = torch.full_like(field, float("nan"))
    enc.decode(out)
    torch.cuda.synchronize()
    assert not torch.isnan(out).any().item()
    err = max((field[:, t].double() - out[:, t].double()).abs().max().item() for t in range(NT))
    assert err <= eps, (err, eps)
    stream = enc.finalize()
    enc.close()
    back = dls.decompress(stream)
    assert torch.equal(back.view(torch.int32), out.view(torch.int32))


def test_l2_many_slices(field):
    print("case 8192 x 8192 x 48 FP32, 4 x 4 patches, L2 mode", flush=True)
    enc = dls.Encoder()
    enc.encode(field, _params([1e-3], l2=True))
    out = torch.full_like(field, float("nan"))
    enc.decode(out)
    torch.cuda.synchronize()
    assert not torch.isnan(out).any().item()
    num = sum((field[:, t].double() - out[:, t].double()).pow(2).sum().item() for t in range(NT))
    den = sum(field[:, t].double().pow(2).sum().item() for t in range(NT))
    d = (num / den) ** 0.5
    assert d <= 1e-3, d
    enc.close()
