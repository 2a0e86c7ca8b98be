"""The device-side decode (dls_decode) against the oracle's decoder.

dls_decode reconstructs the last encode's field straight from the context's
device payload.  On every parity case, on blocks with escapes and raw
blocks, and with the escape-heavy tiny bound it must give bitwise the
values the FP64 oracle's decoder (Alg. 2, Eq. (7)) computes from the stream
dls_finalize writes for the same encode, bitwise the values dls_decompress
gives for that stream, and hold the bound.  It refuses an output buffer
smaller than the encoded field.
"""
import ctypes
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
from test_gpu_parity import CASES, _case  # noqa: E402

pytestmark = pytest.mark.gpu


def _device_vs_stream(f, p):
    lp = H.to_lib_params(p)
    t = torch.from_numpy(f).cuda()
    enc = dls.Encoder()
    enc.encode(t, lp)
    out = torch.full_like(t, float("nan"))
    enc.decode(out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    stream = enc.finalize()
    ref_or = odls.decompress(stream)
    assert np.array_equal(got.view(np.uint8), ref_or.view(np.uint8))
    ref = dls.decompress(stream).cpu().numpy()
    assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))
    return got


@pytest.mark.parametrize("name", CASES)
def test_device_decode_matches_stream_decode(name):
    print("device decode", name, flush=True)
    f, p = _case(name)
    got = _device_vs_stream(f, p)
    for v in range(p.nvars):
        assert np.all(np.abs(got[v].astype(np.float64) - f[v].astype(np.float64)) <= p.eps[v])


def test_device_decode_raw_blocks_and_escapes():
    print("device decode raw blocks and escapes", flush=True)
    f, p = _case("c1_64x64x32_f64")
    f = f.copy()
    f[0, 3, 0, 10, 10] = np.nan
    f[0, 20, 0, 40, 50] = 1e12
    got = _device_vs_stream(f, p)
    assert got[0, 20, 0, 40, 50] == 1e12
    assert np.isnan(got[0, 3, 0, 10, 10])


def test_device_decode_tiny_bound():
    print("device decode tiny bound", flush=True)
    f = synth.blobs2d(nx=32, ny=32, nt=16, seed=5, dtype=np.float32) * 1000.0
    p = odls.Params(nx=32, ny=32, nz=1, nt=16, nvars=1, dtype="f32", px=8, py=8, pz=1, window=16, eps=[1e-5])
    got = _device_vs_stream(f, p)
    assert np.all(np.abs(got.astype(np.float64) - f.astype(np.float64)) <= 1e-5)


def test_device_decode_requires_a_result():
    enc = dls.Encoder()
    out = torch.empty(16, device="cuda")
    with pytest.raises(dls.DlsError):
        enc.decode(out)


def test_device_decode_refuses_a_short_buffer():
    """Through the C ABI: an output byte count below the encoded field's size
    is rejected with DLS_EINVAL before any device work."""
    f, p = _case("c1_64x64x32_f64")
    enc = dls.Encoder()
    enc.encode(torch.from_numpy(f).cuda(), H.to_lib_params(p))
    small = torch.zeros(f.size - 1, dtype=torch.float64, device="cuda")
    st = dls.lib().dls_decode(enc._h, ctypes.c_void_p(small.data_ptr()), small.numel() * 8, None)
    assert st == dls.DLS_EINVAL
    assert bool((small == 0).all())
    with pytest.raises(ValueError):
        enc.decode(small)


@pytest.mark.parametrize("name", ["adaptive_quad_f32_96x80x20", "blobs_f32_96x64x20"])
def test_device_decode_batched_small_slices(name):
    """The batched form (DLS_PERSISTENT) puts slices of at most 64 points in
    small-slice classes, which the device decode runs in 16-lane teams: the
    result equals the oracle's decoder on the stream, bit for bit, on two
    calls in a row (the second replays the captured encode)."""
    print("batched decode", name, flush=True)
    f, p = _case(name)
    lp = H.to_lib_params(p)
    lp.persistent = True
    t = torch.from_numpy(f).cuda()
    enc = dls.Encoder()
    for call in range(2):
        enc.encode(t, lp)
        out = torch.full_like(t, float("nan"))
        enc.decode(out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        stream = enc.finalize()
        assert np.array_equal(got.view(np.uint8), odls.decompress(stream).view(np.uint8)), call
        assert np.all(np.abs(got.astype(np.float64) - f.astype(np.float64)) <= np.array(p.eps)[:, None, None, None, None])
