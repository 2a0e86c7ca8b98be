"""The plain eigensolve's sweep statistics and the host-set sweep cap,
through the C ABI.

* With the default cap every block of a drifting FP32 field (ranks 2-6)
  converges: no unconverged block is reported, the sweeps taken lie between
  one and the cap per solved block, and the Jacobi launch has a time.
* Capped at one sweep from the host, the kernel still ends normally, the
  unconverged blocks are counted, every basis is orthonormal to 1e-12 (a
  product of rotations), every decoded value lies within eps, and the
  oracle's decoder gives the library's bits from the stream.
* The cap is refused outside [1, 64].
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
from oracle import dls as odls  # noqa: E402

pytestmark = pytest.mark.gpu


def _field():
    f = np.concatenate([synth.spectrum(48, 40, 32, 32, nmodes=16, seed=s, drift=True) for s in (31, 32)])
    e = [1e-3 * r for r in synth.range_of(f)]
    p = odls.Params(nx=48, ny=40, nz=32, nt=32, nvars=2, dtype="f32", px=16, py=16, pz=16, window=16, eps=e)
    return f, p


def _encode(enc, f, p):
    t = torch.from_numpy(f).cuda()
    enc.encode(t, H.to_lib_params(p, "fp32"), keep_coef=True)
    return enc.info()


def _bases_orthonormal(inf):
    nb, wp = inf.nblocks, inf.wpad
    rank = dls.d2h(inf.d_rank, nb)
    basis = dls.d2h(inf.d_basis, nb * wp * wp * 8).view(np.float64).reshape(nb, wp, wp)
    desc = dls.d2h(inf.d_desc, nb * 32).view(np.int32).reshape(nb, 8)
    for b in range(nb):
        if rank[b] == 0:
            continue
        w = (int(desc[b, 4]) >> 24) & 255
        V = basis[b][:w, :w].T
        assert np.abs(V.T @ V - np.eye(w)).max() <= 1e-12, b


def test_default_cap_converges():
    print("jacobi statistics, default cap", flush=True)
    f, p = _field()
    enc = dls.Encoder()
    inf = _encode(enc, f, p)
    solved = inf.nblocks - inf.nraw
    print("blocks %d, sweeps %d (%.2f per block), unconverged %d, jacobi %.3f ms"
          % (inf.nblocks, inf.jacobi_sweeps, inf.jacobi_sweeps / solved, inf.jacobi_unconverged, inf.jacobi_ms),
          flush=True)
    assert inf.jacobi_unconverged == 0
    assert solved <= inf.jacobi_sweeps <= 12 * solved
    assert inf.jacobi_ms > 0.0
    ranks = dls.d2h(inf.d_rank, inf.nblocks)
    assert ranks.max() >= 2     # the field needs more than one sweep's worth of work


def test_capped_sweeps_counted_and_bound_holds():
    print("jacobi capped at one sweep", flush=True)
    f, p = _field()
    enc = dls.Encoder()
    enc.set_jacobi_sweeps(1)
    inf = _encode(enc, f, p)
    solved = inf.nblocks - inf.nraw
    print("blocks %d, sweeps %d, unconverged %d" % (inf.nblocks, inf.jacobi_sweeps, inf.jacobi_unconverged),
          flush=True)
    assert inf.jacobi_sweeps <= solved
    assert inf.jacobi_unconverged >= solved // 2
    _bases_orthonormal(inf)
    stream = enc.finalize()
    out = dls.decompress(stream).cpu().numpy()
    err = np.abs(out.astype(np.float64) - f.astype(np.float64))
    assert np.all(err <= np.array(p.eps)[:, None, None, None, None])
    assert np.array_equal(odls.decompress(stream).view(np.uint8), out.view(np.uint8))
    # back to the default: converged again in the same context
    enc.set_jacobi_sweeps(12)
    inf = _encode(enc, f, p)
    assert inf.jacobi_unconverged == 0


@pytest.mark.parametrize("cap", [0, 65, -3])
def test_cap_out_of_range_refused(cap):
    enc = dls.Encoder()
    with pytest.raises(dls.DlsError):
        enc.set_jacobi_sweeps(cap)
