"""The single-pass encode (DLS_PERSISTENT on plans of large FP32 blocks,
W <= 16; reading R28) against the FP64 oracle, through the C ABI.

Per block the oracle runs the same procedure (oracle.dls.encode_block_sketch:
the rank-1 basis of the sketch -- the block's first whole x-rows, at most
1024 points -- verified on the whole block's Gram; the plain eigensolve when
it fails), in FP32 and in bf16-Gram mode:

* the verdict agrees with the oracle's on >= 99 % of blocks (a block whose
  discarded energy sits within rounding of tau may flip), and the GPU's own
  counts add up (verified + deferred = blocks, launch mode 2);
* verified blocks: rank 1, the rank-1 reconstruction q A^T within the
  Davis-Kahan bound of the sketch's FP32-accumulated Gram of the oracle's
  (when the sketch's leading subspace is determined, reading R5);
* deferred blocks: ranks agree on >= 95 % with the plain oracle, coefficients
  within 1e-5 on gap-qualified equal-rank blocks;
* every basis column orthonormal; every decoded value within eps; the
  oracle's decoder and the library's give bit-identical fields from the GPU
  stream; the device decode of the context gives the same bits; escapes as
  many as the oracle's (up to a few on a block with a 1e9 outlier); the
  ratio within 1 % of the oracle's;
* escapes the single pass wrote for blocks it then deferred are dropped (a
  NaN, a huge outlier), those of verified blocks kept (a moderate bump);
* a block the sketch alone rules out is deferred; when more than half the
  blocks are predicted to fail (every variable drifting) the call runs
  two-pass and matches the plain oracle;
* two encodes give the same stream; a field that needs more payload than the
  buffers hold is encoded again two-pass, with the same guarantees.
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
from oracle import container, dls as odls  # noqa: E402

pytestmark = pytest.mark.gpu


def _field(drift, seeds=(11, 12), nx=72, ny=64, nz=48, nt=40):
    """drift: False (every variable rank 1 in time), True (every variable
    drifting), or a tuple of per-variable flags."""
    flags = drift if isinstance(drift, tuple) else (drift,) * len(seeds)
    f = np.concatenate([synth.spectrum(nx, ny, nz, nt, nmodes=16, seed=s, drift=d) for s, d in zip(seeds, flags)])
    e = [1e-3 * r for r in synth.range_of(f)]
    p = odls.Params(nx=nx, ny=ny, nz=nz, nt=nt, nvars=len(seeds), dtype="f32", px=32, py=32, pz=32,
                    window=16, eps=e)
    return f, p


def _lib_params(p, precision):
    lp = H.to_lib_params(p, precision)
    lp.persistent = True
    return lp


def _check(f, p, precision, enc=None):
    bf16 = precision == "bf16"
    enc = enc or dls.Encoder()
    t = torch.from_numpy(f).cuda()
    enc.encode(t, _lib_params(p, precision), keep_coef=True)
    inf = enc.info()
    nb, wp = inf.nblocks, inf.wpad
    print("launch mode %d: %d blocks, %d solved at rank 1 in the single pass, %d deferred; sketch: %d predicted "
          "to fail, %d ruled out, declined %d" % (inf.launch_mode, nb, inf.nfast_accept, inf.ndeferred,
                                                  inf.npredicted_deferred, inf.npruned, inf.fused_declined),
          flush=True)
    assert inf.npruned <= inf.npredicted_deferred <= nb
    assert bool(inf.fused_declined) == (inf.npredicted_deferred > nb / 2)
    rank = dls.d2h(inf.d_rank, nb).copy()
    basis = dls.d2h(inf.d_basis, nb * wp * wp * 8).view(np.float64).reshape(nb, wp, wp).copy()
    qa_off = dls.d2h(inf.d_qa_off, nb * 8).view(np.int64).copy()
    coef = dls.d2h(inf.d_coef, inf.qa_bytes).view(np.float32).copy()
    blocks, _ = odls.plan(f, p)
    assert len(blocks) == nb
    codes, acc_or = [], []
    acc_mism, proj, errs, dmism, ndef = 0, [], [], 0, 0
    for b, blk in enumerate(blocks):
        xs = odls.gather(f, blk)
        if inf.launch_mode == 2:
            code, acc = odls.encode_block_sketch(xs, p.eps[blk.var], p.resolved_rmax(), np.float32, blk.px, bf16)
        else:  # encoded again two-pass: the plain method
            code, acc = odls.encode_block(xs, p.eps[blk.var], p.resolved_rmax(), np.float32, bf16), False
        codes.append(code)
        acc_or.append(acc)
        w, m, r = blk.w, blk.m, int(rank[b])
        acc_gpu = r == 1 and not np.any(basis[b][1:]) and inf.launch_mode == 2
        A = coef[qa_off[b] // 4: qa_off[b] // 4 + r * m].reshape(r, m).T
        V = basis[b][:r, :w].T
        if r:
            assert np.abs(V.T @ V - np.eye(r)).max() <= 1e-12
        if acc_gpu != acc:
            acc_mism += 1
            continue
        if acc:
            xg = xs.astype(np.float64)
            if bf16:
                xg = odls.round_bf16(xg)
            sk = xg[:, :odls.sketch_points(m, blk.px)]
            lam_s = odls.eig_desc(sk @ sk.T)[0]     # the spectrum of the sketch's Gram, which gives q
            tr_full = float(np.sum(xg * xg))
            tol = H.projector_tol(lam_s, 1, w, energy_ratio=tr_full / max(float(code.lam[0]), 1e-300))
            if np.all(np.isfinite(lam_s)) and tol is not None:
                proj.append(H.projector_rel_err(A, V, code.A, code.V) / tol)
            continue
        ndef += 1
        if r != code.r:
            dmism += 1
        elif r > 0 and H.gap_qualified(code.lam, r):
            errs.append(H.coef_rel_err(A, V, code.A, code.V[:, :r]))
    print("acceptance mismatches %d / %d (oracle accepts %d); accepted: projector max %.3g of its bound over %d; deferred %d: "
          "rank mismatches %d, coef max %.3g over %d"
          % (acc_mism, nb, sum(acc_or), max(proj, default=0), len(proj), ndef, dmism, max(errs, default=0),
             len(errs)), flush=True)
    assert acc_mism <= 0.01 * nb
    assert not proj or max(proj) <= 1.0
    assert dmism <= max(1, 0.05 * ndef)
    assert not errs or max(errs) <= 1e-5
    if inf.launch_mode == 2:
        assert inf.nfast_accept + inf.ndeferred == nb
        # a block the sketch rules out is one the whole block fails
        assert inf.ndeferred >= inf.npruned
    stream = enc.finalize()
    out = dls.decompress(stream).cpu().numpy()
    fin = np.isfinite(f)
    assert np.array_equal(np.isnan(out), np.isnan(f))
    err = np.where(fin, np.abs(out.astype(np.float64) - f.astype(np.float64)), 0.0)
    assert np.all(err <= np.array(p.eps)[:, None, None, None, None])
    assert np.array_equal(odls.decompress(stream).view(np.uint8), out.view(np.uint8))
    dev = torch.full_like(t, float("nan"))
    enc.decode(dev)
    torch.cuda.synchronize()
    assert np.array_equal(dev.cpu().numpy().view(np.uint8), out.view(np.uint8))
    # escapes: as many as the oracle's, up to a few on blocks whose FP32 Gram
    # and FP64 Gram pick visibly different bases (a 1e9 outlier)
    nesc_or = sum(c.esc_values.size for c in codes)
    assert abs(inf.nescapes - nesc_or) <= max(8, nesc_or // 1000), (inf.nescapes, nesc_or)
    pb = odls.Params(**{**p.__dict__, "precision": precision})
    ref = container.pack(odls.Encoded(pb, blocks, codes, [[] for _ in range(p.nvars)]))
    cr_g, cr_o = f.nbytes / len(stream), f.nbytes / len(ref)
    print("CR gpu %.4f oracle %.4f escapes %d" % (cr_g, cr_o, inf.nescapes), flush=True)
    assert abs(cr_g / cr_o - 1.0) <= 0.01
    return enc, stream


MIXED = (False, False, True)   # two rank-1 variables and one drifting: a third of the blocks deferred


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("drift", [False, MIXED], ids=["rank1", "mixed"])
def test_fused_parity(drift, precision):
    print("fused single pass, drift %s, %s" % (drift, precision), flush=True)
    f, p = _field(drift, seeds=(11, 12, 13) if drift else (11, 12))
    enc, _ = _check(f, p, precision)
    # the same context again: buffers fit now, the single pass is used
    enc2, s2 = _check(f, p, precision, enc)
    inf = enc2.info()
    assert inf.launch_mode == 2
    if drift:
        assert 0 < inf.ndeferred < inf.nblocks / 2


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_fused_declined_when_most_blocks_fail(precision):
    """Every variable drifting: the sketch predicts most blocks to fail, so
    the call runs two-pass (the plain method, against the plain oracle)."""
    print("fused single pass declined, %s" % precision, flush=True)
    f, p = _field(True)
    enc, _ = _check(f, p, precision)
    inf = enc.info()
    assert inf.fused_declined == 1 and inf.launch_mode != 2 and inf.nfast_accept == 0
    assert inf.npredicted_deferred > inf.nblocks / 2


def test_fused_deterministic_and_regrows():
    """Two encodes of one field give one stream; a field with more payload
    than the buffers hold (higher ranks) is encoded again two-pass on the
    first call and in a single pass on the next."""
    f1, p1 = _field(False, seeds=(21, 22, 23))
    enc = dls.Encoder()
    t = torch.from_numpy(f1).cuda()
    lp = _lib_params(p1, "fp32")
    enc.encode(t, lp)
    a = enc.finalize()
    enc.encode(t, lp)
    assert enc.info().launch_mode == 2
    assert enc.finalize() == a
    f2, p2 = _field(MIXED, seeds=(21, 22, 23))
    _, _ = _check(f2, p2, "fp32", enc)
    assert enc.info().launch_mode != 2     # the deferred blocks' payload did not fit
    _, _ = _check(f2, p2, "fp32", enc)
    assert enc.info().launch_mode == 2


def test_fused_escapes_kept_and_dropped():
    """A moderate bump in a verified block escapes and is kept; a NaN and a
    1e9 outlier make their blocks fail verification, so the escapes the
    single pass wrote for them are dropped and the two-pass path encodes
    them again (the NaN block raw); a block whose sketch is noisy is ruled
    out before the single pass encodes it."""
    f, p = _field(False)
    f = f.copy()
    e0 = p.eps[0]
    f[0, 3, 5, 40, 37] += 300.0 * e0          # block (var 0, window 0, patch (1, 1, 0)): stays rank 1
    f[0, 20, 40, 10, 10] = np.nan             # window 1, a slice after the sketch's
    f[1, 2, 1, 1, 70] = 1e9                   # var 1, window 0, inside the sketch
    # broadband noise of 30 eps over the sketch (the first z-plane) of block
    # (var 0, window 0, patch (1, 0, 0)): the sketch alone rules rank 1 out
    rng = np.random.default_rng(5)
    f[0, 0:16, 0, 0:32, 32:64] += (30.0 * e0 * rng.standard_normal((16, 32, 32))).astype(np.float32)
    enc, _ = _check(f, p, "fp32")            # first call: the deferred blocks need more room
    enc, _ = _check(f, p, "fp32", enc)       # then the single pass, dropping their escapes
    inf = enc.info()
    assert inf.launch_mode == 2 and inf.ndeferred >= 3 and inf.nraw == 1 and inf.nescapes > 0
    # the noisy sketch rules its block out; the outlier's sketch does not
    # resolve its discarded energy against the outlier's (tr ~ 1e18)
    assert inf.npruned >= 1
