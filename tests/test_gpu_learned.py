"""The learned warm start on the GPU against the FP64 oracle.

* features of every block vs oracle.learned.features (FP32 output);
* network gradients: FP32 products vs the FP64 oracle (normwise <= 1e-4),
  bf16 products vs the oracle with the same bf16 rounding (<= 2e-2);
* training on the GPU lowers the loss;
* warm-started eigensolve: with a model whose output ignores its input
  (fixed rank guess 4, V0 = the unit vectors) the GPU and the oracle start
  from identical V0 (both attempts); accepted/rejected blocks, ranks,
  coefficients (1e-5 on gap-qualified blocks), the bound and bit-identical
  decoding are compared.
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
from oracle import dls as odls, learned as L  # noqa: E402

pytestmark = pytest.mark.gpu


def _fields():
    f1 = synth.blobs2d(nx=64, ny=64, nt=32, seed=1)
    p1 = odls.Params(nx=64, ny=64, nz=1, nt=32, nvars=1, dtype="f64", px=8, py=8, pz=1, window=16,
                     eps=list(1e-3 * synth.range_of(f1)))
    f2 = synth.blobs2d(nx=70, ny=45, nt=21, seed=3, nblobs=6, dtype=np.float32)
    p2 = odls.Params(nx=70, ny=45, nz=1, nt=21, nvars=1, dtype="f32", px=16, py=16, pz=1, window=16,
                     eps=list(1e-3 * synth.range_of(f2)))
    f3 = synth.spectrum(20, 18, 12, 10, nmodes=8, seed=5, drift=True, dtype=np.float64)
    p3 = odls.Params(nx=20, ny=18, nz=12, nt=10, nvars=1, dtype="f64", px=8, py=8, pz=4, window=10,
                     eps=list(1e-3 * synth.range_of(f3)))
    # blocks of at most 16 points (16 lanes per block): 4 x 4 patches with
    # truncated edges (4 x 3, 1 x 4, 1 x 3) and a short last window; 3 x 2 x 2
    # patches of a 3D field with 1 x 2 x 2 edges
    f4 = synth.blobs2d(nx=29, ny=27, nt=19, seed=7, nblobs=5, dtype=np.float32)
    p4 = odls.Params(nx=29, ny=27, nz=1, nt=19, nvars=1, dtype="f32", px=4, py=4, pz=1, window=16,
                     eps=list(1e-3 * synth.range_of(f4)))
    f5 = synth.spectrum(10, 6, 8, 7, nmodes=6, seed=9, drift=True, dtype=np.float64)
    p5 = odls.Params(nx=10, ny=6, nz=8, nt=7, nvars=1, dtype="f64", px=3, py=2, pz=2, window=7,
                     eps=list(1e-3 * synth.range_of(f5)))
    return [(f1, p1), (f2, p2), (f3, p3), (f4, p4), (f5, p5)]


@pytest.mark.parametrize("case", [0, 1, 2, 3, 4])
def test_features_match_oracle(case):
    f, p = _fields()[case]
    print("features case", case, flush=True)
    enc = dls.Encoder()
    t = torch.from_numpy(f).cuda()
    enc.encode(t, H.to_lib_params(p))
    got = enc.features(t).cpu().numpy().astype(np.float64)
    blocks, _ = odls.plan(f, p)
    assert got.shape == (len(blocks), 80)
    for b, blk in enumerate(blocks):
        if blk.m > L.WARM_MAX_POINTS:   # never warm-started: no features
            assert np.all(got[b] == 0.0)
            continue
        ref = L.features(odls.gather(f, blk), blk.px, blk.py, blk.pz, p.eps[blk.var])
        err = np.abs(got[b] - ref)
        assert np.all(err <= 2e-6 * np.maximum(1.0, np.abs(ref))), (b, np.argmax(err), got[b][np.argmax(err)],
                                                                    ref[np.argmax(err)])


def _rand_batch(seed, n=96):
    rng = np.random.default_rng(seed)
    feat = rng.normal(size=(n, 80)).astype(np.float32)
    rank = rng.integers(1, 17, size=n).astype(np.int32)
    basis = rng.normal(size=(n, 256)).astype(np.float32)
    wb = rng.integers(3, 17, size=n).astype(np.int32)
    return feat, rank, basis, wb


def _net_for_test(seed):
    net = L.init_net(seed)
    rng = np.random.default_rng(seed + 1)
    net.b1[:] = rng.normal(0, 0.1, net.b1.shape)
    net.b2[:] = rng.normal(0, 0.1, net.b2.shape)
    net.b3[:] = rng.normal(0, 0.1, net.b3.shape)
    net.mom_mean[:] = rng.normal(0, 0.5, 16)
    net.mom_std[:] = rng.uniform(0.5, 2.0, 16)
    return net


def _flat(net):
    return np.concatenate([a.ravel() for a in net.params()]).astype(np.float32), \
        np.concatenate([net.mom_mean, net.mom_std]).astype(np.float32)


@pytest.mark.parametrize("bf16", [False, True])
def test_gradients_match_oracle(bf16):
    net = _net_for_test(3)
    feat, rank, basis, wb = _rand_batch(4)
    # the oracle sees the same FP32 parameters and inputs the GPU sees
    P, N = _flat(net)
    sizes = [a.size for a in net.params()]
    parts = np.split(P.astype(np.float64), np.cumsum(sizes)[:-1])
    net32 = L.Net(*[q.reshape(a.shape) for q, a in zip(parts, net.params())],
                  N[:16].astype(np.float64), N[16:].astype(np.float64))
    z = L.normalise(net32, feat.astype(np.float64))
    h1, h2, out = L.forward(net32, z, round_bf16=bf16)
    loss_ref, gout = L.loss_and_grad_out(out, rank, basis.reshape(-1, 16, 16).astype(np.float64), wb)
    g_ref = L.backward(net32, z, h1, h2, gout, round_bf16=bf16)
    m = dls.Model()
    m.set(P, N)
    g, loss = m.grad(torch.from_numpy(feat).cuda(), torch.from_numpy(rank).cuda(),
                     torch.from_numpy(basis).cuda(), torch.from_numpy(wb).cuda(), bf16=bf16)
    g = g.cpu().numpy().astype(np.float64)
    tol = 2e-2 if bf16 else 1e-4
    assert abs(loss - loss_ref) <= tol * abs(loss_ref)
    off = 0
    for name, G in zip(["W1", "b1", "W2", "b2", "W3", "b3"], g_ref):
        got = g[off:off + G.size].reshape(G.shape)
        off += G.size
        rel = np.linalg.norm(got - G) / max(np.linalg.norm(G), 1e-30)
        print("grad %s rel %.2e" % (name, rel), flush=True)
        assert rel <= tol, name


def test_fused_forward_matches_layers_and_oracle():
    """The fused inference kernel reproduces the layer-by-layer bf16 forward
    bit for bit, and the FP64 oracle with the same bf16 roundings."""
    net = _net_for_test(9)
    P, N = _flat(net)
    m = dls.Model()
    m.set(P, N)
    rng = np.random.default_rng(10)
    feat = rng.normal(size=(1000, 80)).astype(np.float32)   # not a multiple of 64 rows
    tf = torch.from_numpy(feat).cuda()
    fused = m.forward(tf, bf16=True).cpu().numpy()
    layers = m.forward(tf, bf16=2).cpu().numpy()
    assert np.array_equal(fused.view(np.uint32), layers.view(np.uint32))
    sizes = [a.size for a in net.params()]
    parts = np.split(P.astype(np.float64), np.cumsum(sizes)[:-1])
    net32 = L.Net(*[q.reshape(a.shape) for q, a in zip(parts, net.params())],
                  N[:16].astype(np.float64), N[16:].astype(np.float64))
    ref = L.forward(net32, L.normalise(net32, feat.astype(np.float64)), round_bf16=True)[2]
    rel = np.linalg.norm(fused - ref) / np.linalg.norm(ref)
    print("fused forward vs oracle rel %.2e" % rel, flush=True)
    assert rel <= 1e-4


def test_training_lowers_the_loss():
    rng = np.random.default_rng(5)
    n = 512
    feat = rng.normal(size=(n, 80)).astype(np.float32)
    rank = (1 + (feat[:, 0] > 0) + 2 * (feat[:, 1] > 0.5)).astype(np.int32)
    basis = np.tile(np.eye(16, dtype=np.float32).reshape(1, 256), (n, 1))
    wb = np.full(n, 16, np.int32)
    net = L.init_net(7)
    P, N = _flat(net)
    m = dls.Model()
    m.set(P, N)
    tf, tr, tb, tw = (torch.from_numpy(a).cuda() for a in (feat, rank, basis, wb))
    first = m.train_step(tf, tr, tb, tw, lr=3e-3)
    for _ in range(300):
        last = m.train_step(tf, tr, tb, tw, lr=3e-3)
    print("loss %.4f -> %.4f" % (first, last), flush=True)
    assert last < 0.25 * first


def _fixed_guess_model(rhat=4):
    P = np.zeros(dls.NPARAM, np.float32)
    off_b3 = 80 * 128 + 128 + 128 * 128 + 128 + 128 * 272
    P[off_b3 + rhat - 1] = 10.0                 # rank logit
    for k in range(16):
        P[off_b3 + 16 + k * 16 + k] = 1.0       # V0 = identity columns
    m = dls.Model()
    m.set(P, np.concatenate([np.zeros(16), np.ones(16)]).astype(np.float32))
    return m


@pytest.mark.parametrize("case", [0, 1])
def test_warm_start_parity(case):
    f, p = _fields()[case]
    print("warm-start case", case, flush=True)
    rhat, iters = 4, 2
    m = _fixed_guess_model(rhat)
    enc = dls.Encoder()
    enc.set_model(m, iters, margin=0)
    lp = H.to_lib_params(p)
    lp.learned = True
    t = torch.from_numpy(f).cuda()
    enc.encode(t, lp, keep_coef=True)
    inf = enc.info()
    nb = inf.nblocks
    rank = dls.d2h(inf.d_rank, nb).copy()
    basis = dls.d2h(inf.d_basis, nb * 256 * 8).view(np.float64).reshape(nb, 16, 16)
    qa_off = dls.d2h(inf.d_qa_off, nb * 8).view(np.int64)
    coef = dls.d2h(inf.d_coef, inf.qa_bytes).view(np.float32)
    stream = enc.finalize()
    blocks, _ = odls.plan(f, p)
    V0 = np.eye(16)   # the model's 16 starting columns (a retry uses more than rhat)
    n_acc, mism, errs = 0, 0, []
    for b, blk in enumerate(blocks):
        code, acc = L.encode_block_learned(odls.gather(f, blk), p.eps[blk.var], p.resolved_rmax(),
                                           p.np_dtype, rhat, V0, iters)
        n_acc += acc
        if code.r != rank[b]:
            mism += 1
            continue
        r = code.r
        Vg = basis[b][:r, :blk.w].T
        Ag = coef[qa_off[b] // 4: qa_off[b] // 4 + r * blk.m].reshape(r, blk.m).T
        xb = odls.gather(f, blk).astype(np.float64)
        lam_plain = odls.eig_desc(xb @ xb.T)[0]
        if acc and H.gap_qualified(lam_plain, r):
            errs.append(H.coef_rel_err(Ag, Vg, code.A, code.V[:, :r]))
    print("accepted oracle %d gpu %d of %d; rank mismatches %d; coef max %.2e"
          % (n_acc, inf.nwarm_accept, nb, mism, max(errs) if errs else 0), flush=True)
    assert abs(inf.nwarm_accept - n_acc) <= max(1, nb // 100)
    assert inf.nwarm_accept + inf.nwarm_reject == nb
    assert mism <= 0.05 * nb
    assert not errs or max(errs) <= 1e-5
    out = dls.decompress(stream).cpu().numpy()
    assert np.all(np.abs(out.astype(np.float64) - f.astype(np.float64)) <= p.eps[0])
    assert np.array_equal(odls.decompress(stream).view(np.uint8), out.view(np.uint8))


def test_compress_with_model_equals_context_route():
    """dls_compress with the model in dls_params runs the full form (learned
    warm start) in one call: its stream equals the context route's (set_model
    + encode + finalize) byte for byte, warm starts are accepted, and the
    bound holds."""
    f, p = _fields()[0]
    print("compress route with a model", flush=True)
    m = _fixed_guess_model(4)
    lp = H.to_lib_params(p)
    lp.learned = True
    lp.model = m
    lp.warm_iters = 2
    lp.rank_margin = 0
    t = torch.from_numpy(f).cuda()
    one = dls.compress(t, lp)
    enc = dls.Encoder()
    enc.set_model(m, 2, margin=0)
    enc.encode(t, lp)
    assert enc.info().nwarm_accept > 0
    assert enc.finalize() == one
    out = dls.decompress(one).cpu().numpy()
    assert np.all(np.abs(out.astype(np.float64) - f.astype(np.float64)) <= p.eps[0])
    # without a model the learned form is refused
    lp.model = None
    with pytest.raises(dls.DlsError):
        dls.compress(t, lp)
