"""Pins of the learned-warm-start oracle: library statistics, closed forms,
finite differences and the exact-energy identity of the acceptance test."""
import math

import numpy as np
import pytest
import scipy.stats

import synth
from oracle import dls, learned as L


def _block(seed=0, w=16, px=8, py=8, pz=1):
    rng = np.random.default_rng(seed)
    t = np.arange(w)[:, None]
    p = np.arange(px * py * pz)[None, :]
    x = np.cos(0.2 * t + 0.05 * p) + 0.3 * np.sin(0.07 * t * p / 7.0) + 0.01 * rng.normal(size=(w, px * py * pz))
    return x


def test_moments_match_library_statistics():
    x = _block(1)
    f = L.moments(x, 8, 8, 1, 1e-3)
    v = x.ravel()
    sd = v.std()
    assert f[0] == pytest.approx(v.mean(), rel=1e-12)
    assert f[1] == pytest.approx(sd, rel=1e-12)
    assert (f[2], f[3]) == (v.min(), v.max())
    assert f[4] == pytest.approx(scipy.stats.skew(v), rel=1e-9)
    assert f[5] == pytest.approx(scipy.stats.kurtosis(v, fisher=True, bias=True), rel=1e-9)
    d = np.diff(x, axis=0).ravel()
    assert f[6] == pytest.approx(np.abs(d).mean() / sd, rel=1e-12)
    assert f[7] == pytest.approx(d.std() / sd, rel=1e-12)
    img = x.reshape(16, 8, 8)
    assert f[8] == pytest.approx(np.abs(np.diff(img, axis=2)).mean() / sd, rel=1e-12)
    assert f[9] == pytest.approx(np.abs(np.diff(img, axis=1)).mean() / sd, rel=1e-12)
    a = x[:-1].ravel() - v.mean()
    b = x[1:].ravel() - v.mean()
    assert f[10] == pytest.approx(np.mean(a * b) / sd ** 2, rel=1e-12)
    assert f[12] == pytest.approx(math.log10(np.mean(v * v) / 1e-6), rel=1e-12)
    assert f[14] == pytest.approx(np.sum(x.mean(axis=0) ** 2) * 16 / np.sum(v * v), rel=1e-12)
    assert f[15] == 6.0


def test_moments_degenerate_blocks():
    f = L.moments(np.full((4, 16), 2.5), 4, 4, 1, 1e-3)
    assert f[1] == 0 and np.all(f[4:12] == 0)
    g = L.moments(np.ones((1, 8)), 8, 1, 1, 1e-3)
    assert g[6] == g[7] == g[10] == g[11] == 0


def test_pooled_equals_direct_averages():
    x = _block(2, w=6, px=16, py=16)
    got = L.pooled(x, 16, 16, 1).reshape(8, 8)
    y = x.reshape(6, 16, 16).mean(axis=0)
    ref = y.reshape(8, 2, 8, 2).mean(axis=(1, 3))
    ref = (ref - x.mean()) / x.std()
    assert np.allclose(got, ref, rtol=0, atol=1e-13)
    # edge 4: every pixel is replicated over a 2 x 2 group of cells
    x4 = _block(3, w=5, px=4, py=4)
    got4 = L.pooled(x4, 4, 4, 1).reshape(8, 8)
    y4 = (x4.reshape(5, 4, 4).mean(axis=0) - x4.mean()) / x4.std()
    assert np.allclose(got4, np.kron(y4, np.ones((2, 2))), rtol=0, atol=1e-13)
    # 3D: averaged over z as well
    x3 = _block(4, w=3, px=8, py=8, pz=4)
    got3 = L.pooled(x3, 8, 8, 4).reshape(8, 8)
    y3 = (x3.reshape(3, 4, 8, 8).mean(axis=(0, 1)) - x3.mean()) / x3.std()
    assert np.allclose(got3, y3, rtol=0, atol=1e-13)


def _batch(seed, B=6):
    rng = np.random.default_rng(seed)
    z = rng.normal(size=(B, L.NFEAT))
    rank = rng.integers(1, 17, size=B)
    basis = rng.normal(size=(B, 16, 16))
    wb = rng.integers(4, 17, size=B)
    return z, rank, basis, wb


def test_gradients_match_central_differences():
    net = L.init_net(5)
    net.b1[:] = 0.1
    net.b2[:] = 0.05
    z, rank, basis, wb = _batch(6)

    def loss_of():
        _, _, out = L.forward(net, z)
        return L.loss_and_grad_out(out, rank, basis, wb)[0]

    h1, h2, out = L.forward(net, z)
    _, gout = L.loss_and_grad_out(out, rank, basis, wb)
    grads = L.backward(net, z, h1, h2, gout)
    rng = np.random.default_rng(7)
    for P, G in zip(net.params(), grads):
        idx = [tuple(rng.integers(0, s) for s in P.shape) for _ in range(6)]
        for i in idx:
            old = P[i]
            h = 1e-6 * max(1.0, abs(old))
            P[i] = old + h
            lp = loss_of()
            P[i] = old - h
            lm = loss_of()
            P[i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - G[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (P.shape, i, fd, G[i])


def test_loss_closed_forms():
    out = np.zeros((1, L.NOUT))
    out[0, 3] = 2.0
    basis = np.zeros((1, 16, 16))
    l, g = L.loss_and_grad_out(out, np.array([4]), basis, np.array([16]))
    ce = -math.log(math.exp(2.0) / (15 + math.exp(2.0)))
    assert l == pytest.approx(ce, rel=1e-12)
    out2 = np.zeros((1, L.NOUT))
    out2[0, 16:16 + 16] = 1.0        # mode 0, every t
    out2[0, 16 + 16:16 + 32] = 5.0   # mode 1: masked when r = 1
    l2, g2 = L.loss_and_grad_out(out2, np.array([1]), basis, np.array([8]))
    assert l2 == pytest.approx(math.log(16.0) + 1.0, rel=1e-12)   # 8 unmasked entries of (1 - 0)^2
    assert np.all(g2[0, 16 + 8:] == 0.0) and np.allclose(g2[0, 16:16 + 8], 2.0 / 8)


def test_adam_first_step_closed_form():
    P = [np.array([1.0, -2.0, 0.5])]
    G = [np.array([0.3, -1e-3, 0.0])]
    m = [np.zeros(3)]
    v = [np.zeros(3)]
    L.adam_step(P, G, m, v, 1, lr=0.01)
    want = np.array([1.0, -2.0, 0.5]) - 0.01 * G[0] / (np.abs(G[0]) + 1e-8)
    assert np.allclose(P[0], want, rtol=0, atol=1e-15)


def test_bf16_rounding_matches_bit_truncation_rules():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.14159, 1e-40])
    r = L.bf16(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0            # tie -> even
    assert r[2] == 1.0 + 2 ** -7  # above the tie -> up
    assert abs(r[3] + 3.140625) < 1e-12


def _gram_case(seed, r0=3, w=16, m=64):
    rng = np.random.default_rng(seed)
    a, _ = np.linalg.qr(rng.normal(size=(w, r0)))
    b, _ = np.linalg.qr(rng.normal(size=(m, r0)))
    x = (a * np.array([10.0, 3.0, 1.0][:r0])) @ b.T + 1e-4 * rng.normal(size=(w, m))
    return x


def test_warm_start_exact_energy_and_acceptance():
    x = _gram_case(1)
    G = x @ x.T
    lam, V = dls.eig_desc(G)
    for eps in (1e-3, 1e-5):
        tau = eps * eps * x.size
        r_plain = dls.choose_rank(lam, tau, 16)
        rng = np.random.default_rng(2)
        V0 = V[:, :r_plain] + 0.05 * rng.normal(size=(16, r_plain))
        ok, r, th, Z = L.warm_start_eig(G, V0, tau, iters=3)
        assert ok and r == r_plain
        # discarded energy of the accepted basis, computed explicitly
        Zr = Z[:, :r]
        e = np.sum((x - Zr @ (Zr.T @ x)) ** 2)
        assert abs(e - (np.trace(G) - th[:r].sum())) <= 1e-9 * np.trace(G)
        assert e <= tau * (1 + 1e-12)
        assert np.abs(Zr.T @ Zr - np.eye(r)).max() <= 1e-12
    # a too-small predicted rank is rejected (falls back to the full solve)
    ok, r, _, _ = L.warm_start_eig(G, V[:, :1], 1e-8 * x.size, iters=3)
    assert not ok
    # a too-large predicted rank is cut by the downward check
    tau = 1e-3 ** 2 * x.size
    ok, r, _, _ = L.warm_start_eig(G, V[:, :8], tau, iters=2)
    assert ok and r == dls.choose_rank(lam, tau, 16)


def test_mgs_handles_dependent_columns():
    Y = np.zeros((5, 3))
    Y[:, 0] = 1.0
    Y[:, 1] = 2.0
    Y[0, 2] = 1.0
    Q = L.mgs(Y)
    assert np.abs(Q.T @ Q - np.eye(3)).max() <= 1e-14


def test_learned_encode_keeps_the_bound():
    f = synth.blobs2d(nx=32, ny=32, nt=16, seed=9)
    eps = 1e-3 * synth.range_of(f)[0]
    p = dls.Params(nx=32, ny=32, nz=1, nt=16, nvars=1, dtype="f64", px=8, py=8, pz=1, window=16, eps=[eps])
    blocks, _ = dls.plan(f, p)
    rng = np.random.default_rng(3)
    for b in blocks:
        xb = dls.gather(f, b)
        V0 = rng.normal(size=(16, 16))
        code, acc = L.encode_block_learned(xb, eps, 16, np.float64, 2, V0)
        out = dls.decode_block(code.r, code.qV, code.qA, code.codes, code.esc_values, eps, np.float64)
        assert np.all(np.abs(out - xb) <= eps)


def test_learned_retry_and_limits():
    """A rank-6 block: rhat 1 is rejected, the retry with 5 columns is
    rejected too (tail of mode 6 > tau), so the plain eigensolve decides; a
    prediction above WARM_MAX columns falls back at once; rhat 3 is rejected
    and its retry with 7 columns accepted, returning the plain rank."""
    rng = np.random.default_rng(12)
    a, _ = np.linalg.qr(rng.normal(size=(16, 6)))
    bvec, _ = np.linalg.qr(rng.normal(size=(64, 6)))
    x = (a * np.array([50.0, 30, 20, 10, 5, 2])) @ bvec.T
    eps = 1e-3
    V0 = rng.normal(size=(16, 16))
    plain = dls.encode_block(x, eps, 16, np.float64)
    assert plain.r == 6
    code, acc = L.encode_block_learned(x, eps, 16, np.float64, 1, V0)
    assert not acc and code.r == plain.r
    code, acc = L.encode_block_learned(x, eps, 16, np.float64, L.WARM_MAX + 1, V0)
    assert not acc and code.r == plain.r
    code, acc = L.encode_block_learned(x, eps, 16, np.float64, 3, V0)
    assert acc and code.r == plain.r


def test_large_blocks_take_the_plain_eigensolve():
    """Blocks above WARM_MAX_POINTS points are not warm-started: the result
    is the plain encode, reported as not accepted."""
    rng = np.random.default_rng(21)
    x = rng.normal(size=(16, L.WARM_MAX_POINTS + 1))
    V0 = np.eye(16)
    code, acc = L.encode_block_learned(x, 1e-2, 16, np.float64, 2, V0)
    plain = dls.encode_block(x, 1e-2, 16, np.float64)
    assert not acc and code.r == plain.r and np.array_equal(code.qA, plain.qA)


def test_bf16_gram_mode_forms_the_gram_from_rounded_values():
    """With bf16_gram the warm start sees the Gram of the bfloat16-rounded
    snapshots, as the plain oracle's mixed-precision mode does: for the
    1 x 2 block [1 + 2^-8, 3] that Gram is 1 + 9 = 10 exactly (1 + 2^-8 is a
    tie that rounds to the even 1), while the full-precision one is larger."""
    x = np.array([[1 + 2.0 ** -8, 3.0]])
    V0 = np.ones((1, 16))
    code, acc = L.encode_block_learned(x, 1e-3, 1, np.float64, 1, V0, 2, bf16_gram=True)
    assert acc and code.r == 1 and code.lam[0] == 10.0
    code, acc = L.encode_block_learned(x, 1e-3, 1, np.float64, 1, V0, 2)
    assert acc and code.lam[0] > 10.0
