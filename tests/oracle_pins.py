"""Pins of the FP64 oracle against facts outside the oracle itself.

Each ``pin_*`` function raises AssertionError when the oracle disagrees with
a library routine, a closed form, an invariant of the method or a brute-force
answer.  ``test_oracle_pins.py`` runs them; ``test_oracle_mutations.py``
plants plausible mistakes in the oracle and checks that some pin fails.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

import synth
from oracle import container, dls, l2
from oracle import globalbasis as gb
from oracle.jacobi import cyclic_jacobi

SHAPES = [(16, 64), (16, 16), (4, 64), (32, 128), (5, 7), (1, 9), (16, 512)]


def _rand_block(rng, w, m, kind="smooth"):
    if kind == "smooth":
        t = np.arange(w)[:, None]
        p = np.arange(m)[None, :]
        x = np.zeros((w, m))
        for _ in range(4):
            x += rng.normal() * np.cos(rng.uniform(0, 0.3) * t + rng.uniform(0, 0.2) * p
                                       + rng.uniform(0, 6.28))
        return x + 1e-4 * rng.normal(size=(w, m))
    return rng.normal(size=(w, m))


# -- eigenpairs -----------------------------------------------------------
def pin_eigenvalues_vs_svd():
    """lam_k(X X^T) = sigma_k(X)^2 (LAPACK gesdd, a different driver)."""
    rng = np.random.default_rng(7)
    for (w, m) in SHAPES:
        for kind in ("smooth", "normal"):
            x = _rand_block(rng, w, m, kind)
            lam, V = dls.eig_desc(x @ x.T)
            s = np.linalg.svd(x, compute_uv=False)
            ref = np.zeros(w)
            ref[:s.size] = s ** 2
            assert np.allclose(lam, ref, rtol=0, atol=1e-12 * ref[0]), (w, m, kind)


def pin_eigenvectors_orthonormal_and_residual():
    """||V^T V - I||_max <= 1e-12 and G V = V diag(lam) to 1e-12 ||G||."""
    rng = np.random.default_rng(8)
    for (w, m) in SHAPES:
        x = _rand_block(rng, w, m)
        G = x @ x.T
        lam, V = dls.eig_desc(G)
        assert np.abs(V.T @ V - np.eye(w)).max() <= 1e-12
        assert np.abs(G @ V - V * lam[None, :]).max() <= 1e-12 * max(1.0, lam[0])
        for k in range(w):
            i = int(np.argmax(np.abs(V[:, k])))
            assert V[i, k] > 0


def pin_eigenvalues_vs_jacobi():
    """LAPACK eigenvalues equal an independent cyclic Jacobi's."""
    rng = np.random.default_rng(9)
    for (w, m) in [(16, 64), (8, 8), (5, 7)]:
        x = _rand_block(rng, w, m, "normal")
        G = x @ x.T
        lam, _ = dls.eig_desc(G)
        jl, jv = cyclic_jacobi(G)
        jl = np.sort(jl)[::-1]
        assert np.allclose(lam, np.maximum(jl, 0), rtol=0, atol=1e-11 * lam[0])


# -- rank rule ------------------------------------------------------------
def pin_rank_bruteforce():
    """Chosen r is the smallest with ||X - V_r V_r^T X||_F^2 <= tau.

    The discarded energy is computed by explicit projection (Eckart-Young
    says it equals the eigenvalue tail) and the answer is cross-checked by a
    bisection over the monotone criterion, the search the paper uses.
    """
    rng = np.random.default_rng(10)
    for (w, m) in SHAPES:
        x = _rand_block(rng, w, m)
        lam, V = dls.eig_desc(x @ x.T)
        rcap = min(w, m)
        errs = []
        for r in range(0, rcap + 1):
            P = V[:, :r] @ V[:, :r].T
            e = float(np.sum((x - P @ x) ** 2))
            errs.append(e)
            tail = dls.tail_energies(lam)[r]
            assert abs(e - tail) <= 1e-10 * max(1.0, lam[0]), (w, m, r)
        for eps in (1e-1, 1e-2, 1e-3, 3e-5):
            tau = dls.KAPPA * eps * eps * m * w
            r = dls.choose_rank(lam, tau, rcap)
            ok = [rr for rr in range(1, rcap + 1) if errs[rr] <= tau + 1e-12 * lam[0]]
            expect = ok[0] if ok else rcap
            assert r == expect, (w, m, eps, r, expect)
            lo, hi = 1, rcap
            while lo < hi:
                mid = (lo + hi) // 2
                if dls.tail_energies(lam)[mid] <= tau:
                    hi = mid
                else:
                    lo = mid + 1
            assert lo == r


def pin_exact_rank_data():
    """X = sum_{k<=r0} s_k a_k b_k^T reconstructs to round-off with r = r0.

    eps = 1e-6 puts tau = eps^2 M W far above the Gram's round-off
    eigenvalues (~1e-16 lam_1) and far below s_min^2 >= 1.
    """
    rng = np.random.default_rng(11)
    for (w, m, r0) in [(16, 64, 3), (16, 512, 1), (32, 128, 7), (8, 8, 8)]:
        a, _ = np.linalg.qr(rng.normal(size=(w, r0)))
        b, _ = np.linalg.qr(rng.normal(size=(m, r0)))
        s = rng.uniform(1, 10, size=r0)
        x = (a * s) @ b.T
        c = dls.encode_block(x, 1e-6, min(w, 32), np.float64)
        assert c.r == r0
        rec = c.V[:, :c.r] @ c.A.T
        assert np.abs(rec - x).max() <= 1e-12 * np.abs(x).max()
        assert np.abs(c.V[:, :c.r].T @ c.V[:, :c.r] - np.eye(c.r)).max() <= 1e-12


# -- quantizers and the absolute bound -----------------------------------
def _blocks_for_bound(rng):
    out = []
    for (w, m) in SHAPES:
        x = _rand_block(rng, w, m)
        out.append((x, 1e-3 * np.ptp(x)))
        out.append((x, 1e-6 * np.ptp(x)))
        out.append((x + 1e7, 1e-3 * np.ptp(x)))           # large offset
        out.append((_rand_block(rng, w, m, "normal"), 0.5))
    return out


def pin_pointwise_bound():
    """|x - out| <= eps at every point, for both storage dtypes."""
    rng = np.random.default_rng(12)
    for x, eps in _blocks_for_bound(rng):
        for dt in (np.float64, np.float32):
            xs = x.astype(dt)
            c = dls.encode_block(xs, float(eps), 32, dt)
            out = dls.decode_block(c.r, c.qV, c.qA, c.codes, c.esc_values, float(eps), dt)
            err = np.abs(xs.astype(np.float64) - out.astype(np.float64)).max()
            assert err <= eps, (x.shape, eps, dt, err)
            assert np.array_equal(out, c.out)


def pin_escapes_rare_on_smooth_data():
    """With a sound residual step, FP64 smooth data needs no escapes."""
    rng = np.random.default_rng(13)
    for (w, m) in SHAPES:
        x = _rand_block(rng, w, m)
        c = dls.encode_block(x, 1e-3 * float(np.ptp(x)), 32, np.float64)
        assert c.esc_values.size == 0
        q = dls.unzigzag8(c.codes)
        assert np.abs(q).max() <= 4


def pin_escape_threshold():
    """Residual codes are one byte: |q| <= 127 is coded, |q| >= 128 escapes.

    X = [[100, 0], [0, v]], eps = 0.1, rank capped at 1: lam = (10^4, v^2),
    V_1 = e_1, A = (100, 0), qA = (1000, 0), S = [[65536000, 0], [0, 0]], so
    the point (1, 1) keeps its whole value as residual, q = rint(v / 0.2).
    v = 25.4 gives q = 127 (code 254); v = 25.6 gives q = 128, an escape that
    stores v verbatim; the decoder returns it exactly.
    """
    for v, q_want in ((25.4, 127), (-25.4, -127), (25.6, None), (-30.0, None)):
        x = np.array([[100.0, 0.0], [0.0, v]])
        c = dls.encode_block(x, 0.1, 1, np.float64)
        assert c.r == 1 and c.qA[:, 0].tolist() == [1000, 0]
        assert c.codes[0, 0] == 0 and c.codes[0, 1] == 0 and c.codes[1, 0] == 0
        if q_want is None:
            assert c.codes[1, 1] == dls.ESC_CODE
            assert c.esc_values.tolist() == [v]
        else:
            assert c.esc_values.size == 0
            assert int(c.codes[1, 1]) == (2 * q_want if q_want >= 0 else -2 * q_want - 1)
        out = dls.decode_block(c.r, c.qV, c.qA, c.codes, c.esc_values, 0.1, np.float64)
        assert np.array_equal(out, c.out)
        assert np.abs(out - x).max() <= 0.1
        if q_want is None:
            assert out[1, 1] == v


def pin_lattice_one_rounding():
    """out = round(exact (S + 2^17 q) * eps * 2^-16): one correctly rounded product.

    Checked with exact rational arithmetic on tiny blocks whose S and q are
    recomputed here with Python integers.  The rank is capped at 1 on a rank-2
    block so that the residual codes are nonzero and the code step (2 eps =
    2^17 c) is exercised.
    """
    base = np.array([[1.0, 2.0, -1.0], [2.0, 4.0, 0.5]])
    for pert, eps, rcap in ((1e-3, 0.01, 2), (0.07, 0.01, 1), (0.3, 0.02, 1)):
        x = base + np.array([[0.0, pert, 0.0], [-pert, 0.0, 2 * pert]])
        c = dls.encode_block(x, eps, rcap, np.float64)
        qV = [[int(v) for v in row] for row in c.qV]
        qA = [[int(v) for v in row] for row in c.qA]
        q = dls.unzigzag8(c.codes)
        if rcap == 1:
            assert np.abs(q).max() >= 1
        cf = Fraction(eps) / (1 << 16)
        for t in range(2):
            for p in range(3):
                S = sum(qV[t][k] * qA[p][k] for k in range(c.r))
                exact = Fraction(S + (1 << 17) * int(q[t, p])) * cf
                assert float(exact) == c.out[t, p]
                assert abs(Fraction(x[t, p]) - Fraction(c.out[t, p])) <= Fraction(eps)
        # basis and coefficient quantizers: round half to even of V 2^16 and A / eps
        assert np.array_equal(c.qV, np.rint(c.V[:, :c.r] * 65536.0).astype(np.int64))
        assert np.array_equal(c.qA, np.rint(c.A / eps).astype(np.int64))


def pin_hand_worked_rank_one():
    """X = [[1, 2], [2, 4]]: G = [[5, 10], [10, 20]], lam = (25, 0), v1 = (1, 2)/sqrt 5.

    A = X^T v1 = (sqrt 5, 2 sqrt 5); with eps = 0.5: qV = rint(65536 v1) =
    (29309, 58617) (65536/sqrt 5 = 29308.59), qA = rint(2 A) = (4, 9).
    """
    x = np.array([[1.0, 2.0], [2.0, 4.0]])
    c = dls.encode_block(x, 0.5, 2, np.float64)
    assert c.r == 1
    assert np.allclose(c.lam, [25.0, 0.0], atol=1e-13)
    assert np.allclose(c.V[:, 0], np.array([1.0, 2.0]) / math.sqrt(5.0), atol=1e-15)
    assert np.allclose(c.A[:, 0], [math.sqrt(5.0), 2 * math.sqrt(5.0)], atol=1e-14)
    assert c.qV[:, 0].tolist() == [29309, 58617]
    assert c.qA[:, 0].tolist() == [4, 9]
    S = np.array([[29309 * 4, 29309 * 9], [58617 * 4, 58617 * 9]])
    xhat = S * (0.5 / 65536.0)
    q = np.rint((x - xhat) / 1.0)
    assert np.array_equal(dls.unzigzag8(c.codes), q)


def pin_special_blocks():
    """Constant block: r = 1, lam_1 = c^2 M W.  Zero block: r = 1, qA = 0.  W_b = 1: r = 1."""
    w, m, cst = 16, 64, 0.75
    x = np.full((w, m), cst)
    c = dls.encode_block(x, 1e-3, 16, np.float64)
    assert c.r == 1 and abs(c.lam[0] - cst * cst * m * w) <= 1e-12 * cst * cst * m * w
    assert np.all(c.lam[1:] <= 1e-12)
    assert c.esc_values.size == 0
    z = dls.encode_block(np.zeros((w, m)), 1e-3, 16, np.float64)
    assert z.r == 1 and not z.qA.any() and not z.codes.any()
    one = dls.encode_block(np.random.default_rng(3).normal(size=(1, m)), 1e-3, 16, np.float64)
    assert one.r == 1
    nan = np.ones((4, 8))
    nan[2, 3] = np.nan
    rb = dls.encode_block(nan, 1e-3, 16, np.float64)
    assert rb.r == 0 and rb.esc_values.size == 32
    out = dls.decode_block(0, rb.qV, rb.qA, rb.codes, rb.esc_values, 1e-3, np.float64)
    assert np.array_equal(out, nan, equal_nan=True)


# -- plan -----------------------------------------------------------------
def pin_gradient_and_percentile():
    rng = np.random.default_rng(14)
    f = rng.normal(size=(5, 6, 7))
    g = dls.gradient_magnitude(f)
    gz, gy, gx = np.gradient(f, edge_order=1)
    assert np.allclose(g, np.sqrt(gx ** 2 + gy ** 2 + gz ** 2), rtol=1e-14, atol=0)
    f2 = rng.normal(size=(1, 9, 11))
    g2 = dls.gradient_magnitude(f2)
    gy2, gx2 = np.gradient(f2[0], edge_order=1)
    assert np.allclose(g2[0], np.sqrt(gx2 ** 2 + gy2 ** 2), rtol=1e-14, atol=0)
    for n in (1000, 1001, 37, 2):
        v = rng.normal(size=n)
        assert dls.percentile80(v) == np.percentile(v, 80, method="lower")


def _localized_field(nx, ny, nz):
    """A few narrow Gaussian bumps on a smooth background (refines locally)."""
    rng = np.random.default_rng(15)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    f = 0.01 * np.sin(0.05 * x + 0.03 * y + 0.02 * z)
    for _ in range(3):
        c = rng.uniform(0, 1, 3) * [nx, ny, nz]
        w = rng.uniform(1.5, 3.0)
        d2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + ((z - c[2]) ** 2 if nz > 1 else 0)
        f += np.exp(-d2 / (2 * w * w))
    return f


def pin_adaptive_plan():
    """Leaves tile the domain once, respect [pmin, pmax], are sorted, follow the rule."""
    for (nz, ny, nx, pmax, pmin) in [(1, 64, 96, 32, 4), (1, 50, 37, 16, 4), (24, 20, 32, 16, 4)]:
        f = _localized_field(nx, ny, nz)
        p = dls.Params(nx=nx, ny=ny, nz=nz, nt=1, nvars=1, dtype="f64", px=pmax,
                       py=pmax, pz=pmax if nz > 1 else 1, window=1, eps=[1.0],
                       pmin=pmin, adaptive=True)
        leaves, bits = dls.adaptive_leaves(f, p)
        cover = np.zeros((nz, ny, nx), np.int32)
        for (x0, y0, z0, ex, ey, ez, e) in leaves:
            cover[z0:z0 + ez, y0:y0 + ey, x0:x0 + ex] += 1
        assert (cover == 1).all()
        keys = [(L[2], L[1], L[0]) for L in leaves]
        assert keys == sorted(keys)
        g = dls.gradient_magnitude(f)
        thr = float(np.percentile(g, 80, method="lower"))
        nsplit = 0
        for (x0, y0, z0, ex, ey, ez, e) in leaves:
            assert pmin <= e <= pmax and e & (e - 1) == 0
            assert x0 % e == 0 and y0 % e == 0 and (nz == 1 or z0 % e == 0)
            assert ex == min(e, nx - x0) and ey == min(e, ny - y0)
            if e > pmin:      # not split: mean gradient at or below the threshold
                assert g[z0:z0 + ez, y0:y0 + ey, x0:x0 + ex].mean() <= thr
            if e < pmax:      # its parent was split: parent mean above the threshold
                h = 2 * e
                px0, py0 = x0 - x0 % h, y0 - y0 % h
                pz0 = z0 - z0 % h if nz > 1 else 0
                pz1 = pz0 + h if nz > 1 else 1
                assert g[pz0:pz1, py0:py0 + h, px0:px0 + h].mean() > thr
                nsplit += 1
        assert nsplit > 0
        assert dls.leaves_from_bits(p, bits) == leaves


# -- container ------------------------------------------------------------
def _c1_small(adaptive=False, dtype=np.float64):
    f = synth.blobs2d(nx=40, ny=36, nt=20, seed=2, dtype=dtype)
    rng_ = synth.range_of(f)
    p = dls.Params(nx=40, ny=36, nz=1, nt=20, nvars=1,
                   dtype="f64" if dtype == np.float64 else "f32",
                   px=16 if adaptive else 8, py=16 if adaptive else 8, pz=1,
                   window=16, eps=[1e-3 * rng_[0]], pmin=4, adaptive=adaptive)
    return f, p


def pin_container_round_trip():
    for adaptive in (False, True):
        for dt in (np.float64, np.float32):
            f, p = _c1_small(adaptive, dt)
            enc = dls.encode(f, p)
            buf = container.pack(enc)
            dec = container.unpack(buf)
            assert len(dec.blocks) == len(enc.blocks)
            for a, b in zip(enc.codes, dec.codes):
                assert a.r == b.r
                assert np.array_equal(a.qV, b.qV) and np.array_equal(a.qA, b.qA)
                assert np.array_equal(a.codes, b.codes)
                assert np.array_equal(a.esc_values, b.esc_values)
            out = dls.reconstruct(dec)
            assert np.array_equal(out, dls.reconstruct(enc))
            assert np.abs(out.astype(np.float64) - f.astype(np.float64)).max() <= p.eps[0]




def pin_round_bf16():
    """The oracle's bfloat16 rounding (mantissa arithmetic) agrees with the
    float32 bit rule (add 0x7FFF plus the lowest kept bit, truncate) on
    random normal values, and with hand-worked cases."""
    from oracle import learned
    rng = np.random.default_rng(4)
    x = rng.normal(size=20000) * np.exp(rng.uniform(-30, 30, 20000))
    assert np.array_equal(dls.round_bf16(x), learned.bf16(x))
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa (1) wins;
    # 1 + 3 * 2^-8 ties between 1 + 2^-7 and 1 + 2^-6: even (1 + 2^-6) wins
    assert dls.round_bf16(np.array([1 + 2.0 ** -8]))[0] == 1.0
    assert dls.round_bf16(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6
    assert dls.round_bf16(np.array([-(1 + 2.0 ** -8 + 2.0 ** -20)]))[0] == -(1 + 2.0 ** -7)
    assert dls.round_bf16(np.array([0.0, 3.0]))[1] == 3.0

    # the bf16-Gram mode forms G from the rounded values: a 1 x 2 block
    # [1 + 2^-8, 3] has G = 1 + 9 = 10 exactly (the full-precision G is larger)
    x = np.array([[1 + 2.0 ** -8, 3.0]])
    c = dls.encode_block(x, 1e-3, 1, np.float64, bf16_gram=True)
    assert c.lam[0] == 10.0
    assert dls.encode_block(x, 1e-3, 1, np.float64).lam[0] > 10.0


# -- hand-worked fixtures: input statistics, NRMSE, sign ties ---------------
def _golden(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)) as fh:
        return json.load(fh)


def pin_moments_hand_case():
    """The 16 statistics of a 4 x 2 block against values worked by hand
    (golden moments_4x2.json), and the temporal autocorrelations and
    log10(std / eps) of a random block against explicit loops over the
    definitions."""
    from oracle import learned
    g = _golden("moments_4x2.json")
    i = g["inputs"]
    f = learned.moments(np.array(i["x"]), i["px"], i["py"], i["pz"], i["eps"])
    assert np.allclose(f, g["expected"]["f"], rtol=0, atol=1e-12), f
    rng = np.random.default_rng(21)
    w, m = 7, 12
    x = rng.normal(size=(w, m)) + np.arange(w)[:, None] * 0.3
    f = learned.moments(x, 4, 3, 1, 0.05)
    vals = [float(v) for v in x.ravel()]
    mu = sum(vals) / len(vals)
    var = sum((v - mu) ** 2 for v in vals) / len(vals)
    for lag, k in ((1, 10), (2, 11)):
        acc, n = 0.0, 0
        for t in range(w - lag):
            for q in range(m):
                acc += (x[t + lag, q] - mu) * (x[t, q] - mu)
                n += 1
        assert abs(f[k] - acc / n / var) <= 1e-12, (lag, f[k], acc / n / var)
    assert abs(f[13] - math.log10(math.sqrt(var) / 0.05)) <= 1e-12


def pin_nrmse_hand_case():
    """NRMSE (Sec. 2.4) of the hand-worked 2 x 2 case (golden nrmse_2x2.json)
    and of a field off by a constant fraction (closed form 100 * |s|)."""
    g = _golden("nrmse_2x2.json")
    got = dls.nrmse(np.array(g["inputs"]["u"]), np.array(g["inputs"]["u_hat"]))
    assert abs(got - g["expected"]["nrmse"]) <= 1e-12, got
    u = np.random.default_rng(3).normal(size=(2, 5, 1, 4, 3))
    assert abs(dls.nrmse(u, u * (1 - 0.025)) - 2.5) <= 1e-12


def pin_sign_tie():
    """Canonical signs on an exact magnitude tie (golden sign_tie_2x2.json):
    the lowest index among the largest magnitudes is made positive,
    whichever sign the solver returned."""
    g = _golden("sign_tie_2x2.json")
    want = np.array(g["expected"]["V_sign"], dtype=float) / math.sqrt(2.0)
    got = dls.canonical_signs(np.array(g["inputs"]["flipped"]))
    assert np.array_equal(np.sign(got), np.sign(want)), got
    lam, V = dls.eig_desc(np.array(g["inputs"]["G"]))
    assert np.allclose(lam, g["expected"]["lam"], rtol=0, atol=1e-12)
    assert np.array_equal(np.sign(V), np.array(g["expected"]["V_sign"])), V


# -- the single-pass form: rank-1 basis, exact verification, sketch ---------
def pin_rank_one_single_pass():
    """The rank-1 basis and its verification (reading R28) against the
    hand-worked 2 x 2 cases (golden rank1_attempt_2x2.json), an exactly
    rank-1 Gram with a zero component, the energy identity checked by
    explicit projection, convergence to the leading eigenvector, the rank
    rule an accepted block implies, and the sketch: on exactly rank-1 data
    the sketch's basis passes the whole block; a block whose later rows add
    a second mode beyond tau fails."""
    g = _golden("rank1_attempt_2x2.json")
    x = np.array(g["inputs"]["x"])
    e = g["expected"]
    tau = g["inputs"]["eps"] ** 2 * x.size
    q = dls.leading_vector(x @ x.T)
    ok, th = dls.rank_one_verify(x @ x.T, q, tau)
    assert ok == e["accepted"] and abs(th - e["theta"]) <= 1e-12 and np.allclose(q, e["q"], rtol=0, atol=1e-15)
    ok, _ = dls.rank_one_verify(np.eye(2), dls.leading_vector(np.eye(2)), g["inputs"]["identity_tau"])
    assert ok == e["identity_accepted"]
    q = dls.leading_vector(np.zeros((3, 3)))
    ok, th = dls.rank_one_verify(np.zeros((3, 3)), q, 0.0)
    assert ok and th == 0.0 and q.tolist() == e["zero_q"] + [0.0]
    a = np.array([0.0, 3.0, -4.0, 0.0, 12.0]) / 13.0
    q = dls.leading_vector(49.0 * np.outer(a, a))
    ok, th = dls.rank_one_verify(49.0 * np.outer(a, a), q, 1e-9)
    assert ok and abs(th - 49.0) <= 1e-12 and np.allclose(q, a * np.sign(a[4]), rtol=0, atol=1e-15)
    rng = np.random.default_rng(31)
    for w, m in [(16, 64), (7, 40), (16, 1024)]:
        xs = _rand_block(rng, w, m)
        G = xs @ xs.T
        q = dls.leading_vector(G)
        _, th = dls.rank_one_verify(G, q, 0.0)
        r_ = xs - np.outer(q, q @ xs)          # exact discarded energy, by projection
        assert abs(np.sum(r_ * r_) - (np.trace(G) - th)) <= 1e-10 * np.trace(G)
        lam, V = dls.eig_desc(G)
        assert th <= lam[0] * (1 + 1e-14)
        # power iteration from e_i (i = largest diagonal entry; the start
        # column G e_i is its first step): tan of the angle to v_1 shrinks by
        # lam_2 / lam_1 per step (Golub & Van Loan, Sec. 8.2.1)
        i = int(np.argmax(np.diag(G)))
        v1 = V[:, 0]
        tan0 = math.sqrt(max(1.0 - v1[i] ** 2, 0.0)) / abs(v1[i])
        bound = tan0 * (lam[1] / lam[0]) ** (dls.FAST_ITERS + 1)
        assert np.linalg.norm(q - v1) <= bound + 1e-12, (np.linalg.norm(q - v1), bound)
        tau = np.trace(G) - th                 # an accepted block: the rank rule picks 1 too
        ok, _ = dls.rank_one_verify(G, q, tau)
        assert ok and dls.choose_rank(lam, tau, w) == 1
    # sketch: the first floor(1024 / px) rows of px points
    assert dls.sketch_points(32768, 32) == 1024 and dls.sketch_points(640, 24) == 640
    assert dls.sketch_points(4096, 24) == 42 * 24 and dls.sketch_points(50, 100) == 50
    t = np.arange(16)[:, None]
    prof = np.exp(-0.02 * t)
    amp = rng.normal(size=(1, 2048))
    xs = prof * amp                               # exactly rank 1 in time
    code, ok = dls.encode_block_sketch(xs, 1e-6, 16, np.float64, 32)
    assert ok and code.r == 1 and np.allclose(code.V[:, 0], prof[:, 0] / np.linalg.norm(prof), rtol=0, atol=1e-14)
    xs2 = xs.copy()
    xs2[:, 1024:] += np.cos(0.7 * t) * rng.normal(size=(1, 1024))   # a second mode outside the sketch
    code, ok = dls.encode_block_sketch(xs2, 1e-6, 16, np.float64, 32)
    assert not ok and code.r >= 2


# -- L2 / NRMSE-bounded mode (oracle.l2) -----------------------------------
def _l2_gold():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "l2_block_2x2.json")
    with open(path) as fh:
        return json.load(fh)


def pin_l2_eckart_young():
    """The eigenvalue tail after r modes is the squared error of the rank-r
    projection (Eckart-Young), computed directly."""
    rng = np.random.default_rng(3)
    for W, M, rank in [(6, 40, 6), (8, 30, 3), (5, 5, 5)]:
        X = rng.standard_normal((W, rank)) @ rng.standard_normal((rank, M)) + 1e-3 * rng.standard_normal((W, M))
        lam, V = dls.eig_desc(X @ X.T)
        tail = dls.tail_energies(lam)
        for r in range(W + 1):
            Vr = V[:, :r]
            R = X - Vr @ (Vr.T @ X)
            assert abs(float(np.sum(R * R)) - tail[r]) <= 1e-10 * float(np.sum(X * X)), (W, M, r)


def _l2_hand(target):
    u = np.array([[2.0, 0.0], [0.0, 1.0]]).reshape(1, 2, 1, 1, 2)
    p = dls.Params(nx=2, ny=1, nz=1, nt=2, nvars=1, dtype="f64", px=2, py=1, pz=1, window=2, eps=[target])
    return u, p


def pin_l2_hand_case():
    """The one-block field of tests/golden/l2_block_2x2.json, worked by hand
    (cases A and B) and the rank rule's hand cases."""
    g = _l2_gold()
    for target, e in ((g["inputs"]["target"], g["expected"]), (g["inputs"]["target_b"], g["expected"]["b"])):
        u, p = _l2_hand(target)
        enc = l2.encode(u, p)
        c = enc.codes[0]
        assert abs(c.e2 - e["e2"]) <= 1e-12 * e["e2"]
        assert c.r == e["rank"]
        # decimal hand values fix the numbers to ~1e-15, not the last bit of FP64
        assert abs(c.step - e["step"]) <= 1e-14 * e["step"]
        qa = e["qA"] if isinstance(e["qA"][0], list) else [[q] for q in e["qA"]]
        assert c.qA.tolist() == qa
        if "qV" in e:
            assert c.qV[:, 0].tolist() == e["qV"]
        out = l2.reconstruct(enc)
        assert np.allclose(out.reshape(2, 2), np.array(e["out"]), rtol=1e-14, atol=0.0)
        assert abs(c.err - e["err"]) <= 1e-8
    u, p = _l2_hand(g["inputs"]["target"])
    assert abs(l2.nrmse_fraction(u, l2.reconstruct(l2.encode(u, p))) - g["expected"]["nrmse"]) <= 1e-4
    for e2, r in g["expected"]["rank_rule"]:
        assert l2.first_rank(np.array([4.0, 1.0]), e2, 2) == r, (e2, r)


def pin_l2_budgets_sum():
    """sum_b e2_b = (eps_t ||u||)^2: the block budgets are equal shares of
    the variable's squared global budget."""
    f = synth.blobs2d(nx=70, ny=45, nt=37, seed=3, nblobs=6)
    p = dls.Params(nx=70, ny=45, nz=1, nt=37, nvars=1, dtype="f64", px=16, py=16, pz=1, window=16,
                   eps=[0.01], pmin=4, adaptive=True)
    blocks, _ = dls.plan(f, p)
    c = l2.variable_budgets(f, p.eps)
    total = sum(l2.block_budget(c[b.var], b) for b in blocks)
    want = (0.01 ** 2) * float(np.sum(f.astype(np.float64) ** 2))
    assert abs(total - want) <= 1e-12 * want


def _l2_fields():
    a = synth.blobs2d(nx=48, ny=40, nt=20, seed=4, nblobs=8, dtype=np.float32)
    pa = dict(nx=48, ny=40, nz=1, nt=20, nvars=1, dtype="f32", px=16, py=8, pz=1, window=16)
    b = np.concatenate([synth.spectrum(20, 18, 12, 14, nmodes=12, seed=s, drift=True) for s in (5, 6)])
    pb = dict(nx=20, ny=18, nz=12, nt=14, nvars=2, dtype="f32", px=8, py=8, pz=8, window=8)
    return [(a, pa), (b, pb)]


def pin_l2_bound_and_round_trip(targets=(1e-2, 1e-4)):
    """Every block's exact error within its budget, every variable's NRMSE
    within its target, the stream reproduces the decoded field bit for bit;
    the precision parameter has no effect in this mode (FP64 Gram)."""
    for target in targets:
        for f, kw in _l2_fields():
            p = dls.Params(eps=[target] * kw["nvars"], **kw)
            enc = l2.encode(f, p)
            out = l2.reconstruct(enc)
            for b, c in zip(enc.blocks, enc.codes):
                xb = dls.gather(f, b).astype(np.float64)
                ob = dls.gather(out, b).astype(np.float64)
                assert float(np.sum((xb - ob) ** 2)) <= c.e2
            for v in range(p.nvars):
                assert l2.nrmse_fraction(f[v], out[v]) <= target
            assert np.array_equal(l2.decompress(container.pack_l2(enc)).view(np.uint8), out.view(np.uint8))
    f, kw = _l2_fields()[1]
    a = container.pack_l2(l2.encode(f, dls.Params(eps=[1e-3] * kw["nvars"], precision="bf16", **kw)))
    b = container.pack_l2(l2.encode(f, dls.Params(eps=[1e-3] * kw["nvars"], **kw)))
    assert a == b


def pin_l2_ranks_grow():
    """A tighter target never takes fewer modes on average."""
    f, kw = _l2_fields()[1]
    means = []
    for target in (1e-1, 1e-2, 1e-3):
        enc = l2.encode(f, dls.Params(eps=[target] * kw["nvars"], **kw))
        means.append(np.mean([c.r for c in enc.codes if c.r != l2.RAW]))
    assert means[0] < means[1] < means[2]


def pin_l2_special_blocks():
    """A non-finite block is raw and returned exactly; a zero block takes
    rank 0; a target below the 2^-24 basis grid makes the block raw."""
    f = synth.blobs2d(nx=16, ny=8, nt=8, seed=7, nblobs=3)
    f[0, :, 0, :, 8:] = 0.0
    f[0, 3, 0, 2, 1] = np.nan
    p = dls.Params(nx=16, ny=8, nz=1, nt=8, nvars=1, dtype="f64", px=8, py=8, pz=1, window=8, eps=[1e-2])
    enc = l2.encode(f, p)
    assert [c.r for c in enc.codes] == [l2.RAW, 0]
    out = l2.reconstruct(enc)
    assert np.array_equal(np.isnan(out), np.isnan(f))
    assert np.array_equal(np.nan_to_num(out), np.nan_to_num(f))
    g = synth.blobs2d(nx=8, ny=8, nt=8, seed=8, nblobs=2) + 10.0
    q = dls.Params(nx=8, ny=8, nz=1, nt=8, nvars=1, dtype="f64", px=8, py=8, pz=1, window=8, eps=[1e-12])
    enc = l2.encode(g, q)
    assert enc.codes[0].r == l2.RAW
    assert np.array_equal(l2.reconstruct(enc), g)


# ---------------------------------------------------------------- global basis

def pin_splitmix64_published():
    """The generator's first outputs from state 0, as published with it."""
    g = gb.SplitMix64(0)
    assert [g.next() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def pin_cosine_basis():
    """The cosine basis is the orthonormal DCT-II: its 1D factor equals the
    library's orthonormal DCT-II matrix, the tensor basis is orthonormal and
    the 2 x 2 case is the hand-worked one."""
    from scipy.fft import dct
    for n in (1, 2, 5, 8):
        assert np.allclose(gb.cosine_basis(n, 1, 1), dct(np.eye(n), type=2, norm="ortho", axis=0).T, atol=1e-15)
    phi = gb.cosine_basis(4, 3, 2)
    assert np.abs(phi.T @ phi - np.eye(24)).max() < 1e-14
    h = np.array([[0.5, 0.5, 0.5, 0.5], [0.5, -0.5, 0.5, -0.5], [0.5, 0.5, -0.5, -0.5], [0.5, -0.5, -0.5, 0.5]]).T
    assert np.abs(gb.cosine_basis(2, 2, 1) - h).max() < 1e-15


def pin_global_sampling_and_svd_basis():
    """Q holds S = 4M patches of snapshot 0 at in-range positions (checked
    against the field by brute force); the learned basis diagonalises Q^T Q
    with eigenvalues equal to the squared singular values from the library's
    SVD, descending, canonical signs, orthonormal to the 2^-24 grid."""
    f = synth.blobs2d(nx=20, ny=12, nt=3, seed=3, nblobs=3)
    p = dls.Params(nx=20, ny=12, nz=1, nt=3, nvars=1, dtype="f64", px=4, py=3, pz=1, window=1, eps=[1e-3])
    pos = gb.sample_positions(p, 0, 5, 48)
    assert len(pos) == 48 and all(0 <= x <= 16 and 0 <= y <= 9 and z == 0 for x, y, z in pos)
    assert len(set(pos)) > 30
    Q = gb.sample_matrix(f, p, 0, 5)
    assert Q.shape == (48, 12)
    for r, (x0, y0, _) in enumerate(pos):
        for j in range(3):
            for i in range(4):
                assert Q[r, j * 4 + i] == f[0, 0, 0, y0 + j, x0 + i]
    phi = gb.learn_basis(f, p, 0, gb.KIND_SVD, 5)
    sv = np.linalg.svd(Q, compute_uv=False)
    lam = np.diag(phi.T @ (Q.T @ Q) @ phi)
    assert np.all(np.diff(lam) <= 1e-9 * lam[0])
    assert np.allclose(lam, sv ** 2, rtol=1e-6, atol=1e-9 * sv[0] ** 2)
    assert np.abs(phi.T @ phi - np.eye(12)).max() < 1e-6
    for k in range(12):
        i = int(np.argmax(np.abs(phi[:, k])))
        assert phi[i, k] > 0
    assert np.all(np.rint(phi * 2.0 ** 24) == phi * 2.0 ** 24)
    # the random basis: eigenbasis of a uniform [-1, 1) matrix, orthonormal
    R = gb.random_matrix(p, 0, 5)
    assert R.shape == (12, 12) and R.min() >= -1.0 and R.max() < 1.0 and abs(R.mean()) < 0.2
    pr = gb.learn_basis(f, p, 0, gb.KIND_RANDOM, 5)
    assert np.abs(pr.T @ pr - np.eye(12)).max() < 1e-6


def pin_global_hand_case():
    """The hand-worked 2 x 2 patch (tests/golden/global_patch_2x2.json)."""
    fx = _golden("global_patch_2x2.json")
    u = np.array(fx["inputs"]["u"]).reshape(1, 1, 1, 2, 2)
    for t, ex in ((fx["inputs"]["target"], fx["expected"]), (fx["inputs"]["target_b"], fx["expected"]["b"])):
        p = dls.Params(nx=2, ny=2, nz=1, nt=1, nvars=1, dtype="f64", px=2, py=2, pz=1, window=1, eps=[t])
        enc = gb.encode(u, p, gb.KIND_COSINE)
        c = enc.codes[0]
        assert (c.n, c.k, list(c.kept), list(c.q)) == (ex["n"], ex["k"], ex["kept"], ex["q"])
        assert c.e2 == ex["e2"] and c.err == ex["err"]
        assert list(gb.reconstruct(enc).ravel()) == ex["xhat"]
    assert list(enc.bases[0].T @ np.array(fx["inputs"]["u"])) == fx["expected"]["alpha"]
    assert np.abs(gb.cosine_basis(2, 2, 1).T @ np.array(fx["inputs"]["u"]) - fx["expected"]["alpha"]).max() < 1e-14


def _global_fields():
    a = synth.blobs2d(nx=40, ny=24, nt=6, seed=9, nblobs=5, dtype=np.float32)
    pa = dict(nx=40, ny=24, nz=1, nt=6, nvars=1, dtype="f32", px=8, py=8, pz=1, window=1)
    b = np.concatenate([synth.spectrum(12, 10, 8, 3, nmodes=8, seed=s, drift=True) for s in (3, 4)])
    pb = dict(nx=12, ny=10, nz=8, nt=3, nvars=2, dtype="f32", px=4, py=4, pz=4, window=1)
    return [(a, pa), (b, pb)]


def pin_global_bound_and_round_trip():
    """For every basis kind: every patch's exact error within its e2 (the
    sum of the e2 is the squared global budget), every variable's NRMSE
    within its target, the kept count never below the energy rule's, and
    the stream reproduces the decoded field bit for bit (edge patches of
    the 3D field are truncated)."""
    for kind in (gb.KIND_SVD, gb.KIND_COSINE, gb.KIND_RANDOM):
        for target in (1e-2, 1e-4):
            for f, kw in _global_fields():
                p = dls.Params(eps=[target] * kw["nvars"], **kw)
                enc = gb.encode(f, p, kind, seed=11)
                out = gb.reconstruct(enc)
                for b, c in zip(enc.blocks, enc.codes):
                    xb = dls.gather(f, b).astype(np.float64)
                    ob = dls.gather(out, b).astype(np.float64)
                    assert float(np.sum((xb - ob) ** 2)) <= c.e2
                    assert c.n == gb.RAW or c.n >= c.n0
                for v in range(p.nvars):
                    e2sum = sum(c.e2 for b, c in zip(enc.blocks, enc.codes) if b.var == v)
                    want = target ** 2 * float(np.sum(f[v].astype(np.float64) ** 2))
                    assert abs(e2sum - want) <= 1e-9 * want
                    assert l2.nrmse_fraction(f[v], out[v]) <= target
                assert np.array_equal(gb.decompress(container.pack_global(enc)).view(np.uint8), out.view(np.uint8))


def pin_global_parseval_selection():
    """With an orthonormal basis the energy rule's dropped energy is the
    squared projection error of the kept coefficients (before rounding),
    and no other set of the same size drops less (brute force over all
    subsets of a 6-point patch)."""
    import itertools
    rng = np.random.default_rng(4)
    phi = gb.cosine_basis(3, 2, 1)
    for _ in range(20):
        u = rng.normal(size=6)
        alpha = phi.T @ u
        order = np.argsort(-np.abs(alpha), kind="stable")
        for n in range(7):
            kept = order[:n]
            proj = phi[:, kept] @ alpha[kept]
            dropped = float(np.sum(alpha[order[n:]] ** 2))
            assert abs(float(np.sum((u - proj) ** 2)) - dropped) <= 1e-12 * float(u @ u)
            best = min(float(np.sum(np.delete(alpha, list(c)) ** 2)) for c in itertools.combinations(range(6), n))
            assert dropped <= best + 1e-12


def pin_global_special_patches():
    """A non-finite patch is raw and returned exactly; a zero patch keeps
    no coefficient; a target below the dtype's resolution makes patches
    raw; the SVD basis beats the random one on a smooth field (fewer kept
    coefficients), the study's qualitative ordering."""
    f = synth.blobs2d(nx=16, ny=8, nt=2, seed=7, nblobs=3)
    f[0, :, 0, :, 8:] = 0.0
    f[0, 1, 0, 2, 1] = np.nan
    p = dls.Params(nx=16, ny=8, nz=1, nt=2, nvars=1, dtype="f64", px=8, py=8, pz=1, window=1, eps=[1e-2])
    enc = gb.encode(f, p, gb.KIND_COSINE)
    ns = [c.n for c in enc.codes]
    assert ns[1] == 0 and ns[3] == 0 and ns[2] == gb.RAW and ns[0] not in (0, gb.RAW)
    out = gb.reconstruct(enc)
    assert np.array_equal(np.isnan(out), np.isnan(f))
    g = (synth.blobs2d(nx=8, ny=8, nt=1, seed=8, nblobs=2) + 1e6).astype(np.float32)
    q = dls.Params(nx=8, ny=8, nz=1, nt=1, nvars=1, dtype="f32", px=8, py=8, pz=1, window=1, eps=[1e-12])
    enc = gb.encode(g, q, gb.KIND_SVD, seed=1)
    assert enc.codes[0].n == gb.RAW and np.array_equal(gb.reconstruct(enc), g)
    h = synth.blobs2d(nx=48, ny=48, nt=2, seed=2, nblobs=6)
    r = dls.Params(nx=48, ny=48, nz=1, nt=2, nvars=1, dtype="f64", px=8, py=8, pz=1, window=1, eps=[1e-3])
    svd = np.mean([c.n for c in gb.encode(h, r, gb.KIND_SVD, seed=2).codes])
    rnd = np.mean([c.n for c in gb.encode(h, r, gb.KIND_RANDOM, seed=2).codes])
    assert svd < rnd


ALL_PINS = [
    pin_eigenvalues_vs_svd, pin_eigenvectors_orthonormal_and_residual,
    pin_eigenvalues_vs_jacobi, pin_rank_bruteforce, pin_exact_rank_data,
    pin_pointwise_bound, pin_escapes_rare_on_smooth_data, pin_escape_threshold, pin_lattice_one_rounding,
    pin_hand_worked_rank_one, pin_special_blocks, pin_gradient_and_percentile,
    pin_adaptive_plan, pin_container_round_trip, pin_round_bf16, pin_moments_hand_case,
    pin_nrmse_hand_case, pin_sign_tie, pin_rank_one_single_pass, pin_l2_eckart_young, pin_l2_hand_case,
    pin_l2_budgets_sum, pin_l2_bound_and_round_trip, pin_l2_ranks_grow, pin_l2_special_blocks,
    pin_splitmix64_published, pin_cosine_basis, pin_global_sampling_and_svd_basis, pin_global_hand_case,
    pin_global_bound_and_round_trip, pin_global_parseval_selection, pin_global_special_patches,
]
