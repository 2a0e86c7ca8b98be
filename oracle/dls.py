"""FP64 oracle of the DLS local-subspace encoder (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
module; the product path never does.

What is computed, per variable v, per spatial block x time window b:

 1. plan    -- uniform tiling with domain-edge truncation, or adaptive
               quadtree/octree leaves (Sec. 2.3 partitions the domain into
               patches; Alg. 1 step 2 "partition the domain").
 2. gather  -- X_b in R^{W_b x M_b}: row t is the flattened patch at time
               t0+t, point index p = (k*Py + j)*Px + i.  This is the sample
               matrix Q of Sec. 2.3 with snapshots as rows.
 3. Gram    -- G = X X^T, the cross-product form of the SVD (Sec. 2.7.1,
               cross-product SVD; Eq. (2) gives the same nonzero spectrum).
 4. eigh    -- G = V diag(lam) V^T, lam descending, clipped at 0, canonical
               signs (largest-magnitude component positive).  Orthonormal by
               construction (Sec. 2.3, Eq. (3) and the remark after it).
 5. rank    -- smallest r in [1, rcap] whose discarded energy
               sum_{k>r} lam_k <= tau, tau = KAPPA eps^2 M_b W_b.  This is the
               local L2 tolerance of Sec. 2.4, Eq. (4) (equal share of an RMS
               budget eps per point), applied with "<=" as in Alg. 1 step 3;
               the energies are sorted, so the bisection of Sec. 2.5 returns
               the same r as this scan.
 6. project -- A = X^T V_r (Sec. 2.5, Eq. (5); Alg. 1 "project onto basis").
 7. quantize-- qV = rint(V_r 2^16), qA = rint(A / eps) (the bit-grooming step
               of Sec. 2.5 read as uniform quantization, round half to even).
 8. lattice -- S = qV qA^T in exact integers; xhat = float64(S) * c with
               c = eps 2^-16 (reconstruction sum of Sec. 2.6 / Alg. 2).
 9. residual-- q = rint((x - xhat) * (1/(2 eps))); out = dtype(float64(S +
               2^17 q) * c); a point with |q| > 127 or |x - out| > eps
               (checked in FP64 on the returned dtype value) is an escape and
               is stored verbatim.  This enforces an absolute pointwise bound,
               a reading beyond the paper's L2 control.
10. pack    -- batches of 1000 blocks, each zlib-compressed (Sec. 2.5 gzip,
               Sec. 2.7.2 batches of 1000 and an addressable header); see
               ``oracle.container``.

A block with a non-finite value is a raw block (rank byte 0): every point is
an escape.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field as dc_field
from typing import List, Optional, Sequence

import numpy as np

KAPPA = 1.0            # tau = KAPPA * eps^2 * M_b * W_b
BASIS_BITS = 16        # qV = rint(V * 2^16)
RES_SHIFT = 17         # 2 eps = 2^17 * c
QA_LIMIT = 2.0 ** 31   # |rint(A/eps)| must stay below this, else the row is zeroed
Q_LIMIT = 127          # residual codes are one byte (zigzag int8); larger |q| -> escape
ESC_CODE = 0xFF        # zigzag code value reserved for escapes
BATCH_BLOCKS = 1000    # Sec. 2.7.2: patches are processed in batches of 1000


# --------------------------------------------------------------------------
# Parameters and plan
# --------------------------------------------------------------------------
@dataclass
class Params:
    """Problem statement: field shape, patch / window sizes, error bound.

    Mirrors Alg. 1's inputs (snapshots, patch size, target error), extended
    with the time window and an absolute per-variable bound.
    """
    nx: int
    ny: int
    nz: int
    nt: int
    nvars: int
    dtype: str                  # 'f32' or 'f64'
    px: int
    py: int
    pz: int
    window: int
    eps: Sequence[float]
    pmin: int = 0               # adaptive: smallest leaf edge
    r_max: int = 0              # 0 -> min(window, 32)
    adaptive: bool = False
    precision: str = "fp32"     # 'bf16': the Gram contraction takes bfloat16 operands

    @property
    def ndim(self) -> int:
        return 3 if self.nz > 1 else 2

    @property
    def np_dtype(self):
        return np.float32 if self.dtype == "f32" else np.float64

    def resolved_rmax(self) -> int:
        return self.r_max if self.r_max > 0 else min(self.window, 32)


@dataclass
class Block:
    var: int
    x0: int
    y0: int
    z0: int
    px: int
    py: int
    pz: int
    t0: int
    w: int

    @property
    def m(self) -> int:
        return self.px * self.py * self.pz


def windows(nt: int, w: int):
    """Time windows (t0, W_b); the last one is truncated."""
    return [(t0, min(w, nt - t0)) for t0 in range(0, nt, w)]


def uniform_leaves(p: Params):
    """Uniform patches in (z0, y0, x0) order, truncated at the domain edges."""
    out = []
    for z0 in range(0, p.nz, p.pz):
        for y0 in range(0, p.ny, p.py):
            for x0 in range(0, p.nx, p.px):
                out.append((x0, y0, z0, min(p.px, p.nx - x0),
                            min(p.py, p.ny - y0), min(p.pz, p.nz - z0), p.px))
    return out


def gradient_magnitude(f0: np.ndarray) -> np.ndarray:
    """|grad f| of one snapshot (shape (nz, ny, nx)) in grid units, float64.

    Central differences (f[i+1] - f[i-1]) * 0.5 inside, one-sided
    differences at the two ends of each axis, 0 along an axis of size 1;
    g = sqrt(dx^2 + dy^2 + dz^2) summed left to right.
    """
    f = f0.astype(np.float64)

    def deriv(axis):
        n = f.shape[axis]
        d = np.zeros_like(f)
        if n == 1:
            return d
        sl = [slice(None)] * 3

        def s(a, b):
            q = list(sl)
            q[axis] = slice(a, b)
            return tuple(q)
        d[s(1, n - 1)] = (f[s(2, n)] - f[s(0, n - 2)]) * 0.5
        d[s(0, 1)] = f[s(1, 2)] - f[s(0, 1)]
        d[s(n - 1, n)] = f[s(n - 1, n)] - f[s(n - 2, n - 1)]
        return d

    dz, dy, dx = deriv(0), deriv(1), deriv(2)
    return np.sqrt(dx * dx + dy * dy + dz * dz)


def percentile80(g: np.ndarray) -> float:
    """sorted(g)[floor(0.8 (n - 1))]: an exact order statistic, no interpolation."""
    v = np.sort(g.ravel())
    return float(v[int(math.floor(0.8 * (v.size - 1)))])


def adaptive_leaves(f0: np.ndarray, p: Params):
    """Quadtree (2D) / octree (3D) leaves for one variable, plus split bits.

    Start from pmax-edge tiles (pmax = px); a node of nominal edge e > pmin
    is split into its 4 / 8 half-edge children (those whose origin lies in
    the domain) while the mean gradient magnitude over its in-domain region
    exceeds the 80th percentile of the snapshot.  Returns (leaves sorted
    lexicographically by (z0, y0, x0), split bits in depth-first pre-order
    over the roots in (z0, y0, x0) order, children in (z, y, x) order).
    A leaf is (x0, y0, z0, ex, ey, ez, e): origin, in-domain extent and
    nominal edge.
    """
    nz, ny, nx = f0.shape
    g = gradient_magnitude(f0)
    thr = percentile80(g)
    e0 = p.px
    is3d = nz > 1
    bits: List[int] = []
    leaves = []

    def visit(x0, y0, z0, e):
        ex, ey, ez = min(e, nx - x0), min(e, ny - y0), (min(e, nz - z0) if is3d else 1)
        if e > p.pmin:
            region = g[z0:z0 + ez, y0:y0 + ey, x0:x0 + ex]
            split = bool(region.sum() / region.size > thr)
            bits.append(1 if split else 0)
            if split:
                h = e // 2
                for dz in ((0, h) if is3d else (0,)):
                    for dy in (0, h):
                        for dx in (0, h):
                            cx, cy, cz = x0 + dx, y0 + dy, z0 + dz
                            if cx < nx and cy < ny and cz < nz:
                                visit(cx, cy, cz, h)
                return
        leaves.append((x0, y0, z0, ex, ey, ez, e))

    for z0 in range(0, nz, e0 if is3d else 1):
        for y0 in range(0, ny, e0):
            for x0 in range(0, nx, e0):
                visit(x0, y0, z0, e0)
    leaves.sort(key=lambda L: (L[2], L[1], L[0]))
    return leaves, bits


def leaves_from_bits(p: Params, bits: Sequence[int]):
    """Rebuild the leaf list of one variable from its split bits (decoder side)."""
    it = iter(bits)
    leaves = []
    is3d = p.nz > 1

    def visit(x0, y0, z0, e):
        ex, ey, ez = min(e, p.nx - x0), min(e, p.ny - y0), (min(e, p.nz - z0) if is3d else 1)
        if e > p.pmin:
            split = next(it)
            if split:
                h = e // 2
                for dz in ((0, h) if is3d else (0,)):
                    for dy in (0, h):
                        for dx in (0, h):
                            cx, cy, cz = x0 + dx, y0 + dy, z0 + dz
                            if cx < p.nx and cy < p.ny and cz < p.nz:
                                visit(cx, cy, cz, h)
                return
        leaves.append((x0, y0, z0, ex, ey, ez, e))

    e0 = p.px
    for z0 in range(0, p.nz, e0 if is3d else 1):
        for y0 in range(0, p.ny, e0):
            for x0 in range(0, p.nx, e0):
                visit(x0, y0, z0, e0)
    leaves.sort(key=lambda L: (L[2], L[1], L[0]))
    return leaves


def make_blocks(p: Params, leaves_per_var) -> List[Block]:
    """Block order: variable, then window, then leaf (lexicographic)."""
    blocks = []
    for v in range(p.nvars):
        for (t0, wb) in windows(p.nt, p.window):
            for (x0, y0, z0, ex, ey, ez, _e) in leaves_per_var[v]:
                blocks.append(Block(v, x0, y0, z0, ex, ey, ez, t0, wb))
    return blocks


def plan(field: np.ndarray, p: Params):
    """Block list and per-variable split bits (empty lists when uniform)."""
    if p.adaptive:
        lv, bits = [], []
        for v in range(p.nvars):
            L, B = adaptive_leaves(field[v, 0], p)
            lv.append(L)
            bits.append(B)
    else:
        L = uniform_leaves(p)
        lv = [L] * p.nvars
        bits = [[] for _ in range(p.nvars)]
    return make_blocks(p, lv), bits


def gather(field: np.ndarray, b: Block) -> np.ndarray:
    """X_b (W_b x M_b) in the storage dtype, p = (k*Py + j)*Px + i."""
    sub = field[b.var, b.t0:b.t0 + b.w, b.z0:b.z0 + b.pz,
                b.y0:b.y0 + b.py, b.x0:b.x0 + b.px]
    return sub.reshape(b.w, b.m)


def scatter(out: np.ndarray, b: Block, xb: np.ndarray) -> None:
    """Snapshot assembly, Eq. (7): place a decoded block back into the field."""
    out[b.var, b.t0:b.t0 + b.w, b.z0:b.z0 + b.pz,
        b.y0:b.y0 + b.py, b.x0:b.x0 + b.px] = xb.reshape(b.w, b.pz, b.py, b.px)


# --------------------------------------------------------------------------
# Per-block encode
# --------------------------------------------------------------------------
@dataclass
class BlockCode:
    r: int                       # 0 = raw block
    qV: np.ndarray               # int64 (W_b, r)
    qA: np.ndarray               # int64 (M_b, r)
    codes: np.ndarray            # uint8 (W_b, M_b), zigzag residual codes / ESC_CODE
    esc_values: np.ndarray       # storage dtype, escaped x in (t, p) order
    # diagnostics (not stored in the stream)
    lam: Optional[np.ndarray] = None
    V: Optional[np.ndarray] = None
    A: Optional[np.ndarray] = None
    tau: float = 0.0
    out: Optional[np.ndarray] = None


def canonical_signs(V: np.ndarray) -> np.ndarray:
    """Flip each column so its largest-magnitude entry is positive (first index on ties)."""
    V = V.copy()
    for k in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, k])))
        if V[i, k] < 0:
            V[:, k] = -V[:, k]
    return V


def eig_desc(G: np.ndarray):
    """Eigenpairs of the symmetric Gram matrix, eigenvalues descending, >= 0."""
    lam, V = np.linalg.eigh(G)
    order = np.argsort(-lam, kind="stable")
    lam = np.maximum(lam[order], 0.0)
    return lam, canonical_signs(V[:, order])


def tail_energies(lam: np.ndarray) -> np.ndarray:
    """tail[r] = sum_{k > r} lam_k for r = 0..W, as suffix sums."""
    t = np.zeros(lam.size + 1)
    for r in range(lam.size - 1, -1, -1):
        t[r] = t[r + 1] + lam[r]
    return t


def choose_rank(lam: np.ndarray, tau: float, rcap: int) -> int:
    """Smallest r in [1, rcap] with discarded energy <= tau, else rcap."""
    tail = tail_energies(lam)
    for r in range(1, rcap + 1):
        if tail[r] <= tau:
            return r
    return rcap


def zigzag8(q: np.ndarray) -> np.ndarray:
    """Residual code of q, |q| <= Q_LIMIT: 0, -1, 1, -2, ... -> 0, 1, 2, 3, ..."""
    q = q.astype(np.int64)
    return np.where(q >= 0, 2 * q, -2 * q - 1).astype(np.uint8)


def unzigzag8(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.int64)
    return np.where(z % 2 == 0, z // 2, -(z + 1) // 2)


def lattice_values(S: np.ndarray, q: np.ndarray, eps: float, dtype) -> np.ndarray:
    """dtype(float64(S + 2^17 q) * c), c = eps 2^-16: one FP64 rounding, one cast."""
    c = math.ldexp(eps, -BASIS_BITS)
    n = S + q * (1 << RES_SHIFT)                     # exact integers < 2^53
    return (n.astype(np.float64) * c).astype(dtype)


def round_bf16(a: np.ndarray) -> np.ndarray:
    """Values rounded to bfloat16 (8 significant bits, round half to even),
    after a first rounding to float32; normal range only."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)
    m, e = np.frexp(f)                       # f = m 2^e, 0.5 <= |m| < 1
    return np.where(f == 0.0, f, np.ldexp(np.rint(np.ldexp(m, 8)), e - 8))


def encode_block(xs: np.ndarray, eps: float, rcap: int, dtype, bf16_gram: bool = False) -> BlockCode:
    """Encode one block X_b (storage dtype, W_b x M_b) under the bound eps.
    With bf16_gram the Gram matrix is formed from the bfloat16-rounded
    snapshots (mixed precision); every later step uses the exact values."""
    wb, m = xs.shape
    x = xs.astype(np.float64)
    if not np.all(np.isfinite(x)):
        return _raw_block(xs)
    xg = round_bf16(x) if bf16_gram else x
    G = xg @ xg.T                                                 # step 3
    lam, V = eig_desc(G)                                          # step 4
    tau = KAPPA * eps * eps * m * wb
    r = choose_rank(lam, tau, min(rcap, wb, m))                   # step 5
    code = encode_with_basis(xs, eps, V[:, :r], lam, tau, dtype)
    code.V = V
    return code


FAST_ITERS = 6        # power steps of the rank-1 basis after its start column
SKETCH_POINTS = 1024  # the sketch is the block's first whole x-rows, at most this many points


def leading_vector(G: np.ndarray, iters: int = FAST_ITERS):
    """The rank-1 basis of the single-pass form (reading R28): q starts as the
    Gram column of the largest diagonal entry (the lowest index on ties;
    e_i itself when that column is zero), normalised, and takes `iters`
    power steps q = G q / ||G q||.  Returned with the canonical sign, or
    None when G is not finite."""
    w = G.shape[0]
    if not np.all(np.isfinite(G)):
        return None
    i = int(np.argmax(np.diag(G)))
    q = G[:, i].astype(np.float64).copy()
    n = math.sqrt(float(q @ q))
    if n > 0.0:
        q = q / n
    else:
        q = np.zeros(w)
        q[i] = 1.0
    for _ in range(iters):
        y = G @ q
        n = math.sqrt(float(y @ y))
        if n > 0.0:
            q = y / n
    return canonical_signs(q[:, None])[:, 0]


def rank_one_verify(G: np.ndarray, q: np.ndarray, tau: float):
    """Exact test of a unit vector q as the block's basis: theta = q^T G q is
    the energy it keeps, so trace(G) - theta = ||X - q q^T X||_F^2 is its
    discarded energy; accepted when that is <= tau (the local tolerance of
    Sec. 2.4 Eq. (4), '<=' as in Alg. 1).  Since lambda_1 >= theta, an
    accepted block has tail_1 <= tau too: rank 1 is what the rank rule
    chooses.  Returns (accepted, theta)."""
    if q is None or not np.all(np.isfinite(G)):
        return False, 0.0
    theta = float(q @ (G @ q))
    return float(np.trace(G)) - theta <= tau, theta


def sketch_points(m: int, px: int) -> int:
    """Points of the sketch: the first floor(SKETCH_POINTS / px) x-rows of
    the block (p order), all of it when smaller."""
    return min(m, max(1, SKETCH_POINTS // px) * px)


def encode_block_sketch(xs: np.ndarray, eps: float, rcap: int, dtype, px: int, bf16_gram: bool = False):
    """encode_block as the single-pass form does it (reading R28): the rank-1
    basis q of the sketch's Gram (the block's first x-rows), verified on the
    whole block's Gram; a block it does not pass takes the plain eigensolve.
    Returns (BlockCode, accepted)."""
    wb, m = xs.shape
    x = xs.astype(np.float64)
    if not np.all(np.isfinite(x)):
        return _raw_block(xs), False
    xg = round_bf16(x) if bf16_gram else x
    G = xg @ xg.T
    s = sketch_points(m, px)
    q = leading_vector(xg[:, :s] @ xg[:, :s].T)
    tau = KAPPA * eps * eps * m * wb
    ok, theta = rank_one_verify(G, q, tau)
    if ok:
        return encode_with_basis(xs, eps, q[:, None], np.array([max(theta, 0.0)]), tau, dtype), True
    return encode_block(xs, eps, rcap, dtype, bf16_gram), False


def encode_with_basis(xs: np.ndarray, eps: float, Vr: np.ndarray, lam: np.ndarray, tau: float,
                      dtype) -> BlockCode:
    """Steps 6-9 for a chosen orthonormal basis V_r (W_b x r)."""
    x = xs.astype(np.float64)
    r = Vr.shape[1]
    A = x.T @ Vr                                                  # step 6 (M x r)
    qV = np.rint(Vr * float(1 << BASIS_BITS)).astype(np.int64)    # step 7
    qa_f = np.rint(A * (1.0 / eps))
    bad = ~np.all(np.abs(qa_f) < QA_LIMIT, axis=1)                # overflow rows -> 0
    qa_f[bad, :] = 0.0
    qA = qa_f.astype(np.int64)
    S = qV @ qA.T                                                 # step 8, exact int64
    c = math.ldexp(eps, -BASIS_BITS)
    xhat = S.astype(np.float64) * c
    q = np.rint((x - xhat) * (1.0 / (2.0 * eps)))                 # step 9
    big = np.abs(q) > Q_LIMIT
    q[big] = 0.0
    qi = q.astype(np.int64)
    out = lattice_values(S, qi, eps, dtype)
    esc = big | (np.abs(x - out.astype(np.float64)) > eps)
    codes = zigzag8(qi)
    codes[esc] = ESC_CODE
    out = np.where(esc, xs, out)
    return BlockCode(r, qV, qA, codes, xs[esc].copy(), lam=lam, V=Vr, A=A,
                     tau=tau, out=out)


def _raw_block(xs: np.ndarray) -> BlockCode:
    wb, m = xs.shape
    return BlockCode(0, np.zeros((wb, 0), np.int64), np.zeros((m, 0), np.int64),
                     np.full((wb, m), ESC_CODE, np.uint8), xs.ravel().copy(),
                     out=xs.copy())


def decode_block(r: int, qV: np.ndarray, qA: np.ndarray, codes: np.ndarray,
                 esc_values: np.ndarray, eps: float, dtype) -> np.ndarray:
    """Alg. 2 for one block: S = qV qA^T, lattice values, then escapes in order."""
    wb, m = codes.shape
    if r == 0:
        S = np.zeros((wb, m), np.int64)
    else:
        S = qV.astype(np.int64) @ qA.astype(np.int64).T
    esc = codes == ESC_CODE
    q = unzigzag8(np.where(esc, 0, codes))
    out = lattice_values(S, q, eps, dtype)
    if esc.any():
        out[esc] = esc_values
    return out


# --------------------------------------------------------------------------
# Whole-field drivers
# --------------------------------------------------------------------------
@dataclass
class Encoded:
    params: Params
    blocks: List[Block]
    codes: List[BlockCode]
    split_bits: list = dc_field(default_factory=list)


def encode(field: np.ndarray, p: Params) -> Encoded:
    """Alg. 1, step 3, over every block of the plan (no container)."""
    assert field.shape == (p.nvars, p.nt, p.nz, p.ny, p.nx)
    assert field.dtype == p.np_dtype
    blocks, bits = plan(field, p)
    rmax = p.resolved_rmax()
    codes = [encode_block(gather(field, b), float(p.eps[b.var]), rmax, p.np_dtype, p.precision == "bf16")
             for b in blocks]
    return Encoded(p, blocks, codes, bits)


def reconstruct(enc: Encoded) -> np.ndarray:
    """Field from an Encoded (decoder arithmetic, Alg. 2 and Eq. (7))."""
    p = enc.params
    out = np.zeros((p.nvars, p.nt, p.nz, p.ny, p.nx), dtype=p.np_dtype)
    for b, c in zip(enc.blocks, enc.codes):
        xb = decode_block(c.r, c.qV, c.qA, c.codes, c.esc_values,
                          float(p.eps[b.var]), p.np_dtype)
        scatter(out, b, xb)
    return out


def nrmse(u: np.ndarray, uh: np.ndarray) -> float:
    """NRMSE of Sec. 2.4: 100 ||u - uh||_2 / ||u||_2 (in FP64)."""
    a = u.astype(np.float64)
    d = a - uh.astype(np.float64)
    return 100.0 * float(np.sqrt(np.sum(d * d)) / np.sqrt(np.sum(a * a)))


def compress(field: np.ndarray, p: Params) -> bytes:
    from . import container
    return container.pack(encode(field, p))


def decompress(buf: bytes) -> np.ndarray:
    from . import container
    return reconstruct(container.unpack(buf))
