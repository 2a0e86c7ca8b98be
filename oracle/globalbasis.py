"""FP64 oracle of the global-basis mode (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
module; the product path never does.

This is the paper's own method (Sec. 2.2-2.5, Alg. 1): ONE basis per
variable, learned once, applied to every patch of every snapshot.

 1. learn    -- Alg. 1 step 1: S = 4M patches of M = Px Py Pz points at random
                positions of the first snapshot (reading R1: S = 4M) form
                Q (S x M, rows = flattened patches); Q = U Sigma V^T, and the
                compression matrix is the full V (Eqs. (2)-(3): no mode is
                dropped).  V comes from the cross-product Q^T Q (Sec. 2.7.1),
                eigenvalues descending, canonical signs (largest-|v_i| entry
                positive, first index on ties).  Alternatives of Sec. 4's
                basis study: the orthonormal DCT-II tensor basis ("cosine")
                and the eigenbasis of a uniform random matrix ("random").
                The basis is stored on the 2^-24 grid: Phi = rint(V 2^24) 2^-24.
 2. budget   -- the L2 target of Sec. 2.4 per variable: e2 = c_v M_b with
                c_v = (eps_t,v ||u_v||)^2 / K_v, the equal share of each value
                (the same reading as ``oracle.l2``; a patch of one snapshot
                has W_b = 1).
 3. per patch and snapshot (Alg. 1 step 3, Eqs. (5)-(6)):
                alpha = Phi^T u (u zero-padded to M at the domain edges);
                coefficients sorted by decreasing |alpha| (ties: lower index
                first); n = the smallest count whose dropped energy (the sum
                of the other alpha^2, the squared projection error for an
                orthonormal basis) is <= TAIL_SHARE e2;
                bit grooming: the kept alpha on the grid d = 2^k with
                k = floor(log2(STEP_SHARE sqrt(e2 / n))), q = rint(alpha / d);
                decode xhat_i = dtype(sum_{s kept, ascending s} Phi[i][s] (q_s d))
                summed in order in FP64; the exact squared error over the
                patch's in-domain points must be <= e2, else n + 1 (the next
                coefficient in magnitude order), and the patch is stored raw
                (values verbatim) past n = M, on |q| >= 2^31 or on non-finite
                input.

Random draws: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), state
advanced by the golden gamma 0x9E3779B97F4A7C15 and mixed by the published
finaliser; the library implements the same generator independently.
Variable v's sequence starts from state seed + v.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import dls

TAIL_SHARE = 0.36
STEP_SHARE = 0.4
BASIS_BITS = 24
RAW = 0xFFFF              # coefficient count of a patch stored verbatim
QA_LIMIT = 2.0 ** 31
MAX_M = 1024              # largest patch (points) of the mode

KIND_SVD, KIND_COSINE, KIND_RANDOM = 0, 1, 2
KINDS = {"svd": KIND_SVD, "cosine": KIND_COSINE, "random": KIND_RANDOM}

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


class SplitMix64:
    """The SplitMix64 generator (64-bit state, one output per step)."""

    def __init__(self, state: int):
        self.state = state & _MASK

    def next(self) -> int:
        self.state = (self.state + _GAMMA) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)


def sample_positions(p: dls.Params, v: int, seed: int, count: int):
    """Top-left corners of the learning patches of variable v: three draws
    per patch, x0 = draw mod (nx - px + 1), then y0, then z0."""
    g = SplitMix64(seed + v)
    out = []
    for _ in range(count):
        x0 = g.next() % (p.nx - p.px + 1)
        y0 = g.next() % (p.ny - p.py + 1)
        z0 = g.next() % (p.nz - p.pz + 1)
        out.append((x0, y0, z0))
    return out


def sample_matrix(field: np.ndarray, p: dls.Params, v: int, seed: int) -> np.ndarray:
    """Q (S x M): the flattened learning patches of snapshot 0, rows in draw
    order, point index (k Py + j) Px + i."""
    m = p.px * p.py * p.pz
    rows = []
    for x0, y0, z0 in sample_positions(p, v, seed, 4 * m):
        patch = field[v, 0, z0:z0 + p.pz, y0:y0 + p.py, x0:x0 + p.px]
        rows.append(patch.astype(np.float64).ravel())
    return np.array(rows)


def random_matrix(p: dls.Params, v: int, seed: int) -> np.ndarray:
    """M x M entries uniform in [-1, 1): (draw >> 11) 2^-52 - 1, row-major."""
    m = p.px * p.py * p.pz
    g = SplitMix64(seed + v)
    return np.array([[(g.next() >> 11) * 2.0 ** -52 - 1.0 for _ in range(m)] for _ in range(m)])


def cosine_basis(px: int, py: int, pz: int) -> np.ndarray:
    """Orthonormal DCT-II tensor basis: column (c Py + b) Px + a is
    C_a(i) C_b(j) C_c(k) with C_a(i) = sqrt((2 - [a = 0]) / P) cos(pi (2i + 1) a / 2P)."""
    def c1(n):
        out = np.zeros((n, n))
        for a in range(n):
            for i in range(n):
                out[i, a] = math.sqrt((1.0 if a == 0 else 2.0) / n) * math.cos(math.pi * (2 * i + 1) * a / (2 * n))
        return out
    cx, cy, cz = c1(px), c1(py), c1(pz)
    m = px * py * pz
    phi = np.zeros((m, m))
    for k in range(pz):
        for j in range(py):
            for i in range(px):
                row = (k * py + j) * px + i
                for c in range(pz):
                    for b in range(py):
                        for a in range(px):
                            phi[row, (c * py + b) * px + a] = cx[i, a] * cy[j, b] * cz[k, c]
    return phi


def learn_basis(field: np.ndarray, p: dls.Params, v: int, kind: int, seed: int) -> np.ndarray:
    """Alg. 1 step 1 (or a fixed basis of Sec. 4): Phi (M x M) on the 2^-24
    grid, columns = basis vectors."""
    if kind == KIND_COSINE:
        V = cosine_basis(p.px, p.py, p.pz)
    else:
        Q = sample_matrix(field, p, v, seed) if kind == KIND_SVD else random_matrix(p, v, seed)
        _, V = dls.eig_desc(Q.T @ Q)
    return np.rint(V * 2.0 ** BASIS_BITS) * 2.0 ** -BASIS_BITS


def variable_budgets(field: np.ndarray, targets: Sequence[float]) -> np.ndarray:
    """c_v = (eps_t,v ||u_v||)^2 / K_v over the finite values (Sec. 2.4, Eq. (4))."""
    c = []
    for v in range(field.shape[0]):
        x = field[v].astype(np.float64)
        x = x[np.isfinite(x)]
        c.append(float(targets[v]) ** 2 * float(np.sum(x * x)) / float(field[v].size))
    return np.array(c)


def embed(b: dls.Block, p: dls.Params) -> np.ndarray:
    """Full-patch index (k Py + j) Px + i of each of the block's points (its
    own order (k Py_b + j) Px_b + i)."""
    idx = []
    for k in range(b.pz):
        for j in range(b.py):
            for i in range(b.px):
                idx.append((k * p.py + j) * p.px + i)
    return np.array(idx, np.int64)


def step_exponent(e2: float, n: int) -> int:
    """k = floor(log2(STEP_SHARE sqrt(e2 / n))), from the binary exponent."""
    m, e = math.frexp(STEP_SHARE * math.sqrt(e2 / n))
    return e - 1


def decode_patch(phi: np.ndarray, idx: np.ndarray, kept: np.ndarray, q: np.ndarray, k: int, dtype) -> np.ndarray:
    """xhat at the patch's in-domain points: the kept terms in ascending
    index order, one FP64 product and one sum per term, then the cast."""
    d = math.ldexp(1.0, k)
    acc = np.zeros(idx.size)
    for s, qs in zip(kept, q):
        acc = acc + phi[idx, s] * (float(qs) * d)
    return acc.astype(dtype)


@dataclass
class PatchCode:
    n: int                       # kept coefficients, or RAW
    k: int                       # step exponent (d = 2^k)
    kept: np.ndarray             # int64, ascending basis indices
    q: np.ndarray                # int64, quantized coefficients in that order
    raw: Optional[np.ndarray]    # (M_b,) storage dtype, for RAW
    err: float = 0.0
    e2: float = 0.0
    n0: int = 0                  # count from the energy rule, before the check


def encode_patch(xs: np.ndarray, idx: np.ndarray, phi: np.ndarray, e2: float, dtype) -> PatchCode:
    """Step 3 for one patch of one snapshot (xs: its M_b values)."""
    x = xs.astype(np.float64)
    empty = np.zeros(0, np.int64)
    if not np.all(np.isfinite(x)):
        return PatchCode(RAW, 0, empty, empty, xs.copy(), 0.0, e2)
    m = phi.shape[0]
    u = np.zeros(m)
    u[idx] = x
    alpha = phi.T @ u
    order = np.argsort(-np.abs(alpha), kind="stable")
    e = alpha[order] ** 2
    tail = np.zeros(m + 1)
    for j in range(m - 1, -1, -1):
        tail[j] = tail[j + 1] + e[j]
    n = next(j for j in range(m + 1) if tail[j] <= TAIL_SHARE * e2) if tail[m] <= TAIL_SHARE * e2 else m
    n0 = n
    while n <= m:
        if n == 0:
            err = float(np.sum(x * x))
            if err <= e2:
                return PatchCode(0, 0, empty, empty, None, err, e2, n0)
            n = 1
            continue
        if not e2 > 0.0:
            break
        k = step_exponent(e2, n)
        d = math.ldexp(1.0, k)
        kept = np.sort(order[:n])
        qa = np.rint(alpha[kept] / d)
        if np.any(np.abs(qa) >= QA_LIMIT):
            break
        q = qa.astype(np.int64)
        out = decode_patch(phi, idx, kept, q, k, dtype).astype(np.float64)
        err = float(np.sum((x - out) ** 2))
        if err <= e2:
            return PatchCode(n, k, kept, q, None, err, e2, n0)
        n += 1
    return PatchCode(RAW, 0, empty, empty, xs.copy(), 0.0, e2, n0)


@dataclass
class GlobalEncoded:
    params: dls.Params           # window 1; eps holds the targets eps_t,v
    kind: int
    seed: int
    bases: List[np.ndarray]      # Phi per variable (M x M, on the 2^-24 grid)
    budgets: np.ndarray          # c_v
    blocks: List[dls.Block]
    codes: List[PatchCode]


def global_params(p: dls.Params) -> dls.Params:
    """The problem with one snapshot per block (patch x snapshot)."""
    return dls.Params(nx=p.nx, ny=p.ny, nz=p.nz, nt=p.nt, nvars=p.nvars, dtype=p.dtype, px=p.px, py=p.py,
                      pz=p.pz, window=1, eps=list(p.eps), r_max=1)


def encode(field: np.ndarray, p: dls.Params, kind: int = KIND_SVD, seed: int = 0) -> GlobalEncoded:
    """Alg. 1 steps 1-3 for every variable, snapshot and patch."""
    assert field.shape == (p.nvars, p.nt, p.nz, p.ny, p.nx)
    gp = global_params(p)
    m = p.px * p.py * p.pz
    assert m <= MAX_M and p.nx >= p.px and p.ny >= p.py and p.nz >= p.pz
    bases = [learn_basis(field, gp, v, kind, seed) for v in range(p.nvars)]
    c = variable_budgets(field, p.eps)
    blocks = dls.make_blocks(gp, [dls.uniform_leaves(gp)] * p.nvars)
    codes = [encode_patch(dls.gather(field, b)[0], embed(b, gp), bases[b.var], c[b.var] * b.m, gp.np_dtype)
             for b in blocks]
    return GlobalEncoded(gp, kind, seed, bases, c, blocks, codes)


def reconstruct(enc: GlobalEncoded) -> np.ndarray:
    p = enc.params
    out = np.zeros((p.nvars, p.nt, p.nz, p.ny, p.nx), dtype=p.np_dtype)
    for b, cd in zip(enc.blocks, enc.codes):
        if cd.n == RAW:
            vals = np.asarray(cd.raw, p.np_dtype)
        elif cd.n == 0:
            vals = np.zeros(b.m, p.np_dtype)
        else:
            vals = decode_patch(enc.bases[b.var], embed(b, p), cd.kept, cd.q, cd.k, p.np_dtype)
        dls.scatter(out, b, vals.reshape(1, b.m))
    return out


def compress(field: np.ndarray, p: dls.Params, kind: int = KIND_SVD, seed: int = 0) -> bytes:
    from . import container
    return container.pack_global(encode(field, p, kind, seed))


def decompress(buf: bytes) -> np.ndarray:
    from . import container
    return reconstruct(container.unpack_global(buf))
