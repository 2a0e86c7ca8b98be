"""FP64 oracle of the L2 / NRMSE-bounded mode (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
module; the product path never does.

The paper controls a global L2 error (Sec. 2.4): the user's target eps_t is
a relative L2 error (the NRMSE, Sec. 2.4, as a fraction here rather than a
percentage), the global budget is eps = eps_t ||u|| (Eq. (4) and the text
after it), and each patch receives the local tolerance
eps_l = eps (patch size / number of points)^(1/2), an equal share of the
squared budget per point.  Alg. 1 step 3 keeps, per patch, the fewest
coefficients whose reconstruction meets eps_l, testing candidate sets until
it does.  Here the patch is a block (spatial patch x time window) with its
own basis, so per block and variable v:

 1. budget   -- e2 = c_v M_b W_b with c_v = (eps_t,v ||u_v||)^2 / K_v, K_v the
                number of values of the variable and ||u_v|| the L2 norm of
                its finite values; sum_b e2 = (eps_t,v ||u_v||)^2.
 2. Gram, eigenpairs as in the absolute mode (``oracle.dls``), FP64 whatever
                the precision parameter: the rank test below compares tails with
                a share of e2, which at tight targets is ~1e-8 of the block's
                energy, far below what a Gram of rounded operands resolves (the
                paper fixes no reduced precision for this step).
 3. rank     -- r = 0 if the whole energy sum(lam) <= TAIL_SHARE e2, else the
                smallest r >= 1 with sum_{k>r} lam_k <= TAIL_SHARE e2 (at most
                rcap): by Eckart-Young that tail is the squared Frobenius error
                of the best rank-r approximation, so the truncation uses
                TAIL_SHARE of the budget.
 4. quantize -- basis qV = rint(V_r 2^24); coefficients A = X^T V_r (FP64),
                step d = STEP_SHARE sqrt(e2 / (r M_b)), qA = rint(A / d):
                their rounding adds at most STEP_SHARE/2 sqrt(e2) in norm.
 5. decode   -- xhat[t][p] = dtype(sum_k (qV[t][k] 2^-24) (qA[p][k] d)),
                summed over k in order in FP64, one rounding per operation.
 6. check    -- the exact squared error sum (x - xhat)^2 (FP64, on the
                returned dtype values) must be <= e2; if not, the block is
                encoded again at r + 1 (the paper's "test candidate sets until
                the tolerance is met"), and stored raw (values verbatim) once
                r would exceed rcap, or when a coefficient overflows int32.

So every block meets its e2 and the field meets sqrt(sum err) <= eps_t ||u||,
i.e. NRMSE <= eps_t, for every variable.  A block with a non-finite value is
raw.

Stream: the container of ``oracle.container`` with header flag bit 1; per
batch: ranks (u8, RAW = 255), steps (f64), qV planes, qA planes (zigzag
int32, four byte planes each, as in the absolute mode), then the raw blocks'
values in (t, p) order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import dls

TAIL_SHARE = 0.36      # the truncation tail may use 0.6^2 of the block's squared budget
STEP_SHARE = 0.4       # coefficient step d = 0.4 sqrt(e2 / (r M))
BASIS_BITS = 24        # qV = rint(V * 2^24)
RAW = 255              # rank byte of a block stored verbatim
QA_LIMIT = 2.0 ** 31


@dataclass
class L2Code:
    r: int                        # 0..W, or RAW
    step: float                   # d (0 when r is 0 or RAW)
    qV: np.ndarray                # int64 (W_b, r)
    qA: np.ndarray                # int64 (M_b, r)
    raw: Optional[np.ndarray]     # (W_b, M_b) storage dtype, for RAW
    err: float = 0.0              # sum (x - xhat)^2 of the stored result
    e2: float = 0.0               # the block's squared budget
    r0: int = 0                   # rank chosen from the eigenvalues, before the check
    lam: Optional[np.ndarray] = None
    V: Optional[np.ndarray] = None


def variable_budgets(field: np.ndarray, targets: Sequence[float]) -> np.ndarray:
    """c_v = (eps_t,v ||u_v||)^2 / K_v for every variable (Sec. 2.4, Eq. (4))."""
    c = []
    for v in range(field.shape[0]):
        x = field[v].astype(np.float64)
        x = x[np.isfinite(x)]
        norm2 = float(np.sum(x * x))
        c.append(float(targets[v]) ** 2 * norm2 / float(field[v].size))
    return np.array(c)


def block_budget(c_v: float, b: dls.Block) -> float:
    """e2 = c_v M_b W_b: the block's equal share of the squared budget."""
    return c_v * b.m * b.w


def first_rank(lam: np.ndarray, e2: float, rcap: int) -> int:
    """Step 3: the rank the eigenvalues ask for (0 when the block's energy
    fits the truncation share itself)."""
    tail = dls.tail_energies(lam)
    tau = TAIL_SHARE * e2
    if tail[0] <= tau:
        return 0
    for r in range(1, rcap + 1):
        if tail[r] <= tau:
            return r
    return rcap


def decode_block(r: int, step: float, qV: np.ndarray, qA: np.ndarray, raw, wb: int, m: int, dtype) -> np.ndarray:
    """Step 5: the decoder's reconstruction of one block."""
    if r == RAW:
        return np.asarray(raw, dtype=dtype).reshape(wb, m)
    acc = np.zeros((wb, m), np.float64)
    for k in range(r):
        vt = qV[:, k].astype(np.float64) * 2.0 ** -BASIS_BITS
        ck = qA[:, k].astype(np.float64) * step
        acc = acc + np.outer(vt, ck)
    return acc.astype(dtype)


def encode_block(xs: np.ndarray, e2: float, rcap: int, dtype) -> L2Code:
    """Steps 2-6 for one block X_b (W_b x M_b, storage dtype)."""
    wb, m = xs.shape
    x = xs.astype(np.float64)
    if not np.all(np.isfinite(x)):
        return L2Code(RAW, 0.0, np.zeros((wb, 0), np.int64), np.zeros((m, 0), np.int64), xs.copy())
    lam, V = dls.eig_desc(x @ x.T)
    r = first_rank(lam, e2, min(rcap, wb))
    r0 = r
    while True:
        if r == 0:
            if e2 <= 0.0 and np.any(x != 0.0):
                r = 1
                continue
            out = np.zeros((wb, m), dtype)
            err = float(np.sum((x - out.astype(np.float64)) ** 2))
            if err <= e2:
                return L2Code(0, 0.0, np.zeros((wb, 0), np.int64), np.zeros((m, 0), np.int64), None, err, e2, r0,
                              lam, V)
            r = 1
            continue
        if r > min(rcap, wb) or e2 <= 0.0:
            break
        step = STEP_SHARE * math.sqrt(e2 / (r * m))
        Vr = V[:, :r]
        qV = np.rint(Vr * 2.0 ** BASIS_BITS).astype(np.int64)
        A = x.T @ Vr
        qa = np.rint(A / step)
        if np.any(np.abs(qa) >= QA_LIMIT):
            break
        qA = qa.astype(np.int64)
        out = decode_block(r, step, qV, qA, None, wb, m, dtype)
        err = float(np.sum((x - out.astype(np.float64)) ** 2))
        if err <= e2:
            return L2Code(r, step, qV, qA, None, err, e2, r0, lam, V)
        r += 1
    return L2Code(RAW, 0.0, np.zeros((wb, 0), np.int64), np.zeros((m, 0), np.int64), xs.copy(), 0.0, e2, r0, lam, V)


@dataclass
class L2Encoded:
    params: dls.Params            # eps holds the targets eps_t,v
    blocks: List[dls.Block]
    codes: List[L2Code]
    split_bits: list
    budgets: np.ndarray           # c_v


def encode(field: np.ndarray, p: dls.Params) -> L2Encoded:
    """Alg. 1 steps 2-3 with the L2 tolerance, every block of the plan."""
    assert field.shape == (p.nvars, p.nt, p.nz, p.ny, p.nx)
    blocks, bits = dls.plan(field, p)
    c = variable_budgets(field, p.eps)
    rcap = p.resolved_rmax()
    codes = [encode_block(dls.gather(field, b), block_budget(c[b.var], b), rcap, p.np_dtype) for b in blocks]
    return L2Encoded(p, blocks, codes, bits, c)


def reconstruct(enc: L2Encoded) -> np.ndarray:
    p = enc.params
    out = np.zeros((p.nvars, p.nt, p.nz, p.ny, p.nx), dtype=p.np_dtype)
    for b, cd in zip(enc.blocks, enc.codes):
        dls.scatter(out, b, decode_block(cd.r, cd.step, cd.qV, cd.qA, cd.raw, b.w, b.m, p.np_dtype))
    return out


def nrmse_fraction(u: np.ndarray, uh: np.ndarray) -> float:
    """||u - uh|| / ||u|| over the finite values of u (the NRMSE of Sec. 2.4
    as a fraction)."""
    a = u.astype(np.float64)
    fin = np.isfinite(a)
    d = np.where(fin, a - uh.astype(np.float64), 0.0)
    return float(np.sqrt(np.sum(d * d)) / np.sqrt(np.sum(np.where(fin, a * a, 0.0))))


def compress(field: np.ndarray, p: dls.Params) -> bytes:
    from . import container
    return container.pack_l2(encode(field, p))


def decompress(buf: bytes) -> np.ndarray:
    from . import container
    return reconstruct(container.unpack_l2(buf))
