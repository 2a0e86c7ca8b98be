"""FP64 oracle of the learned warm start (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
module; the product path never does.

The paper learns its basis by an SVD of sampled patches (Sec. 2.3, Eq. (2));
the learned warm start replaces the per-block eigensolve by a few steps of
subspace iteration started from a basis that a small network predicts from
per-block statistics.  Whatever the network predicts, the plain method judges
the result: the rank is the smallest r whose discarded energy meets the local
tolerance (Sec. 2.4 Eq. (4), Alg. 1 step 3), computed exactly for the basis
actually used, and the residual quantization keeps the pointwise bound.

Contents:
  features(x, px, py, pz, eps)      -- 16 moments + 8 x 8 pooled time-mean
  Net / forward / backward / loss   -- 80 -> 128 -> 128 -> 272 MLP, ReLU
  adam_step                         -- Adam (Kingma & Ba, 2015)
  warm_start_eig(G, V0, rhat, ...)  -- subspace iteration + Rayleigh-Ritz +
                                       acceptance with the downward check
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import dls

NFEAT = 80
NMOM = 16
HID = 128
NOUT = 16 + 256
WMAX = 16


# --------------------------------------------------------------------------
# Features
# --------------------------------------------------------------------------
def moments(x: np.ndarray, px: int, py: int, pz: int, eps: float) -> np.ndarray:
    """The 16 per-block statistics, FP64, before z-scoring.

    x is X_b (W x M), p = (k*Py + j)*Px + i.  Differences are divided by the
    block standard deviation (0 when it vanishes):
      0 mean, 1 std, 2 min, 3 max, 4 skewness, 5 excess kurtosis,
      6 mean|dt|/std, 7 std(dt)/std, 8 mean|dx|/std, 9 mean|dy|/std,
      10 lag-1 and 11 lag-2 temporal autocorrelation,
      12 log10(mean(x^2)/eps^2), 13 log10(std/eps),
      14 time-mean energy fraction sum_p (sum_t x)^2 / (W sum x^2),
      15 log2(M).
    """
    x = x.astype(np.float64)
    w, m = x.shape
    mu = float(np.mean(x))
    var = float(np.mean((x - mu) ** 2))
    sd = math.sqrt(var)
    f = np.zeros(NMOM)
    f[0], f[1], f[2], f[3] = mu, sd, float(x.min()), float(x.max())
    inv = 1.0 / sd if sd > 0 else 0.0
    if sd > 0:
        f[4] = float(np.mean((x - mu) ** 3)) / sd ** 3
        f[5] = float(np.mean((x - mu) ** 4)) / sd ** 4 - 3.0
    if w > 1:
        d = x[1:] - x[:-1]
        f[6] = float(np.mean(np.abs(d))) * inv
        f[7] = float(np.std(d)) * inv
    cube = x.reshape(w, pz, py, px)
    if px > 1:
        f[8] = float(np.mean(np.abs(cube[..., 1:] - cube[..., :-1]))) * inv
    if py > 1:
        f[9] = float(np.mean(np.abs(cube[:, :, 1:, :] - cube[:, :, :-1, :]))) * inv
    if w > 1 and sd > 0:
        f[10] = float(np.mean((x[1:] - mu) * (x[:-1] - mu))) / var
    if w > 2 and sd > 0:
        f[11] = float(np.mean((x[2:] - mu) * (x[:-2] - mu))) / var
    ms = float(np.mean(x * x))
    f[12] = math.log10(max(ms / (eps * eps), 1e-30))
    f[13] = math.log10(max(sd / eps, 1e-15))
    tot = float(np.sum(x * x))
    f[14] = float(np.sum(np.sum(x, axis=0) ** 2)) / (w * tot) if tot > 0 else 0.0
    f[15] = math.log2(m)
    return f


def pooled(x: np.ndarray, px: int, py: int, pz: int) -> np.ndarray:
    """8 x 8 pooled time-mean image, normalised by the block mean and std.

    Y = mean over t and z; cell (b, a) averages rows j with floor(8 j / Py) = b
    and columns i with floor(8 i / Px) = a, or, when that set is empty
    (edge < 8), the single row floor(b Py / 8) / column floor(a Px / 8).
    Returned in [b][a] order as 64 values (Y - mean) / std (0 if std = 0).
    """
    x = x.astype(np.float64)
    w, m = x.shape
    y = x.reshape(w, pz, py, px).mean(axis=(0, 1))
    mu = float(np.mean(x))
    sd = float(np.sqrt(np.mean((x - mu) ** 2)))
    out = np.zeros((8, 8))
    for b in range(8):
        rows = [j for j in range(py) if (8 * j) // py == b] or [(b * py) // 8]
        for a in range(8):
            cols = [i for i in range(px) if (8 * i) // px == a] or [(a * px) // 8]
            out[b, a] = float(np.mean(y[np.ix_(rows, cols)]))
    if sd > 0:
        out = (out - mu) / sd
    else:
        out[:] = 0.0
    return out.ravel()


def features(x: np.ndarray, px: int, py: int, pz: int, eps: float) -> np.ndarray:
    """80 raw inputs: 16 moments then 64 pooled values."""
    return np.concatenate([moments(x, px, py, pz, eps), pooled(x, px, py, pz)])


# --------------------------------------------------------------------------
# Network
# --------------------------------------------------------------------------
@dataclass
class Net:
    W1: np.ndarray   # (80, 128)
    b1: np.ndarray
    W2: np.ndarray   # (128, 128)
    b2: np.ndarray
    W3: np.ndarray   # (128, 272)
    b3: np.ndarray
    mom_mean: np.ndarray   # (16,) z-scoring of the moments
    mom_std: np.ndarray

    def params(self):
        return [self.W1, self.b1, self.W2, self.b2, self.W3, self.b3]


def init_net(seed: int) -> Net:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, PCG64 draws in
    the order W1, W2, W3; identity z-scoring until statistics are set."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0.0, math.sqrt(2.0 / NFEAT), size=(NFEAT, HID))
    W2 = rng.normal(0.0, math.sqrt(2.0 / HID), size=(HID, HID))
    W3 = rng.normal(0.0, math.sqrt(2.0 / HID), size=(HID, NOUT))
    return Net(W1, np.zeros(HID), W2, np.zeros(HID), W3, np.zeros(NOUT),
               np.zeros(NMOM), np.ones(NMOM))


def normalise(net: Net, raw: np.ndarray) -> np.ndarray:
    """z-score the 16 moments; the pooled part is already normalised."""
    z = np.array(raw, dtype=np.float64, copy=True)
    z[..., :NMOM] = (z[..., :NMOM] - net.mom_mean) / net.mom_std
    return z


def bf16(a: np.ndarray) -> np.ndarray:
    """Round float64 values to bfloat16 (round to nearest even via float32)."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(net: Net, z: np.ndarray, round_bf16: bool = False):
    """Activations of a batch z (B, 80): returns (h1, h2, out).

    With round_bf16 the operands of each product (inputs and weights) are
    rounded to bfloat16 first, as the matrix cores consume them."""
    r = bf16 if round_bf16 else (lambda a: a)
    a1 = r(z) @ r(net.W1) + net.b1
    h1 = np.maximum(a1, 0.0)
    a2 = r(h1) @ r(net.W2) + net.b2
    h2 = np.maximum(a2, 0.0)
    out = r(h2) @ r(net.W3) + net.b3
    return h1, h2, out


def loss_and_grad_out(out: np.ndarray, rank: np.ndarray, basis: np.ndarray, wb: np.ndarray):
    """Batch-mean loss CE(logits, r-1) + masked MSE of the basis, and dL/dout.

    out (B, 272): 16 rank logits then V0[k][t] (mode-major, k, t < 16).
    rank (B,) in [1, 16]; basis (B, 16, 16) target [k][t]; wb (B,) window
    lengths.  The MSE averages over the entries k < r, t < W_b.
    """
    B = out.shape[0]
    logits = out[:, :16]
    mx = logits.max(axis=1, keepdims=True)
    e = np.exp(logits - mx)
    p = e / e.sum(axis=1, keepdims=True)
    ce = -np.log(p[np.arange(B), rank - 1])
    g = np.zeros_like(out)
    g[:, :16] = p
    g[np.arange(B), rank - 1] -= 1.0
    pred = out[:, 16:].reshape(B, 16, 16)
    k = np.arange(16)[None, :, None]
    t = np.arange(16)[None, None, :]
    mask = (k < rank[:, None, None]) & (t < wb[:, None, None])
    cnt = np.maximum(mask.sum(axis=(1, 2)), 1)
    diff = np.where(mask, pred - basis, 0.0)
    mse = (diff ** 2).sum(axis=(1, 2)) / cnt
    g[:, 16:] = (2.0 * diff / cnt[:, None, None]).reshape(B, 256)
    return float(np.mean(ce + mse)), g / B


def backward(net: Net, z, h1, h2, gout, round_bf16: bool = False):
    """Gradients of the loss w.r.t. (W1, b1, W2, b2, W3, b3)."""
    r = bf16 if round_bf16 else (lambda a: a)
    dW3 = r(h2).T @ r(gout)
    db3 = gout.sum(axis=0)
    dh2 = (r(gout) @ r(net.W3).T) * (h2 > 0)
    dW2 = r(h1).T @ r(dh2)
    db2 = dh2.sum(axis=0)
    dh1 = (r(dh2) @ r(net.W2).T) * (h1 > 0)
    dW1 = r(z).T @ r(dh1)
    db1 = dh1.sum(axis=0)
    return [dW1, db1, dW2, db2, dW3, db3]


def adam_step(params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam update; `step` counts from 1."""
    for P, G, M, V in zip(params, grads, m, v):
        M *= b1
        M += (1 - b1) * G
        V *= b2
        V += (1 - b2) * G * G
        mh = M / (1 - b1 ** step)
        vh = V / (1 - b2 ** step)
        P -= lr * mh / (np.sqrt(vh) + eps)


# --------------------------------------------------------------------------
# Warm-started eigensolve
# --------------------------------------------------------------------------
def mgs(Y: np.ndarray) -> np.ndarray:
    """Modified Gram-Schmidt, twice; a column whose remainder collapses below
    1e-12 of its norm is replaced by the unit vector e_j (smallest j) that
    keeps the set independent."""
    w, r = Y.shape
    Q = np.zeros((w, r))
    for k in range(r):
        y = Y[:, k].copy()
        n0 = float(np.linalg.norm(y))
        for _ in range(2):
            for j in range(k):
                y -= (Q[:, j] @ y) * Q[:, j]
        n = float(np.linalg.norm(y))
        if not (n > 1e-12 * n0) or n0 == 0.0:
            for j in range(w):
                y = np.zeros(w)
                y[j] = 1.0
                for _ in range(2):
                    for i in range(k):
                        y -= (Q[:, i] @ y) * Q[:, i]
                n = float(np.linalg.norm(y))
                if n > 0.5:
                    break
        Q[:, k] = y / n
    return Q


def warm_start_eig(G: np.ndarray, V0: np.ndarray, tau: float, iters: int = 2):
    """Subspace iteration from V0, Rayleigh-Ritz, acceptance.

    Q = mgs(V0); `iters` times Q = mgs(G Q); H = Q^T G Q = U diag(theta) U^T
    (theta descending); Ritz vectors Z = Q U.  For the basis Z_r the
    discarded energy is exactly E(r) = trace(G) - sum_{k<=r} theta_k.  The
    accepted rank is the smallest r <= rhat with E(r) <= tau (this includes
    the downward check); if E(rhat) > tau the warm start is rejected and the
    caller falls back to the full eigensolve.
    Returns (accepted, r, theta, Z) with canonical signs on Z.
    """
    Q = mgs(V0)
    for _ in range(iters):
        Q = mgs(G @ Q)
    H = Q.T @ G @ Q
    H = 0.5 * (H + H.T)
    th, U = np.linalg.eigh(H)
    order = np.argsort(-th, kind="stable")
    th = th[order]
    Z = dls.canonical_signs(Q @ U[:, order])
    tr = float(np.trace(G))
    rhat = V0.shape[1]
    for r in range(1, rhat + 1):
        if tr - float(np.sum(th[:r])) <= tau:
            return True, r, th, Z
    return False, rhat, th, Z


WARM_MAX = 8      # most columns the warm start iterates; larger predictions fall back
WARM_MAX_POINTS = 256    # larger blocks take the plain eigensolve directly
RETRY_EXTRA = 4   # columns added by the second attempt
RETRY_ITERS = 2   # subspace iterations added by the second attempt


def encode_block_learned(xs: np.ndarray, eps: float, rcap: int, dtype, rhat: int, V0: np.ndarray,
                         iters: int = 2, bf16_gram: bool = False):
    """encode_block with the warm-started eigensolve.

    V0 holds the network's starting columns (W x 16, or at least as many
    columns as an attempt uses).  Attempt 1 iterates the first rhat columns
    `iters` times; if it is rejected, attempt 2 iterates the first
    min(rhat + RETRY_EXTRA, WARM_MAX, cap) columns `iters + RETRY_ITERS`
    times (only when that is more columns).  An attempt with more than
    WARM_MAX columns is not made.  If no attempt is accepted the block takes
    the plain eigensolve.  With bf16_gram the Gram matrix is formed from the
    bfloat16-rounded snapshots, as in dls.encode_block (mixed precision: the
    acceptance test then sees that Gram).  Returns (BlockCode, accepted)."""
    wb, m = xs.shape
    x = xs.astype(np.float64)
    if not np.all(np.isfinite(x)):
        return dls._raw_block(xs), False
    if m > WARM_MAX_POINTS:
        return dls.encode_block(xs, eps, rcap, dtype, bf16_gram), False
    xg = dls.round_bf16(x) if bf16_gram else x
    G = xg @ xg.T
    tau = dls.KAPPA * eps * eps * m * wb
    cap = min(rcap, wb, m)
    rhat = max(1, min(rhat, cap))
    attempts = [(rhat, iters)]
    r2 = min(rhat + RETRY_EXTRA, WARM_MAX, cap)
    if r2 > rhat:
        attempts.append((r2, iters + RETRY_ITERS))
    for k, it in attempts:
        if k > WARM_MAX:
            break
        ok, r, th, Z = warm_start_eig(G, V0[:wb, :k], tau, it)
        if ok:
            return dls.encode_with_basis(xs, eps, Z[:, :r], np.maximum(th[:r], 0.0), tau, dtype), True
    return dls.encode_block(xs, eps, rcap, dtype, bf16_gram), False
