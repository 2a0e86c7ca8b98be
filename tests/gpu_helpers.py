"""Shared helpers of the GPU tests: run the HIP path through the C ABI and
fetch its per-block diagnostics; compare with the oracle."""
from __future__ import annotations

import numpy as np
import torch

import paper_2601_20113_amd as dls
from oracle import container, dls as odls


def to_lib_params(p: odls.Params, precision="fp32") -> dls.Params:
    return dls.Params(nx=p.nx, ny=p.ny, nz=p.nz, nt=p.nt, nvars=p.nvars, dtype=p.dtype,
                      px=p.px, py=p.py, pz=p.pz, window=p.window, eps=list(p.eps),
                      pmin=p.pmin, r_max=p.r_max, precision=precision, adaptive=p.adaptive)


class GpuRun:
    """One dls_encode + dls_finalize, with the diagnostics copied to host."""

    def __init__(self, field: np.ndarray, p: odls.Params, precision="fp32", enc=None):
        self.p = p
        lp = to_lib_params(p, precision)
        t = torch.from_numpy(field).cuda()
        self.enc = enc or dls.Encoder()
        self.enc.encode(t, lp, keep_coef=True)
        torch.cuda.synchronize()
        inf = self.enc.info()
        nb, wp = inf.nblocks, inf.wpad
        self.nb, self.wp = nb, wp
        self.rank = dls.d2h(inf.d_rank, nb).copy()
        self.lam = dls.d2h(inf.d_lam, nb * wp * 8).view(np.float64).reshape(nb, wp).copy()
        self.basis = dls.d2h(inf.d_basis, nb * wp * wp * 8).view(np.float64).reshape(nb, wp, wp).copy()
        self.qa_off = dls.d2h(inf.d_qa_off, nb * 8).view(np.int64).copy()
        self.coef = dls.d2h(inf.d_coef, inf.qa_bytes).view(np.float32).copy() if inf.qa_bytes else np.zeros(0, np.float32)
        self.nescapes, self.nraw, self.gpu_ms = inf.nescapes, inf.nraw, inf.gpu_ms
        self.stream = self.enc.finalize()
        self.field_t = t

    def coef_of(self, b: int, m: int) -> np.ndarray:
        r = int(self.rank[b])
        o = int(self.qa_off[b]) // 4
        return self.coef[o:o + r * m].reshape(r, m).T  # (M, r)

    def basis_of(self, b: int, w: int) -> np.ndarray:
        return self.basis[b][:, :w].T  # (W, wp): column k = mode k


def predicted_coef_err(lam: np.ndarray, r: int, eta: float = 2.0 ** -23) -> float:
    """First-order error of the kept coefficients when the Gram carries
    perturbations of size eta * lam_1 (an FP32-accurate Gram).

    dA_k = X^T dv_k with dv_k = sum_{j != k} (v_j^T dG v_k) / (lam_k - lam_j) v_j
    and ||X^T v_j|| = sqrt(lam_j), so ||dA_k||^2 <= sum_j lam_j (eta lam_1)^2 /
    (lam_k - lam_j)^2; returned relative to ||A||_F = sqrt(sum_{k<=r} lam_k).
    """
    lam = np.maximum(np.asarray(lam, dtype=np.float64), 0.0)
    l1 = max(lam[0], 1e-300)
    tot = 0.0
    for k in range(r):
        d = lam[k] - lam
        d[k] = np.inf
        d = np.where(np.abs(d) < 1e-300, 1e-300, d)
        tot += float(np.sum(lam * (eta * l1) ** 2 / d ** 2))
    return float(np.sqrt(tot) / np.sqrt(max(np.sum(lam[:r]), 1e-300)))


def gap_qualified(lam: np.ndarray, r: int, limit: float = 1e-6) -> bool:
    """The kept subspace is well separated: predicted FP32 error <= limit."""
    return predicted_coef_err(lam, r) <= limit


def coef_rel_err(A_gpu, V_gpu, A_or, V_or) -> float:
    """||A_gpu - A_or||_F / ||A_or||_F after per-mode sign alignment."""
    s = np.sign(np.sum(V_gpu * V_or, axis=0))
    s[s == 0] = 1.0
    d = A_gpu.astype(np.float64) * s[None, :] - A_or
    return float(np.linalg.norm(d) / max(np.linalg.norm(A_or), 1e-300))


U32 = 2.0 ** -24
GAMMA64 = 64 * U32 / (1 - 64 * U32)   # FP32 accumulation of a 64-point chunk


def projector_tol(lam: np.ndarray, r: int, w: int, energy_ratio=None):
    """Bound on ||P_gpu X - P_or X||_F / ||P_or X||_F for the rank-r
    reconstruction P X = V_r V_r^T X when the Gram is formed from FP32 (or
    bf16) products accumulated in FP32 over 64-point chunks; None when the
    rank-r subspace is not determined (reading R5: several results correct).

    Each Gram entry is off by at most GAMMA64 sqrt(G_aa G_bb) (Cauchy-Schwarz
    on the chunk's products), so ||dG||_2 <= ||dG||_F <= GAMMA64 W trace(G).
    Davis-Kahan: the sine of the angle between the exact and the perturbed
    rank-r subspaces is at most ||dG|| / (lam_r - lam_{r+1} - ||dG||), and
    ||(P_g - P_o) X||_F <= sqrt(2) sin(theta) ||X||_F.  Relative to ||P_o X||_F
    = sqrt(sum_{k<=r} lam_k) (or sqrt(trace / energy_ratio) given), plus 1e-6
    for the FP32 projection itself.  Unlike the coefficients, the projector
    shows a rotation of even the dominant mode at full weight, which an FP32
    Gram makes of order 1e-5."""
    lam = np.maximum(np.asarray(lam, dtype=np.float64), 0.0)
    tr = float(np.sum(lam))
    if not tr > 0.0:
        return None
    dg = GAMMA64 * w * tr
    nxt = lam[r] if r < lam.size else 0.0
    gap = lam[r - 1] - nxt - dg
    if not gap > 0.0:
        return None
    sin = dg / gap
    ratio = energy_ratio if energy_ratio is not None else tr / max(float(np.sum(lam[:r])), 1e-300)
    return float(np.sqrt(2.0) * sin * np.sqrt(ratio) + 1e-6)


def projector_rel_err(A_gpu, V_gpu, A_or, V_or) -> float:
    """||V_g A_g^T - V_o A_o^T||_F / ||V_o A_o^T||_F: the rank-r reconstructions
    before quantization (unique when the kept and discarded spectra are
    separated, whatever the basis inside the kept subspace)."""
    Pg = V_gpu.astype(np.float64) @ A_gpu.astype(np.float64).T
    Po = V_or @ A_or.T
    return float(np.linalg.norm(Pg - Po) / max(np.linalg.norm(Po), 1e-300))
