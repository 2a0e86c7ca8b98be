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


def projector_unique(lam: np.ndarray, r: int, limit: float = 1e-6) -> bool:
    """Reading R5: the rank-r subspace (and with it V_r V_r^T X) is unique
    when the relative gap (lam_r - lam_{r+1}) / lam_1 at r is at least 1e-6;
    below that several results are correct and only the bound judges."""
    lam = np.maximum(np.asarray(lam, dtype=np.float64), 0.0)
    nxt = lam[r] if r < lam.size else 0.0
    return (lam[r - 1] - nxt) >= limit * max(lam[0], 1e-300)


def projector_rel_err(A_gpu, V_gpu, A_or, V_or) -> float:
    """||V_g A_g^T - V_o A_o^T||_F / ||V_o A_o^T||_F: the rank-r reconstructions
    before quantization (unique when the kept and discarded spectra are
    separated, whatever the basis inside the kept subspace)."""
    Pg = V_gpu.astype(np.float64) @ A_gpu.astype(np.float64).T
    Po = V_or @ A_or.T
    return float(np.linalg.norm(Pg - Po) / max(np.linalg.norm(Po), 1e-300))
