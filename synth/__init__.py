"""Seeded synthetic input fields for the DLS block encoder.

This module holds only input generation: no step of the compression method
lives here.  Both the FP64 oracle tests and the GPU runs draw their inputs from
it, so the two sides always see identical bytes.

The paper evaluates on an LES of flow past a cylinder (Sec. 3), which is not
available; these generators stand in for it with fields of the same kind
(smooth, multi-scale, time-dependent, several variables):

* ``blobs2d``     -- moving Gaussian blobs plus white noise (2D, any dtype).
* ``spectrum``    -- random-phase Fourier modes with a k^(-5/3) amplitude
                     spectrum and exp(-0.02 t) decay (2D or 3D), optionally with
                     a per-mode temporal drift so that windows are not rank 1.

Field layout everywhere: ``F[var][t][z][y][x]`` (x fastest), numpy shape
``(nvars, nt, nz, ny, nx)``.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "blob_params",
    "blobs2d",
    "blobs2d_truncated",
    "spectrum_params",
    "spectrum",
    "range_of",
    "philox4x32",
    "philox_normal",
]


# --------------------------------------------------------------------------
# Gaussian blobs
# --------------------------------------------------------------------------
def blob_params(nx: int, ny: int, nblobs: int, seed: int):
    """Draw blob centres, widths and velocities.

    Draw order (PCG64 ``default_rng(seed)``), per blob: centre x ~ U[0,nx),
    centre y ~ U[0,ny), width ~ U[4,12], velocity x ~ U[-1,1], velocity y ~
    U[-1,1].  Returns float64 array of shape (nblobs, 5): cx, cy, w, vx, vy.
    The generator object is returned too so the caller can continue the
    stream (the noise is drawn right after the blobs).
    """
    rng = np.random.default_rng(seed)
    p = np.empty((nblobs, 5), dtype=np.float64)
    for b in range(nblobs):
        p[b, 0] = rng.uniform(0.0, nx)
        p[b, 1] = rng.uniform(0.0, ny)
        p[b, 2] = rng.uniform(4.0, 12.0)
        p[b, 3] = rng.uniform(-1.0, 1.0)
        p[b, 4] = rng.uniform(-1.0, 1.0)
    return p, rng


def blobs2d(nx: int = 64, ny: int = 64, nt: int = 32, nblobs: int = 4,
            seed: int = 1, noise_std: float = 1e-4,
            dtype=np.float64) -> np.ndarray:
    """2D scalar field of moving Gaussian blobs plus N(0, noise_std) noise.

    f(x, y, t) = sum_b exp(-|(x, y) - (c_b + v_b t)|^2 / (2 w_b^2)) + n(t, y, x)
    with integer cell coordinates x, y and t = 0..nt-1, amplitude 1,
    non-periodic.  The noise is drawn after the blob parameters from the same
    PCG64 stream, in [t][y][x] order.  Returns shape (1, nt, 1, ny, nx).
    """
    p, rng = blob_params(nx, ny, nblobs, seed)
    noise = rng.normal(0.0, noise_std, size=(nt, ny, nx))
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    f = np.zeros((nt, ny, nx), dtype=np.float64)
    for t in range(nt):
        acc = np.zeros((ny, nx), dtype=np.float64)
        for b in range(nblobs):
            cx = p[b, 0] + p[b, 3] * t
            cy = p[b, 1] + p[b, 4] * t
            w = p[b, 2]
            acc += np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * w * w))
        f[t] = acc
    f += noise
    return f.astype(dtype)[None, :, None, :, :]


def blobs2d_truncated(nx: int, ny: int, nt: int, nblobs: int, seed: int,
                      noise_std: float = 1e-4, trunc: float = 6.0,
                      dtype=np.float32) -> np.ndarray:
    """Large-domain variant of ``blobs2d`` that a GPU can generate quickly.

    Same blob parameters (``blob_params``), but each blob only contributes
    inside the box |x - cx_b(t)| <= trunc w_b, |y - cy_b(t)| <= trunc w_b
    (outside it the Gaussian is below exp(-18) ~ 1.5e-8, far under the noise),
    blobs are summed in index order, and the noise is counter-based:
    ``philox_normal(t*ny*nx + y*nx + x, seed, noise_std)``.  Evaluated in
    float64 and rounded once to ``dtype``.  Returns shape (1, nt, 1, ny, nx).
    """
    p, _ = blob_params(nx, ny, nblobs, seed)
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    out = np.empty((nt, ny, nx), dtype=dtype)
    for t in range(nt):
        acc = np.zeros((ny, nx), dtype=np.float64)
        for b in range(nblobs):
            cx = p[b, 0] + p[b, 3] * t
            cy = p[b, 1] + p[b, 4] * t
            w = p[b, 2]
            R = trunc * w
            inside = (np.abs(x - cx) <= R) & (np.abs(y - cy) <= R)
            g = np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * w * w))
            acc = acc + np.where(inside, g, 0.0)
        idx = (np.uint64(t) * np.uint64(ny * nx)
               + np.arange(ny * nx, dtype=np.uint64)).reshape(ny, nx)
        acc = acc + philox_normal(idx.ravel(), seed, noise_std).reshape(ny, nx)
        out[t] = acc.astype(dtype)
    return out[None, :, None]


# --------------------------------------------------------------------------
# Random-phase spectrum
# --------------------------------------------------------------------------
def spectrum_params(shape_zyx, nmodes: int, seed: int):
    """Draw integer wave vectors, phases and drift rates.

    Per axis of size n > 1 the wave number is uniform in {-K..K} with
    K = max(1, n // 16); axes of size 1 get 0.  The all-zero vector is
    redrawn.  Draw order (PCG64 ``default_rng(seed)``): for each mode the
    three components (x, y, z) then the phase ~ U[0, 2 pi); after all modes,
    the drift rates omega ~ U[0, 0.2] rad/step.
    Returns (k int64 (nmodes,3) as (kx,ky,kz), phi (nmodes,), omega (nmodes,)).
    """
    nz, ny, nx = shape_zyx
    kmax = [max(1, n // 16) if n > 1 else 0 for n in (nx, ny, nz)]
    rng = np.random.default_rng(seed)
    k = np.zeros((nmodes, 3), dtype=np.int64)
    phi = np.zeros(nmodes, dtype=np.float64)
    for j in range(nmodes):
        while True:
            kk = [int(rng.integers(-m, m + 1)) if m > 0 else 0 for m in kmax]
            if any(kk):
                break
        k[j] = kk
        phi[j] = rng.uniform(0.0, 2.0 * math.pi)
    omega = rng.uniform(0.0, 0.2, size=nmodes)
    return k, phi, omega


def spectrum(nx: int, ny: int, nz: int, nt: int, nmodes: int = 64,
             seed: int = 11, drift: bool = False, decay: float = 0.02,
             dtype=np.float32) -> np.ndarray:
    """One variable of the random-phase Fourier field.

    u(x, t) = sum_j |k_j|^(-5/3) cos(2 pi sum_d (k_jd x_d mod n_d) / n_d
                                       + phi_j [+ omega_j t]) * exp(-decay t)

    evaluated in float64 and rounded once to ``dtype``.  Without drift every
    time window of this field is exactly rank one in time (up to the final
    rounding).  Returns shape (1, nt, nz, ny, nx).
    """
    k, phi, omega = spectrum_params((nz, ny, nx), nmodes, seed)
    amp = np.linalg.norm(k.astype(np.float64), axis=1) ** (-5.0 / 3.0)
    ix = np.arange(nx, dtype=np.int64)
    iy = np.arange(ny, dtype=np.int64)
    iz = np.arange(nz, dtype=np.int64)
    out = np.empty((nt, nz, ny, nx), dtype=dtype)
    two_pi = 2.0 * math.pi

    def phase_of(j):
        px = (k[j, 0] * ix) % nx / nx
        py = (k[j, 1] * iy) % ny / ny
        pz = (k[j, 2] * iz) % nz / nz
        return two_pi * (pz[:, None, None] + py[None, :, None] + px[None, None, :])

    if not drift:
        base = np.zeros((nz, ny, nx), dtype=np.float64)
        for j in range(nmodes):
            base += amp[j] * np.cos(phase_of(j) + phi[j])
        for t in range(nt):
            out[t] = (base * math.exp(-decay * t)).astype(dtype)
    else:
        phases = [phase_of(j) + phi[j] for j in range(nmodes)]
        for t in range(nt):
            acc = np.zeros((nz, ny, nx), dtype=np.float64)
            for j in range(nmodes):
                acc += amp[j] * np.cos(phases[j] + omega[j] * t)
            out[t] = (acc * math.exp(-decay * t)).astype(dtype)
    return out[None]


def range_of(field: np.ndarray) -> np.ndarray:
    """Per-variable value range max - min of the stored values, as float64."""
    f = field.reshape(field.shape[0], -1)
    return (f.max(axis=1).astype(np.float64) - f.min(axis=1).astype(np.float64))


# --------------------------------------------------------------------------
# Counter-based normal noise (Philox4x32-10, Salmon et al., SC'11)
# --------------------------------------------------------------------------
_PHILOX_M0 = np.uint64(0xD2511F53)
_PHILOX_M1 = np.uint64(0xCD9E8D57)
_PHILOX_W0 = np.uint32(0x9E3779B9)
_PHILOX_W1 = np.uint32(0xBB67AE85)


def philox4x32(counter: np.ndarray, key0: int, key1: int) -> np.ndarray:
    """Philox4x32 with 10 rounds.

    ``counter`` is a uint32 array of shape (n, 4); returns uint32 (n, 4).
    Used where the GPU must draw the same random numbers as the host
    (large fields generated on the device).
    """
    c = counter.astype(np.uint32).copy()
    k0 = np.uint32(key0)
    k1 = np.uint32(key1)
    mask = np.uint64(0xFFFFFFFF)
    for _ in range(10):
        p0 = c[:, 0].astype(np.uint64) * _PHILOX_M0
        p1 = c[:, 2].astype(np.uint64) * _PHILOX_M1
        hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
        lo0 = (p0 & mask).astype(np.uint32)
        hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
        lo1 = (p1 & mask).astype(np.uint32)
        n0 = hi1 ^ c[:, 1] ^ k0
        n1 = lo1
        n2 = hi0 ^ c[:, 3] ^ k1
        n3 = lo0
        c = np.stack([n0, n1, n2, n3], axis=1)
        k0 = np.uint32((int(k0) + int(_PHILOX_W0)) & 0xFFFFFFFF)
        k1 = np.uint32((int(k1) + int(_PHILOX_W1)) & 0xFFFFFFFF)
    return c


def philox_normal(index: np.ndarray, seed: int, std: float) -> np.ndarray:
    """N(0, std) draws addressed by a global element index (uint64 array).

    Counter = (index low 32 bits, index high 32 bits, 0, 0), key = (seed,
    0x5EED).  Two uniforms u1 = (x0 + 1) 2^-32, u2 = x1 2^-32 feed one
    Box-Muller transform: std * sqrt(-2 ln u1) cos(2 pi u2), in float64.
    """
    idx = np.asarray(index, dtype=np.uint64)
    ctr = np.zeros((idx.size, 4), dtype=np.uint32)
    ctr[:, 0] = (idx & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    ctr[:, 1] = (idx >> np.uint64(32)).astype(np.uint32)
    r = philox4x32(ctr, seed & 0xFFFFFFFF, 0x5EED)
    u1 = (r[:, 0].astype(np.float64) + 1.0) * 2.0 ** -32
    u2 = r[:, 1].astype(np.float64) * 2.0 ** -32
    return std * np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)
