"""Device-side generation of the large synthetic fields (harness only).

The field is written straight into a torch CUDA tensor by the generator
kernel in ``synth_kernels.hip``; the per-mode constants come from
``synth.spectrum_params`` on the host, exactly as the NumPy generator draws
them.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np
import torch

from . import blob_params, spectrum_params

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(_HERE, "libdls_synth.so")
_lib = None


def build(verbose: bool = False) -> str:
    cmd = [os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"), "--offload-arch=gfx950", "-O3", "-std=c++17",
           "-fPIC", "-shared", "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", os.path.join(_HERE, "synth_kernels.hip"), "-o", LIB + ".tmp"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("synth build failed:\n" + r.stdout)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError("libdls_synth.so is not built")
        _lib = ctypes.CDLL(LIB)
        _lib.synth_spectrum.argtypes = [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_int64] * 4 + \
            [ctypes.c_int] + [ctypes.c_void_p] * 5 + [ctypes.c_int, ctypes.c_void_p]
        _lib.synth_spectrum.restype = ctypes.c_int
        _lib.synth_blobs.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_double, ctypes.c_uint32, ctypes.c_double, ctypes.c_void_p]
        _lib.synth_blobs.restype = ctypes.c_int
    return _lib


def blobs_into(out: torch.Tensor, nblobs: int, seed: int, noise_std: float = 1e-4,
               trunc: float = 6.0) -> torch.Tensor:
    """Fill ``out`` (shape (nt, 1, ny, nx), CUDA) with ``synth.blobs2d_truncated``."""
    nt, nz, ny, nx = out.shape
    assert nz == 1
    p, _ = blob_params(nx, ny, nblobs, seed)
    # per 64x64 tile: every blob whose truncated box can reach the tile
    tiles_x, tiles_y = (nx + 63) // 64, (ny + 63) // 64
    R = trunc * p[:, 2]
    xs = np.stack([p[:, 0], p[:, 0] + p[:, 3] * (nt - 1)])
    ys = np.stack([p[:, 1], p[:, 1] + p[:, 4] * (nt - 1)])
    bx0 = np.clip(np.floor((xs.min(0) - R) / 64), 0, tiles_x - 1).astype(np.int64)
    bx1 = np.clip(np.floor((xs.max(0) + R) / 64), 0, tiles_x - 1).astype(np.int64)
    by0 = np.clip(np.floor((ys.min(0) - R) / 64), 0, tiles_y - 1).astype(np.int64)
    by1 = np.clip(np.floor((ys.max(0) + R) / 64), 0, tiles_y - 1).astype(np.int64)
    lists = [[] for _ in range(tiles_x * tiles_y)]
    for b in range(nblobs):
        for ty in range(by0[b], by1[b] + 1):
            for tx in range(bx0[b], bx1[b] + 1):
                lists[ty * tiles_x + tx].append(b)
    tstart = np.zeros(len(lists) + 1, np.int32)
    tstart[1:] = np.cumsum([len(l) for l in lists])
    tlist = np.array([b for l in lists for b in l] or [0], np.int32)
    dev = out.device
    tb = torch.from_numpy(np.ascontiguousarray(p.reshape(-1))).to(dev)
    ts = torch.from_numpy(tstart).to(dev)
    tl = torch.from_numpy(tlist).to(dev)
    st = torch.cuda.current_stream(dev).cuda_stream
    rc = _L().synth_blobs(ctypes.c_void_p(out.data_ptr()), 0 if out.dtype == torch.float32 else 1, nx, ny, nt,
                          ctypes.c_void_p(tb.data_ptr()), ctypes.c_void_p(ts.data_ptr()),
                          ctypes.c_void_p(tl.data_ptr()), trunc, seed & 0xFFFFFFFF, noise_std,
                          ctypes.c_void_p(st))
    if rc != 0:
        raise RuntimeError("synth_blobs failed: %d" % rc)
    torch.cuda.synchronize(dev)
    return out


def spectrum_into(out: torch.Tensor, seed: int, nmodes: int = 64, drift: bool = False,
                  decay: float = 0.02) -> torch.Tensor:
    """Fill ``out`` (shape (nt, nz, ny, nx), float32/float64, CUDA) with one
    variable of the random-phase spectrum field (same formula as
    ``synth.spectrum``)."""
    nt, nz, ny, nx = out.shape
    k, phi, omega = spectrum_params((nz, ny, nx), nmodes, seed)
    amp = np.linalg.norm(k.astype(np.float64), axis=1) ** (-5.0 / 3.0)
    dec = np.array([math.exp(-decay * t) for t in range(nt)], dtype=np.float64)
    dev = out.device
    tk = torch.from_numpy(np.ascontiguousarray(k.reshape(-1))).to(dev)
    ta = torch.from_numpy(amp).to(dev)
    tp = torch.from_numpy(phi).to(dev)
    to = torch.from_numpy(omega).to(dev)
    td = torch.from_numpy(dec).to(dev)
    st = torch.cuda.current_stream(dev).cuda_stream
    rc = _L().synth_spectrum(ctypes.c_void_p(out.data_ptr()), 0 if out.dtype == torch.float32 else 1,
                             nx, ny, nz, nt, nmodes, ctypes.c_void_p(tk.data_ptr()),
                             ctypes.c_void_p(ta.data_ptr()), ctypes.c_void_p(tp.data_ptr()),
                             ctypes.c_void_p(to.data_ptr()), ctypes.c_void_p(td.data_ptr()),
                             1 if drift else 0, ctypes.c_void_p(st))
    if rc != 0:
        raise RuntimeError("synth_spectrum failed: %d" % rc)
    torch.cuda.synchronize(dev)
    return out
