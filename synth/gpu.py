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

from . import spectrum_params

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
    return _lib


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
