"""Python binding of libdls (the MI355X DLS encoder / decoder).

Argument marshalling only: every step of compression and decompression runs
in the library's HIP kernels and host code.  PyTorch supplies device memory
and streams.  Importing torch first makes the library share torch's HIP
runtime.

    import paper_2601_20113_amd as dls
    p = dls.Params(nx=64, ny=64, nz=1, nt=32, nvars=1, dtype="f64",
                   px=8, py=8, pz=1, window=16, eps=[1e-3])
    buf = dls.compress(field_cuda_tensor, p)       # bytes
    out = dls.decompress(buf)                      # cuda tensor
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field as dc_field
from typing import Optional, Sequence

import torch  # noqa: F401  (load torch's HIP runtime before libdls)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdls.so")

DLS_OK, DLS_EINVAL, DLS_ENOMEM, DLS_EDEVICE, DLS_ECORRUPT, DLS_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
DLS_F32, DLS_F64 = 0, 1
DLS_PREC_FP32, DLS_PREC_BF16 = 0, 1
DLS_PERSISTENT = 4
DLS_ADAPTIVE = 1
DLS_LEARNED = 2
DLS_L2 = 8
DLS_GLOBAL = 16
BASIS_KINDS = {"svd": 0, "cosine": 1, "random": 2}
NPARAM = 61968
WARM_MAX_POINTS = 256   # the warm start applies to blocks of at most this many points

EXPORTS = ["dls_ctx_create", "dls_ctx_destroy", "dls_encode", "dls_encode_info_get", "dls_range",
           "dls_finalize", "dls_compress", "dls_query", "dls_decompress", "dls_stats",
           "dls_free", "dls_last_error", "dls_model_create", "dls_model_destroy", "dls_model_set",
           "dls_model_get", "dls_model_forward", "dls_model_grad", "dls_model_train_step",
           "dls_features", "dls_ctx_set_model", "dls_decode", "dls_range_noalloc",
           "dls_ctx_set_jacobi_sweeps", "dls_ctx_set_graphs", "dls_ctx_set_launch"]


class DlsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("dls status %d: %s" % (status, msg))
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("nvars", ctypes.c_int32),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("nt", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("px", ctypes.c_int32), ("py", ctypes.c_int32), ("pz", ctypes.c_int32),
                ("pmin", ctypes.c_int32), ("window", ctypes.c_int32), ("r_max", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("abs_eps", ctypes.POINTER(ctypes.c_double)), ("basis", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("model", ctypes.c_void_p), ("warm_iters", ctypes.c_int32),
                ("rank_margin", ctypes.c_int32)]


class _EncodeInfo(ctypes.Structure):
    _fields_ = [("nblocks", ctypes.c_int64), ("nescapes", ctypes.c_int64), ("nraw", ctypes.c_int64),
                ("wpad", ctypes.c_int64), ("d_rank", ctypes.c_void_p), ("d_lam", ctypes.c_void_p),
                ("d_basis", ctypes.c_void_p), ("d_desc", ctypes.c_void_p),
                ("qa_bytes", ctypes.c_int64), ("codes_bytes", ctypes.c_int64),
                ("d_qa", ctypes.c_void_p), ("d_codes", ctypes.c_void_p),
                ("d_qa_off", ctypes.c_void_p), ("d_code_off", ctypes.c_void_p),
                ("d_coef", ctypes.c_void_p), ("nwarm_accept", ctypes.c_int64),
                ("nwarm_reject", ctypes.c_int64), ("gpu_ms", ctypes.c_double),
                ("stage_ms", ctypes.c_double * 5), ("nfast_accept", ctypes.c_int64),
                ("ndeferred", ctypes.c_int64), ("launch_mode", ctypes.c_int32),
                ("jacobi_sweeps", ctypes.c_int64), ("jacobi_unconverged", ctypes.c_int64),
                ("jacobi_ms", ctypes.c_double), ("fused_ms", ctypes.c_double),
                ("npredicted_deferred", ctypes.c_int64), ("npruned", ctypes.c_int64),
                ("fused_declined", ctypes.c_int32), ("l2_passes", ctypes.c_int32)]


class _StreamStats(ctypes.Structure):
    _fields_ = [("nblocks", ctypes.c_int64), ("nbatches", ctypes.c_int64), ("nraw", ctypes.c_int64),
                ("nescapes", ctypes.c_int64), ("rank_hist", ctypes.c_int64 * 33),
                ("payload_bytes", ctypes.c_int64), ("stream_bytes", ctypes.c_int64)]


_lib = None


def lib():
    """The loaded libdls; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libdls.so is not built (run __graft_entry__.build() or "
                              "python -m paper_2601_20113_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        c_void_pp = ctypes.POINTER(ctypes.c_void_p)
        L.dls_ctx_create.argtypes = [ctypes.c_int, c_void_pp]
        L.dls_ctx_destroy.argtypes = [ctypes.c_void_p]
        L.dls_ctx_destroy.restype = None
        L.dls_ctx_set_jacobi_sweeps.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.dls_ctx_set_graphs.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.dls_ctx_set_launch.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.dls_encode.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_Params),
                                 ctypes.c_void_p, ctypes.c_int]
        L.dls_encode_info_get.argtypes = [ctypes.c_void_p, ctypes.POINTER(_EncodeInfo)]
        L.dls_finalize.argtypes = [ctypes.c_void_p, c_void_pp, ctypes.POINTER(ctypes.c_size_t)]
        L.dls_compress.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Params), ctypes.c_void_p,
                                   c_void_pp, ctypes.POINTER(ctypes.c_size_t)]
        L.dls_query.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(_Params),
                                ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                ctypes.POINTER(ctypes.c_int64)]
        L.dls_decompress.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]
        L.dls_stats.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(_StreamStats)]
        L.dls_range.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.dls_range_noalloc.argtypes = L.dls_range.argtypes
        vp = ctypes.c_void_p
        L.dls_model_create.argtypes = [ctypes.c_int, c_void_pp]
        L.dls_model_destroy.argtypes = [vp]
        L.dls_model_destroy.restype = None
        L.dls_model_set.argtypes = [vp, vp, vp]
        L.dls_model_get.argtypes = [vp, vp, vp]
        L.dls_model_forward.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int, vp, vp]
        L.dls_model_grad.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int64, ctypes.c_int, vp,
                                     ctypes.POINTER(ctypes.c_float), vp]
        L.dls_model_train_step.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int64, ctypes.c_float, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_float), vp]
        L.dls_features.argtypes = [vp, vp, ctypes.c_size_t, vp, ctypes.c_size_t, vp]
        L.dls_decode.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.dls_ctx_set_model.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int]
        L.dls_free.argtypes = [ctypes.c_void_p]
        L.dls_free.restype = None
        L.dls_last_error.restype = ctypes.c_char_p
        for name in ("dls_model_create", "dls_model_set", "dls_model_get", "dls_model_forward", "dls_model_grad",
                     "dls_model_train_step", "dls_features", "dls_ctx_set_model", "dls_decode",
                     "dls_ctx_create", "dls_encode", "dls_encode_info_get", "dls_finalize", "dls_range",
                     "dls_compress", "dls_query", "dls_decompress", "dls_stats", "dls_range_noalloc"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != DLS_OK:
        raise DlsError(status, lib().dls_last_error().decode(errors="replace"))


@dataclass
class Params:
    """Problem statement: grid, patch and window sizes, absolute bounds."""
    nx: int
    ny: int
    nz: int
    nt: int
    nvars: int
    dtype: str            # "f32" | "f64"
    px: int
    py: int
    pz: int
    window: int
    eps: Sequence[float]
    pmin: int = 0
    r_max: int = 0
    precision: str = "fp32"   # "fp32" | "bf16"
    adaptive: bool = False
    learned: bool = False
    persistent: bool = False  # device-driven (batched) encode launch
    l2: bool = False          # L2 / NRMSE-bounded mode: eps holds the NRMSE targets (fractions)
    global_basis: bool = False  # the paper's global-basis method (window 1, eps = NRMSE targets)
    basis: str = "svd"        # global basis: "svd" | "cosine" | "random"
    seed: int = 0             # global basis: state of the learning draws
    model: object = None      # dls_compress with learned: the warm-start Model
    warm_iters: int = 0       # with model: 0 -> 2
    rank_margin: int = 1      # with model
    _keep: list = dc_field(default_factory=list, repr=False)

    def to_c(self) -> _Params:
        arr = (ctypes.c_double * len(self.eps))(*[float(e) for e in self.eps])
        self._keep = [arr]
        return _Params(ctypes.sizeof(_Params), self.nvars, self.nx, self.ny, self.nz, self.nt,
                       DLS_F32 if self.dtype == "f32" else DLS_F64, self.px, self.py, self.pz,
                       self.pmin, self.window, self.r_max,
                       DLS_PREC_BF16 if self.precision == "bf16" else DLS_PREC_FP32,
                       (DLS_ADAPTIVE if self.adaptive else 0) | (DLS_LEARNED if self.learned else 0)
                       | (DLS_PERSISTENT if self.persistent else 0) | (DLS_L2 if self.l2 else 0)
                       | (DLS_GLOBAL if self.global_basis else 0),
                       ctypes.cast(arr, ctypes.POINTER(ctypes.c_double)), BASIS_KINDS[self.basis],
                       int(self.seed) & ((1 << 64) - 1),
                       self.model._h if self.model is not None else None, self.warm_iters, self.rank_margin)

    @property
    def torch_dtype(self):
        return torch.float32 if self.dtype == "f32" else torch.float64

    @property
    def shape(self):
        return (self.nvars, self.nt, self.nz, self.ny, self.nx)


def _stream_handle(stream) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _take_bytes(out: ctypes.c_void_p, n: ctypes.c_size_t) -> bytes:
    """Copy a library-allocated host buffer of n bytes into a bytes object
    (ctypes.string_at takes a C int length, so streams of 2 GiB and more need
    this route)."""
    if n.value == 0:
        return b""
    return (ctypes.c_char * n.value).from_address(out.value).raw


def _check_field(t: torch.Tensor, p: Params):
    if not t.is_cuda:
        raise ValueError("field must be a device tensor")
    if not t.is_contiguous():
        raise ValueError("field must be contiguous")
    if t.dtype != p.torch_dtype or tuple(t.shape) != p.shape:
        raise ValueError("field dtype/shape %s %s does not match params %s %s"
                         % (t.dtype, tuple(t.shape), p.torch_dtype, p.shape))


class Encoder:
    """A reusable encoder context (device workspace lives here)."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().dls_ctx_create(device, ctypes.byref(h)))
        self._h = h

    def close(self):
        if self._h:
            lib().dls_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def encode(self, field: torch.Tensor, p: Params, stream=None, keep_coef: bool = False):
        _check_field(field, p)
        cp = p.to_c()
        self._last_params = None
        _check(lib().dls_encode(self._h, ctypes.c_void_p(field.data_ptr()), ctypes.byref(cp),
                                _stream_handle(stream), 1 if keep_coef else 0))
        self._last_params = p

    def set_model(self, model: "Model", iters: int = 2, margin: int = 1):
        """Attach a model for encodes with learned=True (None detaches)."""
        self._model = model
        _check(lib().dls_ctx_set_model(self._h, model._h if model is not None else None, iters, margin))

    def set_launch(self, device_driven_max_items: int):
        """Plans of at most this many slices take the device-driven encode."""
        _check(lib().dls_ctx_set_launch(self._h, ctypes.c_int64(int(device_driven_max_items))))

    def set_graphs(self, enabled: bool):
        """Graph replay of the global basis's Jacobi sweeps (default on)."""
        _check(lib().dls_ctx_set_graphs(self._h, int(enabled)))

    def set_jacobi_sweeps(self, max_sweeps: int):
        """Cap the plain eigensolve's sweeps for later encodes (default 12)."""
        _check(lib().dls_ctx_set_jacobi_sweeps(self._h, int(max_sweeps)))

    def _last(self) -> Params:
        p = getattr(self, "_last_params", None)
        if p is None:
            raise DlsError(DLS_EINVAL, "no encode result in this context")
        return p

    def decode(self, out: torch.Tensor, stream=None) -> torch.Tensor:
        """Reconstruct the last encode's field into `out` (device tensor of the
        field's shape and dtype) on the device, enqueued on `stream`."""
        _check_field(out, self._last())
        _check(lib().dls_decode(self._h, ctypes.c_void_p(out.data_ptr()), out.numel() * out.element_size(),
                                _stream_handle(stream)))
        return out

    def features(self, field: torch.Tensor, stream=None) -> torch.Tensor:
        """Raw features (nblocks x 80) of the blocks of the last encode."""
        _check_field(field, self._last())
        nb = self.info().nblocks
        out = torch.empty((nb, 80), dtype=torch.float32, device=field.device)
        _check(lib().dls_features(self._h, ctypes.c_void_p(field.data_ptr()), field.numel() * field.element_size(),
                                  ctypes.c_void_p(out.data_ptr()), out.numel() * 4, _stream_handle(stream)))
        return out

    def info(self) -> _EncodeInfo:
        inf = _EncodeInfo()
        _check(lib().dls_encode_info_get(self._h, ctypes.byref(inf)))
        return inf

    def finalize(self) -> bytes:
        out = ctypes.c_void_p()
        n = ctypes.c_size_t()
        _check(lib().dls_finalize(self._h, ctypes.byref(out), ctypes.byref(n)))
        try:
            return _take_bytes(out, n)
        finally:
            lib().dls_free(out)


def value_range(field: torch.Tensor, stream=None):
    """Per-variable (min, max) of a (nvars, ...) device field, computed on the device."""
    if not field.is_cuda or not field.is_contiguous() or field.dtype not in (torch.float32, torch.float64):
        raise ValueError("field must be a contiguous float32/float64 device tensor")
    nv = field.shape[0]
    lo = (ctypes.c_double * nv)()
    hi = (ctypes.c_double * nv)()
    _check(lib().dls_range(ctypes.c_void_p(field.data_ptr()), nv, field.numel() // nv,
                           DLS_F32 if field.dtype == torch.float32 else DLS_F64,
                           _stream_handle(stream), lo, hi))
    return [lo[i] for i in range(nv)], [hi[i] for i in range(nv)]


def compress(field: torch.Tensor, p: Params, stream=None) -> bytes:
    _check_field(field, p)
    cp = p.to_c()
    out = ctypes.c_void_p()
    n = ctypes.c_size_t()
    _check(lib().dls_compress(ctypes.c_void_p(field.data_ptr()), ctypes.byref(cp),
                              _stream_handle(stream), ctypes.byref(out), ctypes.byref(n)))
    try:
        return _take_bytes(out, n)
    finally:
        lib().dls_free(out)


def query(buf: bytes):
    """(Params, nblocks) from a stream header."""
    cp = _Params()
    eps = (ctypes.c_double * 65536)()
    nb = ctypes.c_int64()
    _check(lib().dls_query(buf, len(buf), ctypes.byref(cp), eps, 65536, ctypes.byref(nb)))
    p = Params(nx=cp.nx, ny=cp.ny, nz=cp.nz, nt=cp.nt, nvars=cp.nvars,
               dtype="f32" if cp.dtype == DLS_F32 else "f64", px=cp.px, py=cp.py, pz=cp.pz,
               window=cp.window, eps=[eps[i] for i in range(cp.nvars)], pmin=cp.pmin,
               r_max=cp.r_max, adaptive=bool(cp.flags & DLS_ADAPTIVE), l2=bool(cp.flags & DLS_L2),
               global_basis=bool(cp.flags & DLS_GLOBAL),
               basis={v: k for k, v in BASIS_KINDS.items()}.get(cp.basis, "svd"))
    return p, nb.value


def stats(buf: bytes) -> dict:
    s = _StreamStats()
    _check(lib().dls_stats(buf, len(buf), ctypes.byref(s)))
    return {"nblocks": s.nblocks, "nbatches": s.nbatches, "nraw": s.nraw, "nescapes": s.nescapes,
            "rank_hist": list(s.rank_hist), "payload_bytes": s.payload_bytes,
            "stream_bytes": s.stream_bytes}


def decompress(buf: bytes, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    p, _ = query(buf)
    if out is None:
        out = torch.empty(p.shape, dtype=p.torch_dtype, device="cuda")
    _check_field(out, p)
    _check(lib().dls_decompress(buf, len(buf), ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


_hiplib = None


def d2h(ptr: int, nbytes: int):
    """Copy device memory (a pointer from Encoder.info()) to a host uint8 numpy array."""
    import numpy as np
    global _hiplib
    if _hiplib is None:
        # the runtime torch already loaded, so both sides share one HIP instance
        _hiplib = ctypes.CDLL(os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so"))
        _hiplib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hiplib.hipMemcpy.restype = ctypes.c_int
    out = np.empty(max(int(nbytes), 1), dtype=np.uint8)
    if nbytes:
        st = _hiplib.hipMemcpy(out.ctypes.data, ctypes.c_void_p(ptr), int(nbytes), 2)
        if st != 0:
            raise RuntimeError("hipMemcpy failed: %d" % st)
    return out[:int(nbytes)]


def d2d(dst: torch.Tensor, ptr: int, nbytes: int):
    """Copy nbytes of device memory at ptr (from Encoder.info()) into dst."""
    d2h(0, 0)  # loads the runtime handle
    st = _hiplib.hipMemcpy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(ptr), int(nbytes), 3)
    if st != 0:
        raise RuntimeError("hipMemcpy failed: %d" % st)
    return dst


class Model:
    """The warm-start network on a device (parameters, Adam state)."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().dls_model_create(device, ctypes.byref(h)))
        self._h = h

    def close(self):
        if self._h:
            lib().dls_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set(self, params, norm=None):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == NPARAM
        n = None if norm is None else np.ascontiguousarray(norm, dtype=np.float32)
        _check(lib().dls_model_set(self._h, ctypes.c_void_p(p.ctypes.data),
                                   None if n is None else ctypes.c_void_p(n.ctypes.data)))

    def get(self):
        import numpy as np
        p = np.empty(NPARAM, np.float32)
        n = np.empty(32, np.float32)
        _check(lib().dls_model_get(self._h, ctypes.c_void_p(p.ctypes.data), ctypes.c_void_p(n.ctypes.data)))
        return p, n

    def forward(self, feat: torch.Tensor, bf16=True, stream=None) -> torch.Tensor:
        """bf16: False (FP32 products), True (bf16, fused kernel) or 2 (bf16, layer by layer)."""
        feat = feat.contiguous()
        out = torch.empty((feat.shape[0], 272), dtype=torch.float32, device=feat.device)
        _check(lib().dls_model_forward(self._h, ctypes.c_void_p(feat.data_ptr()), feat.shape[0], int(bf16),
                                       ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def grad(self, feat, rank, basis, wb, bf16: bool = False, stream=None):
        g = torch.empty(NPARAM, dtype=torch.float32, device=feat.device)
        loss = ctypes.c_float()
        _check(lib().dls_model_grad(self._h, ctypes.c_void_p(feat.data_ptr()), ctypes.c_void_p(rank.data_ptr()),
                                    ctypes.c_void_p(basis.data_ptr()), ctypes.c_void_p(wb.data_ptr()),
                                    feat.shape[0], int(bf16), ctypes.c_void_p(g.data_ptr()), ctypes.byref(loss),
                                    _stream_handle(stream)))
        return g, loss.value

    def train_step(self, feat, rank, basis, wb, lr: float = 1e-3, bf16: bool = True, want_loss: bool = True,
                   stream=None):
        loss = ctypes.c_float()
        _check(lib().dls_model_train_step(self._h, ctypes.c_void_p(feat.data_ptr()),
                                          ctypes.c_void_p(rank.data_ptr()), ctypes.c_void_p(basis.data_ptr()),
                                          ctypes.c_void_p(wb.data_ptr()), feat.shape[0], lr, int(bf16),
                                          ctypes.byref(loss) if want_loss else None, _stream_handle(stream)))
        return loss.value if want_loss else None
