"""dls_range_noalloc (no device allocation) against dls_range, through the C ABI.

Two calls in a row on the same GPU, the second on a smaller field with fewer
variables (the fixed scratch keeps the first call's partials, which the
second must not see), then the first field again; each result must equal
dls_range's bitwise (min and max are exact).  Non-finite values are skipped
by both.
"""
import ctypes
import os
import sys

import numpy as np
import pytest
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import paper_2601_20113_amd as dls  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu


def _range(fn, t, nvars):
    lo = (ctypes.c_double * nvars)()
    hi = (ctypes.c_double * nvars)()
    st = fn(ctypes.c_void_p(t.data_ptr()), nvars, t.numel() // nvars,
            dls.DLS_F32 if t.dtype == torch.float32 else dls.DLS_F64, None, lo, hi)
    assert st == dls.DLS_OK, dls.lib().dls_last_error()
    return list(lo), list(hi)


def test_noalloc_range_matches_allocating_range():
    L = dls.lib()
    f = synth.blobs2d(nx=300, ny=200, nt=40, seed=8, dtype=np.float32)
    big = np.concatenate([f * (v + 1) - v for v in range(5)])      # 5 variables, 2.4M values each
    big[3, 7, 0, 9, 11] = np.nan
    small = synth.blobs2d(nx=20, ny=10, nt=3, seed=9)[:, :, :, :, :] * 0.5 + 7.0   # 1 variable, 600 values, f64
    tb = torch.from_numpy(big).cuda()
    ts = torch.from_numpy(small).cuda()
    for t, nv in ((tb, 5), (ts, 1), (tb, 5)):
        print("noalloc range: %d variables x %d values, %s" % (nv, t.numel() // nv, t.dtype), flush=True)
        a = _range(L.dls_range_noalloc, t, nv)
        b = _range(L.dls_range, t, nv)
        assert a == b
        for v in range(nv):
            x = t[v].double().cpu().numpy()
            x = x[np.isfinite(x)]
            assert a[0][v] == x.min() and a[1][v] == x.max()


def test_noalloc_range_rejects_too_many_variables():
    L = dls.lib()
    t = torch.zeros(65, 4, dtype=torch.float32, device="cuda")
    lo = (ctypes.c_double * 65)()
    hi = (ctypes.c_double * 65)()
    st = L.dls_range_noalloc(ctypes.c_void_p(t.data_ptr()), 65, 4, dls.DLS_F32, None, lo, hi)
    assert st == dls.DLS_EINVAL
    assert b"64" in L.dls_last_error()
