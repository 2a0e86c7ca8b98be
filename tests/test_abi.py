"""libdls loads, exports what include/dls.h declares, and its host-side stream
parser (dls_query, dls_stats) agrees with streams the oracle writes.  No GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import container, dls as odls

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dls.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dls_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    import paper_2601_20113_amd as pkg
    return pkg


def test_library_exports_every_declared_symbol(L):
    lib = L.lib()
    names = _declared()
    assert "dls_encode" in names and "dls_decompress" in names
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(L.EXPORTS) == names


def test_param_struct_layout_matches_header(L, tmp_path):
    """The ctypes mirror of dls_params has the C compiler's size and field
    offsets (compiled from include/dls.h with gcc)."""
    import subprocess
    names = [f[0] for f in L._Params._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"dls.h\"\nint main(void) {\n"
                   "  printf(\"%zu\\n\", sizeof(dls_params));\n"
                   + "".join("  printf(\"%%zu\\n\", offsetof(dls_params, %s));\n" % n for n in names)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.check_call(["gcc", "-std=c11", "-I", inc, str(src), "-o", str(exe)])
    vals = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert vals[0] == ctypes.sizeof(L._Params)
    assert vals[1:] == [getattr(L._Params, n).offset for n in names]


def _oracle_stream(dtype=np.float64, adaptive=False):
    f = synth.blobs2d(nx=40, ny=36, nt=20, seed=2, dtype=dtype)
    e = 1e-3 * synth.range_of(f)[0]
    p = odls.Params(nx=40, ny=36, nz=1, nt=20, nvars=1,
                    dtype="f64" if dtype == np.float64 else "f32",
                    px=16 if adaptive else 8, py=16 if adaptive else 8, pz=1, window=16,
                    eps=[e], pmin=4, adaptive=adaptive)
    enc = odls.encode(f, p)
    return enc, container.pack(enc)


@pytest.mark.parametrize("adaptive", [False, True])
def test_query_and_stats_of_oracle_stream(L, adaptive):
    enc, buf = _oracle_stream(adaptive=adaptive)
    p, nb = L.query(buf)
    assert nb == len(enc.blocks)
    assert (p.nx, p.ny, p.nz, p.nt, p.nvars, p.dtype) == (40, 36, 1, 20, 1, "f64")
    assert p.eps[0] == enc.params.eps[0] and p.adaptive == adaptive
    st = L.stats(buf)
    ranks = [c.r for c in enc.codes]
    assert st["nblocks"] == len(ranks)
    assert st["rank_hist"][:17] == list(np.bincount(ranks, minlength=17))
    assert st["nescapes"] == sum(c.esc_values.size for c in enc.codes)
    assert st["stream_bytes"] == len(buf)


def test_corrupt_streams_are_rejected(L):
    _, buf = _oracle_stream()
    bad = [buf[:50], b"XXXX" + buf[4:], buf[:-10], buf[:200] + bytes(len(buf) - 200)]
    flip = bytearray(buf)
    flip[-20] ^= 0xFF
    bad.append(bytes(flip))
    for b in bad:
        with pytest.raises(L.DlsError) as e:
            L.stats(b)
        assert e.value.status == L.DLS_ECORRUPT


def test_invalid_params_rejected_before_device_work(L):
    lib = L.lib()
    good = L.Params(nx=64, ny=64, nz=1, nt=32, nvars=1, dtype="f64", px=8, py=8, pz=1,
                    window=16, eps=[1e-3])
    cases = [dict(eps=[0.0]), dict(eps=[float("nan")]), dict(window=0), dict(window=33),
             dict(px=0), dict(pz=2), dict(nx=0), dict(r_max=40)]
    for kw in cases:
        p = L.Params(**{**good.__dict__, **kw})
        cp = p.to_c()
        out = ctypes.c_void_p()
        n = ctypes.c_size_t()
        st = lib.dls_compress(ctypes.c_void_p(16), ctypes.byref(cp), None, ctypes.byref(out), ctypes.byref(n))
        assert st == L.DLS_EINVAL, kw
    cp = good.to_c()
    cp.struct_size = 12
    st = lib.dls_compress(ctypes.c_void_p(16), ctypes.byref(cp), None, ctypes.byref(ctypes.c_void_p()),
                          ctypes.byref(ctypes.c_size_t()))
    assert st == L.DLS_EINVAL
    assert b"struct_size" in lib.dls_last_error()


def test_null_context_refused(L):
    """Entry points that take a context refuse NULL before any device call."""
    lib = L.lib()
    assert lib.dls_ctx_set_jacobi_sweeps(None, 4) == L.DLS_EINVAL
    assert lib.dls_encode(None, ctypes.c_void_p(16), None, None, 0) == L.DLS_EINVAL
    info = L._EncodeInfo()
    assert lib.dls_encode_info_get(None, ctypes.byref(info)) == L.DLS_EINVAL


def test_large_host_buffer_copied_whole(L):
    """Streams of 2 GiB and more come back whole (ctypes.string_at takes a C
    int length, which wraps there)."""
    n = (1 << 31) + 4096
    buf = ctypes.create_string_buffer(n)
    ctypes.memset(ctypes.addressof(buf) + n - 3, 0x5A, 3)
    b = L._take_bytes(ctypes.c_void_p(ctypes.addressof(buf)), ctypes.c_size_t(n))
    assert len(b) == n and b[-3:] == b"\x5a\x5a\x5a" and b[0] == 0
    del b, buf
    assert L._take_bytes(ctypes.c_void_p(None), ctypes.c_size_t(0)) == b""


def test_query_and_stats_of_oracle_l2_stream(L):
    """An L2-mode stream written by the oracle: the header carries the mode,
    the stats count its ranks and raw blocks."""
    from oracle import l2
    f = synth.blobs2d(nx=40, ny=36, nt=20, seed=2)
    f[0, 2, 0, 3, 4] = np.nan
    p = odls.Params(nx=40, ny=36, nz=1, nt=20, nvars=1, dtype="f64", px=8, py=8, pz=1, window=16, eps=[1e-3])
    enc = l2.encode(f, p)
    buf = container.pack_l2(enc)
    q, nb = L.query(buf)
    assert nb == len(enc.blocks) and q.l2 and q.eps[0] == 1e-3
    st = L.stats(buf)
    ranks = [c.r for c in enc.codes]
    assert st["nraw"] == ranks.count(l2.RAW) == 1
    assert st["rank_hist"][:17] == [ranks.count(r) for r in range(17)]
    assert st["nescapes"] == 0


def test_l2_with_learned_rejected_before_device_work(L):
    lib = L.lib()
    p = L.Params(nx=64, ny=64, nz=1, nt=32, nvars=1, dtype="f64", px=8, py=8, pz=1, window=16, eps=[1e-3],
                 l2=True, learned=True)
    cp = p.to_c()
    st = lib.dls_compress(ctypes.c_void_p(16), ctypes.byref(cp), None, ctypes.byref(ctypes.c_void_p()),
                          ctypes.byref(ctypes.c_size_t()))
    assert st == L.DLS_EINVAL and b"DLS_L2" in lib.dls_last_error()


@pytest.mark.parametrize("kind", ["svd", "cosine", "random"])
def test_query_and_stats_of_oracle_global_stream(L, kind):
    """The library's host parser reads a global-basis stream the oracle
    wrote: the problem statement, the basis kind, the patch count, the raw
    patches and the coefficient-count histogram."""
    from oracle import globalbasis as gb
    f = synth.blobs2d(nx=24, ny=16, nt=3, seed=5, nblobs=3)
    f[0, 1, 0, 3, 3] = np.nan
    p = odls.Params(nx=24, ny=16, nz=1, nt=3, nvars=1, dtype="f64", px=8, py=8, pz=1, window=1, eps=[1e-3])
    enc = gb.encode(f, p, gb.KINDS[kind], seed=3)
    buf = container.pack_global(enc)
    q, nb = L.query(buf)
    assert nb == len(enc.blocks) == 18
    assert q.global_basis and q.basis == kind and q.window == 1 and not q.l2
    st = L.stats(buf)
    ns = [c.n for c in enc.codes]
    assert st["nraw"] == sum(n == gb.RAW for n in ns) == 1
    hist = [0] * 33
    for n in ns:
        if n != gb.RAW:
            hist[min(n, 32)] += 1
    assert st["rank_hist"] == hist
    # a corrupted basis kind is refused
    bad = bytearray(buf)
    bad[100] = 7
    with pytest.raises(L.DlsError):
        L.stats(bytes(bad))
