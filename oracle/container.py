"""Oracle side of the DLS stream format (test infrastructure only).

Sec. 2.7.2 describes the paper's file: a fixed-size, addressable header that
records where each patch's compressed coefficient array sits, followed by the
tightly packed arrays, written in batches of 1000 patches.  This format keeps
that shape: a header with the problem statement, the adaptive split bits and
a (offset, size) entry per batch of 1000 blocks, then one independently
decodable zlib stream (deflate, level 6 -- gzip's algorithm, Sec. 2.5) per
batch.

Header (little-endian):
    char[4] "DLS1"; u32 version=2; u32 header_bytes; u32 flags (bit0 adaptive,
    bit1 L2 mode: eps holds the per-variable NRMSE targets, see oracle.l2)
    i32 ndim, nvars, dtype (0 f32, 1 f64), r_max
    i64 nx, ny, nz, nt
    i32 px, py, pz, pmin, window, batch_blocks
    u64 nblocks; u32 nbatches; u32 extra (the basis kind in the global-basis
    mode, else 0)
    f64 eps[nvars]
    per variable: u32 nbits, then ceil(nbits/8) bytes of split bits (LSB first)
    per batch:    u64 offset (from header end), u64 compressed size,
                  u64 uncompressed size

Uncompressed batch payload for blocks [b0, b0 + nb):
    ranks      nb x u8 (0 = raw block)
    esc counts nb x u32
    qV         per block, zigzag(int32) of qV[k][t] (k < r, t < W_b), as 4
               byte planes (all low bytes, then the next bytes, ...)
    qA         per block, zigzag(int32) of qA[k][p] (k < r, p < M_b), 4 planes
    codes      per block, u8 codes[t][p] (one plane)
    escapes    escaped input values of the batch, block then (t, p) order,
               in the storage dtype

Global-basis mode (flag bit 2; window 1, so a block is one patch of one
snapshot; see oracle.globalbasis): the batch table lists ceil(nblocks / 1000)
patch batches, then one basis batch per variable.  Patch batch payload:
    counts     nb x u16, 2 planes (0xFFFF = raw patch, values verbatim)
    exponents  nb x i16, 2 planes (coefficient step 2^k; 0 when none)
    indices    the kept basis indices of every patch, ascending, u16, 2 planes
    coeffs     their zigzag(int32) coefficients, 4 planes
    raw        the raw patches' values, patch then point order, storage dtype
Basis batch payload: u32 kind (0 svd, 1 cosine, 2 random), u32 M, f64 c_v,
then zigzag(int32) of rint(Phi 2^24), Phi[i][s] row-major, 4 planes.

L2 mode (flag bit 1), uncompressed batch payload:
    ranks      nb x u8 (255 = raw block, values verbatim)
    steps      nb x f64 (coefficient step d; 0 for rank 0 and raw blocks)
    qV         per block, zigzag(int32) of qV[k][t] (k < r, t < W_b), 4 planes
    qA         per block, zigzag(int32) of qA[k][p] (k < r, p < M_b), 4 planes
    raw        the raw blocks' values, block then (t, p) order, storage dtype
"""
from __future__ import annotations

import struct
import zlib

import numpy as np

from . import dls, globalbasis, l2

MAGIC = b"DLS1"
VERSION = 2
ZLIB_LEVEL = 6
_FIXED = struct.Struct("<4sIII iiii qqqq iiiiii QII")


class CorruptStream(ValueError):
    """The byte stream is truncated or inconsistent."""


def zigzag32(a: np.ndarray) -> np.ndarray:
    a = a.astype(np.int64)
    return np.where(a >= 0, 2 * a, -2 * a - 1).astype(np.uint32)


def unzigzag32(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.int64)
    return np.where(z % 2 == 0, z // 2, -(z + 1) // 2)


def planes(a: np.ndarray, nbytes: int) -> bytes:
    """Byte-plane split: byte j of every element, for j = 0..nbytes-1."""
    le = np.ascontiguousarray(a).astype("<u%d" % nbytes)
    return np.frombuffer(le.tobytes(), np.uint8).reshape(-1, nbytes).T.tobytes()


def unplanes(buf: bytes, n: int, nbytes: int, dtype) -> np.ndarray:
    b = np.frombuffer(buf, np.uint8).reshape(nbytes, n).T.copy()
    return np.frombuffer(b.tobytes(), dtype="<u%d" % nbytes).astype(dtype)


def batch_payload(codes) -> bytes:
    """Uncompressed payload of one batch (list of dls.BlockCode)."""
    parts = [bytes(np.array([c.r for c in codes], np.uint8)),
             np.array([c.esc_values.size for c in codes], "<u4").tobytes()]
    for c in codes:
        parts.append(planes(zigzag32(c.qV.T.ravel()), 4))
    for c in codes:
        parts.append(planes(zigzag32(c.qA.T.ravel()), 4))
    for c in codes:
        parts.append(planes(c.codes.ravel(), 1))
    for c in codes:
        parts.append(c.esc_values.astype(c.esc_values.dtype.newbyteorder("<")).tobytes())
    return b"".join(parts)


def _bits_bytes(bits) -> bytes:
    n = len(bits)
    arr = np.zeros((n + 7) // 8, np.uint8)
    for i, bit in enumerate(bits):
        if bit:
            arr[i >> 3] |= 1 << (i & 7)
    return struct.pack("<I", n) + arr.tobytes()


def pack(enc: "dls.Encoded") -> bytes:
    p = enc.params
    nb = len(enc.blocks)
    nbatches = (nb + dls.BATCH_BLOCKS - 1) // dls.BATCH_BLOCKS
    streams, table = [], []
    off = 0
    for i in range(nbatches):
        raw = batch_payload(enc.codes[i * dls.BATCH_BLOCKS:(i + 1) * dls.BATCH_BLOCKS])
        z = zlib.compress(raw, ZLIB_LEVEL)
        streams.append(z)
        table.append((off, len(z), len(raw)))
        off += len(z)
    plan_bytes = b"".join(_bits_bytes(enc.split_bits[v] if p.adaptive else [])
                          for v in range(p.nvars))
    hdr_len = (_FIXED.size + 8 * p.nvars + len(plan_bytes) + 24 * nbatches)
    fixed = _FIXED.pack(MAGIC, VERSION, hdr_len, 1 if p.adaptive else 0,
                        p.ndim, p.nvars, 0 if p.dtype == "f32" else 1,
                        p.resolved_rmax(), p.nx, p.ny, p.nz, p.nt,
                        p.px, p.py, p.pz, p.pmin, p.window, dls.BATCH_BLOCKS,
                        nb, nbatches, 0)
    eps = struct.pack("<%dd" % p.nvars, *[float(e) for e in p.eps])
    tab = b"".join(struct.pack("<QQQ", *t) for t in table)
    return fixed + eps + plan_bytes + tab + b"".join(streams)


def _pack(p, nb, bits, payloads, flags, extra=0):
    streams, table = [], []
    off = 0
    for raw in payloads:
        z = zlib.compress(raw, ZLIB_LEVEL)
        streams.append(z)
        table.append((off, len(z), len(raw)))
        off += len(z)
    plan_bytes = b"".join(_bits_bytes(bits[v] if p.adaptive else []) for v in range(p.nvars))
    hdr_len = (_FIXED.size + 8 * p.nvars + len(plan_bytes) + 24 * len(payloads))
    fixed = _FIXED.pack(MAGIC, VERSION, hdr_len, flags,
                        p.ndim, p.nvars, 0 if p.dtype == "f32" else 1,
                        p.resolved_rmax(), p.nx, p.ny, p.nz, p.nt,
                        p.px, p.py, p.pz, p.pmin, p.window, dls.BATCH_BLOCKS,
                        nb, len(payloads), extra)
    eps = struct.pack("<%dd" % p.nvars, *[float(e) for e in p.eps])
    tab = b"".join(struct.pack("<QQQ", *t) for t in table)
    return fixed + eps + plan_bytes + tab + b"".join(streams)


def l2_batch_payload(codes, dtype) -> bytes:
    """Uncompressed payload of one L2-mode batch (list of l2.L2Code)."""
    parts = [bytes(np.array([c.r for c in codes], np.uint8)),
             np.array([c.step for c in codes], "<f8").tobytes()]
    for c in codes:
        if c.r != l2.RAW:
            parts.append(planes(zigzag32(c.qV.T.ravel()), 4))
    for c in codes:
        if c.r != l2.RAW:
            parts.append(planes(zigzag32(c.qA.T.ravel()), 4))
    for c in codes:
        if c.r == l2.RAW:
            parts.append(np.asarray(c.raw, dtype=np.dtype(dtype).newbyteorder("<")).tobytes())
    return b"".join(parts)


def pack_l2(enc: "l2.L2Encoded") -> bytes:
    p = enc.params
    nb = len(enc.blocks)
    payloads = [l2_batch_payload(enc.codes[i:i + dls.BATCH_BLOCKS], p.np_dtype)
                for i in range(0, nb, dls.BATCH_BLOCKS)]
    return _pack(p, nb, enc.split_bits, payloads, (1 if p.adaptive else 0) | 2)


def stream_flags(buf: bytes) -> int:
    if len(buf) < _FIXED.size:
        raise CorruptStream("stream shorter than the fixed header")
    return _FIXED.unpack_from(buf, 0)[3]


def _batches(buf, p, bits, nblocks, table, hdr_len):
    if p.adaptive:
        try:
            lv = [dls.leaves_from_bits(p, bits[v]) for v in range(p.nvars)]
        except StopIteration:
            raise CorruptStream("split bits exhausted")
    else:
        lv = [dls.uniform_leaves(p)] * p.nvars
    blocks = dls.make_blocks(p, lv)
    if len(blocks) != nblocks:
        raise CorruptStream("block count mismatch")
    if len(table) != (nblocks + dls.BATCH_BLOCKS - 1) // dls.BATCH_BLOCKS:
        raise CorruptStream("batch count mismatch")
    for i, (off, csz, usz) in enumerate(table):
        s = hdr_len + off
        if s + csz > len(buf):
            raise CorruptStream("batch beyond end of stream")
        try:
            raw = zlib.decompress(buf[s:s + csz])
        except zlib.error as e:
            raise CorruptStream("zlib: %s" % e)
        if len(raw) != usz:
            raise CorruptStream("batch size mismatch")
        yield blocks, blocks[i * dls.BATCH_BLOCKS:(i + 1) * dls.BATCH_BLOCKS], raw


def unpack_l2(buf: bytes) -> "l2.L2Encoded":
    p, bits, nblocks, table, hdr_len = parse_header(buf)
    if not stream_flags(buf) & 2:
        raise CorruptStream("not an L2-mode stream")
    dtype = p.np_dtype
    esz = np.dtype(dtype).itemsize
    codes, blocks = [], []
    for blocks, bl, raw in _batches(buf, p, bits, nblocks, table, hdr_len):
        nb = len(bl)
        pos = 0

        def take(n):
            nonlocal pos
            if pos + n > len(raw):
                raise CorruptStream("batch payload truncated")
            out = raw[pos:pos + n]
            pos += n
            return out
        ranks = np.frombuffer(take(nb), np.uint8)
        steps = np.frombuffer(take(8 * nb), "<f8")
        for b, r in zip(bl, ranks):
            if r != l2.RAW and r > min(p.resolved_rmax(), b.w):
                raise CorruptStream("rank out of range")
        rk = [0 if r == l2.RAW else int(r) for r in ranks]
        qVs = [unzigzag32(unplanes(take(4 * r * b.w), r * b.w, 4, np.uint32)).reshape(r, b.w).T
               for b, r in zip(bl, rk)]
        qAs = [unzigzag32(unplanes(take(4 * r * b.m), r * b.m, 4, np.uint32)).reshape(r, b.m).T
               for b, r in zip(bl, rk)]
        for j, b in enumerate(bl):
            rv = None
            if ranks[j] == l2.RAW:
                rv = np.frombuffer(take(esz * b.w * b.m), dtype=np.dtype(dtype).newbyteorder("<")).astype(dtype)
                rv = rv.reshape(b.w, b.m)
            codes.append(l2.L2Code(int(ranks[j]), float(steps[j]), qVs[j], qAs[j], rv))
        if pos != len(raw):
            raise CorruptStream("trailing bytes in batch")
    return l2.L2Encoded(p, blocks, codes, bits, np.zeros(p.nvars))


def global_batch_payload(codes, dtype) -> bytes:
    """Uncompressed payload of one global-mode patch batch (list of
    globalbasis.PatchCode)."""
    live = [c for c in codes if c.n not in (0, globalbasis.RAW)]
    idx = np.concatenate([c.kept for c in live]) if live else np.zeros(0, np.int64)
    q = np.concatenate([c.q for c in live]) if live else np.zeros(0, np.int64)
    parts = [planes(np.array([c.n for c in codes], np.uint16), 2),
             planes(np.array([c.k for c in codes], np.int64).astype(np.int16).view(np.uint16), 2),
             planes(idx.astype(np.uint16), 2), planes(zigzag32(q), 4)]
    for c in codes:
        if c.n == globalbasis.RAW:
            parts.append(np.asarray(c.raw, dtype=np.dtype(dtype).newbyteorder("<")).tobytes())
    return b"".join(parts)


def global_basis_payload(kind: int, phi: np.ndarray, cv: float) -> bytes:
    m = phi.shape[0]
    qphi = np.rint(phi * 2.0 ** globalbasis.BASIS_BITS).astype(np.int64)
    return struct.pack("<IId", kind, m, cv) + planes(zigzag32(qphi.ravel()), 4)


def pack_global(enc: "globalbasis.GlobalEncoded") -> bytes:
    p = enc.params
    nb = len(enc.blocks)
    payloads = [global_batch_payload(enc.codes[i:i + dls.BATCH_BLOCKS], p.np_dtype)
                for i in range(0, nb, dls.BATCH_BLOCKS)]
    payloads += [global_basis_payload(enc.kind, enc.bases[v], float(enc.budgets[v])) for v in range(p.nvars)]
    return _pack(p, nb, [[]] * p.nvars, payloads, 4, enc.kind)


def unpack_global(buf: bytes) -> "globalbasis.GlobalEncoded":
    p, bits, nblocks, table, hdr_len = parse_header(buf)
    if not stream_flags(buf) & 4:
        raise CorruptStream("not a global-basis stream")
    if p.window != 1:
        raise CorruptStream("global-basis stream with window != 1")
    m = p.px * p.py * p.pz
    if m > globalbasis.MAX_M or p.px > p.nx or p.py > p.ny or p.pz > p.nz:
        raise CorruptStream("bad patch size")
    npb = (nblocks + dls.BATCH_BLOCKS - 1) // dls.BATCH_BLOCKS
    if len(table) != npb + p.nvars:
        raise CorruptStream("batch count mismatch")
    blocks = dls.make_blocks(p, [dls.uniform_leaves(p)] * p.nvars)
    if len(blocks) != nblocks:
        raise CorruptStream("block count mismatch")

    def inflate(i):
        off, csz, usz = table[i]
        s0 = hdr_len + off
        if s0 + csz > len(buf):
            raise CorruptStream("batch beyond end of stream")
        try:
            raw = zlib.decompress(buf[s0:s0 + csz])
        except zlib.error as e:
            raise CorruptStream("zlib: %s" % e)
        if len(raw) != usz:
            raise CorruptStream("batch size mismatch")
        return raw
    bases, cvs = [], []
    kind = _FIXED.unpack_from(buf, 0)[-1]
    if kind > 2:
        raise CorruptStream("unknown basis kind")
    for v in range(p.nvars):
        raw = inflate(npb + v)
        if len(raw) != 16 + 4 * m * m:
            raise CorruptStream("basis batch size")
        k2, mm, cv = struct.unpack_from("<IId", raw, 0)
        if mm != m or k2 != kind:
            raise CorruptStream("basis batch header")
        q = unzigzag32(unplanes(raw[16:], m * m, 4, np.uint32)).reshape(m, m)
        bases.append(q.astype(np.float64) * 2.0 ** -globalbasis.BASIS_BITS)
        cvs.append(cv)
    dtype = p.np_dtype
    esz = np.dtype(dtype).itemsize
    codes = []
    for i in range(npb):
        raw = inflate(i)
        bl = blocks[i * dls.BATCH_BLOCKS:(i + 1) * dls.BATCH_BLOCKS]
        nb = len(bl)
        pos = 0

        def take(n):
            nonlocal pos
            if pos + n > len(raw):
                raise CorruptStream("batch payload truncated")
            out = raw[pos:pos + n]
            pos += n
            return out
        counts = unplanes(take(2 * nb), nb, 2, np.int64)
        exps = unplanes(take(2 * nb), nb, 2, np.uint16).astype(np.uint16).view(np.int16).astype(np.int64)
        for c in counts:
            if c != globalbasis.RAW and c > m:
                raise CorruptStream("coefficient count out of range")
        live = [int(c) for c in counts if c != globalbasis.RAW]
        tot = sum(live)
        idx = unplanes(take(2 * tot), tot, 2, np.int64)
        qs = unzigzag32(unplanes(take(4 * tot), tot, 4, np.uint32))
        if tot and (idx.max() >= m):
            raise CorruptStream("basis index out of range")
        at = 0
        for b, c, k in zip(bl, counts, exps):
            if c == globalbasis.RAW:
                rv = np.frombuffer(take(esz * b.m), dtype=np.dtype(dtype).newbyteorder("<")).astype(dtype)
                codes.append(globalbasis.PatchCode(globalbasis.RAW, 0, np.zeros(0, np.int64), np.zeros(0, np.int64),
                                                   rv))
                continue
            kept = idx[at:at + c]
            if c > 1 and np.any(np.diff(kept) <= 0):
                raise CorruptStream("basis indices not ascending")
            codes.append(globalbasis.PatchCode(int(c), int(k), kept, qs[at:at + c], None))
            at += int(c)
        if pos != len(raw):
            raise CorruptStream("trailing bytes in batch")
    return globalbasis.GlobalEncoded(p, int(kind), 0, bases, np.array(cvs), blocks, codes)


def parse_header(buf: bytes):
    """(Params, split bits per var, nblocks, batch table, header length)."""
    if len(buf) < _FIXED.size:
        raise CorruptStream("stream shorter than the fixed header")
    (magic, ver, hdr_len, flags, ndim, nvars, dt, rmax, nx, ny, nz, nt,
     px, py, pz, pmin, window, bblocks, nblocks, nbatches, _res) = _FIXED.unpack_from(buf, 0)
    if magic != MAGIC or ver != VERSION:
        raise CorruptStream("bad magic or version")
    if not (1 <= nvars <= 1 << 16) or dt not in (0, 1) or bblocks != dls.BATCH_BLOCKS:
        raise CorruptStream("bad header fields")
    if min(nx, ny, nz, nt, px, py, pz, window) < 1 or hdr_len > len(buf):
        raise CorruptStream("bad sizes")
    pos = _FIXED.size
    if pos + 8 * nvars > hdr_len:
        raise CorruptStream("truncated eps")
    eps = struct.unpack_from("<%dd" % nvars, buf, pos)
    pos += 8 * nvars
    bits = []
    for _ in range(nvars):
        if pos + 4 > hdr_len:
            raise CorruptStream("truncated plan")
        (n,) = struct.unpack_from("<I", buf, pos)
        pos += 4
        nbyte = (n + 7) // 8
        if pos + nbyte > hdr_len:
            raise CorruptStream("truncated plan bits")
        arr = np.frombuffer(buf, np.uint8, nbyte, pos)
        bits.append([(int(arr[i >> 3]) >> (i & 7)) & 1 for i in range(n)])
        pos += nbyte
    if pos + 24 * nbatches != hdr_len:
        raise CorruptStream("header length mismatch")
    table = [struct.unpack_from("<QQQ", buf, pos + 24 * i) for i in range(nbatches)]
    p = dls.Params(nx=nx, ny=ny, nz=nz, nt=nt, nvars=nvars,
                   dtype="f32" if dt == 0 else "f64", px=px, py=py, pz=pz,
                   window=window, eps=eps, pmin=pmin, r_max=rmax,
                   adaptive=bool(flags & 1))
    return p, bits, nblocks, table, hdr_len


def unpack(buf: bytes) -> "dls.Encoded":
    p, bits, nblocks, table, hdr_len = parse_header(buf)
    if stream_flags(buf) & 2:
        raise CorruptStream("an L2-mode stream (decode with oracle.l2)")
    if stream_flags(buf) & 4:
        raise CorruptStream("a global-basis stream (decode with oracle.globalbasis)")
    if p.adaptive:
        try:
            lv = [dls.leaves_from_bits(p, bits[v]) for v in range(p.nvars)]
        except StopIteration:
            raise CorruptStream("split bits exhausted")
    else:
        lv = [dls.uniform_leaves(p)] * p.nvars
    blocks = dls.make_blocks(p, lv)
    if len(blocks) != nblocks:
        raise CorruptStream("block count mismatch")
    if len(table) != (nblocks + dls.BATCH_BLOCKS - 1) // dls.BATCH_BLOCKS:
        raise CorruptStream("batch count mismatch")
    dtype = p.np_dtype
    esz = np.dtype(dtype).itemsize
    codes = []
    for i, (off, csz, usz) in enumerate(table):
        s = hdr_len + off
        if s + csz > len(buf):
            raise CorruptStream("batch beyond end of stream")
        try:
            raw = zlib.decompress(buf[s:s + csz])
        except zlib.error as e:
            raise CorruptStream("zlib: %s" % e)
        if len(raw) != usz:
            raise CorruptStream("batch size mismatch")
        bl = blocks[i * dls.BATCH_BLOCKS:(i + 1) * dls.BATCH_BLOCKS]
        nb = len(bl)
        pos = 0

        def take(n):
            nonlocal pos
            if pos + n > len(raw):
                raise CorruptStream("batch payload truncated")
            out = raw[pos:pos + n]
            pos += n
            return out
        ranks = np.frombuffer(take(nb), np.uint8)
        nesc = np.frombuffer(take(4 * nb), "<u4")
        qVs, qAs, cds = [], [], []
        for b, r in zip(bl, ranks):
            if r > min(p.resolved_rmax(), b.w, b.m):
                raise CorruptStream("rank out of range")
            n = int(r) * b.w
            qVs.append(unzigzag32(unplanes(take(4 * n), n, 4, np.uint32))
                       .reshape(int(r), b.w).T)
        for b, r in zip(bl, ranks):
            n = int(r) * b.m
            qAs.append(unzigzag32(unplanes(take(4 * n), n, 4, np.uint32))
                       .reshape(int(r), b.m).T)
        for b in bl:
            n = b.w * b.m
            cds.append(unplanes(take(n), n, 1, np.uint8).reshape(b.w, b.m))
        for j, b in enumerate(bl):
            ne = int(nesc[j])
            if ne != int(np.count_nonzero(cds[j] == dls.ESC_CODE)):
                raise CorruptStream("escape count mismatch")
            ev = np.frombuffer(take(esz * ne), dtype=np.dtype(dtype).newbyteorder("<"))
            codes.append(dls.BlockCode(int(ranks[j]), qVs[j], qAs[j], cds[j],
                                       ev.astype(dtype)))
        if pos != len(raw):
            raise CorruptStream("trailing bytes in batch")
    return dls.Encoded(p, blocks, codes, bits)
