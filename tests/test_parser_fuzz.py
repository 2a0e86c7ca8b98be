"""Seeded corrupt-stream fuzz of the host stream parser under the address
and undefined-behaviour sanitizers (CPU only).

tests/fuzz/parse_fuzz.cpp is built with g++ -fsanitize=address,undefined
together with the library's host format unit (csrc/dls_format.cpp:
parse_header, leaves_from_bits, plan_from_header, build_blocks).  The seed
streams are the oracle's (absolute mode uniform and adaptive, L2 mode,
global-basis mode); each mutant flips, overwrites or truncates bytes of its
header region (where the parser reads sizes, counts, split bits and the
batch table) or of the whole stream.  The harness must exit 0 with no
sanitizer report; every intact seed must parse with its block count.
"""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import synth  # noqa: E402
from oracle import container, dls as odls, globalbasis as gb, l2  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2601_20113_amd", "csrc")


def _seeds():
    f = synth.blobs2d(nx=40, ny=36, nt=20, seed=2)
    e = [1e-3 * synth.range_of(f)[0]]
    out = []
    for adaptive in (False, True):
        p = odls.Params(nx=40, ny=36, nz=1, nt=20, nvars=1, dtype="f64", px=16 if adaptive else 8,
                        py=16 if adaptive else 8, pz=1, window=16, eps=e, pmin=4, adaptive=adaptive)
        enc = odls.encode(f, p)
        out.append((container.pack(enc), len(enc.blocks)))
    p = odls.Params(nx=40, ny=36, nz=1, nt=20, nvars=1, dtype="f64", px=8, py=8, pz=1, window=16, eps=[1e-3])
    enc = l2.encode(f, p)
    out.append((container.pack_l2(enc), len(enc.blocks)))
    g = f[:, :4]
    q = odls.Params(nx=40, ny=36, nz=1, nt=4, nvars=1, dtype="f64", px=8, py=8, pz=1, window=1, eps=[1e-3])
    enc = gb.encode(g, q, gb.KIND_COSINE)
    out.append((container.pack_global(enc), len(enc.blocks)))
    return out


def _mutants(buf, rng, n):
    hdr = int.from_bytes(buf[8:12], "little")
    for _ in range(n):
        b = bytearray(buf)
        kind = rng.integers(0, 4)
        if kind == 0:      # flip bits in the header
            for _ in range(rng.integers(1, 4)):
                i = int(rng.integers(0, min(hdr, len(b))))
                b[i] ^= 1 << int(rng.integers(0, 8))
        elif kind == 1:    # overwrite a header word with an extreme value
            i = int(rng.integers(0, max(1, min(hdr, len(b)) - 8)))
            b[i:i + 8] = rng.choice([b"\xff" * 8, b"\x00" * 8, b"\x7f" + b"\xff" * 7,
                                     (2 ** 31).to_bytes(8, "little")])
        elif kind == 2:    # truncate
            b = b[:int(rng.integers(0, len(b)))]
        else:              # random bytes anywhere
            for _ in range(rng.integers(1, 16)):
                b[int(rng.integers(0, len(b)))] = int(rng.integers(0, 256))
        yield bytes(b)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_parser_under_sanitizers(tmp_path):
    exe = tmp_path / "parse_fuzz"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", CSRC, os.path.join(HERE, "fuzz", "parse_fuzz.cpp"), os.path.join(CSRC, "dls_format.cpp"),
           "-o", str(exe)]
    subprocess.check_call(cmd)
    rng = np.random.default_rng(20260113)
    files, expect = [], []
    for k, (buf, nb) in enumerate(_seeds()):
        fn = tmp_path / ("seed%d" % k)
        fn.write_bytes(buf)
        files.append(str(fn))
        expect.append("ok %d" % nb)
        for j, m in enumerate(_mutants(buf, rng, 150)):
            fm = tmp_path / ("m%d_%d" % (k, j))
            fm.write_bytes(m)
            files.append(str(fm))
            expect.append(None)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)] + files, capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    lines = r.stdout.splitlines()
    assert len(lines) == len(files)
    for line, want in zip(lines, expect):
        if want is not None:
            assert line == want
        else:
            assert line.startswith("ok ") or line.startswith("corrupt ")
    print("mutants: %d parsed, %d refused" % (sum(l.startswith("ok") for l in lines) - 4,
                                             sum(l.startswith("corrupt") for l in lines)))
