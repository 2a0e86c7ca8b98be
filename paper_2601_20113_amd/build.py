"""Build libdls.so (gfx950) in-tree: ``python -m paper_2601_20113_amd.build``."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libdls.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HIP_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    # packed FP32 (v_pk_*_f32) stays off on this target
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-pass-failed",
]
HIP_SOURCES = ["dls_kernels.hip", "dls_plan.hip", "dls_learned.hip", "dls_l2.hip", "dls_global.hip", "dls_api.hip"]
# dls_codec.hip holds the encode / decode kernels; it is compiled once per
# (padded window, element type, part) so that its rank-class instantiations
# build in parallel: (tag, W, element type, points per thread)
CODEC_TYPES = [("w16_f32", 16, "float", 4), ("w16_f64", 16, "double", 2), ("w32_f32", 32, "float", 2),
               ("w32_f64", 32, "double", 2)]
CODEC_PARTS = 3  # 0 large-slice encode, 1 small-slice encode, 2 decode
FUSED_TAG = "w16_f32"  # part 3, the fused single-pass encode, exists for this pair only
CXX_SOURCES = ["dls_format.cpp"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), out))
    if verbose and out.strip():
        print(out, flush=True)


def build(verbose: bool = False) -> str:
    """Compile every HIP source for gfx950 and link libdls.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append((obj, [HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]))
    for tag, wp, ty, ppt in CODEC_TYPES:
        for part in range(CODEC_PARTS + (1 if tag == FUSED_TAG else 0)):
            obj = os.path.join(BUILD, "dls_codec_%s_%d.o" % (tag, part))
            defs = ["-DDLS_CODEC_TAG=" + tag, "-DDLS_CODEC_WP=%d" % wp, "-DDLS_CODEC_T=" + ty,
                    "-DDLS_CODEC_PPT=%d" % ppt, "-DDLS_CODEC_PART=%d" % part]
            jobs.append((obj, [HIPCC] + HIP_FLAGS + defs + ["-c", os.path.join(CSRC, "dls_codec.hip"), "-o", obj]))
    for src in CXX_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append((obj, ["g++", "-O2", "-std=c++17", "-fPIC", "-c", os.path.join(CSRC, src), "-o", obj]))
    jobs.sort(key=lambda j: "dls_codec_w32" not in j[0])  # the longest units first
    nproc = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=nproc) as ex:
        for f in [ex.submit(_run, cmd, verbose) for _, cmd in jobs]:
            f.result()
    objs = [obj for obj, _ in jobs]
    tmp = OUT + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lz", "-lpthread"], verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
