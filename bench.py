#!/usr/bin/env python
"""Device compression throughput of the DLS hot path on one MI355X.

One step = one dls_encode over the whole synthetic field (plan, Gram,
eigensolve + rank, offset scan, projection / quantization / lattice
reconstruction / residual codes), input already resident in HBM.  Prints one
JSON line with the throughput, the roofline of the dominant kernel (measured
with HIP events on the stream the kernels run on), and the FP64 CPU oracle
timed on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "compress GB/s at abs bound 1e-3·range, learned+mixed vs plain GPU; ratio"

CONFIGS = {
    "c1": dict(desc="2D FP64 64x64 x 32 steps, 4 moving Gaussian blobs + N(0,1e-4) noise, "
                    "8x8 patches x 16-step windows (128 blocks), eps = 1e-3*range",
               kind="blobs", nx=64, ny=64, nz=1, nt=32, nvars=1, dtype="f64", px=8, py=8, pz=1,
               window=16, seeds=[1], rel_eps=1e-3),
    "c2": dict(desc="3D FP32 256^3 x 64 steps, 3 variables (u, v, p), 64 random-phase modes "
                    "k^-5/3, exp(-0.02 t) decay, 16^3 patches x 32-step windows, eps = 1e-3*range",
               kind="spectrum", nx=256, ny=256, nz=256, nt=64, nvars=3, dtype="f32", px=16, py=16,
               pz=16, window=32, seeds=[11, 12, 13], rel_eps=1e-3),
    "c3": dict(desc="2D FP32 4096x2048 x 100 steps, 8192 moving Gaussian blobs (4 per 64^2) + "
                    "N(0,1e-4) counter-based noise, quadtree 32^2..4^2 split where the mean "
                    "|grad| of snapshot 0 exceeds its 80th percentile, 16-step windows "
                    "(last one 4), eps = 1e-3*range",
               kind="blobs_gpu", nx=4096, ny=2048, nz=1, nt=100, nvars=1, dtype="f32", px=32, py=32,
               pz=1, pmin=4, adaptive=True, window=16, seeds=[31], nblobs=8192, rel_eps=1e-3),
    "c5": dict(desc="3D FP32 512^3 x 48 steps, 2 variables (u, v), 64 random-phase modes k^-5/3, "
                    "exp(-0.02 t) decay, octree 32^3..8^3 split where the mean |grad| of "
                    "snapshot 0 exceeds its 80th percentile, 16-step windows, eps = 1e-3*range "
                    "(51.5 GB resident in HBM)",
               kind="spectrum", nx=512, ny=512, nz=512, nt=48, nvars=2, dtype="f32", px=32, py=32,
               pz=32, pmin=8, adaptive=True, window=16, seeds=[11, 12], rel_eps=1e-3),
}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def make_field(cfg):
    import numpy as np
    import torch
    import synth
    shape = (cfg["nvars"], cfg["nt"], cfg["nz"], cfg["ny"], cfg["nx"])
    dt = torch.float32 if cfg["dtype"] == "f32" else torch.float64
    if cfg["kind"] == "blobs":
        f = synth.blobs2d(nx=cfg["nx"], ny=cfg["ny"], nt=cfg["nt"], seed=cfg["seeds"][0],
                          dtype=np.float32 if cfg["dtype"] == "f32" else np.float64)
        t = torch.from_numpy(f).cuda()
    elif cfg["kind"] == "blobs_gpu":
        from synth import gpu as sg
        t = torch.empty(shape, dtype=dt, device="cuda")
        sg.blobs_into(t[0], nblobs=cfg["nblobs"], seed=cfg["seeds"][0])
    else:
        from synth import gpu as sg
        t = torch.empty(shape, dtype=dt, device="cuda")
        for v, seed in enumerate(cfg["seeds"]):
            sg.spectrum_into(t[v], seed=seed, nmodes=64, drift=cfg.get("drift", False))
    import paper_2601_20113_amd as dls
    lo, hi = dls.value_range(t)
    eps = [cfg["rel_eps"] * (h - l) for l, h in zip(lo, hi)]
    torch.cuda.synchronize()
    return t, eps


def cpu_baseline(field, cfg, eps, seconds):
    """The FP64 oracle, as it stands, on blocks of variable 0, window 0, in
    plan order, until ~`seconds` of CPU time; BLAS pinned to one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import dls as odls
    W = min(cfg["window"], cfg["nt"])
    sub = field[0:1, 0:W, 0:min(cfg["pz"], cfg["nz"])].cpu().numpy()
    p = odls.Params(nx=cfg["nx"], ny=cfg["ny"], nz=sub.shape[2], nt=W, nvars=1, dtype=cfg["dtype"],
                    px=cfg["px"], py=cfg["py"], pz=cfg["pz"] if cfg["nz"] > 1 else 1, window=W,
                    eps=[eps[0]], pmin=cfg.get("pmin", 0), adaptive=cfg.get("adaptive", False))
    done, nbytes = 0, 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        blocks, _ = odls.plan(sub, p)
        for b in blocks:
            xb = odls.gather(sub, b)
            odls.encode_block(xb, eps[0], p.resolved_rmax(), p.np_dtype)
            done += 1
            nbytes += xb.nbytes
            if time.perf_counter() - t0 > seconds:
                break
        dt = time.perf_counter() - t0
    return {"value": nbytes / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": "%d of %d blocks of variable 0, window 0, first z-slab (the oracle's own "
                      "plan of that slab included), %.1f MB in %.1f s"
                      % (done, len(blocks), nbytes / 1e6, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ratio", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(blocks are independent; sharding is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2601_20113_amd as dls
    cfg = CONFIGS[args.config]
    log("generating %s" % args.config)
    field, eps = make_field(cfg)
    in_bytes = field.numel() * field.element_size()
    p = dls.Params(nx=cfg["nx"], ny=cfg["ny"], nz=cfg["nz"], nt=cfg["nt"], nvars=cfg["nvars"],
                   dtype=cfg["dtype"], px=cfg["px"], py=cfg["py"], pz=cfg["pz"],
                   window=cfg["window"], eps=eps, pmin=cfg.get("pmin", 0),
                   adaptive=cfg.get("adaptive", False))
    enc = dls.Encoder()
    stream = torch.cuda.current_stream()
    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        enc.encode(field, p, stream=stream)
    torch.cuda.synchronize()
    stage = [0.0] * 5
    log("timing %d steps" % args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        enc.encode(field, p, stream=stream)
        inf = enc.info()
        for i in range(5):
            stage[i] += inf.stage_ms[i]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt * 1e3 / args.steps
    stage = [s / args.steps for s in stage]
    inf = enc.info()
    gbs = in_bytes / (ms * 1e-3) / 1e9

    # roofline of the dominant kernel, from algorithmic bytes per launch
    es = field.element_size()
    nvals = field.numel()
    names = ["plan", "gram", "eigen", "scan", "encode"]
    dom = max(range(5), key=lambda i: stage[i])
    if names[dom] == "encode":
        traffic_alg = nvals * (es + 2) + inf.qa_bytes
    elif names[dom] == "gram":
        traffic_alg = nvals * es
    else:
        traffic_alg = None
    roof = None
    if traffic_alg is not None:
        ach = traffic_alg / (stage[dom] * 1e-3) / 1e9
        roof = {"kernel": "k_" + names[dom], "bound": "hbm", "achieved": round(ach, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": None, "alg_bytes_per_launch": int(traffic_alg),
                "launch_ms": round(stage[dom], 4)}
    else:
        roof = {"kernel": "k_" + names[dom], "bound": "alu", "achieved": None, "peak": None,
                "unit": "TFLOP/s", "frac": None, "traffic": None, "launch_ms": round(stage[dom], 4)}

    ratio = None
    if not args.no_ratio:
        log("finalize for the compression ratio")
        t1 = time.perf_counter()
        buf = enc.finalize()
        ratio = in_bytes / len(buf)
        log("finalize %.1f s" % (time.perf_counter() - t1))

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline")
        cpu = cpu_baseline(field, cfg, eps, args.cpu_seconds)

    out = {
        "metric": METRIC, "value": round(gbs, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": cfg["dtype"], "data": "synthetic",
        "config": {"workload": args.config + ": " + cfg["desc"], "form": "plain",
                   "input_bytes": in_bytes, "blocks": int(inf.nblocks)},
        "stage_ms": {n: round(s, 4) for n, s in zip(names, stage)},
        "compression_ratio": None if ratio is None else round(ratio, 3),
        "escapes": int(inf.nescapes),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
