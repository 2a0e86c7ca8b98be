#!/usr/bin/env python
"""Device compression throughput of the DLS hot path on one MI355X.

One step = one dls_encode over the whole synthetic field (plan, Gram,
eigensolve + rank, offset scan, projection / quantization / lattice
reconstruction / residual codes), input already resident in HBM.  Two forms
are timed on the same field: the plain GPU form and the full form (learned
warm start, bf16 Gram, device-driven launch).  Prints one JSON line with the
full form's throughput, the plain form's and their ratio, the roofline of the
dominant kernel (measured with HIP events on the stream the kernels run on),
and the FP64 CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c5]
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
METRIC = ("device compress GB/s at abs bound 1e-3*range (learned + mixed + batched form; "
          "ratio_vs_plain = its GB/s over the plain GPU form)")

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
    """The FP64 oracle, as it stands, on variable 0: window by window and
    z-slab by z-slab (each with the oracle's own plan), block by block in plan
    order, until ~`seconds` of CPU time; BLAS pinned to one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import dls as odls
    W = cfg["window"]
    pz = cfg["pz"] if cfg["nz"] > 1 else 1
    slabs = [(t0, z0) for t0 in range(0, cfg["nt"], W) for z0 in range(0, cfg["nz"], pz)]
    done, total, nbytes, nslab = 0, 0, 0, 0
    with threadpool_limits(limits=1):
        t0c = time.perf_counter()
        for (t0, z0) in slabs:
            w = min(W, cfg["nt"] - t0)
            sub = field[0:1, t0:t0 + w, z0:z0 + pz].cpu().numpy()
            p = odls.Params(nx=cfg["nx"], ny=cfg["ny"], nz=sub.shape[2], nt=w, nvars=1, dtype=cfg["dtype"],
                            px=cfg["px"], py=cfg["py"], pz=pz, window=w, eps=[eps[0]], pmin=cfg.get("pmin", 0),
                            adaptive=cfg.get("adaptive", False))
            blocks, _ = odls.plan(sub, p)
            total += len(blocks)
            nslab += 1
            for b in blocks:
                xb = odls.gather(sub, b)
                odls.encode_block(xb, eps[0], p.resolved_rmax(), p.np_dtype)
                done += 1
                nbytes += xb.nbytes
                if time.perf_counter() - t0c > seconds:
                    break
            if time.perf_counter() - t0c > seconds:
                break
        dt = time.perf_counter() - t0c
    return {"value": nbytes / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": "variable 0, %d window x z-slab pieces in order (each with the oracle's own plan): %d "
                      "blocks encoded, %.1f MB in %.1f s; full-workload time extrapolates at this rate"
                      % (nslab, done, nbytes / 1e6, dt)}


FORMS = {
    "plain": "FP32 Gram, full Jacobi eigensolve, host-driven launches",
    "full": "learned warm start (windows <= 16) + bf16 Gram + device-driven launch",
}


def params_for(cfg, eps, form):
    import paper_2601_20113_amd as dls
    full = form == "full"
    return dls.Params(nx=cfg["nx"], ny=cfg["ny"], nz=cfg["nz"], nt=cfg["nt"], nvars=cfg["nvars"],
                      dtype=cfg["dtype"], px=cfg["px"], py=cfg["py"], pz=cfg["pz"],
                      window=cfg["window"], eps=eps, pmin=cfg.get("pmin", 0),
                      adaptive=cfg.get("adaptive", False),
                      precision="bf16" if full else "fp32",
                      learned=full and cfg["window"] <= 16, persistent=full)


def train_model(cfg, log):
    """The warm-start network for this workload: fields of the same generator
    and block shape with seeds disjoint from the timed field's, labelled by
    the plain method, trained on the device."""
    import numpy as np
    import torch
    import paper_2601_20113_amd as dls
    from paper_2601_20113_amd import train as T
    from synth import gpu as sg
    t0 = time.perf_counter()
    enc = dls.Encoder()
    parts = []
    if cfg["kind"] == "blobs":
        data = T.collect(np.arange(100000, 100160))
    else:
        for i in range(4):
            if cfg["kind"] == "blobs_gpu":
                shape = (1, min(cfg["nt"], 48), 1, 1024, 1024)
                f = torch.empty(shape, dtype=torch.float32, device="cuda")
                sg.blobs_into(f[0], nblobs=cfg["nblobs"] * 1024 * 1024 // (cfg["nx"] * cfg["ny"]), seed=5000 + i)
            else:
                shape = (1, cfg["nt"], cfg["nz"] // 2, cfg["ny"] // 2, cfg["nx"] // 2)
                f = torch.empty(shape, dtype=torch.float32, device="cuda")
                sg.spectrum_into(f[0], seed=5000 + i, nmodes=64)
            lo, hi = dls.value_range(f)
            c = dict(cfg, nt=shape[1], nz=shape[2], ny=shape[3], nx=shape[4], nvars=1)
            parts.append(T.label_blocks(enc, f, params_for(c, [cfg["rel_eps"] * (hi[0] - lo[0])], "plain")))
            del f
        data = T.merge(parts)
    model, losses = T.fit_data(data, epochs=12, batch=512, lr=2e-3, seed=1)
    log("model: %d labelled blocks, loss %.3f -> %.3f, %.1f s"
        % (data["feat"].shape[0], losses[0], losses[-1], time.perf_counter() - t0))
    return model


def run_form(field, cfg, eps, form, steps, warmup, model, log):
    """Time `steps` encodes (after `warmup`); returns the measurements."""
    import torch
    import paper_2601_20113_amd as dls
    p = params_for(cfg, eps, form)
    enc = dls.Encoder()
    if p.learned:
        enc.set_model(model, 2, margin=1)
    stream = torch.cuda.current_stream()
    log("%s: warmup %d" % (form, warmup))
    for _ in range(warmup):
        enc.encode(field, p, stream=stream)
    torch.cuda.synchronize()
    stage = [0.0] * 5
    log("%s: timing %d steps" % (form, steps))
    t0 = time.perf_counter()
    for _ in range(steps):
        enc.encode(field, p, stream=stream)
        inf = enc.info()
        for i in range(5):
            stage[i] += inf.stage_ms[i]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return {"enc": enc, "ms": ms, "stage": [s / steps for s in stage], "info": enc.info(), "params": p}


def source_sha():
    import hashlib
    h = hashlib.sha256()
    for name in ("dls_kernels.hip", "dls_device.h", "dls_internal.h"):
        with open(os.path.join(ROOT, "paper_2601_20113_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summary, or None when the kernel sources changed
    since the counters were taken (or there is no entry)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        tab = json.load(fh)
    e = tab.get("%s/%s" % (kernel, workload))
    if not e or e.get("source_sha") != source_sha():
        return None
    return int(e["fetch_bytes"] + e["write_bytes"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c5", choices=sorted(CONFIGS))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ratio", action="store_true", help="skip the compression ratios (host zlib)")
    ap.add_argument("--forms", default="plain,full")
    ap.add_argument("--no-decode", action="store_true", help="skip the device decode measurement")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 4 GiB device-to-device copy twice (the reference the "
                         "HBM byte counters are scaled by) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.empty(1 << 30, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(2):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4, "copies": 2}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(blocks are independent; sharding is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    cfg = CONFIGS[args.config]
    forms = [f for f in args.forms.split(",") if f]
    model = None
    if "full" in forms and cfg["window"] <= 16:
        log("training the warm-start network")
        model = train_model(cfg, log)
        torch.cuda.empty_cache()
    log("generating %s" % args.config)
    field, eps = make_field(cfg)
    in_bytes = field.numel() * field.element_size()
    res = {}
    for form in forms:
        r = run_form(field, cfg, eps, form, args.steps, args.warmup, model, log)
        r["gbs"] = in_bytes / (r["ms"] * 1e-3) / 1e9
        if not args.no_ratio:
            log("%s: finalize for the compression ratio" % form)
            t1 = time.perf_counter()
            r["cr"] = in_bytes / len(r["enc"].finalize())
            log("%s: finalize %.1f s" % (form, time.perf_counter() - t1))
        res[form] = r
        log("%s: %.3f ms/step, %.1f GB/s, stages %s" % (form, r["ms"], r["gbs"], [round(s, 3) for s in r["stage"]]))
    head = res["full"] if "full" in res else res[forms[0]]
    head_form = "full" if "full" in res else forms[0]

    # roofline of the headline form's dominant kernel: algorithmic bytes per
    # launch over the launch time measured with HIP events on the encode stream
    es = field.element_size()
    nvals = field.numel()
    names = ["plan", "gram", "eigen", "scan", "encode"]
    stage = head["stage"]
    inf = head["info"]
    dom = max(range(5), key=lambda i: stage[i])
    if names[dom] == "encode":
        alg = nvals * (es + 1) + inf.qa_bytes + (inf.qv_bytes if hasattr(inf, "qv_bytes") else 0)
        kern = "k_encode"
    elif names[dom] == "gram":
        alg, kern = nvals * es, "k_gram"
    else:
        alg, kern = None, "k_" + names[dom]
    if alg is not None:
        ach = alg / (stage[dom] * 1e-3) / 1e9
        roof = {"kernel": kern, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(kern, args.config),
                "alg_bytes_per_launch": int(alg), "launch_ms": round(stage[dom], 4)}
    else:
        roof = {"kernel": kern, "bound": "alu", "achieved": None, "peak": None, "unit": "TFLOP/s",
                "frac": None, "traffic": None, "launch_ms": round(stage[dom], 4)}

    # device decode (the inverse, Alg. 2) of the headline form's last encode:
    # the context's device payload back to a field, timed with events on the
    # stream the kernels run on; every point checked against the bound
    dec = None
    if not args.no_decode:
        log("device decode of the %s form" % head_form)
        outbuf = torch.empty_like(field)
        stream = torch.cuda.current_stream()
        for _ in range(max(1, args.warmup)):
            head["enc"].decode(outbuf, stream=stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            head["enc"].decode(outbuf, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        dms = e0.elapsed_time(e1) / args.steps
        ok = True
        for v in range(field.shape[0]):
            for t in range(field.shape[1]):
                d = (outbuf[v, t].double() - field[v, t].double()).abs().max().item()
                ok = ok and d <= eps[v]
        del outbuf
        torch.cuda.empty_cache()
        # algorithmic bytes: residual codes (1 B/value) and the coefficient
        # payload read, the field written, escapes (16 B each)
        dalg = nvals * (1 + es) + inf.qa_bytes + 16 * int(inf.nescapes)
        dach = dalg / (dms * 1e-3) / 1e9
        dec = {"value": round(in_bytes / (dms * 1e-3) / 1e9, 2), "unit": "GB/s (field bytes out)",
               "ms": round(dms, 4), "bound_holds": bool(ok),
               "roofline": {"kernel": "k_decode", "bound": "hbm", "achieved": round(dach, 1), "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": round(dach / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": int(dalg)}}
        log("decode: %.3f ms, %.1f GB/s out, bound %s" % (dms, dec["value"], "holds" if ok else "VIOLATED"))

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline")
        cpu = cpu_baseline(field, cfg, eps, args.cpu_seconds)

    out = {
        "metric": METRIC, "value": round(head["gbs"], 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(head["ms"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": cfg["dtype"], "data": "synthetic",
        "config": {"workload": args.config + ": " + cfg["desc"], "form": head_form + ": " + FORMS[head_form],
                   "input_bytes": in_bytes, "blocks": int(inf.nblocks)},
        "stage_ms": {n: round(s, 4) for n, s in zip(names, stage)},
        "compression_ratio": None if "cr" not in head else round(head["cr"], 3),
        "escapes": int(inf.nescapes),
        "warm_start_accepted": int(inf.nwarm_accept) if head["params"].learned else None,
        "roofline": roof,
        "cpu_baseline": cpu,
        "decode": dec,
    }
    if "plain" in res and head_form != "plain":
        pl = res["plain"]
        out["plain"] = {"value": round(pl["gbs"], 2), "ms_per_step": round(pl["ms"], 3),
                        "stage_ms": {n: round(s, 4) for n, s in zip(names, pl["stage"])},
                        "compression_ratio": None if "cr" not in pl else round(pl["cr"], 3)}
        out["ratio_vs_plain"] = round(head["gbs"] / pl["gbs"], 4)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
