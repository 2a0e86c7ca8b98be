#!/usr/bin/env python
"""Device compression throughput of the DLS hot path on one MI355X.

One step = one dls_encode over the whole synthetic field (plan, Gram,
eigensolve + rank, offset scan, projection / quantization / lattice
reconstruction / residual codes), input already resident in HBM.  Two forms
are timed on the same field: the plain GPU form (FP32 Gram, Jacobi, one
host-driven launch per class) and the full form (bf16 Gram, the batched
launch -- on plans of large FP32 blocks the single pass --, the learned warm
start where blocks are small enough for it).  Prints one JSON line with the
full form's throughput, the plain form's and their ratio, the label of what
actually ran, the roofline of the dominant kernel (its launch timed with HIP
events on the stream the kernels run on), end-to-end throughput (+ device to
host copy and host zlib), the decode, error statistics of the decoded field,
and the FP64 CPU oracle timed on a bounded sample of the same workload on the
host's cores.

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


def _oracle_piece(args):
    """Worker: the FP64 oracle on one piece of variable 0 (its own plan),
    block by block, until the shared deadline; BLAS pinned to one thread.
    Returns (bytes encoded, blocks, busy seconds)."""
    piece, pkw, eps0, deadline = args
    from threadpoolctl import threadpool_limits
    from oracle import dls as odls
    t0 = time.time()
    nbytes = nblk = 0
    with threadpool_limits(limits=1):
        if t0 < deadline:
            p = odls.Params(eps=[eps0], **pkw)
            blocks, _ = odls.plan(piece, p)
            for b in blocks:
                if time.time() >= deadline:
                    break
                xb = odls.gather(piece, b)
                odls.encode_block(xb, eps0, p.resolved_rmax(), p.np_dtype)
                nbytes += xb.nbytes
                nblk += 1
    return nbytes, nblk, time.time() - t0


def host_cores():
    """Cores this process may use, at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_pool():
    """Worker processes for the oracle timing, forked before the GPU is
    touched (a child of a process that holds the device never uses it)."""
    import multiprocessing as mp
    n = host_cores()
    return mp.get_context("fork").Pool(n), n


def cpu_baseline(pool, ncores, field, cfg, eps, seconds):
    """The FP64 oracle, as it stands, on `ncores` processes: pieces of
    variable 0 (window x z-slab x a strip of py rows, each planned by the
    oracle on its own), block by block, until ~`seconds` of wall time."""
    W = cfg["window"]
    pz = cfg["pz"] if cfg["nz"] > 1 else 1
    py = cfg["py"]
    keys = [(t0, z0, y0) for t0 in range(0, cfg["nt"], W) for z0 in range(0, cfg["nz"], pz)
            for y0 in range(0, cfg["ny"], py)]
    keys = keys[:8 * ncores]
    tasks = []
    for (t0, z0, y0) in keys:
        w = min(W, cfg["nt"] - t0)
        piece = field[0:1, t0:t0 + w, z0:z0 + pz, y0:y0 + py].cpu().numpy()
        pkw = dict(nx=cfg["nx"], ny=piece.shape[3], nz=piece.shape[2], nt=w, nvars=1, dtype=cfg["dtype"],
                   px=cfg["px"], py=py, pz=pz, window=w, pmin=cfg.get("pmin", 0),
                   adaptive=cfg.get("adaptive", False))
        tasks.append([piece, pkw, float(eps[0]), None])
    t0w = time.time()
    deadline = t0w + seconds
    for t in tasks:
        t[3] = deadline
    res = pool.map(_oracle_piece, [tuple(t) for t in tasks], chunksize=1)
    wall = time.time() - t0w
    nbytes = sum(r[0] for r in res)
    nblk = sum(r[1] for r in res)
    busy = sum(r[2] for r in res)
    return {"value": round(nbytes / wall / 1e9, 5), "unit": "GB/s", "cores": ncores, "kind": "oracle",
            "value_per_core": round(nbytes / max(busy, 1e-9) / 1e9, 5),
            "os_cpu_count": os.cpu_count(), "cpu_model": cpu_model(), "blas_threads_per_process": 1,
            "sample": "variable 0: %d pieces (%d-step window x %d-deep z-slab x %d-row y strip, whole x), "
                      "each planned by the oracle on its own, on %d processes; %d blocks encoded, %.1f MB in "
                      "%.1f s wall; the full workload extrapolates at this rate"
                      % (len(tasks), W, pz, py, ncores, nblk, nbytes / 1e6, wall)}


def smallest_block_points(cfg):
    """Points of the plan's smallest possible block: the finest leaf
    (adaptive) or the patch, truncated where the grid ends mid-patch."""
    pts = 1
    for n, pk in ((cfg["nx"], "px"), (cfg["ny"], "py"), (cfg["nz"], "pz")):
        if n == 1:
            continue
        ext = cfg.get("pmin", 0) if cfg.get("adaptive") else cfg[pk]
        ext = ext or cfg[pk]
        pts *= min(ext, n % ext) if n % ext else ext
    return pts


def learned_applies(cfg):
    """The warm start serves windows of <= 16 steps and blocks of at most
    WARM_MAX_POINTS points; on a plan without such blocks it never runs."""
    import paper_2601_20113_amd as dls
    return cfg["window"] <= 16 and smallest_block_points(cfg) <= dls.WARM_MAX_POINTS


def params_for(cfg, eps, form):
    import paper_2601_20113_amd as dls
    full = form == "full"
    return dls.Params(nx=cfg["nx"], ny=cfg["ny"], nz=cfg["nz"], nt=cfg["nt"], nvars=cfg["nvars"],
                      dtype=cfg["dtype"], px=cfg["px"], py=cfg["py"], pz=cfg["pz"],
                      window=cfg["window"], eps=eps, pmin=cfg.get("pmin", 0),
                      adaptive=cfg.get("adaptive", False),
                      precision="bf16" if full else "fp32",
                      learned=full and learned_applies(cfg), persistent=full)


LAUNCH = {0: "host-driven launches (one per rank class and slice class)",
          1: "device-driven launch (device-written class lists, one readback)"}


def form_label(form, cfg, p, inf):
    """What the encode actually ran, from its own counters."""
    parts = ["bf16 Gram operands (FP32 MFMA accumulate, FP64 across chunks)" if p.precision == "bf16"
             else "FP32 Gram"]
    if inf.launch_mode == 2:
        parts.append("single pass: %d of %d blocks verified at rank 1 on the sketch basis and encoded in the "
                     "same read, %d deferred to Jacobi and a second read" % (inf.nfast_accept, inf.nblocks,
                                                                            inf.ndeferred))
    else:
        if inf.fused_declined:
            parts.append("single pass declined: the first slices predict %d of %d blocks to fail rank 1 (%d "
                         "proven), so two-pass" % (inf.npredicted_deferred, inf.nblocks, inf.npruned))
        parts.append("Jacobi eigensolve; " + LAUNCH[inf.launch_mode])
    if p.learned:
        parts.append("learned warm start: %d blocks accepted, %d to Jacobi" % (inf.nwarm_accept, inf.nwarm_reject))
    elif form == "full":
        parts.append("no learned warm start (%s)" % (
            "windows above 16 steps" if cfg["window"] > 16 else
            "smallest block %d points > %d" % (smallest_block_points(cfg), 256)))
    return form + ": " + "; ".join(parts)


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


def run_learned(log, n_train=200000, reps=7):
    """The learned warm start at its configured size: the network trained on
    n_train blocks that the plain GPU method encodes from config-1 fields
    (seed A = 100000 + i), evaluated on 256 unseen config-1 fields (seed B =
    200000 + i) against the plain eigensolve and a fixed (non-learned) guess
    of the same warm start; eigensolve-stage times are medians of `reps`
    encodes."""
    import numpy as np
    import torch
    import paper_2601_20113_amd as dls
    from paper_2601_20113_amd import train as T
    t0 = time.perf_counter()
    nf = (n_train + 127) // 128
    model, data, losses = T.fit(np.arange(100000, 100000 + nf), epochs=12, batch=512, lr=2e-3, seed=1)
    train_s = time.perf_counter() - t0
    f, eps = T.c1_fields(np.arange(200000, 200256))
    nv, nt, nz, ny, nx = f.shape
    t = torch.from_numpy(f).cuda()
    base = dict(nx=nx, ny=ny, nz=nz, nt=nt, nvars=nv, dtype="f64", px=8, py=8, pz=1, window=16, eps=eps)
    enc = dls.Encoder()

    def timed(p):
        enc.encode(t, p)
        ms = []
        for _ in range(reps):
            enc.encode(t, p)
            ms.append(enc.info().stage_ms[2])
        inf = enc.info()
        ranks = dls.d2h(inf.d_rank, inf.nblocks).copy()
        return float(np.median(ms)), inf, ranks, len(enc.finalize())

    ms_p, inf_p, r_p, n_p = timed(dls.Params(**base))
    enc.set_model(model, 2, margin=1)
    ms_l, inf_l, r_l, n_l = timed(dls.Params(**base, learned=True))
    fixed = dls.Model()
    P = np.zeros(dls.NPARAM, np.float32)
    ob3 = 80 * 128 + 128 + 128 * 128 + 128 + 128 * 272
    P[ob3 + 2] = 10.0  # rank 3 for every block, the identity's first columns as the guess
    for k in range(16):
        P[ob3 + 16 + 17 * k] = 1.0
    fixed.set(P, np.concatenate([np.zeros(16), np.ones(16)]).astype(np.float32))
    enc.set_model(fixed, 2, margin=0)
    ms_f, inf_f, r_f, n_f = timed(dls.Params(**base, learned=True))
    enc.close()
    nb = int(inf_p.nblocks)
    e = {"workload": "config 4: MLP 3 x 128, trained on %d labelled blocks of config-1 fields (seed A), "
                     "evaluated on 256 config-1 fields (seed B, %d blocks)" % (int(data["feat"].shape[0]), nb),
         "train_s": round(train_s, 2), "loss_first": round(losses[0], 4), "loss_last": round(losses[-1], 4),
         "eigen_ms": {"plain": round(ms_p, 4), "learned": round(ms_l, 4), "fixed_guess": round(ms_f, 4)},
         "warm_accepted": {"learned": int(inf_l.nwarm_accept), "fixed_guess": int(inf_f.nwarm_accept)},
         "rank_agreement_with_plain": round(float(np.mean(r_p == r_l)), 4),
         "mean_rank": {"plain": round(float(np.mean(r_p)), 3), "learned": round(float(np.mean(r_l)), 3),
                       "fixed_guess": round(float(np.mean(r_f)), 3)},
         "compression_ratio": {"plain": round(f.nbytes / n_p, 3), "learned": round(f.nbytes / n_l, 3),
                               "fixed_guess": round(f.nbytes / n_f, 3)}}
    log("learned (config 4): %s" % e)
    return e


def run_form(field, cfg, eps, form, steps, warmup, model, log):
    """Time `steps` encodes (after `warmup`) between device synchronizations;
    returns the wall time per step and the averages of the library's own
    HIP-event times (stages, the fused kernel, the Jacobi launch)."""
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
    fused = jac = 0.0
    log("%s: timing %d steps" % (form, steps))
    t0 = time.perf_counter()
    for _ in range(steps):
        enc.encode(field, p, stream=stream)
        inf = enc.info()
        for i in range(5):
            stage[i] += inf.stage_ms[i]
        fused += inf.fused_ms
        jac += inf.jacobi_ms
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return {"enc": enc, "ms": ms, "stage": [s / steps for s in stage], "fused_ms": fused / steps,
            "jacobi_ms": jac / steps, "info": enc.info(), "params": p,
            "label": form_label(form, cfg, p, enc.info())}


KERNEL_SOURCES = {"k_fused": "dls_codec.hip", "k_encode": "dls_codec.hip", "k_decode": "dls_codec.hip",
                  "k_gram": "dls_kernels.hip", "k_eigen": "dls_kernels.hip"}


def source_sha(kernel):
    """Hash of the sources a kernel is compiled from (its file and the
    shared device headers)."""
    import hashlib
    h = hashlib.sha256()
    for name in (KERNEL_SOURCES[kernel], "dls_kernels.h", "dls_device.h", "dls_internal.h"):
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
    if not e or kernel not in KERNEL_SOURCES or e.get("source_sha") != source_sha(kernel):
        return None
    return int(e["fetch_bytes"] + e["write_bytes"])


FP64_PEAK_TFLOPS = 78.6


def block_shapes(inf):
    """(points M_b, window W_b) of every block, from the device descriptors."""
    import numpy as np
    import paper_2601_20113_amd as dls
    desc = dls.d2h(inf.d_desc, inf.nblocks * 32).view(np.int32).reshape(inf.nblocks, 8)
    return desc[:, 6].astype(np.int64), ((desc[:, 4].astype(np.int64) >> 24) & 255)


def pad16(x):
    return (x + 15) // 16 * 16


def jacobi_stats(r):
    """Sweeps, unconverged blocks and the FP64 rate of the Jacobi launch
    (9 wpad^2 (wpad - 1) flops per sweep of order wpad)."""
    inf = r["info"]
    wp = inf.wpad
    flops = inf.jacobi_sweeps * 9 * wp * wp * (wp - 1)
    ms = r["jacobi_ms"]
    tf = flops / (ms * 1e-3) / 1e12 if ms > 0 else None
    return {"sweeps": int(inf.jacobi_sweeps), "unconverged": int(inf.jacobi_unconverged),
            "ms": round(ms, 4), "flops": int(flops), "achieved_tflops": None if tf is None else round(tf, 3),
            "peak_tflops": FP64_PEAK_TFLOPS, "frac": None if tf is None else round(tf / FP64_PEAK_TFLOPS, 4)}


def roofline(r, field, workload):
    """Roofline of the form's dominant kernel: algorithmic bytes (or flops)
    per launch over the launch's own HIP-event time on the encode stream."""
    import numpy as np
    import paper_2601_20113_amd as dls
    inf, stage = r["info"], r["stage"]
    es, nvals = field.element_size(), field.numel()
    in_bytes = nvals * es
    m, w = block_shapes(inf)
    if inf.launch_mode == 2 and r["fused_ms"] > 0:
        # the fused kernel reads the field once and writes every value's
        # residual code and every block's rank-1 qA and qV
        alg = in_bytes + nvals + int(np.sum(4 * pad16(m) + 4 * pad16(w)))
        kern, ms = "k_fused", r["fused_ms"]
        note = ("field read once + 1 B code per value + rank-1 qA (4 B per point) and qV of every block; "
                "the 2 KiB FP64 Gram partial per slice is not counted")
    else:
        cand = {"k_gram": stage[1], "k_eigen": r["jacobi_ms"], "k_encode": stage[4]}
        kern = max(cand, key=cand.get)
        ms = cand[kern]
        if kern == "k_eigen":
            j = jacobi_stats(r)
            return {"kernel": kern, "bound": "alu", "achieved": j["achieved_tflops"], "peak": FP64_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": j["frac"], "traffic": None, "alg_flops_per_launch": j["flops"],
                    "launch_ms": j["ms"], "note": "FP64 vector peak; 9 wpad^2 (wpad-1) flops per sweep taken"}
        if kern == "k_gram":
            alg, note = in_bytes, "field read once"
        else:
            rank = dls.d2h(inf.d_rank, inf.nblocks).astype(np.int64)
            alg = nvals * (es + 1) + inf.qa_bytes + int(np.sum(4 * pad16(w * rank)))
            note = "field read + 1 B code per value + qA + qV (all rank-class launches of the stage)"
    ach = alg / (ms * 1e-3) / 1e9
    return {"kernel": kern, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(kern, workload),
            "alg_bytes_per_launch": int(alg), "launch_ms": round(ms, 4), "note": note}


def error_stats(field, out, eps, rel_eps):
    """Per variable, over every point: max |x - x_hat| / eps and the NRMSE
    (root-mean-square error over the variable's range), on the device in FP64."""
    res = []
    for v in range(field.shape[0]):
        mx, se, n = 0.0, 0.0, 0
        for t in range(field.shape[1]):
            d = out[v, t].double() - field[v, t].double()
            fin = d.isfinite()
            d = d.masked_fill(~fin, 0.0)
            mx = max(mx, d.abs().max().item())
            se += (d * d).sum().item()
            n += int(fin.sum().item())
        rng = eps[v] / rel_eps
        res.append({"max_abs_err_over_eps": round(mx / eps[v], 6), "within_eps": bool(mx <= eps[v]),
                    "nrmse": float("%.6g" % (math.sqrt(se / max(n, 1)) / rng))})
    return res


def nrmse(field, out):
    """Per variable, ||u - u_hat|| / ||u|| over the finite values (the NRMSE
    of Sec. 2.4 as a fraction), on the device in FP64."""
    res = []
    for v in range(field.shape[0]):
        se = ss = 0.0
        for t in range(field.shape[1]):
            x = field[v, t].double()
            fin = x.isfinite()
            d = (out[v, t].double() - x).masked_fill(~fin, 0.0)
            x = x.masked_fill(~fin, 0.0)
            se += (d * d).sum().item()
            ss += (x * x).sum().item()
        res.append(math.sqrt(se / ss) if ss > 0 else 0.0)
    return res


def run_l2(field, cfg, targets, steps, warmup, no_ratio, log):
    """The L2 / NRMSE-bounded mode (Sec. 2.4) on the same field: per target,
    the encode time (wall, between synchronizations), the passes it took,
    the decoded field's NRMSE per variable and the compression ratio."""
    import torch
    import paper_2601_20113_amd as dls
    in_bytes = field.numel() * field.element_size()
    curve = []
    stream = torch.cuda.current_stream()
    for tg in targets:
        p = dls.Params(nx=cfg["nx"], ny=cfg["ny"], nz=cfg["nz"], nt=cfg["nt"], nvars=cfg["nvars"],
                       dtype=cfg["dtype"], px=cfg["px"], py=cfg["py"], pz=cfg["pz"], window=cfg["window"],
                       eps=[tg] * cfg["nvars"], pmin=cfg.get("pmin", 0), adaptive=cfg.get("adaptive", False),
                       l2=True)
        enc = dls.Encoder()
        for _ in range(warmup):
            enc.encode(field, p, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            enc.encode(field, p, stream=stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        inf = enc.info()
        out = torch.empty_like(field)
        enc.decode(out, stream=stream)
        torch.cuda.synchronize()
        nr = nrmse(field, out)
        del out
        e = {"target": tg, "ms": round(ms, 3), "value": round(in_bytes / (ms * 1e-3) / 1e9, 2), "unit": "GB/s",
             "passes": int(inf.l2_passes), "raw_blocks": int(inf.nraw),
             "nrmse": [float("%.4g" % x) for x in nr], "within_target": bool(all(x <= tg for x in nr)),
             "stage_ms": {"gram": round(inf.stage_ms[1], 4), "eigen": round(inf.stage_ms[2], 4),
                          "encode+check": round(inf.stage_ms[4], 4)}}
        # the two field reads of the mode: the FP64 Gram (with the norm) and
        # the encode; HIP-event time of each stage on the launch stream
        gb = in_bytes  # the field read once
        ach_g = gb / (inf.stage_ms[1] * 1e-3) / 1e9
        eb = in_bytes + int(inf.qa_bytes)
        ach_e = eb / (inf.stage_ms[4] * 1e-3) / 1e9
        e["roofline"] = {"gram": {"kernel": "k_l2_gram (+ k_l2_fsq_part, k_l2_budget)", "bound": "hbm",
                                  "achieved": round(ach_g, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": round(ach_g / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": int(gb)},
                         "encode": {"kernel": "k_l2_encode (+ k_l2_params, scans, k_l2_check)", "bound": "hbm",
                                    "achieved": round(ach_e, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": round(ach_e / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": int(eb)}}
        if not no_ratio:
            t1 = time.perf_counter()
            e["compression_ratio"] = round(in_bytes / len(enc.finalize()), 3)
            e["finalize_s"] = round(time.perf_counter() - t1, 3)
        enc.close()
        torch.cuda.empty_cache()
        log("l2 %g: %.3f ms, %.1f GB/s, %d passes, NRMSE %s, CR %s" % (tg, ms, e["value"], e["passes"], e["nrmse"],
                                                                     e.get("compression_ratio")))
        curve.append(e)
    return {"workload": "the headline field", "what": "L2 / NRMSE-bounded mode (DLS_L2): per-variable target "
            "eps_t on ||u - u_hat|| / ||u||, FP64 Gram, rank by the eigenvalue tail, exact block error check",
            "curve": curve}


def global_params(nx, ny, nt, px, target, kind, seed=1):
    import paper_2601_20113_amd as dls
    return dls.Params(nx=nx, ny=ny, nz=1, nt=nt, nvars=1, dtype="f32", px=px, py=px, pz=1, window=1,
                      eps=[target], global_basis=True, basis=kind, seed=seed)


def run_global_one(field, p, steps, warmup, no_ratio):
    """Encode time (wall, between synchronizations), stage times, kept
    coefficients, NRMSE and compression ratio of one global-basis setting."""
    import torch
    import paper_2601_20113_amd as dls
    enc = dls.Encoder()
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        enc.encode(field, p, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        enc.encode(field, p, stream=stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    inf = enc.info()
    out = torch.empty_like(field)
    enc.decode(out, stream=stream)
    torch.cuda.synchronize()
    nr = nrmse(field, out)[0]
    del out
    in_bytes = field.numel() * field.element_size()
    e = {"ms": round(ms, 3), "value": round(in_bytes / (ms * 1e-3) / 1e9, 2), "unit": "GB/s",
         "nrmse": float("%.4g" % nr), "within_target": bool(nr <= p.eps[0]),
         "learn_ms": round(inf.jacobi_ms, 3), "jacobi_sweeps": int(inf.jacobi_sweeps),
         "stage_ms": {"budget+basis": round(inf.stage_ms[1], 3), "coefficients": round(inf.stage_ms[2], 3),
                      "selection": round(inf.stage_ms[3], 3), "pack": round(inf.stage_ms[4], 3)},
         "raw_patches": int(inf.nraw)}
    # the payload holds 6 bytes per kept coefficient (index, value) and the
    # raw patches' values
    m = p.px * p.py * p.pz
    kept = (inf.qa_bytes - inf.nraw * m * field.element_size()) / 6.0
    e["mean_kept"] = round(kept / max(inf.nblocks - inf.nraw, 1), 2)
    if not no_ratio:
        buf = enc.finalize()
        e["compression_ratio"] = round(in_bytes / len(buf), 3)
    enc.close()
    return e


def run_global(steps, warmup, no_ratio, log):
    """The paper's global-basis method (Alg. 1) on 2D FP32 blob fields:
    throughput on the 4096 x 2048 x 100 field with 8 x 8 patches and the
    learned (SVD) basis at NRMSE 1e-3, and the basis study of Sec. 4 (SVD,
    cosine and random bases; patch edges 4, 8, 16; NRMSE 1e-2 and 1e-3) on a
    1024 x 1024 x 16 field of the same generator."""
    import torch
    from synth import gpu as sg
    res = {"what": "global-basis mode (DLS_GLOBAL): one basis per variable learned from 4M random patches of "
                   "snapshot 0, every patch of every snapshot projected on it, coefficients kept in decreasing "
                   "magnitude until the local L2 share holds, power-of-two grooming, exact error check"}
    f = torch.empty((1, 100, 1, 2048, 4096), dtype=torch.float32, device="cuda")
    sg.blobs_into(f[0], nblobs=8192, seed=31)
    p = global_params(4096, 2048, 100, 8, 1e-3, "svd")
    e = run_global_one(f, p, steps, warmup, no_ratio)
    log("global 4096x2048x100 svd 8x8 1e-3: %s" % e)
    res["throughput"] = dict(e, workload="2D FP32 4096x2048 x 100 steps, 8192 moving Gaussian blobs, 8x8 patches, "
                                         "SVD basis, NRMSE 1e-3")
    # the launch-strategy autotuner on the same field as the quadtree
    # workload (absolute bound, bf16 Gram, batched form without a model)
    import paper_2601_20113_amd as dls
    from paper_2601_20113_amd import autotune
    c3 = CONFIGS["c3"]
    lo, hi = dls.value_range(f)
    pq = params_for(dict(c3), [c3["rel_eps"] * (hi[0] - lo[0])], "full")
    pq.learned = False
    enc = dls.Encoder()
    choice = autotune.tune(f, pq, enc, reps=3, cache=None, check_streams=True)
    enc.close()
    log("launch tuning on the quadtree workload: %s" % choice)
    res["launch_tuning"] = dict(choice, workload="c3 field, absolute bound 1e-3*range, quadtree, bf16 Gram, batched "
                                                "form without the warm start",
                                what="time per encode (median of 3) for each device-driven limit (slices) / graph "
                                     "replay; every candidate wrote the same stream")
    del f
    torch.cuda.empty_cache()
    g = torch.empty((1, 16, 1, 1024, 1024), dtype=torch.float32, device="cuda")
    sg.blobs_into(g[0], nblobs=1024, seed=41)
    study = []
    for px in (4, 8, 16):
        for kind in ("svd", "cosine", "random"):
            for tg in (1e-2, 1e-3):
                e = run_global_one(g, global_params(1024, 1024, 16, px, tg, kind), 1, 1, no_ratio)
                e.update(patch=px, basis=kind, target=tg)
                log("basis study %s %dx%d %g: CR %s NRMSE %s kept %s" % (kind, px, px, tg,
                                                                        e.get("compression_ratio"), e["nrmse"],
                                                                        e.get("mean_kept")))
                study.append(e)
    res["basis_study"] = {"workload": "2D FP32 1024x1024 x 16 steps, 1024 moving Gaussian blobs",
                          "rows": study}
    del g
    torch.cuda.empty_cache()
    return res


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
    ap.add_argument("--no-drift", action="store_true",
                    help="skip the drift variant (modes with a per-step phase drift) of the spectrum workloads")
    ap.add_argument("--l2-targets", default="1e-2,1e-3,1e-4",
                    help="NRMSE targets of the L2-bounded mode measured on the headline field (empty: skip)")
    ap.add_argument("--no-global", action="store_true",
                    help="skip the global-basis mode (its throughput and the basis study)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned warm start at its configured training size")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 4 GiB device-to-device copy twice (the reference the "
                         "HBM byte counters are scaled by) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (blocks are independent; "
              "a multi-GPU run would give each GPU a contiguous range of windows or z-slabs)", file=sys.stderr)
        sys.exit(2)
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

    # the oracle's worker processes start before anything touches the GPU
    pool, ncores = (None, 0) if args.no_cpu_baseline else cpu_pool()
    # host threads of the back-end (device-to-host copy, zlib per batch)
    os.environ.setdefault("DLS_HOST_THREADS", str(host_cores()))
    import torch
    cfg = CONFIGS[args.config]
    forms = [f for f in args.forms.split(",") if f]
    model = None
    if "full" in forms and learned_applies(cfg):
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
            log("%s: finalize (device-to-host copy + host zlib) for the compression ratio" % form)
            t1 = time.perf_counter()
            r["cr"] = in_bytes / len(r["enc"].finalize())
            r["finalize_s"] = time.perf_counter() - t1
            log("%s: finalize %.2f s" % (form, r["finalize_s"]))
        res[form] = r
        log("%s: %.3f ms/step, %.1f GB/s, stages %s, fused %.3f ms, jacobi %.3f ms; %s"
            % (form, r["ms"], r["gbs"], [round(x, 3) for x in r["stage"]], r["fused_ms"], r["jacobi_ms"],
               r["label"]))
    head_form = "full" if "full" in res else forms[0]
    head = res[head_form]
    inf = head["info"]
    roof = roofline(head, field, args.config)
    names = ["plan", "gram", "eigen", "scan", "encode"]

    # device decode (the inverse, Alg. 2) of the headline form's last encode:
    # the context's device payload back to a field, timed with events on the
    # stream the kernels run on; every point checked against the bound
    dec, err = None, None
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
        err = error_stats(field, outbuf, eps, cfg["rel_eps"])
        ok = all(e["within_eps"] for e in err)
        del outbuf
        torch.cuda.empty_cache()
        # algorithmic bytes: residual codes (1 B/value) and the coefficient
        # payload read, the field written, escapes (16 B each)
        nvals = field.numel()
        dalg = nvals * (1 + field.element_size()) + inf.qa_bytes + 16 * int(inf.nescapes)
        dach = dalg / (dms * 1e-3) / 1e9
        dec = {"value": round(in_bytes / (dms * 1e-3) / 1e9, 2), "unit": "GB/s (field bytes out)",
               "ms": round(dms, 4), "bound_holds": bool(ok),
               "roofline": {"kernel": "k_decode", "bound": "hbm", "achieved": round(dach, 1), "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": round(dach / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": int(dalg),
                            "traffic": measured_traffic("k_decode", args.config)}}
        log("decode: %.3f ms, %.1f GB/s out, bound %s, error %s" % (dms, dec["value"], "holds" if ok else "VIOLATED",
                                                                  err))

    cpu = None
    if pool is not None:
        log("cpu baseline: the FP64 oracle on %d processes" % ncores)
        cpu = cpu_baseline(pool, ncores, field, cfg, eps, args.cpu_seconds)
        pool.close()
        pool.join()
        log("cpu baseline: %s" % cpu)

    out = {
        "metric": METRIC, "value": round(head["gbs"], 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(head["ms"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": cfg["dtype"], "data": "synthetic",
        "config": {"workload": args.config + ": " + cfg["desc"], "form": head["label"],
                   "input_bytes": in_bytes, "blocks": int(inf.nblocks)},
        "stage_ms": {n: round(x, 4) for n, x in zip(names, head["stage"])},
        "kernel_ms": {"k_fused": round(head["fused_ms"], 4), "k_eigen": round(head["jacobi_ms"], 4)},
        "compression_ratio": None if "cr" not in head else round(head["cr"], 3),
        "escapes": int(inf.nescapes),
        "warm_start_accepted": int(inf.nwarm_accept) if head["params"].learned else None,
        "roofline": roof,
        "jacobi": jacobi_stats(head),
        "end_to_end": None if "finalize_s" not in head else {
            "value": round(in_bytes / (head["ms"] * 1e-3 + head["finalize_s"]) / 1e9, 3), "unit": "GB/s",
            "finalize_s": round(head["finalize_s"], 3), "host_threads": int(os.environ["DLS_HOST_THREADS"]),
            "what": "device encode + device-to-host copy of the payload + host zlib (level 6, 1000-block "
                    "batches) + container"},
        "error": err,
        "decode": dec,
        "cpu_baseline": cpu,
    }
    if "plain" in res and head_form != "plain":
        pl = res["plain"]
        out["plain"] = {"value": round(pl["gbs"], 2), "ms_per_step": round(pl["ms"], 3), "form": pl["label"],
                        "stage_ms": {n: round(x, 4) for n, x in zip(names, pl["stage"])},
                        "roofline": roofline(pl, field, args.config), "jacobi": jacobi_stats(pl),
                        "compression_ratio": None if "cr" not in pl else round(pl["cr"], 3)}
        out["ratio_vs_plain"] = round(head["gbs"] / pl["gbs"], 4)
    for r in res.values():
        r["enc"].close()
    res.clear()
    torch.cuda.empty_cache()

    targets = [float(x) for x in args.l2_targets.split(",") if x]
    if targets:
        out["l2"] = run_l2(field, cfg, targets, min(args.steps, 3), 1, args.no_ratio, log)
    if not args.no_global:
        del field
        torch.cuda.empty_cache()
        out["global"] = run_global(min(args.steps, 3), 1, args.no_ratio, log)
        field = None

    if not args.no_learned:
        field = None
        torch.cuda.empty_cache()
        out["learned"] = run_learned(log)

    # the drift variant: every mode's phase advances per step, so windows
    # have ranks above 1 (the literal generator is rank 1 in time)
    if cfg["kind"] == "spectrum" and not args.no_drift:
        field = None
        torch.cuda.empty_cache()
        dcfg = dict(cfg, drift=True)
        log("generating the drift variant of %s" % args.config)
        field, deps = make_field(dcfg)
        drift = {"workload": "the same with a per-step phase drift of every mode (U[0, 0.2] rad/step)"}
        for form in forms:
            r = run_form(field, dcfg, deps, form, args.steps, args.warmup, model, log)
            r["gbs"] = in_bytes / (r["ms"] * 1e-3) / 1e9
            e = {"value": round(r["gbs"], 2), "ms_per_step": round(r["ms"], 3), "form": r["label"],
                 "stage_ms": {n: round(x, 4) for n, x in zip(names, r["stage"])},
                 "roofline": roofline(r, field, args.config + "-drift"), "jacobi": jacobi_stats(r)}
            if not args.no_ratio and form == head_form:
                e["compression_ratio"] = round(in_bytes / len(r["enc"].finalize()), 3)
            log("drift %s: %.3f ms/step, %.1f GB/s; %s" % (form, r["ms"], r["gbs"], r["label"]))
            drift[form] = e
            r["enc"].close()
        if "plain" in drift and head_form in drift and head_form != "plain":
            drift["ratio_vs_plain"] = round(drift[head_form]["value"] / drift["plain"]["value"], 4)
        out["drift"] = drift
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
