"""Launch-strategy autotuner with a JSON cache.

The encode's results do not depend on how its kernels are launched, only
its time does: the device-driven encode (no host round trip, looping
workgroups over device-written lists) against the host-driven one (one
workgroup per slice, sized from a readback), with or without graph replay.
The crossover between the two depends on the plan (slice count and size
mix), so this module times the choices on the caller's own workload and
keeps the fastest per workload signature (grid, dtype, patch, window,
flags, precision) in a JSON file.  Every candidate writes the same stream
(checked here on every tuning run).
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Optional

import torch

from . import Encoder, Params

# candidate device-driven limits (slices): 0 = always host-driven
LIMITS = (0, 1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 31)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "dls_autotune.json")


def signature(p: Params) -> str:
    """The workload key of a choice."""
    return "%s|%dx%dx%dx%d|v%d|p%dx%dx%d|w%d|pmin%d|a%d|l%d|ps%d|l2%d|g%d|%s" % (
        p.dtype, p.nx, p.ny, p.nz, p.nt, p.nvars, p.px, p.py, p.pz, p.window, p.pmin, int(p.adaptive),
        int(p.learned), int(p.persistent), int(p.l2), int(p.global_basis), p.precision)


def _load(path: str) -> Dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def apply(enc: Encoder, choice: Dict) -> None:
    enc.set_launch(int(choice["device_driven_max_items"]))
    enc.set_graphs(bool(choice["graphs"]))


def tune(field: torch.Tensor, p: Params, enc: Encoder, reps: int = 5, cache: Optional[str] = DEFAULT_CACHE,
         retune: bool = False, check_streams: bool = True) -> Dict:
    """Times every (device-driven limit, graphs) candidate on `field` with
    `enc` (its model, if any, stays attached), checks that all of them
    write the same stream (unless check_streams is False), stores and
    returns the fastest:
    {"device_driven_max_items", "graphs", "ms", "candidates": {...}}."""
    key = signature(p)
    tab = _load(cache) if cache else {}
    if not retune and key in tab:
        apply(enc, tab[key])
        return tab[key]
    ref = None
    res = {}
    for limit in LIMITS:
        for graphs in (True, False):
            enc.set_launch(limit)
            enc.set_graphs(graphs)
            enc.encode(field, p)
            if check_streams:
                stream = enc.finalize()
                if ref is None:
                    ref = stream
                elif stream != ref:
                    raise RuntimeError("launch strategy changed the stream (limit %d, graphs %d)" % (limit, graphs))
            for _ in range(2):
                enc.encode(field, p)
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                enc.encode(field, p)
                torch.cuda.synchronize()
                ts.append((time.perf_counter() - t0) * 1e3)
            ts.sort()
            res["%d/%d" % (limit, int(graphs))] = ts[len(ts) // 2]
    best = min(res, key=res.get)
    limit, graphs = best.split("/")
    choice = {"device_driven_max_items": int(limit), "graphs": bool(int(graphs)), "ms": round(res[best], 4),
              "candidates": {k: round(v, 4) for k, v in res.items()}}
    if cache:
        tab = _load(cache)
        tab[key] = choice
        d = os.path.dirname(cache)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(cache + ".tmp", "w") as fh:
            json.dump(tab, fh, indent=1, sort_keys=True)
        os.replace(cache + ".tmp", cache)
    apply(enc, choice)
    return choice
