"""Train the warm-start network on the GPU.

The plain method labels the data: every training field is encoded with the
plain GPU path, and each block contributes (features -> rank r, leading
basis columns).  Training uses the library's forward, backward and Adam
kernels; this module only moves tensors around.

    python -m paper_2601_20113_amd.train --n-train 200000 --out model.npz
"""
from __future__ import annotations

import argparse
import math
import time

import numpy as np
import torch

import paper_2601_20113_amd as dls
import synth

W1_SHAPE, W2_SHAPE, W3_SHAPE = (80, 128), (128, 128), (128, 272)


def he_init(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, flat FP32."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in (W1_SHAPE, W2_SHAPE, W3_SHAPE):
        parts.append(rng.normal(0.0, math.sqrt(2.0 / shape[0]), size=shape).ravel())
        parts.append(np.zeros(shape[1]))
    return np.concatenate(parts).astype(np.float32)


def c1_fields(seeds, nx=64, ny=64, nt=32):
    """Stack config-1 fields (one variable per seed) and their 1e-3 * range bounds."""
    f = np.concatenate([synth.blobs2d(nx=nx, ny=ny, nt=nt, seed=int(s)) for s in seeds])
    eps = [1e-3 * r for r in synth.range_of(f)]
    return f, eps


def label_blocks(enc: "dls.Encoder", field: torch.Tensor, p: "dls.Params") -> dict:
    """Encode `field` with the plain method and return its labelled blocks
    (raw blocks dropped): device tensors feat (n x 80), rank (n,),
    basis (n x 256, [k][t]) and wb (n,)."""
    enc.encode(field, p)
    inf = enc.info()
    nb = inf.nblocks
    rank = torch.empty(nb, dtype=torch.uint8, device=field.device)
    dls.d2d(rank, inf.d_rank, nb)
    basis = torch.empty((nb, 16, 16), dtype=torch.float64, device=field.device)
    dls.d2d(basis, inf.d_basis, nb * 256 * 8)
    desc = torch.empty((nb, 8), dtype=torch.int32, device=field.device)
    dls.d2d(desc, inf.d_desc, nb * 32)
    feat = enc.features(field)
    keep = rank > 0
    return {"feat": feat[keep], "rank": rank[keep].to(torch.int32),
            "basis": basis[keep].reshape(-1, 256).to(torch.float32),
            "wb": ((desc[keep, 4] >> 24) & 255).to(torch.int32)}


def merge(parts) -> dict:
    return {k: torch.cat([q[k] for q in parts]) for k in ("feat", "rank", "basis", "wb")}


def collect(seeds, chunk: int = 64, px: int = 8, window: int = 16):
    """Labelled blocks of config-1 fields (see label_blocks)."""
    enc = dls.Encoder()
    parts = []
    for i in range(0, len(seeds), chunk):
        f, eps = c1_fields(seeds[i:i + chunk])
        nv, nt, nz, ny, nx = f.shape
        p = dls.Params(nx=nx, ny=ny, nz=nz, nt=nt, nvars=nv, dtype="f64", px=px, py=px, pz=1,
                       window=window, eps=eps)
        parts.append(label_blocks(enc, torch.from_numpy(f).cuda(), p))
    return merge(parts)


def zscore(feat: torch.Tensor) -> np.ndarray:
    """Mean and standard deviation of the 16 statistics (32 values)."""
    m = feat[:, :16].double().mean(dim=0)
    s = feat[:, :16].double().std(dim=0).clamp_min(1e-6)
    return torch.cat([m, s]).float().cpu().numpy()


def train(model: "dls.Model", data: dict, epochs: int = 10, batch: int = 1024, lr: float = 1e-3,
          seed: int = 0, log=None):
    """Shuffled mini-batch Adam; returns the mean loss of every epoch."""
    n = data["feat"].shape[0]
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    losses = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g, device="cuda")
        tot, cnt = 0.0, 0
        for i in range(0, n - batch + 1, batch):
            idx = perm[i:i + batch]
            want = (i // batch) % 16 == 0
            l = model.train_step(data["feat"][idx].contiguous(), data["rank"][idx].contiguous(),
                                 data["basis"][idx].contiguous(), data["wb"][idx].contiguous(),
                                 lr=lr, bf16=True, want_loss=want)
            if want:
                tot += l
                cnt += 1
        losses.append(tot / max(cnt, 1))
        if log:
            log("epoch %d loss %.4f" % (ep, losses[-1]))
    return losses


def fit_data(data: dict, epochs=10, batch=1024, lr=1e-3, seed=0, log=None):
    """Set the z-scoring from `data`, train from He initialisation; returns (model, losses)."""
    model = dls.Model()
    model.set(he_init(seed), zscore(data["feat"]))
    batch = max(1, min(batch, int(data["feat"].shape[0])))
    losses = train(model, data, epochs, batch, lr, seed, log)
    return model, losses


def fit(train_seeds, epochs=10, batch=1024, lr=1e-3, seed=0, log=None):
    """Collect labels, set the z-scoring, train; returns (model, data, losses)."""
    t0 = time.perf_counter()
    data = collect(train_seeds)
    if log:
        log("collected %d blocks in %.1f s" % (data["feat"].shape[0], time.perf_counter() - t0))
    model, losses = fit_data(data, epochs, batch, lr, seed, log)
    return model, data, losses


def save(path: str, model: "dls.Model"):
    p, n = model.get()
    np.savez(path, params=p, norm=n)


def load(path: str) -> "dls.Model":
    z = np.load(path)
    m = dls.Model()
    m.set(z["params"], z["norm"])
    return m


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seed-a", type=int, default=100000)
    ap.add_argument("--n-train", type=int, default=200000)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--out", default="model.npz")
    a = ap.parse_args()
    nfields = (a.n_train + 127) // 128
    model, data, _ = fit(np.arange(a.seed_a, a.seed_a + nfields), epochs=a.epochs, log=print)
    save(a.out, model)


if __name__ == "__main__":
    main()
