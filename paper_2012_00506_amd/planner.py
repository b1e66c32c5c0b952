"""Learned slice planner: training data from exact inertia, GPU training.

A small network (80 -> 256 -> 256 -> 64) maps cheap band features (Chebyshev
moments of the density of states, Gershgorin bounds, band statistics) to the
fraction of eigenvalues below 64 evenly spaced shifts of the Gershgorin
interval.  Its labels are exact Sylvester inertia counts produced by the
library itself, and its only use is to seed the bisection of
``slice_plan(mode="learned")``: every boundary it proposes is judged by exact
inertia and certified, so the plan is exact whatever the network predicts.

Command line (trains on the seeded matrix family and reports the gain):

    python -m paper_2012_00506_amd.planner --train 1600 --test 200 --out w.npz
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np
import torch

from . import api

N_SHIFTS = 64
SIZES = (80, 256, 256, 64)


def init_weights(seed: int = 0, device="cuda") -> torch.Tensor:
    """Packed FP32 weights (W1, b1, W2, b2, W3, b3): He-uniform weights
    (fan_in x fan_out, row-major), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(3):
        fi, fo = SIZES[l], SIZES[l + 1]
        lim = math.sqrt(6.0 / fi)
        parts.append(rng.uniform(-lim, lim, (fi, fo)).ravel())
        parts.append(np.zeros(fo))
    w = np.concatenate(parts).astype(np.float32)
    assert w.nbytes == api.planner_bytes()
    return torch.from_numpy(w).to(device)


def label_shifts(gersh) -> np.ndarray:
    lo, hi = float(gersh[0]), float(gersh[1])
    return lo + (np.arange(N_SHIFTS) + 0.5) * (hi - lo) / N_SHIFTS


def sample(ab, seed: int):
    """(features (80,), labels (64,)) of one band matrix: labels are exact
    inertia counts n_-(s_k)/n on the GPU."""
    B = api.DeviceBand.from_band(ab)
    x = api.band_features(B, seed=seed)
    _, gersh = api.cheb_moments(B, K=0, P=1, seed=seed)
    neg, _, _ = api.band_inertia(B, label_shifts(gersh))
    return x, neg.astype(np.float64) / B.n


def build_dataset(indices, make_matrix, log=None):
    X, Y = [], []
    t0 = time.time()
    for c, i in enumerate(indices):
        ab = make_matrix(i)
        x, y = sample(ab, seed=i)
        X.append(x)
        Y.append(y)
        if log and (c + 1) % 50 == 0:
            log(f"  {c + 1}/{len(indices)} samples, {time.time() - t0:.1f} s")
    return np.array(X), np.array(Y)


def train(X, Y, epochs=200, batch=64, lr=1e-3, seed=0, device="cuda", log=None, on_epoch=None):
    """Adam on the GPU with the library's own forward/backward kernels;
    on_epoch(epoch, weights) is called after every epoch."""
    w = init_weights(seed, device)
    opt = torch.zeros(2 * w.numel(), dtype=torch.float32, device=device)
    Xt = torch.as_tensor(X, dtype=torch.float32, device=device)
    Yt = torch.as_tensor(Y, dtype=torch.float32, device=device)
    rng = np.random.default_rng(seed + 1)
    t = 0
    hist = []
    n = len(X)
    for ep in range(epochs):
        perm = rng.permutation(n)
        tot = 0.0
        for s in range(0, n - batch + 1 if n >= batch else 1, batch):
            idx = torch.as_tensor(perm[s:s + batch], device=device)
            t += 1
            tot += api.planner_train_step(w, opt, Xt[idx], Yt[idx], lr, t) * len(idx)
        hist.append(tot / max(1, (n // batch) * batch if n >= batch else n))
        if on_epoch:
            on_epoch(ep, w)
        if log and (ep + 1) % 50 == 0:
            log(f"  epoch {ep + 1}: train mse {hist[-1]:.3e}")
    return w, hist


def predict(w, X) -> np.ndarray:
    Xt = torch.as_tensor(np.asarray(X), dtype=torch.float32, device=w.device)
    return api.planner_forward(w, Xt).cpu().numpy()


def gain(w, matrices, K_list=(16, 64), count_tol=0.05):
    """Inertia evaluations of equal-count planning by bisection, by
    interpolation under a uniform prior and by the network's prediction, per
    held-out matrix and K."""
    rows = []
    for i, ab in matrices:
        B = api.DeviceBand.from_band(ab)
        for K in K_list:
            eb, ec, ne = api.slice_plan(B, K, "equal_count", count_tol=count_tol)
            ub, uc, nu = api.slice_plan(B, K, "learned", count_tol=count_tol, planner=None)
            lb, lc, nl = api.slice_plan(B, K, "learned", count_tol=count_tol, planner=w, seed=i)
            rows.append({"matrix": i, "K": K, "bisection": ne, "uniform": nu, "learned": nl,
                         "total_equal": int(ec.sum()) == int(lc.sum()) == int(uc.sum())})
    return rows


def main():
    """Train on the seeded planner family (indices 0..train-1), select the
    epoch by validation loss (the next `val` indices) and report the test
    loss and the inertia-evaluation gain on the `gain` first test matrices."""
    import synth
    p = argparse.ArgumentParser()
    p.add_argument("--train", type=int, default=1600)
    p.add_argument("--val", type=int, default=200)
    p.add_argument("--test", type=int, default=200)
    p.add_argument("--gain", type=int, default=50)
    p.add_argument("--epochs", type=int, default=300)
    p.add_argument("--scale", type=int, default=1, help="n divisor of the family (quick runs)")
    p.add_argument("--out", default=None)
    a = p.parse_args()
    log = lambda s: print(s, flush=True)
    make = lambda i: synth.planner_matrix(i, scale=a.scale)[0]
    t0 = time.time()
    log(f"building {a.train} training samples")
    X, Y = build_dataset(range(a.train), make, log)
    i0 = a.train
    log(f"building {a.val} validation and {a.test} test samples")
    Xv, Yv = build_dataset(range(i0, i0 + a.val), make, log)
    Xt, Yt = build_dataset(range(i0 + a.val, i0 + a.val + a.test), make, log)
    t_data = time.time() - t0
    t0 = time.time()
    best = {"mse": float("inf")}

    def keep_best(ep, w):
        mse = float(np.mean((predict(w, Xv) - Yv) ** 2))
        if mse < best["mse"]:
            best.update(mse=mse, epoch=ep, w=w.clone())

    w, hist = train(X, Y, epochs=a.epochs, log=log, on_epoch=keep_best)
    t_train = time.time() - t0
    w = best["w"]
    test_mse = float(np.mean((predict(w, Xt) - Yt) ** 2))
    t0 = time.time()
    ids = range(i0 + a.val, i0 + a.val + min(a.gain, a.test))
    rows = gain(w, [(i, make(i)) for i in ids])
    t_gain = time.time() - t0
    out = {"train": a.train, "val": a.val, "test": a.test, "scale": a.scale,
           "train_mse": hist[-1], "val_mse": best["mse"], "best_epoch": best["epoch"],
           "test_mse": test_mse, "seconds": {"labels": t_data, "train": t_train, "gain": t_gain}}
    for K in sorted({r["K"] for r in rows}):
        rk = [r for r in rows if r["K"] == K]
        out[f"K{K}"] = {m: float(np.mean([r[m] for r in rk]))
                        for m in ("bisection", "uniform", "learned")}
    print(json.dumps(out), flush=True)
    if a.out:
        np.save(a.out, w.cpu().numpy())


if __name__ == "__main__":
    main()
