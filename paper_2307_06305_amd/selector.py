"""Kernel-variant selector: collect autotuner timings, train the network on
the GPU, evaluate it, load the shipped weights.

    python -m paper_2307_06305_amd.selector collect --count 5000 --out times.npz
    python -m paper_2307_06305_amd.selector train --data times.npz --out weights.npy
    python -m paper_2307_06305_amd.selector evaluate --data times.npz --weights weights.npy

Each generated matrix gives two samples: its SpMV timings (nrhs = 1,
classes 0..62) and its SpMM timings for its own nrhs (2..8, classes 63..69).
All timing is done by the library's autotuner, all network arithmetic by the
library's kernels.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import (CLASS_SPMM, F64, MLP_NPARAMS, NCLASS, NFEAT, VAR_STREAM, Matrix, Mlp, autotune,
               encode, features)

DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")
WEIGHTS = os.path.join(DATA_DIR, "selector_weights.npy")
DATASET = os.path.join(DATA_DIR, "selector_times.npz")

LANES = (1, 2, 4, 8, 16, 32, 64)
TILES = (1024, 2048, 4096)


def config_class(cfg, nrhs):
    """Class index of a handle configuration (as get_config returns it)."""
    li = LANES.index(cfg["lanes"])
    if nrhs > 1:
        return CLASS_SPMM + li
    if cfg["variant"] == VAR_STREAM:
        paired = 21 if cfg["unroll"] == 2 else 0
        return 21 + paired + 3 * li + TILES.index(cfg["tile"])
    return 3 * li + (1, 2, 4).index(cfg["unroll"])


def _log(msg):
    print(f"[selector] {msg}", flush=True)


def collect(count, seed, n_lo=1e3, n_hi=2e5, reps=3, start=0):
    """Autotune `count` generated matrices of the batched family."""
    import torch

    from workloads.matrices import batch_matrix, batch_member

    dev = torch.device("cuda:0")
    F, T, D, M_ID = [], [], [], []
    t0 = time.time()
    for i in range(start, start + count):
        d = batch_member(seed, i, n_lo=n_lo, n_hi=n_hi)
        A = batch_matrix(d)
        e = encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, allow_rcm=False)
        M = Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], e["vals"], store=F64)
        default = M.get_config()
        g = torch.Generator().manual_seed(seed * 100003 + i)
        for k in sorted({1, d["nrhs"]}):
            if k == 1:
                X = torch.rand(A.ncols, generator=g, dtype=torch.float64).to(dev)
                Y = torch.zeros(A.nrows, dtype=torch.float64, device=dev)
            else:
                X = torch.rand(A.ncols, k, generator=g, dtype=torch.float64).to(dev)
                Y = torch.zeros(A.nrows, k, dtype=torch.float64, device=dev)
            T.append(autotune(M, k, X, Y, reps=reps))
            F.append(features(A.nrows, A.ncols, A.rowptr, A.colids, k))
            D.append(config_class(default, k))
            M_ID.append(i)
        M.destroy()
        if (i - start + 1) % 250 == 0:
            _log(f"collected {i - start + 1}/{count} matrices ({time.time() - t0:.0f}s)")
    return {"F": np.array(F, dtype=np.float32), "T": np.array(T, dtype=np.float32),
            "default": np.array(D, dtype=np.int32), "matrix": np.array(M_ID, dtype=np.int32),
            "seed": seed}


def split(data, holdout=0.2):
    """Train / held-out split by matrix (the last fraction of matrices)."""
    mid = data["matrix"]
    cut = np.quantile(mid, 1.0 - holdout)
    tr = mid < cut
    return tr, ~tr


def train(F, T, epochs=300, batch=256, lr=3e-3, tau=0.05, seed=1):
    net = Mlp(seed=seed)
    losses = net.train(F, T, epochs=epochs, batch=batch, lr=lr, tau=tau, seed=seed)
    params = net.params()
    net.destroy()
    return params, losses


def evaluate(params, F, T, default):
    """Slowdown t(chosen) / t(best) - 1 of the network and of the default
    configuration on samples with measured times."""
    net = Mlp(params)
    cls = net.select(F)
    net.destroy()
    idx = np.arange(len(F))
    best = T.min(axis=1)
    reg = T[idx, cls] / best - 1.0
    reg_def = T[idx, default] / best - 1.0
    return {"samples": int(len(F)), "mean_regret": float(reg.mean()),
            "p95_regret": float(np.quantile(reg, 0.95)),
            "within_5pct": float(np.mean(reg <= 0.05)),
            "default_mean_slowdown": float(reg_def.mean()),
            "default_p95_slowdown": float(np.quantile(reg_def, 0.95)),
            "time_ratio_default_over_selected": float((T[idx, default]).sum() / T[idx, cls].sum())}


def evaluate_fallback(params, F, T, threshold):
    """The selector with the exhaustive autotuner behind it: rows whose
    chosen class has probability below `threshold` are autotuned (regret 0,
    the autotuner's choice is the fastest measured class), the rest take the
    network's choice."""
    net = Mlp(params)
    cls, prob = net.select(F, with_prob=True)
    net.destroy()
    idx = np.arange(len(F))
    reg = T[idx, cls] / T.min(axis=1) - 1.0
    fb = prob < threshold
    reg = np.where(fb, 0.0, reg)
    return {"threshold": float(threshold), "fallback_fraction": float(fb.mean()),
            "mean_regret": float(reg.mean()), "p95_regret": float(np.quantile(reg, 0.95)),
            "within_5pct": float(np.mean(reg <= 0.05))}


def choose(net, A, M, nrhs, X, Y, threshold=0.2, reps=3):
    """Configure handle M for its product with nrhs right-hand sides: the
    network's class when its probability reaches `threshold`, else the
    exhaustive autotuner's (which times every class on X, Y and overwrites
    Y).  A: the host CSR arrays of M's matrix (for the features).  Returns
    (class, probability, autotuned)."""
    from . import class_config, features

    f = features(A.nrows, A.ncols, A.rowptr, A.colids, nrhs)
    cls, prob = net.select(f, with_prob=True)
    cls, prob = int(cls[0]), float(prob[0])
    if prob < threshold:
        t = autotune(M, nrhs, X, Y, reps=reps)
        return int(np.argmin(t)), prob, True
    v, lanes, unroll, tile, _ = class_config(cls)
    if v == VAR_STREAM and unroll == 2 and not M.takes_paired:
        unroll = 1  # a cell without paired gathers: the same launch, interleaved
    M.set_config(v, lanes, unroll, tile)
    return cls, prob, False


def load_weights(path=WEIGHTS):
    p = np.load(path, allow_pickle=False)
    if p.shape != (MLP_NPARAMS,) or p.dtype != np.float32:
        raise ValueError(f"{path}: expected {MLP_NPARAMS} float32 parameters")
    return p


def load_net(path=WEIGHTS):
    return Mlp(load_weights(path))


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2307_06305_amd.selector")
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--count", type=int, default=5000)
    c.add_argument("--seed", type=int, default=5004)
    c.add_argument("--reps", type=int, default=3)
    c.add_argument("--out", default=DATASET)
    t = sub.add_parser("train")
    t.add_argument("--data", default=DATASET)
    t.add_argument("--out", default=WEIGHTS)
    t.add_argument("--epochs", type=int, default=300)
    t.add_argument("--batch", type=int, default=256)
    t.add_argument("--lr", type=float, default=3e-3)
    t.add_argument("--tau", type=float, default=0.05)
    t.add_argument("--seed", type=int, default=1)
    ev = sub.add_parser("evaluate")
    ev.add_argument("--data", default=DATASET)
    ev.add_argument("--weights", default=WEIGHTS)
    a = ap.parse_args(argv)
    if a.cmd == "collect":
        data = collect(a.count, a.seed, reps=a.reps)
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        np.savez_compressed(a.out, **data)
        _log(f"wrote {a.out}: {len(data['F'])} samples")
    elif a.cmd == "train":
        d = np.load(a.data, allow_pickle=False)
        data = {k: d[k] for k in d.files}
        tr, ho = split(data)
        params, losses = train(data["F"][tr], data["T"][tr], a.epochs, a.batch, a.lr, a.tau,
                               a.seed)
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        np.save(a.out, params)
        res = {"loss_first": float(losses[0]), "loss_last": float(losses[-1]),
               "train": evaluate(params, data["F"][tr], data["T"][tr], data["default"][tr]),
               "heldout": evaluate(params, data["F"][ho], data["T"][ho], data["default"][ho])}
        print(json.dumps(res), flush=True)
    else:
        d = np.load(a.data, allow_pickle=False)
        data = {k: d[k] for k in d.files}
        _, ho = split(data)
        print(json.dumps(evaluate(load_weights(a.weights), data["F"][ho], data["T"][ho],
                                  data["default"][ho])), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
