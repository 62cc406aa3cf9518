"""Train the per-pair degree model on the GPU from errors the method measures.

    python -m paper_2012_06925_amd.train_degree_model [--out models/coulomb_degree.bin]

Training data: for seeded 1E5-particle Coulomb problems (uniform cube,
Gaussian, unit sphere; theta 0.6 / 0.75 / 0.9; leaf sizes 500 and 2000) the
library traverses each problem and measures, on the GPU, the relative l2
error of every separated pair's cluster-cluster approximation at degrees
2..12 against the pair's direct sum (bldtt_pair_errors).  The model is then
trained on the GPU by the library's own forward/backward/Adam kernels
(bldtt_mlp_train).  Seeds >= 20127000 keep training data apart from every
evaluation workload.
"""
from __future__ import annotations

import argparse
import json
import os
import struct
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

MAGIC = b"BLDTTMLP"
VERSION = 1
DEFAULT_MODEL = os.path.join(HERE, "models", "coulomb_degree.bin")
TRAIN_SEED = 20127000


def save_model(path: str, model: np.ndarray, meta: dict) -> None:
    model = np.ascontiguousarray(model, dtype="<f4")
    with open(path, "wb") as f:
        f.write(MAGIC + struct.pack("<II", VERSION, model.size) + model.tobytes())
    with open(os.path.splitext(path)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)


def load_model(path: str = DEFAULT_MODEL) -> np.ndarray:
    """Read a model record; raises on a missing, truncated or foreign file."""
    with open(path, "rb") as f:
        head = f.read(16)
        if len(head) != 16 or head[:8] != MAGIC:
            raise ValueError(f"{path}: not a degree model file")
        version, n = struct.unpack("<II", head[8:])
        if version != VERSION:
            raise ValueError(f"{path}: unsupported version {version}")
        data = np.frombuffer(f.read(), dtype="<f4")
    if data.size != n:
        raise ValueError(f"{path}: truncated ({data.size} of {n} floats)")
    return data.astype(np.float32)


def measure(problems, log=print):
    import torch
    from paper_2012_06925_amd import api, inputs
    feats, errs = [], []
    for i, (dist, n, theta, leaf) in enumerate(problems):
        p = inputs.particles(n, dist, seed=TRAIN_SEED + i)
        src = [torch.from_numpy(a).cuda() for a in (p.x, p.y, p.z, p.q)]
        t0 = time.perf_counter()
        with api.Plan(None, src, theta=theta, degree=8, leaf=leaf) as plan:
            f, e = plan.pair_errors()
        log(f"  {dist:8s} n={n} theta={theta} leaf={leaf}: {f.shape[0]} pairs ({time.perf_counter() - t0:.1f} s)")
        feats.append(f)
        errs.append(e)
    return np.concatenate(feats), np.concatenate(errs)


def default_problems(n=100_000):
    return [(dist, n, theta, leaf) for dist in ("uniform", "gaussian", "sphere") for theta in (0.6, 0.75, 0.9)
            for leaf in (500, 2000)]


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_MODEL)
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=1)
    args = ap.parse_args()
    from paper_2012_06925_amd import api
    print("measuring pair errors", flush=True)
    f, e = measure(default_problems())
    print(f"training on {f.shape[0]} pairs", flush=True)
    t0 = time.perf_counter()
    model, hist = api.mlp_train(f, e, epochs=args.epochs, batch=args.batch, lr=args.lr, seed=args.seed)
    dt = time.perf_counter() - t0
    print(f"loss {hist[0]:.4f} -> {hist[-1]:.4f} in {dt:.1f} s", flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    save_model(args.out, model, {
        "kernel": "coulomb", "pairs": int(f.shape[0]), "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
        "seed": args.seed, "train_seed_base": TRAIN_SEED, "problems": default_problems(),
        "loss_first": float(hist[0]), "loss_last": float(hist[-1]), "train_seconds": round(dt, 2),
        "feature_range_lo": model[-8:-4].tolist(), "feature_range_hi": model[-4:].tolist()})
    print("wrote", args.out, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
