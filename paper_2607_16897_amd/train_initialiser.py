"""Train the learned start-pose network on tracker-labelled pairs and evaluate
it against the constant-velocity prior.

    python -m paper_2607_16897_amd.train_initialiser --refs 20000 --per-ref 10 --out DIR

Writes DIR/initialiser.npy (flat FP32 parameters) and DIR/initialiser.json
(training configuration, loss history, validation loss, evaluation).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--refs", type=int, default=20000)
    ap.add_argument("--per-ref", type=int, default=10)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=5000)
    ap.add_argument("--time-limit", type=float, default=300.0, help="seconds of training at most")
    ap.add_argument("--eval-streams", type=int, default=64)
    ap.add_argument("--eval-frames", type=int, default=100)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()

    import torch

    from . import Cnn
    from . import initialiser as ini

    os.makedirs(args.out, exist_ok=True)
    log = lambda m: print(m, flush=True)
    t0 = time.perf_counter()
    pairs, targets, dstat = ini.make_dataset(args.refs, args.per_ref, seed=args.seed, log=log)
    n = pairs.shape[0]
    n_val = max(args.batch, n // 20)
    tr_p, tr_t = pairs[:n - n_val], targets[:n - n_val]
    va_p, va_t = pairs[n - n_val:], targets[n - n_val:]
    log(f"dataset ready: {n} pairs ({dstat['seconds']:.1f} s), label failures {dstat['label_failures']}")
    net = Cnn(max_batch=args.batch)
    net.set_params(ini.init_params(args.seed))
    val0 = ini.validation_loss(net, va_p, va_t)
    hist = []
    t_train = time.perf_counter()
    lr = args.lr
    for ep in range(args.epochs):
        if ep == int(0.8 * args.epochs):
            lr = args.lr * 0.1
        hist += ini.train(net, tr_p, tr_t, epochs=1, batch=args.batch, lr=lr, seed=args.seed + ep, log=None)
        val = ini.validation_loss(net, va_p, va_t)
        log(f"epoch {ep}: train {hist[-1]:.4f} val {val:.4f} lr {lr:g} ({time.perf_counter() - t_train:.1f} s)")
        if time.perf_counter() - t_train > args.time_limit:
            break
    train_s = time.perf_counter() - t_train
    val = ini.validation_loss(net, va_p, va_t)
    log("evaluating against the constant-velocity prior")
    ev = ini.evaluate(net, args.eval_streams, args.eval_frames, seed=args.seed + 777)
    log(json.dumps(ev))
    meta = {"pairs": n, "train_pairs": n - n_val, "val_pairs": n_val, "epochs_run": len(hist),
            "batch": args.batch, "lr": args.lr, "seed": args.seed, "dataset_seconds": dstat["seconds"],
            "label_failures": dstat["label_failures"], "train_seconds": train_s, "loss_history": hist,
            "val_loss_initial": val0, "val_loss": val, "evaluation": ev,
            "total_seconds": time.perf_counter() - t0}
    ini.save_checkpoint(os.path.join(args.out, "initialiser"), net.get_params(), meta)
    log(f"saved {args.out}/initialiser.npy")


if __name__ == "__main__":
    sys.exit(main())
