"""Learned warm start of permeability runs (experiment driver).

    python -m paper_2506_17713_amd.warmstart --train 96 --size 128 --epochs 6 \
        --test 8 --test-size 256 --out results.json

1. Training data: seeded periodic sphere packs (radii 6-14, porosity
   U(0.3, 0.5)), each solved from rest to a residual of 1e-6 by the fused LBM
   step (single phase, BGK tau = 1, body acceleration 1e-5 along x); target
   u nu / a.
2. Train the surrogate (paper_2506_17713_amd.surrogate) with the library's
   forward / backward / Adam kernels.
3. Held-out packs (seeds 1000+): the plain solver from rest (cold) and from
   f^eq(1, u_pred) (warm) to the same residual; Darcy permeability
   k = nu <u_x> / a of both.  Warm seconds include inference and the upload
   of the predicted field.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import inputs, nn
from .surrogate import NU, Surrogate, make_dataset, solve_steady, train


def evaluate(model: Surrogate, n_test: int, size: int, accel=1e-5, seed0=1000, log=print):
    rng = np.random.default_rng(777)
    out = []
    for s in range(n_test):
        por = float(rng.uniform(0.3, 0.5))
        solid = inputs.sphere_pack((size,) * 3, (6.0, 14.0), por, seed0 + s)
        cold = solve_steady(solid, accel=accel)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mask = torch.tensor((solid == 0).astype(np.float32)[None], device="cuda")
        u_pred = model.predict(mask).reshape(3, -1) * (accel / NU)
        t_inf = time.perf_counter() - t0
        warm = solve_steady(solid, accel=accel, u0=u_pred)
        warm_s = warm["seconds"] + t_inf
        rec = {"seed": seed0 + s, "porosity": float((solid == 0).mean()),
               "cold_steps": cold["steps"], "cold_s": cold["seconds"], "k_cold": cold["k"],
               "warm_steps": warm["steps"], "warm_s": warm_s, "inference_s": t_inf, "k_warm": warm["k"],
               "k_rel_err": abs(warm["k"] - cold["k"]) / abs(cold["k"]),
               "k_pred": float(NU * 0 + u_pred[0].mean() * NU / accel)}
        out.append(rec)
        log(json.dumps(rec))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=96)
    ap.add_argument("--size", type=int, default=128)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--test", type=int, default=8)
    ap.add_argument("--test-size", type=int, default=256)
    ap.add_argument("--out", default="warmstart_results.json")
    ap.add_argument("--prec", default="bf16", choices=["bf16", "fp32"])
    a = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)
    t0 = time.perf_counter()
    xs, ys, info = make_dataset(a.train, a.size, log=log)
    t_data = time.perf_counter() - t0
    model = Surrogate(prec=nn.BF16 if a.prec == "bf16" else nn.FP32)
    log(f"surrogate parameters: {model.n_params()}")
    t1 = time.perf_counter()
    hist = train(model, xs, ys, a.epochs, lr=a.lr, log=log)
    t_train = time.perf_counter() - t1
    del xs, ys
    res = evaluate(model, a.test, a.test_size, log=log)
    summ = {
        "n_train": a.train, "train_size": a.size, "epochs": a.epochs, "params": model.n_params(),
        "data_seconds": t_data, "train_seconds": t_train, "train_mse": hist,
        "test": res,
        "mean_steps_cold": float(np.mean([r["cold_steps"] for r in res])),
        "mean_steps_warm": float(np.mean([r["warm_steps"] for r in res])),
        "mean_seconds_cold": float(np.mean([r["cold_s"] for r in res])),
        "mean_seconds_warm": float(np.mean([r["warm_s"] for r in res])),
        "max_k_rel_err": float(np.max([r["k_rel_err"] for r in res])),
        "train_info": info,
    }
    with open(a.out, "w") as fh:
        json.dump(summ, fh, indent=1)
    log(json.dumps({k: v for k, v in summ.items() if k not in ("test", "train_info", "train_mse")}))
    return summ


if __name__ == "__main__":
    main(sys.argv[1:])
