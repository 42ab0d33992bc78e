"""Learned warm start of permeability runs (experiment driver).

    python -m paper_2506_17713_amd.warmstart --train 256 --size 128 --epochs 12 \
        --test 32 --test-size 256 --out results.json

1. Training data: seeded periodic sphere packs (radii 6-14, porosity
   U(0.3, 0.5)), each solved from rest to a residual of 1e-6 by the fused LBM
   step (single phase, BGK tau = 1, body acceleration 1e-5 along x); targets
   u nu / a and (rho - 1) c_s^2 / a.
2. Train the surrogate (paper_2506_17713_amd.surrogate) with the library's
   forward / backward / Adam kernels, then fit its velocity gain to the
   permeabilities of the training packs (calibrate_flow).
3. Held-out packs (seeds 1000+): the plain solver from rest (cold) and from
   f^eq(rho_pred, u_pred - a/2) (warm; the start is formed on the GPU and
   loaded with lbm_reset).  Two stopping rules are reported for
   both: the residual rule (r < 1e-6), the time-to-permeability rule (k
   changes by less than 1e-4 relative over two consecutive 100-step checks),
   and the time to a permeability within 1 % of the cold run's converged one
   (the accuracy the warm start is asked for).
   Darcy permeability k = nu <u_x>_V / a; its error is taken against the
   cold run at r < 1e-6.  Warm seconds include inference and the forming of
   the initial state; both runs include the solver set-up.

--save-model / --load-model split training and evaluation over runs.  A
loaded model is only evaluated unless --train is given explicitly (then it is
trained further, with fresh Adam moments); --test-first selects the first
held-out seed offset.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import inputs, nn
from .surrogate import (NU, Surrogate, calibrate_flow, first_within, make_dataset, solve_steady, train,
                        warm_start_device)


def evaluate(model: Surrogate, n_test: int, size: int, accel=1e-5, seed0=1000, first=0, log=print,
             warm_max_steps=100000, layout="FLUID"):
    rng = np.random.default_rng(777)
    pors = [float(rng.uniform(0.3, 0.5)) for _ in range(first + n_test)]
    out = []
    for s in range(first, first + n_test):
        solid = inputs.sphere_pack((size,) * 3, (6.0, 14.0), pors[s], seed0 + s)
        cold = solve_steady(solid, accel=accel, layout=layout)
        mask = torch.tensor((solid == 0).astype(np.float32)[None], device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rho0, u0 = warm_start_device(model, mask, accel)
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t0
        # the network's own k: nu <u_x>_V / a of the predicted velocity
        k_pred = float(((u0[0] + 0.5 * accel) * mask.reshape(-1)).sum()) * NU / accel / solid.size
        warm = solve_steady(solid, accel=accel, u0=u0, rho0=rho0, max_steps=warm_max_steps, layout=layout)
        kc = cold["k"]
        c1 = first_within(cold["history"], kc) or (cold["steps"], cold["seconds"])
        w1 = first_within(warm["history"], kc) or (warm["steps"], warm["seconds"])
        rec = {"seed": seed0 + s, "porosity": float((solid == 0).mean()), "k_cold": kc,
               "warm_reached_residual": bool(warm["residual"] < 1e-6),
               "cold_1pct_steps": c1[0], "cold_1pct_s": c1[1], "warm_1pct_steps": w1[0],
               "warm_1pct_s": w1[1] + t_inf,
               "k_pred": k_pred, "inference_s": t_inf,
               "cold_steps": cold["steps"], "cold_s": cold["seconds"],
               "warm_steps": warm["steps"], "warm_s": warm["seconds"] + t_inf, "k_warm": warm["k"],
               "cold_k_steps": cold["k_steps"], "cold_k_s": cold["k_seconds"],
               "warm_k_steps": warm["k_steps"], "warm_k_s": warm["k_seconds"] + t_inf,
               "k_rel_err": abs(warm["k"] - kc) / abs(kc),
               "k_rel_err_cold_k_rule": abs(cold["k_at_k_steps"] - kc) / abs(kc),
               "k_rel_err_warm_k_rule": abs(warm["k_at_k_steps"] - kc) / abs(kc),
               "k_rel_err_pred": abs(k_pred - kc) / abs(kc),
               "warm_history": warm["history"][:30]}
        out.append(rec)
        log(json.dumps({k: (round(v, 6) if isinstance(v, float) else v) for k, v in rec.items()
                        if k != "warm_history"}))
    return out


def summarise(res: list) -> dict:
    m = lambda key: float(np.mean([r[key] for r in res]))
    return {"n_test": len(res),
            "mean_steps_cold": m("cold_steps"), "mean_steps_warm": m("warm_steps"),
            "mean_seconds_cold": m("cold_s"), "mean_seconds_warm": m("warm_s"),
            "mean_k_steps_cold": m("cold_k_steps"), "mean_k_steps_warm": m("warm_k_steps"),
            "mean_k_seconds_cold": m("cold_k_s"), "mean_k_seconds_warm": m("warm_k_s"),
            "mean_inference_s": m("inference_s"),
            "mean_1pct_steps_cold": m("cold_1pct_steps"), "mean_1pct_steps_warm": m("warm_1pct_steps"),
            "mean_1pct_seconds_cold": m("cold_1pct_s"), "mean_1pct_seconds_warm": m("warm_1pct_s"),
            "warm_faster_1pct_rule": int(sum(r["warm_1pct_s"] < r["cold_1pct_s"] for r in res)),
            "max_k_rel_err": float(np.max([r["k_rel_err"] for r in res])),
            "max_k_rel_err_cold_k_rule": float(np.max([r["k_rel_err_cold_k_rule"] for r in res])),
            "max_k_rel_err_warm_k_rule": float(np.max([r["k_rel_err_warm_k_rule"] for r in res])),
            "mean_k_rel_err_pred": m("k_rel_err_pred"),
            "warm_faster_residual_rule": int(sum(r["warm_s"] < r["cold_s"] and r["warm_reached_residual"]
                                                 for r in res)),
            "warm_reached_residual": int(sum(r["warm_reached_residual"] for r in res)),
            "warm_faster_k_rule": int(sum(r["warm_k_s"] < r["cold_k_s"] for r in res))}


def parse_args(argv=None) -> argparse.Namespace:
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=None,
                    help="training packs (default 256, or 0 with --load-model)")
    ap.add_argument("--size", type=int, default=128)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--test", type=int, default=32)
    ap.add_argument("--test-first", type=int, default=0)
    ap.add_argument("--test-size", type=int, default=256)
    ap.add_argument("--out", default="warmstart_results.json")
    ap.add_argument("--prec", default="bf16", choices=["bf16", "fp32"])
    ap.add_argument("--save-model", default=None)
    ap.add_argument("--load-model", default=None)
    ap.add_argument("--augment", action="store_true", help="train under random symmetries of the problem")
    ap.add_argument("--warm-max-steps", type=int, default=100000,
                    help="cap on the warm runs (the residual rule may then be left unreached)")
    ap.add_argument("--layout", default="FLUID", choices=["FLUID", "DENSE"],
                    help="population layout of the held-out solves (FLUID: fluid nodes only)")
    ap.add_argument("--calibrate", type=int, default=None,
                    help="training-distribution packs for the velocity gain (default: the training set after "
                         "training; 0 keeps the model's gain)")
    a = ap.parse_args(argv)
    if a.train is None:
        a.train = 0 if a.load_model else 256
    return a


def main(argv=None):
    a = parse_args(argv)
    log = lambda m: print(m, flush=True)
    model = Surrogate(prec=nn.BF16 if a.prec == "bf16" else nn.FP32)
    log(f"surrogate parameters: {model.n_params()}")
    summ = {"params": model.n_params(), "prec": a.prec}
    if a.load_model:
        with np.load(a.load_model, allow_pickle=False) as z:
            model.load_state({k: z[k] for k in z.files})
        summ["model"] = a.load_model
    if a.train > 0:
        # (with --load-model this continues training from the saved weights;
        # the Adam moments restart from zero)
        t0 = time.perf_counter()
        xs, ys, info = make_dataset(a.train, a.size, log=log)
        t_data = time.perf_counter() - t0
        t1 = time.perf_counter()
        hist = train(model, xs, ys, a.epochs, lr=a.lr, log=log, augment=a.augment)
        t_train = time.perf_counter() - t1
        if a.calibrate is None:
            gain = calibrate_flow(model, xs, ys)
            log(f"velocity gain {gain:.4f} (training set)")
            summ["flow_gain"] = gain
        del xs, ys
        summ.update({"n_train": a.train, "train_size": a.size, "epochs": a.epochs, "lr": a.lr, "augment": a.augment,
                     "data_seconds": t_data, "train_seconds": t_train, "train_mse": hist,
                     "train_info": info})
    if a.calibrate:
        xs, ys, _ = make_dataset(a.calibrate, a.size, log=log)
        gain = calibrate_flow(model, xs, ys)
        log(f"velocity gain {gain:.4f} ({a.calibrate} training-distribution packs)")
        summ["flow_gain"] = gain
        del xs, ys
    if a.save_model:
        np.savez(a.save_model, **model.state())
    if a.test > 0:
        res = evaluate(model, a.test, a.test_size, first=a.test_first, log=log, warm_max_steps=a.warm_max_steps,
                       layout=a.layout)
        summ["test"] = res
        summ.update(summarise(res))
    with open(a.out, "w") as fh:
        json.dump(summ, fh, indent=1)
    log(json.dumps({k: v for k, v in summ.items() if k not in ("test", "train_info", "train_mse")}))
    return summ


if __name__ == "__main__":
    main(sys.argv[1:])
