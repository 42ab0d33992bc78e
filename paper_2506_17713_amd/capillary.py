"""Capillary pressure - wetting saturation curve measured in place during a
drainage run (Sec. 3.4.3).

The pack between two reservoirs (inputs.pcsw_pack) starts saturated with the
wetting component.  The inlet reservoir holds the non-wetting bulk
composition; its major density, and with it the inlet pressure, is raised in
stages.  Every `sample` steps lbm_stats returns the capillary pressure (mean
pressure of the non-wetting nodes minus that of the wetting nodes) and the
wetting saturation over the pack's planes, computed on the GPU from the
state in HBM: nothing is copied back but the reduction's few numbers.

  python -m paper_2506_17713_amd.capillary --n 128 --stages 0,0.02,0.04 \\
      --steps 4000 --sample 1000 --out pcsw.json
"""
from __future__ import annotations

import argparse
import json
import time

from . import inputs, lbm


def drainage(n: int, buffer: int, stages, steps: int, sample: int, storage: str = "F32", log=print,
             layout: str = "FLUID") -> dict:
    import torch

    w, mask, rho = inputs.pcsw_pack(n=n, buffer=buffer, storage=storage, dp_rho=float(stages[0]))
    w = w.with_(layout=layout)
    minor = w.res_rho[0][1]
    sol = lbm.Solver(w, mask, rho, device="cuda:0")
    rows = []
    t_run = 0.0
    for dp in stages:
        sol.set_reservoir(0, (1.0 + float(dp), minor))
        for _ in range(max(1, steps // sample)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sol.step(sample)
            st = sol.stats()  # synchronises
            t_run += time.perf_counter() - t0
            row = {"dp_rho": float(dp), "step": st["step"], "p_c": st["capillary_pressure"],
                   "s_w": st["s_wetting"], "p_nw": st["p_nonwetting"], "p_w": st["p_wetting"],
                   "mass": st["mass"], "nonfinite": st["nonfinite"]}
            rows.append(row)
            log(f"dp {dp:.3f} step {row['step']} Pc {row['p_c']:.5f} Sw {row['s_w']:.4f}")
            if st["nonfinite"] or st["negative"]:
                raise RuntimeError(f"non-finite or negative density at step {st['step']}")
    sol.close()
    total = rows[-1]["step"]
    return {"workload": {"n": n, "buffer": buffer, "shape": list(w.shape), "window": list(w.window),
                         "storage": storage, "layout": layout, "fluid_nodes": int((mask == 0).sum())},
            "stages": [float(s) for s in stages], "steps_per_stage": steps, "sample": sample,
            "seconds": t_run, "ms_per_step": 1e3 * t_run / total, "curve": rows}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--buffer", type=int, default=8)
    ap.add_argument("--stages", default="0,0.02,0.04,0.06,0.08,0.1,0.12,0.14")
    ap.add_argument("--steps", type=int, default=4000, help="steps per pressure stage")
    ap.add_argument("--sample", type=int, default=1000)
    ap.add_argument("--storage", default="F32")
    ap.add_argument("--layout", default="FLUID", choices=["FLUID", "DENSE"],
                    help="population layout (FLUID: fluid nodes only, twice as fast on packs)")
    ap.add_argument("--out", default="pcsw.json")
    a = ap.parse_args(argv)
    res = drainage(a.n, a.buffer, [float(s) for s in a.stages.split(",")], a.steps, a.sample, a.storage,
                   log=lambda m: print(m, flush=True), layout=a.layout)
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps({k: v for k, v in res.items() if k != "curve"}))


if __name__ == "__main__":
    main()
