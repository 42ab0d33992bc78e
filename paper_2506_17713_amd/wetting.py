"""Contact angles of sessile droplets: the wetting sweep of the D3Q19 MRT
sessile-drop workload (Carnahan-Starling at T = 0.8 T_c, 256^3, drop radius
30 on the solid wall z = 0, 20,000 steps) over five virtual-density settings
of the improved wetting scheme (Sec. 2.4, Eq. 17) chosen to give contact
angles of about 30, 60, 90, 120 and 150 degrees.

The solver runs on the GPU through the library; this module only forms the
inputs, reads the final density back and measures the angle on the host:
the paper describes no angle measurement for a plate, so a circle is fitted
by least squares to the rho = (rho_l + rho_v) / 2 iso-contour in the central
xz and yz slices, using contour points at least 3 lattice units above the
wall, and cos(theta) = (z_wall - z_centre) / R with the halfway bounce-back
wall at z = 0.5; the angle is the mean of the two slices.

  python -m paper_2506_17713_amd.wetting calibrate   # grid + interpolation per target, writes data/wetting_c2.json
  python -m paper_2506_17713_amd.wetting sweep       # the five calibrated runs, one JSON line each
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from pathlib import Path

import numpy as np

from . import inputs

DATA = Path(__file__).resolve().parent / "data" / "wetting_c2.json"
TARGETS = (30.0, 60.0, 90.0, 120.0, 150.0)


def _circle_angle(sl: np.ndarray, mid: float, zmin: float = 3.5, z_wall: float = 0.5) -> float:
    """Angle of the iso-contour sl = mid in a (z, s) slice over the wall z = 0."""
    nz, ns = sl.shape
    pts = []
    for s in range(ns):  # crossings along z
        col = sl[:, s]
        for z in range(1, nz - 2):
            a, b = col[z] - mid, col[z + 1] - mid
            if a * b < 0:
                zz = z + (mid - col[z]) / (col[z + 1] - col[z])
                if zz >= zmin:
                    pts.append((s, zz))
    for z in range(int(math.ceil(zmin)), nz - 1):  # crossings along s
        row = sl[z]
        for s in range(ns - 1):
            if (row[s] - mid) * (row[s + 1] - mid) < 0:
                pts.append((s + (mid - row[s]) / (row[s + 1] - row[s]), float(z)))
    P = np.array(pts)
    if len(P) < 6:
        return float("nan")
    M = np.column_stack([P[:, 0], P[:, 1], np.ones(len(P))])
    b = -(P[:, 0] ** 2 + P[:, 1] ** 2)
    D, E, F = np.linalg.lstsq(M, b, rcond=None)[0]
    sc, zc = -D / 2, -E / 2
    R = math.sqrt(max(sc * sc + zc * zc - F, 1e-30))
    return math.degrees(math.acos(max(-1.0, min(1.0, (z_wall - zc) / R))))


def contact_angle(rho: np.ndarray, mid: float) -> float:
    """Mean contact angle of the central xz and yz slices of rho[z, y, x]
    through the drop's centre of liquid mass."""
    liquid = np.clip(rho - mid, 0.0, None)
    nz, ny, nx = rho.shape
    tot = liquid.sum()
    cy = int(round((liquid.sum(axis=(0, 2)) * np.arange(ny)).sum() / tot))
    cx = int(round((liquid.sum(axis=(0, 1)) * np.arange(nx)).sum() / tot))
    a = _circle_angle(rho[:, cy, :], mid)
    b = _circle_angle(rho[:, :, cx], mid)
    return 0.5 * (a + b)


def run(mode: str, val: float, n: int = 256, r: float = 30.0, steps: int = 20000, storage: str = "F32"):
    """One sessile-drop run on the GPU; returns (angle, seconds, MLUPS)."""
    import torch

    from . import lbm

    rv = inputs.load_coexistence()["CS"]["0.8"]["rho_v"]
    w, solid, rho = inputs.sessile_3d(n=n, r=r, storage=storage, wet_mode=mode, wet=val,
                                      vapour=VAPOUR_FACTOR * rv)
    sol = lbm.Solver(w, solid, rho)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol.step(steps)
    r_gpu, _ = sol.moments_numpy(0)
    secs = time.perf_counter() - t0
    st = sol.stats()
    sol.close()
    if st["nonfinite"] or st["negative"]:
        return float("nan"), secs, 0.0
    mid = 0.5 * (w.rho_min[0] + w.rho_max[0])
    th = contact_angle(r_gpu.reshape(w.shape), mid)
    return th, secs, w.N * steps / secs / 1e6


PHI_GRID = (1.0, 1.1, 1.2, 1.3, 1.45, 1.6)
DRHO_GRID = (0.005, 0.01, 0.02, 0.03, 0.04, 0.05)
# Initial vapour density relative to Maxwell's.  A drop of radius 30 in a
# 256^3 box started in Maxwell vapour evaporates completely within 15,000
# steps: a curved drop is in equilibrium with supersaturated vapour (Kelvin),
# and the box holds 150 times the drop's volume of vapour to saturate.  At
# 1.063 rho_v the phi = 1 drop neither grows nor shrinks over 20,000 steps
# (measured: 1.055 loses 3 %, 1.073 gains 26 % of its liquid volume), so the
# sweep measures wetting rather than evaporation.
VAPOUR_FACTOR = 1.063


def calibrate(n: int, r: float, steps: int, log=print) -> list:
    """Wetting parameters for the target angles: the angle is mapped on a grid
    of phi >= 1 (it falls with phi) and of drho >= 0 (it rises with drho),
    each target is interpolated linearly on the side it falls on, and the
    interpolated setting is run once more to measure the angle it gives."""
    grid = []
    for v in PHI_GRID:
        th = run("PHI", v, n, r, steps)[0]
        grid.append(("PHI", v, th))
        log(f"  PHI {v}: {th:.2f}")
    for v in DRHO_GRID:
        th = run("DRHO", v, n, r, steps)[0]
        grid.append(("DRHO", v, th))
        log(f"  DRHO {v}: {th:.2f}")
    th1 = grid[0][2]
    out = []
    for t in TARGETS:
        if t <= th1:
            pts = [(th, v) for m, v, th in grid if m == "PHI" and np.isfinite(th)]
            mode = "PHI"
        else:
            pts = [(th1, 0.0)] + [(th, v) for m, v, th in grid if m == "DRHO" and np.isfinite(th)]
            mode = "DRHO"
        pts.sort()
        ths = np.array([p[0] for p in pts])
        vs = np.array([p[1] for p in pts])
        val = float(np.interp(t, ths, vs))
        th = run(mode, val, n, r, steps)[0]
        log(f"target {t}: {mode} {val:.5f} -> {th:.2f}")
        out.append({"target": t, "mode": mode, "value": val, "angle": th})
    return out, grid


def main(argv=None) -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["calibrate", "sweep"])
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--r", type=float, default=30.0)
    ap.add_argument("--steps", type=int, default=20000)
    args = ap.parse_args(argv)
    if args.what == "calibrate":
        settings, grid = calibrate(args.n, args.r, args.steps, log=lambda s: print(s, flush=True))
        out = {"n": args.n, "r": args.r, "steps": args.steps, "vapour_factor": VAPOUR_FACTOR, "settings": settings,
               "grid": [{"mode": m, "value": v, "angle": th} for m, v, th in grid]}
        DATA.parent.mkdir(exist_ok=True)
        DATA.write_text(json.dumps(out, indent=1) + "\n")
        print(json.dumps(out), flush=True)
    else:
        cal = json.loads(DATA.read_text())
        for s in cal["settings"]:
            th, secs, mlups = run(s["mode"], s["value"], args.n, args.r, args.steps)
            print(json.dumps({"target": s["target"], "mode": s["mode"], "value": s["value"], "angle": round(th, 2),
                              "seconds": round(secs, 2), "MLUPS": round(mlups, 1)}), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
