"""Write c4_crop32_cstep.json: FP64 oracle derivatives of the adjoint
workload's observable on a 32^3 crop, by complex-step differentiation.

Workload: the adjoint sphere pack (128^3, porosity 0.4, radii 6-14, seed 1)
cropped to x, y, z in [0, 32) and run as its own periodic domain; single
component Carnahan-Starling at T_r = 0.8, d'Humieres MRT at tau = 1, liquid
slab x < 16 (tanh width 5), uniform wetting phi = 1.2; 1,000 steps.
Observable: the smooth vapour saturation S = (1/N_fluid) sum_fluid
sigma((rho_mid - rho) / delta) of the final density, rho_mid and delta from the
Maxwell densities (Sec. 3.4.3 segments by threshold; the logistic version has
a derivative).  Derivatives: dS/d(phi at 20 seeded boundary-solid voxels on
the vapour side, x >= 22) and dS/dT (absolute temperature), each from one
complex-step run of the oracle (h = 1e-30).

Run from the repository root: python tests/golden/make_c4_crop32.py
Uses only oracle/ and the seeded input generators."""
import hashlib
import json
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

from oracle import oracle  # noqa: E402
from paper_2506_17713_amd import inputs  # noqa: E402

STEPS = 1000
NVOX = 20


def crop_workload():
    full = inputs.sphere_pack((128, 128, 128), (6.0, 14.0), 0.4, 1)
    solid = np.ascontiguousarray(full[:32, :32, :32])
    w, solid, rho = inputs.adjoint_pack(shape=(32, 32, 32), storage="F64", solid=solid)
    return w, solid, rho


def boundary_voxels(solid, xmin, count, seed):
    s = solid.astype(bool)
    touch = np.zeros_like(s)
    for ax in range(3):
        for sh in (-1, 1):
            touch |= np.roll(~s, sh, axis=ax)
    cand = np.flatnonzero((s & touch).reshape(-1))
    x = cand % s.shape[2]
    cand = cand[x >= xmin]
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(cand, size=count, replace=False))


def saturation(st, fluid, rho_mid, delta):
    r = st.fields()["rho"][0]
    z = (rho_mid - r[fluid]) / delta
    return (1.0 / (1.0 + np.exp(-z))).sum() / fluid.sum()


def main():
    w, solid, rho = crop_workload()
    fluid = solid.reshape(-1) == 0
    rl, rv = w.rho_max[0], w.rho_min[0]
    rho_mid, delta = 0.5 * (rl + rv), 0.05 * (rl - rv)
    vox = boundary_voxels(solid, 22, NVOX, seed=3)
    base = np.full((1, w.N), w.wet[0], dtype=np.complex128)
    h = 1e-30
    t0 = time.time()
    st = oracle.State(w, solid, rho)
    st.step(STEPS)
    S = float(saturation(st, fluid, rho_mid, delta))
    dphi = []
    for v in vox:
        ww = base.copy()
        ww[0, v] += 1j * h
        st = oracle.State(w, solid, rho, wet=ww, cstep=True)
        st.step(STEPS)
        dphi.append(float(saturation(st, fluid, rho_mid, delta).imag / h))
        print(f"voxel {v}: {dphi[-1]:.6e} ({time.time() - t0:.0f} s)", flush=True)
    st = oracle.State(w, solid, rho, wet=base, cstep=True, T_im=h)
    st.step(STEPS)
    dT = float(saturation(st, fluid, rho_mid, delta).imag / h)
    out = {
        "what": "FP64 oracle complex-step derivatives of the smooth vapour saturation, adjoint pack 32^3 crop",
        "steps": STEPS, "phi": w.wet[0], "rho_mid": rho_mid, "delta": delta,
        "solid_sha256": hashlib.sha256(solid.tobytes()).hexdigest(),
        "S": S, "voxels": [int(v) for v in vox], "dS_dphi": dphi, "dS_dT": dT,
    }
    path = Path(__file__).with_name("c4_crop32_cstep.json")
    path.write_text(json.dumps(out, indent=1) + "\n")
    print("wrote", path, f"({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
