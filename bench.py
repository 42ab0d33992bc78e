"""Benchmark of the fused D3Q19 Shan-Chen step on one MI355X.

Workload: the sessile-droplet case -- D3Q19, MRT, Carnahan-Starling EOS at
T = 0.8 T_c, 256^3 nodes, FP32 populations, a droplet of radius 30 resting on
the solid wall z = 0 (second wall at z = 255, x and y periodic), improved
virtual-density wetting (phi = 1.1).  A step is one launch of the fused
kernel (moments, virtual densities, pseudopotential, force, MRT collision with
exact-difference forcing, pull streaming with bounce-back).

--workload droplet2d (D2Q9 BGK FP64 droplet, 128^2), --workload pack2
(two-component D3Q19 sphere pack, 400^3, BGK) and --workload pcsw (the
two-component drainage pack between reservoirs, 256^3 + buffers) time the
other configurations the same way; the two packs run on the fluid-only layout
(three kernels per step) unless --layout DENSE is given.

Prints one JSON line: MLUPS (n_components * nx * ny * nz * steps / time / 1e6,
all nodes counted as the paper does), the HBM roofline of the fused kernel
(algorithmic bytes per launch / mean launch time from HIP events on the
library's stream), and the FP64 CPU oracle timed on a bounded sample of the
same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 500; 1000 for adjoint)")
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=None, help="lattice size (default: 256, 128 for droplet2d, "
                                                         "400 for pack2)")
    ap.add_argument("--workload", default="sessile",
                    choices=["sessile", "droplet2d", "pack2", "pcsw", "adjoint", "surrogate"],
                    help="sessile: D3Q19 MRT sessile droplet (the headline line); droplet2d: D2Q9 BGK FP64 "
                         "droplet; pack2: D3Q19 two-component sphere pack; pcsw: two-component drainage of "
                         "an n^3 pack between reservoirs (open boundaries, in-situ capillary pressure); "
                         "adjoint: gradient of the saturation over 1000 steps of the 128^3 pack (checkpoint "
                         "every 100)")
    ap.add_argument("--storage", default="F32", choices=["F32", "F64", "F32F64", "F16DEV", "BF16DEV"])
    ap.add_argument("--collision", default="MRT", choices=["MRT", "BGK"])
    ap.add_argument("--layout", default=None, choices=["DENSE", "FLUID"],
                    help="population layout: every node (DENSE) or fluid nodes only (FLUID); default FLUID for "
                         "the porous packs (pack2, pcsw), DENSE otherwise")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-table", action="store_true",
                    help="no GPU work: time the FP64 oracle on the host at the sizes of the parity runs (the "
                         "128^2 droplet, 64^3 and 128^3 sessile drops, the two-component 64^3 pack crop), on all "
                         "threads and on one, and print one JSON line per case")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="after the run, two plain device copies of this many GiB (hardware-counter calibration)")
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None,
                    help="no GPU work: read the rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE output of two runs of "
                         "'bench.py --copy-gib 1' and write profiles/k_step_traffic.json for the kernel sources "
                         "in this tree")
    return ap.parse_args()


def algorithmic_bytes(w, solid) -> float:
    """Bytes the method must move per step: every fluid node's populations
    read once and written once (plus rho* for 16-bit deviation storage), and
    one mask byte per node."""
    import numpy as np

    n_fluid = int((np.asarray(solid) == 0).sum())
    q = w.q
    if w.storage in ("F16DEV", "BF16DEV"):
        per_fluid = w.nc * 2 * (q * 2 + 4)
    else:
        per_fluid = w.nc * 2 * q * (8 if w.storage == "F64" else 4)
    return float(n_fluid * per_fluid + w.N)


KERNEL_SOURCES = ("paper_2506_17713_amd/csrc/lbm_device.hpp", "paper_2506_17713_amd/csrc/lbm_api.hip",
                  "paper_2506_17713_amd/csrc/lbm_internal.hpp")
HEADLINE_KERNEL = "k_step<1, 1, 1, 1, false"  # D3Q19, one component, FP32, MRT, step


def sources_sha256() -> str:
    import hashlib

    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update((ROOT / p).read_bytes())
    return h.hexdigest()


def record_traffic(fetch_dir: str, write_dir: str) -> dict:
    """Per-dispatch FETCH_SIZE and WRITE_SIZE (KiB) of the headline kernel from
    two rocprofv3 --pmc runs of 'bench.py --copy-gib 1', each scaled by the
    same counter on the run's two plain 1 GiB copies (which read and write
    exactly 1 GiB each); written with the hash of the kernel sources of this
    tree, which bench.py compares before reporting roofline.traffic."""
    import csv
    import statistics

    def rows(d, counter):
        out = []
        for f in sorted(Path(d).rglob("*counter_collection.csv")):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    if r.get("Counter_Name") == counter:
                        out.append((r["Kernel_Name"], float(r["Counter_Value"])))
        return out

    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rs = rows(d, counter)
        k = [v for n, v in rs if HEADLINE_KERNEL in n]
        cp = [v for n, v in rs if "copyBuffer" in n]
        if not k or len(cp) < 2:
            raise SystemExit(f"{counter}: kernel or copy dispatches not found under {d}")
        res[counter] = (statistics.mean(k), cp[-2:])
    copy_bytes = 1 << 30
    rf = copy_bytes / (1024.0 * statistics.mean(res["FETCH_SIZE"][1]))
    wf = copy_bytes / (1024.0 * statistics.mean(res["WRITE_SIZE"][1]))
    rec = {
        "kernel": HEADLINE_KERNEL + ", ...> (sessile droplet D3Q19 MRT FP32 256^3, bench.py default)",
        "kernel_source_sha256": sources_sha256(),
        "fetch_kib_per_dispatch": res["FETCH_SIZE"][0], "write_kib_per_dispatch": res["WRITE_SIZE"][0],
        "copy_fetch_kib": res["FETCH_SIZE"][1], "copy_write_kib": res["WRITE_SIZE"][1], "copy_bytes": copy_bytes,
        "read_factor": rf, "write_factor": wf,
        "traffic_bytes_per_launch": res["FETCH_SIZE"][0] * 1024 * rf + res["WRITE_SIZE"][0] * 1024 * wf,
        "command_fetch": "rocprofv3 --pmc FETCH_SIZE --output-format csv -d " + fetch_dir +
                         " -o run -- python3 -u bench.py --steps 5 --warmup 1 --no-cpu-baseline --copy-gib 1",
        "command_write": "rocprofv3 --pmc WRITE_SIZE --output-format csv -d " + write_dir +
                         " -o run -- python3 -u bench.py --steps 5 --warmup 1 --no-cpu-baseline --copy-gib 1",
        "command_record": f"python bench.py --record-traffic {fetch_dir} {write_dir}",
    }
    (ROOT / "profiles" / "k_step_traffic.json").write_text(json.dumps(rec, indent=1) + "\n")
    return rec


def measured_traffic(w, name: str) -> float | None:
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE
    measurement (profiles/k_step_traffic.json), scaled by the same counters on
    a 1 GiB copy; None if the kernel sources changed since, or for another
    workload."""
    path = ROOT / "profiles" / "k_step_traffic.json"
    if (not path.exists() or name != "sessile" or w.storage != "F32" or w.collision != "MRT"
            or w.shape != (256, 256, 256)):
        return None
    rec = json.loads(path.read_text())
    return rec["traffic_bytes_per_launch"] if sources_sha256() == rec["kernel_source_sha256"] else None


def make_workload(name: str, n: int, storage: str, collision: str):
    from paper_2506_17713_amd import inputs

    if name == "sessile":
        r = max(15, 30 * n // 256)  # 30 at 256^3 (the configuration), 15 on the small oracle sample
        w, solid, rho = inputs.sessile_3d(n=n, r=float(r), storage=storage, collision=collision,
                                          wet_mode="PHI", wet=1.1)
        desc = f"sessile droplet D3Q19 {collision} Shan-Chen CS T=0.8Tc {n}^3 r={r} wall z=0 phi=1.1"
    elif name == "pcsw":
        w, solid, rho = inputs.pcsw_pack(n=n, buffer=8, storage=storage, dp_rho=0.05)
        desc = (f"capillary pressure - saturation drainage, two-component Shan-Chen D3Q19 BGK, {n}^3 sphere pack "
                f"porosity 0.381 radii 8-16, 8-plane buffers, reservoir planes (inlet +0.05), walls on x/y")
    elif name == "droplet2d":
        w, solid, rho = inputs.droplet_2d(n=n, storage=storage, collision=collision)
        desc = f"droplet D2Q9 {collision} Shan-Chen CS T=0.7Tc {n}^2 r=20 periodic"
    else:
        w, solid, rho = inputs.two_component_pack(n=n, storage=storage)
        desc = (f"two-component Shan-Chen D3Q19 {w.collision} sphere pack {n}^3 radii 8-16 porosity 0.35, "
                f"body force 1e-6")
    return w, solid, rho, desc


def cpu_model() -> str:
    """The host CPU's model name, from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(budget_s: float, name: str) -> dict:
    """FP64 oracle on a small version of the same workload (64^3 sessile,
    full 128^2 droplet, 48^3 two-component pack), as many steps as fit the
    time budget (first step excluded), on all the host threads; then on one
    thread for a quarter of the budget."""
    from oracle import oracle

    n = {"sessile": 64, "droplet2d": 128, "pack2": 48, "pcsw": 48}[name]
    w, solid, rho, desc = make_workload(name, n, "F64", "BGK" if name == "droplet2d" else "MRT")
    if name == "pack2":
        w = w.with_(collision="BGK")
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    st = oracle.State(w, solid, rho)

    def rate(threads: int, budget: float):
        oracle.set_threads(threads)
        st.step(1)
        t0 = time.perf_counter()
        st.step(3)
        dt3 = time.perf_counter() - t0
        k = max(2, int(budget / max(dt3 / 3, 1e-6)))
        t0 = time.perf_counter()
        st.step(k)
        dt = time.perf_counter() - t0
        return w.nc * w.N * k / dt / 1e6, k, dt

    v, k, dt = rate(cores, budget_s)
    v1, k1, dt1 = rate(1, budget_s / 4)
    oracle.set_threads(cores)
    return {"value": v, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{desc}, {k} steps FP64, {dt:.1f} s",
            "value_1thread": v1, "sample_1thread": f"{k1} steps, {dt1:.1f} s", "cpu": cpu_model()}


def cpu_table() -> None:
    """The FP64 oracle's rate on the host at the sizes of the parity runs:
    all threads (OMP_NUM_THREADS) and one thread, first step excluded."""
    import numpy as np

    from oracle import oracle
    from paper_2506_17713_amd import inputs

    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    full = inputs.sphere_pack((400, 400, 400), (8.0, 16.0), 0.35, 0)
    crop = np.ascontiguousarray(full[:64, :64, :64])
    cases = [
        ("D2Q9 BGK droplet 128^2 (full configuration)", make_workload("droplet2d", 128, "F64", "BGK")[:3], 2000, 200),
        ("D3Q19 MRT sessile drop 64^3", make_workload("sessile", 64, "F64", "MRT")[:3], 100, 10),
        ("D3Q19 MRT sessile drop 128^3", make_workload("sessile", 128, "F64", "MRT")[:3], 100, 5),
        ("D3Q19 two-component pack, 64^3 crop of the 400^3 pack",
         inputs.two_component_pack(shape=(64, 64, 64), storage="F64", solid=crop), 100, 10),
    ]
    for name, (w, solid, rho), k_all, k_one in cases:
        st = oracle.State(w, solid, rho)
        row = {"case": name, "cpu": cpu_model(), "cores": cores, "kind": "oracle", "unit": "MLUPS"}
        for threads, k in ((cores, k_all), (1, k_one)):
            oracle.set_threads(threads)
            st.step(1)
            t0 = time.perf_counter()
            st.step(k)
            dt = time.perf_counter() - t0
            row["value" if threads == cores else "value_1thread"] = w.nc * w.N * k / dt / 1e6
            row["steps" if threads == cores else "steps_1thread"] = k
        oracle.set_threads(cores)
        print(json.dumps(row), flush=True)


def run_adjoint(args) -> dict:
    """Gradient of the smooth non-wetting saturation after `steps` (default
    1000) FP32 steps of the 128^3 single-component pack (porosity 0.4, CS at
    T_r = 0.8, MRT) with respect to the per-voxel wetting parameter and T_r,
    with a checkpoint every 100 steps: the forward run stores checkpoints,
    then each segment is recomputed and back-propagated."""
    import torch

    from paper_2506_17713_amd import inputs, lbm

    steps = args.steps
    w, solid, rho = inputs.adjoint_pack(n=args.n or 128, storage="F32")
    rho_mid = 0.5 * (w.rho_min[0] + w.rho_max[0])
    delta = 0.05 * (w.rho_max[0] - w.rho_min[0])
    sol = lbm.Solver(w, solid, rho, device="cuda:0")
    sol.step(args.warmup)  # forward warm-up of the kernels (the gradient starts after it)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(sol.stream)
    sol.step(100)
    ev1.record(sol.stream)
    torch.cuda.synchronize()
    fwd_ms = ev0.elapsed_time(ev1) / 100
    t0 = time.perf_counter()
    L, dwet, dT = sol.grad(steps, 100, "saturation", rho_mid, delta)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    sol.close()
    # forward 'steps' (checkpoints) + recompute 'steps' + reverse 'steps'
    rev_ms = (secs * 1e3 - 2 * steps * fwd_ms) / steps
    return {
        "metric": "MLUPS of the reverse-mode gradient through the fused D3Q19 step (forward, recompute "
                  "and adjoint per step)",
        "value": round(w.N * steps / secs / 1e6, 1), "unit": "MLUPS", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": round(secs * 1e3 / steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"adjoint: CS T=0.8Tc MRT 128^3 sphere pack porosity 0.4 radii 6-14, {steps} "
                               f"steps, checkpoint every 100, dS/d(wet) and dS/dT_r",
                   "nodes": w.N, "components": 1, "storage": "F32", "fluid_nodes": int((solid == 0).sum()),
                   "grad_seconds": round(secs, 3), "forward_ms_per_step": round(fwd_ms, 4),
                   "reverse_ms_per_step_est": round(rev_ms, 4), "S": L,
                   # lbm_grad gives dS/dT (absolute temperature); T = T_r T_c
                   "dS_dTr": dT * inputs.load_coexistence()["CS"]["Tc"]},
        # dominant kernel: the fused forward step (run twice per step: checkpointing
        # pass and segment recomputation), timed above with events on its stream
        "roofline": {"bound": "hbm", "achieved": round(algorithmic_bytes(w, solid) / (fwd_ms * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(algorithmic_bytes(w, solid) / (fwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None, "bytes_per_launch": algorithmic_bytes(w, solid),
                     "kernel": "k_step (forward and recompute; about half of the gradient's time)"},
        "cpu_baseline": None,
    }


def conv_flops(arch, size: int) -> dict:
    """Multiply-add FLOPs (2 per MAC) of the surrogate's 3x3x3 convolutions on
    a size^3 input: forward, and a training step's backward (data gradient of
    every layer but the first, weight gradient of every layer)."""
    level = {"enc0": 0, "dec0": 0, "head": 0, "enc1": 1, "dec1": 1, "enc2": 2, "dec2": 2, "bot": 3}
    fwd = bwd = 0.0
    for name, ci, co in arch:
        lv = next(v for k, v in level.items() if name.startswith(k))
        f = 2.0 * ci * co * 27 * (size >> lv) ** 3
        fwd += f
        bwd += f + (f if name != "enc0a" else 0.0)
    return {"forward": fwd, "backward": bwd}


def run_surrogate(args) -> dict:
    """Surrogate throughput: inference on a 256^3 pack and training steps
    (forward, masked MSE, backward, Adam) on 128^3 packs, BF16 MFMA.  The
    timed regions hold every kernel of the pass (pooling, upsampling, ReLU and
    skip additions besides the convolutions); the FLOPs counted are the
    convolutions'."""
    import numpy as np
    import torch

    from paper_2506_17713_amd import inputs, nn
    from paper_2506_17713_amd.surrogate import ARCH, Surrogate

    model = Surrogate(prec=nn.BF16, seed=0)
    st = torch.cuda.current_stream()

    def timed(fn, reps):
        for _ in range(max(args.warmup, 1)):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    big = torch.tensor((inputs.sphere_pack((256,) * 3, (6.0, 14.0), 0.4, 1000) == 0).astype(np.float32)[None],
                       device="cuda")
    t_inf = timed(lambda: model.forward(big), args.steps)
    small = torch.tensor((inputs.sphere_pack((128,) * 3, (6.0, 14.0), 0.4, 7) == 0).astype(np.float32)[None],
                         device="cuda")
    target = torch.zeros((4, 128, 128, 128), dtype=torch.float32, device="cuda")

    def train_step():
        tape = []
        out = model.forward(small, tape)
        _, dout = nn.mse(out, target, small[0])
        model.adam_step(model.backward(tape, dout), 1e-4)

    t_train = timed(train_step, args.steps)
    f256, f128 = conv_flops(ARCH, 256), conv_flops(ARCH, 128)
    inf_tf = f256["forward"] / t_inf / 1e12
    train_tf = (f128["forward"] + f128["backward"]) / t_train / 1e12
    return {
        "metric": "TFLOP/s of the surrogate's 3x3x3 convolutions (BF16 MFMA, FP32 accumulation), inference",
        "value": round(inf_tf, 2), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t_inf * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "surrogate U-Net (15 periodic 3x3x3 convolutions, 1.32 M parameters), inference "
                               "on a 256^3 pack; training steps on 128^3",
                   "inference_ms": round(t_inf * 1e3, 3), "inference_conv_TFLOP": round(f256["forward"] / 1e12, 4),
                   "train_step_ms": round(t_train * 1e3, 3),
                   "train_step_conv_TFLOP": round((f128["forward"] + f128["backward"]) / 1e12, 4),
                   "train_TFLOP_s": round(train_tf, 2)},
        "roofline": {"bound": "mfma", "achieved": round(inf_tf, 2), "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": round(inf_tf / 2500.0, 4), "traffic": None,
                     "kernel": "whole inference pass (convolutions' FLOPs over all kernels' time)"},
        "cpu_baseline": None,
    }


def main():
    args = parse()
    if args.record_traffic:
        print(json.dumps(record_traffic(*args.record_traffic), indent=1))
        return
    if args.cpu_table:
        cpu_table()
        return
    if args.steps is None:
        args.steps = {"adjoint": 1000, "surrogate": 20}.get(args.workload, 500)
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU only; sharding over GPUs (x-slabs with a "
                                   "face exchange over RCCL) is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2506_17713_amd import inputs, lbm

    if args.workload == "adjoint":
        print(json.dumps(run_adjoint(args)), flush=True)
        return
    if args.workload == "surrogate":
        print(json.dumps(run_surrogate(args)), flush=True)
        return
    n = args.n or {"sessile": 256, "droplet2d": 128, "pack2": 400, "pcsw": 256}[args.workload]
    storage = args.storage if args.workload != "droplet2d" or args.storage != "F32" else "F64"
    collision = "BGK" if args.workload != "sessile" else args.collision
    w, solid, rho, desc = make_workload(args.workload, n, storage, collision)
    layout = args.layout or ("FLUID" if args.workload in ("pack2", "pcsw") else "DENSE")
    if layout != "DENSE":
        w = w.with_(layout=layout)
        desc += ", fluid-only layout"
    sol = lbm.Solver(w, solid, rho, device="cuda:0")
    stream = sol.stream
    print(f"# init done {w.shape} {w.storage} {w.collision}", file=sys.stderr, flush=True)
    sol.step(1)  # first step excluded (the paper excludes the compile step)
    sol.step(args.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    sol.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    stats = sol.stats()
    ms_step = ms / args.steps
    mlups = w.nc * w.N * args.steps / (ms * 1e-3) / 1e6
    b_alg = algorithmic_bytes(w, solid)
    achieved = b_alg / (ms_step * 1e-3) / 1e9
    print(f"# {args.steps} steps: {ms:.2f} ms (events), wall {wall:.3f} s, mass {stats['mass'][0]:.6e}, "
          f"nonfinite {stats['nonfinite']}", file=sys.stderr, flush=True)
    traffic = measured_traffic(w, args.workload)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_seconds, args.workload)
    dtype = {"F32": "f32", "F64": "f64", "F32F64": "f32 storage, f64 arithmetic", "F16DEV": "f16dev+f32",
             "BF16DEV": "bf16dev+f32"}[w.storage]
    lat = "D2Q9" if args.workload == "droplet2d" else "D3Q19"
    line = {
        "metric": f"MLUPS of fused {lat} Shan-Chen step (% HBM roofline)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": desc, "nodes": w.N, "components": w.nc,
                   "storage": w.storage, "fluid_nodes": int((solid == 0).sum()),
                   "fluid_MLUPS": round(w.nc * int((solid == 0).sum()) * args.steps / (ms * 1e-3) / 1e6, 1)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "bytes_per_launch": b_alg,
                     "kernel": "k_step (fused step)" if w.layout == "DENSE" else
                     "one step = k_fl_rho + k_fl_solid + k_fl_step (fluid-only layout)"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    sol.close()
    if args.copy_gib > 0:
        # reference traffic for FETCH_SIZE / WRITE_SIZE: each copy reads and
        # writes exactly copy_gib GiB
        n = int(args.copy_gib * (1 << 30)) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"# {2} copies of {args.copy_gib} GiB done", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
