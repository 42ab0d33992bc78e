"""3-D convolutional encoder-decoder that predicts steady single-phase flow in
a porous medium, trained on fields the solver generates, used to warm-start
permeability runs.

The paper computes permeability by running the solver from rest to steady
state and applying Darcy's law, k = nu <u_x> / a (Sec. 3.4.1: 50,000 steps).
Here the network maps the pore mask to u nu / a; the solver then starts from
f = f^eq(1, u_pred) and runs to the same residual, so the plain solver
remains the judge of the permeability.

Network (about 1.3 M parameters; every convolution 3x3x3, periodic):
  encoder  16 -> 16 | pool | 32, 32 | pool | 64, 64 | pool | 128, 128
  decoder  up | 64 (+ skip) 64 | up | 32 (+ skip) 32 | up | 16 (+ skip) 16 | head 3
with ReLU after every convolution but the head.  Forward, backward and Adam
run in the library's kernels (paper_2506_17713_amd.nn); torch only holds
memory.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import inputs, lbm, nn

ARCH = [("enc0a", 1, 16), ("enc0b", 16, 16), ("enc1a", 16, 32), ("enc1b", 32, 32),
        ("enc2a", 32, 64), ("enc2b", 64, 64), ("bota", 64, 128), ("botb", 128, 128),
        ("dec2a", 128, 64), ("dec2b", 64, 64), ("dec1a", 64, 32), ("dec1b", 32, 32),
        ("dec0a", 32, 16), ("dec0b", 16, 16), ("head", 16, 3)]


class Surrogate:
    def __init__(self, device="cuda", prec=nn.BF16, seed=0):
        self.device = torch.device(device)
        self.prec = prec
        rng = np.random.default_rng(seed)
        self.W, self.b, self.m, self.v = {}, {}, {}, {}
        for name, ci, co in ARCH:
            std = math.sqrt(2.0 / (ci * 27)) if name != "head" else math.sqrt(1.0 / (ci * 27))
            self.W[name] = torch.tensor(rng.normal(0.0, std, size=(co, ci, 27)), dtype=torch.float32,
                                        device=self.device)
            self.b[name] = torch.zeros(co, dtype=torch.float32, device=self.device)
            for d in (self.m, self.v):
                d[name] = (torch.zeros_like(self.W[name]), torch.zeros_like(self.b[name]))
        self.t = 0
        self.scale = 1.0  # target normalisation (u nu / a per unit output)
        self.repack()

    def n_params(self) -> int:
        return sum(self.W[n].numel() + self.b[n].numel() for n, _, _ in ARCH)

    def repack(self):
        self.pk = {n: nn.pack(self.W[n], False, self.prec) for n, _, _ in ARCH}
        self.pkT = {n: nn.pack(self.W[n], True, self.prec) for n, _, _ in ARCH}

    # ---- forward ------------------------------------------------------------
    def _conv(self, name, x, relu, tape):
        y = nn.conv(x, self.pk[name], self.W[name].shape[0], bias=self.b[name], relu=relu, prec=self.prec)
        if tape is not None:
            tape.append(("conv", name, x, y, relu))
        return y

    def _pool(self, x, tape):
        y = nn.pool(x)
        if tape is not None:
            tape.append(("pool", x, y))
        return y

    def _up(self, x, tape):
        y = nn.up(x)
        if tape is not None:
            tape.append(("up", x, y))
        return y

    def _add(self, a, s, tape):
        y = a.clone()  # device copy
        nn.add_(y, s)
        if tape is not None:
            tape.append(("add", a, s, y))
        return y

    def forward(self, mask: torch.Tensor, tape=None) -> torch.Tensor:
        """mask: float32 [1, D, H, W] (1 = pore).  D, H, W divisible by 8."""
        c = self._conv
        a = c("enc0a", mask, True, tape)
        s0 = c("enc0b", a, True, tape)
        a = c("enc1a", self._pool(s0, tape), True, tape)
        s1 = c("enc1b", a, True, tape)
        a = c("enc2a", self._pool(s1, tape), True, tape)
        s2 = c("enc2b", a, True, tape)
        a = c("bota", self._pool(s2, tape), True, tape)
        a = c("botb", a, True, tape)
        a = self._add(c("dec2a", self._up(a, tape), True, tape), s2, tape)
        a = c("dec2b", a, True, tape)
        a = self._add(c("dec1a", self._up(a, tape), True, tape), s1, tape)
        a = c("dec1b", a, True, tape)
        a = self._add(c("dec0a", self._up(a, tape), True, tape), s0, tape)
        a = c("dec0b", a, True, tape)
        return c("head", a, False, tape)

    # ---- backward -------------------------------------------------------------
    def backward(self, tape, dout: torch.Tensor) -> dict:
        grads = {}
        dact = {id(tape[-1][3]): dout}

        def acc(t, g):
            k = id(t)
            if k in dact:
                nn.add_(dact[k], g)
            else:
                dact[k] = g

        for op in reversed(tape):
            kind = op[0]
            if kind == "conv":
                _, name, x, y, relu = op
                dy = dact.pop(id(y))
                if relu:
                    nn.relu_bwd(y, dy)
                grads[name] = (nn.wgrad(x, dy, self.prec), nn.bias_grad(dy))
                if name != "enc0a":
                    acc(x, nn.conv(dy, self.pkT[name], x.shape[0], prec=self.prec))
            elif kind == "pool":
                _, x, y = op
                dy = dact.pop(id(y))
                if id(x) in dact:
                    nn.pool_bwd(dy, dact[id(x)], accumulate=True)
                else:
                    dx = torch.empty_like(x)
                    nn.pool_bwd(dy, dx, accumulate=False)
                    dact[id(x)] = dx
            elif kind == "up":
                _, x, y = op
                acc(x, nn.up_bwd(dact.pop(id(y))))
            else:  # add
                _, a, s, y = op
                dy = dact.pop(id(y))
                acc(s, dy.clone())
                acc(a, dy)
        return grads

    def adam_step(self, grads: dict, lr: float) -> None:
        self.t += 1
        for name, _, _ in ARCH:
            gW, gb = grads[name]
            nn.adam_(self.W[name], gW, self.m[name][0], self.v[name][0], self.t, lr)
            nn.adam_(self.b[name], gb, self.m[name][1], self.v[name][1], self.t, lr)
        self.repack()

    def predict(self, mask: torch.Tensor) -> np.ndarray:
        """u nu / a on the host, float64 [3, D, H, W], zero in solids."""
        out = self.forward(mask)
        return out.cpu().numpy().astype(np.float64) * self.scale * mask.cpu().numpy()

    def state(self) -> dict:
        return {"scale": self.scale, "t": self.t,
                **{f"W_{n}": self.W[n].cpu().numpy() for n, _, _ in ARCH},
                **{f"b_{n}": self.b[n].cpu().numpy() for n, _, _ in ARCH}}


# ---------------------------------------------------------------------------
# Solver side: steady single-phase flow and Darcy permeability.
# ---------------------------------------------------------------------------
NU = (1.0 - 0.5) / 3.0  # BGK tau = 1


def solve_steady(solid: np.ndarray, accel=1e-5, u0=None, tol=1e-6, check=100, max_steps=100000, device="cuda",
                 storage="F64"):
    """Run single-phase flow (BGK tau = 1, rho = 1, body acceleration along x)
    until the residual sum|u_x(t) - u_x(t-100)| / sum|u_x| < tol.
    FP64 populations by default: with u ~ 1e-4 the FP32 rounding noise of the
    velocity alone keeps this residual near 3e-5.
    Returns dict(u [3, N] torch tensor, steps, seconds, k, residual)."""
    w, solid, rho = inputs.single_phase_pack(shape=solid.shape, solid=solid, accel=accel, storage=storage)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol = lbm.Solver(w, solid, rho, u0=u0, device=device)
    sol.stats()  # first reduction sets the reference velocity
    steps, res = 0, 1.0
    while steps < max_steps:
        sol.step(check)
        steps += check
        st = sol.stats()
        res = st["residual"]
        if res < tol:
            break
    _, u = sol.moments(-1, rho=False)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    porosity = float((solid == 0).mean())
    k = NU * st["mean_ux"] * porosity / accel
    sol.close()
    return {"u": u, "steps": steps, "seconds": secs, "k": k, "residual": res}


def make_dataset(n_samples: int, size=128, seed0=0, accel=1e-5, log=print, device="cuda"):
    """Seeded packs (radii 6-14, porosity U(0.3, 0.5)) and their steady u nu / a."""
    xs, ys, info = [], [], []
    rng = np.random.default_rng(12345)
    for s in range(n_samples):
        por = float(rng.uniform(0.3, 0.5))
        solid = inputs.sphere_pack((size,) * 3, (6.0, 14.0), por, seed0 + s)
        r = solve_steady(solid, accel=accel, device=device)
        mask = torch.tensor((solid == 0).astype(np.float32)[None], device=device)
        target = r["u"].cpu().numpy().astype(np.float64).reshape(3, size, size, size) * (NU / accel)
        xs.append(mask)
        ys.append(target)
        info.append({"seed": seed0 + s, "porosity": float((solid == 0).mean()), "steps": r["steps"],
                     "seconds": r["seconds"], "k": r["k"]})
        log(f"sample {s}: porosity {info[-1]['porosity']:.3f} steps {r['steps']} k {r['k']:.4f} "
            f"({r['seconds']:.1f} s)")
    return xs, ys, info


def train(model: Surrogate, xs, ys, epochs: int, lr=1e-3, log=print, seed=0):
    """ys: host float64 targets u nu / a [3, D, H, W]; normalised to unit RMS
    over pore voxels on the host and kept on the device in FP32."""
    s2 = sum(float((y * y).sum()) for y in ys) / sum(3.0 * float(x.sum()) for x in xs)
    model.scale = math.sqrt(s2)
    ys_n = [torch.tensor((y / model.scale).astype(np.float32), device=xs[0].device) for y in ys]
    order = np.random.default_rng(seed).permutation
    hist = []
    for ep in range(epochs):
        tot = 0.0
        for i in order(len(xs)):
            tape = []
            out = model.forward(xs[i], tape)
            loss, dout = nn.mse(out, ys_n[i], xs[i][0])
            grads = model.backward(tape, dout)
            model.adam_step(grads, lr)
            tot += float(loss)
        hist.append(tot / len(xs))
        log(f"epoch {ep}: mse {hist[-1]:.5f}")
    return hist
