"""3-D convolutional encoder-decoder that predicts steady single-phase flow in
a porous medium, trained on fields the solver generates, used to warm-start
permeability runs.

The paper computes permeability by running the solver from rest to steady
state and applying Darcy's law, k = nu <u_x> / a (Sec. 3.4.1: 50,000 steps).
Here the network maps the pore mask to the steady fields in units that do not
depend on the forcing: u nu / a (three channels) and the pressure deviation
(rho - 1) c_s^2 / a (one channel, a length).  The solver then starts from
f = f^eq(rho_pred, u_pred - a/2) and runs to the same stopping rule, so the
plain solver remains the arbiter of the permeability.  The pressure channel
matters: the steady density is not uniform (about +-0.2 % in these packs),
and a start from the exact velocity with rho = 1 converges no faster than a
start from rest because the pressure has to build up first.

Network (about 1.3 M parameters; every convolution 3x3x3, periodic):
  encoder  16 -> 16 | pool | 32, 32 | pool | 64, 64 | pool | 128, 128
  decoder  up | 64 (+ skip) 64 | up | 32 (+ skip) 32 | up | 16 (+ skip) 16 | head 4
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
        ("dec0a", 32, 16), ("dec0b", 16, 16), ("head", 16, 4)]
OUT_CH = 4  # u nu / a (x, y, z), (rho - 1) c_s^2 / a


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
        self.scale = np.ones(OUT_CH)  # per-channel target normalisation
        self.flow_gain = 1.0  # velocity calibration (calibrate_flow)
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

    def _conv_add(self, name, x, s, tape):
        """relu(conv(x)) + s.  Inference adds the skip in the convolution's
        epilogue (the same operations in the same order); training keeps the
        two steps, whose intermediate the backward pass reads."""
        if tape is not None:
            return self._add(self._conv(name, x, True, tape), s, tape)
        return nn.conv(x, self.pk[name], self.W[name].shape[0], bias=self.b[name], skip=s, relu=True, prec=self.prec)

    def _forward_chain(self, mask: torch.Tensor) -> torch.Tensor:
        """Inference in BF16: each convolution hands its successor the BF16
        channels-innermost copy of its output (lbm_nn_conv_x), pooling and
        upsampling write that layout too, and FP32 tensors are written only
        where pooling, upsampling, a skip or the result reads them.  The same
        operations and roundings as forward()."""
        def cv(name, dhw, X=None, xb=None, skip=None, relu=True, want_y=True, want_yb=True):
            co, ci = self.W[name].shape[0], self.W[name].shape[1]
            return nn.conv_x(self.pk[name], co, ci, dhw, X=X, xb=xb, bias=self.b[name], skip=skip, relu=relu,
                             want_y=want_y, want_yb=want_yb)

        d0 = tuple(mask.shape[1:])
        d1, d2, d3 = (tuple(v // 2 for v in d0), tuple(v // 4 for v in d0), tuple(v // 8 for v in d0))
        _, b = cv("enc0a", d0, X=mask, want_y=False)
        s0, _ = cv("enc0b", d0, xb=b, want_yb=False)
        _, b = cv("enc1a", d1, xb=nn.pool_x(s0), want_y=False)
        s1, _ = cv("enc1b", d1, xb=b, want_yb=False)
        _, b = cv("enc2a", d2, xb=nn.pool_x(s1), want_y=False)
        s2, _ = cv("enc2b", d2, xb=b, want_yb=False)
        _, b = cv("bota", d3, xb=nn.pool_x(s2), want_y=False)
        a, _ = cv("botb", d3, xb=b, want_yb=False)
        _, b = cv("dec2a", d2, xb=nn.up_x(a), skip=s2, want_y=False)
        a, _ = cv("dec2b", d2, xb=b, want_yb=False)
        _, b = cv("dec1a", d1, xb=nn.up_x(a), skip=s1, want_y=False)
        a, _ = cv("dec1b", d1, xb=b, want_yb=False)
        _, b = cv("dec0a", d0, xb=nn.up_x(a), skip=s0, want_y=False)
        _, b = cv("dec0b", d0, xb=b, want_y=False)
        y, _ = cv("head", d0, xb=b, relu=False, want_yb=False)
        return y

    def forward(self, mask: torch.Tensor, tape=None) -> torch.Tensor:
        """mask: float32 [1, D, H, W] (1 = pore).  D, H, W divisible by 8."""
        if tape is None and self.prec == nn.BF16:
            return self._forward_chain(mask)
        c = self._conv
        a = c("enc0a", mask, True, tape)
        s0 = c("enc0b", a, True, tape)
        a = c("enc1a", self._pool(s0, tape), True, tape)
        s1 = c("enc1b", a, True, tape)
        a = c("enc2a", self._pool(s1, tape), True, tape)
        s2 = c("enc2b", a, True, tape)
        a = c("bota", self._pool(s2, tape), True, tape)
        a = c("botb", a, True, tape)
        a = self._conv_add("dec2a", self._up(a, tape), s2, tape)
        a = c("dec2b", a, True, tape)
        a = self._conv_add("dec1a", self._up(a, tape), s1, tape)
        a = c("dec1b", a, True, tape)
        a = self._conv_add("dec0a", self._up(a, tape), s0, tape)
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
        """Steady fields on the host, float64 [4, D, H, W], zero in solids:
        u nu / a (channels 0-2) and (rho - 1) c_s^2 / a (channel 3)."""
        out = self.forward(mask)
        gain = np.array([self.flow_gain] * 3 + [1.0])
        return out.cpu().numpy().astype(np.float64) * (self.scale * gain)[:, None, None, None] * mask.cpu().numpy()

    def state(self) -> dict:
        return {"scale": self.scale, "t": self.t, "flow_gain": self.flow_gain,
                **{f"W_{n}": self.W[n].cpu().numpy() for n, _, _ in ARCH},
                **{f"b_{n}": self.b[n].cpu().numpy() for n, _, _ in ARCH}}

    def load_state(self, st: dict) -> None:
        self.scale = np.asarray(st["scale"], dtype=np.float64)
        self.t = int(st["t"])
        self.flow_gain = float(st["flow_gain"]) if "flow_gain" in st else 1.0
        for n, _, _ in ARCH:
            self.W[n].copy_(torch.as_tensor(np.asarray(st[f"W_{n}"]), dtype=torch.float32))
            self.b[n].copy_(torch.as_tensor(np.asarray(st[f"b_{n}"]), dtype=torch.float32))
        self.repack()


# ---------------------------------------------------------------------------
# Solver side: steady single-phase flow and Darcy permeability.
# ---------------------------------------------------------------------------
NU = (1.0 - 0.5) / 3.0  # BGK tau = 1


def solve_steady(solid: np.ndarray, accel=1e-5, u0=None, rho0=None, tol=1e-6, check=100, max_steps=100000,
                 device="cuda", storage="F64", k_tol=1e-4, layout="DENSE"):
    """Run single-phase flow (BGK tau = 1, body acceleration along x) from
    f^eq(rho0, u0) (rest at rho = 1 by default; host arrays, or device
    tensors of the compute type as from warm_start_device) until the residual
    sum|u_x(t) - u_x(t-100)| / sum|u_x| < tol.  FP64 populations by default:
    with u ~ 1e-4 the FP32 rounding noise of the velocity alone keeps this
    residual near 3e-5.

    Along the way it records when the permeability estimate k(t) first
    changed by less than k_tol (relative) over two consecutive checks: the
    time-to-permeability stopping rule, which needs no converged answer.
    Returns dict(u [3, N] and rho [N] torch tensors, steps, seconds, k,
    residual, k_steps, k_seconds, k_at_k_steps, history of (steps, residual,
    k, seconds) per check).  layout="FLUID" stores the fluid nodes only
    (lbm_params.layout: the same step, faster on packs)."""
    w, solid, rho = inputs.single_phase_pack(shape=solid.shape, solid=solid, accel=accel, storage=storage)
    w = w.with_(layout=layout)
    on_device = isinstance(rho0, torch.Tensor)
    if rho0 is not None and not on_device:
        rho = np.asarray(rho0, dtype=np.float64).reshape(rho.shape)
    porosity = float((solid == 0).mean())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol = lbm.Solver(w, solid, rho, u0=None if on_device else u0, device=device)
    if on_device:
        sol.reset(rho0, u0)
    sol.stats()  # first reduction sets the reference velocity
    steps, res, calm = 0, 1.0, 0
    hist, k_prev, k_hit = [], None, None
    while steps < max_steps:
        sol.step(check)
        steps += check
        st = sol.stats()
        res = st["residual"]
        k = NU * st["mean_ux"] * porosity / accel
        now = time.perf_counter() - t0
        hist.append((steps, res, k, now))
        if k_prev is not None and abs(k - k_prev) < k_tol * abs(k):
            calm += 1
            if calm == 2 and k_hit is None:
                k_hit = (steps, now, k)
        else:
            calm = 0
        k_prev = k
        if res < tol:
            break
    r, u = sol.moments(0)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    sol.close()
    if k_hit is None:
        k_hit = (steps, secs, k)
    return {"u": u, "rho": r, "steps": steps, "seconds": secs, "k": k, "residual": res,
            "k_steps": k_hit[0], "k_seconds": k_hit[1], "k_at_k_steps": k_hit[2], "history": hist}


def targets_of(sol_out: dict, solid: np.ndarray, accel: float) -> np.ndarray:
    """Network targets from a steady solution, computed on the host: u nu / a
    and (rho - 1) c_s^2 / a at pore nodes (zero in solids), float32
    [4, D, H, W]."""
    shape = solid.shape
    fl = (solid == 0)
    u = sol_out["u"].cpu().numpy().astype(np.float64).reshape((3,) + shape) * (NU / accel)
    p = (sol_out["rho"].cpu().numpy().astype(np.float64).reshape(shape) - 1.0) / (3.0 * accel)
    return (np.concatenate([u, p[None]]) * fl).astype(np.float32)


def warm_fields(pred: np.ndarray, solid: np.ndarray, accel: float):
    """Initial (rho0 [1, N], u0 [3, N]) for the solver from predicted fields
    (Surrogate.predict units): the pressure channel is shifted to zero mean
    over the pores so the start holds the same mass as rho = 1, and the
    velocity is turned into the equilibrium velocity j/rho = u - F/(2 rho)."""
    fl = (solid == 0).reshape(-1)
    u = pred[:3].reshape(3, -1) * (accel / NU)
    u[0] -= 0.5 * accel
    u *= fl
    p = pred[3].reshape(-1).copy()
    p -= p[fl].mean()
    rho = np.where(fl, 1.0 + 3.0 * accel * p, 1.0)
    return rho[None], u


def warm_start_device(model: Surrogate, mask: torch.Tensor, accel: float, dtype=torch.float64):
    """The start of warm_fields(model.predict(mask), ...) computed on the GPU
    from the network output (lbm_nn_warm_fields): device (rho0 [1, N],
    u0 [3, N]) of the solver's compute type, for solve_steady / Solver.reset."""
    out = model.forward(mask)
    g = model.flow_gain
    c = [float(model.scale[d]) * g * accel / NU for d in range(3)] + [3.0 * accel * float(model.scale[3])]
    return nn.warm_fields(out, mask[0], c, 0.5 * accel, dtype)


def make_dataset(n_samples: int, size=128, seed0=0, accel=1e-5, log=print, device="cuda",
                 radii=(6.0, 14.0)):
    """Seeded packs (porosity U(0.3, 0.5)) and their steady fields (targets_of)."""
    xs, ys, info = [], [], []
    rng = np.random.default_rng(12345)
    for s in range(n_samples):
        por = float(rng.uniform(0.3, 0.5))
        solid = inputs.sphere_pack((size,) * 3, radii, por, seed0 + s)
        r = solve_steady(solid, accel=accel, device=device)
        xs.append(torch.tensor((solid == 0).astype(np.float32)[None], device=device))
        ys.append(targets_of(r, solid, accel))
        info.append({"seed": seed0 + s, "porosity": float((solid == 0).mean()), "steps": r["steps"],
                     "seconds": r["seconds"], "k": r["k"]})
        log(f"sample {s}: porosity {info[-1]['porosity']:.3f} steps {r['steps']} k {r['k']:.4f} "
            f"({r['seconds']:.1f} s)")
    return xs, ys, info


def calibrate_flow(model: Surrogate, xs, ys) -> float:
    """Set model.flow_gain, the one factor on the predicted velocity that best
    reproduces the permeabilities of the given samples (least squares over
    k_i = <u_x nu / a>_V; targets as from targets_of), and return it.

    The masked MSE of training weighs the field voxel by voxel and leaves the
    volume mean, which is k, loosely pinned: trained models carry a common k
    bias of 10-20 % of either sign, the same on their training packs as on
    held-out ones, with a few percent scatter around it."""
    model.flow_gain = 1.0
    kp = np.array([model.predict(x)[0].mean() for x in xs])
    kt = np.array([float(np.asarray(y[0], dtype=np.float64).mean()) for y in ys])
    model.flow_gain = float((kp * kt).sum() / (kp * kp).sum())
    return model.flow_gain


def symmetry(rng, shape):
    """A random symmetry of the steady problem (periodic pack, body force
    along +x): periodic shift, axis flips and, for D == H, the exchange of the
    z and y axes.  Returns the lbm_nn_augment arguments for the four target
    channels (u_x, u_y, u_z, p).  The velocity maps as A u(g^-1 r) with A the
    flips after the exchange; flipping x also reverses the forcing, and since
    the flow is linear in the forcing (Stokes regime) every channel is then
    negated, which keeps u_x as it is."""
    D, H, W = shape
    shift = [int(rng.integers(n)) for n in shape]
    flip = [int(rng.integers(2)) for _ in range(3)]  # along (z, y, x)
    swap = bool(D == H and rng.integers(2))
    return symmetry_args(shift, flip, swap)


def symmetry_args(shift, flip, swap: bool):
    """lbm_nn_augment arguments of one symmetry (see symmetry())."""
    sz, sy, sx = (-1.0 if f else 1.0 for f in flip)
    src = [0, 2 if swap else 1, 1 if swap else 2, 3]
    sign = [1.0, sx * sy, sx * sz, sx]
    return list(shift), list(flip), bool(swap), src, sign


def train(model: Surrogate, xs, ys, epochs: int, lr=1e-3, log=print, seed=0, augment=False):
    """xs: device masks [1, D, H, W]; ys: host float32 targets [4, D, H, W]
    (targets_of).  Each channel is normalised on the host to unit RMS over the
    pore voxels of the whole set, then the set is uploaded once.  With
    augment, every sample is seen under a fresh random symmetry (symmetry())."""
    npore = sum(float(x.sum()) for x in xs)
    s2 = sum((y.astype(np.float64) ** 2).sum(axis=(1, 2, 3)) for y in ys) / npore
    model.scale = np.sqrt(np.maximum(s2, 1e-30))
    inv = (1.0 / model.scale)[:, None, None, None]
    ys_n = [torch.tensor((y * inv).astype(np.float32), device=xs[0].device) for y in ys]
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        tot = 0.0
        for i in rng.permutation(len(xs)):
            x, y = xs[i], ys_n[i]
            if augment:
                shift, flip, swap, src, sign = symmetry(rng, tuple(x.shape[1:]))
                x = nn.augment(x, shift, flip, swap, [0], [1.0])
                y = nn.augment(y, shift, flip, swap, src, sign)
            tape = []
            out = model.forward(x, tape)
            loss, dout = nn.mse(out, y, x[0])
            grads = model.backward(tape, dout)
            model.adam_step(grads, lr)
            tot += float(loss)
        hist.append(tot / len(xs))
        log(f"epoch {ep}: mse {hist[-1]:.5f}")
    return hist


def first_within(history, k_ref: float, tol: float = 0.01):
    """(steps, seconds) of the first check whose permeability lies within tol
    (relative) of k_ref, or None: the time to a permeability estimate within
    1 % of the plain solver's converged one."""
    for steps, _res, k, secs in history:
        if abs(k - k_ref) < tol * abs(k_ref):
            return steps, secs
    return None
