"""Seeded synthetic inputs and workload descriptions.

This module feeds the same bytes to the GPU library and to the CPU oracle.  It
holds no arithmetic of the method itself -- no equilibrium, force, collision or
streaming -- only geometry, initial density fields, noise and the parameter
sets of the workloads.

Arrays are in (z, y, x) order with x fastest; a D2Q9 domain has nz = 1.

Initial fields follow the paper's tanh interface profile (Sec. 3.1, Eq. 18),
read as rho = (rho_in + rho_out)/2 - (rho_in - rho_out)/2 tanh(2 (d - r) / w):
the printed form subtracts the two halves and would give zero in the vapour.

Porous media stand in for the Digital Rocks sphere packs the paper uses
(Sec. 3.4): periodic Boolean models of overlapping spheres with uniformly
distributed radii; a voxel is solid if its centre lies inside a sphere
(minimum-image distance).  The number of spheres follows the Boolean-model
porosity phi = exp(-n E[V_sphere] / V).
"""
from __future__ import annotations

import json
import math
from dataclasses import dataclass, field, replace
from pathlib import Path

import numpy as np

_COEX = Path(__file__).resolve().parent / "data" / "cs_coexistence.json"


def load_coexistence() -> dict:
    """Carnahan-Starling (a=1, b=4, R=1) critical temperature, Maxwell
    coexistence densities and the calibrated Zhang-Chen weight A per reduced
    temperature, as written by tests/golden/make_cs_coexistence.py."""
    with open(_COEX) as fh:
        return json.load(fh)


# --------------------------------------------------------------------------
# Workload description (plain numbers; marshalled by each side separately).
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    lattice: str                      # "D2Q9" or "D3Q19"
    shape: tuple                      # (nz, ny, nx)
    nc: int = 1
    collision: str = "BGK"            # "BGK", "MRT" or "CLBM" (central moments)
    storage: str = "F32"              # "F64", "F32", "F32F64", "F16DEV", "BF16DEV"
    tau: tuple = (1.0, 1.0)
    mrt_s: tuple | None = None        # explicit rates per component, else defaults
    psi_kind: tuple = ("CS", "CS")    # "CS" (Carnahan-Starling EOS) or "DENSITY"
    eos_a: tuple = (1.0, 1.0)
    eos_b: tuple = (4.0, 4.0)
    eos_R: tuple = (1.0, 1.0)
    eos_T: tuple = (0.0, 0.0)         # absolute temperature
    alpha: tuple = (1.0, 1.0)
    A: tuple = (0.0, 0.0)
    g: tuple = ((-1.0, 0.0), (0.0, -1.0))
    body: tuple = (0.0, 0.0, 0.0)     # body acceleration
    wet_mode: tuple = ("PHI", "PHI")
    wet: tuple = (1.0, 1.0)           # uniform phi or drho
    rho_min: tuple = (0.0, 0.0)
    rho_max: tuple = (1e30, 1e30)
    common_velocity: bool = True
    kappa: tuple = (0.0, 0.0)         # surface-tension adjustment (D2Q9 MRT, Eq. 14-16)
    res_rho: tuple = ((0.0, 0.0), (0.0, 0.0))  # fixed densities of reservoirs 0 and 1 (mask 2, 3)
    window: tuple = (0, 0)            # planes of the capillary-pressure measurement (0, 0: all)
    layout: str = "DENSE"             # "DENSE" or "FLUID" (fluid nodes only: porous media)
    steps: int = 100
    extra: dict = field(default_factory=dict)

    @property
    def shape_xyz(self):
        nz, ny, nx = self.shape
        return nx, ny, nz

    @property
    def N(self) -> int:
        return int(np.prod(self.shape))

    @property
    def q(self) -> int:
        return 9 if self.lattice == "D2Q9" else 19

    def mrt_rates(self, k: int) -> tuple:
        """Relaxation rate of each moment row (rows in the order of the
        Lallemand-Luo D2Q9 / d'Humieres D3Q19 bases).  Defaults: 1/tau on the
        conserved and stress rows, 1.0 on every other row."""
        if self.mrt_s is not None:
            return tuple(self.mrt_s[k])
        sv = 1.0 / self.tau[k]
        if self.lattice == "D2Q9":
            # rho, e, eps, jx, qx, jy, qy, pxx, pxy
            return (sv, 1.0, 1.0, sv, 1.0, sv, 1.0, sv, sv)
        # rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy, pyz, pxz, mx, my, mz
        r = [1.0] * 19
        for i in (0, 3, 5, 7, 9, 11, 13, 14, 15):
            r[i] = sv
        return tuple(r)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def dhumieres_rates(tau: float) -> tuple:
    """D3Q19 MRT rates of d'Humieres et al. (2002) in the row order of
    Workload.mrt_rates: s_nu = 1/tau on the stress rows (3p_xx, p_ww, p_xy,
    p_yz, p_xz) and on the conserved rows (where m - m^eq vanishes for one
    component), s_e = 1.19, s_eps = 1.4, s_q = 1.2, s_pi = 1.4, s_m = 1.98."""
    sv = 1.0 / tau
    return (sv, 1.19, 1.4, sv, 1.2, sv, 1.2, sv, 1.2, sv, 1.4, sv, 1.4, sv, sv, sv, 1.98, 1.98, 1.98)


# --------------------------------------------------------------------------
# Geometry and initial-field generators.
# --------------------------------------------------------------------------
def grid(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)


def tanh_profile(d: np.ndarray, r: float, w: float, rho_in: float, rho_out: float) -> np.ndarray:
    return 0.5 * (rho_in + rho_out) - 0.5 * (rho_in - rho_out) * np.tanh(2.0 * (d - r) / w)


def droplet(shape, center_xyz, r, w, rho_in, rho_out) -> np.ndarray:
    x, y, z = grid(shape)
    cx, cy, cz = center_xyz
    d = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2)
    return tanh_profile(d, r, w, rho_in, rho_out)


def slab(shape, axis: str, lo: float, hi: float, w: float, rho_in, rho_out) -> np.ndarray:
    """rho_in on lo <= c < hi along the axis (periodic distance to the faces)."""
    x, y, z = grid(shape)
    c = {"x": x, "y": y, "z": z}[axis]
    L = {"x": shape[2], "y": shape[1], "z": shape[0]}[axis]
    mid, half = 0.5 * (lo + hi - 1), 0.5 * (hi - lo)
    dc = np.abs(c - mid)
    dc = np.minimum(dc, L - dc)
    return tanh_profile(dc, half, w, rho_in, rho_out)


def uniform_noise(shape, amp: float, seed: int) -> np.ndarray:
    """Additive U(-amp, amp) noise from numpy's PCG64 stream."""
    return np.random.default_rng(seed).uniform(-amp, amp, size=shape)


def walls(shape, axis: str, planes) -> np.ndarray:
    solid = np.zeros(shape, dtype=np.uint8)
    for p in planes:
        if axis == "z":
            solid[p, :, :] = 1
        elif axis == "y":
            solid[:, p, :] = 1
        else:
            solid[:, :, p] = 1
    return solid


def sphere_pack(shape, radii=(8.0, 16.0), porosity=0.35, seed=0, count=None) -> np.ndarray:
    """Periodic Boolean model of overlapping spheres (uint8 mask, 1 = solid)."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    a, b = radii
    er3 = (b ** 4 - a ** 4) / (4.0 * (b - a)) if b > a else a ** 3
    if count is None:
        count = int(round(-math.log(porosity) * nx * ny * nz / (4.0 / 3.0 * math.pi * er3)))
    centers = rng.uniform(0.0, 1.0, size=(count, 3)) * np.array([nx, ny, nz])
    rad = rng.uniform(a, b, size=count)
    solid = np.zeros(shape, dtype=np.uint8)
    for (cx, cy, cz), r in zip(centers, rad):
        ri = int(math.ceil(r)) + 1
        xs = np.arange(int(math.floor(cx)) - ri, int(math.floor(cx)) + ri + 2)
        ys = np.arange(int(math.floor(cy)) - ri, int(math.floor(cy)) + ri + 2)
        zs = np.arange(int(math.floor(cz)) - ri, int(math.floor(cz)) + ri + 2)
        dx2 = (xs - cx) ** 2
        dy2 = (ys - cy) ** 2
        dz2 = (zs - cz) ** 2
        inside = (dz2[:, None, None] + dy2[None, :, None] + dx2[None, None, :]) <= r * r
        iz, iy, ix = np.nonzero(inside)
        solid[zs[iz] % nz, ys[iy] % ny, xs[ix] % nx] = 1
    return solid


# --------------------------------------------------------------------------
# Named workloads.
# --------------------------------------------------------------------------
def _cs(tr: float):
    c = load_coexistence()
    key = f"{tr:.1f}"
    e = c["CS"][key]
    return c["CS"]["Tc"] * tr, e["rho_v"], e["rho_l"], e["A"]


def droplet_2d(n=128, steps=2000, storage="F64", r=20.0, w=5.0, tr=0.7, seed=0, noise=1e-4,
               collision="BGK"):
    """D2Q9 single-component Carnahan-Starling droplet in its vapour, periodic,
    BGK tau = 1 (the small double-precision case)."""
    T, rv, rl, A = _cs(tr)
    shape = (1, n, n)
    wl = Workload("droplet2d", "D2Q9", shape, storage=storage, collision=collision,
                  tau=(1.0, 1.0), eos_T=(T, T), A=(A, A), rho_min=(rv, rv), rho_max=(rl, rl),
                  steps=steps)
    rho = droplet(shape, (n / 2, n / 2, 0.0), r, w, rl, rv) + uniform_noise(shape, noise, seed)
    solid = np.zeros(shape, dtype=np.uint8)
    return wl, solid, rho[None]


def sessile_3d(n=256, steps=20000, storage="F32", r=30.0, w=5.0, tr=0.8, wet_mode="PHI",
               wet=1.0, collision="MRT", nxy=None, center=None, vapour=None):
    """D3Q19 Carnahan-Starling droplet resting on a solid wall at z = 0 (and a
    second wall at z = nz-1); x and y periodic.  MRT takes the d'Humieres
    rates at tau = 1 (with tau = 1 and every other rate 1 it would reduce to
    BGK).  The vapour starts at the Maxwell density unless `vapour` is given
    (the limiter bounds stay at the Maxwell pair)."""
    T, rv, rl, A = _cs(tr)
    rv_init = rv if vapour is None else vapour
    nx = ny = nxy or n
    shape = (n, ny, nx)
    dh = dhumieres_rates(1.0)
    wl = Workload("sessile3d", "D3Q19", shape, storage=storage, collision=collision,
                  tau=(1.0, 1.0), mrt_s=(dh, dh), eos_T=(T, T), A=(A, A), wet_mode=(wet_mode, wet_mode),
                  wet=(wet, wet), rho_min=(rv, rv), rho_max=(rl, rl), steps=steps)
    solid = walls(shape, "z", (0, n - 1))
    c = center or (nx / 2, ny / 2, r + 1.0)
    rho = droplet(shape, c, r, w, rl, rv_init)
    return wl, solid, rho[None]


def two_component_pack(n=400, steps=100, storage="F32", seed=0, porosity=0.35, radii=(8.0, 16.0),
                       rho_major=1.0, minor_frac=0.03, phi_w=1.2, drho_nw=0.1, shape=None,
                       solid=None):
    """D3Q19 two-component Shan-Chen (psi = rho) in a periodic sphere pack.
    Component 0 is non-wetting and fills pores with x < 0.4 nx; component 1 is
    wetting.  g_kk = -0.027, g_12 = 0.57, A = 0 (Sec. 3.3.2); body force 1e-6
    along x; each component is present at minor_frac of rho_major where the
    other dominates.  With G_i = w_i / c_s^2, rho_major = 1 makes 3 % the
    equilibrium solubility of these strengths (the fraction Sec. 3.3.2 uses);
    the wall densities are limited to [0, 1.1 rho_major]."""
    shape = shape or (n, n, n)
    nz, ny, nx = shape
    if solid is None:
        solid = sphere_pack(shape, radii, porosity, seed)
    minor = minor_frac * rho_major
    front = slab(shape, "x", 0, int(round(0.4 * nx)), 3.0, 1.0, 0.0)  # tanh edges, width 3
    rho = np.empty((2,) + tuple(shape))
    rho[0] = minor + (rho_major - minor) * front
    rho[1] = minor + (rho_major - minor) * (1.0 - front)
    g = ((-0.027, 0.57), (0.57, -0.027))
    wl = Workload("twocomp_pack", "D3Q19", tuple(shape), nc=2, storage=storage, collision="BGK",
                  tau=(1.0, 1.0), psi_kind=("DENSITY", "DENSITY"), A=(0.0, 0.0), g=g,
                  body=(1e-6, 0.0, 0.0), wet_mode=("DRHO", "PHI"), wet=(drho_nw, phi_w),
                  rho_min=(0.0, 0.0), rho_max=(1.1 * rho_major, 1.1 * rho_major), steps=steps)
    return wl, solid, rho


def pcsw_pack(n=256, buffer=8, steps=1000, storage="F32", seed=3, porosity=0.381, radii=(8.0, 16.0),
              rho_major=1.0, minor_frac=0.03, phi_w=1.2, drho_nw=0.1, dp_rho=0.0, shape=None,
              collision="BGK", outlet="reservoir", body=0.0):
    """Drainage for a capillary pressure - saturation curve (Sec. 3.4.3):
    D3Q19 two-component Shan-Chen (psi = rho; g_kk = -0.027, g_12 = 0.57,
    A = 0, both components of the same density) in a sphere pack of
    porosity 0.381 along z, with buffers of `buffer` fluid planes at both
    ends and a reservoir plane beyond each: reservoir 0 (z = 0, the inlet)
    holds the non-wetting bulk composition with its major density raised
    by dp_rho, reservoir 1 (the last plane, the outlet) the wetting bulk.
    Solid walls close the x and y faces (one solid layer at x = 0 and at
    y = 0, which the periodic wrap puts on both sides).  The pores and the
    outlet buffer start filled with the wetting component 1, the inlet
    buffer with the non-wetting component 0.  The measurement window is the
    pack's planes.  Wetting as in two_component_pack (wetting phi_w,
    non-wetting drho_nw).  outlet="convective" puts a convective outlet
    plane (mask 4) in place of reservoir 1, and body > 0 adds a body
    acceleration along +z: the body-force drainage of Sec. 3.4.2.  Returns
    (workload, mask with values 0-4, rho)."""
    if shape is None:
        shape = (n + 2 * buffer + 2, n, n)
    nz, ny, nx = shape
    z0, z1 = 1 + buffer, nz - 1 - buffer  # the pack's planes [z0, z1)
    pack = sphere_pack((z1 - z0, ny, nx), radii, porosity, seed)
    mask = np.zeros(shape, np.uint8)
    mask[z0:z1] = pack
    mask[:, :, 0] = 1
    mask[:, 0, :] = 1
    mask[0] = 2
    mask[nz - 1] = 4 if outlet == "convective" else 3
    minor = minor_frac * rho_major
    nw = np.zeros(shape, bool)
    nw[:z0] = True
    rho = np.empty((2,) + tuple(shape))
    rho[0] = np.where(nw, rho_major, minor)
    rho[1] = np.where(nw, minor, rho_major)
    g = ((-0.027, 0.57), (0.57, -0.027))
    wl = Workload("pcsw_pack", "D3Q19", tuple(shape), nc=2, storage=storage, collision=collision,
                  tau=(1.0, 1.0), psi_kind=("DENSITY", "DENSITY"), A=(0.0, 0.0), g=g,
                  wet_mode=("DRHO", "PHI"), wet=(drho_nw, phi_w), rho_min=(0.0, 0.0),
                  rho_max=(1.1 * rho_major, 1.1 * rho_major),
                  res_rho=((rho_major + dp_rho, minor), (minor, rho_major)), window=(z0, z1), steps=steps,
                  body=(0.0, 0.0, body))
    return wl, mask, rho


def adjoint_pack(n=128, steps=1000, storage="F32", seed=1, porosity=0.4, radii=(6.0, 14.0),
                 tr=0.8, phi=1.2, w=5.0, collision="MRT", shape=None, solid=None):
    """D3Q19 single-component CS at T_r = 0.8 in a periodic sphere pack; liquid
    slab x < nx/2, vapour elsewhere; uniform wetting phi; MRT with the
    d'Humieres rates at tau = 1, as the sessile droplet."""
    T, rv, rl, A = _cs(tr)
    shape = shape or (n, n, n)
    nz, ny, nx = shape
    if solid is None:
        solid = sphere_pack(shape, radii, porosity, seed)
    rho = slab(shape, "x", 0, nx // 2, w, rl, rv)
    dh = dhumieres_rates(1.0)
    wl = Workload("adjoint_pack", "D3Q19", tuple(shape), storage=storage, collision=collision,
                  tau=(1.0, 1.0), mrt_s=(dh, dh), eos_T=(T, T), A=(A, A), wet_mode=("PHI", "PHI"),
                  wet=(phi, phi), rho_min=(rv, rv), rho_max=(rl, rl), steps=steps)
    return wl, solid, rho[None]


def single_phase_pack(n=128, seed=0, porosity=0.4, radii=(6.0, 14.0), accel=1e-5, storage="F32",
                      steps=100, shape=None, solid=None):
    """Single-phase flow (no interaction force) through a periodic sphere pack,
    BGK tau = 1, rho = 1, driven by a body acceleration along x."""
    shape = shape or (n, n, n)
    if solid is None:
        solid = sphere_pack(shape, radii, porosity, seed)
    wl = Workload("single_phase_pack", "D3Q19", tuple(shape), storage=storage, collision="BGK",
                  tau=(1.0, 1.0), psi_kind=("DENSITY", "DENSITY"), g=((0.0, 0.0), (0.0, 0.0)),
                  A=(0.0, 0.0), body=(accel, 0.0, 0.0), rho_min=(0.0, 0.0), rho_max=(1e30, 1e30),
                  steps=steps)
    rho = np.ones((1,) + tuple(shape))
    return wl, solid, rho
