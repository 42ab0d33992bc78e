"""Python access to the FP64 CPU oracle (lbm_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  Nothing here is shared
with the GPU path: the oracle library is compiled from its own C source with
gcc (-O2, no fast-math, no FMA contraction) and driven through ctypes.

Two builds of the same source:
  liblbmref.so        real_t = double               (oref_* symbols)
  liblbmref_cstep.so  real_t = double _Complex      (orefc_* symbols),
                      complex-step derivatives of the step.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
BUILD = HERE / "_build"
SRC = HERE / "lbm_oracle.c"
LIB = BUILD / "liblbmref.so"
LIB_CSTEP = BUILD / "liblbmref_cstep.so"

MAXQ, MAXC = 19, 2


def build(force: bool = True) -> None:
    """Compile both oracle libraries with gcc."""
    BUILD.mkdir(exist_ok=True)
    flags = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
             "-std=c11", "-Wall"]
    for out, extra in ((LIB, []), (LIB_CSTEP, ["-DORACLE_CSTEP"])):
        if force or not out.exists() or out.stat().st_mtime < SRC.stat().st_mtime:
            tmp = out.with_suffix(".so.tmp")
            subprocess.check_call(["gcc", *flags, *extra, str(SRC), "-o", str(tmp), "-lm"])
            os.replace(tmp, out)


class OrefParams(C.Structure):
    _fields_ = [
        ("lattice", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("nc", C.c_int), ("collision", C.c_int),
        ("psi_kind", C.c_int * MAXC), ("wet_mode", C.c_int * MAXC),
        ("common_velocity", C.c_int),
        ("tau", C.c_double * MAXC),
        ("mrt_s", (C.c_double * MAXQ) * MAXC),
        ("eos_a", C.c_double * MAXC), ("eos_b", C.c_double * MAXC), ("eos_R", C.c_double * MAXC),
        ("eos_T", C.c_double * MAXC), ("eos_T_im", C.c_double * MAXC),
        ("alpha", C.c_double * MAXC),
        ("A", C.c_double * MAXC),
        ("g", (C.c_double * MAXC) * MAXC),
        ("body", C.c_double * 3),
        ("rho_min", C.c_double * MAXC), ("rho_max", C.c_double * MAXC),
        ("kappa", C.c_double * MAXC),
        ("res_rho", (C.c_double * MAXC) * 2),
    ]


_libs: dict = {}


def _lib(cstep: bool = False):
    key = "c" if cstep else "r"
    if key not in _libs:
        path = LIB_CSTEP if cstep else LIB
        if not path.exists() or path.stat().st_mtime < SRC.stat().st_mtime:
            build(force=False)
        _libs[key] = C.CDLL(str(path))
    return _libs[key]


def params_from(w, T_im: float | tuple = 0.0) -> OrefParams:
    """Marshal a Workload (paper_2506_17713_amd.inputs.Workload) into the C struct."""
    p = OrefParams()
    p.lattice = 0 if w.lattice == "D2Q9" else 1
    nx, ny, nz = w.shape_xyz
    p.nx, p.ny, p.nz = nx, ny, nz
    p.nc = w.nc
    p.collision = {"BGK": 0, "MRT": 1, "CLBM": 2}[w.collision]
    p.common_velocity = 1 if w.common_velocity else 0
    tim = T_im if isinstance(T_im, (tuple, list)) else (T_im, T_im)
    for k in range(w.nc):
        p.psi_kind[k] = 0 if w.psi_kind[k] == "CS" else 1
        p.wet_mode[k] = 0 if w.wet_mode[k] == "PHI" else 1
        p.tau[k] = w.tau[k]
        rates = w.mrt_rates(k)
        for a in range(len(rates)):
            p.mrt_s[k][a] = rates[a]
        p.eos_a[k], p.eos_b[k], p.eos_R[k] = w.eos_a[k], w.eos_b[k], w.eos_R[k]
        p.eos_T[k] = w.eos_T[k]
        p.eos_T_im[k] = tim[k]
        p.alpha[k] = w.alpha[k]
        p.A[k] = w.A[k]
        for kk in range(w.nc):
            p.g[k][kk] = w.g[k][kk]
        p.rho_min[k], p.rho_max[k] = w.rho_min[k], w.rho_max[k]
        p.kappa[k] = w.kappa[k]
        for r in range(2):
            p.res_rho[r][k] = w.res_rho[r][k]
    for d in range(3):
        p.body[d] = w.body[d]
    return p


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def lattice(lat: str):
    """(e[q,3], w[q], opp[q]) built by the oracle from the velocity-set definition."""
    e = np.zeros((MAXQ, 3), dtype=np.int32)
    w = np.zeros(MAXQ)
    opp = np.zeros(MAXQ, dtype=np.int32)
    q = C.c_int()
    _lib().oref_lattice(0 if lat == "D2Q9" else 1, C.byref(q), _ptr(e), _ptr(w), _ptr(opp))
    n = q.value
    return e[:n].copy(), w[:n].copy(), opp[:n].copy()


def mrt_matrix(lat: str):
    q = 9 if lat == "D2Q9" else 19
    M = np.zeros((q, q))
    Mi = np.zeros((q, q))
    rc = _lib().oref_mrt_matrix(0 if lat == "D2Q9" else 1, _ptr(M), _ptr(Mi))
    assert rc == 0
    return M, Mi


def feq(lat: str, rho: float, u) -> np.ndarray:
    q = 9 if lat == "D2Q9" else 19
    out = np.zeros(q)
    uu = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(3))
    lib = _lib()
    lib.oref_feq.argtypes = [C.c_int, C.c_double, C.c_void_p, C.c_void_p]
    lib.oref_feq(0 if lat == "D2Q9" else 1, rho, _ptr(uu), _ptr(out))
    return out


def psi(w, k: int, rho: float):
    p = params_from(w)
    ps, U = C.c_double(), C.c_double()
    lib = _lib()
    lib.oref_psi.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_void_p, C.c_void_p]
    lib.oref_psi(C.byref(p), k, rho, C.byref(ps), C.byref(U))
    return ps.value, U.value


def collide_node(w, k: int, fin, u, F) -> np.ndarray:
    p = params_from(w)
    fin = np.ascontiguousarray(fin, dtype=np.float64)
    out = np.zeros_like(fin)
    uu = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(3))
    FF = np.ascontiguousarray(np.asarray(F, dtype=np.float64).reshape(3))
    _lib().oref_collide_node(C.byref(p), C.c_int(k), _ptr(fin), _ptr(uu), _ptr(FF), _ptr(out))
    return out


def set_threads(n: int) -> None:
    """Threads of the oracle's node loops (its results do not depend on it)."""
    _lib(False).oref_set_threads(C.c_int(n))
    _lib(True).orefc_set_threads(C.c_int(n))


class State:
    """Oracle state of one run: populations f[nc, q, N] (post-streaming)."""

    def __init__(self, w, solid: np.ndarray, rho0: np.ndarray, u0: np.ndarray | None = None,
                 wet: np.ndarray | None = None, cstep: bool = False, T_im=0.0):
        self.w = w
        self.cstep = cstep
        self.dtype = np.complex128 if cstep else np.float64
        self.p = params_from(w, T_im)
        self.N = int(np.prod(w.shape_xyz))
        self.q = 9 if w.lattice == "D2Q9" else 19
        self.solid = np.ascontiguousarray(solid.reshape(-1).astype(np.uint8))
        if wet is None:
            wet = np.empty((w.nc, self.N))
            for k in range(w.nc):
                wet[k] = w.wet[k]
        self.wet = np.ascontiguousarray(np.asarray(wet).reshape(w.nc, self.N).astype(self.dtype))
        r0 = np.ascontiguousarray(np.asarray(rho0).reshape(w.nc, self.N).astype(self.dtype))
        u = None if u0 is None else np.ascontiguousarray(np.asarray(u0).reshape(3, self.N).astype(self.dtype))
        self.f = np.zeros((w.nc, self.q, self.N), dtype=self.dtype)
        lib = _lib(cstep)
        fn = lib.orefc_init_feq if cstep else lib.oref_init_feq
        rc = fn(C.byref(self.p), _ptr(self.solid), _ptr(r0), None if u is None else _ptr(u), _ptr(self.f))
        assert rc == 0

    def step(self, n: int = 1) -> None:
        lib = _lib(self.cstep)
        fn = lib.orefc_step if self.cstep else lib.oref_step
        rc = fn(C.byref(self.p), _ptr(self.solid), _ptr(self.wet), _ptr(self.f), C.c_int(n))
        if rc != 0:
            raise RuntimeError(f"oracle step failed rc={rc}")

    def fields(self) -> dict:
        nc, N = self.w.nc, self.N
        out = {
            "rho": np.zeros((nc, N), self.dtype), "F": np.zeros((nc, 3, N), self.dtype),
            "u": np.zeros((nc, 3, N), self.dtype), "umix": np.zeros((3, N), self.dtype),
            "psi": np.zeros((nc, N), self.dtype), "U": np.zeros((nc, N), self.dtype),
        }
        lib = _lib(self.cstep)
        fn = lib.orefc_fields if self.cstep else lib.oref_fields
        rc = fn(C.byref(self.p), _ptr(self.solid), _ptr(self.wet), _ptr(self.f),
                _ptr(out["rho"]), _ptr(out["F"]), _ptr(out["u"]), _ptr(out["umix"]),
                _ptr(out["psi"]), _ptr(out["U"]))
        assert rc == 0
        return out

    def stream_only(self, fpost: np.ndarray) -> np.ndarray:
        fpost = np.ascontiguousarray(fpost.astype(self.dtype))
        out = np.zeros_like(fpost)
        lib = _lib(self.cstep)
        fn = lib.orefc_stream_only if self.cstep else lib.oref_stream_only
        fn(C.byref(self.p), _ptr(self.solid), _ptr(fpost), _ptr(out))
        return out

    def set_reservoir(self, r: int, rho) -> None:
        """New fixed densities (one per component) of reservoir r from the next step on."""
        self.w = self.w.with_(res_rho=tuple(tuple(rho) if i == r else self.w.res_rho[i] for i in range(2)))
        for k in range(self.w.nc):
            self.p.res_rho[r][k] = float(rho[k])

    def mass(self) -> np.ndarray:
        return self.f.sum(axis=(1, 2))


# --------------------------------------------------------------------------
# In-situ capillary pressure and saturation (Sec. 3.4.3).
# --------------------------------------------------------------------------
def pressure(w, fld: dict) -> np.ndarray:
    """Bulk pressure of the Shan-Chen fluid at every node,
    p = c_s^2 sum_k rho^k + (1/2) sum_kk' g_kk' psi^k psi^k' (the pressure of
    the interaction force of Eq. 13; with one component and the EOS
    pseudopotential of Eq. 12 it equals alpha p_EOS(rho))."""
    rho, psi = fld["rho"], fld["psi"]
    p = rho.sum(axis=0) / 3.0
    for k in range(w.nc):
        for kk in range(w.nc):
            p = p + 0.5 * w.g[k][kk] * psi[k] * psi[kk]
    return p


def capillary(w, solid: np.ndarray, fld: dict, window=None) -> dict:
    """Capillary pressure and wetting saturation measured in place
    (Sec. 3.4.3): over the fluid nodes of the planes window[0] <= c <
    window[1] of the slowest lattice axis (z in 3-D, y in 2-D; all planes
    when window is None), a node is non-wetting where rho^0 >= rho^1 (two
    components; component 0 is the non-wetting fluid) or, for one
    component, where rho lies below (rho_min + rho_max)/2 (vapour).
    P_c = mean pressure of the non-wetting nodes - mean pressure of the
    wetting nodes; S_w = wetting nodes / fluid nodes."""
    nz, ny, nx = w.shape
    plane = nx * ny if w.lattice == "D3Q19" else nx
    n = np.arange(w.N)
    c = n // plane
    sel = solid.reshape(-1) == 0
    if window is not None and window[1] > window[0]:
        sel &= (c >= window[0]) & (c < window[1])
    rho = fld["rho"]
    if w.nc > 1:
        nw = rho[0] >= rho[1]
    else:
        nw = rho[0] < 0.5 * (w.rho_min[0] + w.rho_max[0])
    p = pressure(w, fld)
    a, b = sel & nw, sel & ~nw
    n_nw, n_w = int(a.sum()), int(b.sum())
    p_nw = float(p[a].mean()) if n_nw else 0.0
    p_w = float(p[b].mean()) if n_w else 0.0
    return {"p_nw": p_nw, "p_w": p_w, "p_c": p_nw - p_w, "s_w": n_w / max(n_nw + n_w, 1),
            "n_nw": n_nw, "n_w": n_w}
