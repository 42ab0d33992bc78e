"""Python binding of liblbm.so (include/lbm.h): argument marshalling only.

Every step of the method runs in the HIP kernels of the library; torch only
provides device memory (the caller-owned workspace and output buffers) and the
stream the work is enqueued on.  Loading fails loudly if the library has not
been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
LIB_PATH = HERE / "_lib" / "liblbm.so"

LBM_OK = 0
ERRORS = {-1: "LBM_ERR_ARG", -2: "LBM_ERR_UNSUPPORTED", -3: "LBM_ERR_HIP", -4: "LBM_ERR_NONFINITE",
          -5: "LBM_ERR_SPACE", -6: "LBM_ERR_OOM"}
STORAGE = {"F64": 0, "F32": 1, "F16DEV": 2, "BF16DEV": 3, "F32F64": 4}
LAYOUT = {"DENSE": 0, "FLUID": 1}  # lbm_params.layout
EXPORTS = ["lbm_workspace_size", "lbm_init", "lbm_step", "lbm_moments", "lbm_stats", "lbm_sync",
           "lbm_set_reservoir", "lbm_state_bytes", "lbm_get_state", "lbm_set_state", "lbm_reset", "lbm_grad_workspace_size", "lbm_grad",
           "lbm_free", "lbm_strerror"]
OBSERVABLES = {"saturation": 0, "drho": 1}


class LbmError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn} failed: {ERRORS.get(code, code)} ({code})")
        self.code = code


class LbmParams(C.Structure):
    _fields_ = [
        ("lattice", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("n_comp", C.c_int32), ("collision", C.c_int32), ("storage", C.c_int32),
        ("psi_kind", C.c_int32 * 2), ("wet_mode", C.c_int32 * 2),
        ("common_velocity", C.c_int32), ("check_every", C.c_int32), ("reserved", C.c_int32 * 4),
        ("tau", C.c_double * 2), ("mrt_s", (C.c_double * 19) * 2),
        ("eos_a", C.c_double * 2), ("eos_b", C.c_double * 2), ("eos_R", C.c_double * 2),
        ("eos_T", C.c_double * 2), ("alpha", C.c_double * 2), ("A", C.c_double * 2),
        ("g", (C.c_double * 2) * 2), ("body_accel", C.c_double * 3), ("wet", C.c_double * 2),
        ("rho_min", C.c_double * 2), ("rho_max", C.c_double * 2), ("kappa", C.c_double * 2),
        ("res_rho", (C.c_double * 2) * 2), ("window", C.c_int32 * 2), ("layout", C.c_int32), ("reserved2", C.c_int32),
    ]


class LbmStats(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("mass", C.c_double * 2), ("momentum", C.c_double * 3),
        ("residual", C.c_double), ("saturation", C.c_double), ("mean_ux", C.c_double),
        ("n_fluid", C.c_int64), ("nonfinite", C.c_int32), ("negative", C.c_int32),
        ("p_nonwetting", C.c_double), ("p_wetting", C.c_double), ("capillary_pressure", C.c_double),
        ("s_wetting", C.c_double),
    ]

    def as_dict(self) -> dict:
        return {"step": self.step, "mass": list(self.mass), "momentum": list(self.momentum),
                "residual": self.residual, "saturation": self.saturation, "mean_ux": self.mean_ux,
                "n_fluid": self.n_fluid, "nonfinite": self.nonfinite, "negative": self.negative,
                "p_nonwetting": self.p_nonwetting, "p_wetting": self.p_wetting,
                "capillary_pressure": self.capillary_pressure, "s_wetting": self.s_wetting}


class LbmGradReq(C.Structure):
    _fields_ = [
        ("observable", C.c_int32), ("nsteps", C.c_int32), ("ckpt_every", C.c_int32),
        ("reserved", C.c_int32), ("rho_mid", C.c_double), ("delta", C.c_double),
        ("dL_drho", C.c_void_p), ("ws", C.c_void_p), ("ws_bytes", C.c_size_t),
    ]


_lib = None


def load():
    """Load the library (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        lib = C.CDLL(str(LIB_PATH))
        vp, sz = C.c_void_p, C.c_size_t
        lib.lbm_workspace_size.argtypes = [vp, C.POINTER(sz)]
        lib.lbm_init.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp, C.POINTER(vp)]
        lib.lbm_step.argtypes = [vp, C.c_int64]
        lib.lbm_moments.argtypes = [vp, C.c_int, vp, vp]
        lib.lbm_stats.argtypes = [vp, vp]
        lib.lbm_sync.argtypes = [vp]
        lib.lbm_set_reservoir.argtypes = [vp, C.c_int, vp]
        lib.lbm_state_bytes.argtypes = [vp, C.POINTER(sz)]
        lib.lbm_get_state.argtypes = [vp, vp]
        lib.lbm_set_state.argtypes = [vp, vp]
        lib.lbm_reset.argtypes = [vp, vp, vp]
        lib.lbm_grad_workspace_size.argtypes = [vp, vp, C.POINTER(sz)]
        lib.lbm_grad.argtypes = [vp, vp, C.POINTER(C.c_double), vp, C.POINTER(C.c_double)]
        lib.lbm_free.argtypes = [vp]
        lib.lbm_free.restype = None
        lib.lbm_strerror.argtypes = [C.c_int]
        lib.lbm_strerror.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("lbm_free", "lbm_strerror"):
                getattr(lib, name).restype = C.c_int
        _lib = lib
    return _lib


def _check(fn: str, rc: int) -> None:
    if rc != LBM_OK:
        raise LbmError(fn, rc)


def params_from(w, check_every: int = 0) -> LbmParams:
    """lbm_params of a Workload (paper_2506_17713_amd.inputs.Workload)."""
    p = LbmParams()
    p.lattice = 0 if w.lattice == "D2Q9" else 1
    p.nx, p.ny, p.nz = w.shape_xyz
    p.n_comp = w.nc
    p.collision = {"BGK": 0, "MRT": 1, "CLBM": 2}[w.collision]
    p.storage = STORAGE[w.storage]
    p.common_velocity = 1 if w.common_velocity else 0
    p.check_every = check_every
    for k in range(w.nc):
        p.psi_kind[k] = 0 if w.psi_kind[k] == "CS" else 1
        p.wet_mode[k] = 0 if w.wet_mode[k] == "PHI" else 1
        p.tau[k] = w.tau[k]
        for m, s in enumerate(w.mrt_rates(k)):
            p.mrt_s[k][m] = s
        p.eos_a[k], p.eos_b[k], p.eos_R[k] = w.eos_a[k], w.eos_b[k], w.eos_R[k]
        p.eos_T[k] = w.eos_T[k]
        p.alpha[k] = w.alpha[k]
        p.A[k] = w.A[k]
        for kk in range(w.nc):
            p.g[k][kk] = w.g[k][kk]
        p.wet[k] = w.wet[k]
        p.rho_min[k], p.rho_max[k] = w.rho_min[k], min(w.rho_max[k], 1e300)
        p.kappa[k] = w.kappa[k]
        for r in range(2):
            p.res_rho[r][k] = w.res_rho[r][k]
    for d in range(3):
        p.body_accel[d] = w.body[d]
    p.window[0], p.window[1] = w.window
    p.layout = LAYOUT[w.layout]
    return p


def _host(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


class Solver:
    """One lattice on one GPU stream (wraps an lbm_handle)."""

    def __init__(self, w, solid, rho0, u0=None, wet=None, device="cuda", check_every: int = 0):
        import torch

        self.torch = torch
        self.lib = load()
        self.w = w
        self.device = torch.device(device)
        self.p = params_from(w, check_every)
        N = w.N
        mask = _host(np.asarray(solid).reshape(-1), np.uint8)
        rho = _host(np.asarray(rho0).reshape(w.nc, N), np.float64)
        uu = None if u0 is None else _host(np.asarray(u0).reshape(3, N), np.float64)
        ww = None if wet is None else _host(np.asarray(wet).reshape(w.nc, N), np.float64)
        size = C.c_size_t()
        _check("lbm_workspace_size", self.lib.lbm_workspace_size(C.byref(self.p), C.byref(size)))
        self.ws = torch.empty(size.value, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = self.lib.lbm_init(C.byref(self.p), mask.ctypes.data, rho.ctypes.data,
                               None if uu is None else uu.ctypes.data,
                               None if ww is None else ww.ctypes.data,
                               self.ws.data_ptr(), size.value, self.stream.cuda_stream, C.byref(h))
        _check("lbm_init", rc)
        self.h = h
        self.real = torch.float64 if w.storage in ("F64", "F32F64") else torch.float32

    # -- stepping and observation -------------------------------------------
    def step(self, n: int = 1) -> None:
        _check("lbm_step", self.lib.lbm_step(self.h, int(n)))

    def moments(self, comp: int = -1, rho=True, u=True):
        t = self.torch
        N = self.w.N
        r = t.empty(N, dtype=self.real, device=self.device) if rho else None
        v = t.empty((3, N), dtype=self.real, device=self.device) if u else None
        _check("lbm_moments", self.lib.lbm_moments(self.h, comp, None if r is None else r.data_ptr(),
                                                   None if v is None else v.data_ptr()))
        return r, v

    def moments_numpy(self, comp: int = -1):
        r, v = self.moments(comp)
        self.torch.cuda.synchronize(self.device)
        return r.double().cpu().numpy(), v.double().cpu().numpy()

    def stats(self) -> dict:
        s = LbmStats()
        rc = self.lib.lbm_stats(self.h, C.byref(s))
        out = s.as_dict()
        out["rc"] = rc
        if rc not in (LBM_OK, -4):
            _check("lbm_stats", rc)
        return out

    def sync(self) -> int:
        return self.lib.lbm_sync(self.h)

    def set_reservoir(self, r: int, rho) -> None:
        """New fixed densities (one per component) of reservoir r, from the next step on."""
        buf = _host(list(rho)[: self.w.nc], np.float64)
        _check("lbm_set_reservoir", self.lib.lbm_set_reservoir(self.h, int(r), buf.ctypes.data_as(C.c_void_p)))

    def state_bytes(self) -> int:
        b = C.c_size_t()
        _check("lbm_state_bytes", self.lib.lbm_state_bytes(self.h, C.byref(b)))
        return b.value

    def get_state(self):
        buf = self.torch.empty(self.state_bytes(), dtype=self.torch.uint8, device=self.device)
        _check("lbm_get_state", self.lib.lbm_get_state(self.h, buf.data_ptr()))
        return buf

    def set_state(self, buf) -> None:
        assert buf.numel() == self.state_bytes()
        _check("lbm_set_state", self.lib.lbm_set_state(self.h, buf.data_ptr()))

    def reset(self, rho0, u0=None) -> None:
        """Restart from f^eq of device fields (lbm_reset): rho0 [n_comp, N] and
        u0 [3, N] (None: rest), contiguous device tensors of the compute type."""
        N = self.w.N
        assert rho0.dtype == self.real and rho0.is_cuda and rho0.is_contiguous() and rho0.numel() == self.w.nc * N
        if u0 is not None:
            assert u0.dtype == self.real and u0.is_cuda and u0.is_contiguous() and u0.numel() == 3 * N
        _check("lbm_reset", self.lib.lbm_reset(self.h, rho0.data_ptr(), None if u0 is None else u0.data_ptr()))

    def grad(self, nsteps: int, ckpt_every: int, observable: str = "saturation", rho_mid: float = 0.0,
             delta: float = 1.0, dL_drho=None):
        """Run nsteps from the current state and back-propagate (lbm_grad).
        Returns (L, dL/dwet as a device float64 tensor [N], dL/dT)."""
        t = self.torch
        r = LbmGradReq()
        r.observable = OBSERVABLES[observable]
        r.nsteps, r.ckpt_every = int(nsteps), int(ckpt_every)
        r.rho_mid, r.delta = float(rho_mid), float(delta)
        if dL_drho is not None:
            assert dL_drho.dtype == self.real and dL_drho.is_contiguous()
            r.dL_drho = dL_drho.data_ptr()
        size = C.c_size_t()
        _check("lbm_grad_workspace_size", self.lib.lbm_grad_workspace_size(self.h, C.byref(r), C.byref(size)))
        ws = t.empty(size.value, dtype=t.uint8, device=self.device)
        r.ws, r.ws_bytes = ws.data_ptr(), size.value
        dwet = t.empty(self.w.N, dtype=t.float64, device=self.device)
        L, dT = C.c_double(), C.c_double()
        _check("lbm_grad", self.lib.lbm_grad(self.h, C.byref(r), C.byref(L), dwet.data_ptr(), C.byref(dT)))
        del ws
        return L.value, dwet, dT.value

    def close(self) -> None:
        if getattr(self, "h", None):
            self.lib.lbm_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
