"""The C-ABI library loads and exports every function include/lbm.h declares;
the Python structs match the C layout; host-side validation returns the
documented error codes.  No GPU compute is called here."""
import ctypes as C
import re
import subprocess
from pathlib import Path

import numpy as np
import pytest

from paper_2506_17713_amd import inputs, lbm

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "lbm.h"
HEADERS = [ROOT / "include" / "lbm.h", ROOT / "include" / "lbm_nn.h"]


@pytest.fixture(scope="module")
def lib():
    if not lbm.LIB_PATH.exists():
        from paper_2506_17713_amd import build
        build.build()
    return lbm.load()


def declared_functions(headers=None):
    names = set()
    for hd in headers or HEADERS:
        text = re.sub(r"/\*.*?\*/", "", hd.read_text(), flags=re.S)
        names |= set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("lbm_init", "lbm_step", "lbm_moments", "lbm_workspace_size", "lbm_stats", "lbm_free"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", str(lbm.LIB_PATH)], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (lbm_[a-z_]+)\b", out))
    for n in declared_functions():
        assert n in exported, n
        assert hasattr(lib, n)
    from paper_2506_17713_amd import nn
    assert set(lbm.EXPORTS) == set(declared_functions([HEADER]))
    assert set(nn.EXPORTS) == set(declared_functions([HEADERS[1]]))


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    fields = [f[0] for f in lbm.LbmParams._fields_]
    sfields = [f[0] for f in lbm.LbmStats._fields_]
    body = "\n".join(f'printf("%zu ", offsetof(lbm_params, {f}));' for f in fields)
    sbody = "\n".join(f'printf("%zu ", offsetof(lbm_stats_t, {f}));' for f in sfields)
    src.write_text(f"""#include <stdio.h>
#include <stddef.h>
#include "lbm.h"
int main(void) {{ {body} printf("%zu\\n", sizeof(lbm_params));
{sbody} printf("%zu\\n", sizeof(lbm_stats_t)); return 0; }}""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", f"-I{ROOT / 'include'}", str(src), "-o", str(exe)], check=True)
    l1, l2 = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines()
    got = [int(v) for v in l1.split()]
    exp = [getattr(lbm.LbmParams, f).offset for f in fields] + [C.sizeof(lbm.LbmParams)]
    assert got == exp
    got = [int(v) for v in l2.split()]
    exp = [getattr(lbm.LbmStats, f).offset for f in sfields] + [C.sizeof(lbm.LbmStats)]
    assert got == exp


def _params(**kw):
    w, _, _ = inputs.sessile_3d(n=16, r=4, w=3)
    w = w.with_(**kw) if kw else w
    return lbm.params_from(w)


def test_workspace_size_and_validation(lib):
    sz = C.c_size_t()
    p = _params()
    assert lib.lbm_workspace_size(C.byref(p), C.byref(sz)) == 0
    N = 16 ** 3
    assert sz.value >= 2 * 19 * N * 4 + N * 4
    # F64 needs twice the population bytes of F32
    p64 = _params(storage="F64")
    sz64 = C.c_size_t()
    assert lib.lbm_workspace_size(C.byref(p64), C.byref(sz64)) == 0
    assert sz64.value > sz.value
    # invalid parameter sets
    bad = []
    p = _params(); p.n_comp = 3; bad.append(p)
    p = _params(); p.lattice = 7; bad.append(p)
    p = _params(); p.tau[0] = 0.5; bad.append(p)
    p = _params(); p.g[0][0] = 0.5; bad.append(p)          # EOS psi needs g_kk < 0
    p = _params(); p.reserved[1] = 3; bad.append(p)
    p = _params(lattice="D2Q9"); bad.append(p)               # nz != 1 for D2Q9
    p = _params(); p.eos_T[0] = 1.0; bad.append(p)           # psi argument > 0 inside the bounds
    p = _params(collision="MRT"); p.mrt_s[0][9] = 2.5; bad.append(p)
    p = _params(); p.nx, p.ny, p.nz = 1 << 15, 1 << 14, 1; bad.append(p)  # plane of 2^29 nodes
    for p in bad:
        assert lib.lbm_workspace_size(C.byref(p), C.byref(sz)) == -1
    # valid but not provided: central moments beyond one D2Q9 component, the
    # surface-tension source outside D2Q9 MRT
    unsup = []
    p = _params(collision="CLBM"); unsup.append(p)            # D3Q19
    p = _params(); p.kappa[0] = 0.5; unsup.append(p)           # D3Q19
    for p in unsup:
        assert lib.lbm_workspace_size(C.byref(p), C.byref(sz)) == -2


def test_init_rejects_bad_host_fields_before_touching_the_gpu(lib):
    w, solid, rho = inputs.sessile_3d(n=16, r=4, w=3)
    p = lbm.params_from(w)
    sz = C.c_size_t()
    assert lib.lbm_workspace_size(C.byref(p), C.byref(sz)) == 0
    h = C.c_void_p()
    mask = np.ascontiguousarray(solid.reshape(-1).astype(np.uint8))
    fake_ws = C.c_void_p(1 << 20)  # never dereferenced: validation fails first
    for bad_val in (np.nan, -0.1, 0.0):
        r = np.ascontiguousarray(rho.reshape(1, -1).copy())
        r[0, 16 * 16 * 5 + 7] = bad_val
        rc = lib.lbm_init(C.byref(p), mask.ctypes.data, r.ctypes.data, None, None, fake_ws, sz.value,
                          None, C.byref(h))
        assert rc == -1
    r = np.ascontiguousarray(rho.reshape(1, -1))
    rc = lib.lbm_init(C.byref(p), mask.ctypes.data, r.ctypes.data, None, None, fake_ws, sz.value - 256,
                      None, C.byref(h))
    assert rc == -5  # workspace too small


def test_strerror(lib):
    assert lib.lbm_strerror(0) == b"ok"
    assert b"workspace" in lib.lbm_strerror(-5)
    assert b"memory" in lib.lbm_strerror(-6)
    assert lib.lbm_strerror(-99) == b"unknown error"


def test_warm_start_driver_evaluates_a_loaded_model_without_training_it():
    from paper_2506_17713_amd import warmstart
    assert warmstart.parse_args([]).train == 256
    assert warmstart.parse_args(["--load-model", "m.npz"]).train == 0
    assert warmstart.parse_args(["--load-model", "m.npz", "--train", "64"]).train == 64


def test_surrogate_flop_count_matches_the_layer_shapes():
    """bench.py's FLOP count of the surrogate: 2 per multiply-add of every
    3x3x3 convolution at its level's size; a training step adds the weight
    gradient of every layer and the data gradient of all but the first."""
    import importlib.util

    from paper_2506_17713_amd.surrogate import ARCH

    spec = importlib.util.spec_from_file_location("bench", ROOT / "bench.py")
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    sizes = {"enc0a": 16, "enc0b": 16, "enc1a": 8, "enc1b": 8, "enc2a": 4, "enc2b": 4, "bota": 2, "botb": 2,
             "dec2a": 4, "dec2b": 4, "dec1a": 8, "dec1b": 8, "dec0a": 16, "dec0b": 16, "head": 16}
    fwd = sum(2 * ci * co * 27 * sizes[n] ** 3 for n, ci, co in ARCH)
    first = 2 * ARCH[0][1] * ARCH[0][2] * 27 * 16 ** 3
    f = bench.conv_flops(ARCH, 16)
    assert f["forward"] == fwd
    assert f["backward"] == 2 * fwd - first


def test_init_rejects_bad_reservoir_masks(lib):
    # reservoirs fill whole planes of the marching axis, one per plane, with
    # positive densities; no fluid plane lies between two reservoir planes
    w, mask, rho = inputs.pcsw_pack(n=12, buffer=2, shape=(18, 12, 12))
    sz = C.c_size_t()
    h = C.c_void_p()
    fake_ws = C.c_void_p(1 << 20)  # never dereferenced: validation fails first
    r = np.ascontiguousarray(rho.reshape(2, -1))

    def init(p, m):
        m = np.ascontiguousarray(m.reshape(-1).astype(np.uint8))
        assert lib.lbm_workspace_size(C.byref(p), C.byref(sz)) == 0
        return lib.lbm_init(C.byref(p), m.ctypes.data, r.ctypes.data, None, None, fake_ws, sz.value, None,
                            C.byref(h))

    p = lbm.params_from(w)
    bad = []
    m = mask.copy(); m[0, 3, 4] = 0; bad.append((p, m))            # a hole in the reservoir plane
    m = mask.copy(); m[0, 3, 4] = 3; bad.append((p, m))            # two reservoirs in one plane
    m = mask.copy(); m[5, 5, 5] = 4; bad.append((p, m))            # unknown node kind
    m = mask.copy(); m[2] = 3; bad.append((p, m))                  # plane 1 between two reservoirs
    q = lbm.params_from(w.with_(res_rho=((1.0, 0.0), (0.03, 1.0)))); bad.append((q, mask))  # rho_res = 0
    for p_, m in bad:
        assert init(p_, m) == -1
    p = lbm.params_from(w)
    p.reserved2 = 1
    assert lib.lbm_workspace_size(C.byref(p), C.byref(sz)) == -1
    assert lib.lbm_set_reservoir(None, 0, None) == -1


def test_init_rejects_bad_convective_outlets(lib):
    # one outlet plane, the last of the marching axis, with fluid below it
    # and none above across the wrap; not with 16-bit storage
    w, mask, rho = inputs.pcsw_pack(n=12, buffer=2, shape=(18, 12, 12), outlet="convective")
    sz = C.c_size_t()
    h = C.c_void_p()
    fake_ws = C.c_void_p(1 << 20)  # never dereferenced: validation fails first
    r = np.ascontiguousarray(rho.reshape(2, -1))

    def init(p, m):
        m = np.ascontiguousarray(m.reshape(-1).astype(np.uint8))
        assert lib.lbm_workspace_size(C.byref(p), C.byref(sz)) == 0
        return lib.lbm_init(C.byref(p), m.ctypes.data, r.ctypes.data, None, None, fake_ws, sz.value, None,
                            C.byref(h))

    p = lbm.params_from(w)
    m = mask.copy(); m[0] = 4                       # two outlet planes
    assert init(p, m) == -1
    m = np.roll(mask, -1, axis=0)                   # outlet not the last plane
    assert init(p, m) == -1
    m = mask.copy(); m[0] = 0                       # fluid above the outlet across the wrap
    assert init(p, m) == -1
    assert init(lbm.params_from(w.with_(storage="F16DEV")), mask) == -2


def test_fluid_layout_validation(lib):
    # LBM_LAYOUT_FLUID: D3Q19, BGK or MRT; the workspace adds the neighbour
    # table
    sz, szd = C.c_size_t(), C.c_size_t()
    assert lib.lbm_workspace_size(C.byref(_params(layout="FLUID")), C.byref(sz)) == 0
    assert lib.lbm_workspace_size(C.byref(_params()), C.byref(szd)) == 0
    assert sz.value >= szd.value + 18 * 16 ** 3 * 4
    for kw in (dict(storage="F16DEV"), dict(storage="BF16DEV")):
        assert lib.lbm_workspace_size(C.byref(_params(layout="FLUID", **kw)), C.byref(sz)) == 0
    p = _params(layout="FLUID", collision="CLBM")
    assert lib.lbm_workspace_size(C.byref(p), C.byref(sz)) == -2
    p = _params(layout="FLUID")
    p.lattice, p.nz = 0, 1                                  # a valid D2Q9 set
    assert lib.lbm_workspace_size(C.byref(p), C.byref(sz)) == -2
    p.layout = 0
    assert lib.lbm_workspace_size(C.byref(p), C.byref(sz)) == 0
    p = _params()
    p.layout = 2
    assert lib.lbm_workspace_size(C.byref(p), C.byref(sz)) == -1
    # a convective outlet with 16-bit storage: refused before the GPU is touched
    w, mask, rho = inputs.pcsw_pack(n=12, buffer=2, shape=(18, 12, 12), outlet="convective")
    p = lbm.params_from(w.with_(layout="FLUID", storage="F16DEV"))
    assert lib.lbm_workspace_size(C.byref(p), C.byref(sz)) == 0
    m = np.ascontiguousarray(mask.reshape(-1).astype(np.uint8))
    r = np.ascontiguousarray(rho.reshape(2, -1))
    h = C.c_void_p()
    rc = lib.lbm_init(C.byref(p), m.ctypes.data, r.ctypes.data, None, None, C.c_void_p(1 << 20), sz.value, None,
                      C.byref(h))
    assert rc == -2
