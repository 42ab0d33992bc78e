"""Pins of the oracle's MRT collision (Sec. 2.1, Eq. 3, MRT form) at
non-uniform relaxation rates, and of the default rate assignment
(Workload.mrt_rates) that the GPU path and the oracle both receive.

Uniform rates reduce MRT to BGK (test_oracle_lattice), which says nothing
about which moment row a rate acts on.  These tests fix that with flows whose
answers are known in closed form:

* Poiseuille flow between halfway bounce-back walls under a body force.  Its
  amplitude fixes the shear viscosity nu = (1/s_nu - 1/2) c_s^2, so the shear
  row of the wall orientation (p_xy, p_yz or p_xz) must carry s_nu.  With the
  two odd rows of the flow axis (energy flux q_d and, in D3Q19, the ghost
  moment m_d) at the rate s_q that makes (1/s_nu - 1/2)(1/s_q - 1/2) = 3/16,
  the halfway wall sits exactly midway and the parabola is reproduced to
  rounding (the classic exactness of two-rate schemes for Poiseuille flow);
  at any other pair of odd rows it is not.
* A plane shear wave along a lattice diagonal, u parallel to e_a - e_b with
  wavevector along e_a + e_b, is incompressible and strains only the normal
  stresses; its amplitude decays as exp(-nu |k|^2 t).  It fixes the rates of
  the normal-stress rows (3p_xx and p_ww in D3Q19, p_xx in D2Q9).

Rows are in the Lallemand-Luo (D2Q9) and d'Humieres (D3Q19) order:
  D2Q9   rho, e, eps, jx, qx, jy, qy, pxx, pxy
  D3Q19  rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww, piww,
         pxy, pyz, pxz, mx, my, mz
"""
import numpy as np
import pytest

from paper_2506_17713_amd import inputs
from paper_2506_17713_amd.inputs import Workload

TAU = 0.8
SV = 1.0 / TAU
NU = (TAU - 0.5) / 3.0
# odd-row rate with (1/s_nu - 1/2)(1/s_q - 1/2) = 3/16
S_MAGIC = 1.0 / (0.5 + (3.0 / 16.0) / (1.0 / SV - 0.5))


def rates_d3q19(se=1.19, seps=1.4, sq=1.2, sg=1.98, spi=1.0):
    r = [SV, se, seps, SV, sq, SV, sq, SV, sq, SV, spi, SV, spi, SV, SV, SV, sg, sg, sg]
    return r


def rates_d2q9(se=1.19, seps=1.4, sq=1.2):
    return [SV, se, seps, SV, sq, SV, sq, SV, SV]


def _flow_workload(lat, shape, rates, body):
    return Workload("mrt_pin", lat, shape, collision="MRT", tau=(TAU, TAU),
                    mrt_s=(tuple(rates), tuple(rates)), psi_kind=("DENSITY", "DENSITY"),
                    g=((0.0, 0.0), (0.0, 0.0)), body=body)


def poiseuille_error(oracle_mod, lat, flow, wall, rates, H=10, a=1e-6, steps=4000):
    """Max deviation of the steady profile from a/(2 nu) (y - 1/2)(H + 1/2 - y),
    relative to its peak; walls are the solid layers 0 and H + 1."""
    n = H + 2
    dims = {"x": 1, "y": 1, "z": 1}
    dims[wall] = n
    shape = (dims["z"], dims["y"], dims["x"])
    body = [0.0, 0.0, 0.0]
    body["xyz".index(flow)] = a
    w = _flow_workload(lat, shape, rates, tuple(body))
    st = oracle_mod.State(w, inputs.walls(shape, wall, (0, n - 1)), np.ones((1,) + shape))
    st.step(steps)
    u = st.fields()["umix"]["xyz".index(flow)].reshape(n)
    y = np.arange(n, dtype=float)
    exact = a / (2.0 * NU) * (y - 0.5) * (H + 0.5 - y)
    return float(np.abs(u[1:-1] - exact[1:-1]).max() / exact.max())


def shear_wave_viscosity(oracle_mod, lat, plane, rates, L=32, U=1e-4, t1=200, t2=1200):
    """Viscosity measured from the decay of a diagonal shear wave in `plane`."""
    a, b = plane
    dims = {"x": 1, "y": 1, "z": 1}
    dims[a] = dims[b] = L
    shape = (dims["z"], dims["y"], dims["x"])
    w = _flow_workload(lat, shape, rates, (0.0, 0.0, 0.0))
    x, y, z = inputs.grid(shape)
    c = {"x": x, "y": y, "z": z}
    k = 2.0 * np.pi / L
    s = np.sin(k * (c[a] + c[b]))
    ia, ib = "xyz".index(a), "xyz".index(b)
    u0 = np.zeros((3,) + shape)
    u0[ia] = U * s / np.sqrt(2.0)
    u0[ib] = -U * s / np.sqrt(2.0)
    st = oracle_mod.State(w, np.zeros(shape, np.uint8), np.ones((1,) + shape), u0=u0)
    pat = (u0[ia] - u0[ib]).reshape(-1)

    def amplitude():
        u = st.fields()["umix"]
        return float(((u[ia] - u[ib]) * pat).sum() / (pat * pat).sum())

    st.step(t1)
    A1 = amplitude()
    st.step(t2 - t1)
    A2 = amplitude()
    return float(np.log(A1 / A2) / (2.0 * k * k * (t2 - t1)))


# ------------------------------------------------------------ Poiseuille
D3_ORIENT = [("x", "z"), ("x", "y"), ("y", "z"), ("y", "x"), ("z", "x"), ("z", "y")]
ODD_ROWS_D3 = {"x": (4, 16), "y": (6, 17), "z": (8, 18)}


@pytest.mark.parametrize("flow,wall", D3_ORIENT)
def test_d3q19_magic_poiseuille_is_exact(oracle_mod, flow, wall):
    r = rates_d3q19()
    for m in ODD_ROWS_D3[flow]:
        r[m] = S_MAGIC
    assert poiseuille_error(oracle_mod, "D3Q19", flow, wall, r) < 1e-9


@pytest.mark.parametrize("flow", ["x", "y", "z"])
def test_d3q19_poiseuille_exactness_needs_the_flow_axis_odd_rows(oracle_mod, flow):
    # the magic rate on the odd rows of another axis leaves the wall-slip error
    wall = "x" if flow != "x" else "z"
    for other in "xyz":
        if other == flow:
            continue
        r = rates_d3q19()
        for m in ODD_ROWS_D3[other]:
            r[m] = S_MAGIC
        assert poiseuille_error(oracle_mod, "D3Q19", flow, wall, r) > 1e-3


@pytest.mark.parametrize("flow,wall", D3_ORIENT[:3])
def test_d3q19_poiseuille_viscosity_from_distinct_and_default_rates(oracle_mod, flow, wall):
    # distinct energy, flux and ghost rates: the amplitude is still set by s_nu
    # alone (the remaining error, 1e-2 at H = 10, is the wall slip of halfway
    # walls away from the exact rate pair)
    assert poiseuille_error(oracle_mod, "D3Q19", flow, wall, rates_d3q19()) < 1.5e-2
    # the default assignment: s_nu = 1/tau on the stress rows, 1 elsewhere
    default = Workload("d", "D3Q19", (1, 1, 1), tau=(TAU, TAU)).mrt_rates(0)
    assert poiseuille_error(oracle_mod, "D3Q19", flow, wall, default) < 1.5e-2
    # a different s_nu on the shear row moves the profile by the viscosity ratio
    shear_row = {("x", "y"): 13, ("y", "z"): 14, ("x", "z"): 15}[tuple(sorted((flow, wall)))]
    r = rates_d3q19()
    r[shear_row] = 1.0
    assert poiseuille_error(oracle_mod, "D3Q19", flow, wall, r) > 0.3


@pytest.mark.parametrize("flow", ["x", "y"])
def test_d2q9_magic_poiseuille_is_exact(oracle_mod, flow):
    wall = "y" if flow == "x" else "x"
    own, other = (4, 6) if flow == "x" else (6, 4)
    r = rates_d2q9()
    r[own] = S_MAGIC
    assert poiseuille_error(oracle_mod, "D2Q9", flow, wall, r) < 1e-9
    r = rates_d2q9()
    r[other] = S_MAGIC
    assert poiseuille_error(oracle_mod, "D2Q9", flow, wall, r) > 1e-3
    default = Workload("d", "D2Q9", (1, 1, 1), tau=(TAU, TAU)).mrt_rates(0)
    assert poiseuille_error(oracle_mod, "D2Q9", flow, wall, default) < 1.5e-2
    r = rates_d2q9()
    r[8] = 1.0
    assert poiseuille_error(oracle_mod, "D2Q9", flow, wall, r) > 0.3


# ------------------------------------------------------------ shear waves
@pytest.mark.parametrize("plane", [("x", "y"), ("x", "z"), ("y", "z")])
def test_d3q19_diagonal_shear_wave_decays_at_nu(oracle_mod, plane):
    nu = shear_wave_viscosity(oracle_mod, "D3Q19", plane, rates_d3q19())
    assert abs(nu / NU - 1.0) < 5e-3
    default = Workload("d", "D3Q19", (1, 1, 1), tau=(TAU, TAU)).mrt_rates(0)
    assert abs(shear_wave_viscosity(oracle_mod, "D3Q19", plane, default) / NU - 1.0) < 5e-3
    # the normal-stress rows this wave strains: 3pxx (row 9) in the planes
    # containing x, pww (row 11) in all three
    for row in (9, 11):
        r = rates_d3q19()
        r[row] = 1.0
        moved = abs(shear_wave_viscosity(oracle_mod, "D3Q19", plane, r) / NU - 1.0) > 0.1
        assert moved == (row == 11 or "x" in plane), (plane, row)


def test_d2q9_diagonal_shear_wave_decays_at_nu(oracle_mod):
    nu = shear_wave_viscosity(oracle_mod, "D2Q9", ("x", "y"), rates_d2q9())
    assert abs(nu / NU - 1.0) < 5e-3
    r = rates_d2q9()
    r[7] = 1.0
    assert abs(shear_wave_viscosity(oracle_mod, "D2Q9", ("x", "y"), r) / NU - 1.0) > 0.3


# rates of the GPU parity cases at non-unit rates (tests/test_gpu_parity.py)
RATES_GPU = (1.3, 1.19, 1.4, 1.1, 1.2, 1.1, 1.2, 1.1, 1.2, 1.25, 1.05, 1.25, 1.05, 1.25, 1.25, 1.25,
             1.98, 1.98, 1.98)


def test_mrt_rates_change_the_result(oracle_mod):
    """The non-unit rates of the GPU parity cases are not inert on a sessile
    droplet: changing the rate of any class of rows moves the oracle's result,
    so matching the oracle at these rates constrains where each rate acts."""
    c = inputs.load_coexistence()["CS"]["0.8"]
    shape = (16, 18, 20)
    w = Workload("sessile3d_mrt_rates", "D3Q19", shape, collision="MRT", storage="F64",
                 tau=(0.8, 0.8), mrt_s=(RATES_GPU, RATES_GPU), eos_T=(c["T"],) * 2,
                 A=(c["A"],) * 2, wet_mode=("PHI", "PHI"), wet=(1.1, 1.1),
                 rho_min=(c["rho_v"],) * 2, rho_max=(c["rho_l"],) * 2)
    solid = inputs.walls(shape, "z", (0, shape[0] - 1))
    rho = inputs.droplet(shape, (10.0, 9.0, 6.0), 5, 3, c["rho_l"], c["rho_v"])[None]
    base = oracle_mod.State(w, solid, rho)
    base.step(30)
    r0 = base.fields()["rho"][0]
    for rows in ((1,), (2,), (4, 6, 8), (9, 11), (10, 12), (13, 14, 15), (16, 17, 18)):
        s = list(RATES_GPU)
        for m in rows:
            s[m] = 1.0 if abs(s[m] - 1.0) > 1e-9 else 1.5
        st = oracle_mod.State(w.with_(mrt_s=(tuple(s), tuple(s))), solid, rho)
        st.step(30)
        d = np.abs(st.fields()["rho"][0] - r0).max() / np.abs(r0).max()
        assert d > 1e-9, rows
