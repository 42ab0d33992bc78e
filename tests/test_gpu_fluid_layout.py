"""The fluid-only layout (lbm_params.layout = LBM_LAYOUT_FLUID) through the
C-ABI: parity with the FP64 oracle at the dense layout's tolerances (max-norm
relative 1e-10 with FP64 storage, 1e-4 with FP32), agreement with the dense
layout on the same input, state round trip, reset and statistics."""
import numpy as np
import pytest

from paper_2506_17713_amd import inputs

from test_gpu_parity import MRT_D3Q19_2C, _sessile_mrt, assert_tol, run_pair

pytestmark = pytest.mark.gpu


def fluid(w):
    return w.with_(layout="FLUID")


@pytest.mark.parametrize("storage,tol", [("F64", 1e-10), ("F32", 1e-4), ("F32F64", 1e-4)])
@pytest.mark.parametrize("collision", ["BGK", "MRT"])
def test_two_component_pack(oracle_mod, storage, tol, collision):
    # psi = rho, DRHO / PHI wetting, common velocity; MRT at tau = 0.8 with
    # distinct rates (momentum rows relaxed toward u')
    w, solid, rho = inputs.two_component_pack(shape=(34, 37, 45), storage=storage, radii=(4.0, 7.0), seed=3)
    if collision == "MRT":
        w = w.with_(collision="MRT", tau=(0.8, 0.8), mrt_s=(MRT_D3Q19_2C, MRT_D3Q19_2C))
    out, _, _ = run_pair(oracle_mod, fluid(w), solid, rho, 200)
    assert_tol(out, tol)


@pytest.mark.parametrize("storage,tol", [("F64", 1e-10), ("F32", 1e-4)])
def test_eos_sessile_zhang_chen_mrt(oracle_mod, storage, tol):
    # one component, Carnahan-Starling psi with the Zhang-Chen term (the U
    # gather), PHI wetting, MRT at tau = 0.8 with distinct rates
    w, solid, rho = _sessile_mrt(storage)
    out, _, _ = run_pair(oracle_mod, fluid(w), solid, rho, 300)
    assert_tol(out, tol)


def test_per_node_wetting_body_force_and_velocity_f64(oracle_mod):
    # per-node wetting field at the solids, body force, initial velocity
    shape = (24, 26, 35)
    w, solid, rho = inputs.adjoint_pack(shape=shape, storage="F64", radii=(3.0, 6.0), seed=5)
    rng = np.random.default_rng(11)
    wet = rng.uniform(1.0, 1.3, size=(1,) + shape)
    u0 = np.zeros((3,) + shape)
    u0[0] = 0.01 * np.sin(2 * np.pi * np.arange(shape[2]) / shape[2])[None, None, :]
    u0[:, solid == 1] = 0.0
    w = fluid(w.with_(body=(1e-5, -2e-5, 3e-6)))
    out, _, _ = run_pair(oracle_mod, w, solid, rho, 60, u0=u0, wet=wet)
    assert_tol(out, 1e-10)


@pytest.mark.parametrize("collision", ["BGK", "MRT"])
def test_eos_drho_wetting_ragged_f32(oracle_mod, collision):
    # DRHO virtual density with its limiter; extents that are not multiples of 64
    w, solid, rho = inputs.sessile_3d(n=30, r=8, w=3, storage="F32", wet_mode="DRHO", wet=0.1)
    out, _, _ = run_pair(oracle_mod, fluid(w.with_(collision=collision)), solid, rho, 150)
    assert_tol(out, 1e-4)


@pytest.mark.parametrize("storage", ["F64", "F32"])
def test_fluid_layout_agrees_with_dense(storage):
    # the same step on the same input: after one step the two layouts agree
    # (bitwise on the tested build: the node arithmetic is the same; the
    # compiler may contract multiply-adds differently in the two kernels),
    # after 100 steps to rounding, and so do the statistics
    import torch

    from paper_2506_17713_amd import lbm

    w, solid, rho = inputs.two_component_pack(shape=(40, 40, 40), storage=storage, radii=(4.0, 8.0), seed=0)
    w = w.with_(collision="MRT", tau=(0.8, 0.8), mrt_s=(MRT_D3Q19_2C, MRT_D3Q19_2C))
    d = lbm.Solver(w, solid, rho)
    f = lbm.Solver(fluid(w), solid, rho)
    for steps in (1, 99):
        d.step(steps)
        f.step(steps)
        for comp in (-1, 0, 1):
            rd, ud = d.moments(comp)
            rf, uf = f.moments(comp)
            torch.cuda.synchronize()
            er = float((rd - rf).abs().max() / rd.abs().max())
            eu = float((ud - uf).abs().max() / ud.abs().max())
            print(f"layouts steps {d.stats()['step']} comp {comp}: rho {er:.3g} u {eu:.3g} "
                  f"bitwise {bool(torch.equal(rd, rf) and torch.equal(ud, uf))}", flush=True)
            tol = (1e-14 if storage == "F64" else 1e-6) if steps == 1 else (1e-10 if storage == "F64" else 1e-4)
            assert er <= tol and eu <= tol * 10
    sd, sf = d.stats(), f.stats()
    assert sd["n_fluid"] == sf["n_fluid"]
    for k in range(2):
        assert abs(sd["mass"][k] - sf["mass"][k]) <= (1e-12 if storage == "F64" else 1e-6) * sd["mass"][k]
    d.close()
    f.close()


def test_fluid_state_round_trip_and_reset():
    import torch

    from paper_2506_17713_amd import lbm

    w, solid, rho = inputs.two_component_pack(shape=(30, 33, 36), storage="F32", radii=(4.0, 7.0), seed=2)
    w = fluid(w)
    n_fl = int((solid == 0).sum())
    a = lbm.Solver(w, solid, rho)
    assert a.state_bytes() == 2 * 19 * ((w.N + 63) // 64 * 64) * 4
    a.step(30)
    snap = a.get_state().clone()
    a.step(30)
    ra, ua = a.moments(-1)
    c = lbm.Solver(w, solid, np.ones_like(rho))
    c.set_state(snap)
    c.step(30)
    rc, uc = c.moments(-1)
    torch.cuda.synchronize()
    assert torch.equal(ra, rc) and torch.equal(ua, uc)
    # reset from device fields gives the state lbm_init gives
    b = lbm.Solver(w, solid, np.ones_like(rho))
    b.step(5)
    b.reset(torch.tensor(rho.reshape(2, -1), dtype=torch.float32, device="cuda"))
    a2 = lbm.Solver(w, solid, rho)
    sa, sb = a2.get_state(), b.get_state()
    torch.cuda.synchronize()
    assert torch.equal(sa, sb)
    assert a2.stats()["n_fluid"] == n_fl
    for s in (a, b, c, a2):
        s.close()


def test_fluid_layout_grad_is_unsupported():
    from paper_2506_17713_amd import lbm

    w, solid, rho = inputs.adjoint_pack(shape=(16, 16, 16), storage="F64", radii=(3.0, 5.0), seed=1)
    s = lbm.Solver(fluid(w), solid, rho)
    with pytest.raises(lbm.LbmError) as ei:
        s.grad(4, 2)
    assert ei.value.code == -2
    s.close()


# ------------------------------------------------ open boundaries: reservoirs
@pytest.mark.parametrize("storage", ["F64", "F32"])
def test_drainage_pack_between_reservoirs(oracle_mod, storage):
    # the capillary pressure - saturation workload at a small size, inlet
    # pressure raised: anti-bounce-back inflow, reservoir densities in the
    # force and the virtual densities, capillary slots of lbm_stats
    from test_gpu_open_boundary import _RHO, check_capillary, check_fields

    w, mask, rho = inputs.pcsw_pack(n=40, buffer=4, storage=storage, dp_rho=0.08, shape=(50, 37, 40))
    w = fluid(w.with_(name="fl_pcsw_pack"))
    _RHO[w.name] = rho
    out, st, _ = run_pair(oracle_mod, w, mask, rho, 300)
    check_fields(out, storage)
    check_capillary(oracle_mod, w, mask, st, 300)


@pytest.mark.parametrize("storage", ["F64", "F32"])
def test_liquid_reservoir_imbibition_mrt(oracle_mod, storage):
    # one CS component at T_r = 0.8 with the Zhang-Chen term, d'Humieres MRT
    # at tau = 0.8: a vapour tube between a liquid reservoir below and a
    # vapour reservoir above
    from test_gpu_open_boundary import _RHO, check_capillary, check_fields

    coex = inputs.load_coexistence()["CS"]["0.8"]
    T, rv, rl, A = coex["T"], coex["rho_v"], coex["rho_l"], coex["A"]
    shape = (30, 11, 70)
    mask = np.zeros(shape, np.uint8)
    mask[:, 0, :] = 1
    mask[:, :, 0] = 1
    mask[0], mask[-1] = 2, 3
    z = np.arange(shape[0])[:, None, None] * np.ones(shape)
    rho = inputs.tanh_profile(z, 6.0, 4.0, rl, rv)[None]
    dh = inputs.dhumieres_rates(0.8)
    w = inputs.Workload("fl_imbibition3d", "D3Q19", shape, storage=storage, collision="MRT", tau=(0.8, 0.8),
                        mrt_s=(dh, dh), eos_T=(T, T), A=(A, A), wet=(1.1, 1.1), rho_min=(rv, rv), rho_max=(rl, rl),
                        res_rho=((rl, rl), (rv, rv)), window=(2, 28), layout="FLUID")
    _RHO[w.name] = rho
    out, st, _ = run_pair(oracle_mod, w, mask, rho, 300)
    check_fields(out, storage)
    check_capillary(oracle_mod, w, mask, st, 300)


def test_set_reservoir_between_steps(oracle_mod):
    from paper_2506_17713_amd import lbm

    w, mask, rho = inputs.pcsw_pack(n=24, buffer=3, storage="F64", shape=(32, 20, 24))
    w = fluid(w)
    print(f"case fluid set_reservoir {w.shape}", flush=True)
    sol = lbm.Solver(w, mask, rho)
    ref = oracle_mod.State(w, mask, rho)
    sol.step(60)
    ref.step(60)
    sol.set_reservoir(0, (1.12, 0.03))
    ref.set_reservoir(0, (1.12, 0.03))
    sol.step(60)
    ref.step(60)
    r_gpu, u_gpu = sol.moments_numpy(-1)
    sol.close()
    fl = ref.fields()
    fluid_nodes = mask.reshape(-1) == 0
    r_ref = np.where(fluid_nodes, fl["rho"].sum(0), 0.0)
    assert np.abs(r_gpu - r_ref).max() < 1e-10 * r_ref.max()
    assert np.abs(u_gpu - fl["umix"]).max() < 1e-10 * np.abs(fl["umix"]).max()


# ------------------------------------------------------ 16-bit deviations
@pytest.mark.parametrize("storage", ["F16DEV", "BF16DEV"])
def test_deviation_storage_agrees_with_dense(oracle_mod, storage):
    # the same deviation form as the dense layout (h = f* / (w rho*) - 1,
    # rho* of the storing node): one step agrees with the dense layout to
    # one rounding of the stored 16-bit deviations (a last-bit FP32
    # difference between the two kernels' contractions can flip it; measured
    # 6e-6 in rho, 5e-5 in u with FP16); after 300 steps the run stays within
    # the error the dense 16-bit storage reports against the FP64 oracle
    import torch

    from paper_2506_17713_amd import lbm

    w, solid, rho = inputs.two_component_pack(shape=(40, 40, 40), storage=storage, radii=(4.0, 8.0), seed=0)
    d = lbm.Solver(w, solid, rho)
    f = lbm.Solver(fluid(w), solid, rho)
    d.step(1)
    f.step(1)
    for comp in (-1, 0, 1):
        rd, ud = d.moments(comp)
        rf, uf = f.moments(comp)
        torch.cuda.synchronize()
        er = float((rd - rf).abs().max() / rd.abs().max())
        eu = float((ud - uf).abs().max() / ud.abs().max())
        print(f"{storage} one step comp {comp}: rho {er:.3g} u {eu:.3g}", flush=True)
        assert er <= 5e-5 and eu <= 5e-4
    d.close()
    f.close()
    out, st, _ = run_pair(oracle_mod, fluid(w), solid, rho, 300)
    for c, (er, eu) in out.items():
        assert er < 5e-2 and eu < 0.5, (c, er, eu)
    assert st["nonfinite"] == 0 and st["negative"] == 0


# ------------------------------------------------------------ degenerate cases
def test_all_fluid_box_f64(oracle_mod):
    # no solid node (no listed solids, no bounce-back): a periodic
    # two-component box with a non-wetting blob
    shape = (16, 17, 20)
    solid = np.zeros(shape, np.uint8)
    w, _, _ = inputs.two_component_pack(shape=shape, storage="F64", solid=solid)
    z, y, x = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    blob = ((z - 8.0) ** 2 + (y - 8.0) ** 2 + (x - 10.0) ** 2) < 25.0
    rho = np.stack([np.where(blob, 1.0, 0.03), np.where(blob, 0.03, 1.0)])
    out, _, _ = run_pair(oracle_mod, fluid(w), solid, rho, 100)
    assert_tol(out, 1e-10)


def test_all_solid_lattice():
    # no fluid node: steps launch nothing, moments and statistics are zero
    import torch

    from paper_2506_17713_amd import lbm

    shape = (8, 9, 10)
    solid = np.ones(shape, np.uint8)
    w, _, _ = inputs.two_component_pack(shape=shape, storage="F32", solid=solid)
    s = lbm.Solver(fluid(w), solid, np.ones((2,) + shape))
    s.step(5)
    r, u = s.moments(-1)
    torch.cuda.synchronize()
    assert float(r.abs().max()) == 0.0 and float(u.abs().max()) == 0.0
    st = s.stats()
    assert st["n_fluid"] == 0 and st["mass"][0] == 0.0 and st["nonfinite"] == 0
    s.close()


# --------------------------------------------------------- convective outlet
@pytest.mark.parametrize("storage", ["F64", "F32"])
def test_body_force_drainage_with_convective_outlet(oracle_mod, storage):
    # Sec. 3.4.2: the non-wetting fluid of the inlet buffer driven into the
    # wetting-saturated pack by a body force, a convective outlet at the far
    # end (outlet ids pulled from, never collided; their ghost populations
    # formed after each step)
    from test_gpu_open_boundary import _RHO, check_capillary, check_fields

    w, mask, rho = inputs.pcsw_pack(n=40, buffer=4, storage=storage, shape=(50, 37, 40), outlet="convective",
                                    body=2e-4)
    w = fluid(w.with_(name="fl_conv_drainage"))
    _RHO[w.name] = rho
    out, st, _ = run_pair(oracle_mod, w, mask, rho, 300)
    check_fields(out, storage)
    check_capillary(oracle_mod, w, mask, st, 300)


def test_convective_outlet_agrees_with_dense():
    # one step on both layouts from the same start (the outlet's mean
    # velocity is summed in another order: agreement to rounding)
    import torch

    from paper_2506_17713_amd import lbm

    w, mask, rho = inputs.pcsw_pack(n=24, buffer=3, storage="F64", shape=(32, 20, 24), outlet="convective",
                                    body=2e-4)
    d = lbm.Solver(w, mask, rho)
    f = lbm.Solver(fluid(w), mask, rho)
    for steps in (1, 49):
        d.step(steps)
        f.step(steps)
        rd, ud = d.moments(-1)
        rf, uf = f.moments(-1)
        torch.cuda.synchronize()
        er = float((rd - rf).abs().max() / rd.abs().max())
        eu = float((ud - uf).abs().max() / ud.abs().max())
        print(f"outlet layouts after {d.stats()['step']} steps: rho {er:.3g} u {eu:.3g}", flush=True)
        assert er <= 1e-12 and eu <= 1e-10
    d.close()
    f.close()
