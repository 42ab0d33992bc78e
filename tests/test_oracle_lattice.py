"""Pins of the oracle's lattice tables, equilibrium, MRT transform and
exact-difference forcing against closed-form identities."""
import numpy as np
import pytest

from paper_2506_17713_amd.inputs import Workload

CS2 = 1.0 / 3.0


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_lattice_isotropy(oracle_mod, lat):
    e, w, opp = oracle_mod.lattice(lat)
    q = 9 if lat == "D2Q9" else 19
    dim = 2 if lat == "D2Q9" else 3
    assert len(w) == q
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.abs((w[:, None] * e).sum(0)).max() < 1e-15
    second = np.einsum("i,ia,ib->ab", w, e, e)
    assert np.allclose(second[:dim, :dim], CS2 * np.eye(dim), atol=1e-15)
    # fourth-order isotropy: sum w e_a e_b e_c e_d = c_s^4 (d_ab d_cd + d_ac d_bd + d_ad d_bc)
    fourth = np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e)[:dim, :dim, :dim, :dim]
    I = np.eye(dim)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I)
                      + np.einsum("ad,bc->abcd", I, I))
    assert np.allclose(fourth, iso, atol=1e-15)
    # the force stencil G_i = w_i / c_s^2 gives sum_i G_i e_i e_i = I
    assert np.allclose(np.einsum("i,ia,ib->ab", w / CS2, e, e)[:dim, :dim], I, atol=1e-15)
    for i in range(q):
        assert np.array_equal(e[opp[i]], -e[i])


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_equilibrium_moments(oracle_mod, lat):
    e, w, _ = oracle_mod.lattice(lat)
    dim = 2 if lat == "D2Q9" else 3
    rng = np.random.default_rng(3)
    for _ in range(5):
        rho = rng.uniform(0.01, 2.0)
        u = np.zeros(3)
        u[:dim] = rng.uniform(-0.1, 0.1, dim)
        f = oracle_mod.feq(lat, rho, u)
        assert f.sum() == pytest.approx(rho, rel=1e-14)
        assert np.allclose(f @ e, rho * u, atol=1e-15)
        P = np.einsum("i,ia,ib->ab", f, e, e)[:dim, :dim]
        assert np.allclose(P, rho * np.outer(u, u)[:dim, :dim] + CS2 * rho * np.eye(dim), atol=1e-14)


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_mrt_matrix(oracle_mod, lat):
    M, Mi = oracle_mod.mrt_matrix(lat)
    e, w, _ = oracle_mod.lattice(lat)
    q = M.shape[0]
    G = M @ M.T
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-12  # orthogonal rows
    assert np.allclose(M @ Mi, np.eye(q), atol=1e-12)
    assert np.allclose(M[0], 1.0)
    assert np.allclose(M[3], e[:, 0])  # j_x row
    assert np.allclose(M[5], e[:, 1])  # j_y row
    if q == 19:
        assert np.allclose(M[7], e[:, 2])


def _node_workload(lat, coll, tau, rates=None):
    return Workload("node", lat, (1, 2, 2), collision=coll, tau=(tau, tau),
                    mrt_s=None if rates is None else (rates, rates))


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_mrt_uniform_rates_is_bgk(oracle_mod, lat):
    q = 9 if lat == "D2Q9" else 19
    tau = 0.83
    rng = np.random.default_rng(1)
    u = np.array([0.03, -0.02, 0.01 if q == 19 else 0.0])
    fin = oracle_mod.feq(lat, 1.1, u) * (1 + 0.05 * rng.standard_normal(q))
    j = fin @ oracle_mod.lattice(lat)[0]
    ueq = j / fin.sum()
    F = np.array([1e-3, -2e-3, 5e-4 if q == 19 else 0.0])
    bgk = oracle_mod.collide_node(_node_workload(lat, "BGK", tau), 0, fin, ueq, F)
    mrt = oracle_mod.collide_node(_node_workload(lat, "MRT", tau, [1 / tau] * q), 0, fin, ueq, F)
    assert np.allclose(bgk, mrt, rtol=0, atol=1e-15)


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
@pytest.mark.parametrize("coll", ["BGK", "MRT"])
def test_edm_adds_exactly_the_force(oracle_mod, lat, coll):
    # Eq. 5: the EDM term conserves mass and adds exactly F dt to the momentum.
    q = 9 if lat == "D2Q9" else 19
    e, _, _ = oracle_mod.lattice(lat)
    u = np.array([0.05, 0.02, -0.03 if q == 19 else 0.0])
    rng = np.random.default_rng(7)
    fin = oracle_mod.feq(lat, 0.3, u) * (1 + 0.02 * rng.standard_normal(q))
    ueq = (fin @ e) / fin.sum()
    F = np.array([2e-3, -1e-3, 3e-3 if q == 19 else 0.0])
    wl = _node_workload(lat, coll, 0.9)
    f0 = oracle_mod.collide_node(wl, 0, fin, ueq, np.zeros(3))
    f1 = oracle_mod.collide_node(wl, 0, fin, ueq, F)
    dF = f1 - f0
    assert abs(dF.sum()) < 1e-16
    assert np.allclose(dF @ e, F, rtol=0, atol=1e-16)
    # collision itself conserves mass and momentum at the equilibrium velocity
    assert f0.sum() == pytest.approx(fin.sum(), rel=1e-14)
    assert np.allclose(f0 @ e, fin @ e, atol=1e-15)


def test_bgk_tau_one_gives_shifted_equilibrium(oracle_mod):
    # with tau = 1 BGK relaxes fully: f* = f^eq(rho, u + F/rho)
    e, _, _ = oracle_mod.lattice("D3Q19")
    fin = oracle_mod.feq("D3Q19", 0.7, np.array([0.01, 0.0, 0.02])) + 1e-3
    rho = fin.sum()
    ueq = (fin @ e) / rho
    F = np.array([1e-3, 2e-3, 0.0])
    out = oracle_mod.collide_node(_node_workload("D3Q19", "BGK", 1.0), 0, fin, ueq, F)
    assert np.allclose(out, oracle_mod.feq("D3Q19", rho, ueq + F / rho), atol=1e-16)
