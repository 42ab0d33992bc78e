"""Host-side logic of the learned warm start (no GPU): the velocity gain's
least-squares fit, the start formed from predicted fields, and the channel
rules of the training symmetries."""
import numpy as np

from paper_2506_17713_amd.surrogate import NU, calibrate_flow, symmetry_args, warm_fields


class _FixedModel:
    """Stands in for Surrogate.predict: returns gain * a stored field."""

    def __init__(self, fields):
        self.fields = fields
        self.flow_gain = 1.0

    def predict(self, x):
        out = self.fields[x].copy()
        out[:3] *= self.flow_gain
        return out


def test_velocity_gain_is_the_least_squares_fit_of_the_permeabilities():
    rng = np.random.default_rng(0)
    preds = [rng.uniform(0.0, 1.0, size=(4, 3, 4, 5)) for _ in range(5)]
    scale = 0.8
    targets = [np.concatenate([p[:3] * scale * (1 + 0.01 * k), p[3:]]) for k, p in enumerate(preds)]
    m = _FixedModel(preds)
    m.flow_gain = 7.0  # ignored: the fit starts from gain 1
    g = calibrate_flow(m, list(range(5)), targets)
    kp = np.array([p[0].mean() for p in preds])
    kt = np.array([t[0].mean() for t in targets])
    assert np.isclose(g, (kp * kt).sum() / (kp * kp).sum(), rtol=1e-12)
    assert m.flow_gain == g
    assert 0.8 < g < 0.84
    # an exact proportional target is recovered exactly
    m2 = _FixedModel(preds)
    assert np.isclose(calibrate_flow(m2, list(range(5)), [np.concatenate([p[:3] * 1.3, p[3:]]) for p in preds]),
                      1.3, rtol=1e-12)


def test_warm_start_fields():
    """u0 = u_pred a/nu - a/2 along x and rho0 = 1 + 3 a (p - <p>_pores) at pores;
    rest at rho = 1 in solids; the start holds the mass of rho = 1."""
    rng = np.random.default_rng(1)
    solid = (rng.uniform(size=(4, 5, 6)) < 0.3).astype(np.uint8)
    pred = rng.standard_normal((4,) + solid.shape) * (solid == 0)
    a = 1e-5
    rho0, u0 = warm_fields(pred, solid, a)
    fl = solid.reshape(-1) == 0
    assert rho0.shape == (1, solid.size) and u0.shape == (3, solid.size)
    np.testing.assert_allclose(rho0[0][~fl], 1.0)
    np.testing.assert_allclose(u0[:, ~fl], 0.0)
    np.testing.assert_allclose(u0[1:, fl], pred[1:3].reshape(2, -1)[:, fl] * a / NU, rtol=1e-12)
    np.testing.assert_allclose(u0[0, fl], pred[0].reshape(-1)[fl] * a / NU - a / 2, rtol=1e-12)
    assert abs(rho0[0][fl].sum() - fl.sum()) < 1e-9
    p = pred[3].reshape(-1)[fl]
    np.testing.assert_allclose(rho0[0][fl], 1 + 3 * a * (p - p.mean()), rtol=1e-12)


def test_symmetry_channel_rules():
    """Exchanging z and y swaps the u_y and u_z channels; flipping an axis
    negates that velocity component; flipping x also reverses the forcing,
    which negates every channel (Stokes linearity), so u_x keeps its sign."""
    shift, flip, swap, src, sign = symmetry_args([1, 2, 3], [0, 0, 0], False)
    assert (src, sign) == ([0, 1, 2, 3], [1.0, 1.0, 1.0, 1.0])
    _, _, _, src, sign = symmetry_args([0, 0, 0], [1, 0, 0], False)  # flip z
    assert (src, sign) == ([0, 1, 2, 3], [1.0, 1.0, -1.0, 1.0])
    _, _, _, src, sign = symmetry_args([0, 0, 0], [0, 1, 0], False)  # flip y
    assert (src, sign) == ([0, 1, 2, 3], [1.0, -1.0, 1.0, 1.0])
    _, _, _, src, sign = symmetry_args([0, 0, 0], [0, 0, 1], False)  # flip x
    assert (src, sign) == ([0, 1, 2, 3], [1.0, -1.0, -1.0, -1.0])
    _, _, swap, src, sign = symmetry_args([0, 0, 0], [0, 0, 0], True)  # exchange z and y
    assert swap and (src, sign) == ([0, 2, 1, 3], [1.0, 1.0, 1.0, 1.0])
