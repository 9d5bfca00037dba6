"""Pins of the gamma-index and z-score tools used by the parity tests."""
import numpy as np
import pytest

from oracle import analysis


def test_gamma_dose_criterion_uniform_field():
    ref = np.ones((8, 8, 8))
    assert analysis.gamma_pass_rate(ref, ref * 1.019, 0.25) == 1.0
    assert analysis.gamma_pass_rate(ref, ref * 1.021, 0.25) == 0.0
    assert analysis.gamma_pass_rate(ref, ref * 0.981, 0.25) == 1.0


def test_gamma_distance_criterion_on_a_ramp():
    """Shifted ramp, negligible dose tolerance: gamma = shift / DTA."""
    vox = 0.05
    x = np.arange(40) * vox
    ramp = np.broadcast_to(1.0 + 5.0 * x, (6, 6, 40)).copy()
    def shifted(d):
        return np.broadcast_to(1.0 + 5.0 * (x - d), (6, 6, 40)).copy()
    inner = np.zeros(ramp.shape, bool)
    inner[:, :, 8:32] = True
    for d, want in ((0.16, 1.0), (0.24, 0.0)):
        ev = shifted(d)
        r = analysis.gamma_pass_rate(ramp, ev, vox, dose_crit=1e-5, dta=0.2,
                                     threshold=0.0, step=0.01, region=inner)
        assert r == want


def test_gamma_identical():
    rng = np.random.default_rng(1)
    d = rng.random((10, 10, 10))
    assert analysis.gamma_pass_rate(d, d, 0.5) == 1.0


def test_zscore():
    rng = np.random.default_rng(2)
    mu = np.full(20000, 10.0)
    sa = np.full(20000, 0.3)
    a = mu + rng.normal(0, 0.3, mu.shape)
    b = mu + rng.normal(0, 0.4, mu.shape)
    z = analysis.zscore_stats(a, sa, b, np.full(20000, 0.4))
    assert z["frac_le3"] > 0.99
    assert abs(z["mean"]) < 0.05 and 0.95 < z["sd"] < 1.05
    zb = analysis.zscore_stats(a + 1.0, sa, b, np.full(20000, 0.4))
    assert zb["mean"] > 1.5


def test_time_to_uncertainty_worked_example():
    """T_1% = T_run (sigma_bar / 1%)^2 with sigma_bar the mean relative
    uncertainty at or above half the maximum: relative uncertainties 2% and
    4% on the two voxels above half the maximum give sigma_bar = 3%, so a
    1 s run needs 9 s; the voxel below half the maximum does not count."""
    dose = np.array([1.0, 0.8, 0.3])
    sigma = np.array([0.02, 0.032, 0.3])
    t, s = analysis.time_to_uncertainty(1.0, dose, sigma)
    assert s == pytest.approx(0.03, rel=1e-12)
    assert t == pytest.approx(9.0, rel=1e-12)
