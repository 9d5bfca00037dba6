"""Pins of the oracle's azimuthal particle redistribution (Sec. 2.3.1):
the counter-based azimuth against a pure-Python reading of its definition,
uniformity of the azimuth, and the invariants of a turn about the central
axis (radius, transverse direction length, the position-direction angle,
energy, type, w, total weight)."""
import math

import numpy as np
from scipy import stats

import psl_synth as S

M64 = (1 << 64) - 1


def _splitmix64(x):
    z = (x + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def _azimuth(seed, m):
    key = _splitmix64(seed ^ m)
    for t in range(64):
        a = (_splitmix64((key + 2 * t) & M64) >> 11) * 2.0 ** -53 * 2.0 - 1.0
        b = (_splitmix64((key + 2 * t + 1) & M64) >> 11) * 2.0 ** -53 * 2.0 \
            - 1.0
        r2 = a * a + b * b
        if 0.0 < r2 <= 1.0:
            return (a * a - b * b) / r2, 2.0 * a * b / r2
    return 1.0, 0.0


def test_azimuth_matches_its_definition(oracle_lib):
    for seed in (0, 7, 2**63 + 5):
        for m in (0, 1, 2, 1000, 123456789, 2**40 + 3):
            assert oracle_lib.apr_rotation(seed, m) == _azimuth(seed, m)


def test_azimuth_is_uniform(oracle_lib):
    ang = np.array([math.atan2(*oracle_lib.apr_rotation(3, m)[::-1])
                    for m in range(20000)])
    assert stats.kstest((ang + math.pi) / (2 * math.pi), "uniform").pvalue \
        > 1e-3
    cs = np.array([oracle_lib.apr_rotation(3, m) for m in range(2000)])
    np.testing.assert_allclose((cs ** 2).sum(1), 1.0, atol=4e-16)


def test_expanded_copies_are_turned_particles(oracle_lib):
    ps = S.phase_space(3000, 5, 20.0, S.Z_PSL, aim="disk")
    ps.wt[:] = np.linspace(0.5, 2.0, ps.n, dtype=np.float32)
    k = 4
    ex = oracle_lib.apr_expand(ps, k, 99)
    assert ex.n == k * ps.n
    i = np.repeat(np.arange(ps.n), k)
    np.testing.assert_array_equal(ex.type, ps.type[i])
    np.testing.assert_array_equal(ex.E, ps.E[i])
    np.testing.assert_array_equal(ex.w, ps.w[i])
    np.testing.assert_allclose(ex.wt, ps.wt[i] / k, rtol=1e-7)
    assert abs(ex.wt.astype(np.float64).sum() /
               ps.wt.astype(np.float64).sum() - 1) < 1e-6
    x, y = ps.x[i].astype(np.float64), ps.y[i].astype(np.float64)
    u, v = ps.u[i].astype(np.float64), ps.v[i].astype(np.float64)
    X, Y = ex.x.astype(np.float64), ex.y.astype(np.float64)
    U, V = ex.u.astype(np.float64), ex.v.astype(np.float64)
    np.testing.assert_allclose(np.hypot(X, Y), np.hypot(x, y), rtol=1e-6,
                               atol=1e-6)
    np.testing.assert_allclose(np.hypot(U, V), np.hypot(u, v), rtol=1e-6,
                               atol=1e-7)
    # one turn for position and direction: the dot and cross products of
    # the transverse position and direction are kept
    np.testing.assert_allclose(X * U + Y * V, x * u + y * v, atol=2e-6)
    np.testing.assert_allclose(X * V - Y * U, x * v - y * u, atol=2e-6)
    # and the turn is the azimuth of the copy
    c, s = np.array([oracle_lib.apr_rotation(99, m) for m in range(ex.n)]).T
    np.testing.assert_allclose(X, c * x - s * y, atol=2e-6)
    np.testing.assert_allclose(Y, s * x + c * y, atol=2e-6)
    # copies of one particle spread over all azimuths
    phi = np.arctan2(Y, X)[::k]
    assert stats.kstest((phi + math.pi) / (2 * math.pi), "uniform").pvalue \
        > 1e-3
