"""Pins of the oracle's reference-point dose (Sec. 2.5: absolute calibration
and relative output factors): the voxel set against a brute-force loop,
closed forms for constant and linear doses, the fallback to the voxel
holding the point."""
import itertools
import math

import numpy as np
import pytest

import psl_synth as S


def _approx(v):
    return pytest.approx(v, rel=1e-12, abs=1e-300)


def test_point_set_matches_brute_force(oracle_lib):
    rng = np.random.default_rng(3)
    ph = S.water_phantom((7, 6, 5), 0.5, (-1.3, -1.1, 99.6))
    d = rng.random((5, 6, 7))
    s = rng.random((5, 6, 7)) * 0.1
    for point, r in (((0.1, 0.2, 100.7), 0.6), ((0.0, 0.0, 100.0), 1.1),
                     ((-1.2, 1.8, 101.9), 0.8), ((0.3, -0.4, 100.2), 0.0)):
        got = oracle_lib.dose_point(d, s, ph, point, r)
        sel = []
        for k, j, i in itertools.product(range(5), range(6), range(7)):
            c = (-1.3 + (i + 0.5) * 0.5, -1.1 + (j + 0.5) * 0.5,
                 99.6 + (k + 0.5) * 0.5)
            if sum((c[a] - point[a]) ** 2 for a in range(3)) <= r * r:
                sel.append((k, j, i))
        if not sel:
            i = math.floor((point[0] + 1.3) / 0.5)
            j = math.floor((point[1] + 1.1) / 0.5)
            k = math.floor((point[2] - 99.6) / 0.5)
            sel = [(k, j, i)]
        want = np.mean([d[v] for v in sel])
        se = math.sqrt(sum(s[v] ** 2 for v in sel)) / len(sel)
        assert got[2] == len(sel)
        assert got[0] == _approx(want)
        assert got[1] == _approx(se)


def test_point_closed_forms(oracle_lib):
    ph = S.water_phantom((20, 20, 20), 0.25, (-2.5, -2.5, 100.0))
    # constant dose and sigma: the mean is the constant, the standard
    # error sigma / sqrt(n)
    d = np.full((20, 20, 20), 3.0)
    s = np.full((20, 20, 20), 0.2)
    m, se, n = oracle_lib.dose_point(d, s, ph, (0.0, 0.0, 102.5), 0.6)
    assert m == 3.0 and se == pytest.approx(0.2 / math.sqrt(n))
    # a linear dose about a voxel centre: the sphere's voxel set is
    # symmetric, so the mean is the value at the centre
    z, y, x = np.meshgrid(100.0 + (np.arange(20) + 0.5) * 0.25,
                          -2.5 + (np.arange(20) + 0.5) * 0.25,
                          -2.5 + (np.arange(20) + 0.5) * 0.25, indexing="ij")
    lin = 1.0 + 0.3 * x - 0.2 * y + 0.05 * (z - 100.0)
    c = (-2.5 + 10.5 * 0.25, -2.5 + 9.5 * 0.25, 100.0 + 11.5 * 0.25)
    m, _, n = oracle_lib.dose_point(lin, s, ph, c, 0.7)
    want = 1.0 + 0.3 * c[0] - 0.2 * c[1] + 0.05 * (c[2] - 100.0)
    assert n > 20 and m == pytest.approx(want, rel=1e-13)
    # outside the phantom with no centre in reach: nothing
    assert oracle_lib.dose_point(d, s, ph, (9.0, 0.0, 90.0), 0.5) == \
        (0.0, 0.0, 0)


def test_point_radius_is_closed(oracle_lib):
    """Voxel centres at exactly the radius belong to the set: about a voxel
    centre with the radius one voxel, the centre and its six face
    neighbours (all distances exact in binary)."""
    ph = S.water_phantom((8, 8, 8), 0.5, (-2.0, -2.0, 100.0))
    d = np.arange(512, dtype=np.float64).reshape(8, 8, 8)
    s = np.full((8, 8, 8), 0.1)
    m, se, n = oracle_lib.dose_point(d, s, ph, (0.25, 0.25, 102.25), 0.5)
    nb = [(4, 4, 4), (3, 4, 4), (5, 4, 4), (4, 3, 4), (4, 5, 4), (4, 4, 3),
          (4, 4, 5)]
    assert n == 7
    assert m == _approx(np.mean([d[v] for v in nb]))
    assert se == _approx(math.sqrt(7 * 0.01) / 7)


def test_batch_mean_standard_error_and_dose_worked_example(oracle_lib):
    """Eq. (5) and the batch uncertainty on numbers worked by hand: batch
    energies 1, 2, 3 and 6 MeV in a voxel give the mean 3, the sample
    variance (4 + 1 + 0 + 9) / 3 = 14/3 and the standard error of the mean
    sqrt(14/3 / 4) = sqrt(7/6); the dose is energy x 1.602176634e-10 Gy per
    MeV/g over the voxel mass rho V (here 0.5 g/cm^3 x 8 cm^3), times the
    normalisation; a voxel of density 0 has no dose."""
    ph = S.water_phantom((2, 1, 1), 2.0, (0.0, 0.0, 0.0))
    ph.density[0, 0, :] = [0.5, 0.0]
    # (the finaliser divides by rho V before masking the rho = 0 voxel)
    s1 = np.zeros(2)
    s2 = np.zeros(2)
    for e in (1.0, 2.0, 3.0, 6.0):
        oracle_lib.fold(np.array([e, e]), s1, s2)
    assert list(s1) == [12.0, 12.0] and list(s2) == [50.0, 50.0]
    norm = 1e-3
    dose, se = oracle_lib.finalize(s1, s2, 4, ph, norm)
    c = 1.602176634e-10 / (0.5 * 8.0) * norm
    assert dose[0] == pytest.approx(3.0 * c, rel=1e-15, abs=0)
    assert se[0] == pytest.approx(math.sqrt(7.0 / 6.0) * c, rel=1e-15, abs=0)
    assert dose[1] == 0.0 and se[1] == 0.0
