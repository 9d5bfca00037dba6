"""Pins of the oracle's transport physics against closed forms, library
quadrature, textbook values and exact special cases.

Physics model: Compton-only photons (Klein-Nishina, free electrons at
rest), CSDA electrons with the Bethe collision stopping power (I = 75 eV,
no density effect), 1 mm steps, Highland Gaussian multiple scattering,
cut-offs 10 keV (photons) and 0.7 MeV total energy (electrons, Sec. 2.6).
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import psl_synth as S

ME = 0.51099895
RE = 2.8179403262e-13
NE = 3.343e23
TCUT = 0.700 - ME


def dsigma_dcos(E, c):
    """Klein-Nishina differential cross section per electron, per unit
    cos(theta), integrated over azimuth (cm^2)."""
    P = 1.0 / (1.0 + E / ME * (1.0 - c))
    return math.pi * RE * RE * P * P * (P + 1.0 / P - (1.0 - c * c))


# ------------------------------------------------------- photons ---------
@pytest.mark.parametrize("E", [0.011, 0.1, 0.5, 1.0, 2.5, 6.0])
def test_kn_total_equals_integral_of_differential(oracle_lib, E):
    q, _ = integrate.quad(lambda c: dsigma_dcos(E, c), -1, 1,
                          epsabs=0, epsrel=1e-12)
    assert oracle_lib.kn_sigma(E) == pytest.approx(q, rel=1e-9)


def test_kn_thomson_limit(oracle_lib):
    # k -> 0: sigma -> 8 pi r_e^2 / 3 (1 - 2k + 26k^2/5)
    E = 1e-4
    k = E / ME
    thomson = 8 * math.pi / 3 * RE * RE
    assert oracle_lib.kn_sigma(E) == pytest.approx(
        thomson * (1 - 2 * k + 26 * k * k / 5), rel=1e-6)


def test_water_attenuation_textbook(oracle_lib):
    # Compton attenuation of water at 1 MeV: 0.0707 cm^2/g (textbook)
    mu = NE * oracle_lib.kn_sigma(1.0)
    assert mu == pytest.approx(0.0707, rel=2e-3)


def _pencil(oracle, E, n, ph, flags, seed=3):
    nz, ny, nx = ph.density.shape
    x0, y0, z0 = ph.origin
    st = np.zeros((n, 8))
    st[:, 0] = E
    st[:, 1] = x0 + nx * ph.voxel[0] / 2 + 1e-3
    st[:, 2] = y0 + ny * ph.voxel[1] / 2 + 1e-3
    st[:, 3] = z0
    st[:, 6] = 1.0
    st[:, 7] = 1.0
    types = np.zeros(n, np.uint8)
    uid = np.arange(n, dtype=np.uint64)
    return oracle.transport(types, st, uid, seed, ph,
                            oracle.ophys(flags=flags), ledger=True,
                            trace=True)


@pytest.mark.parametrize("E", [0.2, 1.25, 5.0])
def test_beer_lambert_first_interaction_depth(oracle_lib, E):
    """Uncollided fluence falls as exp(-mu d): first-interaction depths of a
    pencil beam follow the exponential law truncated at the exit face."""
    ph = S.water_phantom((4, 4, 40), 1.0, (-2.0, -2.0, 100.0))
    n = 40_000
    _, _, led, tr = _pencil(oracle_lib, E, n, ph,
                            oracle_lib.FLAG_FIRST_COLLISION)
    mu = NE * oracle_lib.kn_sigma(E)
    L = 40.0
    d = tr[:, 0] - 100.0
    hit = ~np.isnan(d)
    # the probability of interacting inside the slab is 1 - exp(-mu L)
    p = 1 - math.exp(-mu * L)
    assert abs(hit.mean() - p) < 4 * math.sqrt(p * (1 - p) / n)
    cdf = lambda z: (1 - np.exp(-mu * z)) / p
    assert stats.kstest(d[hit], cdf).pvalue > 1e-3


@pytest.mark.parametrize("E", [0.1, 1.0, 6.0])
def test_kn_angular_distribution_chi2(oracle_lib, E):
    ph = S.water_phantom((4, 4, 400), 1.0, (-2.0, -2.0, 100.0))
    n = 60_000
    _, _, _, tr = _pencil(oracle_lib, E, n, ph,
                          oracle_lib.FLAG_FIRST_COLLISION)
    c = tr[:, 1]
    c = c[~np.isnan(c)]
    edges = np.linspace(-1, 1, 41)
    obs, _ = np.histogram(c, edges)
    tot = oracle_lib.kn_sigma(E)
    p = np.array([integrate.quad(lambda x: dsigma_dcos(E, x), a, b)[0]
                  for a, b in zip(edges[:-1], edges[1:])]) / tot
    exp = p * len(c)
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, len(obs) - 1) > 1e-3
    # mean energy transfer T/E against sigma_tr / sigma
    tr_frac = integrate.quad(
        lambda x: dsigma_dcos(E, x) *
        (1 - 1 / (1 + E / ME * (1 - x))), -1, 1)[0] / tot
    T = tr[:, 2][~np.isnan(tr[:, 2])] / E
    assert abs(T.mean() - tr_frac) < 4 * T.std() / math.sqrt(len(T))


# ------------------------------------------------------ electrons --------
@pytest.mark.parametrize("T,estar", [(0.01, 22.56), (0.05, 6.603),
                                     (0.1, 4.115), (0.2, 2.793),
                                     (0.5, 2.034)])
def test_stopping_power_textbook(oracle_lib, T, estar):
    """Collision stopping power of water (NIST ESTAR, MeV cm^2/g) where the
    density effect is negligible."""
    assert oracle_lib.stopping_power(T) == pytest.approx(estar, rel=1.5e-3)


def test_stopping_power_nonrelativistic_limit(oracle_lib):
    """For T << mc^2 the Bethe formula tends to the non-relativistic form
    4 pi r_e^2 (mc^2)^2 n_e / (2T) ln(1.166 T / I) ... checked via its
    leading behaviour: S(T) T / ln(T/I) approaches a constant."""
    a = oracle_lib.stopping_power(0.002) * 0.002 / math.log(0.002 / 75e-6)
    b = oracle_lib.stopping_power(0.004) * 0.004 / math.log(0.004 / 75e-6)
    assert a == pytest.approx(b, rel=0.03)
    assert a == pytest.approx(2 * math.pi * RE * RE * ME * NE * ME,
                              rel=0.06)


@pytest.mark.parametrize("T", [0.25, 1.0, 3.0, 6.0])
def test_csda_range_quadrature(oracle_lib, T):
    q, _ = integrate.quad(lambda t: 1.0 / oracle_lib.stopping_power(t),
                          TCUT, T, epsabs=0, epsrel=1e-12)
    assert oracle_lib.csda_range(TCUT, T) == pytest.approx(q, rel=1e-9)


def test_csda_range_textbook(oracle_lib):
    # ESTAR CSDA range of water at 1 MeV: 0.4367 g/cm^2 (radiative loss and
    # density effect are below 1% there)
    assert oracle_lib.csda_range(0.001, 1.0) == pytest.approx(0.4367,
                                                              rel=5e-3)


def test_electron_track_length_and_depth_staircase(oracle_lib):
    """Without scattering a pencil electron travels straight for exactly its
    residual range; the energy it leaves in each voxel follows from the
    range-energy relation (solved here with scipy's ODE integrator)."""
    from scipy.integrate import solve_ivp
    T0 = 2.0
    dz = 0.05
    ph = S.water_phantom((3, 3, 400), dz, (-0.075, -0.075, 100.0))
    st = np.zeros((1, 8))
    st[0] = [T0, 1e-4, 1e-4, 100.0, 0, 0, 1, 1]
    acc, _, led, _ = oracle_lib.transport(
        np.ones(1, np.uint8), st, np.zeros(1, np.uint64), 1, ph,
        oracle_lib.ophys(flags=oracle_lib.FLAG_NO_MSC), ledger=True)
    dep = acc.reshape(400, 3, 3)[:, 1, 1]
    R = oracle_lib.csda_range(TCUT, T0)
    last = int(np.nonzero(dep)[0].max())
    assert last == int(R // dz)
    sol = solve_ivp(lambda s, t: [-oracle_lib.stopping_power(t[0])],
                    (0, last * dz), [T0], dense_output=True, rtol=1e-11,
                    atol=1e-12)
    Ts = sol.sol(np.arange(last + 1) * dz)[0]
    np.testing.assert_allclose(dep[:last], Ts[:-1] - Ts[1:], rtol=2e-6,
                               atol=1e-9)
    assert dep[last] == pytest.approx(Ts[-1], rel=2e-6)
    assert dep.sum() == pytest.approx(T0, rel=1e-12)


def test_highland_worked_value(oracle_lib):
    # 6 MeV electron, 1 mm of water: t/X0 = 0.1/36.08; beta c p =
    # T(T + 2m)/(T + m) = 6.4708 MeV; theta0 = 13.6/6.4708 * sqrt(t/X0)
    # * (1 + 0.038 ln(t/X0)) = 0.08589 rad
    assert oracle_lib.highland(6.0, 0.1) == pytest.approx(0.085889, rel=2e-5)
    # 1 MeV: beta c p = 1.4220 MeV -> 0.41532 rad
    assert oracle_lib.highland(1.0, 0.1) == pytest.approx(0.41532, rel=2e-5)


def test_highland_sampler_projected_variance(oracle_lib):
    """Projected angles of the oracle's scattering sampler are Gaussian with
    standard deviation theta0 (small angles)."""
    th0 = oracle_lib.highland(6.0, 0.1)
    s = oracle_lib.msc_samples(200_000, 6.0, 0.1, seed=11)
    for a in (0, 1):
        assert s[:, a].std() == pytest.approx(th0, rel=0.01)
        assert abs(s[:, a].mean()) < 4 * th0 / math.sqrt(len(s))
        assert stats.kstest(s[:20000, a] / th0, "norm").pvalue > 1e-3


def _slab_then_vacuum(rho, thick):
    """A slab of density rho and thickness `thick` cm over a vacuum layer of
    the same thickness, one 200 cm voxel wide laterally."""
    dens = np.array([rho, 0.0], np.float32).reshape(2, 1, 1)
    return S.Phantom(dens, (200.0, 200.0, thick), (-100.0, -100.0, 100.0))


@pytest.mark.parametrize("T0,rho,step", [(1.0, 1.0, 0.05), (1.0, 0.26, 0.1),
                                         (6.0, 1.0, 0.1), (3.0, 1.85, 0.1)])
def test_highland_deflection_inside_transport(oracle_lib, T0, rho, step):
    """One electron step through a slab exactly one step thick, then
    vacuum (no further energy loss or scattering): the exit direction is the
    one deflection the transport loop applied.  Its projected angles must be
    Gaussian with width theta0 of the Highland formula for the energy at the
    START of the step and the step's mass thickness rho x step.  (theta0 is
    kept below 0.3 rad so that no electron turns back into the slab.)"""
    ph = _slab_then_vacuum(rho, step)
    n = 40_000
    st = np.zeros((n, 8))
    st[:, 0] = T0
    st[:, 1:3] = 1e-3
    st[:, 3] = 100.0
    st[:, 6] = 1.0
    st[:, 7] = 1.0
    O = oracle_lib
    _, _, led, tr = O.transport(np.ones(n, np.uint8), st,
                                np.arange(n, dtype=np.uint64), 17, ph,
                                O.ophys(step=step), ledger=True, trace=True)
    d = tr[:, O.TR_EXIT:O.TR_EXIT + 3]
    assert np.isfinite(d).all()          # every electron left the box
    th = np.arccos(np.clip(d[:, 2], -1.0, 1.0))
    sp = np.hypot(d[:, 0], d[:, 1])
    ax = th * d[:, 0] / sp
    ay = th * d[:, 1] / sp
    th0 = oracle_lib.highland(T0, rho * step)
    for a in (ax, ay):
        # the standard error of a standard deviation is sd / sqrt(2 n)
        assert a.std() == pytest.approx(th0, rel=5 / math.sqrt(2 * n))
        assert abs(a.mean()) < 5 * th0 / math.sqrt(n)
    assert stats.kstest(ax[:20000] / th0, "norm").pvalue > 1e-4
    assert stats.kstest(th[:20000] / th0, "rayleigh").pvalue > 1e-4
    # the electron lost the CSDA energy of the slab and nothing after it
    lost = led[:, 1]
    S_mid = oracle_lib.stopping_power(T0 - 0.5 * lost.mean())
    assert lost.mean() == pytest.approx(S_mid * rho * step, rel=5e-3)


@pytest.mark.parametrize("E", [0.3, 1.0, 6.0])
def test_compton_recoil_electron_direction(oracle_lib, E):
    """Compton kinematics of the recoil electron the transport creates: its
    angle theta_e to the incident photon obeys
    cot(theta_e) = (1 + k) tan(theta / 2), k = E / m c^2, theta the photon's
    scattering angle; it leaves on the opposite side of the incident axis
    from the scattered photon (azimuths differ by pi); and the momentum
    E d0 - E' d' has the magnitude sqrt(T (T + 2 m c^2)) of an electron of
    kinetic energy T = E - E'."""
    O = oracle_lib
    ph = S.water_phantom((4, 4, 400), 1.0, (-2.0, -2.0, 100.0))
    _, _, _, tr = _pencil(O, E, 6000, ph, O.FLAG_FIRST_COLLISION)
    hit = ~np.isnan(tr[:, O.TR_COS])
    assert hit.sum() > 3000
    tr = tr[hit]
    k = tr[:, O.TR_E] / ME
    theta = np.arccos(np.clip(tr[:, O.TR_COS], -1.0, 1.0))
    cot_e = (1.0 + k) * np.tan(theta / 2.0)
    np.testing.assert_allclose(tr[:, O.TR_COSE],
                               cot_e / np.sqrt(1.0 + cot_e ** 2), atol=1e-7)
    side = tr[:, O.TR_SIDE]
    ok = np.abs(np.sin(theta)) > 1e-6
    np.testing.assert_allclose(side[ok], -1.0, atol=1e-9)
    np.testing.assert_allclose(tr[:, O.TR_PNORM], 1.0, rtol=1e-8)
    # energy of the first interaction: E' = E / (1 + k (1 - cos theta))
    np.testing.assert_allclose(
        tr[:, O.TR_T], tr[:, O.TR_E] - tr[:, O.TR_E] /
        (1.0 + k * (1.0 - tr[:, O.TR_COS])), rtol=1e-12, atol=1e-15)


# --------------------------------------------------------- ledger --------
def test_energy_conservation_per_history(oracle_lib):
    ph = S.heterogeneous_phantom((24, 24, 24), 0.5, (-6.0, -6.0, 100.0), 4)
    rng = np.random.default_rng(2)
    n = 3000
    st = np.zeros((n, 8))
    st[:, 0] = rng.uniform(0.05, 6.0, n)
    st[:, 1] = rng.uniform(-5, 5, n)
    st[:, 2] = rng.uniform(-5, 5, n)
    st[:, 3] = 100.0
    d = rng.normal(size=(n, 3))
    d[:, 2] = np.abs(d[:, 2]) + 0.5
    st[:, 4:7] = d / np.linalg.norm(d, axis=1)[:, None]
    st[:, 7] = 1.0
    types = (rng.random(n) < 0.3).astype(np.uint8)
    _, _, led, _ = oracle_lib.transport(types, st,
                                        np.arange(n, dtype=np.uint64), 9, ph,
                                        ledger=True)
    rel = np.abs(led[:, 1] + led[:, 2] + led[:, 3] - led[:, 0]) / led[:, 0]
    assert rel.max() < 1e-12
    assert (led[:, 2] > 0).any() and (led[:, 1] > 0).any()


# -------------------------------------------- first-collision dose -------
def test_first_collision_dose_closed_form(oracle_lib):
    """Broad parallel monoenergetic beam over the whole face of a water
    block, first collision only with local deposit: the expected energy in
    depth layer j is N E (sigma_tr / sigma) (exp(-mu z_j) - exp(-mu z_j+1)),
    and the dose follows from 1 MeV/g = 1.602176634e-10 Gy."""
    E = 1.25
    nx, nz, vox = 8, 20, 1.0
    ph = S.water_phantom((nx, nx, nz), vox, (-4.0, -4.0, 100.0))
    n = 200_000
    rng = np.random.default_rng(7)
    st = np.zeros((n, 8))
    st[:, 0] = E
    st[:, 1] = rng.uniform(-4, 4, n)
    st[:, 2] = rng.uniform(-4, 4, n)
    st[:, 3] = 100.0
    st[:, 6] = 1.0
    st[:, 7] = 1.0
    acc, _, _, _ = oracle_lib.transport(
        np.zeros(n, np.uint8), st, np.arange(n, dtype=np.uint64), 5, ph,
        oracle_lib.ophys(flags=oracle_lib.FLAG_FIRST_COLLISION))
    layer = acc.reshape(nz, nx, nx).sum((1, 2))
    mu = NE * oracle_lib.kn_sigma(E)
    tot = oracle_lib.kn_sigma(E)
    tr_frac = integrate.quad(
        lambda x: dsigma_dcos(E, x) *
        (1 - 1 / (1 + E / ME * (1 - x))), -1, 1)[0] / tot
    z = np.arange(nz + 1) * vox
    want = n * E * tr_frac * (np.exp(-mu * z[:-1]) - np.exp(-mu * z[1:]))
    # Poisson-like spread of the per-layer sums
    sd = np.sqrt(want * E)
    assert np.all(np.abs(layer - want) < 5 * sd)
    # dose normalisation of the finaliser: one batch, Gy per particle
    s1 = acc.copy()
    s2 = acc * acc
    dose, _ = oracle_lib.finalize(s1, s2, 1, ph, 1.0 / n)
    mass = 1.0 * vox ** 3
    np.testing.assert_allclose(
        dose, acc * 1.602176634e-10 / mass / n, rtol=1e-15)


# ------------------------------------- weights, densities, cut-offs ------
def test_deposits_carry_the_particle_weight(oracle_lib):
    """Every deposit is energy x weight: the weighted tally of a history is
    its weight times its (unweighted) deposited energy, for photons with
    their recoil electrons and for electrons alike."""
    ph = S.heterogeneous_phantom((16, 16, 16), 0.5, (-4.0, -4.0, 100.0), 6)
    rng = np.random.default_rng(11)
    n = 400
    st = np.zeros((n, 8))
    st[:, 0] = rng.uniform(0.3, 6.0, n)
    st[:, 1] = rng.uniform(-3, 3, n)
    st[:, 2] = rng.uniform(-3, 3, n)
    st[:, 3] = 100.0
    st[:, 6] = 1.0
    st[:, 7] = rng.uniform(0.1, 3.0, n)
    types = (np.arange(n) % 2).astype(np.uint8)
    hits = {0: 0, 1: 0}
    for i in range(0, n, 13):      # one history at a time
        acc, _, led, _ = oracle_lib.transport(
            types[i:i + 1], st[i:i + 1], np.array([i], np.uint64), 4, ph,
            ledger=True)
        assert acc.sum() == pytest.approx(st[i, 7] * led[0, 1], rel=1e-12)
        hits[int(types[i])] += led[0, 1] > 0
    assert hits[0] >= 3 and hits[1] >= 10   # photons may cross unscattered


@pytest.mark.parametrize("rho", [0.26, 1.85])
def test_attenuation_scales_with_density(oracle_lib, rho):
    """The interaction coefficient is rho n_e sigma_KN: in a uniform slab
    of density rho the first-interaction depths follow exp(-rho mu z)."""
    E = 1.25
    ph = S.water_phantom((4, 4, 60), 1.0, (-2.0, -2.0, 100.0))
    ph.density[:] = rho
    n = 30_000
    _, _, _, tr = _pencil(oracle_lib, E, n, ph,
                          oracle_lib.FLAG_FIRST_COLLISION)
    mu = rho * NE * oracle_lib.kn_sigma(E)
    d = tr[:, 0] - 100.0
    hit = ~np.isnan(d)
    p = 1 - math.exp(-mu * 60.0)
    assert abs(hit.mean() - p) < 4 * math.sqrt(p * (1 - p) / n)
    assert stats.kstest(d[hit], lambda z: (1 - np.exp(-mu * z)) / p
                        ).pvalue > 1e-3


def test_low_energy_photons_deposit_everything_in_a_large_medium(
        oracle_lib):
    """0.3 MeV photons (every recoil below the electron cut-off: the
    largest recoil energy is E 2k / (1 + 2k) = 0.16 MeV) started at the
    centre of a 4 m water cube: nothing escapes (the chance to cross 2 m is
    below 1e-8), so the recoils that stay under the cut-off and the photon
    that ends under its own cut-off deposit where they are, and the
    deposited energy is the photon's energy, history by history."""
    E = 0.3
    k = E / ME
    assert E * 2 * k / (1 + 2 * k) < TCUT
    ph = S.water_phantom((4, 4, 4), 100.0, (-200.0, -200.0, 0.0))
    n = 300
    rng = np.random.default_rng(12)
    st = np.zeros((n, 8))
    st[:, 0] = E
    st[:, 1:4] = [1e-3, 2e-3, 200.0]
    d = rng.normal(size=(n, 3))
    st[:, 4:7] = d / np.linalg.norm(d, axis=1)[:, None]
    st[:, 7] = 1.0
    acc, cnt, led, _ = oracle_lib.transport(
        np.zeros(n, np.uint8), st, np.arange(n, dtype=np.uint64), 8, ph,
        ledger=True)
    assert cnt[0] > 5 * n                  # several Compton events each
    np.testing.assert_allclose(led[:, 1], E, rtol=1e-12)
    assert np.all(led[:, 2] == 0.0) and np.all(led[:, 3] == 0.0)
    assert acc.sum() == pytest.approx(n * E, rel=1e-12)


def test_particle_on_the_far_face_enters_the_last_voxel(oracle_lib):
    """A point on the box surface belongs to the voxel inside: an electron
    started exactly on the far x face, moving inward with a range shorter
    than a voxel, deposits all its energy in the last voxel of its row."""
    ph = S.water_phantom((4, 4, 4), 1.0, (0.0, 0.0, 0.0))
    T = 0.5                                # CSDA range about 0.18 cm
    # inward across the face, and along it (parallel to the face: the
    # electron stays in the last voxel of the row)
    for d, vox in (((-1.0, 0.0, 0.0), (2, 1, 3)), ((0.0, -1.0, 0.0),
                                                   (2, 2, 3))):
        st = np.array([[T, 4.0, 2.5 if d[1] else 1.5, 2.5, *d, 1.0]])
        acc, _, led, _ = oracle_lib.transport(
            np.ones(1, np.uint8), st, np.zeros(1, np.uint64), 2, ph,
            oracle_lib.ophys(flags=oracle_lib.FLAG_NO_MSC), ledger=True)
        assert led[0, 1] == pytest.approx(T, rel=1e-12)
        assert led[0, 2] == 0.0
        assert acc.reshape(4, 4, 4)[vox] == pytest.approx(T, rel=1e-12)


def test_electron_energy_never_falls_below_the_cut_off_in_flight(
        oracle_lib):
    """CSDA steps end at the cut-off: along a straight track (no
    scattering) through 1 mm voxels, the energy lost in each voxel before
    the last equals T_in - T_out from the CSDA energy-range relation and
    the last voxel receives what is left, down from at least the cut-off;
    so every deposit but the last is below T0 - T_cut and their sum never
    exceeds it."""
    ph = S.water_phantom((4, 4, 60), 0.1, (-0.2, -0.2, 0.0))
    T0 = 2.0
    st = np.array([[T0, 1e-3, 2e-3, 0.0, 0.0, 0.0, 1.0, 1.0]])
    acc, _, led, _ = oracle_lib.transport(
        np.ones(1, np.uint8), st, np.zeros(1, np.uint64), 2, ph,
        oracle_lib.ophys(flags=oracle_lib.FLAG_NO_MSC), ledger=True)
    col = acc.reshape(60, 4, 4)[:, 2, 2]
    nz = np.nonzero(col)[0]
    last = nz[-1]
    assert col[:last].sum() <= T0 - TCUT + 1e-12
    # the residual range above the cut-off fixes the depth of the last
    # deposit: r(T0) - r(T_cut) of water, to the voxel
    r = oracle_lib.csda_range(TCUT, T0)
    assert last == int(r / 0.1)
    # and the final deposit is at least the cut-off energy
    assert col[last] >= TCUT - 1e-12
    assert led[0, 1] == pytest.approx(T0, rel=1e-12)
