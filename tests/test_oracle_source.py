"""Pins of the oracle's PSL source: ROI selection (Sec. 2.3.3, Fig. 1),
allocation (Eq. 1-4) and sampling (Sec. 2.2, 2.3.3, 2.4), against exact
rational arithmetic, integer closed forms and brute force."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import psl_synth as S


# ---------------------------------------------------------------- ROI -----
def _roi_exact(lo, hi, zj, sad, zp):
    lo, hi, zj, sad, zp = map(Fr, (lo, hi, zj, sad, zp))
    c = (lo + hi) / 2
    f = (sad - zp) / (sad - zj)
    return c + (lo * zj / sad - c) * f, c + (hi * zj / sad - c) * f


def test_roi_worked_example(oracle_lib):
    # symmetric 10x10 cm field: the X jaw edge sits at 5 * 37/100 = 1.85 cm,
    # the back-projection from the isocentre through it reaches the PSL
    # plane at 1.85 * 75/63 = 2.2023809... cm
    lo, hi = oracle_lib.roi(-5.0, 5.0, 37.0, 100.0, 25.0)
    assert hi == pytest.approx(1.85 * 75.0 / 63.0, rel=1e-15)
    assert lo == pytest.approx(-1.85 * 75.0 / 63.0, rel=1e-15)
    # an off-centre field: centre at 4 cm, edges 2 and 6 at SAD
    lo, hi = oracle_lib.roi(2.0, 6.0, 28.0, 100.0, 25.0)
    elo, ehi = _roi_exact(2.0, 6.0, 28.0, 100.0, 25.0)
    assert lo == pytest.approx(float(elo), abs=1e-13)
    assert hi == pytest.approx(float(ehi), abs=1e-13)
    # centre 4 + (0.56 - 4) * 75/72 = 0.41666..., 4 + (1.68 - 4) * 75/72
    assert float(elo) == pytest.approx(4 + (0.56 - 4) * 75 / 72, abs=1e-12)


def test_cull_matches_exact_overlap(oracle_lib):
    rng = np.random.default_rng(5)
    grid = S.clinical_grid()
    geom = {"sad": 100.0, "z_x": 37.0, "z_y": 28.0}
    fields = []
    for i in range(40):
        X1, X2, Y1, Y2 = S.random_jaws(500 + i)
        fields.append(S.Field(X1, X2, Y1, Y2))
    fields.append(S.square_field(4.0))
    fields.append(S.square_field(30.0))
    mask = oracle_lib.cull(fields, grid, True, geom)
    for fi, f in enumerate(fields):
        xlo, xhi = _roi_exact(f.X1, f.X2, 37.0, 100.0, grid.z_plane)
        ylo, yhi = _roi_exact(f.Y1, f.Y2, 28.0, 100.0, grid.z_plane)
        for iy in range(grid.n_y):
            for ix in range(grid.n_x):
                ex = (Fr(float(grid.x_edges[ix])) < xhi and
                      Fr(float(grid.x_edges[ix + 1])) > xlo and
                      Fr(float(grid.y_edges[iy])) < yhi and
                      Fr(float(grid.y_edges[iy + 1])) > ylo)
                assert mask[fi, iy * grid.n_x + ix] == int(ex), (fi, ix, iy)
    # no cull / no jaws keep everything
    assert oracle_lib.cull(fields[:2], grid, False, geom).all()
    nj = S.Field(-1, 1, -1, 1, jaws=False)
    assert oracle_lib.cull([nj], grid, True, geom).all()


def test_cull_is_lossless_for_point_source(oracle_lib):
    """With a point source (sigma 0) every particle that passes the jaws
    lies in a selected position bin."""
    ps = S.phase_space(200_000, 9, 20.0, S.Z_PSL, sigma_src=0.0)
    grid = S.clinical_grid()
    ph = S.water_phantom((16, 16, 16), 2.0, (-16.0, -16.0, 100.0))
    geom = oracle_lib.geometry(ph)
    perm, off, _ = oracle_lib.build_psl(ps, grid)
    sps = ps.subset(perm)
    for f in [S.square_field(4.0), S.Field(-3.0, 7.0, -12.0, 1.0),
              S.square_field(30.0)]:
        mask_all = oracle_lib.cull([f], grid, False, geom)
        N, g, _ = oracle_lib.alloc([f], 0, int(off[-1]), off, mask_all, grid)
        # one history per particle: every particle read exactly once
        assert np.all(N[0] == np.diff(off))
        smp = oracle_lib.sample([f], geom, off, N, g, 0, 1, sps)
        acc = smp["status"] != 0
        mask = oracle_lib.cull([f], grid, True, geom)[0]
        pos = smp["key"] % (grid.n_x * grid.n_y)
        assert acc.sum() > 0
        assert np.all(mask[pos[acc]] == 1)


# -------------------------------------------------------------- alloc -----
def _alloc_exact(fields, mode, n_sim, offsets, mask, grid):
    n_keys = grid.n_keys
    npos = grid.n_x * grid.n_y
    nk = [int(offsets[k + 1] - offsets[k]) for k in range(n_keys)]
    C = [sum(nk[k] for k in range(n_keys) if mask[f][k % npos])
         for f in range(len(fields))]
    if mode == 0:
        ideal = [Fr(n_sim * sum(C[:i + 1]), sum(C)) for i in range(len(C))]
    else:
        # MU prefix in double, as the reading states
        m, pre = 0.0, []
        tot = sum(f.MU for f in fields)
        for f in fields:
            m += f.MU
            pre.append(math.floor(float(n_sim) * m / tot))
        ideal = pre
    F = [math.floor(v) for v in ideal]
    F[-1] = n_sim
    NF = [F[0]] + [F[i] - F[i - 1] for i in range(1, len(F))]
    N = np.zeros((len(fields), n_keys), np.int64)
    for f in range(len(fields)):
        S_, prev = 0, 0
        for k in range(n_keys):
            if not mask[f][k % npos] or C[f] == 0:
                continue
            S_ += nk[k]
            Fk = (NF[f] * S_) // C[f]
            N[f, k] = Fk - prev
            prev = Fk
    return N, NF, C


@pytest.mark.parametrize("mode", [0, 1])
def test_alloc_matches_integer_closed_form(oracle_lib, mode):
    ps = S.phase_space(100_000, 11, 20.0, S.Z_PSL)
    grid = S.clinical_grid()
    geom = {"sad": 100.0, "z_x": 37.0, "z_y": 28.0}
    _, off, _ = oracle_lib.build_psl(ps, grid)
    fields = [S.square_field(4.0, MU=17.5), S.square_field(10.0, MU=3.25),
              S.Field(-2, 9, -7, 1, MU=60.0)]
    mask = oracle_lib.cull(fields, grid, True, geom)
    n_sim = 1_234_567
    N, g, NF = oracle_lib.alloc(fields, mode, n_sim, off, mask, grid)
    eN, eNF, C = _alloc_exact(fields, mode, n_sim, off, mask, grid)
    np.testing.assert_array_equal(N, eN)
    np.testing.assert_array_equal(NF, eNF)
    assert N.sum() == n_sim
    for f in range(len(fields)):
        assert N[f].sum() == NF[f]
        nk = np.diff(off)
        sel = N[f] > 0
        ideal = NF[f] * nk / C[f]
        assert np.all(N[f][sel] >= np.floor(ideal[sel]))
        assert np.all(N[f][sel] <= np.ceil(ideal[sel]))
        # unbiasedness identity: sum over histories of g equals
        # (MU_f / MU_tot) times the selected population
        mu = fields[f].MU / sum(x.MU for x in fields)
        assert (N[f] * g[f]).sum() == pytest.approx(mu * C[f], rel=1e-12)


# ------------------------------------------------------------- sample -----
def test_splitmix64_published_sequence(oracle_lib):
    # the generator's reference output for seed 1234567 (Vigna's
    # splitmix64.c), as successive states seed + k * golden gamma
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    s = 1234567
    for w in want:
        assert oracle_lib.splitmix64(s) == w
        s = (s + 0x9E3779B97F4A7C15) % 2**64


def _sample_brute(fields, geom, off, N, g, batch, seed, ps, oracle):
    """Pure-Python reading of the sampling rules, exact rationals for the
    jaw and fluence decisions."""
    F, n_keys = N.shape
    out = []
    for f, fd in enumerate(fields):
        for k in range(n_keys):
            if N[f, k] == 0:
                continue
            nk = int(off[k + 1] - off[k])
            Tk = int(N[:, k].sum())
            before = int(N[:f, k].sum())
            sk = oracle.splitmix64(seed ^ k) % nk
            c = batch * Tk + before
            for r in range(int(N[f, k])):
                p = int(off[k]) + (sk + c + r) % nk
                x, y = Fr(float(ps.x[p])), Fr(float(ps.y[p]))
                u, v, w = (Fr(float(ps.u[p])), Fr(float(ps.v[p])),
                           Fr(float(ps.w[p])))
                zp = Fr(geom["z_psl"])
                st = 1
                if fd.jaws:
                    xj = x + u / w * (Fr(geom["z_x"]) - zp)
                    yj = y + v / w * (Fr(geom["z_y"]) - zp)
                    sx = Fr(geom["z_x"]) / Fr(geom["sad"])
                    sy = Fr(geom["z_y"]) / Fr(geom["sad"])
                    if not (Fr(fd.X1) * sx <= xj <= Fr(fd.X2) * sx and
                            Fr(fd.Y1) * sy <= yj <= Fr(fd.Y2) * sy):
                        st = 0
                if st and fd.fluence is not None:
                    xs = x + u / w * (Fr(geom["sad"]) - zp)
                    ys = y + v / w * (Fr(geom["sad"]) - zp)
                    ix = math.floor((xs - Fr(fd.f_x0)) / Fr(fd.f_pix))
                    iy = math.floor((ys - Fr(fd.f_y0)) / Fr(fd.f_pix))
                    nfy, nfx = fd.fluence.shape
                    if 0 <= ix < nfx and 0 <= iy < nfy and \
                            fd.fluence[iy, ix] > 0:
                        pass
                    else:
                        st = 2
                out.append((p, f, st))
    return out


def test_sample_matches_brute_force(oracle_lib):
    ps = S.phase_space(3000, 13, 20.0, S.Z_PSL)
    grid = S.Grid(S.log_edges(0.1, 6.0, 4), S.linear_edges(-5.5, 5.5, 4),
                  S.linear_edges(-5.5, 5.5, 4), S.Z_PSL)
    ph = S.water_phantom((16, 16, 16), 2.0, (-16.0, -16.0, 100.0))
    geom = oracle_lib.geometry(ph)
    perm, off, _ = oracle_lib.build_psl(ps, grid)
    sps = ps.subset(perm)
    fl = S.fluence_map(3)
    fl[::3, ::4] = 0.0
    fields = [S.Field(-4, 6, -8, 3, MU=2.0, fluence=fl),
              S.Field(-10, 10, -10, 10, MU=1.0)]
    mask = oracle_lib.cull(fields, grid, True, geom)
    N, g, _ = oracle_lib.alloc(fields, 1, 7001, off, mask, grid)
    for batch in (0, 3):
        smp = oracle_lib.sample(fields, geom, off, N, g, batch, 77, sps)
        want = _sample_brute(fields, geom, off, N, g, batch, 77, sps,
                             oracle_lib)
        got = list(zip(smp["src"].tolist(), smp["field"].tolist(),
                       [0 if s == 0 else (2 if s == 2 else 1)
                        for s in smp["status"].tolist()]))
        assert got == want
        # the phantom sits under the whole field: nothing misses
        assert not np.any(smp["status"] == 3)


def test_cyclic_usage_counts(oracle_lib):
    """Over consecutive batches each PSL is read cyclically from its random
    start, so after T histories from a PSL of n particles every particle has
    been used floor(T/n) or ceil(T/n) times."""
    ps = S.phase_space(5000, 17, 20.0, S.Z_PSL)
    grid = S.Grid(S.log_edges(0.1, 6.0, 3), S.linear_edges(-5.5, 5.5, 3),
                  S.linear_edges(-5.5, 5.5, 3), S.Z_PSL)
    ph = S.water_phantom((16, 16, 16), 2.0, (-16.0, -16.0, 100.0))
    geom = oracle_lib.geometry(ph)
    perm, off, _ = oracle_lib.build_psl(ps, grid)
    sps = ps.subset(perm)
    fields = [S.square_field(10.0, MU=1.0), S.square_field(6.0, MU=2.0)]
    mask = oracle_lib.cull(fields, grid, True, geom)
    N, g, _ = oracle_lib.alloc(fields, 1, 12_345, off, mask, grid)
    use = np.zeros(off[-1], np.int64)
    B = 4
    for b in range(B):
        smp = oracle_lib.sample(fields, geom, off, N, g, b, 5, sps)
        np.add.at(use, smp["src"], 1)
    for k in range(grid.n_keys):
        nk = off[k + 1] - off[k]
        T = B * N[:, k].sum()
        if nk == 0 or T == 0:
            continue
        u = use[off[k]:off[k + 1]]
        assert u.sum() == T
        assert u.min() >= T // nk and u.max() <= -(-T // nk)


def test_sample_state_rotation_and_projection(oracle_lib):
    """Gantry rotation about the isocentre and the move to the phantom
    surface, checked against an independent construction: the rotated
    particle lies on the rotated ray and on the box surface."""
    ps = S.phase_space(4000, 19, 20.0, S.Z_PSL)
    grid = S.clinical_grid()
    ph = S.water_phantom((32, 32, 32), 1.0, (-16.0, -16.0, 84.0))
    geom = oracle_lib.geometry(ph)
    perm, off, _ = oracle_lib.build_psl(ps, grid)
    sps = ps.subset(perm)
    for gdeg in (0.0, 51.43, 180.0, 300.0):
        f = S.Field(-8, 8, -8, 8, gantry_deg=gdeg)
        mask = oracle_lib.cull([f], grid, True, geom)
        N, g, _ = oracle_lib.alloc([f], 0, 3000, off, mask, grid)
        smp = oracle_lib.sample([f], geom, off, N, g, 0, 3, sps)
        ok = smp["status"] == 1
        st = smp["state"][ok]
        src = smp["src"][ok]
        th = math.radians(gdeg)
        R = np.array([[math.cos(th), 0, math.sin(th)], [0, 1, 0],
                      [-math.sin(th), 0, math.cos(th)]])
        iso = np.array([0, 0, 100.0])
        p0 = np.stack([sps.x[src], sps.y[src],
                       np.full(len(src), 25.0)], 1).astype(np.float64)
        d0 = np.stack([sps.u[src], sps.v[src], sps.w[src]], 1).astype(
            np.float64)
        p1 = (p0 - iso) @ R.T + iso
        d1 = d0 @ R.T
        np.testing.assert_allclose(st[:, 4:7], d1, atol=1e-12)
        # on the ray: (p - p1) parallel to d1 and forward
        dp = st[:, 1:4] - p1
        t = (dp * d1).sum(1)
        assert np.all(t >= -1e-9)
        np.testing.assert_allclose(dp, t[:, None] * d1, atol=1e-9)
        # on the box surface
        lo, hi = np.array(geom["box_lo"]), np.array(geom["box_hi"])
        on = np.isclose(st[:, 1:4], lo, atol=1e-9) | \
            np.isclose(st[:, 1:4], hi, atol=1e-9)
        assert np.all(on.any(1))
        assert np.all(st[:, 1:4] >= lo - 1e-9) and \
            np.all(st[:, 1:4] <= hi + 1e-9)
        # weight: g of the PSL, unit fluence and phase-space weight
        key = smp["key"][ok]
        np.testing.assert_allclose(st[:, 7], g[0, key], rtol=1e-15)


def test_sample_collimator_and_couch_rotations(oracle_lib):
    """Collimator, gantry and couch (Sec. 2.3.3: each particle receives the
    three rotations of its field), checked against rotation matrices built
    here: the phase space turns with the collimator about the central axis
    (so the jaw test is unchanged), then the gantry turns it about +y and
    the couch turns the patient by +angle about the vertical through the
    isocentre (the beam by -angle): p' = iso + Rz(-t) Ry(g) Rz(c) (p - iso).
    The particle lies on the turned ray and on the phantom surface; with all
    three angles zero the state is the unturned one bit for bit."""
    ps = S.phase_space(4000, 43, 20.0, S.Z_PSL)
    grid = S.clinical_grid()
    ph = S.water_phantom((32, 32, 32), 1.0, (-16.0, -16.0, 84.0))
    geom = oracle_lib.geometry(ph)
    perm, off, _ = oracle_lib.build_psl(ps, grid)
    sps = ps.subset(perm)

    def rz(a):
        c, s = math.cos(a), math.sin(a)
        return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])

    def ry(a):
        c, s = math.cos(a), math.sin(a)
        return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])

    base = None
    for gdeg, cdeg, tdeg in ((0, 0, 0), (0, 30, 0), (0, 0, 90), (45, 15, 270),
                             (200, 330, 10)):
        f = S.Field(-6, 7, -5, 8, gantry_deg=gdeg, collimator_deg=cdeg,
                    couch_deg=tdeg)
        mask = oracle_lib.cull([f], grid, True, geom)
        N, g, _ = oracle_lib.alloc([f], 0, 3000, off, mask, grid)
        smp = oracle_lib.sample([f], geom, off, N, g, 0, 3, sps)
        if base is None:
            base = smp
        # the jaw test is in the phase space's own frame: same decisions
        np.testing.assert_array_equal(smp["status"] == 0,
                                      base["status"] == 0)
        ok = smp["status"] == 1
        st, src = smp["state"][ok], smp["src"][ok]
        R = rz(-math.radians(tdeg)) @ ry(math.radians(gdeg)) @ \
            rz(math.radians(cdeg))
        iso = np.array([0, 0, 100.0])
        p0 = np.stack([sps.x[src], sps.y[src],
                       np.full(len(src), 25.0)], 1).astype(np.float64)
        d0 = np.stack([sps.u[src], sps.v[src], sps.w[src]], 1).astype(
            np.float64)
        p1 = (p0 - iso) @ R.T + iso
        d1 = d0 @ R.T
        np.testing.assert_allclose(st[:, 4:7], d1, atol=1e-12)
        dp = st[:, 1:4] - p1
        t = (dp * d1).sum(1)
        assert np.all(t >= -1e-9)
        np.testing.assert_allclose(dp, t[:, None] * d1, atol=1e-9)
        lo, hi = np.array(geom["box_lo"]), np.array(geom["box_hi"])
        on = np.isclose(st[:, 1:4], lo, atol=1e-9) | \
            np.isclose(st[:, 1:4], hi, atol=1e-9)
        assert np.all(on.any(1))
    # couch 90 at gantry 0 turns the beam about its own axis: the state is
    # the unturned particle turned by -90 degrees about z through the
    # isocentre, exactly on the beam's entry plane
    f0 = S.Field(-6, 7, -5, 8)
    f1 = S.Field(-6, 7, -5, 8, couch_deg=90.0)
    m = oracle_lib.cull([f0], grid, True, geom)
    N, g, _ = oracle_lib.alloc([f0], 0, 3000, off, m, grid)
    a = oracle_lib.sample([f0], geom, off, N, g, 1, 3, sps)
    b = oracle_lib.sample([f1], geom, off, N, g, 1, 3, sps)
    ok = (a["status"] == 1) & (b["status"] == 1)
    np.testing.assert_allclose(b["state"][ok, 1], a["state"][ok, 2],
                               atol=1e-9)
    np.testing.assert_allclose(b["state"][ok, 2], -a["state"][ok, 1],
                               atol=1e-9)


# ------------------------------------------------ boundary readings ------
def test_cull_excludes_bins_that_only_touch_the_roi(oracle_lib):
    """A position bin is kept when it overlaps the ROI with positive area:
    with the PSL plane at the jaw plane (magnification 1) a symmetric 6 cm
    field has its ROI at exactly +-1.5 cm, and the bins [1.5, 2] and
    [-2, -1.5] that only touch it are culled."""
    edges = np.arange(-2.0, 2.01, 0.5).astype(np.float32)
    grid = S.Grid(S.log_edges(0.1, 6.0, 4), edges, edges, 50.0)
    geom = {"sad": 100.0, "z_x": 50.0, "z_y": 50.0}
    lo, hi = oracle_lib.roi(-3.0, 3.0, 50.0, 100.0, 50.0)
    assert (lo, hi) == (-1.5, 1.5)
    m = oracle_lib.cull([S.Field(-3, 3, -3, 3)], grid, True, geom)
    m = m.reshape(grid.n_y, grid.n_x)
    inner = np.array([0, 1, 1, 1, 1, 1, 1, 0], np.uint8)
    np.testing.assert_array_equal(m, np.outer(inner, inner))


def _edge_setup(oracle_lib, xs, ys, gantry=0.0, origin_z=100.0):
    from gpu_util import phase_space_arrays
    n = len(xs)
    one = np.ones(n)
    ps = phase_space_arrays(np.zeros(n), one, xs, ys, 0 * one, 0 * one, one,
                            50.0)
    ph = S.water_phantom((16, 16, 16), 1.0, (-8.0, -8.0, origin_z))
    geom = oracle_lib.geometry(ph, z_x=50.0, z_y=50.0, z_psl=50.0)
    return ps, geom


def test_jaw_edges_are_closed(oracle_lib):
    """The jaws are perfect collimators whose edges belong to the opening:
    a particle travelling along the beam axis exactly through the jaw
    edge (here at +-1.5 cm: 3 cm at SAD x 50/100) passes, the next float
    outside it is stopped."""
    e = np.float32(1.5)
    out = np.nextafter(e, np.float32(2.0))
    xs = [-e, e, 0.0, 0.0, -out, out, 0.0, 0.0]
    ys = [0.0, 0.0, -e, e, 0.0, 0.0, -out, out]
    ps, geom = _edge_setup(oracle_lib, xs, ys)
    f = S.Field(-3, 3, -3, 3)
    r = oracle_lib.stream_sample(f, geom, ps, S.log_edges(0.1, 6.0, 2),
                                 len(xs), 0, 0, 100, method=2)
    src = r["src"]
    status = dict(zip(src.tolist(), r["status"].tolist()))
    assert [status[i] for i in range(8)] == [1, 1, 1, 1, 0, 0, 0, 0]


def test_particle_starting_inside_the_phantom_is_not_moved(oracle_lib):
    """The move to the phantom is along the ray only when the particle
    starts outside: one already inside the box (here the PSL plane at
    z = 50 inside a box from z = 40) keeps its position."""
    xs = [0.25, -1.0, 2.5]
    ys = [0.5, 1.0, -3.0]
    ps, geom = _edge_setup(oracle_lib, xs, ys, origin_z=40.0)
    f = S.Field(-10, 10, -10, 10)
    r = oracle_lib.stream_sample(f, geom, ps, S.log_edges(0.1, 6.0, 2), 3,
                                 0, 0, 100, method=2)
    assert np.all(r["status"] == 1)
    st, src = r["state"], r["src"]
    np.testing.assert_array_equal(st[:, 1], np.float32(xs)[src])
    np.testing.assert_array_equal(st[:, 2], np.float32(ys)[src])
    np.testing.assert_array_equal(st[:, 3], 50.0)


def test_fluence_value_multiplies_the_weight(oracle_lib):
    """w' = wt x fluence x g (Sec. 2.4 with Eq. 4): with a map of
    non-uniform values the accepted weight is the product with the value
    of the pixel the ray crosses at the SAD plane (nearest pixel, found by
    exact arithmetic here)."""
    ps = S.phase_space(3000, 77, 20.0, S.Z_PSL)
    rng = np.random.default_rng(3)
    ps.wt[:] = rng.uniform(0.5, 2.0, ps.n).astype(np.float32)
    ph = S.water_phantom((16, 16, 16), 4.0, (-32.0, -32.0, 100.0))
    geom = oracle_lib.geometry(ph, z_psl=S.Z_PSL)
    fl = rng.uniform(0.05, 1.0, (20, 20)).astype(np.float32)
    f = S.Field(-10, 10, -10, 10, fluence=fl)
    r = oracle_lib.stream_sample(f, geom, ps, S.log_edges(0.1, 6.0, 2),
                                 2000, 0, 5, 100, method=2)
    ok = r["status"] == 1
    assert ok.sum() > 80
    zp, sad = Fr(S.Z_PSL), Fr(100.0)
    g = ps.n / 2000
    for st, p in zip(r["state"][ok], r["src"][ok]):
        xs = Fr(float(ps.x[p])) + Fr(float(ps.u[p])) / Fr(float(ps.w[p])) \
            * (sad - zp)
        ys = Fr(float(ps.y[p])) + Fr(float(ps.v[p])) / Fr(float(ps.w[p])) \
            * (sad - zp)
        ix = math.floor((xs - Fr(f.f_x0)) / Fr(f.f_pix))
        iy = math.floor((ys - Fr(f.f_y0)) / Fr(f.f_pix))
        want = float(ps.wt[p]) * float(fl[iy, ix]) * g
        assert st[7] == want
