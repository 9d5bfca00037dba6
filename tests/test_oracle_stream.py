"""Pins of the oracle's Method 1/2 source (Sec. 2.1, 2.2): the phase space
read in file order from a random start, the beam model (Method 2), and the
on-the-fly bins by type and energy, flushed when they reach their capacity
and at the end of the batch.  Checked against a pure-Python reading of the
rules with exact rationals, and against invariants any correct flush
sequence has."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import psl_synth as S


def _brute(field, geom, ps, e_edges, n_hist, batch, seed, cap, method,
           oracle):
    """The state machine as the paper states it, one particle at a time."""
    n = ps.n
    s0 = oracle.splitmix64(seed) % n
    n_e = len(e_edges) - 1
    bins = {b: [] for b in range(2 * n_e)}
    flushes, seq, status = [], [], []
    zp = Fr(geom["z_psl"])
    for r in range(n_hist):
        p = (s0 + batch * n_hist + r) % n
        t, E = int(ps.type[p]), float(ps.E[p])
        if t > 1 or math.isnan(E):
            status.append(4)
            continue
        x, y = Fr(float(ps.x[p])), Fr(float(ps.y[p]))
        u, v, w = (Fr(float(ps.u[p])), Fr(float(ps.v[p])),
                   Fr(float(ps.w[p])))
        st = 1
        if method == 2 and field.jaws:
            xj = x + u / w * (Fr(geom["z_x"]) - zp)
            yj = y + v / w * (Fr(geom["z_y"]) - zp)
            sx = Fr(geom["z_x"]) / Fr(geom["sad"])
            sy = Fr(geom["z_y"]) / Fr(geom["sad"])
            if not (Fr(field.X1) * sx <= xj <= Fr(field.X2) * sx and
                    Fr(field.Y1) * sy <= yj <= Fr(field.Y2) * sy):
                st = 0
        if st and method == 2 and field.fluence is not None:
            xs = x + u / w * (Fr(geom["sad"]) - zp)
            ys = y + v / w * (Fr(geom["sad"]) - zp)
            ix = math.floor((xs - Fr(field.f_x0)) / Fr(field.f_pix))
            iy = math.floor((ys - Fr(field.f_y0)) / Fr(field.f_pix))
            nfy, nfx = field.fluence.shape
            if not (0 <= ix < nfx and 0 <= iy < nfy and
                    field.fluence[iy, ix] > 0):
                st = 2
        status.append(st)
        if st != 1:
            continue
        e = 0
        for k in range(1, n_e):
            if E >= float(e_edges[k]):
                e = k
        b = t * n_e + e
        bins[b].append(r)
        if len(bins[b]) == cap:
            flushes.append((b, cap, r, len(seq)))
            seq += bins[b]
            bins[b] = []
    for b in range(2 * n_e):
        if bins[b]:
            flushes.append((b, len(bins[b]), -1, len(seq)))
            seq += bins[b]
    return status, flushes, seq


def _setup(oracle_lib, n=2500, seed=23):
    ps = S.phase_space(n, seed, 20.0, S.Z_PSL)
    # wide enough that no particle of the 40x40 cm aim misses it
    ph = S.water_phantom((16, 16, 16), 4.0, (-32.0, -32.0, 100.0))
    geom = oracle_lib.geometry(ph, z_psl=S.Z_PSL)
    return ps, geom


def _flush_list(out):
    return list(zip(out["flush_bin"].tolist(), out["flush_count"].tolist(),
                    out["flush_trigger"].tolist(),
                    out["flush_first"].tolist()))


@pytest.mark.parametrize("method,cap", [(2, 7), (2, 64), (1, 5), (2, 10**9)])
def test_stream_matches_brute_force(oracle_lib, method, cap):
    ps, geom = _setup(oracle_lib)
    fl = S.fluence_map(5)
    fl[::3, ::4] = 0.0
    field = S.Field(-6, 4, -3, 8, fluence=fl)
    e_edges = S.log_edges(0.1, 6.0, 5)
    for batch in (0, 2):
        got = oracle_lib.stream_sample(field, geom, ps, e_edges, 1777, batch,
                                       31, cap, method=method)
        st, flushes, seq = _brute(field, geom, ps, e_edges, 1777, batch, 31,
                                  cap, method, oracle_lib)
        assert got["status"].tolist() == st     # nothing misses the phantom
        assert _flush_list(got) == flushes
        assert got["seq"].tolist() == seq


def test_stream_flush_invariants(oracle_lib):
    """Every accepted history is flushed exactly once; a flush holds one
    bin's particles in arrival order; a full flush holds `cap` particles
    and ends with the one whose arrival filled the bin; full flushes come
    in the order of their triggers, then the partial ones by bin."""
    ps, geom = _setup(oracle_lib, n=4000, seed=29)
    field = S.square_field(10.0)
    e_edges = S.log_edges(0.1, 6.0, 8)
    cap = 23
    out = oracle_lib.stream_sample(field, geom, ps, e_edges, 5000, 1, 3, cap)
    acc = np.nonzero(out["status"] == 1)[0]
    seq = out["seq"]
    assert np.array_equal(np.sort(seq), acc)
    E = out["state"][:, 0]
    t = out["type"]
    n_e = len(e_edges) - 1
    prev_trig = -1
    partial = False
    last_bin = -1
    for b, c, trig, first in _flush_list(out):
        part = seq[first:first + c]
        assert np.all(np.diff(part) > 0)
        assert np.all(t[part] * n_e + np.clip(
            np.searchsorted(e_edges, E[part].astype(np.float32),
                            side="right") - 1, 0, n_e - 1) == b)
        if trig >= 0:
            assert not partial and c == cap and part[-1] == trig
            assert trig > prev_trig
            prev_trig = trig
        else:
            partial = True
            assert 0 < c < cap and b > last_bin
            last_bin = b
    # the bins left open at the end hold fewer than cap particles each
    assert sum(c for _, c, _, _ in _flush_list(out)) == len(acc)


def test_stream_reads_file_order_cyclically(oracle_lib):
    """Consecutive batches continue the file from the random start and wrap
    at its end: after B batches of H histories every particle has been read
    floor(BH/n) or ceil(BH/n) times, and batch b starts where b-1 ended."""
    ps, geom = _setup(oracle_lib, n=997, seed=31)
    field = S.square_field(30.0)
    e_edges = S.log_edges(0.1, 6.0, 4)
    H, B = 400, 6
    use = np.zeros(ps.n, np.int64)
    last = None
    for b in range(B):
        out = oracle_lib.stream_sample(field, geom, ps, e_edges, H, b, 9, 50)
        src = out["src"]
        if last is not None:
            assert src[0] == (last + 1) % ps.n
        last = src[-1]
        assert np.all(np.diff(src) % ps.n == 1)
        np.add.at(use, src, 1)
    assert use.sum() == B * H
    assert use.min() >= B * H // ps.n and use.max() <= -(-B * H // ps.n)
    assert out["src"][0] == (oracle_lib.splitmix64(9) % ps.n + 5 * H) % ps.n


def test_stream_drops_bad_particles_and_method1_ignores_the_jaws(oracle_lib):
    ps, geom = _setup(oracle_lib, n=600, seed=37)
    ps.type[5] = 2
    ps.E[7] = np.nan
    field = S.Field(-2, 2, -2, 2, fluence=S.fluence_map(2))
    e_edges = S.log_edges(0.1, 6.0, 4)
    s0 = oracle_lib.splitmix64(4) % ps.n
    r5, r7 = (5 - s0) % ps.n, (7 - s0) % ps.n
    m1 = oracle_lib.stream_sample(field, geom, ps, e_edges, ps.n, 0, 4, 30,
                                  method=1)
    m2 = oracle_lib.stream_sample(field, geom, ps, e_edges, ps.n, 0, 4, 30,
                                  method=2)
    for out in (m1, m2):
        assert out["status"][r5] == 4 and out["status"][r7] == 4
    # Method 1: a collimated phase space, every valid particle accepted
    assert np.all((m1["status"] == 1) | (m1["status"] == 4))
    assert np.sum(m2["status"] == 0) > 0.5 * ps.n
    # the accepted Method-2 particles carry the same state as in Method 1
    # up to the fluence weight
    both = (m2["status"] == 1)
    np.testing.assert_array_equal(m2["state"][both, :7],
                                  m1["state"][both, :7])
    assert np.all(m2["state"][both, 7] <= m1["state"][both, 7])


def test_stream_weight_and_state_geometry(oracle_lib):
    """w' = wt * fluence * g with g = n / n_hist (dose per phase-space
    particle), and the state is the particle rotated by the gantry about
    the isocentre and moved along its ray onto the phantom surface."""
    ps = S.phase_space(3000, 41, 20.0, S.Z_PSL)
    ph = S.water_phantom((32, 32, 32), 1.0, (-16.0, -16.0, 84.0))
    geom = oracle_lib.geometry(ph, z_psl=S.Z_PSL)
    for gdeg in (0.0, 77.0, 233.0):
        f = S.Field(-8, 8, -8, 8, gantry_deg=gdeg)
        out = oracle_lib.stream_sample(f, geom, ps, S.log_edges(0.1, 6, 4),
                                       2000, 0, 8, 100)
        ok = out["status"] == 1
        st, src = out["state"][ok], out["src"][ok]
        np.testing.assert_allclose(st[:, 7], ps.wt[src] * 3000 / 2000,
                                   rtol=1e-15)
        th = math.radians(gdeg)
        R = np.array([[math.cos(th), 0, math.sin(th)], [0, 1, 0],
                      [-math.sin(th), 0, math.cos(th)]])
        iso = np.array([0, 0, 100.0])
        p0 = np.stack([ps.x[src], ps.y[src], np.full(len(src), S.Z_PSL)],
                      1).astype(np.float64)
        d0 = np.stack([ps.u[src], ps.v[src], ps.w[src]], 1).astype(
            np.float64)
        p1 = (p0 - iso) @ R.T + iso
        d1 = d0 @ R.T
        np.testing.assert_allclose(st[:, 4:7], d1, atol=1e-12)
        dp = st[:, 1:4] - p1
        tt = (dp * d1).sum(1)
        assert np.all(tt >= -1e-9)
        np.testing.assert_allclose(dp, tt[:, None] * d1, atol=1e-9)


def test_stream_energy_on_an_edge_joins_the_upper_bin(oracle_lib):
    """Energy bins are closed below: a particle whose energy equals an
    interior edge e_k joins bin k (the largest k with E >= e_k)."""
    ps, geom = _setup(oracle_lib, n=800, seed=53)
    e_edges = S.log_edges(0.1, 6.0, 5)
    ps.E[:] = e_edges[1:5][np.arange(ps.n) % 4]
    out = oracle_lib.stream_sample(S.square_field(30.0), geom, ps, e_edges,
                                   ps.n, 0, 2, 10 ** 6, method=1)
    seq, E, t = out["seq"], out["state"][:, 0], out["type"]
    assert len(seq) == ps.n
    n_e = len(e_edges) - 1
    for b, c, _, first in _flush_list(out):
        part = seq[first:first + c]
        assert np.all(t[part] == b // n_e)
        assert np.all(E[part].astype(np.float32) == e_edges[b % n_e])
