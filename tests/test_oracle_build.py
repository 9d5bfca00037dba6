"""Pins of the oracle's PSL generation (Sec. 2.3.2): against a library
stable sort, brute force on tiny inputs with ties, and invariants."""
import numpy as np
import pytest

import psl_synth as S


def _keys_by_searchsorted(ps, grid):
    """Keys from numpy.searchsorted (an independent library route)."""
    def b(v, edges):
        k = np.searchsorted(edges, v, side="right") - 1
        k = np.where(v == edges[-1], len(edges) - 2, k)
        ok = (v >= edges[0]) & (v <= edges[-1])
        return k, ok
    e, oe = b(ps.E, grid.e_edges)
    ix, ox = b(ps.x, grid.x_edges)
    iy, oy = b(ps.y, grid.y_edges)
    ok = oe & ox & oy & (ps.type <= 1)
    key = ((ps.type.astype(np.int64) * grid.n_e + e) * grid.n_y + iy) \
        * grid.n_x + ix
    return np.where(ok, key, -1)


def _check_against_argsort(oracle, ps, grid):
    perm, off, nd = oracle.build_psl(ps, grid)
    key = _keys_by_searchsorted(ps, grid)
    keep = np.nonzero(key >= 0)[0]
    order = keep[np.argsort(key[keep], kind="stable")]
    assert nd == int((key < 0).sum())
    np.testing.assert_array_equal(perm, order)
    counts = np.bincount(key[keep], minlength=grid.n_keys)
    np.testing.assert_array_equal(np.diff(off), counts)
    assert off[0] == 0 and off[-1] == ps.n - nd
    return perm, off


def test_tiny_workload_matches_stable_argsort(oracle_lib):
    wl = S.workload_tiny()
    _check_against_argsort(oracle_lib, wl.phsp, wl.grid)


def test_clinical_grid_matches_stable_argsort(oracle_lib):
    ps = S.phase_space(200_000, 7, 20.0, S.Z_PSL)
    _check_against_argsort(oracle_lib, ps, S.clinical_grid())


def _brute(ps, grid):
    """Pure-Python reading of the definition for tiny inputs."""
    def b(v, edges):
        n = len(edges) - 1
        if not (edges[0] <= v <= edges[n]):
            return None
        for k in range(n - 1, -1, -1):
            if v >= edges[k]:
                return k
    buckets = {}
    dropped = 0
    for i in range(ps.n):
        t = int(ps.type[i])
        e, ix, iy = (b(ps.E[i], grid.e_edges), b(ps.x[i], grid.x_edges),
                     b(ps.y[i], grid.y_edges))
        if t > 1 or e is None or ix is None or iy is None:
            dropped += 1
            continue
        k = ((t * grid.n_e + e) * grid.n_y + iy) * grid.n_x + ix
        buckets.setdefault(k, []).append(i)
    perm = [i for k in sorted(buckets) for i in buckets[k]]
    return perm, dropped, buckets


def test_brute_force_with_ties_and_outliers(oracle_lib):
    f32 = np.float32
    grid = S.Grid(np.array([0.0, 1.0, 2.0, 4.0], f32),
                  np.array([-1.0, 0.0, 1.0], f32),
                  np.array([-1.0, 0.5, 1.0], f32), 25.0)
    E = np.array([0.0, 1.0, 4.0, 3.999, 2.0, 4.0001, np.nan, 0.5, 1.0, 1.5,
                  -0.1, 2.0], f32)
    x = np.array([-1.0, 0.0, 1.0, 0.999, 0.0, 0.0, 0.0, np.nan, 1.0001,
                  -0.5, 0.0, 0.0], f32)
    y = np.array([-1.0, 0.5, 1.0, 0.5, 0.4999, 0.0, 0.0, 0.0, 0.0, 0.9,
                  0.0, 0.5], f32)
    t = np.array([0, 1, 0, 1, 1, 0, 0, 0, 0, 2, 0, 1], np.uint8)
    one = np.ones(len(E), f32)
    ps = S.PhaseSpace(t, E, x, y, one * 0, one * 0, one, one, 25.0)
    perm, off, nd = oracle_lib.build_psl(ps, grid)
    bperm, bdrop, buckets = _brute(ps, grid)
    assert nd == bdrop == 6
    assert list(perm) == bperm
    for k, members in buckets.items():
        assert off[k + 1] - off[k] == len(members)


def test_invariants_random(oracle_lib):
    rng = np.random.default_rng(3)
    for trial in range(5):
        n = int(rng.integers(0, 3000))
        ps = S.phase_space(n, 100 + trial, 20.0, S.Z_PSL) if n else \
            S.phase_space(0, 1, 20.0, S.Z_PSL)
        grid = S.clinical_grid()
        perm, off, nd = oracle_lib.build_psl(ps, grid)
        assert len(perm) == n - nd
        assert len(np.unique(perm)) == len(perm)           # permutation
        assert np.all(np.diff(off) >= 0)
        for k in np.nonzero(np.diff(off))[0][:50]:
            members = perm[off[k]:off[k + 1]]
            assert np.all(np.diff(members) > 0)               # stable
            t, rest = divmod(k, grid.n_e * grid.n_x * grid.n_y)
            e, rest = divmod(rest, grid.n_x * grid.n_y)
            iy, ix = divmod(rest, grid.n_x)
            assert np.all(ps.type[members] == t)
            for v, edges, j in ((ps.E, grid.e_edges, e),
                                (ps.x, grid.x_edges, ix),
                                (ps.y, grid.y_edges, iy)):
                vv = v[members]
                assert np.all(vv >= edges[j])
                last = j == len(edges) - 2
                assert np.all(vv <= edges[j + 1]) if last else \
                    np.all(vv < edges[j + 1])


def test_empty(oracle_lib):
    ps = S.phase_space(0, 1, 20.0, S.Z_PSL)
    perm, off, nd = oracle_lib.build_psl(ps, S.clinical_grid())
    assert len(perm) == 0 and nd == 0 and np.all(off == 0)
