"""Azimuthal particle redistribution in the PSL build (Sec. 2.3.1): the GPU
build of the redistributed copies is bit-exact against the oracle's
expansion followed by its PSL build, the dose of a redistributed phase
space agrees with the oracle's, and the redistribution lowers the latent
variance of a small cylindrically symmetric phase space."""
import sys

import numpy as np
import pytest

import oracle
import psl_synth as S
from gpu_util import phase_space_arrays

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gpu_build_apr(ps, grid, k, seed):
    import ctypes as C
    import torch
    import paper_1302_1861_amd as P
    g = P.make_grid(grid.e_edges, grid.x_edges, grid.y_edges, grid.z_plane)
    raw = P.Buffers.phsp_from_numpy(ps, "cuda")
    out = P.Buffers.phsp(ps.n * k, "cuda")
    off = torch.zeros(grid.n_keys + 1, dtype=torch.int64, device="cuda")
    nd = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    ws = torch.empty(max(P.lib().psl_build_apr_workspace_bytes(
        ps.n, k, C.byref(g)), 256), dtype=torch.uint8, device="cuda")
    P.psl_build_apr(raw, g, k, seed, out, off, nd, ws)
    torch.cuda.synchronize()
    off = off.cpu().numpy()
    kept = int(off[-1])
    return {k2: v[:kept].cpu().numpy() for k2, v in out.items()}, off, \
        int(nd.item())


@pytest.mark.parametrize("n,k,grid", [(100_003, 1, "clinical"),
                                      (60_000, 7, "clinical"),
                                      (3000, 64, "tiny"), (1, 3, "clinical")])
def test_apr_build_matches_oracle(n, k, grid):
    ps = S.phase_space(n, 71 + k, 20.0, S.Z_PSL, aim="disk")
    g = S.clinical_grid() if grid == "clinical" else S.Grid(
        S.linear_edges(0.0, 6.5, 3), S.linear_edges(-5.5, 5.5, 5),
        S.linear_edges(-5.5, 5.5, 5), S.Z_PSL)
    _say("apr build n=%d k=%d grid=%s" % (n, k, grid))
    ex = oracle.apr_expand(ps, k, 1234)
    perm, off, nd = oracle.build_psl(ex, g)
    got, goff, gnd = _gpu_build_apr(ps, g, k, 1234)
    assert gnd == nd
    np.testing.assert_array_equal(goff, off)
    for c in ("type", "E", "x", "y", "u", "v", "w", "wt"):
        assert got[c].tobytes() == getattr(ex, c)[perm].tobytes(), c


def test_apr_dose_matches_oracle():
    """The dose of the redistributed phase space (4 copies) against the
    oracle's on the same copies, z-scores above the 10% isodose."""
    import torch
    import paper_1302_1861_amd as P
    from oracle import analysis
    ps = S.phase_space(200_000, 81, 20.0, S.Z_PSL, aim="disk")
    wl = S.workload_clinical(side=10.0, n_particles=10)
    wl.phsp = ps
    wl.phantom = S.water_phantom((40, 40, 40), 0.8, (-16.0, -16.0, 100.0))
    eng = P.Engine(wl, histories_per_batch=50_000, apr_copies=4,
                   apr_seed=5)
    for b in range(40):
        eng.step(b)
    d_g, s_g = eng.finalize()
    torch.cuda.synchronize()
    wl_o = S.workload_clinical(side=10.0, n_particles=10)
    wl_o.phsp = oracle.apr_expand(ps, 4, 5)
    wl_o.phantom = wl.phantom
    d_o, s_o, _ = oracle.run_dose(wl_o, histories=2_000_000, batches=40)
    # the oracle's dose is per expanded particle: per original particle it
    # is 4 times that (each copy carries a quarter of the weight, and the
    # normalisation counts the original phase space)
    d_o, s_o = 4.0 * d_o, 4.0 * s_o
    d_g = d_g.cpu().numpy().astype(np.float64)
    s_g = s_g.cpu().numpy().astype(np.float64)
    z = analysis.zscore_stats(d_g, s_g, d_o, s_o,
                              ref_for_threshold=0.5 * (d_g + d_o))
    _say("apr dose z", z)
    assert z["frac_le3"] >= 0.99 and abs(z["mean"]) < 0.1
    assert 0.9 <= z["sd"] <= 1.1


def _latent(P, torch, seeds, k, hist, n, batches=10):
    """Per-voxel doses of independent phase spaces of n particles (one run
    of `hist` histories each) and their batch standard errors."""
    d_all, s_all = [], []
    for s in seeds:
        ps = S.phase_space(n, 500 + s, 10.0, S.Z_PSL, aim="disk")
        wl = S.workload_clinical(side=10.0, n_particles=10)
        wl.phsp = ps
        wl.phantom = S.water_phantom((32, 32, 32), 1.0,
                                     (-16.0, -16.0, 100.0))
        eng = P.Engine(wl, histories_per_batch=hist // batches,
                       apr_copies=k, apr_seed=900 + s)
        d, sg = eng.run(batches=batches)
        torch.cuda.synchronize()
        d_all.append(d.cpu().numpy().astype(np.float64))
        s_all.append(sg.cpu().numpy().astype(np.float64))
        del eng
    return np.array(d_all), np.array(s_all)


def test_apr_lowers_latent_variance():
    """A 20000-particle cylindrically symmetric phase space recycled 100
    times: across 16 independent phase spaces a voxel's dose varies far
    more than its batch standard error says (latent variance, Sec. 2.3.1);
    16 redistributed copies per particle at the same history count cut that
    spread by more than half.  Voxels 2-12 cm deep at or above half the
    maximum there."""
    import torch
    import paper_1302_1861_amd as P
    seeds = range(16)
    n = 20_000
    d0, s0 = _latent(P, torch, seeds, 0, 100 * n, n)
    d1, s1 = _latent(P, torch, seeds, 16, 100 * n, n)
    m = d0.mean(0).reshape(32, 32, 32)
    win = np.zeros((32, 32, 32), bool)
    win[2:12] = True
    sel = (win & (m >= 0.5 * m[2:12].max())).ravel()
    assert sel.sum() > 100
    v0 = d0[:, sel].var(0, ddof=1).mean()
    v1 = d1[:, sel].var(0, ddof=1).mean()
    b0 = (s0[:, sel] ** 2).mean()
    b1 = (s1[:, sel] ** 2).mean()
    _say("voxels %d; no APR: var %.3e batch var %.3e; APR x16: var %.3e "
         "batch var %.3e" % (sel.sum(), v0, b0, v1, b1))
    assert v0 > 3 * b0          # the spread is mostly latent (4.8x)
    assert v1 < 0.5 * v0        # APR removes most of it
