"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
read results back."""
import ctypes as C

import numpy as np

import psl_synth as S


def gpu_build(ps, grid):
    import torch
    import paper_1302_1861_amd as P
    g = P.make_grid(grid.e_edges, grid.x_edges, grid.y_edges, grid.z_plane)
    n_keys = grid.n_keys
    raw = P.Buffers.phsp_from_numpy(ps, "cuda")
    out = P.Buffers.phsp(ps.n, "cuda")
    off = torch.zeros(n_keys + 1, dtype=torch.int64, device="cuda")
    nd = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    ws = torch.empty(max(P.lib().psl_build_workspace_bytes(ps.n, C.byref(g)),
                         256), dtype=torch.uint8, device="cuda")
    P.psl_build(raw, g, out, off, nd, ws)
    torch.cuda.synchronize()
    off = off.cpu().numpy()
    kept = int(off[-1])
    res = {k: v[:kept].cpu().numpy() for k, v in out.items()}
    return res, off, int(nd.item())


def queue_contents(eng):
    """Photon and electron queue entries after psl_sample, as numpy."""
    counts = eng.queue_counts()
    n_ph = int(counts[0])
    ph = {k: v[:n_ph].cpu().numpy() for k, v in eng.ph_buf.items()}
    cap_b = eng.queue.el.capacity // eng.n_ebuckets
    el = {k: [] for k in eng.el_buf}
    el["bucket"] = []
    for b in range(eng.n_ebuckets):
        c = min(int(counts[1 + b]), cap_b)
        for k, v in eng.el_buf.items():
            el[k].append(v[b * cap_b: b * cap_b + c].cpu().numpy())
        el["bucket"].append(np.full(c, b))
    el = {k: np.concatenate(v) for k, v in el.items()}
    return ph, el, counts


def oracle_geom(oracle, phantom, iso=(0.0, 0.0, 100.0)):
    return oracle.geometry(phantom, iso=iso)


def phase_space_arrays(type_, E, x, y, u, v, w, z_plane, wt=None):
    n = len(E)
    f32 = np.float32
    return S.PhaseSpace(np.asarray(type_, np.uint8), np.asarray(E, f32),
                        np.asarray(x, f32), np.asarray(y, f32),
                        np.asarray(u, f32), np.asarray(v, f32),
                        np.asarray(w, f32),
                        np.ones(n, f32) if wt is None else np.asarray(wt, f32),
                        z_plane)
