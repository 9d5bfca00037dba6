"""CPU oracle for the PSL dose path (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product path (``paper_1302_1861_amd``) never
does, and the two share no code; both only read the seeded inputs of
``psl_synth``.

The arithmetic lives in ``oracle.c`` (plain C, double precision, built with
``-ffp-contract=off``); this module marshals numpy arrays to it and adds the
per-batch tally fold and the dose normalisation (Eq. 5), which are plain
numpy.  Every function is pinned by the ``tests/test_oracle_*`` tests.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import List

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
MEV_PER_G_TO_GY = 1.602176634e-10


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP, no FP contraction)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or \
            os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
             "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = C.CDLL(_SO)
        _declare(_lib)
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class OField(C.Structure):
    _fields_ = [("X1", C.c_double), ("X2", C.c_double), ("Y1", C.c_double),
                ("Y2", C.c_double), ("cos_g", C.c_double),
                ("sin_g", C.c_double), ("MU", C.c_double),
                ("jaws_on", C.c_int32), ("nfx", C.c_int32),
                ("nfy", C.c_int32), ("pad", C.c_int32),
                ("f_x0", C.c_double), ("f_y0", C.c_double),
                ("f_pix", C.c_double), ("fluence", C.c_void_p),
                ("cos_c", C.c_double), ("sin_c", C.c_double),
                ("cos_t", C.c_double), ("sin_t", C.c_double)]


class OGeom(C.Structure):
    _fields_ = [("sad", C.c_double), ("z_x", C.c_double),
                ("z_y", C.c_double), ("z_psl", C.c_double),
                ("iso", C.c_double * 3), ("box_lo", C.c_double * 3),
                ("box_hi", C.c_double * 3)]


class OPhantom(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("pad", C.c_int32), ("dx", C.c_double), ("dy", C.c_double),
                ("dz", C.c_double), ("x0", C.c_double), ("y0", C.c_double),
                ("z0", C.c_double), ("rho", C.c_void_p)]


class OPhys(C.Structure):
    _fields_ = [("n_e", C.c_double), ("I_eV", C.c_double),
                ("X0", C.c_double), ("step", C.c_double),
                ("p_cut", C.c_double), ("t_cut", C.c_double),
                ("flags", C.c_int32), ("pad", C.c_int32)]


FLAG_FIRST_COLLISION = 1
FLAG_NO_MSC = 2

# Columns of the per-particle trace of ``transport(..., trace=True)``:
# depth, scattering cosine, recoil energy and incident energy of the first
# photon interaction; the recoil electron's cosine to the incident photon;
# the normalised (d0 x d') . (d0 x p_e) (-1: photon and electron on opposite
# sides of the incident axis); |E d0 - E' d'| over sqrt(T (T + 2 m)); and
# the primary's direction (3) at escape.
TRACE_N = 10
TR_Z, TR_COS, TR_T, TR_E, TR_COSE, TR_SIDE, TR_PNORM, TR_EXIT = range(8)


def _declare(L):
    vp, i64, i32, d, u64 = C.c_void_p, C.c_int64, C.c_int32, C.c_double, \
        C.c_uint64
    L.oracle_splitmix64.argtypes = [u64]
    L.oracle_splitmix64.restype = u64
    L.oracle_build.argtypes = [i64, vp, vp, vp, vp, i32, vp, i32, vp, i32, vp,
                               vp, vp, vp]
    L.oracle_build.restype = i64
    L.oracle_cull.argtypes = [i32, vp, vp, vp, vp, vp, i32, d, d, d, d, i32,
                              vp, i32, vp, vp]
    L.oracle_cull.restype = None
    L.oracle_roi.argtypes = [d, d, d, d, d, C.POINTER(d), C.POINTER(d)]
    L.oracle_roi.restype = None
    L.oracle_alloc.argtypes = [i32, vp, i32, i64, i64, i32, vp, vp, vp, vp,
                               vp]
    L.oracle_alloc.restype = i32
    L.oracle_sample.argtypes = [i32, vp, vp, i64, vp, vp, vp, i64, u64,
                                vp, vp, vp, vp, vp, vp, vp, vp,
                                vp, vp, vp, vp, vp]
    L.oracle_sample.restype = None
    L.oracle_apr_rotation.argtypes = [u64, u64, C.POINTER(d), C.POINTER(d)]
    L.oracle_apr_rotation.restype = None
    L.oracle_apr_expand.argtypes = [i64, i64, u64] + [vp] * 16
    L.oracle_apr_expand.restype = None
    L.oracle_stream.argtypes = [vp, vp, i32, i64] + [vp] * 8 + \
        [i32, vp, i64, i64, u64, d, i64, vp, vp, vp, vp, vp, vp, vp]
    L.oracle_stream.restype = i64
    L.oracle_kn_sigma.argtypes = [d]
    L.oracle_kn_sigma.restype = d
    L.oracle_stopping_power.argtypes = [d, d, d]
    L.oracle_stopping_power.restype = d
    L.oracle_csda_range.argtypes = [d, d, d, d]
    L.oracle_csda_range.restype = d
    L.oracle_highland.argtypes = [d, d, d]
    L.oracle_highland.restype = d
    L.oracle_transport.argtypes = [i64, vp, vp, vp, u64, vp, vp, vp, vp, vp,
                                   vp, i32]
    L.oracle_transport.restype = None
    L.oracle_msc_samples.argtypes = [i64, d, d, d, u64, vp]
    L.oracle_msc_samples.restype = None


# ---------------------------------------------------------------------------
# Sec. 2.3.2: PSL generation
# ---------------------------------------------------------------------------
def build_psl(ps, grid):
    """Returns (perm, offsets, n_dropped): perm[j] = input index of the j-th
    particle in PSL order, offsets[n_keys + 1] int64."""
    n = ps.n
    n_keys = grid.n_keys
    perm = np.zeros(max(n, 1), np.int64)
    offsets = np.zeros(n_keys + 1, np.int64)
    nd = np.zeros(1, np.int64)
    c = np.ascontiguousarray
    t, E, x, y = (c(ps.type, np.uint8), c(ps.E, np.float32),
                  c(ps.x, np.float32), c(ps.y, np.float32))
    ee, xe, ye = (c(grid.e_edges, np.float32), c(grid.x_edges, np.float32),
                  c(grid.y_edges, np.float32))
    kept = lib().oracle_build(n, _p(t), _p(E), _p(x), _p(y), grid.n_e,
                              _p(ee), grid.n_x, _p(xe), grid.n_y, _p(ye),
                              _p(perm), _p(offsets), _p(nd))
    return perm[:kept], offsets, int(nd[0])


def splitmix64(x: int) -> int:
    return int(lib().oracle_splitmix64(C.c_uint64(x & (2**64 - 1))))


# ---------------------------------------------------------------------------
# Sec. 2.3.3: ROI selection, Eq. (1)-(4)
# ---------------------------------------------------------------------------
def roi(lo_at_sad, hi_at_sad, z_jaw, sad, z_psl):
    lo, hi = C.c_double(), C.c_double()
    lib().oracle_roi(lo_at_sad, hi_at_sad, z_jaw, sad, z_psl, C.byref(lo),
                     C.byref(hi))
    return lo.value, hi.value


def cull(fields, grid, cull_on, geom):
    F = len(fields)
    arr = lambda k: np.array([getattr(f, k) for f in fields], np.float64)
    jaws = np.array([1 if f.jaws else 0 for f in fields], np.int32)
    mask = np.zeros((F, grid.n_y * grid.n_x), np.uint8)
    X1, X2, Y1, Y2 = arr("X1"), arr("X2"), arr("Y1"), arr("Y2")
    xe = np.ascontiguousarray(grid.x_edges, np.float32)
    ye = np.ascontiguousarray(grid.y_edges, np.float32)
    lib().oracle_cull(F, _p(X1), _p(X2), _p(Y1), _p(Y2), _p(jaws),
                      1 if cull_on else 0, geom["sad"], geom["z_x"],
                      geom["z_y"], grid.z_plane, grid.n_x, _p(xe), grid.n_y,
                      _p(ye), _p(mask))
    return mask


def alloc(fields, mode, n_sim, offsets, mask, grid):
    F = len(fields)
    n_keys = grid.n_keys
    MU = np.array([f.MU for f in fields], np.float64)
    N = np.zeros((F, n_keys), np.int64)
    g = np.zeros((F, n_keys), np.float64)
    NF = np.zeros(F, np.int64)
    offsets = np.ascontiguousarray(offsets, np.int64)
    mask = np.ascontiguousarray(mask, np.uint8)
    rc = lib().oracle_alloc(F, _p(MU), mode, int(n_sim), n_keys,
                            grid.n_x * grid.n_y, _p(offsets), _p(mask),
                            _p(N), _p(g), _p(NF))
    if rc != 0:
        raise ValueError("no particle selected")
    return N, g, NF


def _ofields(fields):
    keep = []
    arr = (OField * len(fields))()
    for i, f in enumerate(fields):
        a = arr[i]
        a.X1, a.X2, a.Y1, a.Y2 = f.X1, f.X2, f.Y1, f.Y2
        th = math.radians(f.gantry_deg)
        a.cos_g, a.sin_g = math.cos(th), math.sin(th)
        tc = math.radians(getattr(f, "collimator_deg", 0.0))
        a.cos_c, a.sin_c = math.cos(tc), math.sin(tc)
        tt = math.radians(getattr(f, "couch_deg", 0.0))
        a.cos_t, a.sin_t = math.cos(tt), math.sin(tt)
        a.MU = f.MU
        a.jaws_on = 1 if f.jaws else 0
        if f.fluence is not None:
            fl = np.ascontiguousarray(f.fluence, np.float32)
            keep.append(fl)
            a.nfy, a.nfx = fl.shape
            a.fluence = fl.ctypes.data
        else:
            a.nfx = a.nfy = 0
            a.fluence = None
        a.f_x0, a.f_y0, a.f_pix = f.f_x0, f.f_y0, f.f_pix
    return arr, keep


def geometry(phantom, iso=(0.0, 0.0, 100.0), sad=100.0, z_x=37.0,
             z_y=28.0, z_psl=25.0):
    nz, ny, nx = phantom.density.shape
    lo = np.array(phantom.origin, np.float64)
    hi = lo + np.array([nx, ny, nz], np.float64) * np.array(phantom.voxel)
    return {"sad": sad, "z_x": z_x, "z_y": z_y, "z_psl": z_psl,
            "iso": tuple(iso), "box_lo": tuple(lo), "box_hi": tuple(hi)}


def _ogeom(geom):
    g = OGeom()
    g.sad, g.z_x, g.z_y, g.z_psl = (geom["sad"], geom["z_x"], geom["z_y"],
                                    geom["z_psl"])
    for a in range(3):
        g.iso[a] = geom["iso"][a]
        g.box_lo[a] = geom["box_lo"][a]
        g.box_hi[a] = geom["box_hi"][a]
    return g


def sample(fields, geom, offsets, N, g, batch, seed, ps):
    """Canonical history list of one batch.  Returns a dict of per-history
    arrays: src (phase-space index in PSL order), field, key, status
    (0 jaw-rejected, 1 accepted, 2 zero fluence, 3 misses the phantom),
    state [n, 8] = E x y z u v w wt, and uid = batch * n_hist + h."""
    F, n_keys = N.shape
    n_hist = int(N.sum())
    src = np.zeros(n_hist, np.int64)
    fld = np.zeros(n_hist, np.int32)
    key = np.zeros(n_hist, np.int32)
    st = np.zeros(n_hist, np.uint8)
    state = np.zeros((n_hist, 8), np.float64)
    arr, keep = _ofields(fields)
    G = _ogeom(geom)
    c = np.ascontiguousarray
    cols = [c(getattr(ps, k)) for k in ("type", "E", "x", "y", "u", "v", "w",
                                         "wt")]
    N = c(N, np.int64)
    g = c(g, np.float64)
    offsets = c(offsets, np.int64)
    lib().oracle_sample(F, C.cast(arr, C.c_void_p), C.byref(G), n_keys,
                        _p(offsets), _p(N), _p(g), int(batch),
                        C.c_uint64(seed), *[_p(a) for a in cols], _p(src),
                        _p(fld), _p(key), _p(st), _p(state))
    del keep
    uid = np.uint64(batch) * np.uint64(n_hist) + np.arange(n_hist,
                                                           dtype=np.uint64)
    return {"src": src, "field": fld, "key": key, "status": st,
            "state": state, "uid": uid,
            "type": ps.type[src] if n_hist else np.zeros(0, np.uint8)}


def apr_rotation(seed, m):
    """(cos, sin) of the APR azimuth of copy m (Sec. 2.3.1)."""
    c, s = C.c_double(), C.c_double()
    lib().oracle_apr_rotation(C.c_uint64(seed), C.c_uint64(m), C.byref(c),
                              C.byref(s))
    return c.value, s.value


def apr_expand(ps, copies, seed):
    """The APR-expanded phase space (Sec. 2.3.1): `copies` azimuthally
    redistributed copies of every particle, weight wt / copies; the PSLs
    are then built from it by build_psl."""
    from psl_synth import PhaseSpace
    n, k = int(ps.n), int(copies)
    c = np.ascontiguousarray
    cols = [c(getattr(ps, f)) for f in ("type", "E", "x", "y", "u", "v", "w",
                                         "wt")]
    out = [np.zeros(n * k, np.uint8)] + [np.zeros(n * k, np.float32)
                                         for _ in range(7)]
    lib().oracle_apr_expand(n, k, C.c_uint64(seed), *[_p(a) for a in cols],
                            *[_p(a) for a in out])
    return PhaseSpace(*out, z_plane=ps.z_plane)


def stream_sample(field, geom, ps, e_edges, n_hist, batch, seed, cap,
                  method=2, weight=None):
    """Methods 1 and 2 (Sec. 2.1, 2.2) for one batch: the phase space read
    in file order from a random start, the beam model (Method 2), on-the-fly
    bins by type and energy flushed when they hold `cap` particles and at
    the end.  weight: the per-history factor g (default n / n_hist, dose per
    phase-space particle).  Returns per-history status (0 jaw, 1 accepted,
    2 zero fluence, 3 miss, 4 dropped: bad type or NaN energy), state
    [n_hist, 8] = E x y z u v w w', src, uid, type; the flushes (bin, count,
    trigger, first) in order; seq, the flushed sequence of history
    indices."""
    n = int(ps.n)
    n_hist = int(n_hist)
    e_edges = np.ascontiguousarray(e_edges, np.float32)
    n_e = len(e_edges) - 1
    g = float(n) / n_hist if weight is None else float(weight)
    st = np.zeros(n_hist, np.uint8)
    state = np.zeros((max(n_hist, 1), 8), np.float64)
    max_fl = n_hist // max(int(cap), 1) + 2 * n_e + 1
    fb = np.zeros(max_fl, np.int32)
    fc = np.zeros(max_fl, np.int64)
    ft = np.zeros(max_fl, np.int64)
    ff = np.zeros(max_fl, np.int64)
    seq = np.zeros(max(n_hist, 1), np.int64)
    arr, keep = _ofields([field])
    G = _ogeom(geom)
    c = np.ascontiguousarray
    cols = [c(getattr(ps, k)) for k in ("type", "E", "x", "y", "u", "v", "w",
                                         "wt")]
    nf = lib().oracle_stream(C.cast(arr, C.c_void_p), C.byref(G), int(method),
                             n, *[_p(a) for a in cols], n_e, _p(e_edges),
                             n_hist, int(batch), C.c_uint64(seed), g,
                             int(cap), _p(st), _p(state), _p(fb), _p(fc),
                             _p(ft), _p(ff), _p(seq))
    del keep
    s0 = int(splitmix64(seed) % n) if n else 0
    src = (s0 + int(batch) * n_hist + np.arange(n_hist, dtype=np.int64)) % \
        max(n, 1)
    uid = np.uint64(batch) * np.uint64(n_hist) + np.arange(n_hist,
                                                           dtype=np.uint64)
    n_seq = int(fc[:nf].sum())
    return {"status": st, "state": state[:n_hist], "src": src, "uid": uid,
            "type": ps.type[src] if n_hist else np.zeros(0, np.uint8),
            "flush_bin": fb[:nf], "flush_count": fc[:nf],
            "flush_trigger": ft[:nf], "flush_first": ff[:nf],
            "seq": seq[:n_seq], "weight": g}


def dose_point(dose, sigma, phantom, point, radius):
    """Reference-point dose (Sec. 2.5): mean of the dose over the voxels
    whose centres lie within `radius` of `point` (the voxel holding the
    point when none does), standard error sqrt(sum sigma^2) / count.
    Returns (mean, standard error, count)."""
    nz, ny, nx = phantom.density.shape
    dx, dy, dz = phantom.voxel
    x0, y0, z0 = phantom.origin
    d = np.asarray(dose, np.float64).reshape(nz, ny, nx)
    s = np.asarray(sigma, np.float64).reshape(nz, ny, nx)
    cz = z0 + (np.arange(nz) + 0.5) * dz - point[2]
    cy = y0 + (np.arange(ny) + 0.5) * dy - point[1]
    cx = x0 + (np.arange(nx) + 0.5) * dx - point[0]
    r2 = cz[:, None, None] ** 2 + cy[None, :, None] ** 2 + \
        cx[None, None, :] ** 2
    m = r2 <= radius * radius
    n = int(m.sum())
    if n == 0:
        i = math.floor((point[0] - x0) / dx)
        j = math.floor((point[1] - y0) / dy)
        k = math.floor((point[2] - z0) / dz)
        if 0 <= i < nx and 0 <= j < ny and 0 <= k < nz:
            return float(d[k, j, i]), float(s[k, j, i]), 1
        return 0.0, 0.0, 0
    return float(d[m].sum() / n), float(math.sqrt((s[m] ** 2).sum()) / n), n


# ---------------------------------------------------------------------------
# Transport (physics of the workloads; the paper defers to gDPM)
# ---------------------------------------------------------------------------
def kn_sigma(E):
    return lib().oracle_kn_sigma(float(E))


def stopping_power(T, n_e=3.343e23, I_eV=75.0):
    return lib().oracle_stopping_power(float(T), n_e, I_eV)


def csda_range(t_lo, T, n_e=3.343e23, I_eV=75.0):
    return lib().oracle_csda_range(float(t_lo), float(T), n_e, I_eV)


def highland(T, t, X0=36.08):
    return lib().oracle_highland(float(T), float(t), X0)


def msc_samples(n, T, t, X0=36.08, seed=1):
    out = np.zeros((n, 2), np.float64)
    lib().oracle_msc_samples(n, T, t, X0, C.c_uint64(seed), _p(out))
    return out


def ophantom(ph):
    nz, ny, nx = ph.density.shape
    P = OPhantom()
    P.nx, P.ny, P.nz = nx, ny, nz
    P.dx, P.dy, P.dz = ph.voxel
    P.x0, P.y0, P.z0 = ph.origin
    rho = np.ascontiguousarray(ph.density, np.float32)
    P.rho = rho.ctypes.data
    return P, rho


def ophys(n_e=3.343e23, I_eV=75.0, X0=36.08, step=0.1, p_cut=0.010,
          t_cut=0.700 - 0.51099895, flags=0):
    Y = OPhys()
    Y.n_e, Y.I_eV, Y.X0, Y.step, Y.p_cut, Y.t_cut = (n_e, I_eV, X0, step,
                                                     p_cut, t_cut)
    Y.flags = flags
    return Y


def transport(types, state, uid, seed, phantom, phys=None, acc=None,
              ledger=False, trace=False, n_threads=0):
    """Transport particles (rows E x y z u v w wt) and return
    (acc [voxels] MeV*weight, counts[2], ledger or None, trace or None);
    the trace has the TR_* columns above."""
    phys = phys or ophys()
    n = int(len(types))
    nvox = int(np.prod(phantom.density.shape))
    if acc is None:
        acc = np.zeros(nvox, np.float64)
    P, rho = ophantom(phantom)
    led = np.zeros((n, 4), np.float64) if ledger else None
    tr = np.zeros((n, TRACE_N), np.float64) if trace else None
    counts = np.zeros(2, np.int64)
    types = np.ascontiguousarray(types, np.uint8)
    state = np.ascontiguousarray(state, np.float64)
    uid = np.ascontiguousarray(uid, np.uint64)
    lib().oracle_transport(n, _p(types), _p(state), _p(uid),
                           C.c_uint64(seed), C.byref(P), C.byref(phys),
                           _p(acc), _p(led), _p(tr), _p(counts), n_threads)
    del rho
    return acc, counts, led, tr


# ---------------------------------------------------------------------------
# Dose tally (Sec. 2.3.3 batch uncertainty; Eq. 5 normalisation)
# ---------------------------------------------------------------------------
def fold(acc_b, s1, s2):
    """Add one batch's energy tally to the running sums of tally and tally
    squared."""
    s1 += acc_b
    s2 += acc_b * acc_b


def finalize(s1, s2, n_batches, phantom, norm):
    """Mean dose over batches and its standard error, in Gy per unit of
    ``norm`` (norm = 1 / N_incident): D_v = E_v [MeV] 1.602176634e-10 /
    (rho_v V) * norm; sigma from the spread of the batch estimates."""
    B = n_batches
    rho = phantom.density.reshape(-1).astype(np.float64)
    V = float(np.prod(phantom.voxel))
    with np.errstate(divide="ignore"):
        c = np.where(rho > 0, MEV_PER_G_TO_GY / (rho * V), 0.0) * norm
    mean = s1 / B
    var = np.maximum(s2 - s1 * s1 / B, 0.0) / (B - 1) if B > 1 else \
        np.zeros_like(s1)
    return mean * c, np.sqrt(var / B) * c


def run_dose(wl, n_threads=0, histories=None, batches=None, phys=None,
             geom=None):
    """End-to-end oracle dose for a workload: PSL build, cull, allocation,
    then per batch: sampling, transport, fold; finally Eq. (5).  Returns
    (dose, sigma, info)."""
    ps, grid = wl.phsp, wl.grid
    perm, offsets, nd = build_psl(ps, grid)
    sorted_ps = ps.subset(perm)
    geom = geom or geometry(wl.phantom, z_psl=grid.z_plane)
    mask = cull(wl.fields, grid, wl.cull, geom)
    B = batches or wl.batches
    H = histories or wl.histories
    per_batch = H // B
    N, g, NF = alloc(wl.fields, wl.alloc_mode, per_batch, offsets, mask,
                     grid)
    nvox = int(np.prod(wl.phantom.density.shape))
    s1 = np.zeros(nvox)
    s2 = np.zeros(nvox)
    n_acc = 0
    for b in range(B):
        S = sample(wl.fields, geom, offsets, N, g, b, wl.seed, sorted_ps)
        ok = S["status"] == 1
        n_acc += int(ok.sum())
        acc, _, _, _ = transport(S["type"][ok], S["state"][ok], S["uid"][ok],
                                 wl.seed + b, wl.phantom, phys,
                                 n_threads=n_threads)
        fold(acc, s1, s2)
    dose, sigma = finalize(s1, s2, B, wl.phantom, 1.0 / ps.n)
    return dose, sigma, {"accepted": n_acc, "histories": per_batch * B,
                         "n_dropped": nd}
