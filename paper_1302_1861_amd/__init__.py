"""Python binding of the PSL dose library (libpsl.so, gfx950).

Argument marshalling only: every step of the dose path runs in the HIP
kernels behind the C ABI declared in include/psl.h.  PyTorch provides device
memory and the current HIP stream.  The functions below carry the C names
(psl_build, psl_sample, transport_batch, dose_tally, ...) and take torch
tensors; ``Engine`` allocates the buffers one workload needs and chains the
calls.  There is no CPU fallback: if the library is missing or the device is
not a gfx950, calls raise.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsl.so")

PSL_OK, PSL_EINVAL, PSL_ENOSPC, PSL_EHIP, PSL_EUNSUPPORTED = 0, 1, 2, 3, 4
PSL_MAX_EBINS = 64
PSL_MAX_POSBINS = 128
PSL_MAX_QBUCKETS = 16
PSL_QCOUNTS = PSL_MAX_QBUCKETS + 2
PSL_TABLE_BYTES = 64 * 1024
PSL_ALLOC_COUNTS, PSL_ALLOC_MU = 0, 1
PSL_ACC_F64, PSL_ACC_FIXED64, PSL_ACC_TRACE = 0, 1, 2
PSL_TALLY_FOLD, PSL_TALLY_FINALIZE = 0, 1
PSL_FLAG_FIRST_COLLISION, PSL_FLAG_NO_MSC = 1, 2

EXPORTS = ["psl_last_error", "psl_version", "psl_build_workspace_bytes",
           "psl_build", "psl_sample_workspace_bytes", "psl_sample",
           "psl_physics_init", "transport_batch_workspace_bytes",
           "transport_batch", "dose_tally", "psl_profile_enable",
           "psl_profile_read", "psl_bench_atomics_workspace_bytes",
           "psl_bench_atomics", "psl_plan_workspace_bytes", "psl_plan_create",
           "psl_plan_run", "psl_autotune", "psl_plan_get", "psl_plan_destroy",
           "psl_plan_run_pair", "psl_plan_run_set", "psl_plan_copy_tuning",
           "unet_param_count", "unet_workspace_bytes", "unet_init",
           "unet_set_params", "unet_forward", "unet_backward",
           "unet_adam_step", "unet_set_brick_blocks", "dose_denoise",
           "dose_gamma", "psl_sample_noalloc_max_bytes",
           "psl_sample_noalloc", "psl_bench_atomics_replay",
           "psl_stream_workspace_bytes", "psl_stream_sample", "dose_point",
           "psl_build_apr_workspace_bytes", "psl_build_apr"]


class PslError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("psl status %d: %s" % (status, msg))
        self.status = status


# --------------------------------------------------------------- structs --
class psl_phsp(C.Structure):
    _fields_ = [("n", C.c_int64), ("type", C.c_void_p), ("E", C.c_void_p),
                ("x", C.c_void_p), ("y", C.c_void_p), ("u", C.c_void_p),
                ("v", C.c_void_p), ("w", C.c_void_p), ("wt", C.c_void_p)]


class psl_grid(C.Structure):
    _fields_ = [("n_e", C.c_int32), ("n_x", C.c_int32), ("n_y", C.c_int32),
                ("pad", C.c_int32), ("z_plane", C.c_double),
                ("e_edges", C.c_float * (PSL_MAX_EBINS + 1)),
                ("x_edges", C.c_float * (PSL_MAX_POSBINS + 1)),
                ("y_edges", C.c_float * (PSL_MAX_POSBINS + 1))]


class psl_field(C.Structure):
    _fields_ = [("X1", C.c_double), ("X2", C.c_double), ("Y1", C.c_double),
                ("Y2", C.c_double), ("gantry_deg", C.c_double),
                ("MU", C.c_double), ("fluence", C.c_void_p),
                ("nfx", C.c_int32), ("nfy", C.c_int32), ("f_x0", C.c_double),
                ("f_y0", C.c_double), ("f_pix", C.c_double),
                ("jaws_on", C.c_int32), ("pad", C.c_int32),
                ("collimator_deg", C.c_double), ("couch_deg", C.c_double)]


class psl_sample_cfg(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("batch", C.c_int64),
                ("n_histories", C.c_int64), ("cull", C.c_int32),
                ("alloc_mode", C.c_int32), ("sad", C.c_double),
                ("z_jaw_x", C.c_double), ("z_jaw_y", C.c_double),
                ("iso", C.c_double * 3), ("box_lo", C.c_double * 3),
                ("box_hi", C.c_double * 3)]


class psl_stream_cfg(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("batch", C.c_int64),
                ("n_histories", C.c_int64), ("bin_capacity", C.c_int64),
                ("method", C.c_int32), ("n_e", C.c_int32),
                ("e_edges", C.c_void_p), ("weight", C.c_double),
                ("z_plane", C.c_double), ("sad", C.c_double),
                ("z_jaw_x", C.c_double), ("z_jaw_y", C.c_double),
                ("iso", C.c_double * 3), ("box_lo", C.c_double * 3),
                ("box_hi", C.c_double * 3)]


class psl_flush(C.Structure):
    _fields_ = [("bin", C.c_int32), ("pad", C.c_int32),
                ("count", C.c_int64), ("trigger", C.c_int64),
                ("first", C.c_int64)]


class psl_particles(C.Structure):
    _fields_ = [("capacity", C.c_int64)] + \
        [(k, C.c_void_p) for k in ("E", "x", "y", "z", "u", "v", "w", "wt",
                                   "uid", "ctr")]


class psl_queue(C.Structure):
    _fields_ = [("ph", psl_particles), ("el", psl_particles),
                ("n_ebuckets", C.c_int32), ("pad", C.c_int32),
                ("e_bucket_edges", C.c_float * (PSL_MAX_QBUCKETS + 1)),
                ("d_counts", C.c_void_p)]


STATS_FIELDS = ["histories", "jaw_rejected", "fluence_zero", "missed",
                "photons", "electrons", "lost", "interactions", "secondaries",
                "segments", "flights", "runaway", "deposits",
                "photon_deposits", "bucket_peak", "dropped"]


class psl_stats(C.Structure):
    _fields_ = [(k, C.c_uint64) for k in STATS_FIELDS] + \
        [("e_in", C.c_double), ("e_escaped", C.c_double),
         ("e_killed", C.c_double)]


class psl_phantom(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("pad", C.c_int32), ("dx", C.c_double), ("dy", C.c_double),
                ("dz", C.c_double), ("x0", C.c_double), ("y0", C.c_double),
                ("z0", C.c_double), ("density", C.c_void_p),
                ("rho_max", C.c_float), ("rho_min", C.c_float)]


class psl_physics(C.Structure):
    _fields_ = [("n_e", C.c_double), ("I_eV", C.c_double),
                ("X0", C.c_double), ("step", C.c_double),
                ("p_cut", C.c_double), ("t_cut", C.c_double),
                ("e_max", C.c_double), ("flags", C.c_int32),
                ("pad", C.c_int32)]


class psl_dose_acc(C.Structure):
    _fields_ = [("mode", C.c_int32), ("frac_bits", C.c_int32),
                ("data", C.c_void_p), ("trace_capacity", C.c_int64)]


class psl_launch(C.Structure):
    _fields_ = [("block", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("n_cu", C.c_int32), ("rebucket", C.c_int32)]


class psl_tune_result(C.Structure):
    _fields_ = [("launch", psl_launch), ("n_ebuckets", C.c_int32),
                ("configs_tried", C.c_int32),
                ("e_bucket_edges", C.c_float * (PSL_MAX_QBUCKETS + 1)),
                ("ms_per_batch", C.c_double),
                ("el_capacity_suggested", C.c_int64),
                ("bucket_peak", C.c_int64)]


class psl_unet(C.Structure):
    _fields_ = [("levels", C.c_int32), ("base", C.c_int32),
                ("n_params", C.c_int64), ("params", C.c_void_p),
                ("params_bf16", C.c_void_p)]


def make_launch(blocks_per_cu=4, rebucket=1, n_cu=0, block=256):
    L = psl_launch()
    L.block, L.blocks_per_cu, L.n_cu, L.rebucket = block, blocks_per_cu, \
        n_cu, rebucket
    return L


# ------------------------------------------------------------------ load --
_lib = None


def lib():
    """The loaded libpsl.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                "libpsl.so is not built; run "
                "`python -m paper_1302_1861_amd.build_lib` (or "
                "__graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, sz, u64, d = (C.c_void_p, C.c_int32, C.c_int64,
                                     C.c_size_t, C.c_uint64, C.c_double)
        L.psl_last_error.restype = C.c_char_p
        L.psl_version.restype = i32
        L.psl_build_workspace_bytes.argtypes = [i64, vp]
        L.psl_build_workspace_bytes.restype = sz
        L.psl_build.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
        L.psl_build.restype = i32
        L.psl_sample_workspace_bytes.argtypes = [vp, i32, i64]
        L.psl_sample_workspace_bytes.restype = sz
        L.psl_sample.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp,
                                 sz, vp]
        L.psl_sample.restype = i32
        L.psl_sample_noalloc_max_bytes.argtypes = []
        L.psl_sample_noalloc_max_bytes.restype = sz
        L.psl_sample_noalloc.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp,
                                         vp, vp]
        L.psl_sample_noalloc.restype = i32
        L.psl_bench_atomics_replay.argtypes = [vp, i64, i64, vp, i32, i32, vp,
                                               vp, sz, vp]
        L.psl_bench_atomics_replay.restype = i32
        L.psl_stream_workspace_bytes.argtypes = [i64, i32, i64]
        L.psl_stream_workspace_bytes.restype = sz
        L.psl_stream_sample.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp, vp,
                                        sz, vp]
        L.psl_stream_sample.restype = i32
        L.dose_point.argtypes = [vp, vp, vp, d, d, d, d, vp, vp]
        L.dose_point.restype = i32
        L.psl_build_apr_workspace_bytes.argtypes = [i64, i64, vp]
        L.psl_build_apr_workspace_bytes.restype = sz
        L.psl_build_apr.argtypes = [vp, vp, i64, u64, vp, vp, vp, vp, sz, vp]
        L.psl_build_apr.restype = i32
        L.psl_physics_init.argtypes = [vp, vp, vp]
        L.psl_physics_init.restype = i32
        L.transport_batch_workspace_bytes.argtypes = [vp]
        L.transport_batch_workspace_bytes.restype = sz
        L.transport_batch.argtypes = [vp, vp, vp, vp, u64, vp, vp, vp, vp, sz,
                                      vp]
        L.transport_batch.restype = i32
        L.dose_tally.argtypes = [vp, vp, vp, i32, i32, vp, d, vp, vp, vp]
        L.dose_tally.restype = i32
        L.psl_profile_enable.argtypes = [i32]
        L.psl_profile_enable.restype = i32
        L.psl_profile_read.argtypes = [vp, vp, i32]
        L.psl_profile_read.restype = i32
        L.psl_bench_atomics_workspace_bytes.argtypes = [i64]
        L.psl_bench_atomics_workspace_bytes.restype = sz
        L.psl_bench_atomics.argtypes = [i64, vp, vp, sz, vp]
        L.psl_bench_atomics.restype = i32
        L.psl_plan_workspace_bytes.argtypes = [vp, i32, i64, vp]
        L.psl_plan_workspace_bytes.restype = sz
        L.psl_plan_create.argtypes = [vp, vp, vp, vp, vp, i32, vp, vp, vp, vp,
                                      vp, u64, vp, vp, vp, vp, vp, vp, sz, vp]
        L.psl_plan_create.restype = i32
        L.psl_plan_run.argtypes = [vp, i64, i32, i32, vp]
        L.psl_plan_run.restype = i32
        L.psl_autotune.argtypes = [vp, i32, vp, vp]
        L.psl_autotune.restype = i32
        L.psl_plan_get.argtypes = [vp, vp, vp]
        L.psl_plan_get.restype = i32
        L.psl_plan_run_pair.argtypes = [vp, vp, i64, i32, i32, vp]
        L.psl_plan_run_pair.restype = i32
        L.psl_plan_run_set.argtypes = [C.POINTER(vp), i32, i64, i32, vp]
        L.psl_plan_run_set.restype = i32
        L.psl_plan_copy_tuning.argtypes = [vp, vp]
        L.psl_plan_copy_tuning.restype = i32
        L.psl_plan_destroy.argtypes = [vp]
        L.psl_plan_destroy.restype = i32
        L.unet_param_count.argtypes = [i32, i32]
        L.unet_param_count.restype = i64
        L.unet_workspace_bytes.argtypes = [vp, i32, i32, i32, i32, i32]
        L.unet_workspace_bytes.restype = sz
        L.unet_init.argtypes = [vp, u64, vp]
        L.unet_init.restype = i32
        L.unet_set_params.argtypes = [vp, vp]
        L.unet_set_params.restype = i32
        L.unet_set_brick_blocks.argtypes = [i32]
        L.unet_set_brick_blocks.restype = i32
        L.unet_forward.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp, vp, sz,
                                   vp]
        L.unet_forward.restype = i32
        L.unet_backward.argtypes = [vp, vp, vp, vp, i32, i32, i32, i32, vp,
                                    vp, vp, sz, vp]
        L.unet_backward.restype = i32
        L.unet_adam_step.argtypes = [vp, vp, vp, vp, C.c_float, C.c_float,
                                     C.c_float, C.c_float, i32, vp]
        L.unet_adam_step.restype = i32
        L.dose_denoise.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, sz, vp]
        L.dose_denoise.restype = i32
        d = C.c_double
        L.dose_gamma.argtypes = [vp, vp, i32, i32, i32, d, d, d, d, d, d, d,
                                 vp, vp, vp]
        L.dose_gamma.restype = i32
        _lib = L
    return _lib


def _check(status):
    if status != PSL_OK:
        raise PslError(status, lib().psl_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ------------------------------------------------------------- marshals --
def make_grid(e_edges, x_edges, y_edges, z_plane) -> psl_grid:
    g = psl_grid()
    e, x, y = (np.asarray(a, np.float32) for a in (e_edges, x_edges, y_edges))
    if len(e) - 1 > PSL_MAX_EBINS or len(x) - 1 > PSL_MAX_POSBINS or \
            len(y) - 1 > PSL_MAX_POSBINS:
        raise ValueError("grid too large for psl_grid")
    g.n_e, g.n_x, g.n_y = len(e) - 1, len(x) - 1, len(y) - 1
    g.z_plane = float(z_plane)
    for i, v in enumerate(e):
        g.e_edges[i] = float(v)
    for i, v in enumerate(x):
        g.x_edges[i] = float(v)
    for i, v in enumerate(y):
        g.y_edges[i] = float(v)
    return g


PHSP_KEYS = ("type", "E", "x", "y", "u", "v", "w", "wt")
PART_KEYS = ("E", "x", "y", "z", "u", "v", "w", "wt", "uid", "ctr")


def make_phsp(t: Dict, n: Optional[int] = None) -> psl_phsp:
    p = psl_phsp()
    p.n = int(t["E"].shape[0] if n is None else n)
    for k in PHSP_KEYS:
        setattr(p, k, t[k].data_ptr())
    return p


def make_particles(t: Dict) -> psl_particles:
    p = psl_particles()
    p.capacity = int(t["E"].shape[0])
    for k in PART_KEYS:
        setattr(p, k, t[k].data_ptr())
    return p


def make_fields(fields, fluence_tensors) -> "C.Array":
    arr = (psl_field * len(fields))()
    for i, f in enumerate(fields):
        a = arr[i]
        a.X1, a.X2, a.Y1, a.Y2 = f.X1, f.X2, f.Y1, f.Y2
        a.gantry_deg, a.MU = f.gantry_deg, f.MU
        fl = fluence_tensors[i]
        if fl is not None:
            a.fluence = fl.data_ptr()
            a.nfy, a.nfx = fl.shape
        else:
            a.fluence, a.nfx, a.nfy = None, 0, 0
        a.f_x0, a.f_y0, a.f_pix = f.f_x0, f.f_y0, f.f_pix
        a.jaws_on = 1 if f.jaws else 0
        a.collimator_deg = f.collimator_deg
        a.couch_deg = f.couch_deg
    return arr


def make_phantom(density_t, voxel, origin, rho_max=None,
                 rho_min=None) -> psl_phantom:
    """rho_max / rho_min default to the exact extremes of the density."""
    p = psl_phantom()
    p.nz, p.ny, p.nx = density_t.shape
    p.dx, p.dy, p.dz = (float(v) for v in voxel)
    p.x0, p.y0, p.z0 = (float(v) for v in origin)
    p.density = density_t.data_ptr()
    p.rho_max = float(rho_max if rho_max is not None
                      else density_t.max().item())
    p.rho_min = float(rho_min if rho_min is not None
                      else max(density_t.min().item(), 0.0))
    return p


def make_physics(n_e=3.343e23, I_eV=75.0, X0=36.08, step=0.1, p_cut=0.010,
                 t_cut=0.700 - 0.51099895, e_max=6.0, flags=0) -> psl_physics:
    y = psl_physics()
    y.n_e, y.I_eV, y.X0, y.step, y.p_cut, y.t_cut, y.e_max = (
        n_e, I_eV, X0, step, p_cut, t_cut, e_max)
    y.flags = flags
    return y


# ------------------------------------------------------- the C functions --
def psl_build(in_phsp: Dict, grid: psl_grid, out_phsp: Dict, offsets,
              n_dropped, ws, stream=None):
    i, o = make_phsp(in_phsp), make_phsp(out_phsp)
    _check(lib().psl_build(C.byref(i), C.byref(grid), C.byref(o),
                           _ptr(offsets), _ptr(n_dropped), _ptr(ws),
                           ws.numel() * ws.element_size(), _stream(stream)))


def psl_build_apr(in_phsp: Dict, grid: psl_grid, copies: int, seed: int,
                  out_phsp: Dict, offsets, n_dropped, ws, stream=None):
    """psl_build of `copies` azimuthally redistributed copies of every
    particle (Sec. 2.3.1); out holds n * copies entries."""
    i, o = make_phsp(in_phsp), make_phsp(out_phsp)
    _check(lib().psl_build_apr(C.byref(i), C.byref(grid), int(copies),
                               C.c_uint64(seed), C.byref(o), _ptr(offsets),
                               _ptr(n_dropped), _ptr(ws),
                               ws.numel() * ws.element_size(),
                               _stream(stream)))


def psl_sample(sorted_phsp: Dict, offsets, grid: psl_grid, fields_arr,
               cfg: psl_sample_cfg, queue: psl_queue, stats, ws, mask=None,
               alloc=None, n_sorted=None, stream=None):
    s = make_phsp(sorted_phsp, n_sorted)
    _check(lib().psl_sample(C.byref(s), _ptr(offsets), C.byref(grid),
                            fields_arr, len(fields_arr), C.byref(cfg),
                            C.byref(queue), _ptr(mask), _ptr(alloc),
                            _ptr(stats), _ptr(ws),
                            ws.numel() * ws.element_size(), _stream(stream)))


def psl_sample_noalloc(sorted_phsp: Dict, offsets, grid: psl_grid,
                       fields_arr, cfg: psl_sample_cfg, queue: psl_queue,
                       stats, mask=None, alloc=None, n_sorted=None,
                       stream=None):
    """psl_sample with the library's static scratch instead of a
    workspace (for callers that cannot allocate)."""
    s = make_phsp(sorted_phsp, n_sorted)
    _check(lib().psl_sample_noalloc(C.byref(s), _ptr(offsets),
                                    C.byref(grid), fields_arr,
                                    len(fields_arr), C.byref(cfg),
                                    C.byref(queue), _ptr(mask), _ptr(alloc),
                                    _ptr(stats), _stream(stream)))


def psl_stream_sample(phsp: Dict, field_arr, cfg: psl_stream_cfg,
                      queue: psl_queue, flushes, n_flushes, stats, ws,
                      stream=None):
    """Methods 1/2 source of one batch; flushes: device int64 tensor viewed
    as psl_flush records ([max_flushes, 4]), n_flushes: device int64 [1]."""
    s = make_phsp(phsp)
    _check(lib().psl_stream_sample(C.byref(s), field_arr, C.byref(cfg),
                                   C.byref(queue), _ptr(flushes),
                                   int(flushes.shape[0]), _ptr(n_flushes),
                                   _ptr(stats), _ptr(ws),
                                   ws.numel() * ws.element_size(),
                                   _stream(stream)))


def dose_point(dose, sigma, phantom: psl_phantom, point, radius,
               stream=None):
    """Reference-point dose (Sec. 2.5) of device float tensors dose, sigma:
    (mean over the voxel centres within radius, its standard error,
    count)."""
    import torch
    out = torch.zeros(3, dtype=torch.float64, device=dose.device)
    _check(lib().dose_point(_ptr(dose), _ptr(sigma), C.byref(phantom),
                            float(point[0]), float(point[1]),
                            float(point[2]), float(radius), _ptr(out),
                            _stream(stream)))
    m, se, n = (float(v) for v in out.cpu())
    return m, se, int(n)


def calibration_factor(ref_dose_per_particle, dose_per_mu):
    """Absolute calibration (Sec. 2.5): particles per MU, the calibration
    dose (Gy/MU at the reference point under reference conditions) over the
    computed dose there (Gy per particle).  Dose in Gy for a field of M
    monitor units is then D x factor x M / (1 + b), b the field's monitor
    backscatter relative to the reference field."""
    return dose_per_mu / ref_dose_per_particle


def output_factors(ref_doses, reference, backscatter=None):
    """Relative output factors (Sec. 2.5): the reference-point dose of each
    field per monitor unit relative to the reference field's, where a
    field's monitor units per particle grow by (1 + b) with its monitor
    backscatter b (from a table, the paper's BEAMnrc values; none here
    unless given).  ref_doses: {field: (dose, standard error)}; returns
    {field: (ROF, standard error)}."""
    b = backscatter or {}
    d0, s0 = ref_doses[reference]
    k0 = 1.0 + b.get(reference, 0.0)
    out = {}
    for f, (d, s) in ref_doses.items():
        k = 1.0 + b.get(f, 0.0)
        r = (d / k) / (d0 / k0)
        rel = math.hypot(s / d, s0 / d0) if f != reference else 0.0
        out[f] = (r, r * rel)
    return out


def psl_physics_init(phys: psl_physics, tables, stream=None):
    _check(lib().psl_physics_init(C.byref(phys), _ptr(tables),
                                  _stream(stream)))


def transport_batch(queue: psl_queue, phantom: psl_phantom,
                    phys: psl_physics, tables, seed: int, acc: psl_dose_acc,
                    stats, ws, launch: Optional[psl_launch] = None,
                    stream=None):
    _check(lib().transport_batch(
        C.byref(queue), C.byref(phantom), C.byref(phys), _ptr(tables),
        C.c_uint64(seed), C.byref(acc), _ptr(stats),
        C.byref(launch) if launch is not None else None, _ptr(ws),
        ws.numel() * ws.element_size(), _stream(stream)))


def dose_tally(acc: Optional[psl_dose_acc], s1, s2, op, n_batches,
               phantom: psl_phantom, norm=1.0, dose=None, sigma=None,
               stream=None):
    _check(lib().dose_tally(C.byref(acc) if acc is not None else None,
                            _ptr(s1), _ptr(s2), op, n_batches,
                            C.byref(phantom), float(norm), _ptr(dose),
                            _ptr(sigma), _stream(stream)))


class Plan:
    """A psl_plan handle: allocation once, then batches eagerly or under a
    hipGraph (psl_plan_run), optionally autotuned (psl_autotune)."""

    def __init__(self, handle, ws, stream):
        self.handle = handle
        self.ws = ws          # the plan owns its workspace until destroyed
        self.stream = stream

    def run(self, first_batch, n_batches, use_graph=True, stream=None):
        _check(lib().psl_plan_run(self.handle, int(first_batch),
                                  int(n_batches), 1 if use_graph else 0,
                                  _stream(stream or self.stream)))

    def autotune(self, trials=2, stream=None):
        r = psl_tune_result()
        _check(lib().psl_autotune(self.handle, int(trials), C.byref(r),
                                  _stream(stream or self.stream)))
        return r

    def layout(self):
        q, L = psl_queue(), psl_launch()
        _check(lib().psl_plan_get(self.handle, C.byref(q), C.byref(L)))
        return q, L

    def copy_tuning(self, src):
        """This plan takes src's launch shape and electron bucketing."""
        _check(lib().psl_plan_copy_tuning(self.handle, src.handle))

    def destroy(self):
        if self.handle:
            _check(lib().psl_plan_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class PlanPair:
    """Two plans of the same fields and sums with their own queues,
    accumulators, statistics and workspaces: batches alternate between
    them, two in flight at once (psl_plan_run_pair)."""

    def __init__(self, a, b):
        self.a, self.b = a, b
        self.stream = a.stream

    def autotune(self, trials=2, stream=None):
        """Tunes the first plan and gives the second its configuration."""
        r = self.a.autotune(trials, stream)
        self.b.copy_tuning(self.a)
        return r

    def run(self, first_batch, n_batches, use_graph=True, stream=None):
        _check(lib().psl_plan_run_pair(
            self.a.handle, self.b.handle, int(first_batch), int(n_batches),
            1 if use_graph else 0, _stream(stream or self.stream)))

    def destroy(self):
        self.a.destroy()
        self.b.destroy()


class PlanSet:
    """Plans of the same fields and sums, each with its own queues,
    accumulator, statistics and workspace: batch i runs on plan i mod n,
    n batches in flight at once (psl_plan_run_set)."""

    def __init__(self, plans):
        self.plans = list(plans)
        self.stream = self.plans[0].stream

    def autotune(self, trials=2, stream=None):
        """Tunes the first plan and gives the others its configuration."""
        r = self.plans[0].autotune(trials, stream)
        for p in self.plans[1:]:
            p.copy_tuning(self.plans[0])
        return r

    def run(self, first_batch, n_batches, stream=None):
        h = (C.c_void_p * len(self.plans))(*[p.handle for p in self.plans])
        _check(lib().psl_plan_run_set(h, len(self.plans), int(first_batch),
                                      int(n_batches),
                                      _stream(stream or self.stream)))

    def destroy(self):
        for p in self.plans:
            p.destroy()


def dose_gamma(ref, ev, voxel, dose_crit=0.02, dta=0.2, threshold=0.1,
               step=None, gamma2=None):
    """Global 3D gamma of device float tensors ref, ev [nz, ny, nx]: the dose
    criterion is dose_crit * max(ref), voxels with ref >= threshold *
    max(ref) are evaluated.  Returns (pass fraction, evaluated count)."""
    import torch
    assert ref.dtype == torch.float32 and ev.dtype == torch.float32
    assert ref.shape == ev.shape and ref.dim() == 3
    ref = ref.contiguous()
    ev = ev.contiguous()
    nz, ny, nx = ref.shape
    vz, vy, vx = (voxel,) * 3 if np.isscalar(voxel) else voxel
    mx = float(ref.max().item())
    counts = torch.zeros(2, dtype=torch.int64, device=ref.device)
    _check(lib().dose_gamma(_ptr(ref), _ptr(ev), nx, ny, nz, vx, vy, vz,
                            dose_crit * mx, dta, step or dta / 5.0,
                            threshold * mx,
                            _ptr(gamma2) if gamma2 is not None else None,
                            _ptr(counts), _stream()))
    n_eval, n_pass = (int(v) for v in counts.cpu())
    return (n_pass / n_eval if n_eval else 1.0), n_eval


def unet_set_brick_blocks(max_blocks=0):
    """Caps the grid of the finest-level brick-loop convolution (0: as many
    blocks as are resident); the results do not depend on it."""
    _check(lib().unet_set_brick_blocks(int(max_blocks)))


class Denoiser:
    """Device state of the dose denoiser (fp32 master weights, bf16 copy,
    gradients and Adam moments) and the calls on it."""

    def __init__(self, device="cuda", seed=None):
        import torch
        self.torch = torch
        n = lib().unet_param_count(4, 16)
        self.n = n
        self.params = torch.zeros(n, dtype=torch.float32, device=device)
        self.params_bf16 = torch.zeros(n, dtype=torch.int16, device=device)
        self.grads = torch.zeros(n, dtype=torch.float32, device=device)
        self.m = torch.zeros(n, dtype=torch.float32, device=device)
        self.v = torch.zeros(n, dtype=torch.float32, device=device)
        self.step_no = 0
        self.net = psl_unet()
        self.net.levels, self.net.base, self.net.n_params = 4, 16, n
        self.net.params = self.params.data_ptr()
        self.net.params_bf16 = self.params_bf16.data_ptr()
        self._ws = {}
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)
        if seed is not None:
            self.init(seed)

    def init(self, seed):
        _check(lib().unet_init(C.byref(self.net), C.c_uint64(seed),
                               _stream()))

    def set_params(self, blob):
        """Load fp32 master weights (the documented blob layout); the
        library refreshes the bf16 copy (unet_set_params)."""
        a = np.ascontiguousarray(blob, np.float32)
        if a.size != self.n:
            raise ValueError("blob holds %d floats, the network %d" %
                             (a.size, self.n))
        self.params.copy_(self.torch.from_numpy(a))
        _check(lib().unet_set_params(C.byref(self.net), _stream()))

    def _workspace(self, shape, training):
        key = (tuple(shape), training)
        if key not in self._ws:
            n, d, h, w = shape
            nb = lib().unet_workspace_bytes(C.byref(self.net), n, d, h, w,
                                            1 if training else 0)
            self._ws[key] = self.torch.empty(nb, dtype=torch_uint8(),
                                             device=self.params.device)
        return self._ws[key]

    def forward(self, dose, rho):
        """dose, rho: float32 [n, nz, ny, nx] device tensors."""
        out = self.torch.empty_like(dose)
        ws = self._workspace(dose.shape, False)
        n, d, h, w = dose.shape
        _check(lib().unet_forward(C.byref(self.net), _ptr(dose), _ptr(rho),
                                  n, d, h, w, _ptr(out), _ptr(ws), ws.numel(),
                                  _stream()))
        return out

    def backward(self, dose, rho, target):
        """Adds the loss gradient into self.grads; returns the device loss
        tensor (accumulated since the last zeroing)."""
        ws = self._workspace(dose.shape, True)
        n, d, h, w = dose.shape
        _check(lib().unet_backward(C.byref(self.net), _ptr(dose), _ptr(rho),
                                   _ptr(target), n, d, h, w,
                                   _ptr(self.grads), _ptr(self.loss),
                                   _ptr(ws), ws.numel(), _stream()))
        return self.loss

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_no += 1
        _check(lib().unet_adam_step(C.byref(self.net), _ptr(self.grads),
                                    _ptr(self.m), _ptr(self.v), lr, beta1,
                                    beta2, eps, self.step_no, _stream()))

    def denoise(self, dose, rho):
        """dose, rho: float32 [nz, ny, nx]; returns the denoised dose."""
        out = self.torch.empty_like(dose)
        ws = self._workspace((1,) + tuple(dose.shape), False)
        nz, ny, nx = dose.shape
        _check(lib().dose_denoise(_ptr(dose), _ptr(rho), nx, ny, nz,
                                  C.byref(self.net), _ptr(out), _ptr(ws),
                                  ws.numel(), _stream()))
        return out


def torch_uint8():
    import torch
    return torch.uint8


def stats_to_dict(stats_t) -> Dict:
    raw = stats_t.cpu().numpy().tobytes()
    s = psl_stats.from_buffer_copy(raw[:C.sizeof(psl_stats)])
    d = {k: int(getattr(s, k)) for k in STATS_FIELDS}
    d["e_in"], d["e_escaped"], d["e_killed"] = s.e_in, s.e_escaped, \
        s.e_killed
    return d


PROF_GROUPS = ["build", "sample", "alloc", "photons", "electrons", "fold",
               "finalize", "rebucket"]


def bench_atomics(n_addresses, device="cuda"):
    """Measured atomic roofs: (scattered u64 adds/s over n_addresses,
    same-address adds/s)."""
    import torch
    nb = lib().psl_bench_atomics_workspace_bytes(int(n_addresses))
    ws = torch.zeros(nb, dtype=torch.uint8, device=device)
    rates = (C.c_double * 2)()
    _check(lib().psl_bench_atomics(int(n_addresses), rates, _ptr(ws), nb,
                                   _stream()))
    return rates[0], rates[1]


def bench_atomics_replay(trace, n_addresses, blocks_per_cu=(1, 2, 4, 8, 16),
                         reps=3, device="cuda"):
    """Replay of a recorded deposit-address trace (device uint32 tensor) as
    u64 atomic adds over n_addresses counters, at each launch shape:
    {blocks_per_cu: adds/s}."""
    import torch
    assert trace.dtype == torch.int32 or trace.dtype == torch.uint32
    nb = lib().psl_bench_atomics_workspace_bytes(int(n_addresses))
    ws = torch.zeros(nb, dtype=torch.uint8, device=device)
    shapes = (C.c_int32 * len(blocks_per_cu))(*blocks_per_cu)
    rates = (C.c_double * len(blocks_per_cu))()
    _check(lib().psl_bench_atomics_replay(
        _ptr(trace), int(trace.numel()), int(n_addresses), shapes,
        len(blocks_per_cu), int(reps), rates, _ptr(ws), nb, _stream()))
    return {b: rates[i] for i, b in enumerate(blocks_per_cu)}


def profile_enable(on=True):
    _check(lib().psl_profile_enable(1 if on else 0))


def profile_read(reset=True):
    """{group: (milliseconds, launches)} accumulated while profiling."""
    ms = (C.c_double * 8)()
    n = (C.c_int64 * 8)()
    _check(lib().psl_profile_read(ms, n, 1 if reset else 0))
    return {g: (ms[i], n[i]) for i, g in enumerate(PROF_GROUPS)}


from .engine import Engine, Buffers  # noqa: E402,F401
