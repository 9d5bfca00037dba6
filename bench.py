#!/usr/bin/env python
"""Throughput of the PSL Monte Carlo dose path on one MI355X.

Workload: the PSL method at clinical scale -- a seeded synthetic 1e7-particle
linac-like phase space (97% photons, triangular 0.1-6 MeV spectrum, 1 mm
Gaussian source, aimed over 40x40 cm at the SAD plane) pre-sorted into
2 x 32 log energy bins x 22 x 22 position bins of 5 mm at the PSL plane; a
square open field (10x10 cm by default) with ROI culling and the jaw model;
a 128^3 water phantom of 2.5 mm voxels at SSD 100 cm; 1e8 histories per
field in 10 batches of 1e7; FP32 transport, 64-bit fixed-point dose atomics.

One step = one batch of 1e7 histories through the whole hot path: ROI
selection and allocation, sampling, photon and electron transport, and the
fold of the batch tally (psl_sample -> transport_batch -> dose_tally).  The
PSL build is a commissioning step done once, before timing.  Inputs are
resident in HBM before the timed region starts.

Prints one JSON line.  `value` is histories/s of the timed steps.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_clinical_10x10.json")


KERNEL_OF_GROUP = {"photons": "k_photons<1>", "electrons": "k_electrons<1>",
                   "sample": "k_sample", "fold": "k_fold<1>"}
# the sources each kernel is compiled from
SOURCES_OF_KERNEL = {
    "k_photons<1>": ("transport.hip", "common.hpp", "compact.hpp"),
    "k_electrons<1>": ("transport.hip", "common.hpp", "compact.hpp"),
    "k_sample": ("sample.hip", "sample.hpp", "common.hpp", "compact.hpp"),
    "k_fold<1>": ("tally.hip", "common.hpp"),
}


def source_hash(kernel):
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1302_1861_amd", "csrc")
    for f in SOURCES_OF_KERNEL[kernel]:
        h.update(open(os.path.join(csrc, f), "rb").read())
    h.update(open(os.path.join(ROOT, "include", "psl.h"), "rb").read())
    return h.hexdigest()[:16]


def _traffic(group):
    """HBM bytes per launch of the group's kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, each scaled by what the counter reads
    for a plain copy of known size), or None when that kernel's sources
    changed since the counters were taken."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    k = KERNEL_OF_GROUP.get(group)
    rec = t.get("kernels", {}).get(k)
    if rec is None or rec.get("source_hash") != source_hash(k):
        return None
    return rec["bytes_per_launch"]


# Algorithmic HBM bytes (the byte model of the design notes): a queue entry
# is 44 B (E x y z u v w wt f32, uid u64, ctr u32; the queue, not a type
# byte, carries the particle type), read once by the kernel that transports
# it and written once by the kernel that creates it; a dose deposit is one
# 8 B atomic read-modify-write of the accumulator; a sampled history reads
# its 29 B phase-space particle.  Density and table reads are not counted:
# the 8.4 MB (clinical) to 42 MB (heterogeneous) density stays resident in
# the L2 and Infinity Cache.
QUEUE_ENTRY_B = 44
DEPOSIT_B = 8
PARTICLE_B = 29


def _algorithmic_bytes(group, st, nvox):
    """Algorithmic HBM bytes of one launch of a kernel group, from the
    batch statistics."""
    q = QUEUE_ENTRY_B
    if group == "electrons":
        return q * (st["electrons"] + st["secondaries"]) + \
            DEPOSIT_B * st["deposits"]
    if group == "photons":
        return (q * st["photons"] + q * st["secondaries"]
                + DEPOSIT_B * st["photon_deposits"])
    if group == "sample":
        acc = st["photons"] + st["electrons"]
        return PARTICLE_B * st["histories"] + q * acc
    if group == "fold":
        return 48 * nvox
    return None


def unet_forward_flops(shape, base=16, in_c=2):
    """Multiply-add flops of the denoiser's 3x3x3 convolutions for one
    forward pass over a volume of `shape` (4 levels, channels base * 2^l,
    two convolutions per level and side, skip concatenation).  The first
    layer counts the input's two real channels (dose, density); the
    kernels pad them to 16, and those padded products are not counted."""
    c = [base, 2 * base, 4 * base, 8 * base]
    layers = [(0, in_c, c[0]), (0, c[0], c[0]), (1, c[0], c[1]),
              (1, c[1], c[1]), (2, c[1], c[2]), (2, c[2], c[2]),
              (3, c[2], c[3]), (3, c[3], c[3]), (2, c[3] + c[2], c[2]),
              (2, c[2], c[2]), (1, c[2] + c[1], c[1]), (1, c[1], c[1]),
              (0, c[1] + c[0], c[0]), (0, c[0], c[0])]
    nz, ny, nx = shape
    return sum(2 * 27 * ci * co * (nz >> l) * (ny >> l) * (nx >> l)
               for l, ci, co in layers)


def bench_imrt(P, S, torch, hpb, n_batches, wl=None):
    """A batched plan (default: the IMRT plan, 7 beams x 20 segments),
    MU-proportional histories, autotuned: three plans of the plan's fields
    with three batches in flight on three streams (psl_plan_run_set), and
    for comparison two of them replaying a pair's hipGraph
    (psl_plan_run_pair) and one plan's own hipGraph, one batch after
    another."""
    wl = wl or S.workload_imrt()
    # graph capture needs a created stream (not the legacy null stream)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        eng = P.Engine(wl, histories_per_batch=hpb)   # isocentre at SAD
        pset = eng.make_plan_set(3, stream)
        plan = pset.plans[0]
        pair = P.PlanPair(pset.plans[0], pset.plans[1])
        r = pset.autotune(trials=1)

        def timed(run):
            eng.reset_tally()
            run(0, 3)
            stream.synchronize()
            eng.reset_tally()
            stream.synchronize()
            t0 = time.perf_counter()
            run(0, n_batches)
            stream.synchronize()
            return time.perf_counter() - t0

        dt = timed(lambda f, n: pset.run(f, n))
        dt_pair = timed(lambda f, n: pair.run(f, n, use_graph=True))
        dt_single = timed(lambda f, n: plan.run(f, n, use_graph=True))
        # kernel times of one batch run eagerly (the graph replays the same
        # launches; events are not recorded inside a captured graph)
        P.profile_read(reset=True)
        P.profile_enable(True)
        plan.run(n_batches, 1, use_graph=False)
        stream.synchronize()
        P.profile_enable(False)
        groups = _kernel_groups(P.profile_read(reset=True))
    st = eng.stats_dict()
    roof = hbm_roofline(groups, st, eng.nvox)
    atom = atomic_roofline(P, eng, groups, st, 0, replay=False)
    pset.destroy()
    return {"workload": "%s: %d fields, MU-proportional, 128^3 water at "
                        "2.5 mm, %d batches of %d histories"
                        % (wl.name, len(wl.fields), n_batches, hpb),
            "histories": n_batches * hpb, "seconds": dt,
            "histories_per_s": n_batches * hpb / dt,
            "ms_per_batch": 1e3 * dt / n_batches, "graph": False,
            "in_flight": 3,
            "pair_graph": {"histories_per_s": n_batches * hpb / dt_pair,
                           "ms_per_batch": 1e3 * dt_pair / n_batches,
                           "in_flight": 2},
            "single_plan": {"histories_per_s": n_batches * hpb / dt_single,
                            "ms_per_batch": 1e3 * dt_single / n_batches,
                            "graph": True},
            "tuned": {"blocks_per_cu": r.launch.blocks_per_cu,
                      "rebucket": r.launch.rebucket,
                      "n_ebuckets": r.n_ebuckets,
                      "configs_tried": r.configs_tried,
                      "tune_ms_per_batch": r.ms_per_batch},
            "roofline": roof, "atomic_rate": atom["achieved"],
            "kernel_ms": {g: round(v[0] / v[1], 4)
                          for g, v in groups.items()},
            "lost": st["lost"]}


def bench_denoiser(P, torch, dose, density, shape, reps=5):
    """Forward pass of the (untrained: timing does not depend on weights)
    denoiser at the benchmark volume, timed with events on the current
    stream, against the dense bf16 MFMA peak."""
    net = P.Denoiser(seed=1)
    d = dose.view(shape).contiguous()
    r = density.view(shape).contiguous()
    net.denoise(d, r)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), \
        torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        net.denoise(d, r)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    fl = unet_forward_flops(shape)
    tf = fl / (ms * 1e-3) / 1e12
    return {"volume": list(shape), "forward_ms": ms,
            "gflop_per_forward": fl / 1e9, "achieved": tf,
            "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": tf / MFMA_BF16_PEAK_TFLOPS}


def bench_time_to_accuracy(n_draws=3):
    """Live time to 1% RMS dose error (and to gamma 2%/2mm >= 99%) on
    held-out draws of the denoiser's workload (128^3 heterogeneous phantom
    at 2.5 mm, random jaws and fluence map), each judged against an
    independent 1e9-history run, for PSL + the shipped trained denoiser,
    plain MC on the same PSL engine, and the plain-unsorted analogue (file
    order, no cull, no re-bucketing).  Every side runs in the same number of
    batches per history count.  Per-draw records with every rung, and the
    geometric means of the speedups."""
    import math
    import torch
    from paper_1302_1861_amd import denoise as D
    pm = D.PairMaker((128, 128, 128), 0.25)
    pm_u = D.PairMaker((128, 128, 128), 0.25, unsorted=True)
    net = D.load_trained()
    recs = []
    for k in range(n_draws):
        recs.append(D.denoise_vs_plain(pm, net, draw=D.EVAL_SEED0 + 900 + k,
                                       pm_unsorted=pm_u))
        print("time_to_accuracy draw %d done" % k, file=sys.stderr,
              flush=True)
    pm.engines.clear()
    pm_u.engines.clear()
    del pm, pm_u, net
    torch.cuda.empty_cache()

    def gmean(crit, key):
        v = [r[crit][key] for r in recs]
        if not v or any(x is None for x in v):
            return None
        return math.exp(sum(math.log(x) for x in v) / len(v))

    out = {"draws": recs}
    for crit, tag in (("time_to_error", "1pct_rms"),
                      ("time_to_gamma", "gamma99")):
        out["speedup_to_%s_geomean" % tag] = gmean(crit, "speedup")
        out["speedup_vs_unsorted_to_%s_geomean" % tag] = gmean(
            crit, "speedup_vs_unsorted")
        out["psl_over_unsorted_to_%s_geomean" % tag] = gmean(
            crit, "psl_over_unsorted")
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(wl, hist_target_s, threads, single_s):
    """The oracle, as it stands, on a bounded sample of the same workload:
    PSL build (untimed), then one batch of sampling + transport + fold on
    `threads` threads (the headline figure) and one on a single thread."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    perm, off, nd = oracle.build_psl(wl.phsp, wl.grid)
    sps = wl.phsp.subset(perm)
    geom = oracle.geometry(wl.phantom, z_psl=wl.grid.z_plane)
    mask = oracle.cull(wl.fields, wl.grid, wl.cull, geom)
    nvox = wl.phantom.density.size
    s1 = np.zeros(nvox)
    s2 = np.zeros(nvox)

    def batch(b, H, nt):
        N, g, _ = oracle.alloc(wl.fields, wl.alloc_mode, H, off, mask,
                               wl.grid)
        S_ = oracle.sample(wl.fields, geom, off, N, g, b, wl.seed, sps)
        ok = S_["status"] == 1
        acc, _, _, _ = oracle.transport(S_["type"][ok], S_["state"][ok],
                                        S_["uid"][ok], wl.seed, wl.phantom,
                                        n_threads=nt)
        oracle.fold(acc, s1, s2)

    def timed(b, target_s, nt, probe):
        t0 = time.perf_counter()
        batch(b, probe, nt)
        rate0 = probe / max(time.perf_counter() - t0, 1e-6)
        H = int(min(max(rate0 * target_s, 20_000), 50_000_000))
        t0 = time.perf_counter()
        batch(b + 1, H, nt)
        dt = time.perf_counter() - t0
        return H / dt, H, dt

    v, H, dt = timed(0, hist_target_s, threads, 300_000)
    v1, H1, dt1 = timed(2, single_s, 1, 20_000)
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"value": v, "unit": "histories/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d histories of the same workload in one batch "
                      "(sampling + transport + fold, %.1f s, PSL build "
                      "excluded)" % (H, dt),
            "single_thread": {"value": v1, "unit": "histories/s",
                              "sample": "%d histories, %.1f s" % (H1, dt1)},
            "host": {"nproc": os.cpu_count(), "affinity": affinity,
                     "omp_num_threads": os.environ.get("OMP_NUM_THREADS"),
                     "cpu_model": _cpu_model()}}


def _kernel_groups(prof):
    return {g: v for g, v in prof.items() if v[1] > 0}


def hbm_roofline(groups, st, nvox):
    """HBM roofline of the dominant kernel (the one with the most time
    among those with algorithmic bytes defined)."""
    dom = max((g for g in groups if g in KERNEL_OF_GROUP),
              key=lambda g: groups[g][0])
    avg_ms = groups[dom][0] / groups[dom][1]
    nbytes = _algorithmic_bytes(dom, st, nvox)
    achieved = nbytes / (avg_ms * 1e-3) / 1e9
    return {"kernel": dom, "bound": "hbm", "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": _traffic(dom),
            "algorithmic_bytes_per_launch": nbytes, "avg_launch_ms": avg_ms}


def atomic_roofline(P, eng, groups, st, batch, replay=True):
    """Dose atomics of the transport kernels against the roof of their own
    address pattern: one batch's deposit addresses are recorded (trace
    mode) and replayed as u64 atomic adds at 1-16 blocks of 256 per CU;
    the roof is the fastest replay."""
    def avg(g):
        v = groups.get(g)
        return v[0] / v[1] * 1e-3 if v else 0.0
    t_ph, t_el = avg("photons"), avg("electrons")
    n_atom = st["deposits"] + st["photon_deposits"]
    achieved = n_atom / (t_ph + t_el) if t_ph + t_el > 0 else 0.0
    out = {"kernels": "photons+electrons", "achieved": achieved,
           "unit": "u64 atomic adds/s", "atomics_per_step": n_atom}
    if not replay:
        return out
    trace, n = eng.deposit_trace(batch)
    sweep = P.bench_atomics_replay(trace, eng.nvox)
    del trace
    peak = max(sweep.values())
    uniform, same = P.bench_atomics(eng.nvox)
    out.update({
        "peak": peak, "frac": achieved / peak,
        "per_kernel_frac": {
            "photons": st["photon_deposits"] / t_ph / peak if t_ph else 0,
            "electrons": st["deposits"] / t_el / peak if t_el else 0},
        "roof": "replay of %d recorded deposit addresses, best of "
                "blocks_per_cu sweep" % n,
        "replay_by_blocks_per_cu": sweep, "uniform_scatter_peak": uniform,
        "same_address_peak": same})
    return out


def measure_workload(P, torch, wl, H, steps, warmup, launch=None,
                     replay=True, source="psl", pipelined=True):
    """Times `steps` batches of H histories of one workload (after
    `warmup` batches) and derives the rooflines.  pipelined: three batches
    in flight on three streams, one batch sampled while the others are
    transported (Engine.run_pipelined; same histories and dose as one
    batch after another); kernel times are then taken from one more
    sequential pass.
    Returns (record, engine)."""
    eng = P.Engine(wl, histories_per_batch=H, launch=launch, source=source)

    def run(first, n):
        if pipelined:
            eng.run_pipelined(first, n)
        else:
            for k in range(first, first + n):
                eng.step(k)

    run(0, warmup)
    torch.cuda.synchronize()
    eng.reset_tally()
    P.profile_read(reset=True)
    P.profile_enable(not pipelined)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(0, steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if pipelined:
        # per-kernel durations from batches run one after another (events
        # around kernels that share the GPU with another stream would time
        # the sharing); these batches are not folded into the dose
        P.profile_enable(False)
        s1, s2, nf = eng.s1.clone(), eng.s2.clone(), eng.folded
        P.profile_read(reset=True)
        P.profile_enable(True)
        for k in range(steps, steps + min(steps, 5)):
            eng.step(k)
        torch.cuda.synchronize()
        eng.s1.copy_(s1)
        eng.s2.copy_(s2)
        eng.folded = nf
    P.profile_enable(False)
    groups = _kernel_groups(P.profile_read(reset=True))
    st = eng.stats_dict()
    if st["lost"]:
        raise SystemExit("queue overflow: batch invalid (%s)" % wl.name)
    d, s = eng.finalize()
    torch.cuda.synchronize()
    shp = wl.phantom.density.shape
    ref = P.dose_point(d.view(shp), s.view(shp), eng.phantom,
                       REF_POINT, REF_RADIUS)
    d = d.cpu().numpy()
    s = s.cpu().numpy()
    sel = d >= 0.5 * d.max()
    sbar = float((s[sel] / d[sel]).mean())
    rec = {"workload": wl.name, "source": source, "pipelined": pipelined,
           "batches_in_flight": eng.pipeline_depth if pipelined else 1,
           "histories_per_step": H, "steps": steps,
           "histories_per_s": steps * H / elapsed,
           "ms_per_step": 1e3 * elapsed / steps,
           "roofline": hbm_roofline(groups, st, eng.nvox),
           "atomic_roofline": atomic_roofline(P, eng, groups, st, steps,
                                              replay),
           "kernel_ms": {g: round(v[0] / v[1], 4) for g, v in groups.items()},
           "batch_stats": {k: st[k] for k in (
               "histories", "photons", "electrons", "jaw_rejected",
               "interactions", "secondaries", "segments", "deposits",
               "photon_deposits", "flights")},
           "mean_rel_sigma_50pct": sbar,
           "time_to_1pct_s": elapsed * (sbar / 0.01) ** 2,
           "reference_point_dose": {"point_cm": list(REF_POINT),
                                    "radius_cm": REF_RADIUS,
                                    "gy_per_particle": ref[0],
                                    "standard_error": ref[1],
                                    "voxels": ref[2]}}
    return rec, eng


# Reference point of the calibration and output factors: 10 cm deep on the
# central axis (SSD 100 cm), dose averaged over a sphere of 5 mm radius.
REF_POINT = (0.0, 0.0, 110.0)
REF_RADIUS = 0.5
CAL_DOSE_GY_PER_MU = 0.774e-2     # the paper's calibration condition


def output_factors(P, recs):
    """Relative output factors and the calibration factor from the
    reference-point doses of the open-field runs (records with field_cm)."""
    ref = {r["field_cm"]: (r["reference_point_dose"]["gy_per_particle"],
                           r["reference_point_dose"]["standard_error"])
           for r in recs}
    rof = P.output_factors(ref, 10.0)
    cf = P.calibration_factor(ref[10.0][0], CAL_DOSE_GY_PER_MU)
    return {"reference_point_cm": list(REF_POINT), "radius_cm": REF_RADIUS,
            "rof": {str(k): {"value": v[0], "standard_error": v[1]}
                    for k, v in sorted(rof.items())},
            "calibration_factor_particles_per_mu": cf,
            "calibration_dose_gy_per_mu": CAL_DOSE_GY_PER_MU,
            "monitor_backscatter": "none applied (no head model)"}


def bench_apr_latent(P, torch, S, n=20_000, recycling=(10, 100),
                     copies=(0, 16), seeds=8, batches=10):
    """Latent variance of a small cylindrically symmetric phase space (n
    particles aimed over a 10 cm disk) against the recycling factor, with
    and without azimuthal redistribution: for each setting, the per-voxel
    dose variance across independent phase spaces over the mean batch
    variance, voxels 2-12 cm deep at or above half the maximum there (32^3
    water at 1 cm, 10x10 cm field)."""
    import numpy as np
    out = []
    for R in recycling:
        for k in copies:
            ds, ss = [], []
            for sd in range(seeds):
                ps = S.phase_space(n, 500 + sd, 10.0, S.Z_PSL, aim="disk")
                wl = S.workload_clinical(side=10.0, n_particles=10)
                wl.phsp = ps
                wl.phantom = S.water_phantom((32, 32, 32), 1.0,
                                             (-16.0, -16.0, 100.0))
                eng = P.Engine(wl, histories_per_batch=R * n // batches,
                               apr_copies=k, apr_seed=900 + sd)
                d, sg = eng.run(batches=batches)
                torch.cuda.synchronize()
                ds.append(d.cpu().numpy().astype(np.float64))
                ss.append(sg.cpu().numpy().astype(np.float64))
                del eng
            ds, ss = np.array(ds), np.array(ss)
            m = ds.mean(0).reshape(32, 32, 32)
            win = np.zeros((32, 32, 32), bool)
            win[2:12] = True
            sel = (win & (m >= 0.5 * m[2:12].max())).ravel()
            v = float(ds[:, sel].var(0, ddof=1).mean())
            b = float((ss[:, sel] ** 2).mean())
            out.append({"recycling": R, "apr_copies": k, "voxels":
                        int(sel.sum()), "variance_across_phase_spaces": v,
                        "mean_batch_variance": b, "ratio": v / b})
            print("apr latent R=%d k=%d ratio %.2f" % (R, k, v / b),
                  file=sys.stderr, flush=True)
    return out


def bench_methods(P, torch, S, H, steps=10, sides=(4.0, 10.0, 30.0)):
    """The paper's Method 2 against Method 3 (PSL) on the open fields:
    Method 2 reads the phase space in file order and collimates every
    particle with the jaw model (on-the-fly bins of 2^20), PSL samples only
    the PSLs its ROI selects.  Both estimate the same dose; they are
    compared by the time to 1% mean uncertainty above the 50% isodose,
    T_run (sigma / 1%)^2, from `steps` batches of H histories each."""
    out = []
    for side in sides:
        wl = S.workload_clinical(side=side)
        rec = {"field_cm": side}
        for src in ("psl", "method2"):
            r, e = measure_workload(P, torch, wl, H, steps, 2, replay=False,
                                    source=src)
            del e
            torch.cuda.empty_cache()
            rec[src] = {k: r[k] for k in (
                "histories_per_s", "ms_per_step", "mean_rel_sigma_50pct",
                "time_to_1pct_s", "kernel_ms")}
            rec[src]["accepted_per_step"] = (r["batch_stats"]["photons"] +
                                             r["batch_stats"]["electrons"])
        rec["method2_over_psl_time_to_1pct"] = \
            rec["method2"]["time_to_1pct_s"] / rec["psl"]["time_to_1pct_s"]
        out.append(rec)
        print("methods %g cm done" % side, file=sys.stderr, flush=True)
    return out


def bench_build(P, torch, S, sizes=(10_000_000, 100_000_000, 500_000_000),
                reps=3):
    """psl_build (commissioning) at several phase-space sizes: the seeded
    1e7-particle clinical phase space repeated on the device to the size,
    so the key distribution is the clinical one.  Algorithmic bytes: 13
    read for the key (type, E, x, y), 29 read and 29 written for the
    payload."""
    import ctypes as C
    base = S.phase_space(10_000_000, 1002, 20.0, S.Z_PSL)
    grid = S.clinical_grid()
    g = P.make_grid(grid.e_edges, grid.x_edges, grid.y_edges, grid.z_plane)
    raw0 = P.Buffers.phsp_from_numpy(base, "cuda")
    out = []
    for n in sizes:
        rep = -(-n // base.n)
        raw = {k: v.repeat(rep)[:n].contiguous() for k, v in raw0.items()}
        srt = P.Buffers.phsp(n, "cuda")
        off = torch.zeros(grid.n_keys + 1, dtype=torch.int64, device="cuda")
        nd = torch.zeros(1, dtype=torch.int64, device="cuda")
        ws = torch.empty(P.lib().psl_build_workspace_bytes(n, C.byref(g)),
                         dtype=torch.uint8, device="cuda")
        P.psl_build(raw, g, srt, off, nd, ws)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            P.psl_build(raw, g, srt, off, nd, ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = 71.0 * n / (ms * 1e-3) / 1e9
        out.append({"particles": n, "ms": ms, "achieved": gbs,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": gbs / HBM_PEAK_GBS,
                    "algorithmic_bytes_per_particle": 71})
        print("psl_build %d particles: %.2f ms" % (n, ms), file=sys.stderr,
              flush=True)
        del raw, srt, ws
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=6)
    ap.add_argument("--field", type=float, default=10.0)
    ap.add_argument("--histories-per-step", type=int, default=10_000_000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-single-seconds", type=float, default=8.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip every measurement beside the main workload")
    ap.add_argument("--no-replay", action="store_true",
                    help="skip the atomic-roof replay of the main workload")
    ap.add_argument("--rebucket", type=int, default=None, choices=(0, 1),
                    help="re-bucket secondary electrons (default: library)")
    ap.add_argument("--blocks-per-cu", type=int, default=None)
    ap.add_argument("--extras-only", action="store_true",
                    help="only the measurements beside the main workload "
                         "(for profiling them apart from it)")
    ap.add_argument("--build-only", action="store_true",
                    help="time psl_build alone (1e7, 1e8, 5e8 particles) "
                         "and print its JSON record")
    ap.add_argument("--denoiser-only", action="store_true",
                    help="only the denoiser forward timing at 128^3, on a "
                         "synthetic dose (for profiling the denoiser alone)")
    ap.add_argument("--imrt-batches", type=int, default=100)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="device-to-device copy of this size before the "
                         "timed region (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU "
              "path (histories would shard across GPUs with one all-reduce "
              "of the fixed-point dose; not implemented). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import psl_synth as S
    import paper_1302_1861_amd as P

    H = args.histories_per_step
    launch = None
    if args.rebucket is not None or args.blocks_per_cu is not None:
        kw = {}
        if args.rebucket is not None:
            kw["rebucket"] = args.rebucket
        if args.blocks_per_cu is not None:
            kw["blocks_per_cu"] = args.blocks_per_cu
        launch = P.make_launch(**kw)

    def say(msg):
        print(msg, file=sys.stderr, flush=True)

    def extras(out, eng, main_rec=None):
        nz, ny, nx = eng.wl.phantom.density.shape
        out["denoiser"] = bench_denoiser(P, torch, eng.dose, eng.density,
                                         (nz, ny, nx))
        say("denoiser done")
        # the other open fields and the heterogeneous workload at their
        # own sizes (1e8 histories per field; 3e8 for the heterogeneous)
        out["workloads"] = []
        for side in (4.0, 30.0):
            rec, e2 = measure_workload(P, torch,
                                       S.workload_clinical(side=side), H, 10,
                                       2, launch)
            rec["field_cm"] = side
            out["workloads"].append(rec)
            del e2
            say("field %g done" % side)
        if args.field == 10.0 and main_rec is not None:
            main_rec["field_cm"] = 10.0
            out["output_factors"] = output_factors(
                P, [main_rec] + [r for r in out["workloads"]
                                 if "field_cm" in r])
        wl_h = S.workload_heterogeneous()
        rec, e2 = measure_workload(P, torch, wl_h, H,
                                   wl_h.histories // H, 2, launch)
        out["workloads"].append(rec)
        del e2
        torch.cuda.empty_cache()
        say("heterogeneous done")
        out["imrt_plan"] = bench_imrt(P, S, torch, H, args.imrt_batches)
        say("imrt done")
        out["vmat_plan"] = bench_imrt(P, S, torch, H, args.imrt_batches,
                                      wl=S.workload_vmat())
        say("vmat done")
        out["method2_vs_psl"] = bench_methods(P, torch, S, H)
        out["apr_latent_variance"] = bench_apr_latent(P, torch, S)
        out["psl_build"] = bench_build(P, torch, S)
        out["time_to_accuracy"] = bench_time_to_accuracy()

    if args.denoiser_only:
        shape = (128, 128, 128)
        g = torch.Generator(device="cuda").manual_seed(5)
        dose = torch.rand(shape, device="cuda", generator=g) + 0.1
        rho = torch.rand(shape, device="cuda", generator=g) + 0.5
        print(json.dumps({"denoiser": bench_denoiser(P, torch, dose, rho,
                                                     shape)}))
        return
    if args.build_only:
        print(json.dumps({"psl_build": bench_build(P, torch, S)}))
        return
    wl = S.workload_clinical(side=args.field)
    if args.extras_only:
        eng = P.Engine(wl, histories_per_batch=H, launch=launch)
        eng.step(0)
        eng.step(1)
        eng.finalize()
        out = {}
        extras(out, eng)
        print(json.dumps(out))
        return
    torch.cuda.synchronize()
    if args.copy_probe_mib:
        nbytes = args.copy_probe_mib << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    rec, eng = measure_workload(P, torch, wl, H, args.steps, args.warmup,
                                launch, replay=not args.no_replay)
    say("main workload done")
    out = {
        "metric": "MC histories/sec on 1 GPU; time to 1% dose uncertainty, "
                  "PSL+denoise vs plain",
        "value": rec["histories_per_s"],
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "PSL clinical scale: 1e7-particle phase space,"
                               " %gx%g cm open field, 128^3 water at 2.5 mm, "
                               "1e7 histories per step" % (args.field,
                                                           args.field),
                   "histories_per_step": H, "phase_space": wl.phsp.n,
                   "psl_grid": "2x32x22x22", "phantom": "128^3 x 2.5 mm",
                   "tally": "u64 fixed point 2^-32 MeV",
                   "parallelism": "single GPU"},
    }
    for k in ("roofline", "atomic_roofline", "kernel_ms", "batch_stats",
              "time_to_1pct_s", "mean_rel_sigma_50pct",
              "reference_point_dose"):
        out[k] = rec[k]
    # histories that passed the jaws and reached the phantom, per second
    bs = rec["batch_stats"]
    out["accepted_histories_per_s"] = rec["histories_per_s"] * (
        bs["photons"] + bs["electrons"]) / max(1, bs["histories"])
    if not args.no_extras:
        extras(out, eng, rec)
    del eng
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or \
            len(os.sched_getaffinity(0))
        wl_cpu = S.workload_clinical(side=args.field)
        out["cpu_baseline"] = cpu_baseline(wl_cpu, args.cpu_seconds, threads,
                                           args.cpu_single_seconds)
        out["cpu_baseline"]["gpu_over_cpu"] = out["value"] / \
            out["cpu_baseline"]["value"]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
