"""Training pairs, training and evaluation of the dose denoiser.

The pairs come from the engine itself.  Draw k is a seeded heterogeneous
phantom (water with lung ellipsoids and bone slabs) and a random field
(jaws within +-15 cm and a 40x40 fluence map).  The input of the pair is
the dose of ``n_in`` histories.  The target is an independent run of
``n_tgt`` histories with its own seed.

When n_tgt is finite the target is itself noisy.  The noise is zero-mean
and independent of the input, so the mean-squared-error minimiser is
still the noise-free dose (Lehtinen et al. 2018, "Noise2Noise").  A
larger n_tgt only makes training converge faster.

The network is trained by the library's own kernels: unet_backward for
the forward pass, loss and gradients, and unet_adam_step for the update.
Evaluation uses held-out draws.  Both the raw ``n_in`` dose and its
denoised version are compared with an independent plain run of ``n_ref``
histories, using the RMS error above the 10% isodose and the global
gamma 2%/2mm pass rate from dose_gamma.

Run as ``python -m paper_1302_1861_amd.denoise --help``.  The weights the
package ships (data/denoiser_128.npy) were written by

    python -m paper_1302_1861_amd.denoise --draws 2000 --steps 60000 \
        --batch 4 --crop 64 64 64 --save denoiser_128.npy

at the defaults below: 128^3 phantoms at 2.5 mm, 1e7-history inputs and
1e9-history targets.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from typing import Dict, List

import numpy as np

TRAIN_SEED0 = 50_000      # draw k of the training set uses TRAIN_SEED0 + k
EVAL_SEED0 = 90_000       # held-out draws
MC_SEED_OFFSET = 7_919    # transport seeds of input / target / reference
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data",
                       "denoiser_128.npy")


def _say(*a):
    print(*a, flush=True)


class PairMaker:
    """Engines sharing one phase space and geometry, one per history count,
    and the draws of phantoms and fields."""

    def __init__(self, shape=(128, 128, 128), voxel=0.25, n_particles=None,
                 device="cuda", unsorted=False):
        """unsorted=True: the plain-method analogue -- one PSL per particle
        type holding the phase space in file order (one energy bin, one
        position bin), no ROI cull, no electron re-bucketing."""
        import dataclasses
        import psl_synth as S
        from . import make_launch
        from .engine import Engine
        self.S = S
        self.shape = tuple(shape)
        self.voxel = float(voxel)
        kw = {} if n_particles is None else {"n_particles": n_particles}
        self.wl = S.workload_heterogeneous(shape=self.shape, voxel=self.voxel,
                                           **kw)
        self.launch = None
        if unsorted:
            g = self.wl.grid
            one = S.Grid(S.linear_edges(0.0, float(self.wl.phsp.E.max()), 1),
                         g.x_edges[[0, -1]].copy(), g.y_edges[[0, -1]].copy(),
                         g.z_plane)
            self.wl = dataclasses.replace(self.wl, grid=one, cull=False)
            self.launch = make_launch(rebucket=0)
        self.Engine = Engine
        self.device = device
        self.engines: Dict[int, object] = {}

    def engine(self, hpb):
        if hpb not in self.engines:
            self.engines[hpb] = self.Engine(self.wl, device=self.device,
                                            histories_per_batch=hpb,
                                            launch=self.launch)
        return self.engines[hpb]

    def phantom(self, seed):
        nx, ny, nz = self.shape
        v = self.voxel
        return self.S.heterogeneous_phantom(
            self.shape, v, (-nx * v / 2, -ny * v / 2, self.S.SAD), seed)

    def field(self, seed):
        X1, X2, Y1, Y2 = self.S.random_jaws(seed)
        return self.S.Field(X1, X2, Y1, Y2,
                            fluence=self.S.fluence_map(seed))

    def prepare(self, ph, field, histories, batches=10):
        """The engine for `histories` histories in `batches` batches, with
        the phantom and field loaded (host-to-device copies included)."""
        eng = self.engine(int(histories // batches))
        eng.set_phantom(ph)
        eng.set_fields([field])
        return eng

    def run(self, eng, seed, batches=10):
        """Sampling, transport and tally of a prepared engine, three
        batches in flight (Engine.run_pipelined: the dose of the batches run
        one after another): dose (Gy per phase-space particle), its batch
        sigma and the density, device float32 [nz,ny,nx]."""
        eng.reset_tally()
        eng.set_seed(seed)
        eng.run_pipelined(0, batches)
        d, s = eng.finalize()
        nx, ny, nz = self.shape
        return (d.view(nz, ny, nx).clone(), s.view(nz, ny, nx).clone(),
                eng.density.view(nz, ny, nx).clone())

    def dose(self, ph, field, histories, seed, batches=10):
        """prepare() then run()."""
        return self.run(self.prepare(ph, field, histories, batches), seed,
                        batches)


def make_pairs(pm: PairMaker, n_draws, n_in, n_tgt, seed0=TRAIN_SEED0,
               tgt_batches=None):
    """Stacks of (input dose, density, target dose) on the device."""
    import torch
    nx, ny, nz = pm.shape
    X = torch.empty((n_draws, nz, ny, nx), dtype=torch.float32,
                    device=pm.device)
    R = torch.empty_like(X)
    T = torch.empty_like(X)
    for k in range(n_draws):
        s = seed0 + k
        ph, f = pm.phantom(s), pm.field(s)
        X[k], _, R[k] = pm.dose(ph, f, n_in, s)
        T[k], _, _ = pm.dose(ph, f, n_tgt, s + MC_SEED_OFFSET,
                             tgt_batches or batches_for(n_tgt))
        if (k + 1) % max(1, n_draws // 10) == 0:
            _say("pairs %d/%d" % (k + 1, n_draws))
    return X, R, T


def train(net, X, R, T, steps, batch=2, crop=None, lr=1e-3, lr_end=1e-4,
          seed=0, log_every=50):
    """Adam with a cosine-decayed learning rate over random draws, random
    crops (a multiple of 8 per axis) and random flips across the beam
    (x and y).  Returns the loss history (normalised units)."""
    import torch
    g = np.random.default_rng(seed)
    n, nz, ny, nx = X.shape
    cz, cy, cx = (nz, ny, nx) if crop is None else crop
    losses = []
    for it in range(steps):
        idx = torch.as_tensor(g.choice(n, size=batch, replace=n < batch),
                              device=X.device)
        z0, y0, x0 = (int(g.integers(0, d - c + 1)) for d, c in
                      ((nz, cz), (ny, cy), (nx, cx)))
        sl = (idx, slice(z0, z0 + cz), slice(y0, y0 + cy),
              slice(x0, x0 + cx))
        d, r, t = X[sl], R[sl], T[sl]
        dims = [a for a, flip in ((2, g.random() < 0.5), (3, g.random() < 0.5))
                if flip]
        if dims:
            d, r, t = (torch.flip(a, dims) for a in (d, r, t))
        d, r, t = d.contiguous(), r.contiguous(), t.contiguous()
        net.loss.zero_()
        net.backward(d, r, t)
        frac = it / max(1, steps - 1)
        net.adam(lr=lr_end + 0.5 * (lr - lr_end) * (1 + math.cos(math.pi *
                                                                 frac)))
        if (it + 1) % log_every == 0 or it == steps - 1:
            losses.append((it + 1, float(net.loss.item())))
            _say("step %d loss %.4e" % losses[-1])
    return losses


def _rms_rel(a, ref, sel, mx):
    return float(((a - ref)[sel].double().pow(2).mean().sqrt() / mx).item())


def load_trained(path=WEIGHTS, device="cuda"):
    """A Denoiser holding fp32 weights saved by main() (``--save``)."""
    from . import Denoiser
    net = Denoiser(device=device)
    blob = np.load(path)
    if blob.dtype != np.float32 or blob.shape != (net.n,):
        raise ValueError("%s: expected float32[%d], found %s%s"
                         % (path, net.n, blob.dtype, blob.shape))
    net.set_params(blob)
    return net


def evaluate(pm: PairMaker, net, n_draws, n_in, n_ref, seed0=EVAL_SEED0,
             ref_batches=None):
    """Held-out draws: raw and denoised n_in doses against an independent
    n_ref reference.  Returns per-draw records and their means."""
    import torch
    from . import dose_gamma
    recs = []
    pm.engine(int(n_in // 10))
    for k in range(n_draws):
        s = seed0 + k
        ph, f = pm.phantom(s), pm.field(s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        raw, sraw, rho = pm.dose(ph, f, n_in, s)
        torch.cuda.synchronize()
        t_mc = time.perf_counter() - t0
        t0 = time.perf_counter()
        den = net.denoise(raw, rho)
        torch.cuda.synchronize()
        t_den = time.perf_counter() - t0
        ref, sref, _ = pm.dose(ph, f, n_ref, s + 2 * MC_SEED_OFFSET,
                               ref_batches or batches_for(n_ref))
        mx = float(ref.max().item())
        sel = ref >= 0.1 * mx
        sel50 = ref >= 0.5 * mx
        # reference noise (relative to the maximum) inside the region
        s_ref = float(sref[sel].double().pow(2).mean().sqrt().item() / mx)
        e_raw = _rms_rel(raw, ref, sel, mx)
        e_den = _rms_rel(den, ref, sel, mx)
        g_raw, n_ev = dose_gamma(ref, raw, pm.voxel)
        g_den, _ = dose_gamma(ref, den, pm.voxel)
        # mean relative batch sigma of the raw run above 50% (time-to-1%)
        sbar = float((sraw[sel50] / ref[sel50]).mean().item())
        # error of the denoised dose net of the reference's own noise, and
        # the plain histories that reach it (error ~ 1/sqrt(N))
        c_raw = math.sqrt(max(e_raw ** 2 - s_ref ** 2, 1e-30))
        c_den = math.sqrt(max(e_den ** 2 - s_ref ** 2, 1e-30))
        n_eq = n_in * (c_raw / c_den) ** 2
        recs.append({"draw": s, "voxels_evaluated": n_ev,
                     "rms_rel_raw": e_raw, "rms_rel_denoised": e_den,
                     "rms_rel_reference_noise": s_ref,
                     "gamma_raw": g_raw, "gamma_denoised": g_den,
                     "sigma_bar_raw_50pct": sbar,
                     "mc_seconds": t_mc, "denoise_seconds": t_den,
                     "plain_histories_same_error": n_eq,
                     "speedup_same_error": (n_eq / n_in * t_mc)
                     / (t_mc + t_den)})
        _say(json.dumps(recs[-1]))
    keys = [k for k in recs[0] if k != "draw"]
    mean = {k: float(np.mean([r[k] for r in recs])) for k in keys}
    return recs, mean


def batches_for(n, max_hpb=10_000_000):
    """At least 10 batches and at most max_hpb histories per batch."""
    return max(10, -(-int(n) // max_hpb))


def time_to_gamma(pm: PairMaker, ph, field, ref, ladder, seed, target=0.99,
                  voxel=None):
    """Smallest history count of `ladder` whose dose passes gamma 2%/2mm
    against `ref` at >= target, with its GPU seconds (sampling, transport,
    tally), or None; and the pass rate at every rung tried."""
    import torch
    from . import dose_gamma
    for n in ladder:        # engines (PSL build, buffers) outside the timing
        pm.engine(int(n // batches_for(n)))
    rungs = []
    for n in ladder:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d, _, _ = pm.dose(ph, field, n, seed, batches_for(n))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        g, _ = dose_gamma(ref, d, voxel or pm.voxel)
        rungs.append({"histories": n, "seconds": dt, "gamma": g})
        if g >= target:
            return rungs[-1], rungs
    return None, rungs


class _Judge:
    """Error of a dose against an independent plain reference run: the RMS
    difference over voxels at or above 10% of the reference maximum, over
    that maximum, with the reference's own noise (its batch sigma, same
    region) taken out in quadrature; and the gamma 2%/2mm pass rate."""

    def __init__(self, ref, sref, voxel):
        self.ref, self.voxel = ref, voxel
        self.mx = float(ref.max().item())
        self.sel = ref >= 0.1 * self.mx
        self.s_ref = float(sref[self.sel].double().pow(2).mean().sqrt()
                           .item() / self.mx)

    def __call__(self, d):
        from . import dose_gamma
        e = _rms_rel(d, self.ref, self.sel, self.mx)
        g, _ = dose_gamma(self.ref, d, self.voxel)
        return math.sqrt(max(e * e - self.s_ref ** 2, 0.0)), g


PLAIN_LADDER = tuple(int(v) for v in (1e6, 2e6, 3e6, 5e6, 7e6, 1e7, 1.5e7,
                                       2e7, 3e7, 5e7, 7e7, 1e8, 1.5e8, 2e8))
DENOISED_LADDER = tuple(int(v) for v in (3e6, 5e6, 1e7, 2e7, 5e7))


def tally_batches(n, max_hpb=10_000_000):
    """The fewest batches the tally accepts (two) with at most max_hpb
    histories each.  Every side of the time-to-accuracy comparison runs at
    this count: all of them are judged against an independent reference,
    none by its own batch sigma."""
    return max(2, -(-int(n) // max_hpb))


def denoise_vs_plain(pm: PairMaker, net, draw=EVAL_SEED0 + 900,
                     n_ref=int(1e9), target=0.01, gamma_target=0.99,
                     in_ladder=DENOISED_LADDER, plain_ladder=PLAIN_LADDER,
                     pm_unsorted: PairMaker = None):
    """Time to a dose accuracy on one held-out draw, for three variants
    judged the same way:
      * psl_denoise: the PSL engine at `in_ladder` histories, then the
        network;
      * plain: the same PSL engine without the network (plain MC);
      * plain_unsorted (if pm_unsorted is given): the plain-method analogue,
        phase space in file order, no ROI cull, no re-bucketing.
    Every rung runs in the same number of batches for a given history count
    (tally_batches), so the per-batch cost is the same on every side.

    Accuracy is judged against an independent n_ref run (_Judge): RMS error
    <= `target` of the maximum, and gamma 2%/2mm >= `gamma_target`.  Every
    rung is a live, timed run (sampling, transport, tally and, for the
    denoised rungs, the network) with engines built and the phantom and
    field loaded beforehand.  A variant's time to a criterion is the fastest
    rung that meets it; `speedup` is plain's time over psl_denoise's."""
    import torch

    def timed(maker, n, seed, den):
        # the phantom and field upload is common to every side and stays
        # outside the clock
        nb = tally_batches(n)
        eng = maker.prepare(ph, f, n, nb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d, _, rho = maker.run(eng, seed, nb)
        if den:
            d = net.denoise(d, rho)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        err, g = judge(d)
        return {"histories": int(n), "batches": nb, "seconds": dt,
                "rms_error": err, "gamma": g}

    ph, f = pm.phantom(draw), pm.field(draw)
    ref, sref, _ = pm.dose(ph, f, n_ref, draw + 3 * MC_SEED_OFFSET,
                           batches_for(n_ref))
    judge = _Judge(ref, sref, pm.voxel)
    makers = [(pm, plain_ladder), (pm, in_ladder)]
    if pm_unsorted is not None:
        makers.append((pm_unsorted, plain_ladder))
    for maker, ladder in makers:
        for n in ladder:
            maker.engine(int(n // tally_batches(n)))
    timed(pm, in_ladder[0], draw + 5 * MC_SEED_OFFSET, True)       # warm-up
    seed = draw + 4 * MC_SEED_OFFSET
    den = [timed(pm, n, seed, True) for n in in_ladder]
    plain = [timed(pm, n, seed, False) for n in plain_ladder]
    unsorted = []
    if pm_unsorted is not None:
        timed(pm_unsorted, plain_ladder[0], draw + 5 * MC_SEED_OFFSET, False)
        unsorted = [timed(pm_unsorted, n, seed, False) for n in plain_ladder]

    def first(rungs, key, ok):
        hit = [r for r in rungs if ok(r[key])]
        return min(hit, key=lambda r: r["seconds"]) if hit else None

    def ratio(a, b):
        return a["seconds"] / b["seconds"] if a and b else None

    err_ok = (lambda v: v <= target)
    gam_ok = (lambda v: v >= gamma_target)
    out = {"draw": draw, "voxel_cm": pm.voxel, "shape": list(pm.shape),
           "reference_histories": int(n_ref),
           "reference_noise": judge.s_ref,
           "criterion": {"rms_error_of_max": target,
                         "gamma_2pct_2mm": gamma_target},
           "batches": "tally_batches(n) = max(2, ceil(n / 1e7)) on every "
                      "side"}
    for name, key, ok in (("time_to_error", "rms_error", err_ok),
                          ("time_to_gamma", "gamma", gam_ok)):
        rec = {"plain": first(plain, key, ok),
               "psl_denoise": first(den, key, ok)}
        if pm_unsorted is not None:
            rec["plain_unsorted"] = first(unsorted, key, ok)
        rec["speedup"] = ratio(rec["plain"], rec["psl_denoise"])
        if pm_unsorted is not None:
            rec["speedup_vs_unsorted"] = ratio(rec["plain_unsorted"],
                                               rec["psl_denoise"])
            rec["psl_over_unsorted"] = ratio(rec["plain_unsorted"],
                                             rec["plain"])
        out[name] = rec
    out["rungs_denoised"] = den
    out["rungs_plain"] = plain
    if pm_unsorted is not None:
        out["rungs_plain_unsorted"] = unsorted
    return out


def compare_time_to_gamma(pm: PairMaker, pm_plain: PairMaker, net, n_draws,
                          n_in, n_ref, ladder, seed0=EVAL_SEED0 + 500):
    """Time to gamma 2%/2mm >= 99% against an independent n_ref plain run:
    plain method (file order, no cull), PSL, and PSL + denoiser."""
    import torch
    from . import dose_gamma
    out = []
    for k in range(n_draws):
        s = seed0 + k
        ph, f = pm.phantom(s), pm.field(s)
        ref, _, _ = pm.dose(ph, f, n_ref, s + 3 * MC_SEED_OFFSET,
                            batches_for(n_ref))
        hit_psl, r_psl = time_to_gamma(pm, ph, f, ref, ladder, s)
        hit_pl, r_pl = time_to_gamma(pm_plain, ph, f, ref, ladder, s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        raw, _, rho = pm.dose(ph, f, n_in, s + 4 * MC_SEED_OFFSET)
        den = net.denoise(raw, rho)
        torch.cuda.synchronize()
        t_dn = time.perf_counter() - t0
        g_dn, _ = dose_gamma(ref, den, pm.voxel)
        rec = {"draw": s, "psl": hit_psl, "plain_unsorted": hit_pl,
               "psl_denoise": {"histories": n_in, "seconds": t_dn,
                               "gamma": g_dn},
               "ladder_psl": r_psl, "ladder_plain": r_pl}
        out.append(rec)
        _say(json.dumps({k2: rec[k2] for k2 in ("draw", "psl",
                                                "plain_unsorted",
                                                "psl_denoise")}))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--shape", type=int, nargs=3, default=(128, 128, 128))
    ap.add_argument("--voxel", type=float, default=0.25)
    ap.add_argument("--draws", type=int, default=2000)
    ap.add_argument("--n-in", type=float, default=1e7)
    ap.add_argument("--n-tgt", type=float, default=1e9)
    ap.add_argument("--n-ref", type=float, default=1e9)
    ap.add_argument("--eval-draws", type=int, default=8)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=2)
    ap.add_argument("--crop", type=int, nargs=3, default=(64, 64, 64))
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--gamma-draws", type=int, default=4,
                    help="held-out draws for the time-to-gamma comparison")
    ap.add_argument("--ladder", type=float, nargs="+",
                    default=(1e7, 2e7, 5e7, 1e8, 2e8, 5e8, 1e9))
    ap.add_argument("--out", default=None, help="JSON report path")
    ap.add_argument("--save", default=None, help="fp32 weights (.npy)")
    a = ap.parse_args(argv)
    import torch
    from . import Denoiser
    t_all = time.perf_counter()
    pm = PairMaker(tuple(a.shape), a.voxel)
    t0 = time.perf_counter()
    X, R, T = make_pairs(pm, a.draws, int(a.n_in), int(a.n_tgt))
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    net = Denoiser(seed=a.seed)
    t0 = time.perf_counter()
    losses = train(net, X, R, T, a.steps, a.batch, tuple(a.crop), a.lr,
                   seed=a.seed)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del X, R, T
    if a.save:
        np.save(a.save, net.params.cpu().numpy())
        _say("saved", a.save)
    recs, mean = evaluate(pm, net, a.eval_draws, int(a.n_in), int(a.n_ref))
    ttg = []
    if a.gamma_draws:
        pm_plain = PairMaker(tuple(a.shape), a.voxel, unsorted=True)
        ttg = compare_time_to_gamma(pm, pm_plain, net, a.gamma_draws,
                                    int(a.n_in), int(a.n_ref),
                                    [int(n) for n in a.ladder])
    rep = {"shape": list(a.shape), "voxel_cm": a.voxel, "draws": a.draws,
           "n_in": a.n_in, "n_tgt": a.n_tgt, "n_ref": a.n_ref,
           "steps": a.steps, "batch": a.batch, "crop": list(a.crop),
           "pair_seconds": t_pairs, "train_seconds": t_train,
           "ms_per_train_step": 1e3 * t_train / max(1, a.steps),
           "losses": losses, "eval_mean": mean, "eval": recs,
           "time_to_gamma": ttg,
           "total_seconds": time.perf_counter() - t_all}
    _say(json.dumps({"eval_mean": mean}))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rep, f, indent=1)
    return rep


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
