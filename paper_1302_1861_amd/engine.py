"""Buffer management and call sequencing for one workload.

``Engine`` owns the device buffers (torch tensors) of a workload and chains
the C calls: psl_build once, then per batch psl_sample -> transport_batch ->
dose_tally(FOLD), and dose_tally(FINALIZE) at the end.  No arithmetic of the
method happens here.
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Dict, List, Optional

import numpy as np

from . import (PART_KEYS, PHSP_KEYS, PSL_ACC_F64, PSL_ACC_FIXED64,
               PSL_ACC_TRACE,
               PSL_ALLOC_COUNTS, PSL_MAX_QBUCKETS, PSL_QCOUNTS,
               PSL_TABLE_BYTES, PSL_TALLY_FINALIZE, PSL_TALLY_FOLD, lib,
               make_fields, make_grid, make_particles, make_phantom,
               make_physics, make_phsp, psl_build, psl_dose_acc,
               psl_launch, psl_physics_init, psl_queue, psl_sample,
               psl_sample_cfg, psl_stats, dose_tally, transport_batch,
               stats_to_dict, psl_stream_cfg, psl_stream_sample,
               psl_build_apr)

DEFAULT_BUCKET_EDGES = (0.0, 0.3, 0.5, 0.8, 1.2, 1.8, 2.6, 3.8)


class Buffers:
    """Device tensors of a particle SoA."""

    @staticmethod
    def phsp(n, device):
        import torch
        t = {"type": torch.zeros(max(n, 1), dtype=torch.uint8, device=device)}
        for k in PHSP_KEYS[1:]:
            t[k] = torch.zeros(max(n, 1), dtype=torch.float32, device=device)
        return t

    @staticmethod
    def phsp_from_numpy(ps, device):
        import torch
        return {k: torch.from_numpy(np.ascontiguousarray(getattr(ps, k))).to(
            device) for k in PHSP_KEYS}

    @staticmethod
    def particles(n, device):
        import torch
        t = {}
        for k in PART_KEYS:
            dt = torch.int64 if k == "uid" else (
                torch.int32 if k == "ctr" else torch.float32)
            t[k] = torch.zeros(max(n, 1), dtype=dt, device=device)
        return t


def _ws(nbytes, device):
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8,
                       device=device)


class Engine:
    """All buffers and calls for one workload on one GPU."""

    # batches in flight in run_pipelined (three measured 4% faster than two
    # on the clinical workload; four slower)
    pipeline_depth = 3

    def __init__(self, wl, device="cuda", histories_per_batch=None,
                 n_ebuckets=8, bucket_edges=DEFAULT_BUCKET_EDGES,
                 electron_factor=1.5, frac_bits=32, phys_flags=0,
                 launch: Optional[psl_launch] = None, iso=(0.0, 0.0, 100.0),
                 sad=100.0, z_jaw_x=37.0, z_jaw_y=28.0, seed=None,
                 source="psl", bin_capacity=1 << 20, apr_copies=0,
                 apr_seed=0):
        """source: "psl" (Method 3, the PSL source), or "method1" /
        "method2" (the phase space in file order with on-the-fly bins of
        bin_capacity particles, psl_stream_sample; one field).
        apr_copies >= 1 builds the PSLs from that many azimuthally
        redistributed copies of every particle (psl_build_apr, Sec. 2.3.1);
        the dose stays normalised per original phase-space particle."""
        import torch
        self.torch = torch
        self.device = device
        self.wl = wl
        self.launch = launch
        self.seed = wl.seed if seed is None else seed
        lib()
        # phase space and PSL build
        ps = wl.phsp
        self.n_phsp = ps.n
        self.grid = make_grid(wl.grid.e_edges, wl.grid.x_edges,
                              wl.grid.y_edges, wl.grid.z_plane)
        self.n_keys = 2 * self.grid.n_e * self.grid.n_x * self.grid.n_y
        raw = Buffers.phsp_from_numpy(ps, device)
        k = int(apr_copies)
        self.sorted = Buffers.phsp(ps.n * max(k, 1), device)
        self.offsets = torch.zeros(self.n_keys + 1, dtype=torch.int64,
                                   device=device)
        self.n_dropped = torch.zeros(1, dtype=torch.int64, device=device)
        from . import lib as _l
        if k >= 1:
            ws = _ws(_l().psl_build_apr_workspace_bytes(
                ps.n, k, C.byref(self.grid)), device)
            psl_build_apr(raw, self.grid, k, apr_seed, self.sorted,
                          self.offsets, self.n_dropped, ws)
        else:
            ws = _ws(_l().psl_build_workspace_bytes(ps.n,
                                                    C.byref(self.grid)),
                     device)
            psl_build(raw, self.grid, self.sorted, self.offsets,
                      self.n_dropped, ws)
        del ws
        if source not in ("psl", "method1", "method2"):
            raise ValueError("source must be psl, method1 or method2")
        self.source = source
        self.raw = raw if source != "psl" else None
        del raw
        # fields
        self.fluence = [None if f.fluence is None else
                        torch.from_numpy(np.ascontiguousarray(
                            f.fluence, np.float32)).to(device)
                        for f in wl.fields]
        self.fields = make_fields(wl.fields, self.fluence)
        # phantom and physics
        ph = wl.phantom
        self.density = torch.from_numpy(
            np.ascontiguousarray(ph.density, np.float32)).to(device)
        self.phantom = make_phantom(self.density, ph.voxel, ph.origin,
                                    float(ph.density.max()),
                                    max(float(ph.density.min()), 0.0))
        e_max = float(max(6.0, float(ps.E.max()) if ps.n else 6.0))
        self.phys = make_physics(e_max=e_max, flags=phys_flags)
        self.tables = torch.zeros(PSL_TABLE_BYTES, dtype=torch.uint8,
                                  device=device)
        psl_physics_init(self.phys, self.tables)
        # batches and queues
        self.batches = wl.batches
        self.hpb = int(wl.histories // wl.batches if histories_per_batch is None
                       else histories_per_batch)
        self.cfg = psl_sample_cfg()
        self.cfg.seed = self.seed
        self.cfg.n_histories = self.hpb
        self.cfg.cull = 1 if wl.cull else 0
        self.cfg.alloc_mode = wl.alloc_mode
        self.cfg.sad, self.cfg.z_jaw_x, self.cfg.z_jaw_y = sad, z_jaw_x, \
            z_jaw_y
        nz, ny, nx = ph.density.shape
        lo = np.array(ph.origin, np.float64)
        hi = lo + np.array([nx, ny, nz], np.float64) * np.array(ph.voxel)
        for a in range(3):
            self.cfg.iso[a] = iso[a]
            self.cfg.box_lo[a] = lo[a]
            self.cfg.box_hi[a] = hi[a]
        self.n_ebuckets = n_ebuckets
        per_bucket = int(math.ceil(electron_factor * self.hpb)) + 64
        self.ph_buf = Buffers.particles(self.hpb, device)
        self.el_buf = Buffers.particles(per_bucket * n_ebuckets, device)
        self.counts = torch.zeros(PSL_QCOUNTS, dtype=torch.int32,
                                  device=device)
        self.queue = psl_queue()
        self.queue.ph = make_particles(self.ph_buf)
        self.queue.ph.capacity = self.hpb
        self.queue.el = make_particles(self.el_buf)
        self.queue.el.capacity = per_bucket * n_ebuckets
        self.queue.n_ebuckets = n_ebuckets
        edges = list(bucket_edges[:n_ebuckets]) + [1e30]
        for i, e in enumerate(edges):
            self.queue.e_bucket_edges[i] = e
        self.queue.d_counts = self.counts.data_ptr()
        # tallies
        self.nvox = nx * ny * nz
        self.acc_mode = PSL_ACC_FIXED64 if wl.fixed_point else PSL_ACC_F64
        self.acc_t = torch.zeros(self.nvox, dtype=torch.int64 if
                                 wl.fixed_point else torch.float64,
                                 device=device)
        self.acc = psl_dose_acc()
        self.acc.mode = self.acc_mode
        self.acc.frac_bits = frac_bits
        self.acc.data = self.acc_t.data_ptr()
        self.s1 = torch.zeros(self.nvox, dtype=torch.float64, device=device)
        self.s2 = torch.zeros(self.nvox, dtype=torch.float64, device=device)
        self.dose = torch.zeros(self.nvox, dtype=torch.float32, device=device)
        self.sigma = torch.zeros(self.nvox, dtype=torch.float32,
                                 device=device)
        self.stats = torch.zeros(C.sizeof(psl_stats), dtype=torch.uint8,
                                 device=device)
        self.ws_sample = _ws(lib().psl_sample_workspace_bytes(
            C.byref(self.grid), len(wl.fields), self.hpb), device)
        self.ws_transport = _ws(lib().transport_batch_workspace_bytes(
            C.byref(self.queue)), device)
        self.n_kept = None
        self.folded = 0
        if source != "psl":
            if len(wl.fields) != 1:
                raise ValueError("the Method 1/2 source takes one field")
            self.scfg = psl_stream_cfg()
            sc = self.scfg
            sc.seed = self.seed
            sc.n_histories = self.hpb
            sc.bin_capacity = int(bin_capacity)
            sc.method = 1 if source == "method1" else 2
            self._e_edges = (C.c_float * len(wl.grid.e_edges))(
                *[float(v) for v in wl.grid.e_edges])
            sc.n_e = len(wl.grid.e_edges) - 1
            sc.e_edges = C.cast(self._e_edges, C.c_void_p)
            sc.weight = float(ps.n) / self.hpb
            sc.z_plane = wl.grid.z_plane
            sc.sad, sc.z_jaw_x, sc.z_jaw_y = sad, z_jaw_x, z_jaw_y
            for a in range(3):
                sc.iso[a] = iso[a]
                sc.box_lo[a] = lo[a]
                sc.box_hi[a] = hi[a]
            mf = self.hpb // int(bin_capacity) + 2 * sc.n_e
            self.flushes = torch.zeros((mf, 4), dtype=torch.int64,
                                       device=device)
            self.n_flushes = torch.zeros(1, dtype=torch.int64, device=device)
            self.ws_stream = _ws(lib().psl_stream_workspace_bytes(
                self.hpb, sc.n_e, int(bin_capacity)), device)

    # ------------------------------------------------- swapping inputs --
    def set_phantom(self, ph):
        """Replace the phantom by one with the same voxel count (new
        densities, voxel size, origin); the tallies are cleared."""
        nz, ny, nx = ph.density.shape
        if nx * ny * nz != self.nvox:
            raise ValueError("phantom has %d voxels, engine holds %d" %
                             (nx * ny * nz, self.nvox))
        d = self.torch.from_numpy(np.ascontiguousarray(ph.density,
                                                       np.float32))
        self.density = d.to(self.device)
        self.phantom = make_phantom(self.density, ph.voxel, ph.origin,
                                    float(ph.density.max()),
                                    max(float(ph.density.min()), 0.0))
        lo = np.array(ph.origin, np.float64)
        hi = lo + np.array([nx, ny, nz], np.float64) * np.array(ph.voxel)
        for a in range(3):
            self.cfg.box_lo[a] = lo[a]
            self.cfg.box_hi[a] = hi[a]
        self.reset_tally()

    def set_fields(self, fields):
        """Replace the fields (same number); the tallies are cleared."""
        if len(fields) != len(self.wl.fields):
            raise ValueError("field count must stay %d" % len(self.wl.fields))
        self.fluence = [None if f.fluence is None else
                        self.torch.from_numpy(np.ascontiguousarray(
                            f.fluence, np.float32)).to(self.device)
                        for f in fields]
        self.fields = make_fields(fields, self.fluence)
        self.reset_tally()

    def set_seed(self, seed):
        """New random streams (start offsets and transport)."""
        self.seed = int(seed)
        self.cfg.seed = self.seed

    # -------------------------------------------------------------------
    def kept(self) -> int:
        if self.n_kept is None:
            self.n_kept = int(self.offsets[-1].item())
        return self.n_kept

    def sample(self, batch, mask=None, alloc=None):
        if self.source != "psl":
            self.scfg.batch = batch
            psl_stream_sample(self.raw, self.fields, self.scfg, self.queue,
                              self.flushes, self.n_flushes, self.stats,
                              self.ws_stream)
            return
        self.cfg.batch = batch
        psl_sample(self.sorted, self.offsets, self.grid, self.fields,
                   self.cfg, self.queue, self.stats, self.ws_sample,
                   mask=mask, alloc=alloc, n_sorted=self.kept())

    def transport(self, batch, launch=None):
        transport_batch(self.queue, self.phantom, self.phys, self.tables,
                        self.seed, self.acc, self.stats, self.ws_transport,
                        launch if launch is not None else self.launch)

    def pipeline_launch(self, depth=None):
        """The launch shape of each of the `depth` batches in flight: the
        engine's, with its blocks per CU shared between two (4 -> 2 by
        default), so that two persistent transport grids are resident at
        once instead of one waiting for CUs the other holds; with more
        batches in flight, the others are mostly sampling at any time and
        a third grid starts as CUs free up.  The dose does not depend on
        the launch shape."""
        from . import make_launch
        depth = self.pipeline_depth if depth is None else depth
        L = self.launch if self.launch is not None else make_launch()
        return make_launch(
            blocks_per_cu=max(1, L.blocks_per_cu // min(max(depth, 1), 2)),
            rebucket=L.rebucket, n_cu=L.n_cu, block=L.block)

    def fold(self):
        dose_tally(self.acc, self.s1, self.s2, PSL_TALLY_FOLD, 0,
                   self.phantom)
        self.folded += 1

    def step(self, batch):
        """One batch of the whole hot path: sample, transport, fold."""
        self.sample(batch)
        self.transport(batch)
        self.fold()

    def finalize(self, norm=None):
        norm = 1.0 / self.n_phsp if norm is None else norm
        dose_tally(None, self.s1, self.s2, PSL_TALLY_FINALIZE, self.folded,
                   self.phantom, norm, self.dose, self.sigma)
        return self.dose, self.sigma

    def deposit_trace(self, batch, capacity=None):
        """Samples and transports one batch with the accumulator in trace
        mode: returns the voxel index of every deposit in issue order
        (device int32 tensor holding uint32 values) and the deposit count.
        The dose tallies are not touched."""
        torch = self.torch
        cap = int(capacity or 8 * self.hpb)
        buf = torch.zeros(2 + cap, dtype=torch.int32, device=self.device)
        acc = psl_dose_acc()
        acc.mode = PSL_ACC_TRACE
        acc.data = buf.data_ptr()
        acc.trace_capacity = cap
        self.sample(batch)
        transport_batch(self.queue, self.phantom, self.phys, self.tables,
                        self.seed, acc, self.stats, self.ws_transport,
                        self.launch)
        n = int(buf[:2].cpu().numpy().view(np.uint64)[0])
        if n > cap:
            raise ValueError("trace of %d deposits exceeds capacity %d"
                             % (n, cap))
        return buf[2:2 + n], n

    # ------------------------------------------ two-stream pipelining --
    _SET_KEYS = ("queue", "ph_buf", "el_buf", "counts", "stats", "ws_sample",
                 "ws_stream", "flushes", "n_flushes", "acc_t", "acc",
                 "ws_transport")

    def _make_sets(self, depth):
        """Up to `depth` sets of everything one batch holds from sampling
        to the fold (queues, counts, statistics, sampling and transport
        workspaces, the batch accumulator), each with its own stream, so
        that `depth` batches can be in flight at once."""
        torch = self.torch
        if not hasattr(self, "_sets"):
            self._sets = [{k: getattr(self, k, None)
                           for k in self._SET_KEYS}]
            self._streams = [None]       # set 0: the caller's stream
        while len(self._sets) < depth:
            self._sets.append(self._new_set(self._sets[0]))
            self._streams.append(torch.cuda.Stream())

    def _new_set(self, cur):
        torch = self.torch
        ph = {k: torch.empty_like(v) for k, v in self.ph_buf.items()}
        el = {k: torch.empty_like(v) for k, v in self.el_buf.items()}
        counts = torch.zeros_like(self.counts)
        q = psl_queue()
        C.memmove(C.addressof(q), C.addressof(self.queue), C.sizeof(q))
        q.ph = make_particles(ph)
        q.ph.capacity = self.queue.ph.capacity
        q.el = make_particles(el)
        q.el.capacity = self.queue.el.capacity
        q.d_counts = counts.data_ptr()
        acc_t = torch.zeros_like(self.acc_t)
        acc = psl_dose_acc()
        acc.mode, acc.frac_bits = self.acc.mode, self.acc.frac_bits
        acc.data = acc_t.data_ptr()

        def like(t, zero=False):
            if t is None:
                return None
            return torch.zeros_like(t) if zero else torch.empty_like(t)
        two = {"queue": q, "ph_buf": ph, "el_buf": el, "counts": counts,
               "stats": torch.zeros_like(self.stats),
               "ws_sample": like(self.ws_sample),
               "ws_stream": like(cur["ws_stream"]),
               "flushes": like(cur["flushes"], True),
               "n_flushes": like(cur["n_flushes"], True),
               "acc_t": acc_t, "acc": acc,
               "ws_transport": like(self.ws_transport)}
        return two

    def _use(self, i):
        for k, v in self._sets[i].items():
            setattr(self, k, v)

    def run_pipelined(self, first, n, depth=None):
        """Batches first .. first+n-1 on `depth` streams in turn, each with
        its own set of queues, workspaces and accumulator, so that `depth`
        batches are in flight at once (one batch's sampling or transport
        tail runs beside the others' transport); the folds into the running
        sums are chained in batch order.  The histories and, with the
        fixed-point tally, the dose equal those of step() in a loop: every
        batch keeps its own index and accumulator, and integer sums do not
        depend on order.  Each batch is transported with
        pipeline_launch(depth)."""
        torch = self.torch
        if n <= 0:
            return
        depth = self.pipeline_depth if depth is None else depth
        if depth < 1:
            raise ValueError("depth must be >= 1")
        self._make_sets(depth)
        main = torch.cuda.current_stream()
        streams = [main] + self._streams[1:depth]
        for st in streams[1:]:
            st.wait_stream(main)         # inputs and tallies ready
        folded = torch.cuda.Event()
        folded.record(main)
        launch = self.pipeline_launch(depth)
        last = 0
        for b in range(first, first + n):
            q = (b - first) % depth
            st = streams[q]
            self._use(q)
            with torch.cuda.stream(st):
                self.sample(b)
                self.transport(b, launch)
                st.wait_event(folded)
                self.fold()
                folded.record(st)
            last = q
        for st in streams[1:]:
            main.wait_stream(st)
        self._use(last)                  # stats_dict reports the last batch

    def reset_tally(self):
        self.s1.zero_()
        self.s2.zero_()
        self.acc_t.zero_()
        for st in getattr(self, "_sets", ()):
            st["acc_t"].zero_()
        self.folded = 0

    def run(self, batches=None):
        for b in range(batches or self.batches):
            self.step(b)
        return self.finalize()

    def make_plan(self, stream=None):
        """A psl_plan over this engine's fields, queues and tallies."""
        from . import Plan, _check, _ptr, _stream, make_phsp
        import torch
        stream = stream or torch.cuda.current_stream()
        need = lib().psl_plan_workspace_bytes(C.byref(self.grid),
                                              len(self.wl.fields), self.hpb,
                                              C.byref(self.queue))
        ws = _ws(need, self.device)
        h = C.c_void_p()
        srt = make_phsp(self.sorted, self.kept())
        self.cfg.batch = 0
        _check(lib().psl_plan_create(
            C.byref(h), C.byref(srt), _ptr(self.offsets), C.byref(self.grid),
            self.fields, len(self.fields), C.byref(self.cfg),
            C.byref(self.queue), C.byref(self.phantom), C.byref(self.phys),
            _ptr(self.tables), C.c_uint64(self.seed), C.byref(self.acc),
            _ptr(self.s1), _ptr(self.s2), _ptr(self.stats),
            C.byref(self.launch) if self.launch is not None else None,
            _ptr(ws), ws.numel(), _stream(stream)))
        return Plan(h, ws, stream)

    def make_plan_pair(self, stream=None):
        """Two psl_plans over this engine's fields and running sums, on the
        engine's first two sets of queues, accumulators, statistics (and
        their own plan workspaces), for psl_plan_run_pair."""
        from . import PlanPair
        self._make_sets(2)
        cur = {k: getattr(self, k, None) for k in self._SET_KEYS}
        try:
            self._use(0)
            a = self.make_plan(stream)
            self._use(1)
            b = self.make_plan(stream)
        finally:
            for k, v in cur.items():
                setattr(self, k, v)
        return PlanPair(a, b)

    def make_plan_set(self, n, stream=None):
        """n psl_plans over this engine's fields and running sums, on the
        engine's first n sets of queues, accumulators, statistics (and
        their own plan workspaces), for psl_plan_run_set."""
        from . import PlanSet
        self._make_sets(n)
        cur = {k: getattr(self, k, None) for k in self._SET_KEYS}
        plans = []
        try:
            for q in range(n):
                self._use(q)
                plans.append(self.make_plan(stream))
        finally:
            for k, v in cur.items():
                setattr(self, k, v)
        return PlanSet(plans)

    def stats_dict(self):
        """Batch statistics; `lost` includes entries a full queue region
        could not take."""
        d = stats_to_dict(self.stats)
        d["lost"] += int(self.queue_counts()[-1])
        return d

    def queue_counts(self):
        return self.counts.cpu().numpy().view(np.uint32).copy()
