"""Batched plans: one allocation, many batches, eager or replayed from a
hipGraph, and the autotuner.  The fixed-point dose is exact integer
arithmetic and the random numbers are keyed by history, so every path must
give bit-identical tallies."""
import sys

import numpy as np
import pytest

import psl_synth as S

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _imrt(n_particles=500_000):
    wl = S.workload_imrt(n_particles=n_particles)
    wl.phantom = S.water_phantom((64, 64, 64), 0.5, (-16.0, -16.0, 84.0))
    return wl


def _engine(wl, hpb, **kw):
    import paper_1302_1861_amd as P
    return P.Engine(wl, histories_per_batch=hpb, **kw)


def test_plan_eager_equals_individual_calls():
    import torch
    wl = _imrt()
    ref = _engine(wl, 300_000)
    for b in range(3):
        ref.step(b)
    torch.cuda.synchronize()
    want = ref.s1.cpu().numpy()
    eng = _engine(wl, 300_000)
    plan = eng.make_plan()
    plan.run(0, 3, use_graph=False)
    torch.cuda.synchronize()
    got = eng.s1.cpu().numpy()
    _say("plan eager", float(got.sum()), float(want.sum()))
    assert got.any() and np.array_equal(got, want)
    plan.destroy()


def test_plan_graph_replays_equal_eager_every_batch():
    import torch
    wl = _imrt()
    eager = _engine(wl, 250_000)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        p_e = eager.make_plan()
        graphed = _engine(wl, 250_000)
        p_g = graphed.make_plan()
        for b in range(4):
            p_e.run(b, 1, use_graph=False)
            torch.cuda.current_stream().synchronize()
            want = eager.s1.cpu().numpy().copy()
            # some eager work of the program between replays
            x = torch.randn(1 << 20, device="cuda")
            y = (x * 2.0).sum()
            torch.cuda.current_stream().synchronize()
            p_g.run(b, 1, use_graph=True)
            torch.cuda.current_stream().synchronize()
            got = graphed.s1.cpu().numpy()
            _say("replay", b, float(got.sum()), float(y))
            assert np.array_equal(got, want), b
            st = graphed.stats_dict()
            assert st["histories"] == 250_000 and st["lost"] == 0
        # several replays in one call continue the batch sequence
        p_e.run(4, 3, use_graph=False)
        p_g.run(4, 3, use_graph=True)
        torch.cuda.current_stream().synchronize()
        assert np.array_equal(graphed.s1.cpu().numpy(),
                              eager.s1.cpu().numpy())
    p_e.destroy()
    p_g.destroy()


def test_autotune_choice_keeps_the_dose():
    import torch
    wl = _imrt()
    ref = _engine(wl, 200_000)
    p_r = ref.make_plan()
    p_r.run(0, 2, use_graph=False)
    torch.cuda.synchronize()
    want = ref.s1.cpu().numpy()
    eng = _engine(wl, 200_000)
    plan = eng.make_plan()
    r = plan.autotune(trials=1)
    _say("tuned", r.launch.blocks_per_cu, r.launch.rebucket, r.n_ebuckets,
         r.ms_per_batch, r.configs_tried, r.bucket_peak,
         r.el_capacity_suggested)
    assert r.configs_tried >= 20 and r.ms_per_batch > 0
    assert r.el_capacity_suggested >= r.n_ebuckets * r.bucket_peak
    assert not eng.acc_t.any().item()
    assert not eng.s1.any().item()
    plan.run(0, 2, use_graph=False)
    torch.cuda.synchronize()
    assert np.array_equal(eng.s1.cpu().numpy(), want)
    q, L = plan.layout()
    assert q.n_ebuckets == r.n_ebuckets and L.rebucket == r.launch.rebucket
    plan.destroy()
    p_r.destroy()


@pytest.mark.parametrize("use_graph", [False, True])
def test_plan_pair_equals_single_plan(use_graph):
    """Two plans of one engine, batches alternating between them with two
    in flight: the sums equal one plan's over the same batches, for odd and
    even counts, replay after replay, also after the pair's tuning
    changed."""
    import torch
    wl = _imrt()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ref = _engine(wl, 250_000)
        p_r = ref.make_plan()
        eng = _engine(wl, 250_000)
        pair = eng.make_plan_pair()
        p_r.run(0, 5, use_graph=False)
        pair.run(0, 5, use_graph=use_graph)
        torch.cuda.current_stream().synchronize()
        want = ref.s1.cpu().numpy()
        got = eng.s1.cpu().numpy()
        _say("pair", use_graph, float(got.sum()), float(want.sum()))
        assert got.any() and np.array_equal(got, want)
        assert np.array_equal(eng.s2.cpu().numpy(), ref.s2.cpu().numpy())
        # eager torch work between calls, then four more batches
        x = torch.randn(1 << 20, device="cuda")
        float((x * 3.0).sum())
        p_r.run(5, 4, use_graph=False)
        pair.run(5, 4, use_graph=use_graph)
        torch.cuda.current_stream().synchronize()
        assert np.array_equal(eng.s1.cpu().numpy(), ref.s1.cpu().numpy())
        # tuned (the first plan timed, the second given its configuration;
        # the pair's graph is captured again): the same sums
        r = pair.autotune(trials=1)
        qa, la = pair.a.layout()
        qb, lb = pair.b.layout()
        assert (la.blocks_per_cu, la.rebucket, qa.n_ebuckets) == \
            (lb.blocks_per_cu, lb.rebucket, qb.n_ebuckets) == \
            (r.launch.blocks_per_cu, r.launch.rebucket, r.n_ebuckets)
        p_r.run(9, 3, use_graph=False)
        pair.run(9, 3, use_graph=use_graph)
        torch.cuda.current_stream().synchronize()
        assert np.array_equal(eng.s1.cpu().numpy(), ref.s1.cpu().numpy())
    pair.destroy()
    p_r.destroy()


def test_plan_pair_rejects_shared_buffers():
    import paper_1302_1861_amd as P
    wl = _imrt(n_particles=100_000)
    eng = _engine(wl, 50_000)
    a = eng.make_plan()
    b = eng.make_plan()          # same queues, accumulator and statistics
    st = P.lib().psl_plan_run_pair(a.handle, b.handle, 0, 2, 0, None)
    assert st == P.PSL_EINVAL
    assert "own queues" in P.lib().psl_last_error().decode()
    a.destroy()
    b.destroy()


@pytest.mark.parametrize("n_plans,n_batches", [(3, 7), (2, 5), (1, 3),
                                               (4, 2)])
def test_plan_set_equals_single_plan(n_plans, n_batches):
    """n plans of one engine, batch i on plan i mod n, n batches in flight
    on n streams: the sums equal one plan's over the same batches (counts
    below, equal to and above n), and again after eager torch work and the
    set's tuning."""
    import torch
    wl = _imrt()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ref = _engine(wl, 250_000)
        p_r = ref.make_plan()
        eng = _engine(wl, 250_000)
        ps = eng.make_plan_set(n_plans)
        _say("case plan set n_plans=%d n_batches=%d" % (n_plans, n_batches))
        p_r.run(0, n_batches, use_graph=False)
        ps.run(0, n_batches)
        torch.cuda.current_stream().synchronize()
        want = ref.s1.cpu().numpy()
        got = eng.s1.cpu().numpy()
        assert got.any() and np.array_equal(got, want)
        assert np.array_equal(eng.s2.cpu().numpy(), ref.s2.cpu().numpy())
        x = torch.randn(1 << 20, device="cuda")
        float((x * 3.0).sum())
        ps.autotune(trials=1)
        p_r.run(n_batches, 4, use_graph=False)
        ps.run(n_batches, 4)
        torch.cuda.current_stream().synchronize()
        assert np.array_equal(eng.s1.cpu().numpy(), ref.s1.cpu().numpy())
        assert np.array_equal(eng.s2.cpu().numpy(), ref.s2.cpu().numpy())
    ps.destroy()
    p_r.destroy()


def test_plan_set_rejects_bad_sets():
    import ctypes as C
    import paper_1302_1861_amd as P
    wl = _imrt(n_particles=100_000)
    eng = _engine(wl, 50_000)
    a = eng.make_plan()
    b = eng.make_plan()          # same queues, accumulator and statistics
    h = (C.c_void_p * 2)(a.handle, b.handle)
    assert P.lib().psl_plan_run_set(h, 2, 0, 2, None) == P.PSL_EINVAL
    assert "own queues" in P.lib().psl_last_error().decode()
    h = (C.c_void_p * 2)(a.handle, a.handle)
    assert P.lib().psl_plan_run_set(h, 2, 0, 2, None) == P.PSL_EINVAL
    h = (C.c_void_p * 1)(a.handle)
    assert P.lib().psl_plan_run_set(h, 9, 0, 2, None) == P.PSL_EINVAL
    assert P.lib().psl_plan_run_set(h, 0, 0, 2, None) == P.PSL_EINVAL
    assert P.lib().psl_plan_run_set(h, 1, -1, 2, None) == P.PSL_EINVAL
    a.destroy()
    b.destroy()
