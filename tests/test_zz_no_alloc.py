"""psl_sample_noalloc (the sampling call with the library's static scratch,
for callers that cannot allocate) against psl_sample with a caller
workspace: queues, queue counts, statistics, ROI mask and allocation must
be byte-identical, on two calls in a row, the second smaller."""
import sys

import numpy as np
import pytest

import psl_synth as S
from gpu_util import queue_contents

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _outputs(eng, mask, alloc):
    import torch
    torch.cuda.synchronize()
    ph, el, counts = queue_contents(eng)
    return {"ph": ph, "el": el, "counts": counts.copy(),
            "stats": eng.stats.cpu().numpy().tobytes(),
            "mask": mask.cpu().numpy().copy(),
            "alloc": alloc.cpu().numpy().copy()}


def _same(a, b):
    assert np.array_equal(a["counts"], b["counts"])
    assert a["stats"] == b["stats"]
    assert np.array_equal(a["mask"], b["mask"])
    assert np.array_equal(a["alloc"], b["alloc"])
    for side in ("ph", "el"):
        for k in a[side]:
            assert a[side][k].tobytes() == b[side][k].tobytes(), (side, k)


def _run(eng, n_hist, batch, noalloc, mask, alloc):
    import paper_1302_1861_amd as P
    eng.cfg.n_histories = n_hist
    eng.cfg.batch = batch
    # stale results must not survive into the comparison
    for t in list(eng.ph_buf.values()) + list(eng.el_buf.values()):
        t.fill_(7)
    eng.counts.fill_(-1)
    eng.stats.fill_(0xA5)
    mask.fill_(0xCC)
    alloc.fill_(-7)
    if noalloc:
        P.psl_sample_noalloc(eng.sorted, eng.offsets, eng.grid, eng.fields,
                             eng.cfg, eng.queue, eng.stats, mask=mask,
                             alloc=alloc, n_sorted=eng.kept())
    else:
        P.psl_sample(eng.sorted, eng.offsets, eng.grid, eng.fields, eng.cfg,
                     eng.queue, eng.stats, eng.ws_sample, mask=mask,
                     alloc=alloc, n_sorted=eng.kept())
    return _outputs(eng, mask, alloc)


def test_noalloc_sample_matches_workspace_sample_twice():
    import torch
    import paper_1302_1861_amd as P
    wl = S.workload_clinical(side=10.0, n_particles=2_000_000)
    first, second = 1_000_000, 123_457
    eng = P.Engine(wl, histories_per_batch=first)
    n_pos = eng.grid.n_x * eng.grid.n_y
    mask = torch.empty(len(wl.fields) * n_pos, dtype=torch.uint8,
                       device="cuda")
    alloc = torch.empty(len(wl.fields) * eng.n_keys, dtype=torch.int64,
                        device="cuda")
    cap = P.lib().psl_sample_noalloc_max_bytes()
    need = P.lib().psl_sample_workspace_bytes(
        P.C.byref(eng.grid), len(wl.fields), first)
    _say("static scratch", cap, "bytes; first call needs", need)
    assert 0 < need <= cap
    for n_hist, batch in ((first, 3), (second, 4)):
        _say("case n_histories=%d batch=%d" % (n_hist, batch))
        want = _run(eng, n_hist, batch, False, mask, alloc)
        got = _run(eng, n_hist, batch, True, mask, alloc)
        assert int(want["counts"][0]) > 0
        _same(got, want)


def test_noalloc_sample_rejects_requests_beyond_its_scratch():
    import torch
    import paper_1302_1861_amd as P
    wl = S.workload_clinical(side=10.0, n_particles=200_000)
    eng = P.Engine(wl, histories_per_batch=100_000)
    cap = P.lib().psl_sample_noalloc_max_bytes()
    big = 1
    while P.lib().psl_sample_workspace_bytes(
            P.C.byref(eng.grid), len(wl.fields), big) <= cap:
        big *= 2
    eng.cfg.n_histories = big
    eng.counts.fill_(-1)
    torch.cuda.synchronize()
    with pytest.raises(P.PslError) as e:
        P.psl_sample_noalloc(eng.sorted, eng.offsets, eng.grid, eng.fields,
                             eng.cfg, eng.queue, eng.stats,
                             n_sorted=eng.kept())
    assert e.value.status == P.PSL_ENOSPC
    assert "static scratch" in str(e.value)
    torch.cuda.synchronize()
    # nothing was enqueued: the counts keep their fill
    assert np.all(eng.counts.cpu().numpy() == -1)
