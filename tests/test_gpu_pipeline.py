"""Sampling of batch b+1 on a second stream while batch b is transported
(two queue sets in turn, or more) gives exactly the dose of the batches
run one after another: the histories are keyed by batch and history, and
the fixed-point tally sums integers."""
import numpy as np
import pytest

import psl_synth as S

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("source,depth", [("psl", 2), ("method2", 2),
                                          ("psl", 3), ("method2", 3),
                                          ("psl", 4)])
def test_pipelined_batches_equal_sequential(source, depth):
    import torch
    import paper_1302_1861_amd as P
    wl = S.workload_clinical(side=10.0, n_particles=1_000_000)
    wl.phantom = S.water_phantom((64, 64, 64), 0.5, (-16.0, -16.0, 100.0))
    a = P.Engine(wl, histories_per_batch=700_001, source=source)
    b = P.Engine(wl, histories_per_batch=700_001, source=source)
    for k in range(5):
        a.step(k)
    b.run_pipelined(0, 5, depth)
    torch.cuda.synchronize()
    assert a.folded == b.folded == 5
    assert np.array_equal(a.s1.cpu().numpy(), b.s1.cpu().numpy())
    assert np.array_equal(a.s2.cpu().numpy(), b.s2.cpu().numpy())
    sa, sb = a.stats_dict(), b.stats_dict()
    # counts exactly; the energy sums are floating-point sums whose order
    # follows the persistent kernels' work claims
    for k in sa:
        if k.startswith("e_"):
            assert sa[k] == pytest.approx(sb[k], rel=1e-12)
        else:
            assert sa[k] == sb[k], k
    assert sa["lost"] == 0
    # and again, continuing from batch 5 with the sets already made
    for k in range(5, 8):
        a.step(k)
    b.run_pipelined(5, 3, depth)
    torch.cuda.synchronize()
    assert np.array_equal(a.s1.cpu().numpy(), b.s1.cpu().numpy())
    assert a.s1.abs().sum().item() > 0
