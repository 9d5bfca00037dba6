"""The denoiser trained on engine-generated pairs by the library's own
kernels gains over the raw dose it is given: on held-out phantoms and
fields its output is closer to an independent high-history run."""
import sys

import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_trained_denoiser_beats_raw_dose_on_held_out_draws():
    import torch
    import paper_1302_1861_amd as P
    from paper_1302_1861_amd import denoise as D
    pm = D.PairMaker(shape=(48, 48, 48), voxel=0.5, n_particles=1_000_000)
    X, R, T = D.make_pairs(pm, 24, 200_000, 4_000_000)
    net = P.Denoiser(seed=3)
    losses = D.train(net, X, R, T, steps=240, batch=2, crop=(32, 32, 32),
                     lr=2e-3, lr_end=2e-4, log_every=40)
    assert losses[-1][1] < losses[0][1]
    recs, mean = D.evaluate(pm, net, 3, 200_000, 20_000_000)
    _say("mean", mean)
    # the denoised dose is closer to the reference than the raw dose on
    # every held-out draw, and by at least 30% in RMS on average (the
    # quantity the network is trained to reduce).  Gamma pass rates are
    # reported, not asserted: at this size they move by a fraction of a
    # percent either way, and at full size they can fall where the RMS
    # error falls (systematic errors at steep gradients).
    for r in recs:
        assert r["rms_rel_denoised"] < r["rms_rel_raw"], r
    assert mean["rms_rel_denoised"] < 0.7 * mean["rms_rel_raw"]
    _say("gamma raw", mean["gamma_raw"], "denoised", mean["gamma_denoised"])
