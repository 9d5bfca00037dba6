"""The shipped denoiser weights match the network the library builds:
one float32 per parameter of the 4-level, 16-channel U-Net, all finite."""
import os

import numpy as np


def test_shipped_weights_match_the_parameter_count():
    import paper_1302_1861_amd as P
    from paper_1302_1861_amd import denoise as D
    assert os.path.exists(D.WEIGHTS)
    blob = np.load(D.WEIGHTS)
    assert blob.dtype == np.float32
    assert blob.shape == (P.lib().unet_param_count(4, 16),)
    assert np.isfinite(blob).all()
    assert float(np.abs(blob).max()) > 0
