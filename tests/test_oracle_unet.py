"""Pins of the denoiser's reference implementation: convolution against
scipy's n-dimensional correlation, the whole backward pass against central
finite differences (float64), and the parameter layout."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import unet as U


def test_conv3_matches_scipy_correlate():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 6, 5, 7, 3))
    W = rng.normal(size=(4, 27, 3))
    b = rng.normal(size=4)
    y = U.conv3(x, W, b)
    for n in range(2):
        for co in range(4):
            ref = np.full(x.shape[1:4], b[co])
            for ci in range(3):
                K = W[co, :, ci].reshape(3, 3, 3)   # [dz+1, dy+1, dx+1]
                ref += ndimage.correlate(x[n, ..., ci], K, mode="constant")
            np.testing.assert_allclose(y[n, ..., co], ref, rtol=1e-12,
                                       atol=1e-12)


def test_pool_up_adjoints():
    rng = np.random.default_rng(2)
    a = rng.normal(size=(1, 4, 4, 6, 3))
    b = rng.normal(size=(1, 2, 2, 3, 3))
    # <pool(a), b> = <a, pool_back(b)> and <up(b), a> = <b, up_back(a)>
    assert np.isclose((U.pool(a) * b).sum(), (a * U.pool_back(b)).sum())
    assert np.isclose((U.up(b) * a).sum(), (b * U.up_back(a)).sum())


def _problem(seed=3, n=8):
    rng = np.random.default_rng(seed)
    shapes = U.layer_shapes()
    P = {}
    for name, (ci, co) in shapes.items():
        P[name] = (rng.normal(0, np.sqrt(2.0 / (27 * ci)), (co, 27, ci)),
                   rng.normal(0, 0.05, co))
    P["head"] = (rng.normal(0, 0.3, 16), 0.01)
    dose = rng.random((1, n, n, n)) + 0.1
    rho = rng.uniform(0.2, 1.9, (1, n, n, n))
    tgt = dose * 1.1 + 0.05 * rng.random(dose.shape)
    return P, dose, rho, tgt


def test_backward_matches_finite_differences():
    P, dose, rho, tgt = _problem()
    L, G = U.loss_and_grads(P, dose, rho, tgt)
    blob = U.pack(P)
    gblob = U.grads_to_blob(G)
    assert gblob.shape == blob.shape
    rng = np.random.default_rng(4)
    # small enough not to straddle ReLU kinks (many pre-activations sit
    # close to zero), large enough for float64 round-off
    eps = 1e-7
    names = list(U.layer_shapes())
    # random directions: over everything, and confined to single layers
    dirs = [rng.normal(size=blob.shape) for _ in range(3)]
    offs, off = {}, 0
    for name, (ci, co) in U.layer_shapes().items():
        kp = (27 * ci + 31) // 32 * 32
        offs[name] = (off, off + co * kp + co)
        off += co * kp + co
    for name in ("enc0a", "enc3b", "dec2a", "dec0b"):
        d = np.zeros(blob.shape)
        a, b = offs[name]
        d[a:b] = rng.normal(size=b - a)
        dirs.append(d)
    head = np.zeros(blob.shape)
    head[off:off + 17] = rng.normal(size=17)
    dirs.append(head)
    # padding entries of W carry no gradient
    for d in dirs:
        d *= (U.pack(U.unpack(np.ones(blob.shape))) != 0)
        lp = U.loss_and_grads(U.unpack(blob + eps * d), dose, rho, tgt)[0]
        lm = U.loss_and_grads(U.unpack(blob - eps * d), dose, rho, tgt)[0]
        fd = (lp - lm) / (2 * eps)
        an = float(gblob @ d)
        assert fd == pytest.approx(an, rel=1e-5, abs=1e-10), (fd, an)


def test_layout_roundtrip_and_size():
    P, _, _, _ = _problem()
    blob = U.pack(P)
    Q = U.unpack(blob)
    for k in P:
        if k == "head":
            np.testing.assert_array_equal(Q[k][0], P[k][0])
            assert Q[k][1] == P[k][1]
        else:
            np.testing.assert_array_equal(Q[k][0], P[k][0])
            np.testing.assert_array_equal(Q[k][1], P[k][1])
    import os
    lib = os.path.join(os.path.dirname(os.path.dirname(__file__)),
                       "paper_1302_1861_amd", "libpsl.so")
    if os.path.exists(lib):
        import ctypes
        L = ctypes.CDLL(lib)
        L.unet_param_count.restype = ctypes.c_int64
        L.unet_param_count.argtypes = [ctypes.c_int32, ctypes.c_int32]
        assert L.unet_param_count(4, 16) == blob.size


def test_forward_with_zero_kernels_is_residual_plus_head():
    """With every convolution kernel zero each layer outputs ReLU of its
    bias, whatever its input, so the network's output is the input dose
    plus the head applied to ReLU(b_dec0b), in the units of the dose
    normalised by its maximum (per sample) and scaled back: out = dose +
    max(dose) (relu(b_dec0b) . w_head + b_head)."""
    rng = np.random.default_rng(7)
    P = {}
    for name, (ci, co) in U.layer_shapes().items():
        P[name] = (np.zeros((co, 27, ci)), rng.normal(0, 1.0, co))
    wh, bh = rng.normal(0, 0.3, 16), 0.05
    P["head"] = (wh, bh)
    dose = rng.random((2, 8, 8, 8)) * np.array([3.0, 0.5])[:, None, None,
                                                            None] + 0.01
    rho = rng.uniform(0.2, 1.9, dose.shape)
    out = U.forward(P, dose, rho)
    mx = dose.reshape(2, -1).max(1)[:, None, None, None]
    want = dose + mx * (np.maximum(P["dec0b"][1], 0.0) @ wh + bh)
    np.testing.assert_allclose(out, want, rtol=1e-13, atol=1e-15)
