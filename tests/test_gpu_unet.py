"""The denoiser's own kernels against its float64 reference: forward,
gradients, Adam, and the gain of a trained network over the noisy dose."""
import sys

import numpy as np
import pytest

from oracle import unet as U

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _bf16_round(a):
    import torch
    t = torch.as_tensor(np.asarray(a, np.float32))
    return t.to(torch.bfloat16).to(torch.float64).numpy()


def _setup(n=2, size=16, seed=5, shape=None):
    """shape (d, h, w) overrides the cube of side size."""
    import torch
    import paper_1302_1861_amd as P
    rng = np.random.default_rng(seed)
    P_ = {}
    for name, (ci, co) in U.layer_shapes().items():
        P_[name] = (rng.normal(0, np.sqrt(2.0 / (27 * ci)), (co, 27, ci)),
                    rng.normal(0, 0.05, co))
    P_["head"] = (rng.normal(0, 0.3, 16), 0.01)
    blob = U.pack(P_).astype(np.float32)
    net = P.Denoiser()
    net.set_params(blob)
    dims = (n,) + (tuple(shape) if shape else (size, size, size))
    dose = (rng.random(dims) + 0.1).astype(np.float32)
    rho = rng.uniform(0.2, 1.9, dims).astype(np.float32)
    tgt = (dose * 1.1 + 0.05 * rng.random(dose.shape)).astype(np.float32)
    # the reference uses the bf16-rounded weights the kernels compute with
    ref = U.unpack(_bf16_round(blob).astype(np.float64))
    ref["head"] = U.unpack(blob.astype(np.float64))["head"]
    for k in P_:
        if k != "head":
            ref[k] = (ref[k][0], U.unpack(blob.astype(np.float64))[k][1])
    T = lambda a: torch.from_numpy(a).cuda()
    return net, ref, dose, rho, tgt, T


# The LDS-staged brick kernel runs on every level whose volume tiles into
# 16 x 4 x 4 bricks, the direct-gather kernel elsewhere: 16^3 runs both,
# 32^3 adds the 32-channel level on bricks (two channel blocks per wave,
# 32-channel staging), 64^3 (one volume) the 64-channel level (one block
# per wave, several 32-channel stages).
# The last case is not a cube: bricks whose counts differ per axis at the
# finest level, direct gathers below.
# The finest level's 16 -> 16 convolutions run as a loop over bricks, each
# block walking its share with the next halo prefetched: blocks=None keeps
# the default grid (more bricks than resident blocks only at 64^3); a small
# cap puts several bricks on each block at 16^3 (13 blocks: eight XCD
# ranges of unequal length; 3: fewer blocks than XCDs, plain striding).
BLOCKS = [None, None, None, None, 13, 3]
CASES = [(16, 2, None), (32, 2, None), (64, 1, None), (0, 1, (24, 40, 48)),
         (16, 2, None), (16, 2, None)]


def _capped(blocks):
    import paper_1302_1861_amd as P
    P.unet_set_brick_blocks(blocks or 0)


@pytest.mark.parametrize("size,n,shape,blocks",
                         [c + (b,) for c, b in zip(CASES, BLOCKS)])
def test_forward_matches_reference(size, n, shape, blocks):
    import torch
    net, ref, dose, rho, tgt, T = _setup(n=n, size=size, shape=shape)
    _capped(blocks)
    try:
        out = net.forward(T(dose), T(rho))
        torch.cuda.synchronize()
    finally:
        _capped(0)
    got = out.cpu().numpy().astype(np.float64)
    want = U.forward(ref, dose.astype(np.float64), rho.astype(np.float64))
    # The kernels keep activations in bf16 (relative rounding <= 2^-9 per
    # value, rms ~1.1e-3); over 14 convolution layers in a chain the rms
    # error of the network's correction grows to ~sqrt(14) x 1.1e-3 ~ 4e-3.
    # The bound below leaves a factor of 5 on that.
    corr_g, corr_w = got - dose, want - dose
    rel = np.linalg.norm(corr_g - corr_w) / np.linalg.norm(corr_w)
    _say("forward: correction rel l2", rel)
    assert rel < 2e-2
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-2
    # Element by element: the error of each voxel's correction is a sum of
    # bf16 roundings (2^-9 relative each) through the chain, so it scales
    # with the size of the correction there and around it.  The bound is
    # 2^-9 x 32 (|correction| + its rms over the volume), checked on every
    # voxel and reported apart for the voxels on a face of the volume or of
    # a 16x4x4 brick (where the halo is read): a wrong halo, brick edge or
    # skipped offset changes a voxel by a sizeable part of its correction,
    # far above this bound.
    err = np.abs(corr_g - corr_w)
    scale = np.abs(corr_w) + np.sqrt(np.mean(corr_w ** 2))
    ratio = err / scale
    d, h, w = dose.shape[1:]
    zi, yi, xi = np.meshgrid(np.arange(d), np.arange(h), np.arange(w),
                             indexing="ij")
    edge = ((zi % 4 == 0) | (zi % 4 == 3) | (yi % 4 == 0) | (yi % 4 == 3) |
            (xi % 16 == 0) | (xi % 16 == 15) | (zi == d - 1) |
            (yi == h - 1) | (xi == w - 1))
    edge = np.broadcast_to(edge, ratio.shape)
    _say("forward: max err/scale, brick-edge voxels %.3e, interior %.3e"
         % (ratio[edge].max(), ratio[~edge].max() if (~edge).any() else 0))
    # (measured maxima 0.030-0.040 over 8k-262k voxels, alike on brick
    # edges and inside)
    bound = 32 * 2.0 ** -9
    assert ratio.max() <= bound, (ratio.max(), np.unravel_index(
        int(ratio.argmax()), ratio.shape))


@pytest.mark.parametrize("size,n,shape,blocks",
                         [(16, 2, None, None), (32, 2, None, None),
                          (0, 1, (16, 24, 32), None), (16, 2, None, 13),
                          (16, 2, None, 3)])
def test_gradients_match_reference(size, n, shape, blocks):
    import torch
    net, ref, dose, rho, tgt, T = _setup(n=n, size=size, shape=shape)
    net.loss.zero_()
    net.grads.zero_()
    _capped(blocks)
    try:
        net.backward(T(dose), T(rho), T(tgt))
        torch.cuda.synchronize()
    finally:
        _capped(0)
    g = net.grads.cpu().numpy().astype(np.float64)
    L, G = U.loss_and_grads(ref, dose.astype(np.float64),
                            rho.astype(np.float64), tgt.astype(np.float64))
    want = U.grads_to_blob(G)
    _say("loss", float(net.loss.item()), L)
    assert float(net.loss.item()) == pytest.approx(L, rel=2e-2)
    cos = g @ want / (np.linalg.norm(g) * np.linalg.norm(want))
    # per layer, weights and biases apart (all reported before asserting)
    off, bad = 0, []
    for name, (ci, co) in U.layer_shapes().items():
        kp = (27 * ci + 31) // 32 * 32
        for part, n in (("W", co * kp), ("b", co)):
            a, b = off, off + n
            off = b
            c = g[a:b] @ want[a:b] / (np.linalg.norm(g[a:b]) *
                                      np.linalg.norm(want[a:b]) + 1e-300)
            r = np.linalg.norm(g[a:b]) / (np.linalg.norm(want[a:b]) + 1e-300)
            _say(name, part, "cosine %.5f norm ratio %.4f" % (c, r))
            # the scale matters as much as the direction: Adam would hide
            # a wrong factor (a missing 1/N, a bias summed twice)
            if c < 0.99 or abs(r - 1.0) > 2e-2:
                bad.append(name + part)
    _say("gradient cosine", cos)
    assert cos >= 0.999 and not bad, bad


def test_adam_reduces_loss():
    import torch
    net, ref, dose, rho, tgt, T = _setup(n=1, size=16)
    d, r, t = T(dose), T(rho), T(tgt)
    losses = []
    for it in range(30):
        net.loss.zero_()
        net.backward(d, r, t)
        net.adam(lr=2e-3)
        losses.append(float(net.loss.item()))
    _say("losses", losses[:3], losses[-3:])
    assert losses[-1] < 0.5 * losses[0]
