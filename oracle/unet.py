"""Plain float64 reference of the dose denoiser (test infrastructure).

The network is the one the library documents (include/psl.h): 4 levels of
16/32/64/128 channels, two 3x3x3 zero-padded convolutions with ReLU per
level and side, 2x2x2 average pooling, nearest up-sampling with the coarse
features concatenated before the skip, a 1x1 head added to the normalised
input dose, loss = mean squared error in normalised units.  Parameters are
read from the flat blob in the documented layout.  Forward and backward are
written out layer by layer; the backward is pinned by finite differences
and the convolution by scipy's correlation.
"""
from __future__ import annotations

import numpy as np

IN_C = 16
ORDER = ["enc0a", "enc0b", "enc1a", "enc1b", "enc2a", "enc2b", "enc3a",
         "enc3b", "dec2a", "dec2b", "dec1a", "dec1b", "dec0a", "dec0b"]


def layer_shapes(base=16):
    c = [base, 2 * base, 4 * base, 8 * base]
    io = [(IN_C, c[0]), (c[0], c[0]), (c[0], c[1]), (c[1], c[1]),
          (c[1], c[2]), (c[2], c[2]), (c[2], c[3]), (c[3], c[3]),
          (c[3] + c[2], c[2]), (c[2], c[2]), (c[2] + c[1], c[1]),
          (c[1], c[1]), (c[1] + c[0], c[0]), (c[0], c[0])]
    return dict(zip(ORDER, io))


def unpack(blob, base=16):
    """Flat float blob -> {layer: (W [Cout, 27, Cin], b [Cout])}, head."""
    blob = np.asarray(blob, np.float64)
    P, off = {}, 0
    for name, (ci, co) in layer_shapes(base).items():
        kp = (27 * ci + 31) // 32 * 32
        Wp = blob[off:off + co * kp].reshape(co, kp)
        off += co * kp
        P[name] = (Wp[:, :27 * ci].reshape(co, 27, ci).copy(),
                   blob[off:off + co].copy())
        off += co
    P["head"] = (blob[off:off + base].copy(), blob[off + base])
    off += base + 8
    assert off == len(blob), (off, len(blob))
    return P


def pack(P, base=16):
    out = []
    for name, (ci, co) in layer_shapes(base).items():
        kp = (27 * ci + 31) // 32 * 32
        W, b = P[name]
        Wp = np.zeros((co, kp))
        Wp[:, :27 * ci] = W.reshape(co, 27 * ci)
        out += [Wp.ravel(), b]
    wh, bh = P["head"]
    out += [np.asarray(wh, np.float64), np.array([bh]), np.zeros(7)]
    return np.concatenate(out)


# ------------------------------------------------------------- layers -----
def conv3(x, W, b):
    """x [N, D, H, W, Cin], W [Cout, 27, Cin] with offset o = (dz+1)*9 +
    (dy+1)*3 + (dx+1): y[v] = b + sum_o x[v + (dz, dy, dx)] . W[:, o]."""
    N, D, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    y = np.broadcast_to(b, (N, D, H, Wd, W.shape[0])).copy()
    for o in range(27):
        z, yy, xx = o // 9, (o // 3) % 3, o % 3
        y += xp[:, z:z + D, yy:yy + H, xx:xx + Wd, :] @ W[:, o, :].T
    return y


def conv3_back(x, W, dy):
    N, D, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for o in range(27):
        z, yy, xx = o // 9, (o // 3) % 3, o % 3
        xs = xp[:, z:z + D, yy:yy + H, xx:xx + Wd, :]
        dW[:, o, :] = np.einsum("ndhwc,ndhwk->ck", dy, xs)
        dxp[:, z:z + D, yy:yy + H, xx:xx + Wd, :] += dy @ W[:, o, :]
    db = dy.sum((0, 1, 2, 3))
    return dxp[:, 1:-1, 1:-1, 1:-1, :], dW, db


def pool(x):
    N, D, H, W, C = x.shape
    return x.reshape(N, D // 2, 2, H // 2, 2, W // 2, 2, C).mean((2, 4, 6))


def pool_back(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, 1), 2, 2), 2, 3) / 8.0


def up(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 1), 2, 2), 2, 3)


def up_back(dy):
    N, D, H, W, C = dy.shape
    return dy.reshape(N, D // 2, 2, H // 2, 2, W // 2, 2, C).sum((2, 4, 6))


# -------------------------------------------------------------- network ---
def pack_input(dose, rho):
    """dose, rho [N, D, H, W] -> (x [N, D, H, W, 16], scale [N])."""
    N = dose.shape[0]
    mx = dose.reshape(N, -1).max(1)
    scale = np.where(mx > 0, 1.0 / np.where(mx > 0, mx, 1.0), 1.0)
    x = np.zeros(dose.shape + (IN_C,))
    x[..., 0] = dose * scale[:, None, None, None]
    x[..., 1] = rho
    return x, scale


def forward(P, dose, rho, keep=False):
    x, scale = pack_input(dose, rho)
    A = {"x": x}
    h = x
    skips = []
    for l in range(4):
        for s in "ab":
            n = "enc%d%s" % (l, s)
            A[n + "_in"] = h
            h = np.maximum(conv3(h, *P[n]), 0.0)
            A[n] = h
        skips.append(h)
        if l < 3:
            h = pool(h)
    for l in (2, 1, 0):
        cat = np.concatenate([up(h), skips[l]], axis=-1)
        A["cat%d" % l] = cat
        h = cat
        for s in "ab":
            n = "dec%d%s" % (l, s)
            A[n + "_in"] = h
            h = np.maximum(conv3(h, *P[n]), 0.0)
            A[n] = h
    wh, bh = P["head"]
    out = dose * scale[:, None, None, None] + h @ wh + bh
    A["out"] = out
    A["scale"] = scale
    return (out, A) if keep else out / scale[:, None, None, None]


def loss_and_grads(P, dose, rho, target):
    out, A = forward(P, dose, rho, keep=True)
    scale = A["scale"][:, None, None, None]
    e = out - target * scale
    L = float((e * e).mean())
    g = 2.0 * e / e.size
    G = {}
    f = A["dec0b"]
    G["head"] = (np.einsum("ndhw,ndhwc->c", g, f), float(g.sum()))
    dh = g[..., None] * P["head"][0]
    skip_g = {}
    for l in (0, 1, 2):
        for s in "ba":
            n = "dec%d%s" % (l, s)
            dh = dh * (A[n] > 0)
            dx, dW, db = conv3_back(A[n + "_in"], P[n][0], dh)
            G[n] = (dW, db)
            dh = dx
        cc = dh.shape[-1] - skips_channels(l)
        skip_g[l] = dh[..., cc:]
        dh = up_back(dh[..., :cc])
    for l in (3, 2, 1, 0):
        if l < 3:
            dh = pool_back(dh) + skip_g[l]
        for s in "ba":
            n = "enc%d%s" % (l, s)
            dh = dh * (A[n] > 0)
            dx, dW, db = conv3_back(A[n + "_in"], P[n][0], dh)
            G[n] = (dW, db)
            dh = dx
    return L, G


def skips_channels(l, base=16):
    return base * 2 ** l


def grads_to_blob(G, base=16):
    P = {k: (v[0], v[1]) for k, v in G.items() if k != "head"}
    P["head"] = G["head"]
    return pack(P, base)
