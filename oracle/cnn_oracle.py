"""CPU oracle for the learned refinement tagger -- TEST INFRASTRUCTURE ONLY.

Plain FP64 numpy; only tests/, __graft_entry__.smoke() and the CPU-baseline
leg of bench.py may use it.  It shares no code with the library.

What it computes (a small convolutional network that predicts, per patch,
whether the plain tagger of Section 4.1 will ask to refine or coarsen it over
the next 16 steps):

  features   for a leaf at level l: a 24 x 24 pixel window covering the 3 x 3
             block of level-l patch squares centred on the leaf, 8 x 8 pixels
             per patch square (each pixel a square of 4 x 4 level-l cells).
             A pixel holds the mean over its square of the piecewise-constant
             leaf fields: h, hu, hv and b - b_leaf (b_leaf = mean bed of the
             leaf itself), scaled by 1, 1/10, 1/10, 1/10.  Pixels outside the
             domain are 0.
  network    conv 3x3 stride 1, 4 -> 16 channels (24 x 24), ReLU;
             conv 3x3 stride 2, 16 -> 32 (12 x 12), ReLU;
             conv 3x3 stride 2, 32 -> 32 (6 x 6), ReLU;
             mean over the 36 pixels; fully connected 32 -> 3 logits
             (classes: 0 coarsen, 1 keep, 2 refine).  Zero padding of 1.
  loss       class-weighted cross-entropy, sum of w[y_i] (-log p_i[y_i])
             divided by the sum of w[y_i].
  optimiser  Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction.

emulate=True rounds to bfloat16 (round to nearest even, through float32) at the
points where the GPU kernels round: the input features, the three conv weight
tensors, the post-ReLU activations of layers 1 and 2, and the three
pre-activation gradients that enter the matrix products.  Everything else
(biases, layer-3 activations, pooling, the fully connected layer, the loss)
stays unrounded; sums are FP64 here and FP32 on the GPU.

Parameter vector layout (all float): W1[16][3][3][4], b1[16], W2[32][3][3][16],
b2[32], W3[32][3][3][32], b3[32], Wf[3][32], bf[3].
"""
from __future__ import annotations

import numpy as np

C_IN, C1, C2, C3, NCLS = 4, 16, 32, 32, 3
TILE = 24
FEATURE_SCALE = np.array([1.0, 0.1, 0.1, 0.1])

PARAM_SHAPES = [("W1", (C1, 3, 3, C_IN)), ("b1", (C1,)), ("W2", (C2, 3, 3, C1)), ("b2", (C2,)),
                ("W3", (C3, 3, 3, C2)), ("b3", (C3,)), ("Wf", (NCLS, C3)), ("bf", (NCLS,))]
N_PARAMS = int(sum(np.prod(s) for _, s in PARAM_SHAPES))


def unpack(flat: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in PARAM_SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in PARAM_SHAPES])


# ---------------------------------------------------------------------------
# bfloat16 rounding: to float32 (nearest even), then keep the upper 16 bits of
# the float32 pattern, rounding to nearest even on the lower 16.
# ---------------------------------------------------------------------------
def bf16(x) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    nan = np.isnan(a)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    r = u.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, r)


# ---------------------------------------------------------------------------
# features
# ---------------------------------------------------------------------------
def _finest_images(sc, leaves, st, Lf):
    """Fields h, hu, hv, b of the leaves projected (piecewise constant) onto
    the uniform level-Lf grid: arrays (NJ, NI)."""
    m = sc.m
    NI, NJ = sc.mi * m << Lf, sc.mj * m << Lf
    img = np.zeros((4, NJ, NI))
    for k, (t, l, ix, iy) in enumerate(np.asarray(leaves)):
        r = 1 << (Lf - l)
        PI = (t % sc.mi) * (1 << l) + ix
        PJ = (t // sc.mi) * (1 << l) + iy
        for f in range(4):
            img[f, PJ * m * r:(PJ + 1) * m * r, PI * m * r:(PI + 1) * m * r] = np.kron(st[k, f], np.ones((r, r)))
    return img


def features(sc, leaves, st) -> np.ndarray:
    """(n, 24, 24, 4) feature tiles, [y][x][channel], for leaves (n, 4) =
    (tree, level, ix, iy) with states st (n, 4, m, m) = h, hu, hv, b."""
    leaves = np.asarray(leaves)
    m = sc.m
    Lf = int(leaves[:, 1].max())
    img = _finest_images(sc, leaves, st, Lf)
    pix = {}
    out = np.zeros((leaves.shape[0], TILE, TILE, 4))
    for k, (t, l, ix, iy) in enumerate(leaves):
        l = int(l)
        if l not in pix:
            ps = (m // 8) << (Lf - l)          # finest cells per pixel side
            NJ, NI = img.shape[1] // ps, img.shape[2] // ps
            p = img.reshape(4, NJ, ps, NI, ps).mean(axis=(2, 4))
            pix[l] = np.pad(p, ((0, 0), (8, 8), (8, 8)))   # zero outside the domain
        p = pix[l]
        PI = (t % sc.mi) * (1 << l) + ix
        PJ = (t // sc.mi) * (1 << l) + iy
        win = p[:, 8 * PJ:8 * PJ + TILE, 8 * PI:8 * PI + TILE]     # pixel 8 PJ - 8 .. in padded coordinates
        inside = np.zeros((TILE, TILE), bool)
        NJp, NIp = p.shape[1] - 16, p.shape[2] - 16
        yy = np.arange(8 * PJ - 8, 8 * PJ + 16)
        xx = np.arange(8 * PI - 8, 8 * PI + 16)
        inside[:, :] = ((yy >= 0) & (yy < NJp))[:, None] & ((xx >= 0) & (xx < NIp))[None, :]
        bleaf = st[k, 3].mean()
        tile = np.moveaxis(win, 0, -1).copy()
        tile[..., 3] = np.where(inside, tile[..., 3] - bleaf, 0.0)
        out[k] = tile * FEATURE_SCALE
    return out


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def _pad(X):
    return np.pad(X, ((0, 0), (1, 1), (1, 1), (0, 0)))


def conv3x3(X, W, b, stride):
    """Y[n, oy, ox, co] = b[co] + sum over ky, kx, ci of
    X[n, s oy + ky - 1, s ox + kx - 1, ci] W[co, ky, kx, ci] (zero outside)."""
    N, H, Wd, _ = X.shape
    Ho, Wo = (H - 1) // stride + 1, (Wd - 1) // stride + 1
    Xp = _pad(X)
    Y = np.zeros((N, Ho, Wo, W.shape[0])) + b
    for ky in range(3):
        for kx in range(3):
            sl = Xp[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride, :]
            Y += sl @ W[:, ky, kx, :].T
    return Y


def conv3x3_wgrad(X, dY, stride):
    """dW[co, ky, kx, ci] = sum over n, oy, ox of X[n, s oy + ky - 1, s ox + kx - 1, ci] dY[n, oy, ox, co]."""
    N, Ho, Wo, Co = dY.shape
    Xp = _pad(X)
    dW = np.zeros((Co, 3, 3, X.shape[3]))
    for ky in range(3):
        for kx in range(3):
            sl = Xp[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride, :]
            dW[:, ky, kx, :] = np.einsum("nyxo,nyxi->oi", dY, sl)
    return dW


def conv3x3_xgrad(dY, W, stride, in_shape):
    """dX[n, y, x, ci] = sum over the output pixels (oy, ox) and taps (ky, kx)
    with s oy + ky - 1 = y and s ox + kx - 1 = x of dY[n, oy, ox, co] W[co, ky, kx, ci]."""
    N, H, Wd, Ci = in_shape
    _, Ho, Wo, _ = dY.shape
    dXp = np.zeros((N, H + 2, Wd + 2, Ci))
    for ky in range(3):
        for kx in range(3):
            dXp[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride, :] += dY @ W[:, ky, kx, :]
    return dXp[:, 1:-1, 1:-1, :]


def forward(params: np.ndarray, X: np.ndarray, emulate: bool = False):
    """Logits (n, 3) and the values the backward pass needs."""
    p = unpack(params)
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    X0 = r(X)
    W1, W2, W3 = r(p["W1"]), r(p["W2"]), r(p["W3"])
    Y1 = conv3x3(X0, W1, p["b1"], 1)
    A1 = r(np.maximum(Y1, 0.0))
    Y2 = conv3x3(A1, W2, p["b2"], 2)
    A2 = r(np.maximum(Y2, 0.0))
    Y3 = conv3x3(A2, W3, p["b3"], 2)
    A3 = np.maximum(Y3, 0.0)
    P = A3.mean(axis=(1, 2))
    Z = P @ p["Wf"].T + p["bf"]
    cache = dict(X0=X0, W1=W1, W2=W2, W3=W3, A1=A1, A2=A2, Y3=Y3, P=P, Wf=p["Wf"], emulate=emulate)
    return Z, cache


def loss(Z: np.ndarray, y: np.ndarray, class_w: np.ndarray):
    """Weighted cross-entropy and its gradient with respect to the logits."""
    Z = np.asarray(Z, dtype=np.float64)
    e = np.exp(Z - Z.max(axis=1, keepdims=True))
    p = e / e.sum(axis=1, keepdims=True)
    w = np.asarray(class_w, dtype=np.float64)[y]
    W = w.sum()
    L = float(np.sum(w * -np.log(p[np.arange(len(y)), y])) / W)
    onehot = np.zeros_like(p)
    onehot[np.arange(len(y)), y] = 1.0
    dZ = (w / W)[:, None] * (p - onehot)
    return L, dZ


def backward(params: np.ndarray, cache: dict, dZ: np.ndarray) -> np.ndarray:
    """Gradient of the loss with respect to the parameter vector."""
    r = bf16 if cache["emulate"] else (lambda a: np.asarray(a, dtype=np.float64))
    P, Wf = cache["P"], cache["Wf"]
    g = {}
    g["Wf"] = dZ.T @ P
    g["bf"] = dZ.sum(axis=0)
    dP = dZ @ Wf
    npx = cache["Y3"].shape[1] * cache["Y3"].shape[2]
    dY3 = np.broadcast_to(dP[:, None, None, :] / npx, cache["Y3"].shape) * (cache["Y3"] > 0)
    g["b3"] = dY3.sum(axis=(0, 1, 2))
    dY3r = r(dY3)
    g["W3"] = conv3x3_wgrad(cache["A2"], dY3r, 2)
    dA2 = conv3x3_xgrad(dY3r, cache["W3"], 2, cache["A2"].shape)
    dY2 = dA2 * (cache["A2"] > 0)
    g["b2"] = dY2.sum(axis=(0, 1, 2))
    dY2r = r(dY2)
    g["W2"] = conv3x3_wgrad(cache["A1"], dY2r, 2)
    dA1 = conv3x3_xgrad(dY2r, cache["W2"], 2, cache["A1"].shape)
    dY1 = dA1 * (cache["A1"] > 0)
    g["b1"] = dY1.sum(axis=(0, 1, 2))
    dY1r = r(dY1)
    g["W1"] = conv3x3_wgrad(cache["X0"], dY1r, 1)
    return pack(g)


def adam(params, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def predict(params: np.ndarray, X: np.ndarray, emulate: bool = False) -> np.ndarray:
    """Flags -1 (coarsen), 0 (keep), +1 (refine) from the largest logit."""
    Z, _ = forward(params, X, emulate)
    return np.argmax(Z, axis=1).astype(np.int8) - 1
