"""Pins of the learned-tagger oracle (CPU): bfloat16 rounding, convolutions
against brute force and adjoint identities, gradients against finite
differences, loss and optimiser closed forms, features against their
definition on hand-built fields."""
import itertools
import math

import numpy as np
import pytest

from oracle import cnn_oracle as cn
from paper_2403_15435_amd import inputs


# ------------------------------------------------------------------ bf16
def test_bf16_rounding_known_values():
    e = 2.0 ** -8          # half an ulp of bfloat16 at 1
    big = 2.0 ** 100
    cases = [(1.0, 1.0), (1.0 + e, 1.0),                       # tie -> even (down)
             (1.0 + 3 * e, 1.0 + 4 * e),                       # tie -> even (up)
             (1.0 + e + 2.0 ** -20, 1.0 + 2 * e),              # above the tie
             (-1.5, -1.5), (0.0, 0.0),
             (big * (1 + 2 * e), big * (1 + 2 * e)), (big * (1 + e), big)]
    for x, want in cases:
        got = cn.bf16(np.array([x]))[0]
        assert got == want, (x, got, want)


def test_bf16_rounding_bounds():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(10000) * 10.0 ** rng.integers(-10, 10, 10000)
    r = cn.bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-6))
    bits = r.astype(np.float32).view(np.uint32)
    assert np.all(bits & 0xFFFF == 0)
    assert np.array_equal(cn.bf16(r), r)


# ------------------------------------------------------------------ convolutions
def conv_brute(X, W, b, s):
    N, H, Wd, Ci = X.shape
    Co = W.shape[0]
    Ho, Wo = (H - 1) // s + 1, (Wd - 1) // s + 1
    Y = np.zeros((N, Ho, Wo, Co))
    for n, oy, ox, co in itertools.product(range(N), range(Ho), range(Wo), range(Co)):
        acc = b[co]
        for ky, kx, ci in itertools.product(range(3), range(3), range(Ci)):
            y, x = s * oy + ky - 1, s * ox + kx - 1
            if 0 <= y < H and 0 <= x < Wd:
                acc += X[n, y, x, ci] * W[co, ky, kx, ci]
        Y[n, oy, ox, co] = acc
    return Y


@pytest.mark.parametrize("s", [1, 2])
def test_conv_matches_brute_force(s):
    rng = np.random.default_rng(2 + s)
    X = rng.standard_normal((2, 6, 6, 3))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    assert np.allclose(cn.conv3x3(X, W, b, s), conv_brute(X, W, b, s), rtol=1e-12, atol=1e-12)


def test_conv_delta_kernel_copies_channel():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((1, 8, 8, 4))
    W = np.zeros((4, 3, 3, 4))
    for c in range(4):
        W[c, 1, 1, (c + 1) % 4] = 1.0
    Y = cn.conv3x3(X, W, np.zeros(4), 1)
    assert np.array_equal(Y, X[..., [1, 2, 3, 0]])
    Y2 = cn.conv3x3(X, W, np.zeros(4), 2)
    assert np.array_equal(Y2, X[:, ::2, ::2][..., [1, 2, 3, 0]])


@pytest.mark.parametrize("s", [1, 2])
def test_conv_gradients_are_adjoints(s):
    """<conv(X, W), dY> is bilinear: its derivative in W is wgrad(X, dY) and in
    X is xgrad(dY, W)."""
    rng = np.random.default_rng(7 + s)
    X = rng.standard_normal((2, 12, 12, 5))
    W = rng.standard_normal((6, 3, 3, 5))
    Y = cn.conv3x3(X, W, np.zeros(6), s)
    dY = rng.standard_normal(Y.shape)
    lhs = np.sum(Y * dY)
    assert np.sum(W * cn.conv3x3_wgrad(X, dY, s)) == pytest.approx(lhs, rel=1e-12)
    assert np.sum(X * cn.conv3x3_xgrad(dY, W, s, X.shape)) == pytest.approx(lhs, rel=1e-12)


# ------------------------------------------------------------------ loss, optimiser
def test_loss_closed_forms():
    Z = np.zeros((4, 3))
    y = np.array([0, 1, 2, 1])
    L, dZ = cn.loss(Z, y, np.array([1.0, 2.0, 3.0]))
    assert L == pytest.approx(math.log(3.0))
    assert np.allclose(dZ.sum(axis=1), 0.0)
    # one sample: d/dz of -log softmax = p - onehot
    L1, d1 = cn.loss(np.array([[0.0, math.log(2.0), 0.0]]), np.array([1]), np.ones(3))
    assert L1 == pytest.approx(-math.log(0.5))
    assert np.allclose(d1, [[0.25, -0.5, 0.25]])


def test_adam_first_step_moves_by_lr():
    rng = np.random.default_rng(3)
    p0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = cn.adam(p0, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    # bias-corrected moments of one step are g and g^2: a step of lr g / (|g| + eps)
    assert np.allclose(p1, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


# ------------------------------------------------------------------ gradients
def test_backward_matches_finite_differences():
    rng = np.random.default_rng(11)
    params = inputs.cnn_init_params(4)
    params[cn.N_PARAMS - 3:] = rng.standard_normal(3) * 0.1
    X = rng.standard_normal((3, 24, 24, 4))
    y = np.array([0, 1, 2])
    cw = np.array([1.0, 0.5, 2.0])
    Z, cache = cn.forward(params, X)
    _, dZ = cn.loss(Z, y, cw)
    g = cn.backward(params, cache, dZ)
    f = lambda p: cn.loss(cn.forward(p, X)[0], y, cw)[0]
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in cn.PARAM_SHAPES])
    idx = []
    for a, b in zip(offs[:-1], offs[1:]):
        idx += list(rng.choice(np.arange(a, b), size=min(6, b - a), replace=False))
    eps = 1e-6
    for i in idx:
        e = np.zeros_like(params)
        e[i] = eps
        fd = (f(params + e) - f(params - e)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), 1e-3), (i, fd, g[i])


def test_emulated_forward_is_close_to_exact():
    rng = np.random.default_rng(12)
    params = inputs.cnn_init_params(5)
    X = rng.standard_normal((4, 24, 24, 4))
    Ze, _ = cn.forward(params, X, emulate=True)
    Zx, _ = cn.forward(params, X, emulate=False)
    assert np.abs(Ze - Zx).max() <= 0.05 * np.abs(Zx).max()
    assert not np.array_equal(Ze, Zx)


# ------------------------------------------------------------------ features
def _state(sc, leaves, fn):
    st = np.zeros((len(leaves), 4, sc.m, sc.m))
    for k, lf in enumerate(leaves):
        X, Y = sc.cell_centres(lf)
        st[k] = fn(X, Y)
    return st


def test_features_uniform_and_linear_fields():
    sc = inputs.reservoir_fractal(level=2, m=16, L=2000.0, seed=2)
    lv = sc.uniform_leaves(2)
    st = _state(sc, lv, lambda X, Y: np.stack([np.full_like(X, 3.0), np.full_like(X, 20.0),
                                               np.full_like(X, -10.0), 0.01 * X + 0.02 * Y]))
    F = cn.features(sc, lv, st)
    k = int(np.flatnonzero((lv[:, 2] == 1) & (lv[:, 3] == 2))[0])    # an interior leaf
    assert np.allclose(F[k, ..., 0], 3.0) and np.allclose(F[k, ..., 1], 2.0) and np.allclose(F[k, ..., 2], -1.0)
    # a linear bed averages to its value at the pixel centre
    dx = sc.dx(2)
    px = (sc.m // 8) * dx          # a pixel is m/8 cells wide
    xs = (8 * 1 - 8 + np.arange(24) + 0.5) * px
    ys = (8 * 2 - 8 + np.arange(24) + 0.5) * px
    bleaf = st[k, 3].mean()
    want = (0.01 * xs[None, :] + 0.02 * ys[:, None] - bleaf) * 0.1
    assert np.allclose(F[k, ..., 3], want, atol=1e-12)
    # a corner leaf sees zeros outside the domain
    k0 = int(np.flatnonzero((lv[:, 2] == 0) & (lv[:, 3] == 0))[0])
    assert np.all(F[k0, :8, :, :] == 0.0) and np.all(F[k0, :, :8, :] == 0.0)
    assert np.allclose(F[k0, 8:, 8:, 0], 3.0)


def test_features_across_levels_are_area_means():
    """A coarse leaf's window over a refined region holds the means of the fine
    cells under each pixel; a fine leaf's window over a coarse leaf repeats the
    coarse cell values; the centre block is the leaf's own block means."""
    sc = inputs.reservoir_fractal(level=1, m=16, L=2000.0, seed=2)
    sc.min_level, sc.max_level = 1, 2
    lv = np.array([(0, 1, 0, 0), (0, 1, 0, 1), (0, 1, 1, 1)] + [(0, 2, 2 + a, b) for b in range(2) for a in range(2)],
                  np.int32)
    rng = np.random.default_rng(9)
    st = rng.uniform(0.0, 5.0, (len(lv), 4, 16, 16))
    F = cn.features(sc, lv, st)
    # m = 16: a pixel is 2 x 2 cells of the leaf's level.  Level-2 image of the
    # level-1 square (1, 0), which the four level-2 leaves cover:
    img2 = np.zeros((32, 32))
    for k in range(3, 7):
        a, b = lv[k, 2] - 2, lv[k, 3]
        img2[b * 16:(b + 1) * 16, a * 16:(a + 1) * 16] = st[k, 0]
    # coarse leaf (1, 0, 0): window columns 16..23, rows 8..15 are that square;
    # pixel (py, px) covers level-2 cells rows 4 py .. 4 py + 3, columns 4 px .. 4 px + 3
    for py in range(8):
        for px in range(8):
            want = img2[4 * py:4 * py + 4, 4 * px:4 * px + 4].mean()
            assert F[0, 8 + py, 16 + px, 0] == pytest.approx(want, rel=1e-12)
    # fine leaf (2, 2, 1): window columns 0..7, rows 8..15 are the level-2 square
    # (1, 1), inside coarse leaf (1, 0, 0) cells i 8..15, j 8..15: one coarse cell per pixel
    kf = int(np.flatnonzero((lv[:, 1] == 2) & (lv[:, 2] == 2) & (lv[:, 3] == 1))[0])
    assert np.allclose(F[kf, 8:16, 0:8, 0], st[0, 0, 8:16, 8:16], rtol=1e-12)
    own = st[kf, 0].reshape(8, 2, 8, 2).mean(axis=(1, 3))
    assert np.allclose(F[kf, 8:16, 8:16, 0], own, rtol=1e-12)
