"""The learned tagger on the GPU (BF16 matrix cores, FP32 accumulation) against
the CPU oracle in its bfloat16-emulating mode, which rounds at the same points
and sums in FP64.  The two differ by FP32 summation error, and by the rare
value that lands next to a bfloat16 rounding boundary and rounds the other
way, so the comparisons are norm-wise per parameter block: 1e-4, about 30
times under what the rounding points themselves change (emulated vs exact
arithmetic, printed beside)."""
import numpy as np
import pytest

import paper_2403_15435_amd as gf
from paper_2403_15435_amd import inputs
from oracle import cnn_oracle as cn

pytestmark = pytest.mark.gpu


def _ctx():
    sc = inputs.reservoir_fractal(level=2, m=16, L=2000.0, seed=2, radius=300.0)
    ctx = gf.Context([sc], precision=gf.GF_FP32, max_patches=64)
    ctx.set_initial(0)
    return sc, ctx


def _batch(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 24, 24, 4)) * np.array([2.0, 0.5, 0.5, 1.0])
    return cn.bf16(X)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_forward_matches_oracle():
    sc, ctx = _ctx()
    params = inputs.cnn_init_params(1)
    params[cn.N_PARAMS - 3:] = [0.1, -0.2, 0.05]
    ctx.net_set_params(params)
    X = _batch(16, 2)
    Zg = ctx.net_forward(X)
    Ze, _ = cn.forward(params, X, emulate=True)
    Zx, _ = cn.forward(params, X, emulate=False)
    print(f"logits: rel to emulated {_rel(Zg, Ze):.2e}, emulated vs exact {_rel(Ze, Zx):.2e}", flush=True)
    assert _rel(Zg, Ze) <= 1e-4
    assert np.array_equal(np.argmax(Zg, axis=1), np.argmax(Ze, axis=1))


def test_gradients_match_oracle():
    sc, ctx = _ctx()
    params = inputs.cnn_init_params(3)
    ctx.net_set_params(params)
    X = _batch(32, 4)
    y = np.random.default_rng(5).integers(0, 3, 32).astype(np.int8)
    cw = np.array([1.0, 0.5, 2.0])
    loss_g, g = ctx.net_train_step(X, y, cw, lr=0.0, want_grad=True)
    Ze, cache = cn.forward(params, X, emulate=True)
    loss_e, dZ = cn.loss(Ze, y, cw)
    ge = cn.backward(params, cache, dZ)
    Zx, cx = cn.forward(params, X, emulate=False)
    _, dZx = cn.loss(Zx, y, cw)
    gx = cn.backward(params, cx, dZx)
    assert loss_g == pytest.approx(loss_e, rel=1e-5)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in cn.PARAM_SHAPES])
    for (name, _), a, b in zip(cn.PARAM_SHAPES, offs[:-1], offs[1:]):
        rg, rx = _rel(g[a:b], ge[a:b]), _rel(ge[a:b], gx[a:b])
        print(f"{name}: GPU vs emulated {rg:.2e}; emulated vs exact {rx:.2e}", flush=True)
        assert rg <= 1e-4, name


def test_adam_step_and_training():
    """The update applied after a step is the oracle's Adam on the gradient the
    GPU reported; a short training run on a fixed batch drives the loss down."""
    sc, ctx = _ctx()
    params = inputs.cnn_init_params(6)
    ctx.net_set_params(params)
    X = _batch(24, 7)
    y = (np.arange(24) % 3).astype(np.int8)
    cw = np.ones(3)
    loss0, g = ctx.net_train_step(X, y, cw, lr=1e-3, want_grad=True)
    p1 = ctx.net_params()
    want, _, _ = cn.adam(params, g, np.zeros_like(params), np.zeros_like(params), 1, 1e-3)
    assert np.allclose(p1, want, rtol=1e-5, atol=1e-7)
    losses = [loss0]
    for _ in range(60):
        losses.append(ctx.net_train_step(X, y, cw, lr=3e-3))
    print(f"loss {losses[0]:.4f} -> {losses[-1]:.4f}", flush=True)
    assert losses[-1] < 0.5 * losses[0]


def test_features_match_oracle():
    """Feature tiles of an AMR mesh (levels 1-3) from the library's own state."""
    sc = inputs.reservoir_fractal(level=2, m=16, L=2000.0, seed=3, radius=500.0)
    sc.min_level, sc.max_level = 1, 3
    lv = [(0, 1, 0, 0), (0, 1, 1, 1)]
    lv += [(0, 2, 2 + a, b) for b in range(2) for a in range(2)]
    lv += [(0, 2, 0, 2), (0, 2, 1, 2), (0, 2, 1, 3)]
    lv += [(0, 3, a, 6 + b) for b in range(2) for a in range(2)]
    leaves = np.array(lv, np.int32)
    for prec in (gf.GF_FP32, gf.GF_FP64):
        ctx = gf.Context([sc], precision=prec, max_patches=64)
        ctx.set_leaves(0, leaves)
        ctx.set_initial(0)
        ctx.step(10)
        Fg = ctx.net_features()
        Fo = cn.features(sc, ctx.leaves(0), ctx.state(0))
        err = np.abs(Fg - Fo).max()
        print(f"features ({'fp32' if prec == gf.GF_FP32 else 'fp64'} state): max abs diff {err:.2e}, "
              f"max value {np.abs(Fo).max():.2f}", flush=True)
        assert err <= 1e-5 * max(1.0, np.abs(Fo).max())


def test_predict_flags_drive_regrid():
    """Flags from the network stay within the level limits and are what a
    following regrid applies."""
    sc = inputs.reservoir_fractal(level=2, m=16, L=2000.0, seed=3, radius=500.0)
    sc.min_level, sc.max_level = 1, 3
    ctx = gf.Context([sc], precision=gf.GF_FP32, max_patches=256)
    ctx.set_initial(0)
    params = inputs.cnn_init_params(8)
    params[cn.N_PARAMS - 3:] = [0.0, -5.0, 5.0]     # bias every leaf towards "refine"
    ctx.net_set_params(params)
    lv = ctx.leaves(0)
    flags = ctx.net_predict()
    assert flags.shape == (lv.shape[0],)
    assert np.all(flags[lv[:, 1] >= sc.max_level] <= 0)
    assert np.all(flags[lv[:, 1] <= sc.min_level] >= 0)
    F = ctx.net_features()
    Z, _ = cn.forward(params, F, emulate=True)
    want = np.argmax(Z, axis=1) - 1
    want = np.where((want > 0) & (lv[:, 1] >= sc.max_level), 0, want)
    want = np.where((want < 0) & (lv[:, 1] <= sc.min_level), 0, want)
    assert np.mean(flags == want) >= 0.95
    n = ctx.regrid(None)
    assert n > lv.shape[0]
