"""Checkpoint and restart through the boundary: the leaves, the state and the
clock (time and the next step) of a run, read back to the host and loaded
into a new context, continue to the same bits as the run that never stopped,
through steps with the adaptive step controller and through regrids."""
import numpy as np
import pytest

import paper_2403_15435_amd as gf
from paper_2403_15435_amd import inputs

pytestmark = pytest.mark.gpu


def _scenario():
    sc = inputs.reservoir_fractal(level=3, m=16, radius=300.0, L=2000.0, seed=2)
    sc.min_level, sc.max_level, sc.init_level = 1, 4, 1
    return sc


def _advance(ctx, blocks):
    # blocks of 4 adaptive steps, each followed by tagging and a regrid
    for _ in range(blocks):
        ctx.step(4)
        ctx.regrid(ctx.tag())


def _checkpoint(ctx, scen=0):
    t, dt, steps, rej = ctx.time(scen)
    return {"leaves": ctx.leaves(scen).copy(), "state": ctx.state(scen).copy(), "t": t, "dt": dt}


def _restore(ck, sc, prec):
    ctx = gf.Context([sc], precision=prec, max_patches=1024)
    ctx.set_leaves(0, ck["leaves"])
    ctx.set_state(0, ck["state"])
    ctx.set_time(0, ck["t"], ck["dt"])
    return ctx


@pytest.mark.parametrize("prec", [gf.GF_FP64, gf.GF_FP32])
def test_restart_continues_bit_for_bit(prec):
    sc = _scenario()
    a = gf.Context([sc], precision=prec, max_patches=1024)
    a.set_initial(0, max_passes=3)
    print(f"restart, precision {prec}: 6 blocks, checkpoint, 6 more", flush=True)
    _advance(a, 6)
    ck = _checkpoint(a)
    assert len(set(ck["leaves"][:, 1])) >= 2 and ck["t"] > 0 and ck["dt"] > 0
    b = _restore(ck, sc, prec)
    # the restored context reads back what was saved
    assert np.array_equal(b.leaves(0), ck["leaves"])
    assert np.array_equal(b.state(0), ck["state"])
    assert b.time(0)[:2] == (ck["t"], ck["dt"])
    assert b.mass(0)[0] == a.mass(0)[0]
    _advance(a, 6)
    _advance(b, 6)
    ta, tb = a.time(0), b.time(0)
    print(f"t {ta[0]!r} vs {tb[0]!r}, leaves {len(a.leaves(0))} vs {len(b.leaves(0))}", flush=True)
    assert ta[:2] == tb[:2]
    assert np.array_equal(a.leaves(0), b.leaves(0))
    assert np.array_equal(a.state(0), b.state(0))
    assert a.mass(0)[0] == b.mass(0)[0]


def test_restart_into_another_launch_shape():
    """A checkpoint is independent of the step kernel's launch shape: restored
    under other threads, padding and schedule, the run goes on to the same
    bits (FP64)."""
    sc = _scenario()
    a = gf.Context([sc], precision=gf.GF_FP64, max_patches=1024)
    a.set_initial(0, max_passes=3)
    _advance(a, 3)
    ck = _checkpoint(a)
    b = _restore(ck, sc, gf.GF_FP64)
    b.set_step_threads(64)
    b.set_step_pad(1)
    b.set_schedule(0)
    _advance(a, 4)
    _advance(b, 4)
    assert a.time(0)[:2] == b.time(0)[:2]
    assert np.array_equal(a.leaves(0), b.leaves(0))
    assert np.array_equal(a.state(0), b.state(0))
