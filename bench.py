"""Benchmark: cell updates per second of the FP32 batched adaptive patch
update on one MI355X, against the plain FP64 path on the same inputs.

Headline workload (the adaptive one the metric names): the AMR inflow
valley, 20 km x 10 km, side slope 0.05 with 2 m rms fractal
roughness, 16 x 8 trees, levels 0-6 of 32 x 32 patches (finest cells 0.61 m,
about 25 000 leaves), inflow 5000 m^3/s over 200 m on the hydrograph's
plateau, Manning n = 0.04, extrapolation outflow, walls; the mesh built from
level 0 by plain-tagger passes over the initial flood.  One step = one pass
of ghost fill + wave-propagation update + friction + positivity + step control
+ refluxing over every leaf; the job tags and regrids every 4 steps, inside
the timed window.  Reported beside it: the fused FP64 and plain FP64 paths on
the same mesh and state, the step kernel's roofline (its launches timed alone
with HIP events in a repeat of the window, the patches it updated counted in
another), the device's achievable HBM bandwidth (a triad probe), the CPU
oracle on the same valley (all host threads and one), and further sections:
the uniform 2048^2 reservoir, the same grid fully wet, the 256-scenario
ensemble, the floodplain, local time stepping, the learned tagger.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np

METRIC = "cell-updates/s and % HBM roofline, FP32-batched AMR vs FP64 plain, 1 MI355X"
PROFILES = os.path.join(ROOT, "profiles")
VALLEY_COUNTERS = os.path.join(PROFILES, "step_kernel_fp32_valley_counters.txt")
VALLEY_STATS = os.path.join(PROFILES, "step_kernel_fp32_valley_kernel_stats.txt")
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = {"f32": 28.0, "f64": 56.0}
# the method's arithmetic per cell update (two augmented Riemann solves, three
# limited waves and the transverse splits per edge direction, update and
# friction), counted as VALU lane operations with sqrt and division as one
ALGO_OPS_PER_UPDATE = 500.0
# non-packed FP32 VALU issue: 256 CUs x 4 SIMDs x 16 lanes per cycle x 2.4 GHz
VALU_PEAK_GOPS = 256 * 4 * 16 * 2.4
VALLEY_DESC = ("AMR inflow valley: 20 km x 10 km V valley, side slope 0.05, 2 m rms fractal "
               "roughness, 16x8 trees, levels 0-6 of 32x32 patches (finest cells 0.61 m), inflow 5000 m^3/s over "
               "200 m (hydrograph plateau, from t = 4000 s), n = 0.04, extrapolation outflow, walls; mesh built "
               "from level 0 by plain-tagger passes; tag and regrid every 4 steps inside the timed window")


def workload():
    from paper_2403_15435_amd import inputs
    return inputs.reservoir_fractal(level=6, m=32, L=10000.0, seed=2, radius=400.0, h_res=20.0, manning_n=0.033)


def wet_workload():
    from paper_2403_15435_amd import inputs
    return inputs.wet_dambreak(level=6, m=32, L=10000.0, seed=2, radius=400.0, manning_n=0.033)


def _sync():
    import torch
    torch.cuda.synchronize()


def flood_speed_amr(steps, warmup, regrid_every=4, t_spin=1800.0):
    """The floodplain workload (flat 1 km x 2 km, 20 m inlet, trapezoid
    hydrograph to 20 m^3/s, n = 0.03, dry start) on AMR levels 0-3 of 32 x 32
    patches (5.2 m to 0.65 m cells), depth-tagged, the inlet held at the
    finest level: spun up on the FP32 path to t_spin, then timed on the fused
    FP32, fused FP64 and plain FP64 paths from that mesh and state (widened),
    tag and regrid every `regrid_every` steps."""
    import paper_2403_15435_amd as gf
    from paper_2403_15435_amd import inputs
    sc = inputs.flood_speed()
    cap = 8192
    base = gf.Context([sc], precision=gf.GF_FP32, max_patches=cap)
    base.set_initial(0)
    spin = 0
    while base.time(0)[0] < t_spin:
        base.tag()
        base.regrid(None)
        base.step(regrid_every)
        spin += regrid_every
    base.tag()
    base.regrid(None)
    leaves0, state0, t0 = base.leaves(0), base.state(0), base.time(0)[0]
    base.close()
    print(f"[bench] floodplain at t = {t0:.0f} s after {spin} steps: {leaves0.shape[0]} leaves, levels "
          f"{np.bincount(leaves0[:, 1]).tolist()}", file=sys.stderr, flush=True)
    out = {"workload": "floodplain: flat 1000 m x 2000 m, inflow over 990-1010 m of x = 0, trapezoid hydrograph "
                       "0 -> 20 m^3/s (60/180/60 min), n = 0.03, walls, dry start; 6x12 trees, levels 0-3 of 32x32 "
                       "patches (5.2 m to 0.65 m), depth tagging (0.05 m), inlet region at level 3, regrid every 4 "
                       "steps; timed from t = 30 min",
           "t_start_s": t0, "leaves_start": int(leaves0.shape[0]), "steps": steps, "regrid_every": regrid_every}
    for name, prec, plain in (("fp32_fused", gf.GF_FP32, False), ("fp64_fused", gf.GF_FP64, False),
                              ("fp64_plain", gf.GF_FP64, True)):
        ctx = gf.Context([sc], precision=prec, max_patches=cap)
        ctx.set_leaves(0, leaves0)
        ctx.set_state(0, state0[:, :3])
        ctx.set_time(0, t0)
        if not plain:
            ctx.autotune(steps=3)

        def cycle():
            _sync()
            a = time.perf_counter()
            st = ctx.step(regrid_every, plain=plain)
            _sync()
            b = time.perf_counter()
            ctx.tag()
            ctx.regrid(None)
            return st, b - a, time.perf_counter() - b
        for _ in range(max(warmup // regrid_every, 1)):
            cycle()
        m0 = ctx.mass(0)
        t_step = t_regrid = 0.0
        cells = 0
        for _ in range(steps // regrid_every):
            st, ts, tr = cycle()
            t_step += ts
            t_regrid += tr
            cells += int(st.cell_updates)
        M = ctx.mass(0)
        out[name] = {"step_cell_updates_per_s": cells / t_step,
                     "end_to_end_cell_updates_per_s": cells / (t_step + t_regrid), "step_s": t_step,
                     "tag_regrid_s": t_regrid, "leaves_end": int(ctx.leaves(0).shape[0]),
                     "budget_residual_rel": float(((M[0] - m0[0]) - (M[1] - m0[1]) - (M[2] - m0[2])) / M[0])}
        print(f"[bench] floodplain {name}: {out[name]}", file=sys.stderr, flush=True)
        ctx.close()
    out["speedup_fp32_fused_over_fp64_plain"] = (out["fp32_fused"]["step_cell_updates_per_s"]
                                                 / out["fp64_plain"]["step_cell_updates_per_s"])
    return out


def lts_compare(window_steps=64):
    """Local time stepping against the single clock on fixed AMR meshes (no
    regrid inside the window): the valley mesh (levels 0-6) and the
    floodplain mesh at t = 30 min (levels 0-3), FP32 fused path.  The single
    clock takes `window_steps` steps; local time stepping, in one call, the
    number of macro steps that spans about as long (at least 4).  Reported:
    simulated seconds per wall second (the comparison), cell updates per
    second (local time stepping updates each level at its own rate, so it
    does fewer)."""
    import paper_2403_15435_amd as gf
    from paper_2403_15435_amd import inputs
    out = {}
    cases = []
    sc = inputs.v_valley()
    base = gf.Context([sc], precision=gf.GF_FP32, max_patches=48000)
    base.set_initial(0)
    for _ in range(sc.max_level - sc.min_level):
        base.tag()
        base.regrid(None)
        base.set_initial(0)
    cases.append(("valley", sc, base.leaves(0), base.state(0), 4000.0, 48000))
    base.close()
    fs = inputs.flood_speed()
    base = gf.Context([fs], precision=gf.GF_FP32, max_patches=8192)
    base.set_initial(0)
    while base.time(0)[0] < 1800.0:
        base.tag()
        base.regrid(None)
        base.step(4)
    cases.append(("floodplain", fs, base.leaves(0), base.state(0), base.time(0)[0], 8192))
    base.close()
    for name, sc, leaves, state, t0, cap in cases:
        res = {"leaves": int(leaves.shape[0]), "levels": np.bincount(leaves[:, 1]).tolist()}
        for path in ("single_clock", "lts"):
            ctx = gf.Context([sc], precision=gf.GF_FP32, max_patches=cap)
            ctx.set_leaves(0, leaves)
            ctx.set_state(0, state[:, :3])
            ctx.set_time(0, t0)
            ctx.autotune(steps=3)
            lts = path == "lts"
            ctx.step(2, lts=lts)           # warm-up (first use of each launch shape)
            t1 = ctx.time(0)[0]
            _sync()
            a = time.perf_counter()
            if not lts:
                st = ctx.step(window_steps)
            else:
                # about the same stretch of time in one call: a macro step
                # spans up to 2^(L1 - L0) single-clock steps
                span = 1 << int(leaves[:, 1].max() - leaves[:, 1].min())
                st = ctx.step(max(4, window_steps // span), lts=True)
            cells = int(st.cell_updates)
            _sync()
            wall = time.perf_counter() - a
            sim = ctx.time(0)[0] - t1
            res[path] = {"sim_s": sim, "wall_s": wall, "sim_s_per_wall_s": sim / wall, "cell_updates_per_s": cells / wall,
                         "steps": int(ctx.time(0)[2])}
            ctx.close()
        res["lts_speedup_sim_time"] = res["lts"]["sim_s_per_wall_s"] / res["single_clock"]["sim_s_per_wall_s"]
        print(f"[bench] lts {name}: {res}", file=sys.stderr, flush=True)
        out[name] = res
    return out


def ensemble(steps, warmup, n_scen=256):
    """The batched workload: 256 independent dam breaks on seeded fractal
    terrain (grids of 64^2 to 512^2 cells as 32 x 32 patches, n ~ U[0.02,
    0.06], breach widths U[50, 500] m), every scenario with its own adaptive
    step, all in one launch per step on the fused path (one launch per
    scenario on the plain path); the same initial state (FP32, widened) on
    every path."""
    import paper_2403_15435_amd as gf
    from paper_2403_15435_amd import inputs
    scs = inputs.ensemble_dambreaks(n_scen=n_scen)
    cap = sum(int(round((s.x1 - s.x0) / 10.0)) ** 2 // (32 * 32) for s in scs) + 64
    base = gf.Context(scs, precision=gf.GF_FP32, max_patches=cap)
    states = [base.set_initial(k) for k in range(len(scs))]
    base.close()
    out = {"workload": f"ensemble of {n_scen} dam breaks, grids in {{64,128,256,512}}^2 (dx 10 m) as 32x32 patches, "
                       "seeded fractal terrain, n ~ U[0.02,0.06], breach U[50,500] m, walls",
           "patches": cap - 64, "steps_per_scenario": steps}
    for name, prec, plain in (("fp32_fused", gf.GF_FP32, False), ("fp64_fused", gf.GF_FP64, False),
                              ("fp64_plain", gf.GF_FP64, True)):
        ctx = gf.Context(scs, precision=prec, max_patches=cap)
        for k, st0 in enumerate(states):
            ctx.set_state(k, st0[:, :3])
        if not plain:
            ctx.autotune(steps=3)
        ctx.step(warmup, plain=plain)
        _sync()
        a = time.perf_counter()
        st = ctx.step(steps, plain=plain)
        _sync()
        wall = time.perf_counter() - a
        cups = int(st.cell_updates) / wall
        out[name] = {"cell_updates_per_s": cups, "s": wall, "rejected": int(st.rejected)}
        if prec == gf.GF_FP32:
            out[name]["hbm_frac_algorithmic"] = cups * BYTES_PER_UPDATE["f32"] / (HBM_PEAK_GBS * 1e9)
        print(f"[bench] ensemble {name}: {out[name]}", file=sys.stderr, flush=True)
        ctx.close()
    out["speedup_fp32_fused_over_fp64_plain"] = out["fp32_fused"]["cell_updates_per_s"] / out["fp64_plain"]["cell_updates_per_s"]
    return out


def _finest_depth(sc, leaves, st, level):
    """Depth of an AMR state projected (piecewise constant) onto one uniform level."""
    m = sc.m
    out = np.zeros((sc.mj * m << level, sc.mi * m << level))
    for k, (t, l, ix, iy) in enumerate(np.asarray(leaves)):
        r = 1 << (level - l)
        PI = (t % sc.mi) * (1 << l) + ix
        PJ = (t // sc.mi) * (1 << l) + iy
        out[PJ * m * r:(PJ + 1) * m * r, PI * m * r:(PI + 1) * m * r] = np.kron(st[k, 0], np.ones((r, r)))
    return out


def _dilated_flags(sc, lv, fl):
    """Plain flags with every refine request spread to the neighbouring leaves
    (faces and corners) that are as coarse or coarser: a trivial anticipating
    tagger, the baseline the network has to beat."""
    lv = np.asarray(lv)
    pos = {(int(l), int(ix), int(iy)): k for k, (t, l, ix, iy) in enumerate(lv)}
    out = np.asarray(fl, np.int8).copy()
    for k in np.flatnonzero(np.asarray(fl) > 0):
        t, l, ix, iy = (int(v) for v in lv[k])
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                X, Y = ix + dx, iy + dy
                if not (0 <= X < (1 << l) and 0 <= Y < (1 << l)):
                    continue
                for a in range(l, -1, -1):
                    j = pos.get((a, X >> (l - a), Y >> (l - a)))
                    if j is not None:
                        if lv[j, 1] < sc.max_level:
                            out[j] = 1
                        break
    return out


class _RunStats:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def _dilated_run(ctx, sc, nsteps, check=4, regrid_every=16):
    """The plain tagger every regrid_every steps with its refine requests
    dilated by one leaf; misses counted at the checks between (no regrid),
    as gf_run's sparse mode counts them."""
    st = _RunStats(steps=0, regrids=0, forced_regrids=0, checks=0, misses=0, leaf_steps=0, seconds=0.0)
    _sync()
    t0 = time.perf_counter()
    for k in range(0, nsteps, check):
        fl = ctx.tag()
        if k % regrid_every == 0:
            ctx.regrid(_dilated_flags(sc, ctx.leaves(0), fl))
            st.regrids += 1
        else:
            st.checks += fl.size
            st.misses += int((fl > 0).sum())
        ns = min(check, nsteps - k)
        ctx.step(ns)
        st.steps += ns
        st.leaf_steps += ctx.leaves(0).shape[0] * ns
    _sync()
    st.seconds = time.perf_counter() - t0
    return st


def learned_tagger(n_train=50, n_eval=10, steps=2000, window=16, check=4, iters=400, batch=256):
    """The learned tagger on the reservoir geometry as AMR: 10 km square,
    levels 0-6 of 32 x 32 patches (finest 4.88 m), reservoir r = 400 m with
    its centre drawn from U[2.5 km, 7.5 km]^2 by the seed.  Trained on the GPU
    from plain-tagger windows (a sample every 16 steps: every refine label,
    twice as many others drawn at random) of seeds 5001.., evaluated on the
    unseen seeds 5051..: the plain tagger every 4 steps (the reference), every 16
    steps, and the network every 16 steps with the plain-tagger fallback at
    the 4-step checks."""
    import paper_2403_15435_amd as gf
    from paper_2403_15435_amd import inputs
    cap = 12000

    def make(seed):
        sc = inputs.adaptive_reservoir(seed, L=10000.0, m=32, max_level=6, dem_level=6, radius=400.0)
        ctx = gf.Context([sc], precision=gf.GF_FP32, max_patches=cap)
        ctx.set_initial(0)
        for _ in range(sc.max_level):
            ctx.tag()
            ctx.regrid(None)
            ctx.set_initial(0)
        return sc, ctx
    rng = np.random.default_rng(0)
    X, Y = [], []
    t0 = time.perf_counter()
    for j in range(n_train):
        sc, ctx = make(5001 + j)
        for _ in range(steps // window):
            F, y = ctx.net_collect(window, check)
            keep = np.flatnonzero(y == 2)
            rest = np.flatnonzero(y != 2)
            take = min(rest.size, 2 * keep.size + 8)
            keep = np.concatenate([keep, rng.choice(rest, size=take, replace=False)]) if take else keep
            X.append(F[keep].astype(np.float32))
            Y.append(y[keep])
        ctx.close()
        print(f"[bench] learned: collected seed {5001 + j}: {sum(a.shape[0] for a in X)} samples, "
              f"{time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
    X, Y = np.concatenate(X), np.concatenate(Y)
    counts = np.bincount(Y, minlength=3)
    cw = counts.sum() / (3.0 * np.maximum(counts, 1))
    sc, ctx = make(5001)
    ctx.net_set_params(inputs.cnn_init_params(0))
    # the training set on the device once (bfloat16 features, int8 labels);
    # each step trains on a batch gathered there (gf_net_train_step_dev), the
    # loss read back every 10 steps
    import torch
    Xt = torch.from_numpy(X.reshape(Y.size, -1)).to("cuda").to(torch.bfloat16).view(torch.int16)
    Yt = torch.from_numpy(Y.astype(np.int8)).to("cuda")
    losses = []
    _sync()
    t1 = time.perf_counter()
    for it in range(iters):
        idx = torch.from_numpy(rng.choice(Y.size, size=min(batch, Y.size), replace=False)).to("cuda")
        xb, yb = Xt.index_select(0, idx).contiguous(), Yt.index_select(0, idx).contiguous()
        want = it % 10 == 9 or it < 10 or it >= iters - 10
        loss = ctx.net_train_step_dev(xb, yb, cw, lr=3e-3, want_loss=want)
        if want:
            losses.append(loss)
    _sync()
    t_train = time.perf_counter() - t1
    params = ctx.net_params()
    ctx.close()
    print(f"[bench] learned: trained on {Y.size} samples {counts.tolist()}, loss {np.mean(losses[:10]):.3f} -> "
          f"{np.mean(losses[-10:]):.3f}", file=sys.stderr, flush=True)
    names = {gf.GF_RUN_PLAIN: "plain_every_4", gf.GF_RUN_SPARSE: "plain_every_16", gf.GF_RUN_LEARNED: "learned_every_16",
             "dilated": "plain_dilated_every_16"}
    acc = {v: {"regrids": 0, "forced_regrids": 0, "checks": 0, "misses": 0, "leaf_steps": 0, "seconds": 0.0,
               "max_abs_dh_vs_plain": [], "mean_abs_dh_wet": [], "frac_dh_over_10cm": [], "budget_residual_rel": []}
           for v in names.values()}
    for j in range(n_eval):
        hp = None
        for mode in (gf.GF_RUN_PLAIN, gf.GF_RUN_SPARSE, gf.GF_RUN_LEARNED, "dilated"):
            sc, c2 = make(5051 + j)
            c2.net_set_params(params)
            m0 = c2.mass(0)
            if mode == "dilated":
                st = _dilated_run(c2, sc, steps, check, window)
            else:
                st = c2.run(steps, mode, check, window)
            M = c2.mass(0)
            h = _finest_depth(sc, c2.leaves(0), c2.state(0), sc.max_level)
            hp = h if mode == gf.GF_RUN_PLAIN else hp
            a = acc[names[mode]]
            for k in ("regrids", "forced_regrids", "checks", "misses", "leaf_steps"):
                a[k] += int(getattr(st, k))
            a["seconds"] += st.seconds
            d = np.abs(h - hp)
            wet = (h > 1e-2) | (hp > 1e-2)
            a["max_abs_dh_vs_plain"].append(float(d.max()))
            a["mean_abs_dh_wet"].append(float(d[wet].mean()) if wet.any() else 0.0)
            a["frac_dh_over_10cm"].append(float(np.count_nonzero(d[wet] > 0.1)) / max(int(wet.sum()), 1))
            a["budget_residual_rel"].append(float(abs((M[0] - m0[0]) - (M[1] - m0[1]) - (M[2] - m0[2])) / m0[0]))
            c2.close()
        print(f"[bench] learned: evaluated seed {5051 + j}", file=sys.stderr, flush=True)
    for a in acc.values():
        a["miss_rate"] = a["misses"] / max(a["checks"], 1)
        d = a.pop("max_abs_dh_vs_plain")
        a["max_abs_dh_vs_plain_m"] = {"max": max(d), "median": float(np.median(d))}
        a["mean_abs_dh_wet_vs_plain_m"] = float(np.mean(a.pop("mean_abs_dh_wet")))
        a["frac_wet_cells_dh_over_10cm"] = float(np.mean(a.pop("frac_dh_over_10cm")))
        a["budget_residual_rel_max"] = max(a.pop("budget_residual_rel"))
    return {"workload": "reservoir geometry as AMR: 10 km fractal terrain, levels 0-6 of 32x32 patches, reservoir "
                        "h=20 m r=400 m at a seeded centre, n=0.033; FP32",
            "train_seeds": n_train, "eval_seeds": n_eval, "steps_per_run": steps, "samples": int(Y.size),
            "classes_coarsen_keep_refine": counts.tolist(), "train_iters": iters, "batch": batch,
            "train_s": t_train, "loss_start_end": [float(np.mean(losses[:10])), float(np.mean(losses[-10:]))],
            "modes": acc}


def guarded(fn, *a, **kw):
    """An extra workload's section, or the error that stopped it."""
    try:
        return fn(*a, **kw)
    except Exception as e:  # reported in the JSON line, which still prints
        print(f"[bench] {fn.__name__} failed: {e!r}", file=sys.stderr, flush=True)
        return {"error": repr(e)}



def valley_mesh():
    """The valley, its mesh built from level 0 by gf_set_initial's plain-tagger
    passes (FP32 state)."""
    import paper_2403_15435_amd as gf
    from paper_2403_15435_amd import inputs
    sc = inputs.v_valley()
    base = gf.Context([sc], precision=gf.GF_FP32, max_patches=48000)
    base.set_initial(0, max_passes=sc.max_level - sc.min_level)
    leaves, state = base.leaves(0), base.state(0)
    base.close()
    print(f"[bench] valley mesh: {leaves.shape[0]} leaves, levels {np.bincount(leaves[:, 1]).tolist()}",
          file=sys.stderr, flush=True)
    return sc, leaves, state


def amr_window(ctx, steps, regrid_every=4, plain=False):
    """`steps` steps with a plain tag and regrid after every `regrid_every`
    (the adaptive job).  Returns (cell updates, wall time of the whole window,
    time inside the step calls, accepted steps, rejected attempts); each call
    returns synchronised."""
    cells, t_step, done, acc, rej = 0, 0.0, 0, 0, 0
    _sync()
    t0 = time.perf_counter()
    while done < steps:
        n = min(regrid_every, steps - done)
        a = time.perf_counter()
        st = ctx.step(n, plain=plain)
        t_step += time.perf_counter() - a
        cells += int(st.cell_updates)
        acc += int(st.steps)
        rej += int(st.rejected)
        done += n
        ctx.tag()
        ctx.regrid(None)
    _sync()
    return cells, time.perf_counter() - t0, t_step, acc, rej


def _restore(ctx, snap):
    leaves, state, t, dt = snap
    ctx.set_leaves(0, leaves)
    ctx.set_state(0, state[:, :3])
    ctx.set_time(0, t, dt)


def valley_headline(steps, warmup, regrid_every=4, t0=4000.0, paths=("fp32_fused", "fp64_fused", "fp64_plain"),
                    shape=None):
    """The headline: the valley on the fused FP32 path (the timed window),
    then the same window again with the step kernel's launches timed alone,
    and once more with the kernels counting the patches they update; the
    fused FP64 and plain FP64 paths from the same mesh and state.  The fused
    paths take the autotuner's shape, or `shape` = (threads, padding,
    schedule) for the FP32 path when given (profiling runs)."""
    import paper_2403_15435_amd as gf
    sc, leaves0, state0 = valley_mesh()
    cap = 48000
    out = {"workload": VALLEY_DESC, "leaves_start": int(leaves0.shape[0]),
           "levels_start": np.bincount(leaves0[:, 1]).tolist(), "steps": steps, "regrid_every": regrid_every}
    snap = None
    for name in paths:
        prec = gf.GF_FP32 if name == "fp32_fused" else gf.GF_FP64
        plain = name == "fp64_plain"
        ctx = gf.Context([sc], precision=prec, max_patches=cap)
        if snap is None:
            _restore(ctx, (leaves0, state0, t0, 0.0))
        else:
            _restore(ctx, snap)
        res = {}
        if shape is not None and name == "fp32_fused":
            ctx.set_step_threads(shape[0])
            ctx.set_step_pad(shape[1])
            ctx.set_schedule(shape[2])
            res["shape_fixed"] = list(shape)
        elif not plain:
            res["tuned"] = list(ctx.autotune(steps=3))
            res["tuned_pad"] = ctx.autotune_choice()[2]
            res["tune_trials"] = [{"threads": t[0], "schedule": t[1], "pad": t[2], "us_per_step": t[3]}
                                  for t in ctx.autotune_trials()]
        if snap is None:
            # the warm-up, then the window every path starts from
            amr_window(ctx, warmup, regrid_every)
            snap = (ctx.leaves(0), ctx.state(0), *ctx.time(0)[:2])
            _restore(ctx, snap)
        else:
            amr_window(ctx, min(warmup, 8), regrid_every, plain)
            _restore(ctx, snap)
        m0 = ctx.mass(0)
        cells, wall, t_step, acc, rej = amr_window(ctx, steps, regrid_every, plain)
        M = ctx.mass(0)
        res.update({"cell_updates_per_s": cells / wall, "step_cell_updates_per_s": cells / t_step,
                    "wall_s": wall, "step_s": t_step, "tag_regrid_s": wall - t_step, "cell_updates": cells,
                    "accepted_steps": acc, "rejected": rej, "leaves_end": int(ctx.leaves(0).shape[0]),
                    "budget_residual_rel": float(((M[0] - m0[0]) - (M[1] - m0[1]) - (M[2] - m0[2])) / M[0])})
        if name == "fp32_fused":
            res["step_threads"] = ctx.step_threads()
            res["step_pad"] = shape[1] if shape is not None else res["tuned_pad"]
            # repeat 1: the step kernel's launches timed alone (event pairs)
            _restore(ctx, snap)
            ctx.profile_enable(False, kernel=True)
            c2 = amr_window(ctx, steps, regrid_every)[0]
            n_launch, ms = ctx.profile_kernel()
            ctx.profile_enable(False)
            # repeat 2: the patches the step kernel updated
            _restore(ctx, snap)
            ctx.profile_enable(False, patches=True)
            c3 = amr_window(ctx, steps, regrid_every)[0]
            full, stable = ctx.profile_patches()
            ctx.profile_enable(False)
            res.update({"repeat_cell_updates_equal": bool(c2 == cells and c3 == cells),
                        "step_kernel_launches": n_launch, "step_kernel_avg_us": 1e3 * ms / max(n_launch, 1),
                        "patches_full_update": full, "patches_stable_dry": stable})
        print(f"[bench] valley {name}: {res}", file=sys.stderr, flush=True)
        out[name] = res
        ctx.close()
    if "fp64_plain" in out and "fp32_fused" in out:
        out["speedup_fp32_fused_over_fp64_plain"] = (out["fp32_fused"]["cell_updates_per_s"]
                                                     / out["fp64_plain"]["cell_updates_per_s"])
        out["speedup_step_fp32_fused_over_fp64_plain"] = (out["fp32_fused"]["step_cell_updates_per_s"]
                                                          / out["fp64_plain"]["step_cell_updates_per_s"])
    if "fp64_fused" in out and "fp32_fused" in out:
        out["speedup_fp32_over_fp64_fused"] = (out["fp32_fused"]["cell_updates_per_s"]
                                               / out["fp64_fused"]["cell_updates_per_s"])
    return out


def run_reservoir(sc, precision, warmup, steps, plain=False):
    """The uniform 2048^2 reservoir (a further section): `steps` steps timed on
    the host clock; the fused path's step kernel timed alone in a repeat of
    the window, and the patches it updated counted in another."""
    import paper_2403_15435_amd as gf
    ctx = gf.Context([sc], precision=precision, max_patches=4096)
    ctx.set_initial(0)
    if not plain:
        ctx.autotune(steps=5)
    ctx.step(warmup, plain=plain)
    state0 = ctx.state(0)[:, :3]
    t_0, dt_0 = ctx.time(0)[:2]
    _sync()
    t0 = time.perf_counter()
    st = ctx.step(steps, plain=plain)
    _sync()
    wall = time.perf_counter() - t0
    out = {"wall": wall, "cell_updates": int(st.cell_updates), "steps": int(st.steps), "rejected": int(st.rejected)}
    if not plain:
        for kw in ({"kernel": True}, {"patches": True}):
            ctx.set_state(0, state0)
            ctx.set_time(0, t_0, dt_0)
            ctx.profile_enable(False, **kw)
            ctx.step(steps)
            if "kernel" in kw:
                n, ms = ctx.profile_kernel()
                out["step_kernel_launches"], out["step_kernel_avg_us"] = n, 1e3 * ms / max(n, 1)
            else:
                out["patches_full_update"], out["patches_stable_dry"] = ctx.profile_patches()
            ctx.profile_enable(False)
        out["step_threads"] = ctx.step_threads()
        h = ctx.state(0)[:, 0]
        out["wet_cell_fraction_end"] = float(np.count_nonzero(h > 1e-4)) / h.size
    ctx.close()
    return out


def reservoir_section(steps, warmup, wet_steps):
    """The uniform reservoir (most patches dry or stable, a few hundred
    updated per step) and the same grid fully wet, FP32 fused, FP64 fused and
    FP64 plain."""
    import paper_2403_15435_amd as gf
    sc = workload()
    out = {"workload": "uniform 2048x2048 cells (64x64 patches of 32x32), 10 km fractal terrain 100+/-50 m, "
                       "reservoir h=20 m r=400 m, n=0.033, walls, adaptive CFL 0.9", "steps": steps}
    r32 = run_reservoir(sc, gf.GF_FP32, warmup, steps)
    r64 = run_reservoir(sc, gf.GF_FP64, warmup, steps)
    rp = run_reservoir(sc, gf.GF_FP64, warmup, steps, plain=True)
    cups = {k: v["cell_updates"] / v["wall"] for k, v in (("fp32_fused", r32), ("fp64_fused", r64), ("fp64_plain", rp))}
    upd = r32["patches_full_update"] * 1024 / max(r32["step_kernel_launches"], 1)
    t = r32["step_kernel_avg_us"] * 1e-6
    out.update({"cell_updates_per_s": cups, "fp32_fused": r32,
                "speedup_fp32_fused_over_fp64_plain": cups["fp32_fused"] / cups["fp64_plain"],
                "step_kernel_cells_updated_per_launch": upd,
                "step_kernel_hbm_frac": BYTES_PER_UPDATE["f32"] * upd / t / 1e9 / HBM_PEAK_GBS,
                "dense_equivalent_hbm_frac": BYTES_PER_UPDATE["f32"] * 4096 * 1024 / t / 1e9 / HBM_PEAK_GBS})
    if wet_steps > 0:
        w32 = run_reservoir(wet_workload(), gf.GF_FP32, 10, wet_steps)
        tw = w32["step_kernel_avg_us"] * 1e-6
        out["all_wet"] = {"workload": "same grid and terrain under a lake at 155 m (every cell wet), column at 165 m",
                          "fp32_cell_updates_per_s": w32["cell_updates"] / w32["wall"],
                          "step_kernel_avg_us": w32["step_kernel_avg_us"],
                          "step_kernel_hbm_frac": BYTES_PER_UPDATE["f32"] * 4096 * 1024 / tw / 1e9 / HBM_PEAK_GBS}
    print(f"[bench] reservoir: {out}", file=sys.stderr, flush=True)
    return out


# the learned-tagger section: bounded by default (a few seeds and a shorter
# run), the full configuration (50 training and 10 evaluation seeds) on request
LEARNED = {"small": dict(n_train=4, n_eval=2, steps=400, iters=200),
           "full": dict(n_train=50, n_eval=10, steps=2000, iters=400)}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(t0=4000.0, steps_all=4, steps_one=2):
    """The oracle on the same valley (its own mesh from the same refinement
    passes; it takes nothing from the GPU path): `steps_all` adaptive steps on
    every host thread OpenMP offers (OMP_NUM_THREADS, or every core), then
    `steps_one` on one thread."""
    import oracle
    from paper_2403_15435_amd import inputs
    from paper_2403_15435_amd.inputs import initial_state
    oracle.build(force=False)
    sc = inputs.v_valley()
    o = oracle.Oracle(sc)

    def recipe():
        lv = o.leaves()
        for k in range(lv.shape[0]):
            h, hu, hv = initial_state(sc, lv[k], o.get_field(k, 3), "f64")
            o.set_field(k, 0, np.asarray(h, np.float64))
            o.set_field(k, 1, np.asarray(hu, np.float64))
            o.set_field(k, 2, np.asarray(hv, np.float64))
    recipe()
    for _ in range(sc.max_level - sc.min_level):
        f = o.tag()
        if not f.any():
            break
        o.regrid(f)
        recipe()
    o.set_time(t0, 0.0)
    n_leaves = o.n_leaves
    res = {}
    for label, nt, steps in (("all", 0, steps_all), ("one", 1, steps_one)):
        used = oracle.set_threads(nt)
        s0 = o.steps
        a = time.perf_counter()
        o.advance(steps)
        dt = time.perf_counter() - a
        res[label] = {"threads": used, "steps": o.steps - s0, "s": dt,
                      "cell_updates_per_s": (o.steps - s0) * n_leaves * sc.m * sc.m / dt}
    oracle.set_threads(0)
    return {"value": res["all"]["cell_updates_per_s"], "unit": "cell-updates/s", "cores": res["all"]["threads"],
            "kind": "oracle",
            "sample": (f"{res['all']['steps']} adaptive steps of the valley ({n_leaves} leaves, levels 0-6, its own "
                       f"mesh from the same refinement passes; FP64) on {res['all']['threads']} threads "
                       f"({res['all']['s']:.1f} s), then {res['one']['steps']} on one thread ({res['one']['s']:.1f} s)"),
            "one_thread_cell_updates_per_s": res["one"]["cell_updates_per_s"],
            "host": {"cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count(),
                     "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}}


def read_summary(path):
    """Key: value lines of a committed profile summary, or None when it is
    missing or was taken on other kernel sources."""
    from paper_2403_15435_amd.build import source_digest
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", " ")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_digest") != source_digest():
        return None
    return kv


def _num(kv, key):
    try:
        return float(kv[key]) if kv and key in kv else None
    except ValueError:
        return None


def triad_probe(n=1 << 28, reps=10):
    """Achievable HBM bandwidth: the library's triad kernel c = a + s b on
    three arrays of n floats (3 GiB), `reps` launches each timed with a HIP
    event pair on the stream it runs on; 12 n bytes per launch."""
    import torch
    import paper_2403_15435_amd as gf
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.full((n,), 2.0, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)
    gf.probe_triad(a, b, c)
    torch.cuda.synchronize()
    assert float(c[0]) == 7.0 and float(c[-1]) == 7.0
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        gf.probe_triad(a, b, c)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    gbs = [12.0 * n / t / 1e9 for t in times]
    del a, b, c
    torch.cuda.empty_cache()
    return {"kernel": "gf_probe_triad (c = a + s b, float4 grid-stride)", "bytes_per_launch": 12 * n,
            "best_GBps": max(gbs), "median_GBps": float(np.median(gbs)), "launches": reps}


def calibrate_copy(mib=512, reps=5):
    """Device-to-device copy of a known size, run under the same HBM byte
    counters as the step kernel to scale them: each copy reads and writes
    `mib` MiB exactly once."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_kib_read": mib * 1024, "copy_kib_written": mib * 1024, "reps": reps}))


def roofline(v32, probe):
    """The step kernel's roofline from the headline's repeats: cells it
    updated per launch (patch counts), its average launch (event pairs); the
    issued VALU operations and HBM bytes per launch from the committed counter
    summary of this workload when it matches the kernel sources; the bound
    from those counters."""
    n = max(v32["step_kernel_launches"], 1)
    t = v32["step_kernel_avg_us"] * 1e-6
    cells = v32["patches_full_update"] * 1024.0 / n
    dense = v32["cell_updates"] / max(v32["accepted_steps"] + v32["rejected"], 1)
    alg_ops = ALGO_OPS_PER_UPDATE * cells
    hbm_gbs = BYTES_PER_UPDATE["f32"] * cells / t / 1e9
    # the committed summaries count only when taken on the same kernel
    # sources and the same step-kernel shape (threads, LDS row padding)
    shape = f"{v32.get('step_threads')},{v32.get('step_pad')}"
    kv, stats = read_summary(VALLEY_COUNTERS), read_summary(VALLEY_STATS)
    if kv and kv.get("kernel_shape") != shape:
        kv = None
    if stats and stats.get("kernel_shape") != shape:
        stats = None
    valu_per_launch = _num(kv, "valu_lane_ops_per_launch")
    traffic = None
    if kv and _num(kv, "fetch_kib_per_launch") is not None:
        traffic = 1024.0 * (_num(kv, "fetch_kib_per_launch") * _num(kv, "fetch_scale")
                            + _num(kv, "write_kib_per_launch") * _num(kv, "write_scale"))
    issued_frac = valu_per_launch / t / 1e9 / VALU_PEAK_GOPS if valu_per_launch else None
    traffic_frac = traffic / t / 1e9 / HBM_PEAK_GBS if traffic else None
    if issued_frac is not None and traffic_frac is not None:
        bound, source = ("alu", "counters") if issued_frac >= traffic_frac else ("hbm", "counters")
    else:
        bound, source = "alu", ("no counters for these kernel sources and this shape: "
                                "the method's arithmetic intensity")
    achieved = alg_ops / t / 1e9
    return {"bound": bound, "bound_from": source, "achieved": achieved, "peak": VALU_PEAK_GOPS,
            "unit": "Gop/s (VALU lane operations, non-packed FP32)", "frac": achieved / VALU_PEAK_GOPS,
            "traffic": traffic, "traffic_unit": "HBM bytes per launch (counters x copy calibration)",
            "kernel": f"step_kernel<32,{v32.get('step_threads')},{v32.get('step_pad')}> fp32", "launches": n,
            "avg_launch_us": t * 1e6, "rocprof_avg_launch_us": _num(stats, "step_kernel_avg_us"),
            "cells_updated_per_launch": cells, "algorithmic_ops_per_cell": ALGO_OPS_PER_UPDATE,
            "algorithmic_ops_per_launch": alg_ops,
            "issued_valu_ops_per_cell": valu_per_launch / cells if valu_per_launch else None,
            "issued_valu_frac": issued_frac,
            "hbm": {"algorithmic_bytes_per_launch": BYTES_PER_UPDATE["f32"] * cells, "achieved": hbm_gbs,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm_gbs / HBM_PEAK_GBS,
                    "frac_of_achievable": hbm_gbs / probe["best_GBps"] if probe else None,
                    "traffic_frac": traffic_frac,
                    "dense_equivalent_frac": BYTES_PER_UPDATE["f32"] * dense / t / 1e9 / HBM_PEAK_GBS},
            "hbm_achievable": probe}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400, help="timed steps of the headline valley window")
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--reservoir-steps", type=int, default=2000, help="steps of the uniform reservoir section (0: skip)")
    ap.add_argument("--wet-steps", type=int, default=200, help="steps of the all-wet run (0: skip)")
    ap.add_argument("--ensemble-steps", type=int, default=200, help="steps of each ensemble run (0: skip)")
    ap.add_argument("--flood-steps", type=int, default=400, help="steps of each floodplain AMR run (0: skip)")
    ap.add_argument("--lts-steps", type=int, default=64, help="single-clock steps of the local-time-stepping window (0: skip)")
    ap.add_argument("--learned", choices=["off", "small", "full"], default="small",
                    help="learned-tagger section: small (a few seeds, bounded), full (50 + 10 seeds)")
    ap.add_argument("--only", choices=["valley", "fp32", "reservoir", "ensemble", "learned", "flood", "lts", "triad"],
                    default=None, help="run only this section and print it (fp32: the headline's FP32 path only)")
    ap.add_argument("--shape", default=None,
                    help="threads,padding,schedule of the FP32 step kernel instead of the autotuner's (--only fp32)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (for scaling HBM byte counters)")
    args = ap.parse_args()
    shape = tuple(int(v) for v in args.shape.split(",")) if args.shape else None
    if shape is not None and len(shape) != 3:
        ap.error("--shape takes threads,padding,schedule")
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding is not built", file=sys.stderr)
        sys.exit(2)
    only = {"valley": lambda: valley_headline(args.steps, args.warmup),
            "fp32": lambda: valley_headline(args.steps, args.warmup, paths=("fp32_fused",), shape=shape),
            "reservoir": lambda: reservoir_section(args.reservoir_steps, 50, args.wet_steps),
            "ensemble": lambda: ensemble(args.ensemble_steps, 10),
            "lts": lambda: lts_compare(args.lts_steps),
            "flood": lambda: flood_speed_amr(args.flood_steps, 40),
            "learned": lambda: learned_tagger(**LEARNED[args.learned if args.learned != "off" else "small"]),
            "triad": triad_probe}
    if args.only:
        print(json.dumps(only[args.only]()))
        return
    probe = triad_probe()
    print(f"[bench] triad probe: {probe}", file=sys.stderr, flush=True)
    v = valley_headline(args.steps, args.warmup)
    v32 = v["fp32_fused"]
    res = guarded(reservoir_section, args.reservoir_steps, 50, args.wet_steps) if args.reservoir_steps > 0 else None
    ens = guarded(ensemble, args.ensemble_steps, 10) if args.ensemble_steps > 0 else None
    flood = guarded(flood_speed_amr, args.flood_steps, 40) if args.flood_steps > 0 else None
    ltsc = guarded(lts_compare, args.lts_steps) if args.lts_steps > 0 else None
    learned = guarded(learned_tagger, **LEARNED[args.learned]) if args.learned != "off" else None
    cpu = None
    if not args.no_cpu:
        cpu = guarded(cpu_baseline)
        print(f"[bench] cpu baseline: {cpu}", file=sys.stderr, flush=True)
    line = {
        "metric": METRIC, "value": v32["cell_updates_per_s"], "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * v32["wall_s"] / max(args.steps, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": VALLEY_DESC, "leaves": v["leaves_start"], "levels": v["levels_start"],
                   "cells_per_step": v["leaves_start"] * 1024, "regrid_every": 4},
        "roofline": roofline(v32, probe),
        "step_cell_updates_per_s": v32["step_cell_updates_per_s"],
        "fp64_plain": {"value": v["fp64_plain"]["cell_updates_per_s"], "unit": "cell-updates/s",
                       "step_cell_updates_per_s": v["fp64_plain"]["step_cell_updates_per_s"],
                       "path": "gf_step_plain: per step, ghost fill into ghosted tiles in HBM, one step launch per "
                               "level from them, Courant number read back and dt chosen on the host; same tag and "
                               "regrid every 4 steps",
                       "speedup_fp32_fused_over_fp64_plain": v["speedup_fp32_fused_over_fp64_plain"],
                       "speedup_step_fp32_fused_over_fp64_plain": v["speedup_step_fp32_fused_over_fp64_plain"]},
        "fp64_fused": {"value": v["fp64_fused"]["cell_updates_per_s"], "unit": "cell-updates/s",
                       "speedup_fp32_over_fp64_fused": v["speedup_fp32_over_fp64_fused"]},
        "cpu_baseline": cpu,
        "valley": v,
        "reservoir_2048": res,
        "ensemble": ens,
        "amr_floodplain": flood,
        "local_time_stepping": ltsc,
        "learned_tagger": learned,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
