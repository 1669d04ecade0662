"""Benchmark: cell updates per second of the FP32 patch update on one MI355X.

Workload (one step = one full pass of ghost fill + wave-propagation update +
friction + positivity + step control over every patch): uniform 2048 x 2048
cells as 64 x 64 patches of 32 x 32 on a 10 km square of seeded fractal
terrain (100 +/- 50 m), circular reservoir of depth 20 m and radius 400 m,
Manning n = 0.033, walls.  A step is two kernels: the classification and
update of dry patches, then the full update of the others.  Reported beside
it: the same run on the plain FP64 path (ghost fill into ghosted tiles in
device memory, a step launch per level, the step length chosen on the host:
the comparator of the speedup) and on the fused FP64 path, the step's HBM
roofline fraction (algorithmic 28 B per FP32 cell update), the same grid fully
wet, and the CPU oracle timed on a bounded sample of the same workload.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_fp32_reservoir2048_hbm_traffic.txt")
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = {"f32": 28.0, "f64": 56.0}


def workload():
    from paper_2403_15435_amd import inputs
    return inputs.reservoir_fractal(level=6, m=32, L=10000.0, seed=2, radius=400.0, h_res=20.0, manning_n=0.033)


def wet_workload():
    from paper_2403_15435_amd import inputs
    return inputs.wet_dambreak(level=6, m=32, L=10000.0, seed=2, radius=400.0, manning_n=0.033)


def run_gpu(sc, precision, warmup, steps, step_threads=None, wet_fraction=False, plain=False):
    import torch
    import paper_2403_15435_amd as gf
    ctx = gf.Context([sc], precision=precision, max_patches=4096)
    ctx.set_initial(0)
    ctx.step(warmup, plain=plain)
    tuned = None
    if plain:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.step(steps, plain=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out = {"wall": wall, "cell_updates": int(st.cell_updates), "steps": int(st.steps),
               "rejected": int(st.rejected), "mass": ctx.mass(0).tolist()}
        ctx.close()
        return out
    if step_threads:
        ctx.set_step_threads(step_threads)
    else:
        # launch shape from the tuner (state restored after its trials)
        tuned = ctx.autotune(steps=5)
    torch.cuda.synchronize()
    # the timed run: HIP events on the library's stream bracket its launches
    # (nothing is queued between the kernels); a second run of the same window
    # (state and clock restored) has the kernels count patches
    state0 = ctx.state(0)[:, :3]
    t_0, dt_0 = ctx.time(0)[:2]
    ctx.profile_enable(True)
    t0 = time.perf_counter()
    st = ctx.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches, ms = ctx.profile_read()
    ctx.profile_enable(False)
    cells = int(st.cell_updates)
    ctx.set_state(0, state0)
    ctx.set_time(0, t_0, dt_0)
    ctx.profile_enable(False, patches=True)
    st2 = ctx.step(steps)
    torch.cuda.synchronize()
    full, stable = ctx.profile_patches()
    ctx.profile_enable(False)
    assert int(st2.cell_updates) == cells
    mass = ctx.mass(0)
    out = {"wall": wall, "cell_updates": cells, "steps": int(st.steps), "launches": launches, "kernel_ms": ms,
           "rejected": int(st.rejected), "mass": mass.tolist(), "step_threads": ctx.step_threads(), "tuned": tuned,
           "full_patch_updates": full, "stable_dry_patches": stable}
    if wet_fraction:
        h = ctx.state(0)[:, 0]
        out["wet_cell_fraction"] = float(np.count_nonzero(h > 1e-4)) / h.size
    ctx.close()
    return out


def _sync():
    import torch
    torch.cuda.synchronize()


def valley_amr(steps, warmup, regrid_every=4, t0=4000.0):
    """The AMR workload: the inflow valley (20 km x 10 km, 16 x 8 trees, levels
    0-6 of 32 x 32 patches, finest cells 0.61 m), refined from level 0 around
    its normal-depth flood by the plain tagger, started on the hydrograph's
    plateau (5000 m^3/s); tag and regrid every `regrid_every` steps.  Run on
    the fused FP32 path, the fused FP64 path and the plain FP64 path from the
    same mesh and state (the FP32 one, widened)."""
    import paper_2403_15435_amd as gf
    from paper_2403_15435_amd import inputs
    sc = inputs.v_valley()
    cap = 48000
    base = gf.Context([sc], precision=gf.GF_FP32, max_patches=cap)
    base.set_initial(0)
    for _ in range(sc.max_level - sc.min_level):
        base.tag()
        base.regrid(None)
        base.set_initial(0)
    leaves0, state0 = base.leaves(0), base.state(0)
    base.close()
    print(f"[bench] valley mesh: {leaves0.shape[0]} leaves, levels {sorted(set(leaves0[:, 1].tolist()))}",
          file=sys.stderr, flush=True)
    out = {"workload": "AMR inflow valley: 20 km x 10 km V valley (side slope 0.05, 2 m rms fractal roughness), "
                       "16x8 trees, levels 0-6 of 32x32 patches (finest 0.61 m), inflow 5000 m^3/s over 200 m, "
                       "n = 0.04, extrapolation outflow, walls; plain tagger and regrid every 4 steps",
           "leaves_start": int(leaves0.shape[0]), "steps": steps, "regrid_every": regrid_every}
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
        cups = cells / t_step
        out[name] = {"step_cell_updates_per_s": cups, "end_to_end_cell_updates_per_s": cells / (t_step + t_regrid),
                     "step_s": t_step, "tag_regrid_s": t_regrid, "leaves_end": int(ctx.leaves(0).shape[0]),
                     "budget_residual_rel": float(((M[0] - m0[0]) - (M[1] - m0[1]) - (M[2] - m0[2])) / M[0])}
        if prec == gf.GF_FP32:
            out[name]["hbm_frac_algorithmic"] = cups * BYTES_PER_UPDATE["f32"] / (HBM_PEAK_GBS * 1e9)
        print(f"[bench] valley {name}: {out[name]}", file=sys.stderr, flush=True)
        ctx.close()
    out["speedup_fp32_fused_over_fp64_plain"] = (out["fp32_fused"]["step_cell_updates_per_s"]
                                                 / out["fp64_plain"]["step_cell_updates_per_s"])
    return out


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


def learned_tagger(n_train=50, n_eval=10, steps=2000, window=16, check=4, iters=400, batch=256):
    """The learned tagger on the reservoir geometry as AMR: 10 km square,
    levels 0-6 of 32 x 32 patches (finest 4.88 m), reservoir r = 400 m with
    its centre drawn from U[2.5 km, 7.5 km]^2 by the seed.  Trained on the GPU
    from plain-tagger windows (a sample every 16 steps: every refine label,
    twice as many others drawn at random) of seeds 5001.., evaluated on the
    unseen seeds 5051..: the plain tagger every 4 steps (the judge), every 16
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
    losses = []
    t1 = time.perf_counter()
    for _ in range(iters):
        idx = rng.choice(Y.size, size=min(batch, Y.size), replace=False)
        losses.append(ctx.net_train_step(X[idx].astype(np.float64), Y[idx], cw, lr=3e-3))
    _sync()
    t_train = time.perf_counter() - t1
    params = ctx.net_params()
    ctx.close()
    print(f"[bench] learned: trained on {Y.size} samples {counts.tolist()}, loss {np.mean(losses[:10]):.3f} -> "
          f"{np.mean(losses[-10:]):.3f}", file=sys.stderr, flush=True)
    names = {gf.GF_RUN_PLAIN: "plain_every_4", gf.GF_RUN_SPARSE: "plain_every_16", gf.GF_RUN_LEARNED: "learned_every_16"}
    acc = {v: {"regrids": 0, "forced_regrids": 0, "checks": 0, "misses": 0, "leaf_steps": 0, "seconds": 0.0,
               "max_abs_dh_vs_plain": [], "budget_residual_rel": []} for v in names.values()}
    for j in range(n_eval):
        hp = None
        for mode in (gf.GF_RUN_PLAIN, gf.GF_RUN_SPARSE, gf.GF_RUN_LEARNED):
            sc, c2 = make(5051 + j)
            c2.net_set_params(params)
            m0 = c2.mass(0)
            st = c2.run(steps, mode, check, window)
            M = c2.mass(0)
            h = _finest_depth(sc, c2.leaves(0), c2.state(0), sc.max_level)
            hp = h if mode == gf.GF_RUN_PLAIN else hp
            a = acc[names[mode]]
            for k in ("regrids", "forced_regrids", "checks", "misses", "leaf_steps"):
                a[k] += int(getattr(st, k))
            a["seconds"] += st.seconds
            a["max_abs_dh_vs_plain"].append(float(np.abs(h - hp).max()))
            a["budget_residual_rel"].append(float(abs((M[0] - m0[0]) - (M[1] - m0[1]) - (M[2] - m0[2])) / m0[0]))
            c2.close()
        print(f"[bench] learned: evaluated seed {5051 + j}", file=sys.stderr, flush=True)
    for a in acc.values():
        a["miss_rate"] = a["misses"] / max(a["checks"], 1)
        d = a.pop("max_abs_dh_vs_plain")
        a["max_abs_dh_vs_plain_m"] = {"max": max(d), "median": float(np.median(d))}
        a["budget_residual_rel_max"] = max(a.pop("budget_residual_rel"))
    return {"workload": "reservoir geometry as AMR: 10 km fractal terrain, levels 0-6 of 32x32 patches, reservoir "
                        "h=20 m r=400 m at a seeded centre, n=0.033; FP32",
            "train_seeds": n_train, "eval_seeds": n_eval, "steps_per_run": steps, "samples": int(Y.size),
            "classes_coarsen_keep_refine": counts.tolist(), "train_iters": iters, "batch": batch,
            "train_s": t_train, "loss_start_end": [float(np.mean(losses[:10])), float(np.mean(losses[-10:]))],
            "modes": acc}


def guarded(fn, *a):
    """An extra workload's section, or the error that stopped it."""
    try:
        return fn(*a)
    except Exception as e:  # reported in the JSON line, which still prints
        print(f"[bench] {fn.__name__} failed: {e!r}", file=sys.stderr, flush=True)
        return {"error": repr(e)}


def cpu_baseline(sc, steps=48):
    import oracle
    from paper_2403_15435_amd.inputs import initial_state
    oracle.build(force=False)
    o = oracle.Oracle(sc)
    lv = o.leaves()
    for k in range(lv.shape[0]):
        h, hu, hv = initial_state(sc, lv[k], o.get_field(k, 3), "f64")
        o.set_field(k, 0, np.asarray(h, np.float64))
        o.set_field(k, 1, np.asarray(hu, np.float64))
        o.set_field(k, 2, np.asarray(hv, np.float64))
    t0 = time.perf_counter()
    o.advance(steps)
    dt = time.perf_counter() - t0
    cells = o.steps * lv.shape[0] * sc.m * sc.m
    return {"value": cells / dt, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{o.steps} adaptive steps of the full 2048^2 workload (FP64, one thread), {dt:.1f} s"}


def measured_traffic():
    """HBM bytes per step (both kernels) from the committed FETCH_SIZE /
    WRITE_SIZE counter summary, scaled by the copy-kernel calibration; None
    when the summary was taken on different kernel sources."""
    from paper_2403_15435_amd.build import source_digest
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_digest") != source_digest():
        return None
    try:
        fetch = float(kv["fetch_kib_per_step"]) * float(kv["fetch_scale"])
        write = float(kv["write_kib_per_step"]) * float(kv["write_scale"])
    except (KeyError, ValueError):
        return None
    return (fetch + write) * 1024.0


def profiled_kernel_us():
    """Average durations (us) of the reservoir FP32 dry and step kernels in
    the committed rocprofv3 kernel-trace summary; None when it was taken on
    other kernel sources."""
    from paper_2403_15435_amd.build import source_digest
    path = os.path.join(ROOT, "profiles", "step_reservoir2048_kernel_stats.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if source_digest() not in text or "Reservoir, FP32:" not in text:
        return None
    block = text.split("Reservoir, FP32:")[1].split("\n\n")[0]
    out = {}
    for line in block.splitlines():
        f = line.split()
        if "avg_ns" not in f:
            continue
        avg = float(f[f.index("avg_ns") + 1]) * 1e-3
        if "dry_kernel<32>" in line:
            out["dry_kernel_us"] = avg
        elif "step_kernel<32," in line and "512>" in line:
            out["step_kernel_us"] = avg
    return out or None


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--fp64-steps", type=int, default=0, help="steps of the FP64 run (0: the same as --steps)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--step-threads", type=int, default=0, help="step-kernel workgroup size (0: chosen by the tuner)")
    ap.add_argument("--workload", choices=["reservoir", "wet"], default="reservoir",
                    help="run only this grid (counter collection); the JSON line is for the reservoir")
    ap.add_argument("--wet-steps", type=int, default=200, help="steps of the all-wet comparison run (0: skip)")
    ap.add_argument("--precision", choices=["both", "f32", "f64", "plain"], default="both",
                    help="run only one path (for counter collection; plain: the FP64 comparator); "
                         "the JSON line needs all")
    ap.add_argument("--plain-steps", type=int, default=0, help="steps of the plain FP64 run (0: the same as --steps)")
    ap.add_argument("--amr-steps", type=int, default=400, help="steps of each AMR valley run (0: skip)")
    ap.add_argument("--ensemble-steps", type=int, default=200, help="steps of each ensemble run (0: skip)")
    ap.add_argument("--flood-steps", type=int, default=400, help="steps of each floodplain AMR run (0: skip)")
    ap.add_argument("--lts-steps", type=int, default=64, help="single-clock steps of the local-time-stepping window (0: skip)")
    ap.add_argument("--only", choices=["valley", "ensemble", "learned", "flood", "lts"], default=None,
                    help="run only this extra workload and print its section")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding is not built", file=sys.stderr)
        sys.exit(2)
    if args.only == "valley":
        print(json.dumps(valley_amr(args.amr_steps, 40)))
        return
    if args.only == "ensemble":
        print(json.dumps(ensemble(args.ensemble_steps, 10)))
        return
    if args.only == "lts":
        print(json.dumps(lts_compare(args.lts_steps)))
        return
    if args.only == "flood":
        print(json.dumps(flood_speed_amr(args.flood_steps, 40)))
        return
    if args.only == "learned":
        print(json.dumps(learned_tagger()))
        return
    import paper_2403_15435_amd as gf
    sc = workload() if args.workload == "reservoir" else wet_workload()
    print(f"[bench] workload ready: {sc.name}, {4096} patches", file=sys.stderr, flush=True)
    nt = args.step_threads or None
    if args.fp64_steps <= 0:
        args.fp64_steps = args.steps
    if args.plain_steps <= 0:
        args.plain_steps = args.steps
    if args.precision == "plain":
        rp = run_gpu(sc, gf.GF_FP64, min(args.warmup, 20), args.plain_steps, plain=True)
        print(f"[bench] plain fp64 done: {rp}", file=sys.stderr, flush=True)
        return
    if args.precision == "f64":
        r64 = run_gpu(sc, gf.GF_FP64, min(args.warmup, 20), args.fp64_steps, nt)
        print(f"[bench] fp64 done: {r64}", file=sys.stderr, flush=True)
        return
    r32 = run_gpu(sc, gf.GF_FP32, args.warmup, args.steps, nt, wet_fraction=True)
    print(f"[bench] fp32 done: {r32}", file=sys.stderr, flush=True)
    if args.precision == "f32":
        return
    r64 = run_gpu(sc, gf.GF_FP64, args.warmup, args.fp64_steps, nt)
    print(f"[bench] fp64 done: {r64}", file=sys.stderr, flush=True)
    rp = run_gpu(sc, gf.GF_FP64, args.warmup, args.plain_steps, plain=True)
    print(f"[bench] plain fp64 done: {rp}", file=sys.stderr, flush=True)
    wet = None
    if args.wet_steps > 0:
        wsc = wet_workload()
        w32 = run_gpu(wsc, gf.GF_FP32, 10, args.wet_steps, nt)
        w64 = run_gpu(wsc, gf.GF_FP64, 10, max(args.wet_steps // 2, 1), nt)
        print(f"[bench] all-wet fp32 {w32}\n[bench] all-wet fp64 {w64}", file=sys.stderr, flush=True)
        wl = w32["kernel_ms"] / max(w32["launches"], 1) / 1e3
        wet = {"workload": "same grid and terrain under a lake at 155 m (every cell wet), column at 165 m r=400 m",
               "fp32_cell_updates_per_s": w32["cell_updates"] / w32["wall"],
               "fp64_cell_updates_per_s": w64["cell_updates"] / w64["wall"],
               "fp32_step_us": wl * 1e6,
               "fp32_hbm_frac": BYTES_PER_UPDATE["f32"] * 4096 * 1024 / wl / 1e9 / HBM_PEAK_GBS,
               "step_threads": w32["step_threads"]}
    cups32 = r32["cell_updates"] / r32["wall"]
    cups64 = r64["cell_updates"] / r64["wall"]
    cupsp = rp["cell_updates"] / rp["wall"]
    cells_per_launch = 4096 * 32 * 32
    avg_launch_s = r32["kernel_ms"] / max(r32["launches"], 1) / 1e3
    achieved = BYTES_PER_UPDATE["f32"] * cells_per_launch / avg_launch_s / 1e9
    rp_us = profiled_kernel_us()
    rp_step = rp_us["dry_kernel_us"] + rp_us["step_kernel_us"] if rp_us and len(rp_us) == 2 else None
    amr = guarded(valley_amr, args.amr_steps, 40) if args.amr_steps > 0 else None
    ens = guarded(ensemble, args.ensemble_steps, 10) if args.ensemble_steps > 0 else None
    flood = guarded(flood_speed_amr, args.flood_steps, 40) if args.flood_steps > 0 else None
    ltsc = guarded(lts_compare, args.lts_steps) if args.lts_steps > 0 else None
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(sc)
        print(f"[bench] cpu baseline: {cpu}", file=sys.stderr, flush=True)
    line = {
        "metric": METRIC, "value": cups32, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * r32["wall"] / max(r32["steps"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "uniform 2048x2048 cells (64x64 patches of 32x32), 10 km fractal terrain 100+/-50 m, "
                               "reservoir h=20 m r=400 m, n=0.033, walls, adaptive CFL 0.9",
                   "patches": 4096, "cells": cells_per_launch},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "traffic_unit": "HBM bytes per launch (counters x copy calibration)",
                     "algorithmic_bytes_per_launch": BYTES_PER_UPDATE["f32"] * cells_per_launch,
                     "kernel": f"one step = dry_kernel<32> + step_kernel<32,{r32['step_threads']}> (fp32)",
                     # event pair on the library's stream around the timed launches, per step
                     "avg_launch_us": avg_launch_s * 1e6,
                     # the same kernels as rocprofv3 times them (committed summary of this command)
                     # and their sum, which the event figure above includes with the gaps between
                     # launches
                     "rocprof_kernel_us": rp_us,
                     "rocprof_step_us": rp_step,
                     "patches_full_update_per_step": r32["full_patch_updates"] / max(r32["launches"], 1),
                     "patches_stable_dry_per_step": r32["stable_dry_patches"] / max(r32["launches"], 1),
                     "step_kernel_hbm_frac": (BYTES_PER_UPDATE["f32"] * 1024 * r32["full_patch_updates"]
                                              / max(r32["launches"], 1)
                                              / (1e-6 * rp_us["step_kernel_us"]) / 1e9 / HBM_PEAK_GBS
                                              if rp_us and "step_kernel_us" in rp_us else None)},
        "fp64_plain": {"value": cupsp, "unit": "cell-updates/s", "steps": rp["steps"],
                       "path": "gf_step_plain: per step, ghost fill into ghosted tiles in HBM, one step launch per "
                               "level from them, Courant number read back and dt chosen on the host",
                       "speedup_fp32_fused_over_fp64_plain": cups32 / cupsp},
        "fp64_fused": {"value": cups64, "unit": "cell-updates/s", "steps": r64["steps"],
                       "speedup_fp32_over_fp64_fused": cups32 / cups64},
        "cpu_baseline": cpu,
        "wet_cell_fraction_end": r32.get("wet_cell_fraction"),
        "step_threads": r32.get("step_threads"),
        "all_wet": wet,
        "amr_valley": amr,
        "ensemble": ens,
        "amr_floodplain": flood,
        "local_time_stepping": ltsc,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
