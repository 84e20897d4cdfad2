"""Measured cost model for choosing the segment count p (the plan's autotuner).

For every padded block-size class the device is timed on small synthetic
batches (the library's own kernels, one persistent launch per class):
  workers   workgroups of the class's item sweeps for unsegmented systems
            (read back from the plan)
  workers_seg  the same for the items of segmented systems
  t_first   per-stage time of a first segment under full load
            (a batch of `workers` systems, p = 1, timed at horizons 8 and 24)
  t_fill    per-stage time of a segment carrying fill rows under full load
            (workers_seg / 2 systems with p = 2 and a one-stage first segment)
  t_item    fixed cost of an item (intercept of the p = 1 fit)
  t_fill    sigma * t_first, and
  t_red     rho * t_first, where sigma (a stage of a fill-carrying segment over
            a stage of a first segment) and rho (a stage of the reduced chain over
            a first-segment stage) come from the latency of single systems:
            N = 97 with the first or the second segment one stage long, and
            N = 127 cut into 64 one-stage segments
  family    (classes 24 and 32) the sweep family, i.e. the tile shape: the dense
            single-wave sweeps on 32-wide tiles or the row-lane sweeps of the
            class's width, whichever runs a full batch of 32-stage systems faster;
            every other figure of the class is measured with it
  t_level   the fixed cost of one more level of recursive segmentation: the
            latency of the same N = 127 system with its chain of 63 separators
            cut into 8 segments, less what its stages cost by the latencies
            above, in units of t_first
The result is cached as JSON per GPU architecture.  The chooser itself
(makespan = max(total work / workers, longest item)) runs in the C library.
"""
import json
import os
import time

import numpy as np

from . import kkt, workloads

CLASSES = kkt.CLASS_BLOCKS
# classes calibrated on the device (all of them; a class left out gets the stage
# costs of the widest measured class scaled by the cube of the block size)
MEASURED = CLASSES


def _cache_path(arch):
    base = os.environ.get("KKT_CACHE_DIR", os.path.join(os.path.expanduser("~"), ".cache", "kkt_mi355x"))
    return os.path.join(base, "cost_model_%s.json" % arch)


def _time_batch(dims, reps=3, nest=None, plan_out=None, family=None):
    import torch
    rng = np.random.default_rng(7)
    drawn = {}
    for d in dims:                      # one system per distinct shape, repeated
        if d[:3] not in drawn:
            drawn[d[:3]] = workloads.draw_system(rng, d[0], d[1], d[2], alpha=d[1])
    systems = [drawn[d[:3]] for d in dims]
    cm = None if family is None else {"family": list(family)}
    plan = kkt.Plan(dims, nrhs=1, nest=nest, cost_model=cm)
    if plan_out is not None:
        plan_out.append(plan)
    d = kkt.pack_to_device(workloads.pack(systems))
    ws = plan.new_workspace()
    info = torch.zeros(len(dims), dtype=torch.int32, device="cuda")
    x = torch.empty_like(d["r"])

    def run():
        x.copy_(d["r"])
        plan.factor_solve(d["D"], d["C"], d["B"], d["corner"], ws, x, info)

    run()
    torch.cuda.synchronize()
    a, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        run()
    b2.record()
    torch.cuda.synchronize()
    grid = max(g for *_, g in plan.classes(with_grid=True))
    return a.elapsed_time(b2) / reps, grid


def calibrate(verbose=False, classes=MEASURED):
    """Measure the classes in `classes`; any other class gets the stage costs of the
    widest measured class scaled by the cube of the block size (the flop ratio)."""
    keys = ("t_first", "t_fill", "t_red", "t_item", "workers", "workers_seg", "t_level", "family")
    model = {k: [0.0] * len(CLASSES) for k in keys}
    for c, bp in enumerate(CLASSES):
        if bp not in classes:
            continue
        b = bp
        fam = None
        if bp in (24, 32):
            # the tile shape: dense single-wave sweeps on 32-wide tiles or row-lane
            # sweeps of the class's width, each timed on a full batch of whole systems
            ft = {}
            for f in (1, 2):
                fl = [0.0] * len(CLASSES)
                fl[c] = float(f)
                _, Wf = _time_batch([(1, b, 2, 1)] * 8192, reps=1, family=fl)
                ft[f], _ = _time_batch([(32, b, 2, 1)] * max(1, Wf), family=fl)
            best = min(ft, key=ft.get)
            fam = [0.0] * len(CLASSES)
            fam[c] = float(best)
            model["family"][c] = float(best)
            if verbose:
                print("class %2d: dense sweeps %.3f ms, row-lane sweeps %.3f ms per full batch -> family %d"
                      % (bp, ft[1], ft[2], best), flush=True)
        _, W = _time_batch([(1, b, 2, 1)] * 8192, reps=1, family=fam)   # more items than slots: the full grid
        W = max(1, W)
        _, Ws = _time_batch([(3, b, 2, 2, 1)] * 8192, reps=1, family=fam)   # two items per system
        Ws = max(2, Ws)
        t1, _ = _time_batch([(8, b, 2, 1)] * W, family=fam)
        t2, _ = _time_batch([(24, b, 2, 1)] * W, family=fam)
        t_first = max((t2 - t1) / 16.0, 1e-6)
        t_item = max(t1 - 8 * t_first, 0.0)
        # stage-cost ratios from single-system latencies
        l33, _ = _time_batch([(33, b, 2, 1)], reps=5, family=fam)
        l97, _ = _time_batch([(97, b, 2, 1)], reps=5, family=fam)
        a = max((l97 - l33) / 64.0, 1e-6)                           # latency of a first-segment stage
        t0 = max(l33 - 33 * a, 0.0)
        lf, _ = _time_batch([(97, b, 2, 2, 1)], reps=5, family=fam)   # N1 = 1, Nk = 95 (fill rows)
        lh, _ = _time_batch([(97, b, 2, 2, 95)], reps=5, family=fam)  # N1 = 95, Nk = 1
        sigma = min(max(1.0 + (lf - lh) / (94.0 * a), 1.0), 8.0)
        lr, _ = _time_batch([(127, b, 2, 64, 1)], reps=5, family=fam)  # 64 one-stage segments
        rho = max((lr - t0 - max(1.0, sigma) * a) / (63.0 * a), 0.1)
        t_fill, t_red = sigma * t_first, rho * t_first
        # one more level: the chain of 63 separators cut into 8 segments (Eq. 13)
        made = []
        ln, _ = _time_batch([(127, b, 2, 64, 1)], reps=5, nest=[[8]], plan_out=made, family=fam)
        ch, cs, _ = made[0].reduced(0)
        n1, nk = ch.layouts[cs].N1, ch.layouts[cs].Nk
        stages = t0 + max(1.0, sigma) * a + max(n1 * a, nk * sigma * a) + 7 * rho * a
        t_level = max(ln - stages, 0.0) * t_first / a
        model["t_first"][c], model["t_fill"][c], model["t_red"][c] = t_first, t_fill, t_red
        model["t_item"][c], model["workers"][c], model["workers_seg"][c] = t_item, float(W), float(Ws)
        model["t_level"][c] = t_level
        if verbose:
            print("class %2d: workers %d / %d t_first %.4f t_fill %.4f t_red %.4f t_item %.4f t_level %.4f (ms); "
                  "latency per stage %.4f, sigma %.2f, rho %.2f, extra level %.4f"
                  % (bp, W, Ws, t_first, t_fill, t_red, t_item, t_level, a, sigma, rho, ln - stages), flush=True)
    ref = max(c for c, bp in enumerate(CLASSES) if bp in classes)
    for c, bp in enumerate(CLASSES):
        if bp in classes:
            continue
        scale = (bp / CLASSES[ref]) ** 3
        for k in ("t_first", "t_fill", "t_red", "t_item"):
            model[k][c] = model[k][ref] * scale
        model["t_level"][c] = model["t_level"][ref]
        model["workers"][c] = model["workers"][ref]
        model["workers_seg"][c] = model["workers_seg"][ref]
    return model


def cost_model(refresh=False, verbose=False):
    """The cached measured model for this GPU, calibrating it if needed."""
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    path = _cache_path(arch)
    if not refresh and os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    t0 = time.time()
    m = calibrate(verbose=verbose)
    m["arch"] = arch
    m["seconds"] = round(time.time() - t0, 2)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        json.dump(m, fh)
    return m
