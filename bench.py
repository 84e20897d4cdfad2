"""Benchmark: batched FP64 KKT factor + solve throughput on one MI355X.

A step is one pass of the whole hot path over the ragged batch workload
(4096 block-tridiagonal-arrow systems, N ~ U{16..256}, b ~ U{8,16,32},
ng ~ U{0,2,4}, one rhs): load the rhs, then factorization fused with the forward
substitution, the reduced separator/arrow phase and the backward substitution
for every system, through the C ABI (kkt_factor_solve).  Inputs are resident in
HBM before timing starts.  Prints ONE JSON line.

Besides the headline value it reports: the plain single-system GPU path (one
call per system) on a sample of the batch, the graph-replay time of the same
step, the differentiation workload (1024 x (N=64, b=24, ng=4), forward factor +
solve and adjoint backward), the relative residual of every system (gate 1e-10),
the roofline of the dominant persistent kernel (HIP events around it on its own
stream), and the oracle timed on the host (cpu_baseline).
"""
import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 30
SRC_FILES = ("paper_2511_00946_amd/csrc/kkt.hip", "paper_2511_00946_amd/csrc/kkt_wave.h",
             "paper_2511_00946_amd/csrc/kkt_lane.h", "paper_2511_00946_amd/csrc/kkt_kernels.h",
             "paper_2511_00946_amd/csrc/kkt_wave_inst.hip", "paper_2511_00946_amd/csrc/kkt_internal.h",
             "paper_2511_00946_amd/csrc/kkt_dense.h", "paper_2511_00946_amd/csrc/kkt_device.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_ragged4096.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class HipEvents:
    """Raw HIP events (the persistent kernels run on torch's current stream)."""

    def __init__(self):
        self.lib = ctypes.CDLL("libamdhip64.so")
        self.lib.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.lib.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        self.lib.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self):
        ev = ctypes.c_void_p()
        assert self.lib.hipEventCreate(ctypes.byref(ev)) == 0
        return ev.value

    def elapsed_ms(self, a, b):
        self.lib.hipEventSynchronize(ctypes.c_void_p(b))
        ms = ctypes.c_float()
        assert self.lib.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(a), ctypes.c_void_p(b)) == 0
        return float(ms.value)


def oracle_core_seconds(okkt, systems):
    """Seconds the oracle's C core spends on factor + solve of each system (steady
    clock around the factor and solve calls only; the assembly of the block matrix
    through the Python wrapper is left out)."""
    tot = 0.0
    for sy in systems:
        f = okkt.KKTFactor(sy.D, sy.C, sy.B, sy.corner, factor=False)
        t = time.perf_counter()
        f.factor()
        f.solve(sy.r)
        tot += time.perf_counter() - t
    return tot


def _oracle_worker(job):
    """One worker of the all-cores oracle baseline (its own process): the oracle's
    C core on the systems idx of the ragged batch of S systems, timed."""
    S, idx = job
    from oracle import kkt as okkt
    from paper_2511_00946_amd import workloads
    spec = workloads.ragged_batch_spec(S=S)
    systems = [spec.system(i) for i in idx]
    return oracle_core_seconds(okkt, systems)


def oracle_all_cores(S, csamp, max_workers=16):
    """The same oracle sample spread over the host's cores, one process per core
    (the systems are independent; no parallelism inside a system).  Returns
    (systems/s, workers) with the rate taken over the slowest worker."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    n = max(1, min(len(os.sched_getaffinity(0)), max_workers, len(csamp)))
    jobs = [(S, [int(i) for i in csamp[w::n]]) for w in range(n)]
    # fresh interpreters (spawn), never forks of this process; a worker that dies
    # raises here instead of leaving the pool waiting
    with ProcessPoolExecutor(n, mp_context=mp.get_context("spawn")) as pool:
        times = list(pool.map(_oracle_worker, jobs, timeout=600))
    return len(csamp) / max(times), n


def build_pools(spec, idx=None):
    """Pack systems (all, or the index list idx) of a BatchSpec into numpy pools."""
    from paper_2511_00946_amd import workloads
    idx = list(range(len(spec))) if idx is None else list(idx)
    systems = [spec.system(i) for i in idx]
    return systems, workloads.pack(systems)


def alg_bytes(plan, systems, adjoint=False):
    """Algorithmic HBM bytes per system of one fused factor + solve: read Psi once,
    write hat L once, read hat L once in the backward sweep, read r, write x.  With
    adjoint, plus one adjoint solve: read hat L, x and the incoming gradient, write
    lambda and the four gradient pools (the pattern of Psi)."""
    out = []
    for s, sy in enumerate(systems):
        lay = plan.layouts[s]
        N, b, ng, p, nk = lay.N, lay.b, lay.ng, lay.p, lay.Nk
        K = N * b * b + (N - 1) * b * b + N * ng * b + ng * ng
        fill = (p - 1) * (nk - 1) * b * b + max(p - 2, 0) * b * b if p > 1 else 0
        L = K + fill
        n = sy.n * plan.nrhs
        out.append(8.0 * (K + 2 * L + 2 * n + ((L + K + 3 * n) if adjoint else 0)))
    return np.asarray(out)


def source_digest():
    """sha256 over the kernel sources: counters taken from other sources do not apply."""
    import hashlib
    h = hashlib.sha256()
    for f in SRC_FILES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(bp, p, S):
    """HBM bytes per launch of the dominant kernel from the committed FETCH_SIZE /
    WRITE_SIZE passes (scaled by a plain copy's reading), or None when those were
    taken on other kernel sources or another workload."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != source_digest() or t.get("systems") != S or t.get("p") != p:
        return None
    k = t.get("kernels", {}).get(str(bp))
    return None if k is None else k.get("hbm_bytes_per_launch")


KIND_ROWLANE, KIND_DENSE, KIND_DSEG = 0, 1, 2
DENSE_GROUPS = (24, 32)


def in_class(bp, kind, b, p):
    """Whether a system of block size b split into p segments belongs to a launch class."""
    if class_of(b) != bp:
        return False
    if bp not in DENSE_GROUPS:
        return True
    return (p == 1) == (kind == KIND_DENSE)


def class_label(bp, kind):
    return {KIND_DENSE: "dense%d", KIND_DSEG: "dseg%d"}.get(kind, "%d") % bp


def class_of(b):
    for bp in (8, 16, 24, 32, 48):
        if b <= bp:
            return bp
    raise ValueError(b)


def fd_check(torch, kkt, workloads, dsys, dplan, dev, grads, systems=(0, 511, 1023), per_tensor=4, h=1e-6):
    """Central differences (step h) of L = sum(w * x) against the adjoint gradients on
    sampled entries of D, C, B and r; error relative to the largest gradient entry of
    that tensor in that system."""
    rng = np.random.default_rng(3)
    worst = 0.0
    for s in systems:
        sy = dsys[s]
        lay = dplan.layouts[s]
        plan = kkt.Plan([(sy.N, sy.b, sy.ng, lay.p)], nrhs=1)
        ws = plan.new_workspace(dev)
        info = torch.zeros(1, dtype=torch.int32, device=dev)
        base = {k: v.copy() for k, v in workloads.pack([sy]).items()}
        w = base["w"]
        offs = {"D": lay.off_D, "C": lay.off_C, "B": lay.off_B, "r": lay.off_rhs}
        for key in ("D", "C", "B", "r"):
            n = base[key].size
            if n == 0:
                continue
            g_sys = grads[key][offs[key]:offs[key] + n]
            scale = float(np.max(np.abs(g_sys)))
            for idx in rng.choice(n, size=per_tensor, replace=False):
                vals = []
                for sign in (1.0, -1.0):
                    pert = {k: v.copy() for k, v in base.items()}
                    pert[key].reshape(-1)[idx] += sign * h
                    d = kkt.pack_to_device(pert, dev)
                    x = d["r"].clone()
                    plan.factor_solve(d["D"], d["C"], d["B"], d["corner"], ws, x, info)
                    vals.append(float(np.sum(x.cpu().numpy() * w)))
                fd = (vals[0] - vals[1]) / (2 * h)
                worst = max(worst, abs(fd - float(g_sys[idx])) / scale)
    return worst


SINGLE_P = {"small": (1, 2, 4, 8), "race": (1, 2, 4, 8, 16, 32, 64, 128), "chain": (1, 4, 8, 16, 32)}


def nest_levels(plan, s=0):
    """[(p, N1, Nk)] of system s and of every level of its recursive segmentation."""
    out, pl = [], plan
    while True:
        lay = pl.layouts[s]
        out.append([lay.p, lay.N1, lay.Nk])
        r = pl.reduced(s)
        if r is None:
            return out
        pl, s, _ = r


def single_systems(torch, kkt, workloads, okkt, dev, cost_model=None, reps=50):
    """Latency of one factor + solve call on the single-system workloads, per
    segment count p and with the p the cost model picks; speedup vs p = 1."""
    out = {}
    for name, plist in SINGLE_P.items():
        sy = workloads.single(name)
        nrhs = sy.r.shape[1]
        pools = kkt.pack_to_device(workloads.pack([sy]), dev)
        tuned = kkt.Plan([(sy.N, sy.b, sy.ng, 0)], nrhs=nrhs, cost_model=cost_model)
        auto = tuned.segments()[0]
        res = {}
        # every p of the list with the Eq. 13 partition (sigma = 19/7), then the plan
        # the cost model makes (its p, split with its measured sigma)
        cases = [(p, kkt.Plan([(sy.N, sy.b, sy.ng, p)], nrhs=nrhs)) for p in sorted(set(plist) | {auto})]
        cases.append(("cost_model", tuned))
        for p, plan in cases:
            ws = plan.new_workspace(dev)
            info = torch.zeros(1, dtype=torch.int32, device=dev)
            x = torch.empty_like(pools["r"])

            def call():
                x.copy_(pools["r"])
                plan.factor_solve(pools["D"], pools["C"], pools["B"], pools["corner"], ws, x, info)

            for _ in range(5):
                call()
            torch.cuda.synchronize()
            a, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                call()
            b2.record()
            torch.cuda.synchronize()
            us = a.elapsed_time(b2) * 1e3 / reps
            xs = x.cpu().numpy().reshape(sy.n, nrhs)
            rr = okkt.rel_residual(sy.D, sy.C, sy.B, sy.corner, xs, sy.r)
            assert plan.workspace_error(ws) == 0 and int(info.item()) == 0 and rr <= 1e-10, (name, p, rr)
            res[p] = us
        base = res[1]
        out[name] = {"shape": "N=%d b=%d ng=%d nrhs=%d" % (sy.N, sy.b, sy.ng, nrhs),
                     "us_per_factor_solve": {str(p): round(v, 2) for p, v in res.items()},
                     "speedup_vs_p1": {str(p): round(base / v, 3) for p, v in res.items()},
                     "cost_model_p": auto,
                     "cost_model_segments": [tuned.layouts[0].N1, tuned.layouts[0].Nk],
                     "cost_model_levels": nest_levels(tuned)}
        log("single %s: %s" % (name, {p: round(v, 1) for p, v in res.items()}))
    return out


def qp_iteration(torch, kkt, workloads, dev, cost_model=None, reps=30):
    """One interior-point linear-algebra step of a multistage QP with the race-line
    system's shape (N 2048, b 6, ng 8, 4 rhs; 6 equality rows per group, the
    dynamics, and 12 inequality rows, two-sided bounds): assemble Psi, factor it
    once, then two right-hand-side sets (predictor, corrector), each reduced,
    solved and its dy, dz recovered.  The plan is the cost model's (recursive
    segmentation included).  Also the assembly kernel's HBM rate."""
    N, b, ng, pe, me, nrhs = 2048, 6, 8, 6, 12, 4
    rng = np.random.default_rng(6)
    q = workloads.draw_qp(rng, N, b, ng, pe, me)
    plan = kkt.Plan([(N, b, ng, 0)], nrhs=nrhs, cost_model=cost_model)
    qp = kkt.QP(plan, [pe], [me])
    pools = {k: torch.from_numpy(v).to(dev) for k, v in workloads.pack_qp([q]).items()}
    lens = plan.pool_lengths()
    z = lambda n: torch.zeros(n, dtype=torch.float64, device=dev)
    D, C, B, R = z(lens["D"]), z(lens["C"]), z(lens["B"]), z(lens["corner"])
    ws = plan.new_workspace(dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    vec = [(torch.from_numpy(rng.standard_normal(lens["rhs"])).to(dev),
            torch.from_numpy(rng.standard_normal(qp.lengths["ry"])).to(dev),
            torch.from_numpy(rng.standard_normal(qp.lengths["rz"])).to(dev)) for _ in range(2)]
    x, dy, dz = z(lens["rhs"]), z(qp.lengths["ry"]), z(qp.lengths["rz"])
    rho, delta = 1e-6, 1e-6

    def step():
        qp.assemble(pools, rho, delta, D, C, B, R)
        plan.factor(D, C, B, R, ws, info)
        for rx, ry, rz in vec:
            qp.reduce_rhs(pools, delta, rx, ry, rz, x)
            plan.solve(ws, x)
            qp.recover(pools, delta, x, ry, rz, dy, dz)

    def assemble_only():
        qp.assemble(pools, rho, delta, D, C, B, R)

    out = {"shape": "N=%d b=%d ng=%d pe=%d me=%d nrhs=%d" % (N, b, ng, pe, me, nrhs),
           "levels": nest_levels(plan)}
    for name, fn in (("us_per_iteration", step), ("us_assembly", assemble_only)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        a, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b2.record()
        torch.cuda.synchronize()
        out[name] = round(a.elapsed_time(b2) * 1e3 / reps, 2)
    assert int(info.item()) == 0
    # assembly bytes: read the cost and constraint pools, write Psi (and the corner partials)
    rd = sum(int(v.numel()) for v in pools.values()) * 8
    wr = (lens["D"] + lens["C"] + lens["B"] + lens["corner"] + N * ng * ng) * 8
    out["assembly_gbps"] = round((rd + wr) / (out["us_assembly"] * 1e-6) / 1e9, 1)
    log("qp iteration: %s" % out)
    return out


def qp_solves(torch, kkt, workloads, dev, cost_model=None, reps=3):
    """Whole interior-point solves (kkt_ipm_solve, every step on the device) of
    feasible strictly convex multistage QPs: one with the race-line system's shape
    (N 2048, b 6, ng 8, 6 equality and 12 inequality rows per group) on the cost
    model's plan, and a batch of 512 small ones (N 64, b 8, ng 2, 4 and 8 rows)."""
    out = {}
    for name, shape, count in (("race", (2048, 6, 8, 6, 12), 1), ("batch512", (64, 8, 2, 4, 8), 512)):
        rng = np.random.default_rng(7)
        probs = [workloads.draw_qp_problem(rng, *shape) for _ in range(count)]
        qps = [p[0] for p in probs]
        N, b, ng, pe, me = shape
        plan = kkt.Plan([(N, b, ng, 0)] * count, nrhs=1, cost_model=cost_model)
        qp = kkt.QP(plan, [pe] * count, [me] * count)
        pools = {k: torch.from_numpy(v).to(dev) for k, v in workloads.pack_qp(qps).items()}
        c = np.zeros(plan.info.rhs_len)
        beq = np.zeros(qp.lengths["ry"])
        h = np.zeros(qp.lengths["rz"])
        for i, (q, cv, bv, hv) in enumerate(probs):
            lay, off = plan.layouts[i], qp.offsets[i]
            c[lay.off_rhs:lay.off_rhs + cv.size] = cv
            beq[off["ry"]:off["ry"] + bv.size] = bv
            h[off["rz"]:off["rz"] + hv.size] = hv
        cd, bd, hd = (torch.from_numpy(v).to(dev) for v in (c, beq, h))
        ipm = kkt.IPM(plan, qp)
        ws = plan.new_workspace(dev)
        res = ipm.solve(ws, pools, cd, bd, hd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            res = ipm.solve(ws, pools, cd, bd, hd)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        st = res["status"].cpu().numpy()
        assert (st >= 0).all(), "interior-point solve did not converge: %s" % st[:8]
        its = float(np.mean(st))
        out[name] = {"shape": "%d x (N=%d b=%d ng=%d pe=%d me=%d)" % (count, N, b, ng, pe, me),
                     "ms_per_solve": round(ms, 3), "iterations_mean": round(its, 2),
                     "ms_per_iteration": round(ms / max(its, 1.0), 3),
                     "qps_per_s": round(count / (ms * 1e-3), 1), "levels": nest_levels(plan)}
    log("qp solves: %s" % out)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--systems", type=int, default=4096)
    ap.add_argument("--plain-sample", type=int, default=512)
    ap.add_argument("--cpu-sample", type=int, default=2048)
    ap.add_argument("--skip-oracle-all-cores", action="store_true",
                    help="time the oracle on one core only")
    ap.add_argument("--p", type=int, default=0,
                    help="segments per system (1 = sequential; 0 = chosen by the cost model measured on this GPU; "
                         "-1 = chosen by the default flop-ratio model)")
    ap.add_argument("--skip-diff", action="store_true")
    ap.add_argument("--skip-single", action="store_true", help="skip the single-system latency section")
    ap.add_argument("--single-only", action="store_true",
                    help="run only the single-system latencies and the QP iteration (no batch, no headline value)")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay measurement")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (got --gpus %d)" % args.gpus)
        sys.exit(2)

    import torch
    from paper_2511_00946_amd import kkt, workloads
    from oracle import kkt as okkt

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ev = HipEvents()

    if args.copy_calibration:
        n = COPY_BYTES // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES, "launches": 3}))
        return

    if args.single_only:
        from paper_2511_00946_amd import autotune
        cm = autotune.cost_model()
        single = single_systems(torch, kkt, workloads, okkt, dev, cm)
        print(json.dumps({"single_system": single, "qp_iteration": qp_iteration(torch, kkt, workloads, dev, cm),
                          "qp_solve": qp_solves(torch, kkt, workloads, dev, cm)}))
        return

    # ------------------------------------------------------------ ragged batch workload
    t0 = time.time()
    spec = workloads.ragged_batch_spec(S=args.systems)
    systems, pools = build_pools(spec)
    S = len(systems)
    log("generated %d systems in %.1fs (%.2f GB of inputs)" % (S, time.time() - t0,
        sum(v.nbytes for v in pools.values()) / 1e9))
    cost_model, calib_s = None, None
    if args.p == 0:
        from paper_2511_00946_amd import autotune
        t_cal = time.time()
        cost_model = autotune.cost_model()
        calib_s = round(time.time() - t_cal, 1)
        log("cost model (measured, %.1fs): %s" % (calib_s, cost_model))
    plan = kkt.Plan([(sy.N, sy.b, sy.ng, max(args.p, 0)) for sy in systems], nrhs=1, cost_model=cost_model)
    segs = plan.segments()
    uniform_p = segs[0] if len(set(segs)) == 1 else -1   # the counters apply to one p for all
    if args.p <= 0:
        log("segments chosen: %d systems split, max p %d" % (sum(1 for q in segs if q > 1), max(segs)))
    dp = kkt.pack_to_device(pools, dev)
    ws = plan.new_workspace(dev)
    info = torch.zeros(S, dtype=torch.int32, device=dev)
    x = torch.empty_like(dp["r"])
    classes = plan.classes()
    kinds = plan.class_kinds()
    log("plan: %d items, classes %s, workspace %.2f GB" % (plan.info.num_items, classes,
        plan.info.workspace_bytes / 1e9))
    step_flops = float(plan.info.factor_flops + plan.info.solve_flops)   # standard counts, one step

    def step():
        x.copy_(dp["r"])
        plan.factor_solve(dp["D"], dp["C"], dp["B"], dp["corner"], ws, x, info)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # per-step, per-class HIP events around each persistent launch
    K = args.steps
    cls_ev = [[(ev.create(), ev.create()) for _ in classes] for _ in range(K)]
    start, stop = ev.create(), ev.create()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    lib = ctypes.CDLL("libamdhip64.so")
    lib.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.hipEventRecord(ctypes.c_void_p(start), ctypes.c_void_p(st.cuda_stream))
    step_ev = [ev.create() for _ in range(K + 1)]
    for k in range(K):
        lib.hipEventRecord(ctypes.c_void_p(step_ev[k]), ctypes.c_void_p(st.cuda_stream))
        for c in range(len(classes)):
            plan.set_class_events(c, cls_ev[k][c][0], cls_ev[k][c][1])
        step()
    lib.hipEventRecord(ctypes.c_void_p(step_ev[K]), ctypes.c_void_p(st.cuda_stream))
    lib.hipEventRecord(ctypes.c_void_p(stop), ctypes.c_void_p(st.cuda_stream))
    torch.cuda.synchronize()
    step_ms = [ev.elapsed_ms(step_ev[k], step_ev[k + 1]) for k in range(K)]
    for c in range(len(classes)):
        plan.set_class_events(c, None, None)
    total_ms = ev.elapsed_ms(start, stop)
    ms_per_step = total_ms / K
    cls_ms = [np.mean([ev.elapsed_ms(*cls_ev[k][c]) for k in range(K)]) for c in range(len(classes))]
    log("timed %d steps: %.3f ms/step; per-class kernel ms %s" % (K, ms_per_step,
        ["%d:%.3f" % (classes[c][0], cls_ms[c]) for c in range(len(classes))]))

    # graph replay of the same step (capture is required to work: a failure or a
    # replay that differs from the eager result ends the run)
    graph_ms = None
    if not args.no_graph:
        g = torch.cuda.CUDAGraph()
        s2 = torch.cuda.Stream()
        s2.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s2):
            step()
        torch.cuda.current_stream().wait_stream(s2)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            step()
        torch.cuda.synchronize()
        x_eager = x.clone()
        for _ in range(2):
            g.replay()
        torch.cuda.synchronize()
        a, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(K):
            g.replay()
        b2.record()
        torch.cuda.synchronize()
        graph_ms = a.elapsed_time(b2) / K
        if not torch.equal(x, x_eager):
            raise RuntimeError("graph replay differs from the eager result")

    # residual gate on every system + parity with the oracle on a sample
    step()
    torch.cuda.synchronize()
    xh = x.cpu().numpy()
    infoh = info.cpu().numpy()
    assert (infoh == 0).all(), "factorization failed on %d systems" % int((infoh != 0).sum())
    worst = 0.0
    for s, sy in enumerate(systems):
        lay = plan.layouts[s]
        xs = xh[lay.off_rhs:lay.off_rhs + sy.n].reshape(sy.n, 1)
        worst = max(worst, okkt.rel_residual(sy.D, sy.C, sy.B, sy.corner, xs, sy.r))
    rng = np.random.default_rng(0)
    par = 0.0
    for s in rng.choice(S, size=8, replace=False):
        sy = systems[s]
        lay = plan.layouts[s]
        xs = xh[lay.off_rhs:lay.off_rhs + sy.n].reshape(sy.n, 1)
        xo = okkt.solve(sy.D, sy.C, sy.B, sy.corner, sy.r)
        par = max(par, float(np.max(np.abs(xs - xo)) / np.max(np.abs(xo))))
    log("max relative residual %.3e, sampled parity vs oracle %.3e" % (worst, par))
    assert worst <= 1e-10, "residual gate failed: %.3e" % worst

    # roofline of the dominant class kernel
    bytes_sys = alg_bytes(plan, systems)
    dom = int(np.argmax(cls_ms))
    dom_bp, dom_kind = classes[dom][0], kinds[dom]
    dom_dense = dom_kind == KIND_DENSE
    dom_db = 32
    dom_bytes = float(sum(bytes_sys[s] for s, sy in enumerate(systems)
                          if in_class(dom_bp, dom_kind, sy.b, plan.layouts[s].p)))
    achieved = dom_bytes / (cls_ms[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": measured_traffic(("d%d" if dom_dense else "%d") % dom_bp, uniform_p, S),
                "kernel": {KIND_DENSE: "kkt_dense<%d, factor_solve> + kkt_dense_bwd<%d>" % (dom_db, dom_db),
                           KIND_DSEG: "kkt_dense_seg<%d> + kkt_wave_p2<%d> + kkt_dense_seg_bwd<%d>"
                                      % (dom_db, dom_bp, dom_db)}.get(
                               dom_kind, "kkt_wave_p1/p2/p3<%d, factor_solve, 1>" % dom_bp),
                "kernel_ms": round(float(cls_ms[dom]), 4), "alg_bytes": dom_bytes}

    # plain single-system path: one call (one launch) per system, on a sample
    samp = np.random.default_rng(1).choice(S, size=min(args.plain_sample, S), replace=False)
    plain = []
    for s in samp:
        sy = systems[s]
        pl = kkt.Plan([(sy.N, sy.b, sy.ng, 1)], nrhs=1)
        pp = kkt.pack_to_device(workloads.pack([sy]), dev)
        w1 = pl.new_workspace(dev)
        i1 = torch.zeros(1, dtype=torch.int32, device=dev)
        x1 = torch.empty_like(pp["r"])
        plain.append((pl, pp, w1, i1, x1))
    def plain_pass():
        for pl, pp, w1, i1, x1 in plain:
            x1.copy_(pp["r"])
            pl.factor_solve(pp["D"], pp["C"], pp["B"], pp["corner"], w1, x1, i1)
    plain_sps = None
    if plain:
        plain_pass()
        torch.cuda.synchronize()
        a, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        plain_pass()
        b2.record()
        torch.cuda.synchronize()
        plain_ms = a.elapsed_time(b2)
        plain_sps = len(plain) / (plain_ms * 1e-3)
        log("plain path: %d systems in %.2f ms -> %.0f systems/s" % (len(samp), plain_ms, plain_sps))
    del plain

    # oracle on the host (bounded sample): its C core alone, and the whole Python call
    csamp = np.random.default_rng(2).choice(S, size=min(args.cpu_sample, S), replace=False)
    csys = [systems[s] for s in csamp]
    cpu_s = oracle_core_seconds(okkt, csys)
    cpu_sps = len(csamp) / cpu_s if len(csamp) else None
    t1 = time.perf_counter()
    for sy in csys[:256]:
        okkt.solve(sy.D, sy.C, sy.B, sy.corner, sy.r)
    wrapped_sps = min(256, len(csys)) / (time.perf_counter() - t1) if len(csys) else None
    log("oracle C core: %d systems in %.1fs -> %s systems/s (with the Python wrapper %s)"
        % (len(csamp), cpu_s, cpu_sps, wrapped_sps))
    cpu_all = None
    if len(csamp) and not args.skip_oracle_all_cores:
        sps_all, nw = oracle_all_cores(S, csamp)
        cpu_all = {"value": round(sps_all, 2), "unit": "systems/s", "cores": nw, "kind": "oracle",
                   "sample": "the same %d systems, one process per core over systems" % len(csamp)}
        log("oracle on %d cores: %.1f systems/s" % (nw, sps_all))

    del dp, ws, x, info
    torch.cuda.empty_cache()

    single = None if args.skip_single else single_systems(torch, kkt, workloads, okkt, dev, cost_model)
    qp_iter = None if args.skip_single else qp_iteration(torch, kkt, workloads, dev, cost_model)
    qp_solve = None if args.skip_single else qp_solves(torch, kkt, workloads, dev, cost_model)

    # differentiation workload: forward factor + solve, adjoint backward
    diff = None
    if not args.skip_diff:
        dspec = workloads.uniform_batch_spec()
        dsys, dpools = build_pools(dspec)
        dplan = kkt.Plan([(sy.N, sy.b, sy.ng, max(args.p, 0)) for sy in dsys], nrhs=1, cost_model=cost_model)
        dd = kkt.pack_to_device(dpools, dev)
        dws = dplan.new_workspace(dev)
        dinfo = torch.zeros(len(dsys), dtype=torch.int32, device=dev)
        dx = torch.empty_like(dd["r"])
        lam = torch.empty_like(dd["r"])
        gD, gC, gB, gR = (torch.empty_like(dd[k]) for k in ("D", "C", "B", "corner"))

        def dstep():
            dx.copy_(dd["r"])
            dplan.factor_solve(dd["D"], dd["C"], dd["B"], dd["corner"], dws, dx, dinfo)
            lam.copy_(dd["w"])
            dplan.solve_adjoint(dws, dx, lam, gD, gC, gB, gR)

        for _ in range(args.warmup):
            dstep()
        torch.cuda.synchronize()
        a, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(K):
            dstep()
        b2.record()
        torch.cuda.synchronize()
        dms = a.elapsed_time(b2) / K
        # gradient check against the oracle's closed form on a sample of systems
        lam_h, gD_h = lam.cpu().numpy(), gD.cpu().numpy()
        dxh = dx.cpu().numpy()
        gerr = 0.0
        for s in (0, 511, 1023):
            sy = dsys[s]
            lay = dplan.layouts[s]
            xs = dxh[lay.off_rhs:lay.off_rhs + sy.n].reshape(sy.n, 1)
            ref = okkt.adjoint(sy.D, sy.C, sy.B, sy.corner, xs, sy.w)
            got = gD_h[lay.off_D:lay.off_D + sy.N * sy.b * sy.b].reshape(sy.N, sy.b, sy.b)
            gerr = max(gerr, float(np.max(np.abs(got - ref[1])) / np.max(np.abs(ref[1]))))
            gl = lam_h[lay.off_rhs:lay.off_rhs + sy.n].reshape(sy.n, 1)
            gerr = max(gerr, float(np.max(np.abs(gl - ref[0])) / np.max(np.abs(ref[0]))))
        fd_err = fd_check(torch, kkt, workloads, dsys, dplan, dev,
                          {"D": gD.cpu().numpy(), "C": gC.cpu().numpy(), "B": gB.cpu().numpy(), "r": lam_h})
        dbytes = float(np.sum(alg_bytes(dplan, dsys, adjoint=True)))
        dach = dbytes / (dms * 1e-3) / 1e9
        diff = {"workload": "1024 x (N=64, b=24, ng=4)", "fwd_bwd_systems_per_s": round(len(dsys) / (dms * 1e-3), 1),
                "ms_per_step": round(dms, 4), "grad_max_rel_err_vs_oracle": gerr,
                "grad_max_rel_err_vs_central_fd_h1e-6": fd_err,
                "roofline": {"bound": "hbm", "achieved": round(dach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(dach / HBM_PEAK_GBS, 5), "traffic": None,
                             "kernel": "whole step (factor + solve, adjoint solve: every launch)",
                             "alg_bytes": dbytes}}
        assert fd_err <= 1e-6, "finite-difference gradient check failed: %.3e" % fd_err
        log("diff workload: %.3f ms per fwd+bwd -> %.0f systems/s, grad err %.2e" % (dms, len(dsys) / (dms * 1e-3), gerr))

    value = S / (ms_per_step * 1e-3)
    out = {
        "metric": "KKT factor+solve systems/sec FP64 (rel resid <=1e-10), batched vs plain; fwd+bwd/s",
        "value": round(value, 1),
        "unit": "systems/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "ms_per_step_std": round(float(np.std(step_ms)), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "ragged batch: %d systems, N~U{16..256}, b~U{8,16,32}, ng~U{0,2,4}, 1 rhs, seed 4"
                               % S, "segments": "p=%d" % args.p if args.p > 0 else
                                     ("%s cost model: %s" % ("measured" if args.p == 0 else "default",
                                      "p = %d for every system" % uniform_p if uniform_p > 0 else
                                      "%d of %d systems split" % (sum(1 for q in segs if q > 1), S)))},
        "plain_systems_per_s": None if plain_sps is None else round(plain_sps, 1),
        "plain_sample": int(len(samp)),
        "batched_vs_plain": None if plain_sps is None else round(value / plain_sps, 2),
        "graph_ms_per_step": None if graph_ms is None else round(graph_ms, 4),
        "max_rel_residual": worst,
        "sampled_parity_vs_oracle": par,
        "per_class_kernel_ms": {class_label(classes[c][0], kinds[c]): round(float(cls_ms[c]), 4)
                                for c in range(len(classes))},
        "differentiation": diff,
        "single_system": single,
        "qp_iteration": qp_iter,
        "qp_solve": qp_solve,
        "roofline": roofline,
        "cpu_baseline": {"value": None if cpu_sps is None else round(cpu_sps, 2), "unit": "systems/s", "cores": 1,
                         "kind": "oracle",
                         "sample": "%d random systems of the batch, factor + solve each, the oracle's C core "
                                   "timed with a steady clock (block assembly in Python left out)" % len(csamp)},
        "cpu_baseline_python_wrapped": None if wrapped_sps is None else round(wrapped_sps, 2),
        "cpu_baseline_all_cores": cpu_all,
        "fp64": {"achieved_tflops": round(step_flops / (ms_per_step * 1e-3) / 1e12, 4), "peak_tflops": 78.6,
                 "frac": round(step_flops / (ms_per_step * 1e-3) / 1e12 / 78.6, 5),
                 "flops_per_step": step_flops},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
