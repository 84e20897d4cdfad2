"""GPU parity of recursive (multi-level) segmentation: the reduced separator chain
of a system segmented in turn (and its own chain again), through the C ABI,
against the oracle's factor of the nested elimination order.

Tolerances as in the parity tests: factor blocks within 1e-11 of the oracle's
block scaled by its largest entry, solutions within 1e-10 relative with a
relative residual <= 1e-10, adjoint within 1e-9 relative."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kkt as okkt
from paper_2511_00946_amd import workloads

pytestmark = pytest.mark.gpu


def _kkt():
    from paper_2511_00946_amd import kkt
    return kkt


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _gen(seed, dims, nrhs=1, with_w=False):
    rng = np.random.default_rng(seed)
    return [workloads.draw_system(rng, N, b, ng, nrhs=nrhs, alpha=b, s_C=0.05, s_B=0.05, with_w=with_w)
            for (N, b, ng) in dims]


def levels(plan, s):
    """Segment lengths of every level of system s: the system's, then its chain's, ..."""
    out = [plan.segment_lengths(s)]
    r = plan.reduced(s)
    while r is not None:
        ch, cs, _ = r
        out.append(ch.segment_lengths(cs))
        r = ch.reduced(cs)
    return out


def _split(plan, x, systems):
    xh = x.detach().cpu().numpy()
    out = []
    for s, sy in enumerate(systems):
        lay = plan.layouts[s]
        out.append(xh[lay.off_rhs:lay.off_rhs + sy.n * plan.nrhs].reshape(sy.n, plan.nrhs))
    return out


def _run(systems, ps, nest, nrhs, mode="fused"):
    kkt = _kkt()
    _say("gpu case: nested mode=%s dims=%s p=%s nest=%s nrhs=%d"
         % (mode, [(s.N, s.b, s.ng) for s in systems][:6], ps[:6], nest[:6], nrhs))
    plan = kkt.Plan([(s.N, s.b, s.ng, p) for s, p in zip(systems, ps)], nrhs=nrhs, nest=nest)
    pools = kkt.pack_to_device(workloads.pack(systems))
    ws = plan.new_workspace()
    info = torch.full((len(systems),), -7, dtype=torch.int32, device="cuda")
    x = pools["r"].clone()
    if mode == "fused":
        plan.factor_solve(pools["D"], pools["C"], pools["B"], pools["corner"], ws, x, info)
    else:
        plan.factor(pools["D"], pools["C"], pools["B"], pools["corner"], ws, info)
        plan.solve(ws, x)
    torch.cuda.synchronize()
    assert plan.workspace_error(ws) == 0
    return plan, pools, ws, x, info.cpu().numpy()


def _check_solution(plan, x, systems, idx=None):
    for s, (xs, sy) in enumerate(zip(_split(plan, x, systems), systems)):
        if idx is not None and s not in idx:
            continue
        lv = levels(plan, s)
        xo = okkt.solve(sy.D, sy.C, sy.B, sy.corner, sy.r, lv[0], nest=lv[1:])
        rel = float(np.max(np.abs(xs - xo)) / max(1e-300, np.max(np.abs(xo))))
        res = okkt.rel_residual(sy.D, sy.C, sy.B, sy.corner, xs, sy.r)
        assert rel < 1e-10 and res < 1e-10, ("solution", s, (sy.N, sy.b, sy.ng), lv, rel, res)


def _check_factor(plan, ws, systems, idx=None):
    """Every block the library stores equals the oracle's block of the nested
    order, and every nonzero block of the oracle's factor is stored."""
    wsh = ws.cpu().numpy()
    for s, sy in enumerate(systems):
        if idx is not None and s not in idx:
            continue
        lv = levels(plan, s)
        ref = okkt.KKTFactor(sy.D, sy.C, sy.B, sy.corner, lv[0], nest=lv[1:])
        got = plan.factor_blocks(wsh, s)
        for (r, c), blk in got.items():
            rb = ref.block(r, c)
            if rb is None:
                assert np.all(blk == 0.0), (s, r, c)
                continue
            scale = max(1.0, float(np.max(np.abs(rb))))
            err = float(np.max(np.abs(blk - rb))) / scale
            assert err < 1e-11, ("factor block", s, lv, (r, c), err)
        order = ref.order + (["g"] if sy.ng else [])
        for i, ri in enumerate(order):
            for cj in order[: i + 1]:
                rb = ref.block(ri, cj)
                if rb is not None and np.max(np.abs(rb)) > 0.0:
                    assert (ri, cj) in got, ("block not stored", s, (ri, cj))


CASES = [
    # (N, b, ng, p, nest, nrhs)
    (64, 8, 3, 8, [3], 1),           # 8-wide single-wave sweeps, one extra level
    (130, 5, 2, 16, [4, 2], 2),      # two extra levels
    (61, 16, 4, 10, [4], 1),         # 16-wide single-wave sweeps
    (90, 24, 4, 9, [3], 1),          # dense segment sweeps (32-wide tiles) at both levels
    (45, 32, 16, 7, [3], 8),         # the maxima: 32 wide, 16 arrow rows, 8 rhs
    (40, 42, 0, 6, [2], 1),          # 48-wide three-wave sweeps
    (300, 6, 8, 40, [8, 3], 4),      # the race shape, two extra levels
]


@pytest.mark.parametrize("N,b,ng,p,nest,nrhs", CASES)
def test_nested_factor_solve(N, b, ng, p, nest, nrhs):
    systems = _gen(4000 + N + 7 * b + p, [(N, b, ng)], nrhs=nrhs)
    plan, pools, ws, x, info = _run(systems, [p], [nest], nrhs)
    assert plan.nest_depth(0) == len(nest)
    assert info.tolist() == [0]
    _check_factor(plan, ws, systems)
    _check_solution(plan, x, systems)


def test_nested_factor_then_solve_mixed_batch():
    """Nested systems of several classes beside sequential-chain segmented and
    whole systems in one plan; factor, then solve."""
    dims = [(64, 8, 3), (50, 6, 2), (20, 8, 0), (61, 16, 4), (30, 12, 2), (90, 24, 4), (12, 32, 1), (40, 42, 0)]
    ps = [8, 5, 1, 10, 3, 9, 1, 6]
    nest = [[3], None, None, [4], None, [3], None, [2]]
    systems = _gen(4101, dims, nrhs=3)
    plan, pools, ws, x, info = _run(systems, ps, nest, 3, mode="separate")
    assert (info == 0).all()
    assert [plan.nest_depth(s) for s in range(len(dims))] == [1, 0, 0, 1, 0, 1, 0, 1]
    _check_factor(plan, ws, systems)
    _check_solution(plan, x, systems)


@pytest.mark.parametrize("nr", [1, 3])
def test_nested_adjoint_matches_oracle(nr):
    kkt = _kkt()
    dims = [(64, 8, 3), (61, 16, 4), (90, 24, 4), (30, 12, 2), (130, 5, 2)]
    ps = [8, 10, 9, 3, 16]
    nest = [[3], [4], [3], None, [4, 2]]
    systems = _gen(4200 + nr, dims, nrhs=nr, with_w=True)
    plan, pools, ws, x, info = _run(systems, ps, nest, nr)
    assert (info == 0).all()
    gx = torch.from_numpy(workloads.pack(systems)["w"]).cuda()
    lam = gx.clone()
    dD, dC = torch.zeros_like(pools["D"]), torch.zeros_like(pools["C"])
    dB, dR = torch.zeros_like(pools["B"]), torch.zeros_like(pools["corner"])
    _say("gpu case: nested adjoint nr=%d" % nr)
    plan.solve_adjoint(ws, x, lam, dD, dC, dB, dR)
    torch.cuda.synchronize()
    lam_h, dD_h, dC_h, dB_h, dR_h = (t.cpu().numpy() for t in (lam, dD, dC, dB, dR))
    xs = _split(plan, x, systems)
    for s, sy in enumerate(systems):
        lay = plan.layouts[s]
        N, b, ng = sy.N, sy.b, sy.ng
        ref = okkt.adjoint(sy.D, sy.C, sy.B, sy.corner, xs[s], sy.w, plan.segment_lengths(s))
        got = (lam_h[lay.off_rhs:lay.off_rhs + sy.n * nr].reshape(sy.n, nr),
               dD_h[lay.off_D:lay.off_D + N * b * b].reshape(N, b, b),
               dC_h[lay.off_C:lay.off_C + (N - 1) * b * b].reshape(N - 1, b, b),
               dB_h[lay.off_B:lay.off_B + N * ng * b].reshape(N, ng, b),
               dR_h[lay.off_corner:lay.off_corner + ng * ng].reshape(ng, ng))
        for name, g, r in zip(("lambda", "dD", "dC", "dB", "dcorner"), got, ref):
            if r.size == 0:
                continue
            err = float(np.max(np.abs(g - r)) / max(1e-300, np.max(np.abs(r))))
            assert err < 1e-9, (name, s, err)


def test_nested_failures_report_the_first_block_of_the_nested_order():
    """Indefinite blocks in a level-0 segment, at separators (a level-1 segment
    stage and a level-1 separator) and at the corner: info follows the nested
    elimination order and the failed systems' solutions are NaN."""
    dims = [(64, 8, 3)] * 5
    systems = _gen(4301, dims)
    ps, nest = [8] * 5, [[3]] * 5
    kkt = _kkt()
    probe = kkt.Plan([(s.N, s.b, s.ng, p) for s, p in zip(systems, ps)], nest=nest)
    lv = levels(probe, 0)
    _, seps = okkt.stage_layout(64, lv[0])
    segs1, seps1 = okkt.stage_layout(len(seps), lv[1])
    sep_in_seg = seps[segs1[-1][-1]]   # a level-1 segment stage (late in natural order)
    sep_last = seps[seps1[0]]          # a level-1 separator (early in natural order)
    assert sep_last < sep_in_seg
    systems[1].D[2] = -np.eye(8)                      # a level-0 segment stage
    systems[2].D[sep_in_seg] = -np.eye(8)
    systems[2].D[sep_last] = -np.eye(8)
    systems[3].D[sep_last] = -np.eye(8)
    systems[4].corner[:] = -np.eye(3)
    plan, pools, ws, x, info = _run(systems, ps, nest, 1)
    exp = []
    for i, s in enumerate(systems):
        l = levels(plan, i)
        exp.append(okkt.KKTFactor(s.D, s.C, s.B, s.corner, l[0], nest=l[1:]).info)
    assert exp == [0, 3, sep_in_seg + 1, sep_last + 1, 65]
    assert info.tolist() == exp
    xs = _split(plan, x, systems)
    assert np.isfinite(xs[0]).all()
    for i in (1, 2, 3, 4):
        assert np.isnan(xs[i]).all(), i
    _check_solution(plan, x, systems, idx={0})


def test_cost_model_nests_and_solves():
    """A plan whose cost model prices recursion cheaply nests the long chain
    itself; its solution matches the oracle of the order it chose."""
    kkt = _kkt()
    b3 = [float(bp) ** 3 for bp in (8, 16, 24, 32, 48)]
    m = {"t_first": [7 / 3 * x for x in b3], "t_fill": [19 / 3 * x for x in b3],
         "t_red": [10 / 3 * x for x in b3], "t_item": [0.0] * 5, "workers": [1e12] * 5,
         "t_level": [40 * 7 / 3 * 512.0] * 5}
    systems = _gen(4401, [(1024, 6, 4)], nrhs=2)
    plan = kkt.Plan([(1024, 6, 4, 0)], nrhs=2, cost_model=m)
    assert plan.nest_depth(0) >= 1
    _say("gpu case: cost-model nested plan levels=%s" % [len(v) for v in levels(plan, 0)])
    pools = kkt.pack_to_device(workloads.pack(systems))
    ws = plan.new_workspace()
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    x = pools["r"].clone()
    plan.factor_solve(pools["D"], pools["C"], pools["B"], pools["corner"], ws, x, info)
    torch.cuda.synchronize()
    assert info.tolist() == [0]
    _check_solution(plan, x, systems)


def test_nested_call_captured_in_a_graph():
    """factor_solve of a nested plan captured in a HIP graph (first call
    included), replayed with eager work in between: every replay equals the eager
    call bitwise."""
    kkt = _kkt()
    dims = [(130, 5, 2), (61, 16, 4), (20, 8, 0)]
    systems = _gen(4501, dims, nrhs=2)
    plan = kkt.Plan([(130, 5, 2, 16), (61, 16, 4, 10), (20, 8, 0, 1)], nrhs=2, nest=[[4, 2], [4], None])
    pools = kkt.pack_to_device(workloads.pack(systems))
    ws = plan.new_workspace()
    info = torch.zeros(3, dtype=torch.int32, device="cuda")
    x = torch.empty_like(pools["r"])
    _say("gpu case: nested graph capture")
    g = torch.cuda.CUDAGraph()
    s2 = torch.cuda.Stream()
    s2.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s2):
        x.copy_(pools["r"])
        plan.factor_solve(pools["D"], pools["C"], pools["B"], pools["corner"], ws, x, info)
    torch.cuda.synchronize()
    outs = []
    for _ in range(3):
        x.zero_()
        g.replay()
        torch.cuda.synchronize()
        outs.append(x.clone())
        _ = (pools["D"] * 2.0).sum().item()
    xe = pools["r"].clone()
    plan.factor_solve(pools["D"], pools["C"], pools["B"], pools["corner"], ws, xe, info)
    torch.cuda.synchronize()
    assert info.tolist() == [0, 0, 0]
    for o in outs:
        assert torch.equal(o, xe)
    _check_solution(plan, xe, systems)
