"""GPU parity: the HIP path (through the C ABI) against the oracle, element by element.

Tolerances (FP64): factor blocks within 1e-11 of the oracle's block scaled by the
block's largest entry (both are Cholesky factors of the same permuted matrix,
computed in different summation orders; the inputs are well conditioned);
solutions within 1e-10 relative and a relative residual <= 1e-10 (the gate of
the solver); gradients within 1e-9 relative of the oracle's closed form.
"""
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


def gen(seed, dims, nrhs=1, with_w=False):
    rng = np.random.default_rng(seed)
    return [workloads.draw_system(rng, N, b, ng, nrhs=nrhs, alpha=b, s_C=0.05, s_B=0.05, with_w=with_w)
            for (N, b, ng) in dims]


def run(systems, ps, nrhs, mode="fused"):
    kkt = _kkt()
    _say("gpu case: mode=%s dims=%s p=%s nrhs=%d" % (mode, [(s.N, s.b, s.ng) for s in systems][:6], ps[:6], nrhs))
    plan = kkt.Plan([(s.N, s.b, s.ng, p) for s, p in zip(systems, ps)], nrhs=nrhs)
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
    assert plan.workspace_error(ws) == 0, "a worker gave up waiting for a backward-sweep handover"
    return plan, pools, ws, x, info.cpu().numpy()


def split_rhs(plan, x, systems):
    xh = x.detach().cpu().numpy()
    out = []
    for s, sysm in enumerate(systems):
        lay = plan.layouts[s]
        n = sysm.n * plan.nrhs
        out.append(xh[lay.off_rhs:lay.off_rhs + n].reshape(sysm.n, plan.nrhs))
    return out


def check_factor(plan, ws, systems):
    wsh = ws.cpu().numpy()
    for s, sysm in enumerate(systems):
        seg = plan.segment_lengths(s)
        ref = okkt.KKTFactor(sysm.D, sysm.C, sysm.B, sysm.corner, seg)
        got = plan.factor_blocks(wsh, s)
        for (r, c), blk in got.items():
            rb = ref.block(r, c)
            if rb is None:
                assert np.all(blk == 0.0), (s, r, c)
                continue
            scale = max(1.0, float(np.max(np.abs(rb))))
            err = float(np.max(np.abs(blk - rb))) / scale
            assert err < 1e-11, ("factor block", s, seg, (r, c), err)


def check_solution(plan, x, systems):
    for s, (xs, sysm) in enumerate(zip(split_rhs(plan, x, systems), systems)):
        seg = plan.segment_lengths(s)
        xo = okkt.solve(sysm.D, sysm.C, sysm.B, sysm.corner, sysm.r, seg)
        rel = float(np.max(np.abs(xs - xo)) / max(1e-300, np.max(np.abs(xo))))
        res = okkt.rel_residual(sysm.D, sysm.C, sysm.B, sysm.corner, xs, sysm.r)
        assert rel < 1e-10 and res < 1e-10, ("solution", s, (sysm.N, sysm.b, sysm.ng), seg, rel, res)


SINGLE_CASES = [
    # (N, b, ng, p, nrhs)
    (16, 4, 2, 1, 1),
    (16, 4, 2, 2, 1),
    (16, 4, 2, 3, 1),
    (16, 4, 2, 8, 1),
    (1, 4, 2, 1, 1),
    (2, 1, 1, 1, 1),
    (3, 2, 0, 2, 1),
    (7, 3, 2, 3, 2),
    (9, 5, 0, 3, 1),
    (10, 8, 4, 1, 1),
    (10, 8, 4, 3, 1),
    (11, 12, 16, 2, 3),
    (9, 16, 0, 4, 1),
    (8, 20, 3, 2, 1),
    (8, 24, 4, 3, 1),
    (7, 32, 4, 1, 1),
    (9, 32, 2, 3, 1),
    # the 48-wide group (three-wave row-lane sweeps): whole and segmented, every mode
    (5, 42, 0, 2, 1),
    (7, 48, 1, 3, 1),
    (6, 33, 16, 1, 8),
    (11, 45, 5, 3, 3),
    (40, 6, 8, 4, 4),
    # the maxima: block size 32, 16 arrow rows, 8 rhs (whole and segmented, dense path)
    (6, 32, 16, 1, 8),
    (9, 32, 16, 3, 8),
    (7, 24, 16, 2, 5),
    (9, 8, 16, 3, 8),
]


@pytest.mark.parametrize("N,b,ng,p,nrhs", SINGLE_CASES)
def test_single_system_factor_solve(N, b, ng, p, nrhs):
    systems = gen(1000 + N * 31 + b * 7 + p, [(N, b, ng)], nrhs=nrhs)
    plan, pools, ws, x, info = run(systems, [p], nrhs)
    assert info.tolist() == [0]
    check_factor(plan, ws, systems)
    check_solution(plan, x, systems)


@pytest.mark.parametrize("p", [1, 4])
def test_factor_then_solve_matches(p):
    systems = gen(77, [(20, 6, 3)], nrhs=2)
    plan, pools, ws, x, info = run(systems, [p], 2, mode="separate")
    assert info.tolist() == [0]
    check_factor(plan, ws, systems)
    check_solution(plan, x, systems)


def test_factor_then_solve_every_group_segmented():
    """The solve-only mode of segmented systems of every block group (row-lane
    sweeps for all three phases), beside whole systems of the dense groups."""
    dims = [(17, 7, 2), (19, 14, 3), (16, 22, 1), (15, 30, 4), (9, 16, 2), (8, 32, 0), (13, 40, 3), (6, 47, 0)]
    systems = gen(78, dims, nrhs=3)
    ps = [3, 4, 2, 3, 1, 1, 3, 1]
    plan, pools, ws, x, info = run(systems, ps, 3, mode="separate")
    assert (info == 0).all()
    check_factor(plan, ws, systems)
    check_solution(plan, x, systems)


def test_small_workload_all_p():
    s = workloads.single("small")
    for p in (1, 2, 4, 8):
        plan, pools, ws, x, info = run([s], [p], 1)
        assert info.tolist() == [0]
        check_factor(plan, ws, [s])
        check_solution(plan, x, [s])


def test_ragged_batch_mixed_classes():
    rng = np.random.default_rng(5)
    dims, ps = [], []
    for i in range(40):
        N = int(rng.integers(1, 30))
        b = int(rng.choice([1, 3, 6, 8, 11, 16, 24, 32]))
        ng = int(rng.choice([0, 2, 4, 9]))
        pmax = (N + 1) // 2
        p = int(rng.integers(1, min(pmax, 5) + 1))
        dims.append((N, b, ng))
        ps.append(p)
    systems = gen(6, dims)
    plan, pools, ws, x, info = run(systems, ps, 1)
    # more launch classes than side streams: some run on the caller's stream
    assert len(plan.classes()) > 3
    assert (info == 0).all()
    check_factor(plan, ws, systems)
    check_solution(plan, x, systems)


def test_nonsymmetric_blocks_enter_through_their_symmetric_part():
    """D_i and the corner enter as sym(.) (the parametrisation of Eq. 3 used here):
    adding an antisymmetric part to every stored block changes nothing beyond rounding."""
    rng = np.random.default_rng(31)
    dims = [(9, 32, 4), (12, 16, 2), (7, 24, 3), (10, 8, 4), (13, 32, 0), (11, 16, 5), (6, 5, 2)]
    ps = [1, 1, 1, 1, 3, 2, 2]
    systems = gen(32, dims, nrhs=2)
    for sysm in systems:
        K = rng.standard_normal(sysm.D.shape)
        sysm.D[...] = sysm.D + 0.3 * (K - np.swapaxes(K, 1, 2))
        if sysm.ng:
            Kc = rng.standard_normal(sysm.corner.shape)
            sysm.corner[...] = sysm.corner + 0.3 * (Kc - Kc.T)
    assert max(float(np.max(np.abs(s.D - np.swapaxes(s.D, 1, 2)))) for s in systems) > 0.1
    plan, pools, ws, x, info = run(systems, ps, 2)
    assert (info == 0).all()
    check_factor(plan, ws, systems)
    check_solution(plan, x, systems)


def test_indefinite_block_reports_info_and_nan():
    dims = [(12, 6, 2), (12, 6, 2), (12, 6, 2), (12, 6, 2)]
    systems = gen(9, dims)
    systems[1].D[5] = -np.eye(6)          # segment stage
    systems[2].D[4] = -np.eye(6)          # with p = 3 (N1 = 4? see plan): whichever stage it is
    systems[3].corner[:] = -np.eye(2)     # corner
    ps = [1, 3, 3, 2]
    plan, pools, ws, x, info = run(systems, ps, 1)
    exp = []
    for s, p in zip(systems, ps):
        exp.append(okkt.KKTFactor(s.D, s.C, s.B, s.corner, plan.segment_lengths(len(exp))).info)
    assert info.tolist() == exp and exp[0] == 0 and exp[1] == 6 and exp[3] == 13
    xs = split_rhs(plan, x, systems)
    assert np.isfinite(xs[0]).all()
    for i in (1, 2, 3):
        assert np.isnan(xs[i]).all()
    check_solution(plan, x, systems[:1])


def test_indefinite_block_segmented_dense_classes():
    """Failures inside a segment, at a separator and at the corner of segmented
    16/24/32-wide systems (the dense segment sweeps and the sequential phase)."""
    dims = [(14, 12, 2), (14, 12, 2), (14, 20, 3), (14, 28, 2), (14, 12, 0)]
    systems = gen(19, dims)
    ps = [3, 3, 2, 3, 3]
    systems[1].D[2] = -np.eye(12)         # a stage of segment 1
    systems[2].D[9] = -np.eye(20)         # a stage of segment 2
    systems[3].corner[:] = -np.eye(2)     # corner
    plan, pools, ws, x, info = run(systems, ps, 1)
    exp = [okkt.KKTFactor(s.D, s.C, s.B, s.corner, plan.segment_lengths(i)).info for i, s in enumerate(systems)]
    assert info.tolist() == exp and exp[0] == 0 and exp[4] == 0 and all(e != 0 for e in exp[1:4])
    xs = split_rhs(plan, x, systems)
    for i in (1, 2, 3):
        assert np.isnan(xs[i]).all()
    check_solution(plan, x, [systems[0]])
    check_factor(plan, ws, [systems[0]])


def test_repeat_runs_bitwise_identical():
    systems = gen(11, [(30, 8, 4), (25, 16, 0), (17, 6, 2)])
    ps = [3, 2, 1]
    _, _, _, x1, _ = run(systems, ps, 1)
    _, _, _, x2, _ = run(systems, ps, 1)
    assert torch.equal(x1, x2)


ADJ_CASES = {
    # the last three are whole (p = 1) systems of the dense classes
    "mixed": ([(12, 6, 3), (9, 8, 0), (7, 16, 2), (6, 24, 4), (5, 32, 0)], 2, None),
    # the maxima: block size 32, 16 arrow rows, 8 rhs
    "maxima": ([(9, 8, 16), (6, 32, 16), (7, 16, 16)], 8, None),
    # segmented systems of every block group (their adjoint runs on the row-lane sweeps)
    "segmented": ([(12, 12, 3), (14, 20, 2), (13, 28, 4), (11, 5, 1), (15, 32, 16), (9, 44, 2), (7, 36, 4)], 3,
                  [3, 2, 3, 4, 2, 3, 1]),
}


@pytest.mark.parametrize("case", ["mixed", "maxima", "segmented"])
@pytest.mark.parametrize("p", [1, 3])
def test_adjoint_matches_oracle(p, case):
    kkt = _kkt()
    dims, nr, fixed = ADJ_CASES[case]
    if fixed is not None and p == 1:
        pytest.skip("the segmented case fixes its own segment counts")
    systems = gen(21, dims, nrhs=nr, with_w=True)
    ps = fixed if fixed is not None else [p, min(p, 2)] + [1] * (len(dims) - 2)
    plan, pools, ws, x, info = run(systems, ps, nr)
    assert (info == 0).all()
    gx = torch.from_numpy(workloads.pack(systems)["w"]).cuda()
    lam = gx.clone()
    dD = torch.zeros_like(pools["D"])
    dC = torch.zeros_like(pools["C"])
    dB = torch.zeros_like(pools["B"])
    dR = torch.zeros_like(pools["corner"])
    plan.solve_adjoint(ws, x, lam, dD, dC, dB, dR)
    torch.cuda.synchronize()
    lam_h, dD_h, dC_h, dB_h, dR_h = (t.cpu().numpy() for t in (lam, dD, dC, dB, dR))
    xs = split_rhs(plan, x, systems)
    for s, sysm in enumerate(systems):
        lay = plan.layouts[s]
        N, b, ng = sysm.N, sysm.b, sysm.ng
        ref = okkt.adjoint(sysm.D, sysm.C, sysm.B, sysm.corner, xs[s], sysm.w, plan.segment_lengths(s))
        got = (lam_h[lay.off_rhs:lay.off_rhs + sysm.n * nr].reshape(sysm.n, nr),
               dD_h[lay.off_D:lay.off_D + N * b * b].reshape(N, b, b),
               dC_h[lay.off_C:lay.off_C + (N - 1) * b * b].reshape(N - 1, b, b),
               dB_h[lay.off_B:lay.off_B + N * ng * b].reshape(N, ng, b),
               dR_h[lay.off_corner:lay.off_corner + ng * ng].reshape(ng, ng))
        for name, g, r in zip(("lambda", "dD", "dC", "dB", "dcorner"), got, ref):
            if r.size == 0:
                continue
            err = float(np.max(np.abs(g - r)) / max(1e-300, np.max(np.abs(r))))
            assert err < 1e-9, (name, s, err)


def test_foreign_workspace_is_refused_on_device():
    """A workspace re-initialised by another plan still passes the first plan's
    host-side registry; the reset kernel then finds the other plan's tag, every
    kernel of the call returns at once (no output written) and kkt_workspace_error
    reports it.  The first plan's own workspace is unaffected."""
    kkt = _kkt()
    systems = gen(31, [(20, 8, 2), (12, 16, 0)])
    plan_a = kkt.Plan([(20, 8, 2, 2), (12, 16, 0, 1)], nrhs=1)
    plan_b = kkt.Plan([(20, 8, 2, 2), (12, 16, 0, 1)], nrhs=1)
    pools = kkt.pack_to_device(workloads.pack(systems))
    ws = plan_a.new_workspace()
    plan_b.init_workspace(ws)
    info = torch.full((2,), -7, dtype=torch.int32, device="cuda")
    x = pools["r"].clone()
    _say("gpu case: foreign workspace")
    plan_a.factor_solve(pools["D"], pools["C"], pools["B"], pools["corner"], ws, x, info)
    torch.cuda.synchronize()
    assert plan_a.workspace_error(ws) == kkt.WS_FOREIGN
    assert torch.equal(x, pools["r"]) and info.tolist() == [-7, -7]
    plan_a.init_workspace(ws)
    plan_a.factor_solve(pools["D"], pools["C"], pools["B"], pools["corner"], ws, x, info)
    torch.cuda.synchronize()
    assert plan_a.workspace_error(ws) == 0 and info.tolist() == [0, 0]
    check_solution(plan_a, x, systems)


def test_workspaces_keep_their_own_factors():
    """One plan, two workspaces factored with different matrices: each later solve
    uses its own workspace's factor; a fresh workspace is refused."""
    kkt = _kkt()
    dims = [(20, 8, 2), (15, 16, 4)]
    sa, sb = gen(51, dims), gen(52, dims)
    plan = kkt.Plan([d + (2,) for d in dims], nrhs=1)
    _say("gpu case: two workspaces dims=%s p=2" % dims)
    pa, pb = kkt.pack_to_device(workloads.pack(sa)), kkt.pack_to_device(workloads.pack(sb))
    wa, wb = plan.new_workspace(), plan.new_workspace()
    info = torch.zeros(2, dtype=torch.int32, device="cuda")
    plan.factor(pa["D"], pa["C"], pa["B"], pa["corner"], wa, info)
    plan.factor(pb["D"], pb["C"], pb["B"], pb["corner"], wb, info)
    xa, xb = pa["r"].clone(), pb["r"].clone()
    plan.solve(wa, xa)
    plan.solve(wb, xb)
    torch.cuda.synchronize()
    check_solution(plan, xa, sa)
    check_solution(plan, xb, sb)
    with pytest.raises(kkt.KKTError):
        plan.solve(plan.new_workspace(), pa["r"].clone())
    plan.init_workspace(wa)
    with pytest.raises(kkt.KKTError):
        plan.solve(wa, pa["r"].clone())


def test_row_lane_family_for_the_dense_classes():
    """The cost model's family 2 runs the 24- and 32-wide classes on the row-lane
    sweeps (whole and segmented systems, factor then solve): same results."""
    kkt = _kkt()
    dims = [(14, 20, 3), (11, 28, 2), (9, 32, 16), (16, 24, 0)]
    ps = [1, 1, 3, 2]
    systems = gen(83, dims, nrhs=2)
    m = {"family": [0.0, 0.0, 2.0, 2.0, 0.0]}
    _say("gpu case: row-lane family for the 24/32 classes dims=%s" % dims)
    plan = kkt.Plan([(s.N, s.b, s.ng, p) for s, p in zip(systems, ps)], nrhs=2, cost_model=m)
    assert set(plan.class_kinds()) == {0}
    pools = kkt.pack_to_device(workloads.pack(systems))
    ws = plan.new_workspace()
    info = torch.zeros(len(systems), dtype=torch.int32, device="cuda")
    x = pools["r"].clone()
    plan.factor(pools["D"], pools["C"], pools["B"], pools["corner"], ws, info)
    plan.solve(ws, x)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    check_factor(plan, ws, systems)
    check_solution(plan, x, systems)
