"""GPU: calls captured in a HIP graph (torch.cuda.graph), the first call on a
fresh plan and workspace included, replayed several times with eager work and
synchronisations between the replays; every replay is compared with the eager
result (bitwise) and with the oracle.

Tolerances as in the parity tests: solutions within 1e-10 relative of the
oracle with a relative residual <= 1e-10; adjoint within 1e-9 relative."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kkt as okkt
from paper_2511_00946_amd import workloads

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _gen(seed, dims, nrhs=1, with_w=False):
    rng = np.random.default_rng(seed)
    return [workloads.draw_system(rng, N, b, ng, nrhs=nrhs, alpha=b, s_C=0.05, s_B=0.05, with_w=with_w)
            for (N, b, ng) in dims]


def _split(plan, xh, systems):
    out = []
    for s, sy in enumerate(systems):
        lay = plan.layouts[s]
        out.append(xh[lay.off_rhs:lay.off_rhs + sy.n * plan.nrhs].reshape(sy.n, plan.nrhs))
    return out


# more launch classes than side streams (8, dense 16, segmented 16, dense 32, segmented 32)
DIMS = [(20, 6, 3), (31, 8, 2), (12, 16, 2), (18, 13, 4), (9, 32, 0), (16, 28, 3), (11, 24, 1)]
PS = [3, 1, 1, 3, 1, 2, 1]


def test_first_call_captured_factor_solve_and_adjoint():
    from paper_2511_00946_amd import kkt
    nr = 2
    systems = _gen(91, DIMS, nrhs=nr, with_w=True)
    plan = kkt.Plan([(s.N, s.b, s.ng, p) for s, p in zip(systems, PS)], nrhs=nr)
    assert plan.info.num_classes > 3
    pools = kkt.pack_to_device(workloads.pack(systems))
    ws = plan.new_workspace()            # kkt_workspace_init: the plan's launch state is made here
    info = torch.zeros(len(systems), dtype=torch.int32, device="cuda")
    x = torch.empty_like(pools["r"])
    lam = torch.empty_like(pools["r"])
    grads = {k: torch.empty_like(pools[k]) for k in ("D", "C", "B", "corner")}
    _say("gpu case: graph capture of the first factor_solve + solve_adjoint, %d classes" % plan.info.num_classes)
    g = torch.cuda.CUDAGraph()
    s2 = torch.cuda.Stream()
    s2.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s2):
        x.copy_(pools["r"])
        plan.factor_solve(pools["D"], pools["C"], pools["B"], pools["corner"], ws, x, info)
        lam.copy_(pools["w"])
        plan.solve_adjoint(ws, x, lam, grads["D"], grads["C"], grads["B"], grads["corner"])
    torch.cuda.synchronize()
    outs = []
    for rep in range(3):
        x.zero_()
        lam.zero_()
        g.replay()
        torch.cuda.synchronize()
        outs.append((x.clone(), lam.clone(), {k: v.clone() for k, v in grads.items()}, info.clone()))
        # eager work between replays
        _ = (pools["D"] * 2.0).sum().item()
    # eager reference through the same plan and workspace
    xe, lame = pools["r"].clone(), pools["w"].clone()
    ge = {k: torch.empty_like(pools[k]) for k in ("D", "C", "B", "corner")}
    plan.factor_solve(pools["D"], pools["C"], pools["B"], pools["corner"], ws, xe, info)
    plan.solve_adjoint(ws, xe, lame, ge["D"], ge["C"], ge["B"], ge["corner"])
    torch.cuda.synchronize()
    for xr, lr, gr, ir in outs:
        assert (ir.cpu() == 0).all()
        assert torch.equal(xr, xe) and torch.equal(lr, lame)
        for k in ge:
            assert torch.equal(gr[k], ge[k]), k
    xs = _split(plan, xe.cpu().numpy(), systems)
    ls = _split(plan, lame.cpu().numpy(), systems)
    for s, sy in enumerate(systems):
        xo = okkt.solve(sy.D, sy.C, sy.B, sy.corner, sy.r, plan.segment_lengths(s))
        rel = float(np.max(np.abs(xs[s] - xo)) / np.max(np.abs(xo)))
        res = okkt.rel_residual(sy.D, sy.C, sy.B, sy.corner, xs[s], sy.r)
        assert rel < 1e-10 and res < 1e-10, (s, rel, res)
        lo = okkt.adjoint(sy.D, sy.C, sy.B, sy.corner, xs[s], sy.w, plan.segment_lengths(s))[0]
        err = float(np.max(np.abs(ls[s] - lo)) / np.max(np.abs(lo)))
        assert err < 1e-9, (s, err)


def test_captured_solve_with_new_rhs_each_replay():
    """Factor eagerly, capture one kkt_solve, and replay it on three different
    right-hand sides copied into the captured buffer between replays."""
    from paper_2511_00946_amd import kkt
    systems = _gen(92, DIMS, nrhs=1)
    plan = kkt.Plan([(s.N, s.b, s.ng, p) for s, p in zip(systems, PS)], nrhs=1)
    pools = kkt.pack_to_device(workloads.pack(systems))
    ws = plan.new_workspace()
    info = torch.zeros(len(systems), dtype=torch.int32, device="cuda")
    plan.factor(pools["D"], pools["C"], pools["B"], pools["corner"], ws, info)
    torch.cuda.synchronize()
    x = torch.empty_like(pools["r"])
    _say("gpu case: captured solve, three right-hand sides")
    g = torch.cuda.CUDAGraph()
    s2 = torch.cuda.Stream()
    s2.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=s2):
        plan.solve(ws, x)
    rng = np.random.default_rng(5)
    for rep in range(3):
        rh = rng.standard_normal(pools["r"].numel())
        x.copy_(torch.from_numpy(rh))
        g.replay()
        torch.cuda.synchronize()
        xs = _split(plan, x.cpu().numpy(), systems)
        off = 0
        for s, sy in enumerate(systems):
            r = rh[off:off + sy.n].reshape(sy.n, 1)
            off += sy.n
            res = okkt.rel_residual(sy.D, sy.C, sy.B, sy.corner, xs[s], r)
            assert res < 1e-10, (rep, s, res)
