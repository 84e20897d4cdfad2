"""GPU: the no-allocation entry point (kkt_factor_solve_noalloc, its workspace a
file-scope device array inside the library) against kkt_factor_solve with a
caller workspace, through the C ABI, on two calls in a row (the second with a
smaller plan, so the array switches plans), and the size limit.

Both entry points run the same kernels in the same launch order on a single
stream (the no-allocation one runs every class on the caller's stream, which
changes no arithmetic), so the results are compared bitwise, and against the
oracle at the parity tests' bar (relative 1e-10, residual 1e-10)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kkt as okkt
from paper_2511_00946_amd import workloads

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2511_00946_amd import kkt
    return kkt, kkt.lib()


def _gen(seed, dims, nrhs):
    rng = np.random.default_rng(seed)
    return [workloads.draw_system(rng, N, b, ng, nrhs=nrhs, alpha=b, s_C=0.05, s_B=0.05) for (N, b, ng) in dims]


def _run_pair(kkt, L, systems, ps, nrhs, nest=None):
    plan = kkt.Plan([(s.N, s.b, s.ng, p) for s, p in zip(systems, ps)], nrhs=nrhs, nest=nest)
    pools = kkt.pack_to_device(workloads.pack(systems))
    info1 = torch.full((len(systems),), -7, dtype=torch.int32, device="cuda")
    info2 = torch.full((len(systems),), -7, dtype=torch.int32, device="cuda")
    x1 = pools["r"].clone()
    rc = L.kkt_factor_solve_noalloc(plan._h, kkt._ptr(pools["D"]), kkt._ptr(pools["C"]), kkt._ptr(pools["B"]),
                                    kkt._ptr(pools["corner"]), kkt._ptr(x1), kkt._ptr(info1), kkt._stream(None))
    assert rc == 0, rc
    ws = plan.new_workspace()
    x2 = pools["r"].clone()
    plan.factor_solve(pools["D"], pools["C"], pools["B"], pools["corner"], ws, x2, info2)
    torch.cuda.synchronize()
    assert info1.tolist() == [0] * len(systems) and info2.tolist() == [0] * len(systems)
    assert torch.equal(x1, x2)
    xh = x1.cpu().numpy()
    for s, sy in enumerate(systems):
        lay = plan.layouts[s]
        xs = xh[lay.off_rhs:lay.off_rhs + sy.n * nrhs].reshape(sy.n, nrhs)
        xo = okkt.solve(sy.D, sy.C, sy.B, sy.corner, sy.r, plan.segment_lengths(s))
        assert float(np.max(np.abs(xs - xo)) / np.max(np.abs(xo))) < 1e-10
        assert okkt.rel_residual(sy.D, sy.C, sy.B, sy.corner, xs, sy.r) < 1e-10
    return plan


def test_noalloc_matches_workspace_entry_point_twice():
    kkt, L = _lib()
    print("gpu case: no-allocation entry point, two plans", file=sys.stderr, flush=True)
    big = _gen(61, [(40, 6, 8), (30, 16, 4), (25, 32, 2), (20, 42, 0), (16, 4, 2)], 2)
    _run_pair(kkt, L, big, [4, 1, 2, 3, 1], 2)
    small = _gen(62, [(12, 8, 2), (9, 24, 3)], 2)
    _run_pair(kkt, L, small, [2, 1], 2)
    # the first plan again: its tables are copied back in
    _run_pair(kkt, L, big, [4, 1, 2, 3, 1], 2)


def test_noalloc_runs_a_nested_plan():
    """Recursive segmentation through the no-allocation entry point: the child plans'
    tables and workspaces live in the same device array."""
    kkt, L = _lib()
    print("gpu case: no-allocation entry point, nested plan", file=sys.stderr, flush=True)
    systems = _gen(63, [(130, 5, 2), (61, 16, 4), (20, 8, 0)], 2)
    plan = _run_pair(kkt, L, systems, [16, 10, 1], 2, nest=[[4, 2], [4], None])
    assert plan.nest_depth(0) == 2 and plan.nest_depth(1) == 1
    # and a plain plan after it
    _run_pair(kkt, L, _gen(64, [(12, 8, 2), (9, 24, 3)], 2), [2, 1], 2)


def test_noalloc_refuses_a_plan_larger_than_its_array():
    kkt, L = _lib()
    plan = kkt.Plan([(256, 32, 4, 1)] * 200, nrhs=1)
    assert plan.info.workspace_bytes > kkt.NOALLOC_MAX_BYTES
    buf = torch.zeros(8, dtype=torch.float64, device="cuda")
    info = torch.zeros(200, dtype=torch.int32, device="cuda")
    rc = L.kkt_factor_solve_noalloc(plan._h, kkt._ptr(buf), kkt._ptr(buf), kkt._ptr(buf), kkt._ptr(buf),
                                    kkt._ptr(buf), kkt._ptr(info), kkt._stream(None))
    assert rc == -3
