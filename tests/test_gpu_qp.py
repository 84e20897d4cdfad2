"""GPU parity of the multistage-QP KKT path (assembly of Psi, reduced rhs, recovery
of dy and dz) against the oracle, and of one interior-point linear-algebra step
(assemble, factor once, solve two right-hand sides) against LAPACK on the
unreduced saddle-point matrix.

Tolerances (FP64): assembled blocks within 1e-12 of the oracle's scaled by the
pool's largest entry (sums of products in another order); the reduced rhs within
1e-12 relative; the Newton step (dx, dy, dz) within 1e-9 relative of the dense
saddle-point solve."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kkt as okkt
from oracle import qp as oqp
from paper_2511_00946_amd import workloads

pytestmark = pytest.mark.gpu


def _kkt():
    from paper_2511_00946_amd import kkt
    return kkt


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


SHAPES = [
    # (N, b, ng, pe, me)
    (6, 4, 2, 3, 5),
    (9, 8, 4, 8, 8),
    (5, 13, 3, 6, 10),
    (4, 24, 0, 12, 20),
    (3, 32, 16, 32, 32),
    (7, 1, 1, 1, 0),
    (5, 6, 8, 0, 4),
]


def _setup(seed, shapes, nrhs, ps=None):
    kkt = _kkt()
    rng = np.random.default_rng(seed)
    qps = [workloads.draw_qp(rng, *sh) for sh in shapes]
    ps = ps or [1] * len(shapes)
    plan = kkt.Plan([(q.N, q.b, q.ng, p) for q, p in zip(qps, ps)], nrhs=nrhs)
    qp = kkt.QP(plan, [q.pe for q in qps], [q.me for q in qps])
    pools = {k: torch.from_numpy(v).cuda() for k, v in workloads.pack_qp(qps).items()}
    return kkt, plan, qp, qps, pools


def _vec(rng, plan, qp, qps, nrhs):
    """rx in the plan's rhs layout, ry and rz in the QP layouts, and per system views."""
    rx = np.zeros(plan.info.rhs_len)
    ry = np.zeros(qp.lengths["ry"])
    rz = np.zeros(qp.lengths["rz"])
    per = []
    for s, q in enumerate(qps):
        lay, off = plan.layouts[s], qp.offsets[s]
        n = q.N * q.b + q.ng
        a = rng.standard_normal((n, nrhs))
        y = rng.standard_normal((q.N * q.pe, nrhs))
        z = rng.standard_normal((q.N * q.me, nrhs))
        rx[lay.off_rhs:lay.off_rhs + n * nrhs] = a.reshape(-1)
        ry[off["ry"]:off["ry"] + y.size] = y.reshape(-1)
        rz[off["rz"]:off["rz"] + z.size] = z.reshape(-1)
        per.append((a, y, z))
    return rx, ry, rz, per


def test_qp_assembly_matches_oracle():
    kkt, plan, qp, qps, pools = _setup(11, SHAPES, 1)
    lens = plan.pool_lengths()
    D, C = torch.zeros(lens["D"], dtype=torch.float64, device="cuda"), torch.zeros(lens["C"], dtype=torch.float64, device="cuda")
    B, R = torch.zeros(lens["B"], dtype=torch.float64, device="cuda"), torch.zeros(lens["corner"], dtype=torch.float64, device="cuda")
    rho, delta = 1e-3, 0.05
    _say("gpu case: qp assembly shapes=%s" % SHAPES)
    qp.assemble(pools, rho, delta, D, C, B, R)
    torch.cuda.synchronize()
    Dh, Ch, Bh, Rh = (t.cpu().numpy() for t in (D, C, B, R))
    for s, q in enumerate(qps):
        lay = plan.layouts[s]
        N, b, ng = q.N, q.b, q.ng
        rD, rC, rB, rR, _ = oqp.assemble(q.arrays, rho, delta)
        got = (Dh[lay.off_D:lay.off_D + N * b * b].reshape(N, b, b), Ch[lay.off_C:lay.off_C + (N - 1) * b * b].reshape(N - 1, b, b),
               Bh[lay.off_B:lay.off_B + N * ng * b].reshape(N, ng, b), Rh[lay.off_corner:lay.off_corner + ng * ng].reshape(ng, ng))
        for name, g, r in zip(("D", "C", "B", "corner"), got, (rD, rC, rB, rR)):
            if r.size == 0:
                continue
            err = float(np.max(np.abs(g - r))) / max(1.0, float(np.max(np.abs(r))))
            assert err < 1e-12, (name, s, err)


@pytest.mark.parametrize("nrhs", [1, 3])
def test_qp_newton_step_factor_once_solve_twice(nrhs):
    """One interior-point linear-algebra step: assemble Psi, factor it once, then for
    two right-hand-side sets (predictor, corrector) reduce, solve and recover; each
    step equals LAPACK on the unreduced saddle-point matrix."""
    kkt, plan, qp, qps, pools = _setup(12 + nrhs, SHAPES[:5] + [(40, 6, 8, 6, 12)], nrhs, ps=[1, 2, 1, 2, 1, 4])
    lens = plan.pool_lengths()
    zeros = lambda n: torch.zeros(n, dtype=torch.float64, device="cuda")
    D, C, B, R = zeros(lens["D"]), zeros(lens["C"]), zeros(lens["B"]), zeros(lens["corner"])
    rho, delta = 1e-4, 1e-2
    ws = plan.new_workspace()
    info = torch.zeros(plan.S, dtype=torch.int32, device="cuda")
    _say("gpu case: qp newton step nrhs=%d" % nrhs)
    qp.assemble(pools, rho, delta, D, C, B, R)
    plan.factor(D, C, B, R, ws, info)
    rng = np.random.default_rng(7)
    for rep in range(2):
        rx, ry, rz, per = _vec(rng, plan, qp, qps, nrhs)
        rx_d, ry_d, rz_d = (torch.from_numpy(v).cuda() for v in (rx, ry, rz))
        x = zeros(lens["rhs"])
        qp.reduce_rhs(pools, delta, rx_d, ry_d, rz_d, x)
        # the reduced rhs against the oracle's
        xh = x.cpu().numpy()
        for s, q in enumerate(qps):
            lay = plan.layouts[s]
            n = q.N * q.b + q.ng
            ref = oqp.reduce_rhs(q.arrays, delta, *per[s])
            got = xh[lay.off_rhs:lay.off_rhs + n * nrhs].reshape(n, nrhs)
            assert float(np.max(np.abs(got - ref))) / float(np.max(np.abs(ref))) < 1e-12, ("rhs", s)
        plan.solve(ws, x)
        dy, dz = zeros(qp.lengths["ry"]), zeros(qp.lengths["rz"])
        qp.recover(pools, delta, x, ry_d, rz_d, dy, dz)
        torch.cuda.synchronize()
        assert (info.cpu().numpy() == 0).all()
        xh, dyh, dzh = x.cpu().numpy(), dy.cpu().numpy(), dz.cpu().numpy()
        for s, q in enumerate(qps):
            lay, off = plan.layouts[s], qp.offsets[s]
            n = q.N * q.b + q.ng
            fx, fy, fz = oqp.newton_step_full(q.arrays, rho, delta, *per[s])
            got = (xh[lay.off_rhs:lay.off_rhs + n * nrhs].reshape(n, nrhs),
                   dyh[off["ry"]:off["ry"] + fy.size].reshape(fy.shape),
                   dzh[off["rz"]:off["rz"] + fz.size].reshape(fz.shape))
            for name, g, r in zip(("dx", "dy", "dz"), got, (fx, fy, fz)):
                if r.size == 0:
                    continue
                err = float(np.max(np.abs(g - r))) / float(np.max(np.abs(r)))
                assert err < 1e-9, (name, s, rep, err)
