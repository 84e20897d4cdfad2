"""GPU: badly scaled and nearly singular inputs, through the C ABI.

Scaled systems: Psi' = S Psi S with S = diag(s_i^(1/2) I_b, s_g^(1/2) I_ng), the
s_i drawn log-uniformly from [1e-4, 1e4]: every D_i, C_i, B_i and the corner change
scale by up to eight orders of magnitude while Psi' stays symmetric positive
definite.  Cholesky's accuracy does not depend on such a diagonal scaling, so
u = S x' (the solution of the well-conditioned base system Psi u = S^-1 r) must
match the oracle's to the parity bar of the other tests (1e-10 relative, max
norm); a path that mishandles the scales fails this even where the normwise
backward error below, dominated by the largest rows, stays small.
Nearly singular corner: corner = R R^T + delta I with R of rank ng - 1 and
delta = 1e-9 relative, arrow couplings small enough that Psi stays positive
definite; the corner's Schur complement is then ill conditioned (about 1e9) and
x is not expected to match closely.  Gate there: the normwise backward error
    eta = ||r - Psi x||_inf / (||Psi||_inf ||x||_inf + ||r||_inf)
of the GPU solution is at most 10 times the oracle's (plus 1e-15) and below 1e-13.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kkt as okkt
from paper_2511_00946_amd import workloads

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def scaled(sy, rng, lo=-4.0, hi=4.0):
    N, b, ng = sy.N, sy.b, sy.ng
    s = 10.0 ** rng.uniform(lo, hi, size=N)
    sg = 10.0 ** rng.uniform(lo, hi)
    h = np.sqrt(s)
    D = sy.D * s[:, None, None]
    C = sy.C * (h[1:] * h[:-1])[:, None, None]
    B = sy.B * (np.sqrt(sg) * h)[:, None, None] if ng else sy.B
    corner = sy.corner * sg
    scale = np.concatenate([np.repeat(h, b), np.full(ng, np.sqrt(sg))])
    return workloads.System(N, b, ng, D, C, B, corner, sy.r, None), scale


def near_singular_corner(sy, rng):
    ng = sy.ng
    R = rng.standard_normal((ng, ng - 1))
    K = R @ R.T
    corner = K + 1e-9 * np.trace(K) / ng * np.eye(ng)
    # keep Psi positive definite: the arrow couplings scaled down with the corner's smallest direction
    B = sy.B * 1e-5
    return workloads.System(sy.N, sy.b, ng, sy.D, sy.C, B, corner, sy.r, None)


def psi_norm_inf(sy):
    """||Psi||_inf from the blocks (row sums of absolute values)."""
    N, b, ng = sy.N, sy.b, sy.ng
    rows = np.zeros(N * b + ng)
    for i in range(N):
        Ds = 0.5 * (sy.D[i] + sy.D[i].T)
        rows[i * b:(i + 1) * b] += np.abs(Ds).sum(axis=1)
        if i + 1 < N:
            rows[i * b:(i + 1) * b] += np.abs(sy.C[i]).sum(axis=0)        # Psi_{i,i+1} = C_i^T
            rows[(i + 1) * b:(i + 2) * b] += np.abs(sy.C[i]).sum(axis=1)  # Psi_{i+1,i} = C_i
        if ng:
            rows[i * b:(i + 1) * b] += np.abs(sy.B[i]).sum(axis=0)
            rows[N * b:] += np.abs(sy.B[i]).sum(axis=1)
    if ng:
        rows[N * b:] += np.abs(0.5 * (sy.corner + sy.corner.T)).sum(axis=1)
    return float(rows.max())


def backward_error(sy, x):
    res = sy.r - okkt.matvec(sy.D, sy.C, sy.B, sy.corner, x)
    return float(np.max(np.abs(res)) / (psi_norm_inf(sy) * np.max(np.abs(x)) + np.max(np.abs(sy.r))))


def run(systems, ps):
    from paper_2511_00946_amd import kkt
    plan = kkt.Plan([(s.N, s.b, s.ng, p) for s, p in zip(systems, ps)], nrhs=systems[0].r.shape[1])
    pools = kkt.pack_to_device(workloads.pack(systems))
    ws = plan.new_workspace()
    info = torch.full((len(systems),), -7, dtype=torch.int32, device="cuda")
    x = pools["r"].clone()
    plan.factor_solve(pools["D"], pools["C"], pools["B"], pools["corner"], ws, x, info)
    torch.cuda.synchronize()
    xh = x.cpu().numpy()
    out = []
    for s, sy in enumerate(systems):
        lay = plan.layouts[s]
        out.append(xh[lay.off_rhs:lay.off_rhs + sy.n * plan.nrhs].reshape(sy.n, plan.nrhs))
    return out, info.cpu().numpy()


CASES = [(40, 6, 4), (33, 16, 8), (30, 24, 4), (28, 32, 16), (12, 42, 3)]


@pytest.mark.parametrize("p", [1, 3])
def test_scaled_blocks_keep_the_scaled_solution(p):
    rng = np.random.default_rng(11)
    systems, scales = [], []
    for (N, b, ng) in CASES:
        base = workloads.draw_system(rng, N, b, ng, nrhs=2, alpha=b, s_C=0.05, s_B=0.05)
        sy, sc = scaled(base, rng)
        systems.append(sy)
        scales.append(sc)
    _say("gpu case: scaled blocks p=%d dims=%s" % (p, CASES))
    xs, info = run(systems, [p] * len(systems))
    assert (info == 0).all(), info
    for sy, sc, x, dims in zip(systems, scales, xs, CASES):
        xo = okkt.solve(sy.D, sy.C, sy.B, sy.corner, sy.r)
        u, uo = sc[:, None] * x, sc[:, None] * xo
        err = float(np.max(np.abs(u - uo)) / np.max(np.abs(uo)))
        assert err < 1e-10, (p, dims, err)
        eta_gpu, eta_ora = backward_error(sy, x), backward_error(sy, xo)
        assert eta_gpu <= 10.0 * eta_ora + 1e-15, (p, dims, eta_gpu, eta_ora)


@pytest.mark.parametrize("p", [1, 3])
def test_nearly_singular_corner_backward_error(p):
    rng = np.random.default_rng(12)
    systems = []
    for (N, b, ng) in CASES:
        base = workloads.draw_system(rng, N, b, ng, nrhs=2, alpha=b, s_C=0.05, s_B=0.05)
        systems.append(near_singular_corner(base, rng))
    _say("gpu case: nearly singular corner p=%d dims=%s" % (p, CASES))
    xs, info = run(systems, [p] * len(systems))
    assert (info == 0).all(), info
    for sy, x, dims in zip(systems, xs, CASES):
        xo = okkt.solve(sy.D, sy.C, sy.B, sy.corner, sy.r)
        eta_gpu, eta_ora = backward_error(sy, x), backward_error(sy, xo)
        assert eta_gpu <= 10.0 * eta_ora + 1e-15, (p, dims, eta_gpu, eta_ora)
        assert eta_gpu < 1e-13, (p, dims, eta_gpu)
