"""GPU: non-uniform stage sizes (each stage i with its own size n_i) through the
C ABI: kkt_ragged_pad embeds every stage in the plan's block size b = max n_i
(identity on the padded diagonal, zeros elsewhere), the uniform path factors and
solves, kkt_ragged_unpad returns the real entries.

Checks: the padded pools the device writes equal a host padding of the same
blocks bitwise; x matches the non-uniform oracle (solve_ragged, the block
Cholesky with per-stage sizes) within 1e-10 relative; the relative residual
against the non-uniform matrix is at most 1e-10."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kkt as okkt
from paper_2511_00946_amd import workloads

pytestmark = pytest.mark.gpu


def host_pad(sy, plan, s, nr, pools):
    """Write system s's blocks into numpy copies of the plan's pools."""
    lay = plan.layouts[s]
    N, b, ng = lay.N, lay.b, lay.ng
    for i, n in enumerate(sy.sizes):
        D = np.eye(b)
        D[:n, :n] = sy.D[i]
        pools["D"][lay.off_D + i * b * b:lay.off_D + (i + 1) * b * b] = D.ravel()
        if i + 1 < N:
            C = np.zeros((b, b))
            C[:sy.sizes[i + 1], :n] = sy.C[i]
            pools["C"][lay.off_C + i * b * b:lay.off_C + (i + 1) * b * b] = C.ravel()
        B = np.zeros((ng, b))
        B[:, :n] = sy.B[i]
        pools["B"][lay.off_B + i * ng * b:lay.off_B + (i + 1) * ng * b] = B.ravel()
    pools["corner"][lay.off_corner:lay.off_corner + ng * ng] = sy.corner.ravel()
    off = okkt.ragged_offsets(sy.sizes)
    rp = np.zeros((N * b + ng, nr))
    for i, n in enumerate(sy.sizes):
        rp[i * b:i * b + n] = sy.r[off[i]:off[i + 1]]
    rp[N * b:] = sy.r[off[N]:]
    pools["r"][lay.off_rhs:lay.off_rhs + (N * b + ng) * nr] = rp.ravel()


@pytest.mark.parametrize("p", [1, 3])
def test_ragged_systems_match_the_oracle(p):
    from paper_2511_00946_amd import kkt
    rng = np.random.default_rng(41 + p)
    nr = 2
    shapes = [(rng.integers(1, 9, size=30), 3), (rng.integers(5, 17, size=24), 0), (rng.integers(1, 33, size=20), 4),
              (rng.integers(20, 43, size=12), 2), (np.array([1, 7, 1, 7, 1, 7, 1]), 1)]
    systems = [workloads.draw_ragged_system(rng, [int(n) for n in sizes], ng, nrhs=nr) for sizes, ng in shapes]
    dims = [(len(sy.sizes), max(sy.sizes), sy.ng, p) for sy in systems]
    print("gpu case: ragged p=%d dims=%s" % (p, dims), file=sys.stderr, flush=True)
    plan = kkt.Plan(dims, nrhs=nr)
    rag = kkt.Ragged(plan, [sy.sizes for sy in systems])
    src_h = workloads.pack_ragged(systems)
    assert {k: v.size for k, v in src_h.items()} == {k: rag.lengths[k2] for k, k2 in
                                                     (("D", "D"), ("C", "C"), ("B", "B"), ("corner", "corner"),
                                                      ("r", "rhs"))}
    src = kkt.pack_to_device(src_h)
    lens = plan.pool_lengths()
    dst = {k: torch.full((max(1, lens[k2]),), np.nan, dtype=torch.float64, device="cuda")
           for k, k2 in (("D", "D"), ("C", "C"), ("B", "B"), ("corner", "corner"), ("r", "rhs"))}
    rag.pad(src, dst)
    torch.cuda.synchronize()
    ref = {k: np.full(max(1, lens[k2]), np.nan) for k, k2 in
           (("D", "D"), ("C", "C"), ("B", "B"), ("corner", "corner"), ("r", "rhs"))}
    for s, sy in enumerate(systems):
        host_pad(sy, plan, s, nr, ref)
    for k in ref:
        got = dst[k].cpu().numpy()
        n = lens[{"r": "rhs"}.get(k, k)]
        assert np.array_equal(got[:n], ref[k][:n]), k
    ws = plan.new_workspace()
    info = torch.full((len(systems),), -7, dtype=torch.int32, device="cuda")
    x = dst["r"].clone()
    plan.factor_solve(dst["D"], dst["C"], dst["B"], dst["corner"], ws, x, info)
    xr = torch.full((rag.lengths["rhs"],), np.nan, dtype=torch.float64, device="cuda")
    rag.unpad(x, xr)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    xh = xr.cpu().numpy()
    o = 0
    for sy in systems:
        n = (sum(sy.sizes) + sy.ng) * nr
        xs = xh[o:o + n].reshape(-1, nr)
        o += n
        xo = okkt.solve_ragged(sy.D, sy.C, sy.B, sy.corner if sy.ng else None, sy.r)
        assert float(np.max(np.abs(xs - xo)) / np.max(np.abs(xo))) < 1e-10
        res = okkt.matvec_ragged(sy.D, sy.C, sy.B, sy.corner if sy.ng else None, xs) - sy.r
        assert float(np.max(np.linalg.norm(res, axis=0) / np.linalg.norm(sy.r, axis=0))) < 1e-10
