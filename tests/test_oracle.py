"""Pins of the oracle against what the paper and the mathematics fix (CPU only)."""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import kkt, partition, flops
from paper_2511_00946_amd import workloads
from tests import dense_ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny_system(seed, N, b, ng, nrhs=1):
    rng = np.random.default_rng(seed)
    return workloads.draw_system(rng, N, b, ng, nrhs=nrhs, alpha=b, s_C=0.3, s_B=0.3)


CASES = [
    # (N, b, ng, seg_lens)
    (1, 3, 2, [1]),
    (1, 4, 0, [1]),
    (5, 3, 0, [5]),
    (5, 3, 2, [5]),
    (5, 3, 2, [2, 2]),
    (7, 2, 3, [3, 1, 1]),
    (8, 4, 1, [3, 2, 1]),
    (8, 5, 3, [2, 2, 2]),
    (7, 1, 1, [1, 1, 1, 1]),
    (6, 4, 0, [3, 2]),
]


@pytest.mark.parametrize("N,b,ng,seg", CASES)
def test_factor_blocks_equal_dense_cholesky(N, b, ng, seg):
    """Every block of hat L (including fill) equals LAPACK's chol(P Psi P^T); other blocks are 0."""
    s = tiny_system(100 + N * 7 + b, N, b, ng)
    f = kkt.KKTFactor(s.D, s.C, s.B, s.corner, seg)
    assert f.info == 0
    K = dense_ref.assemble(s.D, s.C, s.B, s.corner)
    L = dense_ref.dense_factor(K, dense_ref.scalar_permutation(seg, b, ng))
    order = dense_ref.permuted_stage_order(seg) + (["g"] if ng else [])
    size = {o: (ng if o == "g" else b) for o in order}
    start, o0 = {}, 0
    for o in order:
        start[o] = o0
        o0 += size[o]
    for i, ri in enumerate(order):
        for j, cj in enumerate(order[: i + 1]):
            ref = L[start[ri]:start[ri] + size[ri], start[cj]:start[cj] + size[cj]]
            got = f.block(ri, cj)
            if got is None:
                assert np.all(ref == 0.0) or np.max(np.abs(ref)) < 1e-15, (ri, cj)
            else:
                np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * max(1.0, np.max(np.abs(ref))))


@pytest.mark.parametrize("N,b,ng,seg", CASES)
def test_solve_equals_dense_solve(N, b, ng, seg):
    s = tiny_system(200 + N + b, N, b, ng, nrhs=3)
    K = dense_ref.assemble(s.D, s.C, s.B, s.corner)
    x = kkt.solve(s.D, s.C, s.B, s.corner, s.r, seg)
    np.testing.assert_allclose(x, np.linalg.solve(K, s.r), rtol=1e-12, atol=1e-13)
    assert kkt.rel_residual(s.D, s.C, s.B, s.corner, x, s.r) < 1e-14


def test_matvec_equals_dense():
    s = tiny_system(3, 6, 3, 2, nrhs=2)
    K = dense_ref.assemble(s.D, s.C, s.B, s.corner)
    np.testing.assert_allclose(kkt.matvec(s.D, s.C, s.B, s.corner, s.r), K @ s.r, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("N,b,ng,seg", CASES[3:8])
def test_reconstruction(N, b, ng, seg):
    """hat L hat L^T = P Psi P^T, assembled from the oracle's blocks."""
    s = tiny_system(300 + N, N, b, ng)
    f = kkt.KKTFactor(s.D, s.C, s.B, s.corner, seg)
    order = f.order + (["g"] if ng else [])
    size = {o: (ng if o == "g" else b) for o in order}
    n = N * b + ng
    L = np.zeros((n, n))
    st, o0 = {}, 0
    for o in order:
        st[o] = o0
        o0 += size[o]
    for i, ri in enumerate(order):
        for cj in order[: i + 1]:
            blk = f.block(ri, cj)
            if blk is not None:
                L[st[ri]:st[ri] + size[ri], st[cj]:st[cj] + size[cj]] = blk
    K = dense_ref.assemble(s.D, s.C, s.B, s.corner)
    P = dense_ref.scalar_permutation(seg, b, ng)
    KP = K[np.ix_(P, P)]
    assert np.linalg.norm(L @ L.T - KP) / np.linalg.norm(K) < 1e-15
    assert np.all(np.triu(L, 1) == 0)


@pytest.mark.parametrize("seg", [[9], [4, 4], [3, 2, 2], [1, 1, 1, 1, 1]])
def test_laplacian_closed_form(seg):
    """Psi = T_N (x) I_b with T_N = tridiag(-1, 2, -1): L_ii = sqrt((i+1)/i) I,
    L_{i+1,i} = -sqrt(i/(i+1)) I (1-based, natural order), and
    (T_N^{-1})_{ij} = min(i,j)(N+1-max(i,j))/(N+1)."""
    N, b = sum(seg) + len(seg) - 1, 3
    D = np.repeat(2.0 * np.eye(b)[None], N, 0)
    C = np.repeat(-np.eye(b)[None], N - 1, 0)
    B = np.zeros((N, 0, b))
    f = kkt.KKTFactor(D, C, B, np.zeros((0, 0)), seg)
    if len(seg) == 1:
        for i in range(1, N + 1):
            np.testing.assert_allclose(f.block(i - 1, i - 1), np.sqrt((i + 1) / i) * np.eye(b), rtol=2e-16 * 8)
            if i < N:
                np.testing.assert_allclose(f.block(i, i - 1), -np.sqrt(i / (i + 1)) * np.eye(b), rtol=2e-16 * 8)
    idx = np.arange(1, N + 1)
    Tinv = np.minimum.outer(idx, idx) * (N + 1 - np.maximum.outer(idx, idx)) / (N + 1)
    rng = np.random.default_rng(7)
    r = rng.standard_normal((N * b, 2))
    x_ref = np.einsum("ij,jtq->itq", Tinv, r.reshape(N, b, 2)).reshape(N * b, 2)
    np.testing.assert_allclose(f.solve(r), x_ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("seg", [[10], [5, 4], [2, 2, 2, 2], [4, 1, 1, 1]])
def test_rank_one_arrow_closed_form(seg):
    """ng = 1, B_i = c 1^T, corner = gamma on T_N (x) I_b: hat R = sqrt(gamma - c^2 b N(N+1)(N+2)/12)
    for every block order, since g is eliminated last in all of them."""
    N, b, c, gam = sum(seg) + len(seg) - 1, 2, 0.3, 50.0
    D = np.repeat(2.0 * np.eye(b)[None], N, 0)
    C = np.repeat(-np.eye(b)[None], N - 1, 0)
    B = np.full((N, 1, b), c)
    f = kkt.KKTFactor(D, C, B, np.array([[gam]]), seg)
    expect = np.sqrt(gam - c * c * b * N * (N + 1) * (N + 2) / 12.0)
    np.testing.assert_allclose(f.block("g", "g")[0, 0], expect, rtol=1e-14)


def test_invariants_across_orders():
    """x, hat R and log det Psi do not depend on the segmentation; logdet = numpy slogdet."""
    s = workloads.single("small")
    K = dense_ref.assemble(s.D, s.C, s.B, s.corner)
    sign, ld = np.linalg.slogdet(K)
    assert sign > 0
    xs, Rs = [], []
    for seg in ([16], [7, 8], [6, 4, 4], [4, 3, 3, 3], [2, 1, 1, 1, 1, 1, 1, 1]):
        f = kkt.KKTFactor(s.D, s.C, s.B, s.corner, seg)
        assert abs(f.logdet() - ld) < 1e-12 * abs(ld) + 1e-12
        xs.append(f.solve(s.r))
        Rs.append(f.block("g", "g"))
    for x in xs[1:]:
        np.testing.assert_allclose(x, xs[0], rtol=1e-12, atol=1e-14)
    for R in Rs[1:]:
        np.testing.assert_allclose(R, Rs[0], rtol=1e-13)


@pytest.mark.parametrize("seg,j", [([8], 4), ([3, 2, 1], 2), ([3, 2, 1], 3), ([3, 2, 1], 7), ([2, 2, 2], 6)])
def test_indefinite_block_reports_its_stage(seg, j):
    N, b = sum(seg) + len(seg) - 1, 3
    s = tiny_system(11, N, b, 2)
    D = s.D.copy()
    D[j] = -np.eye(b)
    f = kkt.KKTFactor(D, s.C, s.B, s.corner, seg)
    assert f.info == j + 1


def test_indefinite_corner_reports_N_plus_1():
    s = tiny_system(12, 5, 2, 2)
    f = kkt.KKTFactor(s.D, s.C, s.B, -np.eye(2), [2, 2])
    assert f.info == 6


def _fd_grad(fun, a, idx, h=1e-6):
    ap, am = a.copy(), a.copy()
    ap[idx] += h
    am[idx] -= h
    return (fun(ap) - fun(am)) / (2 * h)


@pytest.mark.parametrize("N,b,ng,seg", [(5, 3, 2, [2, 2]), (6, 2, 0, [6]), (7, 3, 1, [3, 1, 1])])
def test_adjoint_against_central_differences(N, b, ng, seg):
    """Gradients of L = sum(w * x), Psi x = r, against central differences (h = 1e-6) of a dense solve."""
    s = tiny_system(40 + N, N, b, ng, nrhs=2)
    w = np.random.default_rng(41).standard_normal(s.r.shape)
    x = kkt.solve(s.D, s.C, s.B, s.corner, s.r, seg)
    lam, dD, dC, dB, dcorner = kkt.adjoint(s.D, s.C, s.B, s.corner, x, w, seg)

    def loss(D=s.D, C=s.C, B=s.B, corner=s.corner, r=s.r):
        K = dense_ref.assemble(D, C, B, corner)
        return float(np.sum(w * np.linalg.solve(K, r)))

    rng = np.random.default_rng(5)
    checks = [("D", s.D, dD, lambda a: loss(D=a)), ("C", s.C, dC, lambda a: loss(C=a)),
              ("r", s.r, lam, lambda a: loss(r=a))]
    if ng:
        checks += [("B", s.B, dB, lambda a: loss(B=a)), ("corner", s.corner, dcorner, lambda a: loss(corner=a))]
    for name, arr, grad, fun in checks:
        for _ in range(8):
            idx = tuple(int(rng.integers(0, d)) for d in arr.shape)
            fd = _fd_grad(fun, arr, idx)
            assert abs(fd - grad[idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, grad[idx])


def test_adjoint_against_dense_autograd():
    torch = pytest.importorskip("torch")
    s = tiny_system(77, 6, 3, 2, nrhs=2)
    w = np.random.default_rng(78).standard_normal(s.r.shape)
    seg = [2, 1, 1]
    x = kkt.solve(s.D, s.C, s.B, s.corner, s.r, seg)
    lam, dD, dC, dB, dcorner = kkt.adjoint(s.D, s.C, s.B, s.corner, x, w, seg)
    T = lambda a: torch.tensor(a, dtype=torch.float64, requires_grad=True)
    tD, tC, tB, tR, tr = T(s.D), T(s.C), T(s.B), T(s.corner), T(s.r)
    N, b, ng = 6, 3, 2
    rows = []
    for i in range(N):
        blocks = []
        for j in range(N):
            if i == j:
                blocks.append(0.5 * (tD[i] + tD[i].T))
            elif i == j + 1:
                blocks.append(tC[j])
            elif j == i + 1:
                blocks.append(tC[i].T)
            else:
                blocks.append(torch.zeros(b, b, dtype=torch.float64))
        blocks.append(tB[i].T)
        rows.append(torch.cat(blocks, 1))
    rows.append(torch.cat([tB[j] for j in range(N)] + [0.5 * (tR + tR.T)], 1))
    K = torch.cat(rows, 0)
    L = (torch.tensor(w) * torch.linalg.solve(K, tr)).sum()
    L.backward()
    for got, ref in ((dD, tD.grad), (dC, tC.grad), (dB, tB.grad), (dcorner, tR.grad), (lam, tr.grad)):
        np.testing.assert_allclose(got, ref.numpy(), rtol=1e-9, atol=1e-12)


def _read_table2():
    rows = {}
    with open(os.path.join(GOLDEN, "table2_speedups.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            conv = lambda v: None if v == "-" else int(v)
            rows[int(t[0])] = (float(t[1]), conv(t[2]), conv(t[3]), conv(t[4]), conv(t[5]))
    return rows


def test_partition_reproduces_table2():
    """All 40 cells of Table 2 (paper-table mode, see partition.py)."""
    for p, (gmax, n2, n3, n4, n09) in _read_table2().items():
        g = partition.gamma_max(p)
        assert round(float(g), 2) == gmax
        for thr, expect in ((2, n2), (3, n3), (4, n4)):
            got = partition.first_horizon(p, thr) if g > thr else None
            assert got == expect, (p, thr, got, expect)
        assert partition.first_horizon(p, Fraction(9, 10) * g) == n09


def test_partition_production_mode_differs_only_where_n1_would_vanish():
    diffs = []
    for p, (gmax, n2, n3, n4, n09) in _read_table2().items():
        g = partition.gamma_max(p)
        for thr, expect in ((2, n2), (3, n3), (4, n4), (Fraction(9, 10) * g, n09)):
            got = partition.first_horizon(p, thr, paper_table=False) if g > thr else None
            if got != expect:
                diffs.append((p, thr, got, expect))
    assert diffs == [(14, 2, 53, 52), (16, 2, 61, 58)]


def test_partition_rule_properties():
    for p in range(2, 20):
        for N in range(2 * p - 1, 300, 7):
            n1, nk = partition.segment_lengths(N, p)
            assert n1 >= 1 and nk >= 1 and n1 + (p - 1) * nk + p - 1 == N
            nbar = Fraction(N - p + 1) / (p - 1 + partition.SIGMA)
            assert nk in (int(nbar), int(nbar) + 1) or nbar == int(nbar)
        with pytest.raises(ValueError):
            partition.segment_lengths(2 * p - 2, p)
    # the configurations of the chain-shaped workload
    assert partition.segment_lengths(128, 4) == (59, 22)
    assert partition.segment_lengths(128, 8) == (30, 13)
    assert partition.segment_lengths(128, 16) == (8, 7)
    assert partition.segment_lengths(128, 32) == (4, 3)


def _read_table1():
    out = {}
    with open(os.path.join(GOLDEN, "table1_flops.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            ph, fa, fc, sa, sc = line.split()
            out[ph] = tuple(Fraction(v) for v in (fa, fc, sa, sc))
    return out


@pytest.mark.parametrize("seg", [[10, 4, 4, 4], [9, 3, 3], [5, 2], [30, 11, 11, 11, 11, 11], [3, 1, 1]])
def test_op_lists_reproduce_table1(seg):
    t1 = _read_table1()
    p = len(seg)
    fac = flops.phase_totals(flops.factor_ops(seg, 1))
    sol = flops.phase_totals(flops.solve_ops(seg, 1))
    fa, fc, sa, sc = t1["first"]
    assert fac["first"] == fa * seg[0] + fc and sol["first"] == sa * seg[0] + sc
    fa, fc, sa, sc = t1["last"]
    assert fac["last"] == fa * seg[-1] + fc and sol["last"] == sa * seg[-1] + sc
    if p > 2:
        fa, fc, sa, sc = t1["other"]
        assert fac["other"] == sum(fa * n + fc for n in seg[1:-1])
        assert sol["other"] == sum(sa * n + sc for n in seg[1:-1])
    fa, fc, sa, sc = t1["seq"]
    assert fac["seq"] == fa * p + fc and sol["seq"] == sa * p + sc


def test_op_list_p1_equals_sequential_complexity():
    """p = 1 is the sequential method: O_seq = (7/3 N - 2) b^3 (Sec. 3.3)."""
    for N in (1, 2, 5, 40):
        assert flops.phase_totals(flops.factor_ops([N], 1))["first"] == partition.o_seq(N)


# ---- the op lists with an arrow (n_g > 0), against a symbolic block Cholesky

def _symbolic_block_cholesky_flops(N, seg, b, ng):
    """Standard flops of the right-looking block Cholesky of P Psi P^T (Sec. 3.1
    order: segment stages, separators, g) found by a symbolic factorization of the
    block pattern (fill created as it appears), and of the two block triangular
    solves with one rhs.  Written from the textbook definition, not from Algorithms
    1-3: column j factors its diagonal block (potrf), solves every nonzero block
    below it (trsm) and updates every pair of them (syrk on the diagonal, gemm off
    it); a solve takes one trsv per diagonal block and one gemv per nonzero block
    in each direction."""
    order = kkt.elimination_order(N, seg)
    pos = {s: i for i, s in enumerate(order)}
    M = N + (1 if ng else 0)
    size = [b] * N + ([ng] if ng else [])
    nz = set()
    for s in range(N - 1):
        i, j = pos[s + 1], pos[s]
        nz.add((max(i, j), min(i, j)))
    if ng:
        for s in range(N):
            nz.add((N, pos[s]))
    fac = Fraction(0)
    sol = Fraction(0)
    for j in range(M):
        nj = size[j]
        fac += Fraction(nj ** 3, 3)
        sol += 2 * nj * nj
        below = sorted(i for (i, jj) in nz if jj == j)
        for i in below:
            fac += size[i] * nj * nj
            sol += 2 * (2 * size[i] * nj)
        for x, i in enumerate(below):
            for l in below[:x + 1]:
                if i == l:
                    fac += size[i] * size[i] * nj
                else:
                    fac += 2 * size[i] * size[l] * nj
                    nz.add((i, l))
    return fac, sol


@pytest.mark.parametrize("N,seg,b,ng", [(16, [16], 4, 2), (40, [5, 4, 4, 4, 4, 4, 4, 4], 6, 8),
                                        (30, [9, 6, 6, 6], 3, 5), (9, [3, 2, 2], 2, 1), (12, [4, 3, 3], 5, 0),
                                        (21, [6, 4, 4, 4], 3, 4)])
def test_op_lists_with_arrow_equal_symbolic_block_cholesky(N, seg, b, ng):
    """The operation lists of Algorithms 1-3 with a global block (n_g > 0) cost
    exactly what a symbolic right-looking block Cholesky of the permuted matrix
    costs, plus the paper's separate accumulation of the corner partials (gead:
    n_g^2 per segment for the factor, n_g per segment for a solve)."""
    assert sum(seg) + len(seg) - 1 == N and len(set(seg[1:])) <= 1
    p = len(seg)
    fac, sol = _symbolic_block_cholesky_flops(N, seg, b, ng)
    f = sum(flops.std_cost(op, m, n, k) for _, op, m, n, k in flops.factor_ops(seg, b, ng))
    s = sum(flops.std_cost(op, m, n, k) for _, op, m, n, k in flops.solve_ops(seg, b, ng))
    gead_f = ng * ng * p if ng else 0
    gead_s = ng * p if ng else 0
    assert f == fac + gead_f
    assert s == sol + gead_s


def test_symbolic_count_catches_a_dropped_arrow_term():
    """The pin above is sensitive to the arrow terms: removing one gemm(ng, b, b)
    from the op list of a segment with fill rows changes the total."""
    seg, b, ng = [9, 6, 6, 6], 3, 5
    fac, _ = _symbolic_block_cholesky_flops(30, seg, b, ng)
    ops = flops.factor_ops(seg, b, ng)
    i = next(x for x, o in enumerate(ops) if o[0] == "other" and o[1] == "gemm" and o[2] == ng)
    f = sum(flops.std_cost(op, m, n, k) for _, op, m, n, k in ops[:i] + ops[i + 1:])
    assert f != fac + ng * ng * len(seg)


@pytest.mark.parametrize("seg", [None, [9, 4, 4, 4]])
def test_solution_is_invariant_under_symmetric_diagonal_scaling(seg):
    """Invariant: for S = diag(s_i^(1/2) I_b, s_g^(1/2) I_ng), the solution of
    (S Psi S) x' = r is x' = S^-1 u with Psi u = S^-1 r.  The blocks of S Psi S are
    s_i D_i, (s_i s_{i+1})^(1/2) C_i, (s_g s_i)^(1/2) B_i and s_g corner; a dropped or
    misplaced block scale (or a transposed coupling) breaks the identity by far
    more than rounding (scales from 1e-4 to 1e4).  Pins the scale handling of
    every block against the unscaled solve."""
    rng = np.random.default_rng(21)
    N, b, ng = 24, 5, 3
    sy = workloads.draw_system(rng, N, b, ng, nrhs=2, alpha=b, s_C=0.3, s_B=0.3)
    s = 10.0 ** rng.uniform(-4, 4, size=N)
    sg = 10.0 ** rng.uniform(-4, 4)
    h = np.sqrt(s)
    D = sy.D * s[:, None, None]
    C = sy.C * (h[1:] * h[:-1])[:, None, None]
    B = sy.B * (np.sqrt(sg) * h)[:, None, None]
    corner = sy.corner * sg
    S = np.concatenate([np.repeat(h, b), np.full(ng, np.sqrt(sg))])
    xs = kkt.solve(D, C, B, corner, sy.r, seg)
    u = kkt.solve(sy.D, sy.C, sy.B, sy.corner, sy.r / S[:, None], seg)
    assert np.max(np.abs(S[:, None] * xs - u)) <= 1e-12 * np.max(np.abs(u))
    # the check sees a transposed coupling block (the matrix stays definite)
    xb = kkt.solve(D, np.swapaxes(C, 1, 2).copy(), B, corner, sy.r, seg)
    assert np.max(np.abs(S[:, None] * xb - u)) > 1e-6 * np.max(np.abs(u))


def _ragged_system(rng, sizes, ng, nrhs):
    N = len(sizes)
    D = []
    for n in sizes:
        M = rng.standard_normal((n, n))
        D.append(M @ M.T + n * np.eye(n) + np.eye(n))
    C = [0.2 * rng.standard_normal((sizes[i + 1], sizes[i])) for i in range(N - 1)]
    B = [0.2 * rng.standard_normal((ng, n)) for n in sizes]
    R = rng.standard_normal((ng, ng))
    corner = R @ R.T + (ng + N) * np.eye(ng) if ng else None
    r = rng.standard_normal((int(sum(sizes)) + ng, nrhs))
    return D, C, B, corner, r


def _dense_ragged(D, C, B, corner):
    sizes = [d.shape[0] for d in D]
    off = kkt.ragged_offsets(sizes)
    N = len(D)
    ng = 0 if corner is None else corner.shape[0]
    A = np.zeros((off[N] + ng, off[N] + ng))
    for i in range(N):
        A[off[i]:off[i + 1], off[i]:off[i + 1]] = 0.5 * (D[i] + D[i].T)
        if i + 1 < N:
            A[off[i + 1]:off[i + 2], off[i]:off[i + 1]] = C[i]
            A[off[i]:off[i + 1], off[i + 1]:off[i + 2]] = C[i].T
        if ng:
            A[off[N]:, off[i]:off[i + 1]] = B[i]
            A[off[i]:off[i + 1], off[N]:] = B[i].T
    if ng:
        A[off[N]:, off[N]:] = 0.5 * (corner + corner.T)
    return A


@pytest.mark.parametrize("sizes,ng", [([3, 1, 4, 2, 5], 2), ([1, 1, 1], 0), ([6, 2, 6, 3], 3), ([2], 1)])
def test_ragged_solve_matches_lapack(sizes, ng):
    """The non-uniform oracle against LAPACK on the assembled dense matrix (its
    definition), and its mat-vec against the dense product."""
    rng = np.random.default_rng(31)
    D, C, B, corner, r = _ragged_system(rng, sizes, ng, 2)
    A = _dense_ragged(D, C, B, corner)
    x = kkt.solve_ragged(D, C, B, corner, r)
    assert np.allclose(x, np.linalg.solve(A, r), rtol=1e-12, atol=1e-12)
    assert np.allclose(kkt.matvec_ragged(D, C, B, corner, x), A @ x, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seg", [None, [4, 2, 2]])
def test_ragged_equals_identity_padded_uniform_solve(seg):
    """Padding every stage to b = max n_i with the identity on the padded diagonal
    and zeros in the couplings is exact: the uniform solve of the padded system
    (any segmentation), restricted to the real entries, is the ragged solution."""
    rng = np.random.default_rng(32)
    sizes, ng = [3, 5, 1, 4, 5, 2, 3, 4, 2, 5], 3
    D, C, B, corner, r = _ragged_system(rng, sizes, ng, 2)
    N, b = len(sizes), max(sizes)
    Dp = np.zeros((N, b, b))
    Cp = np.zeros((N - 1, b, b))
    Bp = np.zeros((N, ng, b))
    rp = np.zeros((N * b + ng, 2))
    off = kkt.ragged_offsets(sizes)
    for i, n in enumerate(sizes):
        Dp[i] = np.eye(b)
        Dp[i, :n, :n] = D[i]
        Bp[i, :, :n] = B[i]
        rp[i * b:i * b + n] = r[off[i]:off[i + 1]]
        if i + 1 < N:
            Cp[i, :sizes[i + 1], :n] = C[i]
    rp[N * b:] = r[off[N]:]
    xp = kkt.solve(Dp, Cp, Bp, corner, rp, seg)
    x = kkt.solve_ragged(D, C, B, corner, r)
    back = np.concatenate([xp[i * b:i * b + n] for i, n in enumerate(sizes)] + [xp[N * b:]])
    assert np.allclose(back, x, rtol=1e-12, atol=1e-13)
    for i, n in enumerate(sizes):
        assert np.all(np.abs(xp[i * b + n:(i + 1) * b]) < 1e-14)


# ---------------------------------------------------------------- recursive segmentation
def test_nested_order_hand_examples():
    """Two and three levels, written out by hand."""
    assert kkt.nested_order(15, [[3, 3, 3, 3], [1, 1]]) == [0, 1, 2, 4, 5, 6, 8, 9, 10, 12, 13, 14, 3, 11, 7]
    lev0 = [i for i in range(31) if i % 4 != 3]
    assert kkt.nested_order(31, [[3] * 8, [1] * 4, [1, 1]]) == lev0 + [3, 11, 19, 27, 7, 23, 15]
    assert kkt.nested_order(11, [[3, 3, 3]]) == kkt.elimination_order(11, [3, 3, 3])
    # a one-segment level eliminates the whole chain of separators in order
    assert kkt.nested_order(11, [[3, 3, 3], [2]]) == kkt.elimination_order(11, [3, 3, 3])


NEST_CASES = [
    # (N, b, ng, seg_lens, nest)
    (15, 2, 2, [3, 3, 3, 3], [[1, 1]]),
    (19, 3, 0, [2, 2, 2, 2, 2, 2, 1], [[2, 1, 1]]),
    (31, 2, 3, [3] * 8, [[1] * 4, [1, 1]]),
    (23, 3, 1, [4, 3, 3, 3, 3, 2], [[2, 2]]),
]


def _dense_blocks_check(f, N, b, ng, levels, s):
    K = dense_ref.assemble(s.D, s.C, s.B, s.corner)
    L = dense_ref.dense_factor(K, dense_ref.nested_scalar_permutation(N, levels, b, ng))
    order = dense_ref.nested_stage_order(N, levels) + (["g"] if ng else [])
    size = {o: (ng if o == "g" else b) for o in order}
    start, o0 = {}, 0
    for o in order:
        start[o] = o0
        o0 += size[o]
    for i, ri in enumerate(order):
        for cj in order[: i + 1]:
            ref = L[start[ri]:start[ri] + size[ri], start[cj]:start[cj] + size[cj]]
            got = f.block(ri, cj)
            if got is None:
                assert np.max(np.abs(ref), initial=0.0) < 1e-15, (ri, cj)
            else:
                np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * max(1.0, np.max(np.abs(ref))))


@pytest.mark.parametrize("N,b,ng,seg,nest", NEST_CASES)
def test_nested_factor_equals_dense_cholesky(N, b, ng, seg, nest):
    """Every block of the multi-level factor equals LAPACK's Cholesky of the matrix
    permuted by an independently written nested order."""
    s = tiny_system(500 + N + b, N, b, ng)
    f = kkt.KKTFactor(s.D, s.C, s.B, s.corner, seg, nest=nest)
    assert f.info == 0
    _dense_blocks_check(f, N, b, ng, [seg] + nest, s)


@pytest.mark.parametrize("N,b,ng,seg,nest", NEST_CASES)
def test_nested_solve_equals_dense_solve(N, b, ng, seg, nest):
    s = tiny_system(600 + N + b, N, b, ng, nrhs=2)
    x = kkt.solve(s.D, s.C, s.B, s.corner, s.r, seg, nest=nest)
    K = dense_ref.assemble(s.D, s.C, s.B, s.corner)
    np.testing.assert_allclose(x, np.linalg.solve(K, s.r), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("N,b,ng,seg,nest", NEST_CASES)
def test_reduced_system_is_a_chain_and_carries_the_nested_factor(N, b, ng, seg, nest):
    """The Schur complement on the separators couples only neighbouring separators
    (a block-tridiagonal arrow chain); its solution is the separators' part of x;
    and segmenting it gives exactly the separator blocks of the multi-level factor."""
    s = tiny_system(700 + N + b, N, b, ng, nrhs=2)
    # structure, from the dense matrix: separators two apart are not coupled
    K = dense_ref.assemble(s.D, s.C, s.B, s.corner)
    _, seps = kkt.stage_layout(N, seg)
    I = [st * b + t for st in range(N) if st not in seps for t in range(b)]
    S = [st * b + t for st in seps for t in range(b)] + [N * b + t for t in range(ng)]
    Sm = K[np.ix_(S, S)] - K[np.ix_(S, I)] @ np.linalg.solve(K[np.ix_(I, I)], K[np.ix_(I, S)])
    M = len(seps)
    for i in range(M):
        for j in range(i + 2, M):
            assert np.max(np.abs(Sm[j * b:(j + 1) * b, i * b:(i + 1) * b])) < 1e-13
    Dr, Cr, Br, cr, rr = kkt.reduced_system(s.D, s.C, s.B, s.corner, seg, s.r)
    assert Dr.shape == (M, b, b) and Cr.shape == (M - 1, b, b)
    np.testing.assert_allclose(Dr, np.swapaxes(Dr, 1, 2), rtol=0, atol=1e-13)
    # the reduced solve gives the separators and g of the full solution
    x = np.linalg.solve(K, s.r)
    xr = kkt.solve(Dr, Cr, Br, cr, rr, None)
    xs = np.concatenate([x[st * b:(st + 1) * b] for st in seps] + ([x[N * b:]] if ng else []))
    np.testing.assert_allclose(xr, xs, rtol=1e-11, atol=1e-12)
    # the nested factor's separator blocks are the factor of the segmented chain
    f = kkt.KKTFactor(s.D, s.C, s.B, s.corner, seg, nest=nest)
    fr = kkt.KKTFactor(Dr, Cr, Br, cr, nest[0], nest=nest[1:])
    lab = {j: st for j, st in enumerate(seps)}
    keys = list(range(M)) + (["g"] if ng else [])
    for i, ri in enumerate(fr.order + (["g"] if ng else [])):
        for cj in (fr.order + (["g"] if ng else []))[: i + 1]:
            got = fr.block(ri, cj)
            ref = f.block(lab.get(ri, ri), lab.get(cj, cj))
            if got is None:
                assert ref is None or np.max(np.abs(ref)) < 1e-14
            else:
                np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * max(1.0, np.max(np.abs(ref))))
    assert len(keys) == M + (1 if ng else 0)


def test_nested_failure_is_first_in_the_nested_order():
    """Two indefinite separator blocks: the one eliminated first under the nested
    order is reported, which differs from the single-level order's choice."""
    N, b = 15, 2
    s = tiny_system(31, N, b, 2)
    D = s.D.copy()
    D[7] = -np.eye(b)    # level-1 separator: eliminated last
    D[11] = -np.eye(b)   # level-1 segment stage: eliminated before it
    assert kkt.KKTFactor(D, s.C, s.B, s.corner, [3, 3, 3, 3]).info == 8
    assert kkt.KKTFactor(D, s.C, s.B, s.corner, [3, 3, 3, 3], nest=[[1, 1]]).info == 12


# ---------------------------------------------------------------- multistage QP -> KKT (scope row f3)
from oracle import qp as oqp


def _qp(seed, N, b, ng, pe, me):
    return workloads.draw_qp(np.random.default_rng(seed), N, b, ng, pe, me).arrays


@pytest.mark.parametrize("N,b,ng,pe,me", [(4, 3, 2, 2, 3), (1, 2, 1, 1, 2), (5, 2, 0, 3, 1)])
def test_qp_dense_parts_follow_eq1(N, b, ng, pe, me):
    """The Hessian and the stacked constraint rows reproduce Eq. 1 evaluated term by
    term at a random point: the coupled stage costs and the terminal cost, and each
    group's equality and inequality rows."""
    d = _qp(7 + N, N, b, ng, pe, me)
    P, A, G = oqp.dense_parts(d)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((N, b))
    g = rng.standard_normal(ng)
    z = np.concatenate([x.reshape(-1), g])
    cost = 0.0
    for i in range(N - 1):
        v = np.concatenate([x[i], x[i + 1], g])
        H = np.zeros((2 * b + ng, 2 * b + ng))
        H[:b, :b] = d["Q"][i]
        H[b:2 * b, :b] = d["S"][i]
        H[:b, b:2 * b] = d["S"][i].T
        if ng:
            H[2 * b:, :b] = d["T"][i]
            H[:b, 2 * b:] = d["T"][i].T
        cost += 0.5 * v @ H @ v
    v = np.concatenate([x[N - 1], g])
    H = np.zeros((b + ng, b + ng))
    H[:b, :b] = d["Q"][N - 1]
    if ng:
        H[b:, :b] = d["T"][N - 1]
        H[:b, b:] = d["T"][N - 1].T
        H[b:, b:] = d["Qg"]
    cost += 0.5 * v @ H @ v
    assert 0.5 * z @ P @ z == pytest.approx(cost, rel=1e-13)
    for k in range(N):
        eq = d["EL"][k] @ x[k] + (d["ER"][k] @ x[k + 1] if k < N - 1 else 0) + (d["EG"][k] @ g if ng else 0)
        iq = d["IL"][k] @ x[k] + (d["IR"][k] @ x[k + 1] if k < N - 1 else 0) + (d["IG"][k] @ g if ng else 0)
        np.testing.assert_allclose((A @ z)[k * pe:(k + 1) * pe], eq, rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose((G @ z)[k * me:(k + 1) * me], iq, rtol=1e-13, atol=1e-14)


def test_qp_assembly_scalar_closed_form():
    """One stage of size 1, one equality and one inequality row: Psi is the scalar
    Q + rho + EL^2 / delta + w IL^2."""
    d = dict(Q=np.array([[[2.0]]]), S=np.zeros((0, 1, 1)), T=np.zeros((1, 0, 1)), Qg=np.zeros((0, 0)),
             EL=np.array([[[3.0]]]), ER=np.zeros((0, 1, 1)), EG=np.zeros((1, 1, 0)),
             IL=np.array([[[-5.0]]]), IR=np.zeros((0, 1, 1)), IG=np.zeros((1, 1, 0)), w=np.array([[0.25]]))
    D, C, B, corner, _ = oqp.assemble(d, 0.5, 0.1)
    assert D[0, 0, 0] == pytest.approx(2.0 + 0.5 + 9.0 / 0.1 + 0.25 * 25.0, rel=1e-15)


@pytest.mark.parametrize("N,b,ng,pe,me", [(6, 3, 2, 2, 4), (5, 4, 0, 4, 2), (3, 2, 3, 1, 1)])
def test_qp_psi_is_a_block_tridiagonal_arrow_spd_matrix(N, b, ng, pe, me):
    d = _qp(20 + N, N, b, ng, pe, me)
    D, C, B, corner, Psi = oqp.assemble(d, 1e-2, 1e-3)
    for i in range(N):
        for j in range(i + 2, N):
            assert np.max(np.abs(Psi[j * b:(j + 1) * b, i * b:(i + 1) * b])) == 0.0
    np.testing.assert_allclose(Psi, Psi.T, rtol=0, atol=1e-12 * np.max(np.abs(Psi)))
    np.linalg.cholesky(Psi)
    # the block arrays rebuild the same matrix through the KKT oracle's assembly
    x = np.random.default_rng(3).standard_normal((N * b + ng, 2))
    np.testing.assert_allclose(kkt.matvec(D, C, B if ng else None, corner, x), Psi @ x, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("N,b,ng,pe,me", [(6, 3, 2, 2, 4), (7, 2, 1, 3, 3), (4, 4, 0, 2, 5)])
def test_qp_reduced_newton_step_equals_the_full_saddle_point_solve(N, b, ng, pe, me):
    """Reduce the rhs, solve with Psi (block Cholesky oracle), recover dy and dz: the
    same step as LAPACK on the unreduced saddle-point matrix, for several rhs."""
    d = _qp(40 + N, N, b, ng, pe, me)
    rho, delta = 1e-3, 1e-2
    rng = np.random.default_rng(5)
    rx = rng.standard_normal((N * b + ng, 2))
    ry = rng.standard_normal((N * pe, 2))
    rz = rng.standard_normal((N * me, 2))
    D, C, B, corner, _ = oqp.assemble(d, rho, delta)
    r = oqp.reduce_rhs(d, delta, rx, ry, rz)
    dx = kkt.solve(D, C, B if ng else None, corner, r, [N])
    dy, dz = oqp.recover(d, delta, dx, ry, rz)
    fx, fy, fz = oqp.newton_step_full(d, rho, delta, rx, ry, rz)
    for got, ref in ((dx, fx), (dy, fy), (dz, fz)):
        np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-10 * np.max(np.abs(ref)))


# ---------------------------------------------------------------- the interior-point loop (scope row f3)
from oracle import ipm as oipm


def _kkt_residuals(q, c, beq, h, sol):
    P, A, G = oqp.dense_parts(q.arrays)
    x, y, z, s = sol["x"], sol["y"], sol["z"], sol["s"]
    return (np.max(np.abs(P @ x + c + A.T @ y + G.T @ z), initial=0.0), np.max(np.abs(A @ x - beq), initial=0.0),
            np.max(np.abs(G @ x + s - h), initial=0.0), float(s @ z) / max(1, s.size))


@pytest.mark.parametrize("N,b,ng,pe,me", [(5, 3, 2, 1, 4), (8, 2, 1, 1, 3), (4, 4, 0, 2, 6), (6, 3, 2, 2, 0)])
def test_ipm_reaches_a_kkt_point(N, b, ng, pe, me):
    """Stationarity, primal feasibility and complementarity at the loop's result
    (the optimality conditions of the convex QP), with s, z > 0."""
    q, c, beq, h = workloads.draw_qp_problem(np.random.default_rng(80 + N), N, b, ng, pe, me)
    sol = oipm.solve(q.arrays, c, beq, h)
    assert sol["converged"] and sol["iterations"] < 40
    rd, rp, rs, gap = _kkt_residuals(q, c, beq, h, sol)
    assert max(rd, rp, rs, gap) < 1e-8
    if me:
        assert np.all(sol["s"] > 0) and np.all(sol["z"] > 0)


def test_ipm_matches_an_independent_solver():
    """A tiny strictly convex QP: the same minimiser as scipy's SLSQP on the
    dense problem."""
    from scipy.optimize import minimize
    q, c, beq, h = workloads.draw_qp_problem(np.random.default_rng(91), 3, 2, 1, 1, 2)
    P, A, G = oqp.dense_parts(q.arrays)
    sol = oipm.solve(q.arrays, c, beq, h)
    res = minimize(lambda v: 0.5 * v @ P @ v + c @ v, np.zeros(P.shape[0]), jac=lambda v: P @ v + c, method="SLSQP",
                   constraints=[{"type": "eq", "fun": lambda v: A @ v - beq, "jac": lambda v: A},
                                {"type": "ineq", "fun": lambda v: h - G @ v, "jac": lambda v: -G}],
                   options={"ftol": 1e-14, "maxiter": 500})
    assert res.success
    np.testing.assert_allclose(sol["x"], res.x, rtol=0, atol=1e-6)
