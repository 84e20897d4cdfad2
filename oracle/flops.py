"""Operation lists of Algorithms 1-3 and their flop counts (Table 1) -- test infrastructure only.

Not a product module: only tests/ and the benchmark's CPU leg use it.

Each function walks the loop structure of one algorithm and emits the dense block
operations it performs, as (phase, op, m, n, k) tuples, for uniform stage size b
and global size ng.  ``cost`` prices them under the paper's counting convention
(Sec. 3.1, the comments of Algorithms 1-3): potrf n^3/3, trsm m n^2, syrk n^2 k,
gemm 2 m n k, trsv n^2/2, gemv 2 m n, gead m n.  With ng = 0 the per-phase sums
are the polynomials of Table 1.

Phases: "first" (segment 1), "other" (1 < k < p), "last" (segment p, p > 1),
"seq" (sequential phase).  With p = 1 the single segment is reported as "first"
and carries no F / H terms.
"""
from fractions import Fraction


def _phase(k, p):
    if k == 1:
        return "first"
    return "last" if k == p else "other"


def factor_ops(seg_lens, b, ng=0):
    """Algorithm 1 (parallel Cholesky factorization)."""
    p = len(seg_lens)
    ops = []
    for k in range(1, p + 1):
        ph = _phase(k, p)
        nk = seg_lens[k - 1]
        for i in range(1, nk + 1):
            ops.append((ph, "potrf", b, b, b))
            if i < nk:
                ops.append((ph, "trsm", b, b, b))            # hat E
            if ng:
                ops.append((ph, "trsm", ng, b, b))           # hat G
                ops.append((ph, "syrk", ng, ng, b))          # hat R_k
            if i < nk:
                ops.append((ph, "syrk", b, b, b))            # D_{i+1}
                if ng:
                    ops.append((ph, "gemm", ng, b, b))       # G_{i+1}
            if k > 1:
                ops.append((ph, "trsm", b, b, b))            # hat B^T_{ik}
                ops.append((ph, "syrk", b, b, b))            # hat A_k
                if i < nk:
                    ops.append((ph, "gemm", b, b, b))        # B^T_{i+1,k}
                if ng:
                    ops.append((ph, "gemm", ng, b, b))       # hat Q_k
        if k < p:
            ops.append((ph, "trsm", b, b, b))                # hat F_k
        if 1 < k < p:
            ops.append((ph, "gemm", b, b, b))                # hat H_k
    for k in range(2, p + 1):
        ops.append(("seq", "syrk", b, b, b))                 # A_k -= F F^T
        ops.append(("seq", "potrf", b, b, b))
        if k < p:
            ops.append(("seq", "trsm", b, b, b))             # hat H_k
        if ng:
            ops.append(("seq", "gemm", ng, b, b))            # Q_k -= G F^T
            ops.append(("seq", "trsm", ng, b, b))            # hat Q_k
        if k < p:
            ops.append(("seq", "syrk", b, b, b))             # A_{k+1} -= H H^T
            if ng:
                ops.append(("seq", "gemm", ng, b, b))        # Q_{k+1} -= Q H^T
        if ng:
            ops.append(("seq", "syrk", ng, ng, b))           # R -= Q Q^T
    if ng:
        ops.append(("seq", "gead", ng, ng, p))
        ops.append(("seq", "potrf", ng, ng, ng))
    return ops


def solve_ops(seg_lens, b, ng=0):
    """Algorithms 2 and 3 (forward and backward substitution), one rhs."""
    p = len(seg_lens)
    ops = []
    for k in range(1, p + 1):                                # Alg. 2, parallel
        ph = _phase(k, p)
        nk = seg_lens[k - 1]
        for i in range(1, nk + 1):
            ops.append((ph, "trsv", b, b, 1))
            if i < nk:
                ops.append((ph, "gemv", b, b, 1))
            if k > 1:
                ops.append((ph, "gemv", b, b, 1))
            if ng:
                ops.append((ph, "gemv", ng, b, 1))
    for k in range(2, p + 1):                                # Alg. 2, sequential
        ops.append(("seq", "gemv", b, b, 1))
        ops.append(("seq", "trsv", b, b, 1))
        if k < p:
            ops.append(("seq", "gemv", b, b, 1))
        if ng:
            ops.append(("seq", "gemv", ng, b, 1))
    if ng:
        ops.append(("seq", "gead", ng, 1, p))
        ops.append(("seq", "trsv", ng, ng, 1))
        ops.append(("seq", "trsv", ng, ng, 1))               # Alg. 3, hat R^{-T}
    for k in range(p, 1, -1):                                # Alg. 3, sequential
        if ng:
            ops.append(("seq", "gemv", b, ng, 1))
        if k < p:
            ops.append(("seq", "gemv", b, b, 1))
        ops.append(("seq", "trsv", b, b, 1))
    for k in range(1, p + 1):                                # Alg. 3, parallel
        ph = _phase(k, p)
        nk = seg_lens[k - 1]
        if k < p:
            ops.append((ph, "gemv", b, b, 1))
        for i in range(nk, 0, -1):
            if ng:
                ops.append((ph, "gemv", b, ng, 1))
            if k > 1:
                ops.append((ph, "gemv", b, b, 1))
            ops.append((ph, "trsv", b, b, 1))
            if i > 1:
                ops.append((ph, "gemv", b, b, 1))
    return ops


def cost(op, m, n, k):
    """Flops of one operation under the paper's counting convention."""
    if op == "potrf":
        return Fraction(n ** 3, 3)
    if op == "trsm":
        return Fraction(m * n * n)
    if op == "syrk":
        return Fraction(m * n * k) if m == n else Fraction(m * n * k)
    if op == "gemm":
        return Fraction(2 * m * n * k)
    if op == "trsv":
        return Fraction(n * n, 2)
    if op == "gemv":
        return Fraction(2 * m * n)
    if op == "gead":
        return Fraction(m * n * k)
    raise ValueError(op)


def std_cost(op, m, n, k):
    """Flops of one operation under standard counts (the plan's flop totals use
    these): potrf n^3/3, trsm m n^2, syrk n^2 k, gemm 2 m n k, trsv n^2, gemv 2 m n,
    gead m n k.  Only trsv differs from the paper's convention (n^2 / 2 there)."""
    if op == "trsv":
        return Fraction(n * n)
    return cost(op, m, n, k)


def phase_totals(ops):
    tot = {}
    for ph, op, m, n, k in ops:
        tot[ph] = tot.get(ph, Fraction(0)) + cost(op, m, n, k)
    return tot
