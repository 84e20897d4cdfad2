"""Oracle for the block-tridiagonal-arrow KKT system -- test infrastructure only.

Notation (paper, Eq. 3, 1-based there, 0-based here):
  D[i]   = Psi_{i,i}    (b x b, SPD; the matrix uses sym(D[i]) = (D[i] + D[i]^T)/2)
  C[i]   = Psi_{i+1,i}  (b x b, i = 0..N-2; Psi_{i,i+1} = C[i]^T)
  B[i]   = Psi_{g,i}    (ng x b, the arrow; Psi_{i,g} = B[i]^T)
  corner = Psi_{g,g}    (ng x ng, SPD; the matrix uses sym(corner))
  r                     (N*b + ng) x nrhs right-hand side, stages first, g last.

Segmentation (Sec. 3.1): with segment lengths N_1..N_p, segment k holds N_k
consecutive stages and a single separator stage sits between segment k-1 and
segment k, so N = sum_k N_k + p - 1.  The permutation P of Sec. 3.1 (Fig. 1b)
lists the segment stages first (segment 1, then 2, ...), then the separators
(of segments 2..p, in order), then g.  The factor of P Psi P^T is unique
(positive diagonal), so it is computed here by plain block Cholesky in that order
(``blockchol``); p = 1 is the sequential method the paper compares against
(Sec. 3.3, O_seq).

Recursive segmentation (the multi-level method that Sec. 5 names as future
work): the separators' reduced system is again a block-tridiagonal arrow chain
(``reduced_system``), so it is segmented in turn; ``nested_order`` gives the
resulting elimination order and ``KKTFactor(..., nest=...)`` its unique factor.

Readings where the paper is silent:
  * failure: ``info`` is the 1-based natural stage index of the first diagonal
    block, in elimination order, whose pivot is not positive and finite; N + 1
    names the corner.  The paper does not discuss indefinite input.
  * symmetric parametrisation: the matrix uses sym(D[i]) and sym(corner); C[i]
    and B[i] each appear twice.  This fixes the gradient of the adjoint.
"""
import numpy as np

from .blockchol import BlockMatrix


def sym(a):
    return 0.5 * (a + np.swapaxes(a, -1, -2))


def stage_layout(N, seg_lens):
    """Natural 0-based stage indices of every segment, and of the separators.

    Returns (segments, separators): segments[k] is the list of stages of segment
    k+1; separators[k-2] is the separator stage between segments k-1 and k
    (k = 2..p, paper's 1-based k)."""
    seg_lens = [int(v) for v in seg_lens]
    p = len(seg_lens)
    if p < 1 or min(seg_lens) < 1 or sum(seg_lens) + p - 1 != N:
        raise ValueError("segment lengths %s do not tile N=%d" % (seg_lens, N))
    segments, separators = [], []
    s = 0
    for k, nk in enumerate(seg_lens):
        if k > 0:
            separators.append(s)
            s += 1
        segments.append(list(range(s, s + nk)))
        s += nk
    return segments, separators


def elimination_order(N, seg_lens):
    """Stage order of P Psi P^T: all segment stages, then the separators (g is last)."""
    segments, separators = stage_layout(N, seg_lens)
    return [i for seg in segments for i in seg] + separators


def nested_order(N, levels):
    """Stage order of recursive (multi-level) segmentation.

    Sec. 3.1's permutation eliminates the segment stages first and leaves the
    separators, whose reduced system (Eqs. 8, 9) is again block tridiagonal with
    the same arrow.  Segmenting that chain the same way, and so on, is the
    multi-level method that Sec. 5 names as future work.  ``levels[0]`` are the
    segment lengths of the whole chain, ``levels[1]`` those of the chain of its
    p - 1 separators (taken in natural order), and so on; the separators left by
    the last level close the order (g is last).  One level gives
    ``elimination_order``."""
    chain = list(range(N))
    order = []
    for seg_lens in levels:
        segments, separators = stage_layout(len(chain), seg_lens)
        order += [chain[i] for seg in segments for i in seg]
        chain = [chain[j] for j in separators]
    return order + chain


def reduced_system(D, C, B, corner, seg_lens, r=None):
    """The system left on the separators and g once the segment stages of
    ``seg_lens`` are eliminated (Sec. 3.2, Eqs. 8, 9), from its definition: the
    Schur complement S = Psi_SS - Psi_SI Psi_II^{-1} Psi_IS of the assembled matrix
    (I: segment stages, S: separators in natural order, then g) and the reduced
    rhs r_S - Psi_SI Psi_II^{-1} r_I.

    Returned as block arrays of a system with p - 1 stages:
    (D', C', B', corner', r') with D'_j = S_jj, C'_j = S_{j+1,j}, B'_j = S_gj,
    corner' = S_gg (r' is None without r)."""
    D = np.asarray(D, dtype=np.float64)
    N, b, ng = _dims(D, B)
    segments, separators = stage_layout(N, seg_lens)
    if not separators:
        raise ValueError("one segment leaves no reduced system")
    n = N * b + ng
    K = np.zeros((n, n))
    Cm = np.asarray(C, dtype=np.float64).reshape(-1, b, b)
    for i in range(N):
        K[i * b:(i + 1) * b, i * b:(i + 1) * b] = sym(D[i])
    for i in range(N - 1):
        K[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = Cm[i]
        K[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = Cm[i].T
    if ng:
        Bm = np.asarray(B, dtype=np.float64)
        for i in range(N):
            K[N * b:, i * b:(i + 1) * b] = Bm[i]
            K[i * b:(i + 1) * b, N * b:] = Bm[i].T
        K[N * b:, N * b:] = sym(np.asarray(corner, dtype=np.float64))
    I = [s * b + t for seg in segments for s in seg for t in range(b)]
    S = [s * b + t for s in separators for t in range(b)] + [N * b + t for t in range(ng)]
    KII, KSI = K[np.ix_(I, I)], K[np.ix_(S, I)]
    Smat = K[np.ix_(S, S)] - KSI @ np.linalg.solve(KII, KSI.T)
    M = len(separators)
    Dr = np.stack([Smat[j * b:(j + 1) * b, j * b:(j + 1) * b] for j in range(M)])
    Cr = np.stack([Smat[(j + 1) * b:(j + 2) * b, j * b:(j + 1) * b] for j in range(M - 1)]) \
        if M > 1 else np.zeros((0, b, b))
    Br = np.stack([Smat[M * b:, j * b:(j + 1) * b] for j in range(M)]) if ng else None
    cr = Smat[M * b:, M * b:] if ng else None
    rr = None
    if r is not None:
        R = np.asarray(r, dtype=np.float64)
        rr = R[S] - KSI @ np.linalg.solve(KII, R[I])
    return Dr, Cr, Br, cr, rr


def _dims(D, B):
    D = np.asarray(D)
    N, b = D.shape[0], D.shape[1]
    ng = 0 if B is None else int(np.asarray(B).shape[1])
    return N, b, ng


class KKTFactor:
    """hat L = chol(P Psi P^T) for the order given by ``seg_lens`` (default: p = 1);
    ``nest``: segment lengths of the reduced chain at each deeper level
    (``nested_order``), None for the single-level method."""

    def __init__(self, D, C, B, corner, seg_lens=None, factor=True, nest=None):
        D = np.asarray(D, dtype=np.float64)
        C = np.asarray(C, dtype=np.float64).reshape(-1, D.shape[1], D.shape[1])
        N, b, ng = _dims(D, B)
        if seg_lens is None:
            seg_lens = [N]
        self.N, self.b, self.ng = N, b, ng
        self.seg_lens = list(seg_lens)
        self.nest = [list(v) for v in (nest or [])]
        self.order = nested_order(N, [self.seg_lens] + self.nest)
        self.pos = {s: i for i, s in enumerate(self.order)}
        if ng:
            self.pos["g"] = N
        sizes = [b] * N + ([ng] if ng else [])
        M = BlockMatrix(sizes)
        for s in range(N):
            M.set(self.pos[s], self.pos[s], sym(D[s]))
        for s in range(N - 1):
            i, j = self.pos[s + 1], self.pos[s]
            if i > j:
                M.set(i, j, C[s])
            else:
                M.set(j, i, C[s].T)
        if ng:
            B = np.asarray(B, dtype=np.float64)
            for s in range(N):
                M.set(N, self.pos[s], B[s])
            M.set(N, N, sym(np.asarray(corner, dtype=np.float64)))
        self._M = M
        self.info = None
        if factor:
            self.factor()

    def factor(self):
        """Block Cholesky of the assembled P Psi P^T (in place); sets ``info``.
        Separate from the assembly so that a caller can time the C core alone."""
        rc = self._M.cholesky()
        if rc < 0:
            raise RuntimeError("oracle block Cholesky failed on its input")
        if rc == 0:
            self.info = 0
        else:
            col = rc - 1
            self.info = self.order[col] + 1 if col < self.N else self.N + 1

    def block(self, row, col):
        """hat L block at (row stage, col stage), natural labels (ints or 'g').

        Returns None for a structural zero.  Requires row to follow col in the
        elimination order."""
        i, j = self.pos[row], self.pos[col]
        if i < j:
            raise ValueError("(%r, %r) lies above the diagonal of hat L" % (row, col))
        return self._M.get(i, j)

    def _to_perm(self, r):
        N, b, ng = self.N, self.b, self.ng
        r = np.asarray(r, dtype=np.float64)
        rs = r[: N * b].reshape(N, b, *r.shape[1:])
        parts = [rs[s] for s in self.order]
        if ng:
            parts.append(r[N * b:])
        return np.concatenate(parts, axis=0)

    def _from_perm(self, xp):
        N, b = self.N, self.b
        x = np.empty_like(xp)
        for i, s in enumerate(self.order):
            x[s * b:(s + 1) * b] = xp[i * b:(i + 1) * b]
        x[N * b:] = xp[N * b:]
        return x

    def solve(self, r):
        """x with Psi x = r (natural order, any number of columns)."""
        if self.info:
            raise FloatingPointError("matrix is not positive definite (info=%d)" % self.info)
        return self._from_perm(self._M.solve(self._to_perm(r)))

    def logdet(self):
        """log det Psi = 2 * sum log diag(hat L); identical for every block order."""
        tot = 0.0
        keys = list(range(self.N)) + (["g"] if self.ng else [])
        for s in keys:
            tot += 2.0 * np.sum(np.log(np.diag(self.block(s, s))))
        return float(tot)


def solve(D, C, B, corner, r, seg_lens=None, nest=None):
    return KKTFactor(D, C, B, corner, seg_lens, nest=nest).solve(r)


def matvec(D, C, B, corner, x):
    """Psi x with the symmetric parametrisation (block form, natural order)."""
    D = np.asarray(D, dtype=np.float64)
    N, b, ng = _dims(D, B)
    x = np.asarray(x, dtype=np.float64)
    one = x.ndim == 1
    X = x[:, None] if one else x
    xs = X[: N * b].reshape(N, b, -1)
    ys = np.einsum("irc,icq->irq", sym(D), xs)
    if N > 1:
        C = np.asarray(C, dtype=np.float64).reshape(N - 1, b, b)
        ys[1:] += np.einsum("irc,icq->irq", C, xs[:-1])
        ys[:-1] += np.einsum("icr,icq->irq", C, xs[1:])
    out = [ys.reshape(N * b, -1)]
    if ng:
        B = np.asarray(B, dtype=np.float64)
        xg = X[N * b:]
        ys2 = ys + np.einsum("iqr,qk->irk", B, xg)
        out = [ys2.reshape(N * b, -1)]
        yg = np.einsum("iqc,ick->qk", B, xs) + sym(np.asarray(corner, dtype=np.float64)) @ xg
        out.append(yg)
    y = np.concatenate(out, axis=0)
    return y[:, 0] if one else y


def rel_residual(D, C, B, corner, x, r):
    """max over rhs columns of ||Psi x - r||_2 / ||r||_2."""
    res = matvec(D, C, B, corner, x) - np.asarray(r, dtype=np.float64)
    R = np.asarray(r, dtype=np.float64)
    if res.ndim == 1:
        res, R = res[:, None], R[:, None]
    return float(np.max(np.linalg.norm(res, axis=0) / np.maximum(np.linalg.norm(R, axis=0), 1e-300)))


def adjoint(D, C, B, corner, x, gbar, seg_lens=None):
    """Gradients of L = <gbar, x> where Psi x = r (x given, gbar = dL/dx).

    lambda = Psi^{-1} gbar (Psi symmetric), dL/dPsi = -lambda x^T summed over the
    rhs columns, then pulled back through the parametrisation Psi(D, C, B, corner):
      dD[i]   = -sym(lambda_i x_i^T)
      dC[i]   = -(lambda_{i+1} x_i^T + x_{i+1} lambda_i^T)
      dB[i]   = -(lambda_g x_i^T + x_g lambda_i^T)
      dcorner = -sym(lambda_g x_g^T)
      dr      = lambda
    Returns (lambda, dD, dC, dB, dcorner)."""
    D = np.asarray(D, dtype=np.float64)
    N, b, ng = _dims(D, B)
    lam = solve(D, C, B, corner, gbar, seg_lens)
    X = np.asarray(x, dtype=np.float64)
    Lm = lam
    if X.ndim == 1:
        X, Lm = X[:, None], lam[:, None]
    xs = X[: N * b].reshape(N, b, -1)
    ls = Lm[: N * b].reshape(N, b, -1)
    dD = -sym(np.einsum("irq,icq->irc", ls, xs))
    dC = -(np.einsum("irq,icq->irc", ls[1:], xs[:-1]) + np.einsum("irq,icq->irc", xs[1:], ls[:-1]))
    if ng:
        xg, lg = X[N * b:], Lm[N * b:]
        dB = -(np.einsum("rq,icq->irc", lg, xs) + np.einsum("rq,icq->irc", xg, ls))
        dcorner = -sym(lg @ xg.T)
    else:
        dB = np.zeros((N, 0, b))
        dcorner = np.zeros((0, 0))
    return lam, dD, dC, dB, dcorner


# ---------------------------------------------------------------- non-uniform stage sizes
# Sec. 2 (Eqs. 1, 3) lets stage i carry its own size n_i: D[i] is n_i x n_i,
# C[i] = Psi_{i+1,i} is n_{i+1} x n_i, B[i] is ng x n_i, r stacks the stage parts
# (n_0 + ... + n_{N-1}) and then g.  The solution has a plain definition, so the
# oracle is the block Cholesky of the natural-order matrix with those block sizes.


def ragged_offsets(sizes):
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def solve_ragged(D, C, B, corner, r):
    """x with Psi x = r for lists of blocks with per-stage sizes (natural order)."""
    N = len(D)
    sizes = [int(np.asarray(d).shape[0]) for d in D]
    ng = 0 if corner is None else int(np.asarray(corner).shape[0])
    M = BlockMatrix(sizes + ([ng] if ng else []))
    for i in range(N):
        M.set(i, i, sym(np.asarray(D[i], dtype=np.float64)))
    for i in range(N - 1):
        M.set(i + 1, i, np.asarray(C[i], dtype=np.float64))
    if ng:
        for i in range(N):
            M.set(N, i, np.asarray(B[i], dtype=np.float64))
        M.set(N, N, sym(np.asarray(corner, dtype=np.float64)))
    rc = M.cholesky()
    if rc != 0:
        raise FloatingPointError("matrix is not positive definite (block %d)" % rc)
    return M.solve(np.asarray(r, dtype=np.float64))


def matvec_ragged(D, C, B, corner, x):
    """Psi x for lists of blocks with per-stage sizes (symmetric parametrisation)."""
    N = len(D)
    sizes = [int(np.asarray(d).shape[0]) for d in D]
    off = ragged_offsets(sizes)
    ng = 0 if corner is None else int(np.asarray(corner).shape[0])
    x = np.asarray(x, dtype=np.float64)
    X = x[:, None] if x.ndim == 1 else x
    Y = np.zeros_like(X)
    for i in range(N):
        Y[off[i]:off[i + 1]] += sym(np.asarray(D[i])) @ X[off[i]:off[i + 1]]
        if i + 1 < N:
            Ci = np.asarray(C[i])
            Y[off[i + 1]:off[i + 2]] += Ci @ X[off[i]:off[i + 1]]
            Y[off[i]:off[i + 1]] += Ci.T @ X[off[i + 1]:off[i + 2]]
        if ng:
            Bi = np.asarray(B[i])
            Y[off[i]:off[i + 1]] += Bi.T @ X[off[N]:]
            Y[off[N]:] += Bi @ X[off[i]:off[i + 1]]
    if ng:
        Y[off[N]:] += sym(np.asarray(corner)) @ X[off[N]:]
    return Y[:, 0] if x.ndim == 1 else Y
