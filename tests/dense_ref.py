"""Dense references written independently of ``oracle/``: assemble Psi as one dense
matrix, build the permutation of Sec. 3.1 directly, and let LAPACK (numpy) factor
and solve.  Used to pin the oracle on tiny inputs."""
import numpy as np


def assemble(D, C, B, corner):
    """Dense Psi (Eq. 3) with K_ii = (D_i + D_i^T)/2, K_{i+1,i} = C_i, K_{g,i} = B_i."""
    N, b = D.shape[0], D.shape[1]
    ng = 0 if B is None else B.shape[1]
    n = N * b + ng
    K = np.zeros((n, n))
    for i in range(N):
        K[i * b:(i + 1) * b, i * b:(i + 1) * b] = 0.5 * (D[i] + D[i].T)
    for i in range(N - 1):
        K[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = C[i]
        K[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = C[i].T
    if ng:
        for i in range(N):
            K[N * b:, i * b:(i + 1) * b] = B[i]
            K[i * b:(i + 1) * b, N * b:] = B[i].T
        K[N * b:, N * b:] = 0.5 * (corner + corner.T)
    return K


def permuted_stage_order(seg_lens):
    """Segments' stages first, then the separators between consecutive segments."""
    stages, seps, s = [], [], 0
    for k, nk in enumerate(seg_lens):
        if k:
            seps.append(s)
            s += 1
        stages.extend(range(s, s + nk))
        s += nk
    return stages + seps


def scalar_permutation(seg_lens, b, ng):
    order = permuted_stage_order(seg_lens)
    idx = [s * b + t for s in order for t in range(b)]
    N = len(order)
    idx += [N * b + t for t in range(ng)]
    return np.asarray(idx)


def dense_factor(K, perm):
    """numpy (LAPACK) Cholesky of P K P^T."""
    return np.linalg.cholesky(K[np.ix_(perm, perm)])


def nested_stage_order(N, levels):
    """Recursive segmentation, written as a recursion over the chain: the stages
    inside the segments of levels[0], then the same rule applied to the chain of
    the separators with levels[1:], the last separators at the end."""
    def rec(chain, lv):
        if not lv:
            return list(chain)
        inner, seps, pos = [], [], 0
        for k, nk in enumerate(lv[0]):
            if k:
                seps.append(chain[pos])
                pos += 1
            inner.extend(chain[pos:pos + nk])
            pos += nk
        assert pos == len(chain), "segment lengths do not tile the chain"
        return inner + rec(seps, lv[1:])
    return rec(list(range(N)), list(levels))


def nested_scalar_permutation(N, levels, b, ng):
    order = nested_stage_order(N, levels)
    return np.asarray([s * b + t for s in order for t in range(b)] + [N * b + t for t in range(ng)])
