"""Oracle for assembling the KKT matrix of a multistage QP -- test infrastructure only.

The problem is the multistage QP of Sec. 2, Eq. 1: stages x_0 .. x_{N-1} (N
diagonal blocks, the last one the terminal stage), a global variable g, a cost
that couples x_i with x_{i+1} and g, and N groups of equality and inequality
constraints: group k < N-1 couples x_k, x_{k+1} and g, group N-1 (the terminal
one) couples x_{N-1} and g.  Names (0-based; the paper's symbols in brackets):

  Q[i]  (b x b)   Hessian block of x_i               [Q_i, the terminal Q_N at N-1]
  S[i]  (b x b)   Hessian block (x_{i+1}, x_i)       [S_i], i < N-1
  T[i]  (ng x b)  Hessian block (g, x_i)             [T_i, T_N at N-1]
  Qg    (ng x ng) Hessian block of g                 [Q_g]
  EL[k] (pe x b)  equality rows of group k on x_k       [A_k; A_N for the terminal group]
  ER[k] (pe x b)  equality rows of group k on x_{k+1}   [B_k], k < N-1
  EG[k] (pe x ng) equality rows of group k on g         [E_k]
  IL[k] (me x b)  inequality rows on x_k                [C_k; D_N for the terminal group]
  IR[k] (me x b)  inequality rows on x_{k+1}            [D_k], k < N-1
  IG[k] (me x ng) inequality rows on g                  [F_k]
  w[k]  (me)      positive weights of the inequality rows

The paper takes Psi from the solver (PIQP) without deriving it.  The reading
used here is the proximal interior-point Newton system
    [ H   A^T   G^T  ] [dx]   [rx]
    [ A  -d I    0   ] [dy] = [ry]        H = P + rho I,  d = delta > 0,
    [ G    0   -W^-1 ] [dz]   [rz]        W = diag(w) > 0,
whose block elimination of dy = (A dx - ry) / d and dz = W (G dx - rz) gives
    Psi dx = rx + A^T ry / d + G^T W rz,   Psi = P + rho I + A^T A / d + G^T W G,
an SPD matrix with the block-tridiagonal-arrow pattern of Eq. 3 (P is the
Hessian of the cost, A and G the stacked constraint rows).  Every function here
builds the dense matrices and applies these definitions literally.
"""
import numpy as np


def _sizes(Q, T, EL, IL):
    Q = np.asarray(Q)
    N, b = Q.shape[0], Q.shape[1]
    ng = 0 if T is None else int(np.asarray(T).shape[1])
    pe = int(np.asarray(EL).shape[1])
    me = int(np.asarray(IL).shape[1])
    return N, b, ng, pe, me


def dense_parts(qp):
    """Dense P (n x n), A (N pe x n) and G (N me x n), n = N b + ng, natural order
    (stages first, g last)."""
    N, b, ng, pe, me = _sizes(qp["Q"], qp["T"], qp["EL"], qp["IL"])
    n = N * b + ng
    P = np.zeros((n, n))
    for i in range(N):
        P[i * b:(i + 1) * b, i * b:(i + 1) * b] = qp["Q"][i]
        if ng:
            P[N * b:, i * b:(i + 1) * b] = qp["T"][i]
            P[i * b:(i + 1) * b, N * b:] = qp["T"][i].T
    for i in range(N - 1):
        P[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] = qp["S"][i]
        P[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] = qp["S"][i].T
    if ng:
        P[N * b:, N * b:] = qp["Qg"]
    A = np.zeros((N * pe, n))
    G = np.zeros((N * me, n))
    for k in range(N):
        A[k * pe:(k + 1) * pe, k * b:(k + 1) * b] = qp["EL"][k]
        G[k * me:(k + 1) * me, k * b:(k + 1) * b] = qp["IL"][k]
        if k < N - 1:
            A[k * pe:(k + 1) * pe, (k + 1) * b:(k + 2) * b] = qp["ER"][k]
            G[k * me:(k + 1) * me, (k + 1) * b:(k + 2) * b] = qp["IR"][k]
        if ng:
            A[k * pe:(k + 1) * pe, N * b:] = qp["EG"][k]
            G[k * me:(k + 1) * me, N * b:] = qp["IG"][k]
    return P, A, G


def assemble(qp, rho, delta):
    """Psi = P + rho I + A^T A / delta + G^T W G as block arrays (D, C, B, corner):
    D[i] = Psi_{i,i}, C[i] = Psi_{i+1,i}, B[i] = Psi_{g,i}, corner = Psi_{g,g}; also
    returns the dense Psi."""
    N, b, ng, pe, me = _sizes(qp["Q"], qp["T"], qp["EL"], qp["IL"])
    P, A, G = dense_parts(qp)
    w = np.asarray(qp["w"], dtype=np.float64).reshape(-1)
    Psi = P + rho * np.eye(P.shape[0]) + A.T @ A / delta + G.T @ (w[:, None] * G)
    D = np.stack([Psi[i * b:(i + 1) * b, i * b:(i + 1) * b] for i in range(N)])
    C = np.stack([Psi[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] for i in range(N - 1)]) \
        if N > 1 else np.zeros((0, b, b))
    B = np.stack([Psi[N * b:, i * b:(i + 1) * b] for i in range(N)]) if ng else np.zeros((N, 0, b))
    corner = Psi[N * b:, N * b:] if ng else np.zeros((0, 0))
    return D, C, B, corner, Psi


def reduce_rhs(qp, delta, rx, ry, rz):
    """rx + A^T ry / delta + G^T W rz (columns are right-hand sides)."""
    _, A, G = dense_parts(qp)
    w = np.asarray(qp["w"], dtype=np.float64).reshape(-1)
    return np.asarray(rx) + A.T @ np.asarray(ry) / delta + G.T @ (w[:, None] * np.asarray(rz))


def recover(qp, delta, dx, ry, rz):
    """dy = (A dx - ry) / delta, dz = W (G dx - rz)."""
    _, A, G = dense_parts(qp)
    w = np.asarray(qp["w"], dtype=np.float64).reshape(-1)
    dy = (A @ np.asarray(dx) - np.asarray(ry)) / delta
    dz = w[:, None] * (G @ np.asarray(dx) - np.asarray(rz))
    return dy, dz


def newton_step_full(qp, rho, delta, rx, ry, rz):
    """The unreduced saddle-point system solved as one dense matrix (LAPACK)."""
    P, A, G = dense_parts(qp)
    w = np.asarray(qp["w"], dtype=np.float64).reshape(-1)
    n, ma, mg = P.shape[0], A.shape[0], G.shape[0]
    K = np.zeros((n + ma + mg, n + ma + mg))
    K[:n, :n] = P + rho * np.eye(n)
    K[:n, n:n + ma] = A.T
    K[:n, n + ma:] = G.T
    K[n:n + ma, :n] = A
    K[n:n + ma, n:n + ma] = -delta * np.eye(ma)
    K[n + ma:, :n] = G
    K[n + ma:, n + ma:] = -np.diag(1.0 / w)
    rhs = np.concatenate([np.asarray(rx), np.asarray(ry), np.asarray(rz)], axis=0)
    sol = np.linalg.solve(K, rhs)
    return sol[:n], sol[n:n + ma], sol[n + ma:]
