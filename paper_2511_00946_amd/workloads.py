"""Seeded synthetic KKT inputs shaped like the paper's workloads.

This module only draws inputs; it holds none of the solver's arithmetic.  Both
the oracle-side tests and the GPU path consume what it produces.

Recipe (FP64, numpy PCG64; for every system, in this order):
  1. M ~ N(0, 1) [N, b, b]       ->  D_i = M_i M_i^T + alpha I    (SPD, lambda_min >= alpha)
  2. C ~ N(0, s_C^2) [N-1, b, b]     sub-diagonal couplings Psi_{i+1,i}
  3. B ~ N(0, s_B^2) [N, ng, b]      arrow blocks Psi_{g,i}
  4. R ~ N(0, 1) [ng, ng]        ->  corner = R R^T + (ng + N) I
  5. r ~ N(0, 1) [N b + ng, nrhs]    right-hand side
  6. w ~ N(0, 1) [N b + ng, nrhs]    (differentiation workload only) weights of L = sum(w * x)
With alpha >= b and s_C, s_B ~ 0.05-0.1 the matrix is block diagonally dominant,
hence SPD with margin.

Workloads (the paper's chain-of-masses and Silverstone race-line data and its
comparison solvers are not available; these shapes stand in for them):
  small   N=16,   b=4,  ng=2, 1 rhs, alpha=4,  s_C=0.05, s_B=0.1   seed 1
  chain   N=128,  b=42, ng=0, 1 rhs, alpha=42, s_C=0.05            seed 2
  race    N=2048, b=6,  ng=8, 4 rhs, alpha=6,  s_C=0.05, s_B=0.05  seed 3
  batch   4096 systems, N ~ U{16..256}, b ~ U{8,16,32}, ng ~ U{0,2,4},
          alpha=b, s_C=s_B=0.05, 1 rhs                              seed 4
  diff    1024 x (N=64, b=24, ng=4), alpha=24, s_C=s_B=0.05, 1 rhs, plus w   seed 5
A batch draws every system's (N, b, ng) from the master generator first; each
system then draws its blocks from its own child generator
(``SeedSequence(seed).spawn``), so any one system can be regenerated alone.
"""
from dataclasses import dataclass, field

import numpy as np


@dataclass
class System:
    N: int
    b: int
    ng: int
    D: np.ndarray
    C: np.ndarray
    B: np.ndarray
    corner: np.ndarray
    r: np.ndarray
    w: np.ndarray = None

    @property
    def n(self):
        return self.N * self.b + self.ng

    @property
    def nrhs(self):
        return self.r.shape[1]


def draw_system(rng, N, b, ng, nrhs=1, alpha=None, s_C=0.05, s_B=0.05, with_w=False):
    """One system drawn from ``rng`` by the recipe above."""
    alpha = float(b if alpha is None else alpha)
    M = rng.standard_normal((N, b, b))
    D = np.matmul(M, np.swapaxes(M, 1, 2))
    D += alpha * np.eye(b)[None]
    C = s_C * rng.standard_normal((max(N - 1, 0), b, b))
    B = s_B * rng.standard_normal((N, ng, b))
    R = rng.standard_normal((ng, ng))
    corner = R @ R.T + (ng + N) * np.eye(ng)
    r = rng.standard_normal((N * b + ng, nrhs))
    w = rng.standard_normal((N * b + ng, nrhs)) if with_w else None
    return System(N, b, ng, D, C, B, corner, r, w)


SINGLE = {
    "small": dict(seed=1, N=16, b=4, ng=2, nrhs=1, alpha=4.0, s_C=0.05, s_B=0.1),
    "chain": dict(seed=2, N=128, b=42, ng=0, nrhs=1, alpha=42.0, s_C=0.05, s_B=0.05),
    "race": dict(seed=3, N=2048, b=6, ng=8, nrhs=4, alpha=6.0, s_C=0.05, s_B=0.05),
}


def single(name, **over):
    """One of the single-system workloads ('small', 'chain', 'race'); keyword overrides allowed."""
    cfg = dict(SINGLE[name])
    cfg.update(over)
    seed = cfg.pop("seed")
    return draw_system(np.random.default_rng(seed), **cfg)


@dataclass
class BatchSpec:
    """Dims of a batch and how to regenerate each system."""
    seed: int
    dims: list                     # [(N, b, ng)] per system
    nrhs: int = 1
    s_C: float = 0.05
    s_B: float = 0.05
    with_w: bool = False
    children: list = field(default_factory=list)

    def system(self, i):
        N, b, ng = self.dims[i]
        rng = np.random.default_rng(self.children[i])
        return draw_system(rng, N, b, ng, nrhs=self.nrhs, alpha=b, s_C=self.s_C,
                           s_B=self.s_B, with_w=self.with_w)

    def __len__(self):
        return len(self.dims)


def ragged_batch_spec(S=4096, seed=4, N_range=(16, 256), b_choices=(8, 16, 32),
                      ng_choices=(0, 2, 4), nrhs=1):
    """The ragged batching workload (default: 4096 systems)."""
    ss = np.random.SeedSequence(seed)
    master = np.random.default_rng(ss)
    Ns = master.integers(N_range[0], N_range[1] + 1, size=S)
    bs = master.choice(np.asarray(b_choices), size=S)
    gs = master.choice(np.asarray(ng_choices), size=S)
    dims = [(int(a), int(b), int(c)) for a, b, c in zip(Ns, bs, gs)]
    return BatchSpec(seed, dims, nrhs=nrhs, children=ss.spawn(S))


def uniform_batch_spec(S=1024, seed=5, N=64, b=24, ng=4, nrhs=1, with_w=True):
    """The differentiation workload (default: 1024 x (N=64, b=24, ng=4), with weights w)."""
    ss = np.random.SeedSequence(seed)
    np.random.default_rng(ss)   # keep the master stream consumed like the ragged case
    return BatchSpec(seed, [(N, b, ng)] * S, nrhs=nrhs, with_w=with_w, children=ss.spawn(S))


def pack(systems):
    """Concatenate systems into flat pools (D, C, B, corner, r[, w]), system after system.

    Pool layout per system s (FP64, row-major blocks): D [N, b, b], C [N-1, b, b],
    B [N, ng, b], corner [ng, ng], r [N b + ng, nrhs]."""
    cat = lambda xs: np.concatenate([np.ascontiguousarray(x).ravel() for x in xs]) if xs else np.zeros(0)
    pools = dict(D=cat([s.D for s in systems]), C=cat([s.C for s in systems]),
                 B=cat([s.B for s in systems]), corner=cat([s.corner for s in systems]),
                 r=cat([s.r for s in systems]))
    if systems and systems[0].w is not None:
        pools["w"] = cat([s.w for s in systems])
    return pools


@dataclass
class RaggedSystem:
    """A system with a size n_i per stage (lists of blocks)."""
    sizes: list
    ng: int
    D: list
    C: list
    B: list
    corner: np.ndarray
    r: np.ndarray


def draw_ragged_system(rng, sizes, ng, nrhs=1, s_C=0.05, s_B=0.05):
    """One non-uniform system by the recipe above, stage by stage (alpha = n_i)."""
    N = len(sizes)
    D = []
    for n in sizes:
        M = rng.standard_normal((n, n))
        D.append(M @ M.T + n * np.eye(n))
    C = [s_C * rng.standard_normal((sizes[i + 1], sizes[i])) for i in range(N - 1)]
    B = [s_B * rng.standard_normal((ng, n)) for n in sizes]
    R = rng.standard_normal((ng, ng))
    corner = R @ R.T + (ng + N) * np.eye(ng)
    r = rng.standard_normal((int(sum(sizes)) + ng, nrhs))
    return RaggedSystem(list(sizes), ng, D, C, B, corner, r)


def pack_ragged(systems):
    """Non-uniform pools, system after system (the layout of kkt_ragged_pad)."""
    cat = lambda xs: np.concatenate([np.ascontiguousarray(x, dtype=np.float64).ravel() for x in xs]) if xs else np.zeros(0)
    return dict(D=cat([d for s in systems for d in s.D]), C=cat([c for s in systems for c in s.C]),
                B=cat([b for s in systems for b in s.B]), corner=cat([s.corner for s in systems]),
                r=cat([s.r for s in systems]))


# ---------------------------------------------------------------- multistage QP data
@dataclass
class QPData:
    """A multistage QP (Sec. 2, Eq. 1) with N stages of size b, ng global
    variables, pe equality and me inequality rows per constraint group, and the
    positive inequality weights w of one interior-point iteration."""
    N: int
    b: int
    ng: int
    pe: int
    me: int
    arrays: dict


def draw_qp(rng, N, b, ng, pe, me, s=0.3):
    """S_i, T_i ~ N(0, s^2 / b); Q_i = M M^T / b + (1 + |S_{i-1}| + |S_i| + |T_i|) I and
    Qg = R R^T / ng + (1 + sum_i |T_i|) I (spectral norms: P is SPD by block
    Gershgorin, so the QP is strictly convex); constraint rows ~ N(0, s^2);
    weights w log-uniform in [0.1, 10]; drawn in this order (M, S, T, R, rows, w)."""
    M = rng.standard_normal((N, b, b))
    S = s / np.sqrt(b) * rng.standard_normal((max(N - 1, 0), b, b))
    T = s / np.sqrt(b) * rng.standard_normal((N, ng, b))
    R = rng.standard_normal((ng, ng))
    nS = np.array([np.linalg.norm(v, 2) for v in S]) if N > 1 else np.zeros(0)
    nT = np.array([np.linalg.norm(v, 2) if ng else 0.0 for v in T])
    margin = 1.0 + nT + np.concatenate([[0.0], nS]) + np.concatenate([nS, [0.0]])
    Q = np.matmul(M, np.swapaxes(M, 1, 2)) / b + margin[:, None, None] * np.eye(b)[None]
    Qg = R @ R.T / max(ng, 1) + (1.0 + float(np.sum(nT))) * np.eye(ng)
    EL = s * rng.standard_normal((N, pe, b))
    ER = s * rng.standard_normal((max(N - 1, 0), pe, b))
    EG = s * rng.standard_normal((N, pe, ng))
    IL = s * rng.standard_normal((N, me, b))
    IR = s * rng.standard_normal((max(N - 1, 0), me, b))
    IG = s * rng.standard_normal((N, me, ng))
    w = np.exp(rng.uniform(np.log(0.1), np.log(10.0), size=(N, me)))
    return QPData(N, b, ng, pe, me, dict(Q=Q, S=S, T=T, Qg=Qg, EL=EL, ER=ER, EG=EG, IL=IL, IR=IR, IG=IG, w=w))


def pack_qp(qps):
    """QP pools of a batch (system after system, the layouts of the plan and of
    kkt_qp): Q, S, T, Qg, EL, ER, EG, IL, IR, IG, w as flat float64 arrays."""
    out = {}
    for k in ("Q", "S", "T", "Qg", "EL", "ER", "EG", "IL", "IR", "IG", "w"):
        out[k] = np.concatenate([np.asarray(q.arrays[k], dtype=np.float64).reshape(-1) for q in qps])
    return out


def draw_qp_problem(rng, N, b, ng, pe, me, s=0.3):
    """A feasible multistage QP: the data of draw_qp, then c ~ N(0, 1), a point
    x_f ~ N(0, 1) and slacks u ~ U(0.5, 1.5) with beq = A x_f and h = G x_f + u
    (stage by stage, g last; the rows of each constraint group in turn)."""
    q = draw_qp(rng, N, b, ng, pe, me, s)
    a = q.arrays
    n = N * b + ng
    c = rng.standard_normal(n)
    xf = rng.standard_normal(n)
    u = rng.uniform(0.5, 1.5, size=N * me)
    xs, xg = xf[:N * b].reshape(N, b), xf[N * b:]
    beq = np.zeros(N * pe)
    h = np.zeros(N * me)
    for k in range(N):
        e = a["EL"][k] @ xs[k] + (a["ER"][k] @ xs[k + 1] if k < N - 1 else 0.0) + (a["EG"][k] @ xg if ng else 0.0)
        g = a["IL"][k] @ xs[k] + (a["IR"][k] @ xs[k + 1] if k < N - 1 else 0.0) + (a["IG"][k] @ xg if ng else 0.0)
        beq[k * pe:(k + 1) * pe] = e
        h[k * me:(k + 1) * me] = g + u[k * me:(k + 1) * me]
    return q, c, beq, h
