"""Segment lengths (Eq. 13) and the complexity model of Sec. 3.3 -- test infrastructure only.

The flop balance of Table 1 (n_g = 0) between the first segment, (7/3 N_1 - 1) b^3,
and any other segment, (19/3 N_k - 1) b^3, gives sigma = N_1 / N_k = 19/7.  The
other segments all get the same length N_k, rounded from the ideal value

    bar N_k* = (N - p + 1) / (p - 1 + sigma)

to whichever of floor / ceil gives the smaller max{7/3 N_1, 19/3 N_k}, with
N_1 = N - (p - 1) - (p - 1) N_k (Eq. 13: N_1 + (p-1) N_k + p - 1 = N).

Readings (the paper is garbled or silent here):
  * the denominator is (p - 1 + sigma).  The printed (p + sigma) does not give the
    numbers of Table 2; (p - 1 + sigma) follows from N_1 = sigma N_k and
    N_1 + (p-1) N_k = N - p + 1, and reproduces Table 2.
  * equal maxima pick floor (the longer first segment).
  * production mode requires N_1 >= 1 and N_k >= 1, i.e. N >= 2p - 1.  The
    "paper table" mode does not reject a candidate with N_1 < 1; Table 2 was
    evidently computed that way (its p = 14, 16 entries of the N_{gamma=2} row).

Complexities (Sec. 3.3):
    O_par(N; p) = (max{7/3 N_1*, 19/3 N_k*} + 10/3 p - 19/3) b^3
    O_seq(N)    = (7/3 N - 2) b^3
    gamma       = O_seq / O_par
"""
import math
from fractions import Fraction

SIGMA = Fraction(19, 7)


def segment_lengths(N, p, sigma=SIGMA, paper_table=False):
    """(N_1, N_k) of Eq. (13).  p = 1 returns (N, 0)."""
    N, p = int(N), int(p)
    if p < 1:
        raise ValueError("p must be >= 1")
    if p == 1:
        return N, 0
    sigma = Fraction(sigma)
    nbar = Fraction(N - p + 1) / (p - 1 + sigma)
    best = None
    for nk in (math.floor(nbar), math.ceil(nbar)):
        n1 = N - (p - 1) - (p - 1) * nk
        if nk < 1:
            continue
        if not paper_table and n1 < 1:
            continue
        cost = max(Fraction(7, 3) * n1, Fraction(19, 3) * nk)
        if best is None or cost < best[0]:
            best = (cost, n1, nk)
    if best is None:
        raise ValueError("no feasible partition of N=%d into p=%d segments (needs N >= 2p-1)" % (N, p))
    return best[1], best[2]


def seg_lens(N, p, **kw):
    """[N_1, N_k, ..., N_k] (p entries)."""
    n1, nk = segment_lengths(N, p, **kw)
    return [n1] + [nk] * (p - 1)


def o_seq(N):
    return Fraction(7, 3) * N - 2


def o_par(N, p, paper_table=False):
    n1, nk = segment_lengths(N, p, paper_table=paper_table)
    return max(Fraction(7, 3) * n1, Fraction(19, 3) * nk) + Fraction(10, 3) * p - Fraction(19, 3)


def gamma(N, p, paper_table=False):
    return o_seq(N) / o_par(N, p, paper_table=paper_table)


def gamma_max(p):
    """lim_{N -> inf} gamma(N; p) = 7 (p - 1 + sigma) / 19 = 1 + 7 (p - 1) / 19."""
    return 1 + Fraction(7 * (p - 1), 19)


def first_horizon(p, threshold, n_max=20000, paper_table=True):
    """Smallest N >= 2p with gamma(N; p) >= threshold, or None (first crossing)."""
    for N in range(2 * p, n_max):
        if gamma(N, p, paper_table=paper_table) >= threshold:
            return N
    return None
