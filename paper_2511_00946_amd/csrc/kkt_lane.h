// Single-wave row-lane stage sweeps for padded block sizes 8 and 16 (gfx950, FP64).
//
// One 64-lane wave per work item (a segment, a whole system, or the reduced
// separator chain).  Lane t holds row t of the panel of a stage:
//   [0, BP)                D rows  the working diagonal block (its factor after the step)
//   [BP, 2 BP)             E rows  the coupling rows to the next pivot
//   [2 BP, 2 BP + 16)      G rows  the arrow rows
//   [2 BP + 16, 3 BP + 16) F rows  the separator fill rows of a segment k >= 2
// and, with a forward substitution, its right-hand-side entries as extra columns.
//
// Factor sweep, per stage:
//   1. elimination (Algorithm 1: potrf of the diagonal block and the trsm of the
//      panel rows; Algorithm 2 fused): for each column c the pivot row is
//      broadcast from lane c with readlane (by symmetry, row c right of the pivot
//      is column c below it) and every lane below the pivot updates its row and
//      its right-hand sides with one FMA per entry.  No LDS traffic, no selects.
//   2. the rows go to LDS; the Gram of the E, G, F rows (Eqs. 4, 6, 8a, 8b) runs on
//      the FP64 matrix cores as the lower 16 x 16 tiles of -[E; G; F][E; G; F]^T:
//      the tiles of the E columns start from the next stage's blocks (next D, G and
//      F rows), the others from running sums held in registers through the sweep
//      (G G^T -> hat R_k, F G^T -> hat Q_k^T, F F^T -> hat A_k).
// Memory: when a stage starts it issues the stores of the previous stage's
// outputs (from LDS) and the loads of the next stage's blocks together, and waits
// for them only at its end, where the blocks go to LDS: loads and stores share one
// counter, so a wait for a load with a younger store pending waits for every
// memory operation.  Blocks move as lane-contiguous elements through range-checked
// buffer accesses (past a block a load reads zero and a store is dropped).
//
// Forward sweep (solve modes): the same lane layout with the factor rows staged
// from HBM.  Backward sweep: lane c owns column c of the stage's blocks (staged
// through LDS) and the back substitution broadcasts x_c with readlane.
//
// Right-hand sides: the instance count NR (1, 4 or 8) covers nr <= NR; the
// columns past nr hold zeros.
#pragma once
#include "kkt_wave.h"

namespace kkt_dev {

__host__ __device__ constexpr int nr_class(int nr) { return nr <= 1 ? 1 : (nr <= 4 ? 4 : 8); }

template <int BP>
struct LC {
    static constexpr int N2 = 2 * BP + NGM;         // Gram rows: E, G, F
    static constexpr int T2 = N2 / 16;              // 16-row tiles of the Gram
    static constexpr int KS = BP / 4;               // k-steps of 4 columns
    static constexpr int NTL = T2 * (T2 + 1) / 2;   // lower tiles
    static constexpr int NROW = 3 * BP + NGM;       // panel rows (lane t holds row t)
    static constexpr int F0 = BP + NGM;             // Gram coordinate of the first F row
    static constexpr int MB = BP * BP / 64;         // elements per lane of a b x b block
    static constexpr int MG = NGM * BP / 64;        // ... of an ng x b block
    static constexpr int MY = 2;                    // ... of b x nr rhs rows
    static_assert(BP == 8 || BP == 16, "single-wave sweeps cover padded sizes 8 and 16");
    static_assert(NROW <= 64 && N2 % 16 == 0, "row placement");
    static_assert(BP * MAX_NRHS_DEV <= 64 * MY, "rhs rows");
    static_assert(WC<BP>::NW == 1 && WC<BP>::TE == BP && WC<BP>::TG == 2 * BP && WC<BP>::TF == 2 * BP + NGM,
                  "lane t holds panel row t");
};

// Lane-contiguous elements e = t + 64 m of a row-major block with `cols` columns:
// row er, column ec, and the LDS offset (pitch P) of that entry with the row
// clamped to 15 (an element past the block then still reads inside the LDS areas).
template <int M>
struct Elems {
    int er[M], ec[M], lo[M];
    __device__ __forceinline__ void init(int t, int cols, int P)
    {
        const float inv = 1.0f / (float)cols;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            rc_of(t + 64 * m, cols, inv, er[m], ec[m]);
            lo[m] = (er[m] < NGM ? er[m] : NGM - 1) * P + ec[m];
        }
    }
};

// A block of n elements from LDS (offsets in the first MU entries of E) to global
// memory, range-checked; LOWER zeroes the entries right of the diagonal.  Every
// LDS read before the first store.
template <int MU, bool LOWER = false, int M>
__device__ __forceinline__ void lstore(double *dst, long long n, const double *lds, const Elems<M> &E, int t,
                                       double scale = 1.0)
{
    static_assert(MU <= M, "element count");
    const brsrc_t r = brsrc(dst, n);
    double v[MU];
#pragma unroll
    for (int m = 0; m < MU; ++m) {
        const double x = lds[E.lo[m]];
        v[m] = (LOWER && E.ec[m] > E.er[m]) ? 0.0 : scale * x;
    }
    pin_row<MU>(v);
#pragma unroll
    for (int m = 0; m < MU; ++m) bstore(r, t + 64 * m, v[m]);
}

// ---------------------------------------------------------------- elimination
// Column c of the fused elimination, then the columns after it (template
// recursion: every register index is a constant).  f = A[t][c] / A[c][c] on lanes
// below the pivot (t > c: D rows below it and every panel lane), 0 elsewhere, so
// the rows and right-hand sides of finished lanes stay as they are; lane c keeps
// 1 / L_cc in myinv.  After the sweep lane t < BP holds row t of L (entries right
// of the diagonal stale) and w_t^(t) (y_t = w_t myinv), panel lanes hold
// P L^{-T} and w - P y.  A pivot that is not positive and finite gives a NaN myinv
// (see sqrt_rsqrt), tested once after the sweep.  inv is 1 / sqrt of pivot c: each
// step updates the next pivot's column first, reads the pivot from its lane and
// spreads the dependent stages of its square root over its own remaining updates,
// which fill the latencies of that chain.
template <int W, int NR, bool RHS, int c>
__device__ __forceinline__ void lelim(double (&row)[W], double (&w)[NR], double &myinv, int t, double inv)
{
    if constexpr (c < W) {
        const double v = row[c] * inv;
        const double f = (t > c) ? v * inv : 0.0;
        row[c] = v;
        myinv = (t == c) ? inv : myinv;
        if constexpr (c + 1 < W) {
            row[c + 1] = fma(-f, readlane_d(row[c + 1], c), row[c + 1]);
            RsqChain q{readlane_d(row[c + 1], c + 1), 0.0, 0.0, 0.0};
            constexpr int NROWU = W - c - 2, NU = NROWU + (RHS ? NR : 0);
            static_for<0, RSQ_STAGES>([&](auto ss) {
                constexpr int st = decltype(ss)::value;
                rsq_stage(st, q);
                static_for<(NU * st) / RSQ_STAGES, (NU * (st + 1)) / RSQ_STAGES>([&](auto uu) {
                    constexpr int u = decltype(uu)::value;
                    if constexpr (u < NROWU) {
                        row[c + 2 + u] = fma(-f, readlane_d(row[c + 2 + u], c), row[c + 2 + u]);
                    } else {
                        w[u - NROWU] = fma(-f, readlane_d(w[u - NROWU], c), w[u - NROWU]);
                    }
                });
                __builtin_amdgcn_sched_barrier(0);
            });
            lelim<W, NR, RHS, c + 1>(row, w, myinv, t, q.h);
        } else if constexpr (RHS) {
#pragma unroll
            for (int j = 0; j < NR; ++j) w[j] = fma(-f, readlane_d(w[j], c), w[j]);
        }
    }
}

// the elimination from its first pivot
template <int W, int NR, bool RHS>
__device__ __forceinline__ void lelim_all(double (&row)[W], double (&w)[NR], double &myinv, int t)
{
    double d, inv;
    sqrt_rsqrt(readlane_d(row[0], 0), d, inv);
    (void)d;
    lelim<W, NR, RHS, 0>(row, w, myinv, t, inv);
}

// ---------------------------------------------------------------- factor loads
// The blocks of stage j of a factor chain (lane-contiguous elements): the
// diagonal block, the coupling block (its rows are the next E rows), the arrow
// rows and the rhs rows.  Reduced chain: the partials minus hat F hat F^T,
// hat G hat F^T, plus -hat F y of the segment before (Eqs. 7, 8c, 9d).
template <int BP, int NR, bool RED>
struct LanePre {
    using G = LC<BP>;
    static constexpr int MB = G::MB, MG = G::MG, MY = G::MY;
    double d[MB], c[MB], g[MG], r[MY];
    double d2[RED ? MB : 1], g2[RED ? MG : 1], r2[RED ? MY : 1];

    __device__ __forceinline__ void load(const WChain<RED> &ch, int j, bool fwd, int t)
    {
        const Args &a = ch.a;
        const SysDesc &sd = ch.sd;
        const int b = sd.b, ng = sd.ng, nr = a.nr, s = ch.stage(j);
        const long long b2 = (long long)b * b, gb = (long long)ng * b, rb = fwd ? (long long)b * nr : 0;
        const bool hasE = ch.has_next(j);
        const brsrc_t rD = brsrc(RED ? a.F + sd.oLd + s * b2 : a.D + sd.oD + s * b2, b2);
        const brsrc_t rC = brsrc(RED ? a.F + ch.coup_off(j) : a.C + sd.oC + s * b2, hasE ? b2 : 0);
        const brsrc_t rB = brsrc(RED ? a.F + sd.oLb + s * gb : a.B + sd.oB + s * gb, gb);
        const brsrc_t rR = brsrc(a.rhs + sd.oRhs + s * b * nr, rb);
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            d[m] = bload(rD, t + 64 * m);
            c[m] = bload(rC, t + 64 * m);
        }
#pragma unroll
        for (int m = 0; m < MG; ++m) g[m] = bload(rB, t + 64 * m);
#pragma unroll
        for (int m = 0; m < MY; ++m) r[m] = bload(rR, t + 64 * m);
        if constexpr (RED) {
            const double *sc = ch.scr(j + 1);
            const brsrc_t rA = brsrc(sc + scr_dA(b, ng, nr), b2), rQ = brsrc(sc + scr_dQ(b, ng, nr), gb);
            const brsrc_t rY = brsrc(sc + scr_dy(b, ng, nr), rb);
#pragma unroll
            for (int m = 0; m < MB; ++m) d2[m] = bload(rA, t + 64 * m);
#pragma unroll
            for (int m = 0; m < MG; ++m) g2[m] = bload(rQ, t + 64 * m);
#pragma unroll
            for (int m = 0; m < MY; ++m) r2[m] = bload(rY, t + 64 * m);
        }
    }

    // The diagonal block and the arrow rows into cb (rows [0, BP) and [BP, BP + 16),
    // pitch P: the Gram reads them as its accumulator input), the coupling rows into
    // the E rows of the next-row area, the rhs rows into rn (pitch RP).
    __device__ __forceinline__ void commit(double *cb, double *nxt, double *rn, int b, int ng, int nr,
                                          const Elems<LC<BP>::MG> &E, const Elems<LC<BP>::MY> &Y, int t) const
    {
        constexpr int P = WC<BP>::P, RP = WC<BP>::RP;
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            if (t + 64 * m < b * b) {
                cb[E.er[m] * P + E.ec[m]] = RED ? d[m] - d2[m] : d[m];
                nxt[(BP + E.er[m]) * P + E.ec[m]] = c[m];
            }
        }
#pragma unroll
        for (int m = 0; m < MG; ++m)
            if (t + 64 * m < ng * b) cb[(BP + E.er[m]) * P + E.ec[m]] = RED ? g[m] - g2[m] : g[m];
#pragma unroll
        for (int m = 0; m < MY; ++m)
            if (t + 64 * m < b * nr) rn[Y.er[m] * RP + Y.ec[m]] = RED ? r[m] + r2[m] : r[m];
    }
};

// Element (p, q), q < BP, of the E-column tiles as the next stage starts it: the
// symmetrized diagonal block (cb holds the identity on its padded diagonal), the
// arrow rows, or zero for the fill rows.
template <int BP>
__device__ __forceinline__ double lfresh(const double *cb, int pb, int p, int q)
{
    constexpr int P = WC<BP>::P;
    if (pb < BP) return 0.5 * (cb[p * P + q] + cb[q * P + p]);
    if (pb < BP + NGM) return cb[p * P + q];
    return 0.0;
}

// ---------------------------------------------------------------- factor sweep
// Factor (and with FWD forward-substitute) one chain: segment k of a system
// (Algorithm 1 parallel phase, Algorithm 2 fused), the whole system when p = 1,
// or (RED) the reduced separator chain (sequential phases, without the corner).
// Outputs as the multi-wave sweep: the factor blocks in the input pattern, y in
// place of the rhs; for a segment k >= 2 hat A_k, hat Q_k and the separator rhs;
// for a segment ending on hat F_k (k < p) hat F_k hat F_k^T, hat G hat F_k^T,
// -hat F_k y and tilde H_k; the arrow partials -sum hat G hat G^T and -sum hat G y
// in the segment's scratch (RED: in LDS for the corner).  Returns the 1-based
// natural index of the first stage whose pivot failed, 0 if none.
template <int BP, int NR, bool FWD, bool RED>
__device__ __forceinline__ int lane_factor(const Args &a, const SysDesc &sd, int k, const WaveLds &L)
{
    using C = WC<BP>;
    using G = LC<BP>;
    constexpr int P = C::P, RP = C::RP, T2 = G::T2, KS = G::KS, NTL = G::NTL, NROW = G::NROW, F0 = G::F0;
    constexpr int MB = G::MB, MG = G::MG, MY = G::MY;
    const WChain<RED> ch{a, sd, k};
    const int b = sd.b, ng = sd.ng, nr = a.nr;
    const long long b2 = (long long)b * b, gb = (long long)ng * b, rb = (long long)b * nr;
    double *F = a.F;
    const bool hasF = !RED && k > 1;
    const int len = ch.length();
    const int sep = hasF ? sep_of(sd, k) : 0;
    const int tid = threadIdx.x;
    double *cb = L.acc_a;   // (BP + 16) x P: the next diagonal block and arrow rows

    Elems<MG> E;   // elements of blocks with b columns
    Elems<MY> Y;   // elements of rhs rows
    E.init(tid, b, P);
    Y.init(tid, nr, RP);

    // ---- prologue: the next-row area and cb with the identity on the padded
    // diagonal; stage 0's blocks; its diagonal and arrow rows where the Gram leaves
    // them for later stages, its fill rows F_w = C_sep^T; the running sums (hat R_k
    // = 0, hat A_k = sym(D_sep), hat Q_k = B_sep); the separator rhs on the F lanes
    for (int e = tid; e < (C::NROW + 2) * P; e += 64) {
        const int rr = e / P, cc = e - rr * P;
        L.nxt[e] = (rr < BP && rr == cc && rr >= b) ? 1.0 : 0.0;
    }
    for (int e = tid; e < (BP + NGM) * P; e += 64) {
        const int rr = e / P, cc = e - rr * P;
        cb[e] = (rr < BP && rr == cc && rr >= b) ? 1.0 : 0.0;
    }
    // rhs staging: the commits write the rows of the block only, so the padded rows
    // (read by the padded D lanes) must start as zeros
    if (FWD)
        for (int e = tid; e < C::BPX * RP; e += 64) L.w[e] = L.rn[e] = 0.0;
    LanePre<BP, NR, RED> pre;
    pre.load(ch, 0, FWD, tid);
    wave_sync();
    pre.commit(cb, L.nxt, L.rn, b, ng, nr, E, Y, tid);
    wave_sync();
    for (int e = tid; e < (BP + NGM) * BP; e += 64) {
        const int p = e / BP, q = e - p * BP;
        L.nxt[(p < BP ? p : BP + p) * P + q] = lfresh<BP>(cb, p < BP ? 0 : BP, p, q);
    }
    if (hasF) {
        const double *Cs = a.C + sd.oC + (long long)sep * b2;
        for (int e = tid; e < b * b; e += 64) {
            const int rr = e / b, cc = e - rr * b;
            L.nxt[(C::RF + cc) * P + rr] = Cs[e];
        }
    }
    dx4 acc[NTL];
    {
        const int q0 = tid & 15, p0 = tid >> 4;
        const double *Ds = a.D + sd.oD + (long long)sep * b2;
        const double *Bs = a.B + sd.oB + (long long)sep * ng * b;
#pragma unroll
        for (int tr = 0; tr < T2; ++tr)
#pragma unroll
            for (int tc = 0; tc <= tr; ++tc)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int pb = 16 * tr + 4 * v, p = pb + p0, q = 16 * tc + q0;
                    double x = 0.0;
                    if (pb >= F0) {
                        const int r = p - F0;
                        if (q >= F0) {
                            const int c = q - F0;
                            const bool ok = hasF && r < b && c < b;
                            x = 0.5 * (ld_or_zero(Ds, ok ? r * b + c : 0, ok) + ld_or_zero(Ds, ok ? c * b + r : 0, ok));
                        } else if (q >= BP) {
                            const int qq = q - BP;
                            const bool ok = hasF && qq < ng && r < b;
                            x = ld_or_zero(Bs, ok ? qq * b + r : 0, ok);
                        }
                    }
                    acc[tr * (tr + 1) / 2 + tc][v] = x;
                }
    }
    double w[NR];
    {
        const int r = tid - C::TF;
        const bool fl = FWD && hasF && r >= 0 && r < b;
        const double *rs = a.rhs + sd.oRhs + (long long)sep * b * nr;
#pragma unroll
        for (int j = 0; j < NR; ++j) w[j] = ld_or_zero(rs, fl ? r * nr + j : 0, fl && j < nr);
    }
    wave_sync();

    int failed = 0;
    double row[BP];
    for (int i = 0; i < len; ++i) {
        const int gs = ch.stage(i);
        const bool hasE = ch.has_next(i);
        const bool last = i == len - 1;
        const bool endS = !RED && last && hasE;
        const int t = opaque_tid();
        const bool isD = t < BP;
        const bool isE = t >= BP && t < 2 * BP;

        // ---- (1) rows from the next-row area; the D lanes' rhs
        {
            const double *src = L.nxt + (t < NROW ? t : C::ZROW) * P;
#pragma unroll
            for (int m = 0; m < BP; ++m) row[m] = src[m];
            if (FWD) {
                const int tr = isD ? t : 0;
#pragma unroll
                for (int j = 0; j < NR; ++j) {
                    const double x = L.w[tr * RP + j] + L.rn[tr * RP + j];
                    w[j] = isD ? x : (isE ? 0.0 : w[j]);
                }
            }
        }
        wave_sync();
        // ---- (2) the previous stage's outputs leave, the next stage's blocks arrive
        if (i > 0) {
            const int ps = ch.stage(i - 1);
            lstore<MB, true>(F + sd.oLd + (long long)ps * b2, b2, L.pnl + C::RD * P, E, t);
            lstore<MB>(F + ch.coup_off(i - 1), b2, L.pnl + C::RE * P, E, t);
            if (ng) lstore<MG>(F + sd.oLb + (long long)ps * gb, gb, L.pnl + C::RG * P, E, t);
            if (hasF) lstore<MB>(F + ch.fill_off(i - 1), b2, L.pnl + C::RF * P, E, t);
            if (FWD) lstore<MY>(a.rhs + sd.oRhs + (long long)ps * rb, rb, L.y, Y, t);
        }
        if (!last) pre.load(ch, i + 1, FWD, t);

        // ---- (3) elimination (Algorithm 1 potrf / trsm, Algorithm 2)
        double myinv = 1.0;
        lelim_all<BP, NR, FWD>(row, w, myinv, t);
        if (any_bad_pivot(t < b, myinv) && !failed) failed = gs + 1;

        // ---- (4) rows to LDS: the Gram's operands, the factor rows and y for their
        // stores; -hat E y for the next stage's rhs
        if (t < NROW) {
            double *dst = L.pnl + t * P;
#pragma unroll
            for (int m = 0; m < BP; ++m) dst[m] = row[m];
        }
        if (FWD) {
            if (isD) {
#pragma unroll
                for (int j = 0; j < NR; ++j) L.y[t * RP + j] = w[j] * myinv;
            } else if (isE && hasE) {
                const int r = t - BP;
#pragma unroll
                for (int j = 0; j < NR; ++j) L.w[r * RP + j] = w[j];
            }
        }
        // the next stage's blocks (their loads have arrived during the elimination)
        if (!last) pre.commit(cb, L.nxt, L.rn, b, ng, nr, E, Y, t);
        wave_sync();

        // ---- (5) Gram of the E, G, F rows on the matrix cores
        {
            const int q0 = t & 15, p0 = t >> 4;
            double op[T2][KS];
#pragma unroll
            for (int t2 = 0; t2 < T2; ++t2)
#pragma unroll
                for (int s = 0; s < KS; ++s) op[t2][s] = L.pnl[(BP + 16 * t2 + q0) * P + 4 * s + p0];
            bool live[T2];
            if (BP == 16) {
                live[0] = hasE;
                live[1] = ng > 0;
                live[T2 - 1] = hasF;
            } else {
                live[0] = hasE || ng > 0;
                live[T2 - 1] = ng > 8 || hasF;
            }
            const bool fq = BP == 16 || q0 < BP;   // a column of the E rows
            const bool fresh = !endS && !last;
#pragma unroll
            for (int tr = 0; tr < T2; ++tr)
#pragma unroll
                for (int tc = 0; tc <= tr; ++tc) {
                    if (!(live[tr] && live[tc])) continue;
                    const int ix = tr * (tr + 1) / 2 + tc;
                    dx4 cur = acc[ix];
                    if (tc == 0) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int pb = 16 * tr + 4 * v, p = pb + p0;
                            const double fv = fresh ? lfresh<BP>(cb, pb, fq ? p : 0, fq ? q0 : 0) : 0.0;
                            cur[v] = fq ? fv : cur[v];
                        }
                    }
#pragma unroll
                    for (int s = 0; s < KS; ++s) cur = mfma4(-op[tr][s], op[tc][s], cur);
                    acc[ix] = cur;
                    if (tc == 0 && hasE && fq) {
                        // next D, G, F rows (at a segment end the scratch products)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int pb = 16 * tr + 4 * v, p = pb + p0;
                            if (pb < F0 || hasF) L.nxt[(pb < BP ? p : BP + p) * P + q0] = cur[v];
                        }
                    }
                }
        }
        wave_sync();
        if (endS) {
            // hat F_k hat F_k^T, hat G hat F_k^T (Eq. 8c), tilde H_k = -hat F_k hat B (transposed) and -hat F_k y
            double *sc = ch.scr(k);
            wstore<64, BP * BP>(sc + scr_dA(b, ng, nr), L.nxt + C::RD * P, P, b, b, t, -1.0);
            if (ng) wstore<64, NGM * BP>(sc + scr_dQ(b, ng, nr), L.nxt + C::RG * P, P, ng, b, t, -1.0);
            if (hasF) wstore<64, BP * BP, true>(F + sd.oH + (long long)(k - 2) * b2, L.nxt + C::RF * P, P, b, b, t);
            if (FWD) lstore<MY>(sc + scr_dy(b, ng, nr), rb, L.w, Y, t);
        }
    }

    // ---- epilogue: the last stage's outputs, the running sums and the partials
    {
        const int ps = ch.stage(len - 1);
        lstore<MB, true>(F + sd.oLd + (long long)ps * b2, b2, L.pnl + C::RD * P, E, tid);
        if (ch.has_next(len - 1)) lstore<MB>(F + ch.coup_off(len - 1), b2, L.pnl + C::RE * P, E, tid);
        if (ng) lstore<MG>(F + sd.oLb + (long long)ps * gb, gb, L.pnl + C::RG * P, E, tid);
        if (hasF) lstore<MB>(F + ch.fill_off(len - 1), b2, L.pnl + C::RF * P, E, tid);
        if (FWD) lstore<MY>(a.rhs + sd.oRhs + (long long)ps * rb, rb, L.y, Y, tid);
    }
    {
        const int q0 = tid & 15, p0 = tid >> 4;
        double *Rg = RED ? nullptr : ch.scr(k) + scr_Rk(b, ng, nr);
        double *As = F + sd.oLd + (long long)sep * b2, *Qs = F + sd.oLb + (long long)sep * ng * b;
#pragma unroll
        for (int tr = 0; tr < T2; ++tr)
#pragma unroll
            for (int tc = 0; tc <= tr; ++tc)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int pb = 16 * tr + 4 * v, p = pb + p0, q = 16 * tc + q0;
                    const double x = acc[tr * (tr + 1) / 2 + tc][v];
                    if (pb >= BP && pb < F0) {
                        // hat R_k (G x G); an off-diagonal tile holds one triangle only
                        const int ga = p - BP, gc = q - BP;
                        if (q >= BP && q < F0 && ga < ng && gc < ng) {
                            if (RED) {
                                L.racc[ga * (NGM + 1) + gc] = x;
                                if (tr != tc) L.racc[gc * (NGM + 1) + ga] = x;
                            } else {
                                Rg[ga * ng + gc] = x;
                                if (tr != tc) Rg[gc * ng + ga] = x;
                            }
                        }
                    } else if (pb >= F0 && hasF) {
                        const int r = p - F0;
                        if (q >= F0) {
                            const int c = q - F0;   // hat A_k (F x F, a diagonal tile)
                            if (r < b && c < b) As[r * b + c] = x;
                        } else if (q >= BP) {
                            const int gq = q - BP;  // hat Q_k^T (F x G)
                            if (r < b && gq < ng) Qs[gq * b + r] = x;
                        }
                    }
                }
        if (FWD) {
            const int r = tid - C::TG;
            if (r >= 0 && r < NGM) {
                if (RED) {
#pragma unroll
                    for (int j = 0; j < NR; ++j) L.yg[r * RP + j] = w[j];
                } else if (r < ng) {
                    double *yg = ch.scr(k) + scr_yg(b, ng, nr);
#pragma unroll
                    for (int j = 0; j < NR; ++j)
                        if (j < nr) yg[r * nr + j] = w[j];
                }
            }
            const int rf = tid - C::TF;
            if (hasF && rf >= 0 && rf < b) {
#pragma unroll
                for (int j = 0; j < NR; ++j)
                    if (j < nr) a.rhs[sd.oRhs + ((long long)sep * b + rf) * nr + j] = w[j];
            }
        } else if (RED) {
            const int r = tid - C::TG;
            if (r >= 0 && r < NGM) {
#pragma unroll
                for (int j = 0; j < RP; ++j) L.yg[r * RP + j] = 0.0;
            }
        }
    }
    wave_sync();
    return failed;
}

// ---------------------------------------------------------------- forward sweep
// The factor blocks of stage j of a chain (lane-contiguous elements) and the rhs
// rows (RED: plus -hat F y), committed to the staging area: rows of L without
// their diagonal (which goes to dv), hat E, hat G, the fill rows.
template <int BP, int NR, bool RED>
struct LaneRowPre {
    using G = LC<BP>;
    static constexpr int MB = G::MB, MG = G::MG, MY = G::MY;
    double d[MB], e[MB], f[MB], g[MG], r[MY], r2[RED ? MY : 1];

    __device__ __forceinline__ void load(const WChain<RED> &ch, int j, bool hasF, int t)
    {
        const Args &a = ch.a;
        const SysDesc &sd = ch.sd;
        const int b = sd.b, ng = sd.ng, nr = a.nr, s = ch.stage(j);
        const long long b2 = (long long)b * b, gb = (long long)ng * b, rb = (long long)b * nr;
        const bool hasE = ch.has_next(j);
        const brsrc_t rD = brsrc(a.F + sd.oLd + s * b2, b2);
        const brsrc_t rE = brsrc(a.F + ch.coup_off(j), hasE ? b2 : 0);
        const brsrc_t rF = brsrc(a.F + (hasF ? ch.fill_off(j) : 0), hasF ? b2 : 0);
        const brsrc_t rB = brsrc(a.F + sd.oLb + s * gb, gb);
        const brsrc_t rR = brsrc(a.rhs + sd.oRhs + s * rb, rb);
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            d[m] = bload(rD, t + 64 * m);
            e[m] = bload(rE, t + 64 * m);
            f[m] = bload(rF, t + 64 * m);
        }
#pragma unroll
        for (int m = 0; m < MG; ++m) g[m] = bload(rB, t + 64 * m);
#pragma unroll
        for (int m = 0; m < MY; ++m) r[m] = bload(rR, t + 64 * m);
        if constexpr (RED) {
            const brsrc_t rY = brsrc(ch.scr(j + 1) + scr_dy(b, ng, nr), rb);
#pragma unroll
            for (int m = 0; m < MY; ++m) r2[m] = bload(rY, t + 64 * m);
        }
    }

    __device__ __forceinline__ void commit(double *area, double *dv, double *rn, int b, int ng, int nr,
                                          const Elems<LC<BP>::MG> &E, const Elems<LC<BP>::MY> &Y, int t) const
    {
        using C = WC<BP>;
        constexpr int P = C::P, RP = C::RP;
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            if (t + 64 * m < b * b) {
                const int rr = E.er[m], cc = E.ec[m];
                area[(C::RD + rr) * P + cc] = (rr == cc) ? 0.0 : d[m];
                if (rr == cc) dv[rr] = d[m];
                area[(C::RE + rr) * P + cc] = e[m];
                area[(C::RF + rr) * P + cc] = f[m];
            }
        }
#pragma unroll
        for (int m = 0; m < MG; ++m)
            if (t + 64 * m < ng * b) area[(C::RG + E.er[m]) * P + E.ec[m]] = g[m];
#pragma unroll
        for (int m = 0; m < MY; ++m)
            if (t + 64 * m < b * nr) rn[Y.er[m] * RP + Y.ec[m]] = RED ? r[m] + r2[m] : r[m];
    }
};

// Forward substitution of one chain with its factor in place (Algorithm 2,
// parallel phase for a segment, sequential phase for RED): y overwrites the rhs;
// the separator rhs partial, -hat F_k y and the arrow partial -sum hat G y go
// where the factor sweep puts them.
template <int BP, int NR, bool RED>
__device__ __forceinline__ void lane_forward(const Args &a, const SysDesc &sd, int k, const WaveLds &L)
{
    using C = WC<BP>;
    using G = LC<BP>;
    constexpr int P = C::P, RP = C::RP, NROW = G::NROW, MY = G::MY;
    const WChain<RED> ch{a, sd, k};
    const int b = sd.b, ng = sd.ng, nr = a.nr;
    const long long rb = (long long)b * nr;
    const bool hasF = !RED && k > 1;
    const int len = ch.length();
    const int sep = hasF ? sep_of(sd, k) : 0;
    const int tid = threadIdx.x;
    double *area = L.pnl, *dv = L.dinv;
    Elems<G::MG> E;
    Elems<MY> Y;
    E.init(tid, b, P);
    Y.init(tid, nr, RP);
    for (int e = tid; e < NROW * P; e += 64) area[e] = 0.0;
    for (int e = tid; e < C::BPX; e += 64) dv[e] = 1.0;
    // rhs staging: the commits write the rows of the block only, so the padded rows
    // (read by the padded D lanes) must start as zeros
    for (int e = tid; e < C::BPX * RP; e += 64) L.w[e] = L.rn[e] = 0.0;
    double w[NR];
    {
        const int r = tid - C::TF;
        const bool fl = hasF && r >= 0 && r < b;
        const double *rs = a.rhs + sd.oRhs + (long long)sep * b * nr;
#pragma unroll
        for (int j = 0; j < NR; ++j) w[j] = ld_or_zero(rs, fl ? r * nr + j : 0, fl && j < nr);
    }
    LaneRowPre<BP, NR, RED> pre;
    pre.load(ch, 0, hasF, tid);
    wave_sync();
    pre.commit(area, dv, L.rn, b, ng, nr, E, Y, tid);
    wave_sync();
    double row[BP];
    for (int i = 0; i < len; ++i) {
        const bool hasE = ch.has_next(i);
        const bool last = i == len - 1;
        const bool endS = !RED && last && hasE;
        const int t = opaque_tid();
        const bool isD = t < BP;
        const bool isE = t >= BP && t < 2 * BP;
        {
            const double *src = area + (t < NROW ? t : 0) * P;
#pragma unroll
            for (int m = 0; m < BP; ++m) row[m] = t < NROW ? src[m] : 0.0;
            const int tr = isD ? t : 0;
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                const double x = L.w[tr * RP + j] + L.rn[tr * RP + j];
                w[j] = isD ? x : (isE ? 0.0 : w[j]);
            }
        }
        const double myinv = 1.0 / dv[isD ? t : 0];
        wave_sync();
        if (i > 0) lstore<MY>(a.rhs + sd.oRhs + (long long)ch.stage(i - 1) * rb, rb, L.y, Y, t);
        if (!last) pre.load(ch, i + 1, hasF, t);
#pragma unroll
        for (int c = 0; c < BP; ++c) {
            const double ic = readlane_d(myinv, c);
#pragma unroll
            for (int j = 0; j < NR; ++j) w[j] = fma(-row[c], readlane_d(w[j], c) * ic, w[j]);
        }
        if (isD) {
#pragma unroll
            for (int j = 0; j < NR; ++j) L.y[t * RP + j] = w[j] * myinv;
        } else if (isE && hasE) {
            const int r = t - BP;
#pragma unroll
            for (int j = 0; j < NR; ++j) L.w[r * RP + j] = w[j];
        }
        if (!last) pre.commit(area, dv, L.rn, b, ng, nr, E, Y, t);
        wave_sync();
        if (endS) lstore<MY>(ch.scr(k) + scr_dy(b, ng, nr), rb, L.w, Y, t);
    }
    lstore<MY>(a.rhs + sd.oRhs + (long long)ch.stage(len - 1) * rb, rb, L.y, Y, tid);
    {
        const int r = tid - C::TG;
        if (r >= 0 && r < NGM) {
            if (RED) {
#pragma unroll
                for (int j = 0; j < NR; ++j) L.yg[r * RP + j] = w[j];
            } else if (r < ng) {
                double *yg = ch.scr(k) + scr_yg(b, ng, nr);
#pragma unroll
                for (int j = 0; j < NR; ++j)
                    if (j < nr) yg[r * nr + j] = w[j];
            }
        }
        const int rf = tid - C::TF;
        if (hasF && rf >= 0 && rf < b) {
#pragma unroll
            for (int j = 0; j < NR; ++j)
                if (j < nr) a.rhs[sd.oRhs + ((long long)sep * b + rf) * nr + j] = w[j];
        }
    }
    wave_sync();
}

// ---------------------------------------------------------------- backward sweep
// The factor blocks of stage i (lane-contiguous elements) and its y rows (with
// PRIMAL the primal solution rows too), committed to the staging area: L without
// its diagonal (which goes to dv), hat E, hat G, the fill rows; y into Yl.
template <int BP, int NR, bool RED>
struct LaneColPre {
    using G = LC<BP>;
    static constexpr int MB = G::MB, MG = G::MG, MY = G::MY;
    double d[MB], e[MB], f[MB], g[MG], y[MY], px[MY];

    template <bool PRIMAL>
    __device__ __forceinline__ void load(const WChain<RED> &ch, int i, bool hasF, int t)
    {
        const Args &a = ch.a;
        const SysDesc &sd = ch.sd;
        const int b = sd.b, ng = sd.ng, nr = a.nr, s = ch.stage(i);
        const long long b2 = (long long)b * b, gb = (long long)ng * b, rb = (long long)b * nr;
        const bool hasE = ch.has_next(i);
        const brsrc_t rD = brsrc(a.F + sd.oLd + s * b2, b2);
        const brsrc_t rE = brsrc(a.F + ch.coup_off(i), hasE ? b2 : 0);
        const brsrc_t rF = brsrc(a.F + (hasF ? ch.fill_off(i) : 0), hasF ? b2 : 0);
        const brsrc_t rB = brsrc(a.F + sd.oLb + s * gb, gb);
        const brsrc_t rY = brsrc(a.rhs + sd.oRhs + s * rb, rb);
        const brsrc_t rP = brsrc(PRIMAL ? a.xp + sd.oRhs + s * rb : a.rhs, PRIMAL ? rb : 0);
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            d[m] = bload(rD, t + 64 * m);
            e[m] = bload(rE, t + 64 * m);
            f[m] = bload(rF, t + 64 * m);
        }
#pragma unroll
        for (int m = 0; m < MG; ++m) g[m] = bload(rB, t + 64 * m);
#pragma unroll
        for (int m = 0; m < MY; ++m) {
            y[m] = bload(rY, t + 64 * m);
            px[m] = PRIMAL ? bload(rP, t + 64 * m) : 0.0;
        }
    }

    template <bool PRIMAL>
    __device__ __forceinline__ void commit(double *area, double *dv, double *Yl, double *Pl, int b, int ng, int nr,
                                           const Elems<LC<BP>::MG> &E, const Elems<LC<BP>::MY> &Y, int t) const
    {
        using C = WC<BP>;
        constexpr int P = C::P, RP = C::RP;
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            if (t + 64 * m < b * b) {
                const int rr = E.er[m], cc = E.ec[m];
                area[(C::RD + rr) * P + cc] = (rr == cc) ? 0.0 : d[m];
                if (rr == cc) dv[rr] = d[m];
                area[(C::RE + rr) * P + cc] = e[m];
                area[(C::RF + rr) * P + cc] = f[m];
            }
        }
#pragma unroll
        for (int m = 0; m < MG; ++m)
            if (t + 64 * m < ng * b) area[(C::RG + E.er[m]) * P + E.ec[m]] = g[m];
#pragma unroll
        for (int m = 0; m < MY; ++m) {
            if (t + 64 * m < b * nr) {
                Yl[Y.er[m] * RP + Y.ec[m]] = y[m];
                if (PRIMAL) Pl[Y.er[m] * RP + Y.ec[m]] = px[m];
            }
        }
    }
};

// Backward substitution of one chain (Algorithm 3, Eqs. 11, 12): for the chain's
// stages in reverse, x_i = hat D_i^{-T} (y_i - hat E_i^T x_next - hat G_i^T x_g
// [- hat B_i x_sep]); x_g, x at the separator of segment k and x after the chain
// are in place.  Lane c owns column c.  With ADJ the solution is lambda and the
// gradient blocks of the chain's stages are written as by the multi-wave sweep.
template <int BP, int NR, bool ADJ, bool RED>
__device__ __forceinline__ void lane_backward(const Args &a, const SysDesc &sd, int k, const WaveLds &L)
{
    using C = WC<BP>;
    using G = LC<BP>;
    constexpr int P = C::P, RP = C::RP, BPX = C::BPX, MY = G::MY;
    const WChain<RED> ch{a, sd, k};
    const int b = sd.b, ng = sd.ng, nr = a.nr, N = sd.N;
    const long long b2 = (long long)b * b, rb = (long long)b * nr;
    const bool hasF = !RED && k > 1;
    const int len = ch.length();
    const int sep = hasF ? sep_of(sd, k) : 0;
    double *X = a.rhs + sd.oRhs;
    const double *XP = ADJ ? a.xp + sd.oRhs : X;
    double *xn = L.xn, *xc = L.xc, *pn = L.pn, *pc = L.pc;
    double *area = L.pnl;
    double *dv = L.dinv;
    const int tid = threadIdx.x;
    Elems<G::MG> E;
    Elems<MY> Y;
    E.init(tid, b, P);
    Y.init(tid, nr, RP);
    for (int e = tid; e < C::NROW * P; e += 64) area[e] = 0.0;
    for (int e = tid; e < BPX; e += 64) dv[e] = 1.0;
    {
        const long long og = (long long)N * b * nr;
        for (int e = tid; e < NGM * RP; e += 64) {
            const int q = e / RP, j = e - q * RP;
            const bool in = q < ng && j < nr;
            L.xg[e] = in ? X[og + q * nr + j] : 0.0;
            if (ADJ) L.pg[e] = in ? XP[og + q * nr + j] : 0.0;
        }
        const bool after = !RED && ch.has_next(len - 1);
        const long long on = after ? (long long)(ch.stage(len - 1) + 1) * b * nr : 0;
        const long long os = (long long)sep * b * nr;
        for (int e = tid; e < BPX * RP; e += 64) {
            const int rr = e / RP, j = e - rr * RP;
            const bool in = rr < b && j < nr;
            L.xs[e] = (hasF && in) ? X[os + rr * nr + j] : 0.0;
            xn[e] = (after && in) ? X[on + rr * nr + j] : 0.0;
            xc[e] = 0.0;
            if (ADJ) {
                L.ps[e] = (hasF && in) ? XP[os + rr * nr + j] : 0.0;
                pn[e] = (after && in) ? XP[on + rr * nr + j] : 0.0;
                pc[e] = 0.0;
            }
        }
    }
    LaneColPre<BP, NR, RED> pre;
    pre.template load<ADJ>(ch, len - 1, hasF, tid);
    wave_sync();
    for (int i = len - 1; i >= 0; --i) {
        const int gs = ch.stage(i);
        const bool hasE = ch.has_next(i);
        const int t = opaque_tid();
        // ---- (1) stage i's blocks and y into the staging area; x of the stage
        // after it leaves; stage i - 1's blocks arrive
        pre.template commit<ADJ>(area, dv, xc, pc, b, ng, nr, E, Y, t);
        wave_sync();
        if (i < len - 1) lstore<MY>(X + (long long)ch.stage(i + 1) * rb, rb, xn, Y, t);
        if (i > 0) pre.template load<ADJ>(ch, i - 1, hasF, t);
        // ---- (2) lane c: acc = y_c - (hat E^T x_next)_c - (hat G^T x_g)_c - (hat B x_sep)_c
        const int c = t < BP ? t : 0;
        double acc[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j) acc[j] = xc[c * RP + j];
        if (hasE) {
#pragma unroll
            for (int m = 0; m < BP; ++m) {
                const double e = area[(C::RE + m) * P + c];
#pragma unroll
                for (int j = 0; j < NR; ++j) acc[j] = fma(-e, xn[m * RP + j], acc[j]);
            }
        }
        if (ng > 0) {
#pragma unroll
            for (int q = 0; q < NGM; ++q) {
                if (q == 8 && ng <= 8) break;
                const double g = area[(C::RG + q) * P + c];
#pragma unroll
                for (int j = 0; j < NR; ++j) acc[j] = fma(-g, L.xg[q * RP + j], acc[j]);
            }
        }
        if (hasF) {
#pragma unroll
            for (int m = 0; m < BP; ++m) {
                const double f = area[(C::RF + m) * P + c];
#pragma unroll
                for (int j = 0; j < NR; ++j) acc[j] = fma(-f, L.xs[m * RP + j], acc[j]);
            }
        }
        // ---- (3) back substitution with hat D^T: lane c holds column c of L below
        // the diagonal; x_c2 broadcast from lane c2, last column first
        double lc[BP];
#pragma unroll
        for (int m = 0; m < BP; ++m) lc[m] = area[(C::RD + m) * P + c];
        const double myinv = 1.0 / dv[c];
#pragma unroll
        for (int c2 = BP - 1; c2 >= 0; --c2) {
#pragma unroll
            for (int j = 0; j < NR; ++j) acc[j] = fma(-lc[c2], readlane_d(acc[j] * myinv, c2), acc[j]);
        }
        wave_sync();
        if (t < BP) {
#pragma unroll
            for (int j = 0; j < NR; ++j) xc[t * RP + j] = acc[j] * myinv;
        }
        wave_sync();
        if (ADJ && t < b) {
            // dD_i = -sym(lambda_i x_i^T), dB_i = -(lambda_g x_i^T + x_g lambda_i^T),
            // dC_i = -(lambda_{i+1} x_i^T + x_{i+1} lambda_i^T) for natural neighbours,
            // and the separator coupling of the first stage (column c)
            double *dD = a.dD + sd.oD + (long long)gs * b2;
            for (int rr = 0; rr < b; ++rr) {
                double s = 0.0;
                for (int j = 0; j < nr; ++j) s += xc[rr * RP + j] * pc[c * RP + j] + pc[rr * RP + j] * xc[c * RP + j];
                dD[rr * b + c] = -0.5 * s;
            }
            double *dB = a.dB + sd.oB + (long long)gs * ng * b;
            for (int q = 0; q < ng; ++q) {
                double s = 0.0;
                for (int j = 0; j < nr; ++j) s += L.xg[q * RP + j] * pc[c * RP + j] + L.pg[q * RP + j] * xc[c * RP + j];
                dB[q * b + c] = -s;
            }
            if (!RED && hasE) {
                double *dC = a.dC + sd.oC + (long long)gs * b2;
                for (int rr = 0; rr < b; ++rr) {
                    double s = 0.0;
                    for (int j = 0; j < nr; ++j) s += xn[rr * RP + j] * pc[c * RP + j] + pn[rr * RP + j] * xc[c * RP + j];
                    dC[rr * b + c] = -s;
                }
            }
            if (hasF && i == 0) {
                double *dC = a.dC + sd.oC + (long long)sep * b2;
                for (int rr = 0; rr < b; ++rr) {
                    double s = 0.0;
                    for (int j = 0; j < nr; ++j) s += xc[rr * RP + j] * L.ps[c * RP + j] + pc[rr * RP + j] * L.xs[c * RP + j];
                    dC[rr * b + c] = -s;
                }
            }
        }
        wave_sync();
        double *tmp = xn; xn = xc; xc = tmp;
        tmp = pn; pn = pc; pc = tmp;
    }
    lstore<MY>(X + (long long)ch.stage(0) * rb, rb, xn, Y, tid);
    wave_sync();
}

}  // namespace kkt_dev
