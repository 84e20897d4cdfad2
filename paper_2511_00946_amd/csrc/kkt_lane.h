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
// outputs (from LDS) and the loads of the next stage's blocks together, and
// consumes the loads only at its end: loads and stores share one counter, so a
// wait for a load with a younger store pending waits for every memory operation.
//
// Forward sweep (solve modes): the same lane layout with the factor rows fetched
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
    static constexpr int G0 = BP, F0 = BP + NGM;    // Gram coordinate of the first G / F row
    static_assert(BP == 8 || BP == 16, "single-wave sweeps cover padded sizes 8 and 16");
    static_assert(NROW <= 64 && N2 % 16 == 0, "row placement");
    static_assert(WC<BP>::NW == 1 && WC<BP>::TE == BP && WC<BP>::TG == 2 * BP && WC<BP>::TF == 2 * BP + NGM,
                  "lane t holds panel row t");
};

// ---------------------------------------------------------------- elimination
// Column c of the fused elimination, then the columns after it (template
// recursion: every register index is a constant).  f = A[t][c] / A[c][c] on lanes
// below the pivot (t > c: D rows below it and every panel lane), 0 elsewhere, so
// the rows and right-hand sides of finished lanes stay as they are; lane c keeps
// 1 / L_cc in myinv.  After the sweep lane t < BP holds row t of L (entries right
// of the diagonal stale) and w_t^(t) (y_t = w_t myinv), panel lanes hold
// P L^{-T} and w - P y.  A pivot that is not positive and finite gives a NaN myinv
// (see sqrt_rsqrt), tested once after the sweep.
template <int W, int NR, bool RHS, int c>
__device__ __forceinline__ void lelim(double (&row)[W], double (&w)[NR], double &myinv, int t)
{
    if constexpr (c < W) {
        const double dcc = readlane_d(row[c], c);
        double d, inv;
        sqrt_rsqrt(dcc, d, inv);
        (void)d;
        const double v = row[c] * inv;
        const double f = (t > c) ? v * inv : 0.0;
        row[c] = v;
        myinv = (t == c) ? inv : myinv;
#pragma unroll
        for (int m = c + 1; m < W; ++m) row[m] = fma(-f, readlane_d(row[m], c), row[m]);
        if constexpr (RHS) {
#pragma unroll
            for (int j = 0; j < NR; ++j) w[j] = fma(-f, readlane_d(w[j], c), w[j]);
        }
        lelim<W, NR, RHS, c + 1>(row, w, myinv, t);
    }
}

// Rows [0, rows) x [0, cols) of an LDS block (pitch P) to a row-major global block
// from a single wave, with the (row, column) of each lane's elements given; LOWER
// zeroes the entries right of the diagonal.  Every LDS read before the first store.
template <int M, bool LOWER = false>
__device__ __forceinline__ void lstore(double *dst, const double *lds, int P, int rows, int cols, const int (&er)[M],
                                       const int (&ec)[M], double scale = 1.0)
{
    double v[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const bool ok = er[m] < rows;
        const double x = lds[(ok ? er[m] : 0) * P + (ok ? ec[m] : 0)];
        v[m] = (LOWER && ec[m] > er[m]) ? 0.0 : scale * x;
    }
    pin_row<M>(v);
#pragma unroll
    for (int m = 0; m < M; ++m)
        if (er[m] < rows) dst[er[m] * cols + ec[m]] = v[m];
}

// ---------------------------------------------------------------- factor loads
// The blocks of stage j of a factor chain that the stage before consumes at its
// end: the next diagonal block (both triangles, to symmetrize it) and arrow rows
// in the Gram's tile layout (lane l, element v of tile row tr: row 16 tr + 4 v +
// l / 16, column l % 16), the next coupling rows on the E lanes and the next rhs
// rows on the D lanes.  Reduced chain: the partials minus hat F hat F^T, hat G
// hat F^T, plus -hat F y of the segment before (Eqs. 7, 8c, 9d).
template <int BP, int NR, bool RED>
struct LanePre {
    static constexpr int T2 = LC<BP>::T2;
    double x1[T2][4], x2[T2][4], x3[T2][4], x4[T2][4];
    double cr[BP];
    double r1[NR], r2[NR];

    __device__ __forceinline__ void load(const WChain<RED> &ch, int j, bool fwd, int t)
    {
        const Args &a = ch.a;
        const SysDesc &sd = ch.sd;
        const int b = sd.b, ng = sd.ng, nr = a.nr, s = ch.stage(j);
        const long long b2 = (long long)b * b, gb = (long long)ng * b;
        const double *Dp = RED ? a.F + sd.oLd + s * b2 : a.D + sd.oD + s * b2;
        const double *Bp = RED ? a.F + sd.oLb + s * gb : a.B + sd.oB + s * gb;
        const double *sc = RED ? ch.scr(j + 1) : a.F;
        const int q = t & 15, p0 = t >> 4;
#pragma unroll
        for (int tr = 0; tr < T2; ++tr)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int pb = 16 * tr + 4 * v, p = pb + p0;
                if (pb < BP) {
                    const bool ok = p < b && q < b;
                    const int e1 = ok ? p * b + q : 0, e2 = ok ? q * b + p : 0;
                    x1[tr][v] = ld_or_zero(Dp, e1, ok);
                    x2[tr][v] = ld_or_zero(Dp, e2, ok);
                    x3[tr][v] = RED ? ld_or_zero(sc + scr_dA(b, ng, nr), e1, ok) : 0.0;
                    x4[tr][v] = RED ? ld_or_zero(sc + scr_dA(b, ng, nr), e2, ok) : 0.0;
                } else if (pb < BP + NGM) {
                    const int qg = p - BP;
                    const bool ok = qg < ng && q < b;
                    const int e1 = ok ? qg * b + q : 0;
                    x1[tr][v] = ld_or_zero(Bp, e1, ok);
                    x3[tr][v] = RED ? ld_or_zero(sc + scr_dQ(b, ng, nr), e1, ok) : 0.0;
                    x2[tr][v] = 0.0;
                    x4[tr][v] = 0.0;
                } else {
                    x1[tr][v] = x2[tr][v] = x3[tr][v] = x4[tr][v] = 0.0;
                }
            }
        const bool hasE = ch.has_next(j);
        const double *Cp = RED ? a.F + ch.coup_off(j) : a.C + sd.oC + s * b2;
        const int r = t - BP;
        const bool er = hasE && r >= 0 && r < b;
        const int rb = er ? r * b : 0;
#pragma unroll
        for (int m = 0; m < BP; ++m) cr[m] = ld_or_zero(Cp, rb + m, er && m < b);
        const double *Rp = a.rhs + sd.oRhs + (long long)s * b * nr;
        const bool dr = fwd && t < b;
        const int ro = dr ? t * nr : 0;
#pragma unroll
        for (int jj = 0; jj < NR; ++jj) {
            r1[jj] = ld_or_zero(Rp, ro + jj, dr && jj < nr);
            r2[jj] = RED ? ld_or_zero(sc + scr_dy(b, ng, nr), ro + jj, dr && jj < nr) : 0.0;
        }
    }

    // Element v of tile row tr of the E-column tiles as the next stage starts it:
    // the symmetrized diagonal block (identity on the padded diagonal), the arrow
    // rows, or zero (fill rows).
    __device__ __forceinline__ double fresh(int tr, int v, int t, int b) const
    {
        const int pb = 16 * tr + 4 * v, p = pb + (t >> 4), q = t & 15;
        if (pb < BP) return 0.5 * ((x1[tr][v] - x3[tr][v]) + (x2[tr][v] - x4[tr][v])) + ((p == q && p >= b) ? 1.0 : 0.0);
        if (pb < BP + NGM) return x1[tr][v] - x3[tr][v];
        return 0.0;
    }
};

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
    constexpr int MB = BP * BP / 64, MG = NGM * BP / 64;
    const WChain<RED> ch{a, sd, k};
    const int b = sd.b, ng = sd.ng, nr = a.nr;
    const long long b2 = (long long)b * b;
    double *F = a.F;
    const bool hasF = !RED && k > 1;
    const int len = ch.length();
    const int sep = hasF ? sep_of(sd, k) : 0;
    const int tid = threadIdx.x;

    // (row, column) of this lane's elements of a b-column block, for the stores
    int er[MG], ec[MG], yr[2], yc[2];
    {
        const float invb = 1.0f / (float)b, invr = 1.0f / (float)nr;
#pragma unroll
        for (int m = 0; m < MG; ++m) rc_of(tid + 64 * m, b, invb, er[m], ec[m]);
#pragma unroll
        for (int m = 0; m < 2; ++m) rc_of(tid + 64 * m, nr, invr, yr[m], yc[m]);
    }
    int erd[MB], ecd[MB];
#pragma unroll
    for (int m = 0; m < MB; ++m) { erd[m] = er[m]; ecd[m] = ec[m]; }

    // ---- prologue: the next-row area with the identity on the padded diagonal,
    // stage 0's diagonal and arrow rows as the Gram leaves them for later stages,
    // its fill rows F_w = C_sep^T; the running sums (hat R_k = 0, hat A_k =
    // sym(D_sep), hat Q_k = B_sep); the separator rhs on the F lanes
    for (int e = tid; e < (C::NROW + 2) * P; e += 64) {
        const int rr = e / P, cc = e - rr * P;
        L.nxt[e] = (rr < BP && rr == cc && rr >= b) ? 1.0 : 0.0;
    }
    if (FWD)
        for (int e = tid; e < C::BPX * RP; e += 64) L.w[e] = 0.0;
    LanePre<BP, NR, RED> pre;
    pre.load(ch, 0, FWD, tid);
    wave_sync();
    {
        const int q = tid & 15, p0 = tid >> 4;
        if (BP == 16 || q < BP) {
#pragma unroll
            for (int tr = 0; tr < T2; ++tr)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int pb = 16 * tr + 4 * v, p = pb + p0;
                    if (pb < F0) L.nxt[(pb < BP ? p : BP + p) * P + q] = pre.fresh(tr, v, tid, b);
                }
        }
    }
    wave_sync();
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

        // ---- (1) rows: D, G, F rows from the next-row area, E rows from registers
        {
            const double *src = L.nxt + (t < NROW ? t : C::ZROW) * P;
#pragma unroll
            for (int m = 0; m < BP; ++m) {
                const double x = src[m];
                row[m] = isE ? pre.cr[m] : x;
            }
            if (FWD) {
                const double *lw = L.w + (isD ? t : 0) * RP;
#pragma unroll
                for (int j = 0; j < NR; ++j) {
                    const double x = lw[j] + (pre.r1[j] + pre.r2[j]);
                    w[j] = isD ? x : (isE ? 0.0 : w[j]);
                }
            }
        }
        wave_sync();
        // ---- (2) the previous stage's outputs leave, the next stage's blocks arrive
        if (i > 0) {
            const int ps = ch.stage(i - 1);
            lstore<MB, true>(F + sd.oLd + (long long)ps * b2, L.pnl + C::RD * P, P, b, b, erd, ecd);
            lstore<MB>(F + ch.coup_off(i - 1), L.pnl + C::RE * P, P, b, b, erd, ecd);
            if (ng) lstore<MG>(F + sd.oLb + (long long)ps * ng * b, L.pnl + C::RG * P, P, ng, b, er, ec);
            if (hasF) lstore<MB>(F + ch.fill_off(i - 1), L.pnl + C::RF * P, P, b, b, erd, ecd);
            if (FWD) lstore<2>(a.rhs + sd.oRhs + (long long)ps * b * nr, L.y, RP, b, nr, yr, yc);
        }
        if (!last) pre.load(ch, i + 1, FWD, t);

        // ---- (3) elimination (Algorithm 1 potrf / trsm, Algorithm 2)
        double myinv = 1.0;
        lelim<BP, NR, FWD, 0>(row, w, myinv, t);
        if (any_bad_pivot(t < b, myinv) && !failed) failed = gs + 1;

        // ---- (4) rows to LDS: the Gram's operands, the factor rows and y for their stores
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
                // -hat E y: the next stage's rhs once r_{i+1} is added (at a segment
                // end -hat F_k y, for the scratch)
                const int r = t - BP;
#pragma unroll
                for (int j = 0; j < NR; ++j) L.w[r * RP + j] = w[j];
            }
        }
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
                            const double fv = endS ? 0.0 : pre.fresh(tr, v, t, b);
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
            if (FWD) lstore<2>(sc + scr_dy(b, ng, nr), L.w, RP, b, nr, yr, yc);
        }
    }

    // ---- epilogue: the last stage's outputs, the running sums and the partials
    {
        const int ps = ch.stage(len - 1);
        lstore<MB, true>(F + sd.oLd + (long long)ps * b2, L.pnl + C::RD * P, P, b, b, erd, ecd);
        if (ch.has_next(len - 1)) lstore<MB>(F + ch.coup_off(len - 1), L.pnl + C::RE * P, P, b, b, erd, ecd);
        if (ng) lstore<MG>(F + sd.oLb + (long long)ps * ng * b, L.pnl + C::RG * P, P, ng, b, er, ec);
        if (hasF) lstore<MB>(F + ch.fill_off(len - 1), L.pnl + C::RF * P, P, b, b, erd, ecd);
        if (FWD) lstore<2>(a.rhs + sd.oRhs + (long long)ps * b * nr, L.y, RP, b, nr, yr, yc);
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
// The factor rows of stage j on their lanes (the D row without its diagonal, which
// comes separately), fetched from HBM, and the D lanes' rhs rows (RED: plus -hat F y).
template <int BP, int NR, bool RED>
struct LaneRowPre {
    double row[BP], diag, r1[NR], r2[NR];

    __device__ __forceinline__ void load(const WChain<RED> &ch, int j, bool hasF, int t)
    {
        const Args &a = ch.a;
        const SysDesc &sd = ch.sd;
        const int b = sd.b, ng = sd.ng, nr = a.nr, s = ch.stage(j);
        const long long b2 = (long long)b * b;
        const bool hasE = ch.has_next(j);
        const bool isD = t < BP, isE = t >= BP && t < 2 * BP, isG = t >= 2 * BP && t < 2 * BP + NGM;
        const int r = isD ? t : (isE ? t - BP : (isG ? t - 2 * BP : t - 2 * BP - NGM));
        const bool isF = hasF && t >= 2 * BP + NGM && r < BP;
        const bool ok = isD ? r < b : (isE ? hasE && r < b : (isG ? r < ng : isF && r < b));
        const long long off = isD ? sd.oLd + s * b2
                                  : (isE ? ch.coup_off(j) : (isG ? sd.oLb + (long long)s * ng * b : (isF ? ch.fill_off(j) : 0)));
        const double *src = a.F + off;
        const int ro = ok ? r * b : 0;
#pragma unroll
        for (int m = 0; m < BP; ++m) row[m] = ld_or_zero(src, ro + m, ok && m < b && !(isD && m == t));
        const bool dd = isD && t < b;
        diag = dd ? ld_or_zero(src, ro + t, dd) : 1.0;
        const double *Rp = a.rhs + sd.oRhs + (long long)s * b * nr;
        const double *sc = RED ? ch.scr(j + 1) : a.F;
        const int rr = dd ? t * nr : 0;
#pragma unroll
        for (int jj = 0; jj < NR; ++jj) {
            r1[jj] = ld_or_zero(Rp, rr + jj, dd && jj < nr);
            r2[jj] = RED ? ld_or_zero(sc + scr_dy(b, ng, nr), rr + jj, dd && jj < nr) : 0.0;
        }
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
    constexpr int RP = C::RP;
    const WChain<RED> ch{a, sd, k};
    const int b = sd.b, ng = sd.ng, nr = a.nr;
    const bool hasF = !RED && k > 1;
    const int len = ch.length();
    const int sep = hasF ? sep_of(sd, k) : 0;
    const int tid = threadIdx.x;
    int yr[2], yc[2];
    {
        const float invr = 1.0f / (float)nr;
#pragma unroll
        for (int m = 0; m < 2; ++m) rc_of(tid + 64 * m, nr, invr, yr[m], yc[m]);
    }
    for (int e = tid; e < C::BPX * RP; e += 64) L.w[e] = 0.0;
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
    double row[BP];
    for (int i = 0; i < len; ++i) {
        const bool hasE = ch.has_next(i);
        const bool last = i == len - 1;
        const bool endS = !RED && last && hasE;
        const int t = opaque_tid();
        const bool isD = t < BP;
        const bool isE = t >= BP && t < 2 * BP;
#pragma unroll
        for (int m = 0; m < BP; ++m) row[m] = pre.row[m];
        const double diag = pre.diag;
        {
            const double *lw = L.w + (isD ? t : 0) * RP;
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                const double x = lw[j] + (pre.r1[j] + pre.r2[j]);
                w[j] = isD ? x : (isE ? 0.0 : w[j]);
            }
        }
        wave_sync();
        if (i > 0) lstore<2>(a.rhs + sd.oRhs + (long long)ch.stage(i - 1) * b * nr, L.y, RP, b, nr, yr, yc);
        if (!last) pre.load(ch, i + 1, hasF, t);
        const double myinv = 1.0 / diag;
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
        wave_sync();
        if (endS) lstore<2>(ch.scr(k) + scr_dy(b, ng, nr), L.w, RP, b, nr, yr, yc);
    }
    lstore<2>(a.rhs + sd.oRhs + (long long)ch.stage(len - 1) * b * nr, L.y, RP, b, nr, yr, yc);
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
// The factor blocks of stage i (lane-contiguous element loads) and its y rows
// (with PRIMAL the primal solution rows too), committed to the staging area: L
// without its diagonal (which goes to a vector), hat E, hat G, the fill rows.
template <int BP, int NR, bool RED>
struct LaneColPre {
    static constexpr int MB = BP * BP / 64, MG = NGM * BP / 64;
    double d[MB], e[MB], f[MB], g[MG], y[2], px[2];

    template <bool PRIMAL>
    __device__ __forceinline__ void load(const WChain<RED> &ch, int i, bool hasF, int t, const int (&er)[MG],
                                         const int (&ec)[MG], const int (&yr)[2], const int (&yc)[2])
    {
        const Args &a = ch.a;
        const SysDesc &sd = ch.sd;
        const int b = sd.b, ng = sd.ng, nr = a.nr, s = ch.stage(i);
        const long long b2 = (long long)b * b;
        const bool hasE = ch.has_next(i);
        const double *Ld = a.F + sd.oLd + s * b2, *Le = a.F + ch.coup_off(i);
        const double *Lb = a.F + sd.oLb + (long long)s * ng * b;
        const double *Lf = a.F + (hasF ? ch.fill_off(i) : 0);
        const double *Y = a.rhs + sd.oRhs + (long long)s * b * nr;
        const double *XP = PRIMAL ? a.xp + sd.oRhs + (long long)s * b * nr : Y;
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            const bool in = er[m] < b;
            const int x = in ? er[m] * b + ec[m] : 0;
            d[m] = ld_or_zero(Ld, x, in);
            e[m] = ld_or_zero(Le, x, hasE && in);
            f[m] = ld_or_zero(Lf, x, hasF && in);
        }
#pragma unroll
        for (int m = 0; m < MG; ++m) {
            const bool in = er[m] < ng;
            g[m] = ld_or_zero(Lb, in ? er[m] * b + ec[m] : 0, in);
        }
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const bool in = yr[m] < b;
            const int x = in ? yr[m] * nr + yc[m] : 0;
            y[m] = ld_or_zero(Y, x, in);
            px[m] = PRIMAL ? ld_or_zero(XP, x, in) : 0.0;
        }
    }

    template <bool PRIMAL>
    __device__ __forceinline__ void commit(double *area, double *dv, double *Yl, double *Pl, int b, const int (&er)[MG],
                                           const int (&ec)[MG], const int (&yr)[2], const int (&yc)[2]) const
    {
        using C = WC<BP>;
        constexpr int P = C::P;
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            if (er[m] < b) {
                const int rr = er[m], cc = ec[m];
                area[(C::RD + rr) * P + cc] = (rr == cc) ? 0.0 : d[m];
                if (rr == cc) dv[rr] = d[m];
                area[(C::RE + rr) * P + cc] = e[m];
                area[(C::RF + rr) * P + cc] = f[m];
            }
        }
#pragma unroll
        for (int m = 0; m < MG; ++m)
            if (er[m] < NGM) area[(C::RG + er[m]) * P + ec[m]] = g[m];
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            if (yr[m] < b) {
                Yl[yr[m] * C::RP + yc[m]] = y[m];
                if (PRIMAL) Pl[yr[m] * C::RP + yc[m]] = px[m];
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
    constexpr int P = C::P, RP = C::RP, BPX = C::BPX, MG = NGM * BP / 64;
    const WChain<RED> ch{a, sd, k};
    const int b = sd.b, ng = sd.ng, nr = a.nr, N = sd.N;
    const long long b2 = (long long)b * b;
    const bool hasF = !RED && k > 1;
    const int len = ch.length();
    const int sep = hasF ? sep_of(sd, k) : 0;
    double *X = a.rhs + sd.oRhs;
    const double *XP = ADJ ? a.xp + sd.oRhs : X;
    double *xn = L.xn, *xc = L.xc, *pn = L.pn, *pc = L.pc;
    double *area = L.pnl;
    double *dv = L.dinv;
    const int tid = threadIdx.x;
    int er[MG], ec[MG], yr[2], yc[2];
    {
        const float invb = 1.0f / (float)b, invr = 1.0f / (float)nr;
#pragma unroll
        for (int m = 0; m < MG; ++m) rc_of(tid + 64 * m, b, invb, er[m], ec[m]);
#pragma unroll
        for (int m = 0; m < 2; ++m) rc_of(tid + 64 * m, nr, invr, yr[m], yc[m]);
    }
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
    pre.template load<ADJ>(ch, len - 1, hasF, tid, er, ec, yr, yc);
    wave_sync();
    for (int i = len - 1; i >= 0; --i) {
        const int gs = ch.stage(i);
        const bool hasE = ch.has_next(i);
        const int t = opaque_tid();
        // ---- (1) stage i's blocks and y into the staging area; x of the stage
        // after it leaves; stage i - 1's blocks arrive
        pre.template commit<ADJ>(area, dv, xc, pc, b, er, ec, yr, yc);
        wave_sync();
        if (i < len - 1) lstore<2>(X + (long long)ch.stage(i + 1) * b * nr, xn, RP, b, nr, yr, yc);
        if (i > 0) pre.template load<ADJ>(ch, i - 1, hasF, t, er, ec, yr, yc);
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
    lstore<2>(X + (long long)ch.stage(0) * b * nr, xn, RP, b, nr, yr, yc);
    wave_sync();
}

}  // namespace kkt_dev
