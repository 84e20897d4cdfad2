// Dense single-wave stage sweep for whole (p = 1) systems with block sizes 9..32
// (gfx950, FP64).  One 64-lane wave per system; no workgroup barriers.
//
// Per stage i of the sequential block Cholesky (Algorithm 1 with p = 1):
//   1. L = chol(Dw) and L^{-1} in one pass: lanes [0, DB) hold the rows of Dw and
//      eliminate them (right-looking); lanes [DB, 2DB) hold the columns of the
//      identity and run the same updates, which is the forward substitution
//      L X = I column by column (both use the same broadcast column of L).
//   2. hat E = C L^{-T} and hat G = Gw L^{-T} as products with the explicit
//      inverse on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
//   3. Forward substitution y = L^{-1} w and the rhs of the next stage
//      w' = r_{i+1} - hat E y, arrow part y_g -= hat G y (Algorithm 2, Eqs. 9a-9c).
//   4. Gram (Eqs. 4, 6): Dw' = sym(D_{i+1}) - hat E hat E^T (lower tiles),
//      Gw' = B_{i+1} - hat G hat E^T, R_acc -= hat G hat G^T, on the matrix cores.
// C_i is loaded from HBM straight into MFMA operand layout before the block is
// factored, and the next stage's blocks into accumulator layout before the
// forward substitution, so their latency overlaps computation.
//
// MFMA 16x16x4 FP64 lane layout (gfx950): A[i][k] in lane i + 16 k, B[k][j] in
// lane j + 16 k, D[4 v + lane / 16][lane % 16] in element v of lane `lane`.
#pragma once
#include "kkt_device.h"

namespace kkt_dev {

typedef double dx4 __attribute__((ext_vector_type(4)));

// Phase boundary: the scheduler may not move instructions across it, so the live
// ranges of consecutive phases of a stage do not overlap.
__device__ __forceinline__ void phase_fence() { __builtin_amdgcn_sched_barrier(0); }

__device__ __forceinline__ dx4 mfma4(double a, double b, dx4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// sqrt(x) and 1/sqrt(x) from the hardware reciprocal square root refined by two
// Goldschmidt iterations (g -> sqrt(x), h -> 1/(2 sqrt(x))); for x > 0 finite the
// result is within a few ulp of the correctly rounded values.
__device__ __forceinline__ void sqrt_rsqrt(double x, double &d, double &inv)
{
    const double y0 = __builtin_amdgcn_rsq(x);
    double g = x * y0, h = 0.5 * y0;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    d = g;
    inv = h + h;
}

// Dense LDS layout: a panel area of (2 DB + 16) rows with pitch DB + 1 (the
// backward sweep and the corner reuse it as their staging area), then the same
// small vectors as the general layout.  Regions the p = 1 path never touches
// (fill-row accumulators) alias the panel area.
__host__ __device__ __forceinline__ LdsOff lds_offsets_dense(int DB, int nr)
{
    LdsOff o;
    const int PITCH = DB + 1;
    int t = 0;
    o.col = t; t += 2 * (DB > NGM ? DB : NGM);
    o.P = t;   t += (2 * DB + NGM) * PITCH;
    o.A = o.P; o.Q = o.P; o.RP = o.P;
    o.R = t;   t += NGM * NGM;
    o.W = t;   t += (DB > NGM ? DB : NGM) * nr;
    o.Y = t;   t += (DB > NGM ? DB : NGM) * nr;
    o.XN = t;  t += DB * nr;
    o.XS = t;  t += 0;
    o.XC = t;  t += DB * nr;
    o.XG = t;  t += NGM * nr;
    o.PN = t;  t += DB * nr;
    o.PS = t;  t += 0;
    o.PC = t;  t += DB * nr;
    o.PG = t;  t += NGM * nr;
    o.misc = t; t += 8;
    o.total = t;
    return o;
}

__device__ __forceinline__ Lds make_lds_dense(double *base, int DB, int nr)
{
    const LdsOff o = lds_offsets_dense(DB, nr);
    Lds L;
    L.col = base + o.col; L.P = base + o.P; L.A = base + o.A; L.Q = base + o.Q; L.R = base + o.R;
    L.W = base + o.W; L.Y = base + o.Y; L.RP = base + o.RP; L.XN = base + o.XN; L.XS = base + o.XS;
    L.XC = base + o.XC; L.XG = base + o.XG; L.PN = base + o.PN; L.PS = base + o.PS; L.PC = base + o.PC;
    L.PG = base + o.PG; L.misc = reinterpret_cast<int *>(base + o.misc);
    return L;
}

// Factor (and with FWD forward-substitute) a whole system with one wave.  Writes
// the factor blocks, y in place of the rhs, and the arrow partials (-sum hat G
// hat G^T, -sum hat G y) to the scratch of segment 1, exactly as the general
// sweep does for p = 1.  Returns the 1-based index of the first stage whose pivot
// is not positive and finite, 0 if none.
template <int DB, bool FWD>
__device__ __forceinline__ int dense_factor(const Args &a, const SysDesc &sd, const Lds &L)
{
    constexpr int PD = DB + 1, TB = DB / 16, KS = DB / 4, NTL = 64;
    static_assert(DB == 16 || DB == 32, "dense sweep tiles are 16 or 32 wide");
    const int lane = threadIdx.x;
    const int b = sd.b, ng = sd.ng, nr = a.nr, N = sd.N;
    const long long b2 = (long long)b * b;
    double *F = a.F;
    double *RA = L.P;                 // Dw -> L (store staging) -> hat E -> next Dw
    double *RB = L.P + DB * PD;       // L^{-1}
    double *RG = L.P + 2 * DB * PD;   // Gw -> hat G -> next Gw (16 rows)
    double *buf0 = L.col, *buf1 = L.col + DB;

    // ---- prologue: Dw = sym(D_0), Gw = B_0, w = r_0, y_g partial = 0
    {
        const double *D0 = a.D + sd.oD;
        for (int e = lane; e < DB * DB; e += NTL) {
            const int r = e / DB, c = e - r * DB;
            RA[r * PD + c] = (r < b && c < b) ? 0.5 * (D0[r * b + c] + D0[c * b + r]) : (r == c ? 1.0 : 0.0);
        }
        const double *B0 = a.B + sd.oB;
        for (int e = lane; e < NGM * DB; e += NTL) {
            const int q = e / DB, c = e - q * DB;
            RG[q * PD + c] = (q < ng && c < b) ? B0[q * b + c] : 0.0;
        }
        if (FWD) {
            for (int e = lane; e < DB * nr; e += NTL) L.W[e] = (e < b * nr) ? a.rhs[sd.oRhs + e] : 0.0;
            for (int e = lane; e < NGM * nr; e += NTL) L.XG[e] = 0.0;
        }
    }
    wave_sync();

    dx4 accR = {0.0, 0.0, 0.0, 0.0};
    int failed = 0;
    for (int i = 0; i < N; ++i) {
        const bool hasN = i + 1 < N;
        // lane-derived indices and masks are re-derived every stage: hoisting the
        // unrolled per-element addresses and predicates out of the stage loop would
        // keep hundreds of them live across it
        int lane_s = lane;
        asm volatile("" : "+v"(lane_s));
        const int li = lane_s & 15, lk = lane_s >> 4;
        const bool isP = lane_s < DB;
        const bool isI = lane_s >= DB && lane_s < 2 * DB;
        const int ri = isP ? lane_s : lane_s - DB;

        // ---- (0) C_i in MFMA operand layout, in flight during the factorization
        double cA[TB][KS];
        const double *Ci = a.C + sd.oC + (long long)i * b2;
#pragma unroll
        for (int rt = 0; rt < TB; ++rt)
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) {
                const int r = 16 * rt + li, c = 4 * kk + lk;
                cA[rt][kk] = (hasN && r < b && c < b) ? Ci[r * b + c] : 0.0;
            }
        phase_fence();
        // ---- (1) L = chol(Dw) on the row lanes, L^{-1} on the column lanes
        double vec[DB];
        {
            const double *rowp = RA + (isP ? ri : 0) * PD, *colp = RA + (isP ? ri : 0);
#pragma unroll
            for (int c = 0; c < DB; ++c) {
                const double lo = rowp[c], up = colp[c * PD];
                vec[c] = isP ? ((c <= ri) ? lo : up) : ((isI && c == ri) ? 1.0 : 0.0);
            }
        }
        bool bad = false;
        if (isP) buf0[ri] = vec[0];
        wave_sync();
#pragma unroll
        for (int c = 0; c < DB; ++c) {
            double *cur = (c & 1) ? buf1 : buf0;
            double *nxt = (c & 1) ? buf0 : buf1;
            const double dcc = cur[c];
            bad |= !(dcc > 0.0) || !isfinite(dcc);
            double d, inv;
            sqrt_rsqrt(dcc, d, inv);
            double f = 0.0;
            if (isP) {
                if (ri == c) vec[c] = d;
                else if (ri > c) { const double v = vec[c] * inv; vec[c] = v; f = v * inv; }
            } else if (isI && ri <= c) {
                const double x = vec[c] * inv;
                vec[c] = x;
                f = x * inv;
            }
            if (c + 1 < DB) {
                // the next pivot column first, so its broadcast overlaps the rest
                vec[c + 1] = fma(-f, cur[c + 1], vec[c + 1]);
                if (isP && ri >= c + 1) nxt[ri] = vec[c + 1];
#pragma unroll
                for (int l = c + 2; l < DB; ++l) vec[l] = fma(-f, cur[l], vec[l]);
            }
            pin_row<DB>(vec);
            wave_sync();
        }
        if (bad && !failed) failed = i + 1;

        phase_fence();
        // ---- (2) L rows and L^{-1} columns into LDS; store L
        if (isP) {
#pragma unroll
            for (int c = 0; c < DB; ++c) RA[ri * PD + c] = (c <= ri) ? vec[c] : 0.0;
        } else if (isI) {
#pragma unroll
            for (int r = 0; r < DB; ++r) RB[r * PD + ri] = (r >= ri) ? vec[r] : 0.0;
        }
        wave_sync();
        store_block<NTL, DB * DB>(F + sd.oLd + (long long)i * b2, RA, PD, b, b);
        wave_sync();

        phase_fence();
        // ---- (3) hat E = C L^{-T}, hat G = Gw L^{-T}
        dx4 accE[TB][TB], accG[TB];
#pragma unroll
        for (int ct = 0; ct < TB; ++ct) {
            accG[ct] = dx4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int rt = 0; rt < TB; ++rt) accE[rt][ct] = dx4{0.0, 0.0, 0.0, 0.0};
        }
        // B operand: L^{-T}[k][j] = L^{-1}[j][k]
        if (hasN) {
#pragma unroll
            for (int kk = 0; kk < KS; ++kk)
#pragma unroll
                for (int ct = 0; ct < TB; ++ct) {
                    const double bo = RB[(16 * ct + li) * PD + 4 * kk + lk];
#pragma unroll
                    for (int rt = 0; rt < TB; ++rt) accE[rt][ct] = mfma4(cA[rt][kk], bo, accE[rt][ct]);
                }
        }
        if (ng) {
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) {
                const double ga = RG[li * PD + 4 * kk + lk];
#pragma unroll
                for (int ct = 0; ct < TB; ++ct) accG[ct] = mfma4(ga, RB[(16 * ct + li) * PD + 4 * kk + lk], accG[ct]);
            }
        }
        wave_sync();
#pragma unroll
        for (int ct = 0; ct < TB; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = 16 * ct + li;
#pragma unroll
                for (int rt = 0; rt < TB; ++rt) RA[(16 * rt + 4 * v + lk) * PD + c] = accE[rt][ct][v];
                RG[(4 * v + lk) * PD + c] = accG[ct][v];
            }
        wave_sync();
        if (hasN) store_block<NTL, DB * DB>(F + sd.oLc + (long long)i * b2, RA, PD, b, b);
        if (ng) store_block<NTL, NGM * DB>(F + sd.oLb + (long long)i * ng * b, RG, PD, ng, b);

        phase_fence();
        // ---- next stage's blocks, in flight during the forward substitution
        // lower tiles (rt >= ct) of sym(D_{i+1}) in accumulator layout
        constexpr int NLT = TB * (TB + 1) / 2;
        double dn[NLT][4], dt[NLT][4];
        const double *Dn = a.D + sd.oD + (long long)(i + 1) * b2;
#pragma unroll
        for (int rt = 0, t = 0; rt < TB; ++rt)
#pragma unroll
            for (int ct = 0; ct <= rt; ++ct, ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * rt + 4 * v + lk, c = 16 * ct + li;
                    const bool in = hasN && r < b && c < b;
                    dn[t][v] = in ? Dn[r * b + c] : 0.0;
                    dt[t][v] = in ? Dn[c * b + r] : 0.0;
                }
        double bn[TB][4];
        const double *Bn = a.B + sd.oB + (long long)(i + 1) * ng * b;
#pragma unroll
        for (int ct = 0; ct < TB; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int q = 4 * v + lk, c = 16 * ct + li;
                bn[ct][v] = (hasN && q < ng && c < b) ? Bn[q * b + c] : 0.0;
            }
        constexpr int RM = (DB * MAX_NRHS_DEV + NTL - 1) / NTL;
        double rn[RM];
        if (FWD) {
            const double *rs = a.rhs + sd.oRhs + (long long)(i + 1) * b * nr;
#pragma unroll
            for (int m = 0; m < RM; ++m) {
                const int e = lane + m * NTL;
                rn[m] = (hasN && e < b * nr) ? rs[e] : 0.0;
            }
        }


        phase_fence();
        // ---- (4) forward substitution: y = L^{-1} w, w' = r_{i+1} - hat E y, y_g -= hat G y
        if (FWD) {
            for (int e = lane; e < DB * nr; e += NTL) {
                const int r = e / nr, j = e - r * nr;
                double s = 0.0;
                for (int k = 0; k <= r; ++k) s = fma(RB[r * PD + k], L.W[k * nr + j], s);
                L.Y[e] = s;
                if (r < b) a.rhs[sd.oRhs + (long long)i * b * nr + e] = s;
            }
            wave_sync();
            for (int e = lane; e < ng * nr; e += NTL) {
                const int q = e / nr, j = e - q * nr;
                double s = 0.0;
                for (int k = 0; k < b; ++k) s = fma(RG[q * PD + k], L.Y[k * nr + j], s);
                L.XG[e] -= s;
            }
#pragma unroll
            for (int m = 0; m < RM; ++m) {
                const int e = lane + m * NTL;
                if (e < DB * nr) {
                    const int r = e / nr, j = e - r * nr;
                    double s = 0.0;
                    for (int k = 0; k < b; ++k) s = fma(RA[r * PD + k], L.Y[k * nr + j], s);
                    L.W[e] = (r < b) ? rn[m] - s : 0.0;
                }
            }
        }

        phase_fence();
        // ---- (5) Gram: next Dw and Gw, arrow accumulator
        dx4 accD[NLT], accB[TB];
#pragma unroll
        for (int rt = 0, t = 0; rt < TB; ++rt)
#pragma unroll
            for (int ct = 0; ct <= rt; ++ct, ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * rt + 4 * v + lk, c = 16 * ct + li;
                    accD[t][v] = (r < b && c < b) ? 0.5 * (dn[t][v] + dt[t][v]) : (r == c ? 1.0 : 0.0);
                }
#pragma unroll
        for (int ct = 0; ct < TB; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) accB[ct][v] = bn[ct][v];
        if (hasN) {
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) {
                double ek[TB];
#pragma unroll
                for (int t = 0; t < TB; ++t) ek[t] = RA[(16 * t + li) * PD + 4 * kk + lk];
#pragma unroll
                for (int rt = 0, t = 0; rt < TB; ++rt)
#pragma unroll
                    for (int ct = 0; ct <= rt; ++ct, ++t) accD[t] = mfma4(-ek[rt], ek[ct], accD[t]);
            }
        }
        if (ng) {
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) {
                const double gk = RG[li * PD + 4 * kk + lk];
                if (hasN) {
#pragma unroll
                    for (int ct = 0; ct < TB; ++ct)
                        accB[ct] = mfma4(-gk, RA[(16 * ct + li) * PD + 4 * kk + lk], accB[ct]);
                }
                accR = mfma4(-gk, gk, accR);
            }
        }
        wave_sync();
        if (hasN) {
#pragma unroll
            for (int rt = 0, t = 0; rt < TB; ++rt)
#pragma unroll
                for (int ct = 0; ct <= rt; ++ct, ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v) RA[(16 * rt + 4 * v + lk) * PD + 16 * ct + li] = accD[t][v];
#pragma unroll
            for (int ct = 0; ct < TB; ++ct)
#pragma unroll
                for (int v = 0; v < 4; ++v) RG[(4 * v + lk) * PD + 16 * ct + li] = accB[ct][v];
        }
        wave_sync();
    }

    // ---- epilogue: arrow partials into the scratch of segment 1
    if (ng) {
        const int li = lane & 15, lk = lane >> 4;
        double *sc = F + sd.oScr;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int q = 4 * v + lk;
            if (q < ng && li < ng) sc[scr_Rk(b, ng, nr) + q * ng + li] = accR[v];
        }
        if (FWD)
            for (int e = lane; e < ng * nr; e += NTL) sc[scr_yg(b, ng, nr) + e] = L.XG[e];
    }
    wave_sync();
    return failed;
}

}  // namespace kkt_dev
