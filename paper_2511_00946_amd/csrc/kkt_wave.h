// Barrier-free row-lane stage sweeps of the segmented block Cholesky (gfx950, FP64).
//
// One workgroup of NW 64-lane waves processes one work item: a segment of one
// system (Algorithm 1, 2 and 3, parallel phases), the reduced separator chain of
// one system (the sequential phases, Eq. 7) or a whole system (p = 1).  Every
// thread holds one row of the tall panel of a stage in registers:
//   D rows  the working diagonal block (its Cholesky factor after the step)
//   E rows  the coupling rows to the next pivot: C_i -> hat E (hat F_k at the end
//           of a segment k < p, hat H_k on the reduced chain)
//   G rows  the arrow rows: G_w -> hat G (hat Q_k on the reduced chain)
//   F rows  the separator fill rows of a segment k >= 2: F_w -> hat B^T_{ik}
// Placement: with BP <= 16 all 3 BP + 16 rows fit one wave (D at lanes [0, BP),
// E at [BP, 2BP), G at [2BP, 2BP + 16), F after them).  With wider blocks, wave 0
// holds the D and G rows and the E and F rows sit in further waves.
//
// Per stage of a factor sweep:
//   1. elimination of wave 0 (right-looking, one column per step): the pivot and
//      the pivot row are broadcast from lane c with readlane (no LDS round trip,
//      no barrier), so hat D = chol(D_w) and the panel rows P hat D^{-T} (the trsm
//      of Algorithm 1) come out of one sweep; the right-hand sides ride along as
//      extra columns (forward substitution of Algorithm 2: y = hat D^{-1} w, and
//      the E, G and F rows accumulate -hat E y, -hat G y and -hat B^T y).  Further
//      waves solve their rows against hat D from LDS after one barrier.
//   2. the factor rows go to LDS and leave for HBM with lane-contiguous stores.
//   3. Gram of the panel rows (Eqs. 4, 6, 8a, 8b): every thread dots its own row
//      with the rows of hat E, hat G and hat B^T read from LDS as broadcasts, which
//      gives the next diagonal block (E threads), the next arrow rows (G threads),
//      the next fill rows and hat A_k (F threads), hat R_k and hat Q_k (G threads).
// The blocks of the next stage are fetched into registers (lane-contiguous,
// branch-free loads) when a stage starts, and reach LDS before its Gram.
//
// Padding: a block of size b < BP is embedded with identity on the padded
// diagonal and zeros elsewhere; this is exact.
#pragma once
#include "kkt_device.h"

namespace kkt_dev {

template <int BP>
struct WC {
    static constexpr int NW = BP <= 16 ? 1 : (BP <= 32 ? 2 : 3);
    static constexpr int NT = 64 * NW;
    static constexpr int P = BP + 1;                 // LDS row pitch (doubles)
    static constexpr int NROW = 3 * BP + NGM;        // panel rows
    static constexpr int RD = 0, RE = BP, RG = 2 * BP, RF = 2 * BP + NGM;   // LDS row of each group
    static constexpr int TG = NW == 1 ? 2 * BP : BP;                       // first thread of each group
    static constexpr int TE = NW == 1 ? BP : 64;
    static constexpr int TF = NW == 1 ? 2 * BP + NGM : (NW == 2 ? 64 + BP : 128);
    static constexpr int WE = TE / 64, WF = TF / 64;
    static constexpr int BPX = BP > NGM ? BP : NGM;
    static constexpr int RP = 8;                     // pitch of right-hand-side rows in LDS
    static constexpr int ZROW = NROW, SROW = NROW + 1;   // next-row area: a row of zeros, a sink row
    static_assert(TF + BP <= NT && TG + NGM <= (NW == 1 ? NT : 64), "row placement");
};

// LDS layout in doubles.  The backward sweep reuses the panel area for its
// staged blocks and the next-row area for its vectors.
struct WaveLdsOff {
    int pnl, nxt, w, y, rn, dinv, acc_a, acc_q, racc, yg, misc, total;
    int xn, xc, xg, xs, pn, pc, pg, ps;
};

template <int BP>
__host__ __device__ constexpr WaveLdsOff wave_lds_offsets()
{
    using C = WC<BP>;
    WaveLdsOff o{};
    int t = 0;
    o.pnl = t; t += C::NROW * C::P;
    o.nxt = t;
    {
        const int vec = C::BPX * C::RP;
        o.xn = t; o.xc = t + vec; o.xs = t + 2 * vec; o.pn = t + 3 * vec; o.pc = t + 4 * vec; o.ps = t + 5 * vec;
        o.xg = t + 6 * vec; o.pg = o.xg + NGM * C::RP;
        const int bwd = 6 * vec + 2 * NGM * C::RP;
        const int fwd = (C::NROW + 2) * C::P;   // + a zero row (ZROW) and a sink row (SROW)
        t += (fwd > bwd ? fwd : bwd);
    }
    o.w = t;     t += C::BPX * C::RP;
    o.y = t;     t += C::BPX * C::RP;
    o.rn = t;    t += C::NW == 1 ? C::BPX * C::RP : 0;   // single-wave sweeps only
    o.dinv = t;  t += C::BPX;
    o.acc_a = t; t += BP * C::P;
    o.acc_q = t; t += NGM * C::P;
    o.racc = t;  t += NGM * (NGM + 1);
    o.yg = t;    t += NGM * C::RP;
    o.misc = t;  t += 4;
    o.total = t;
    return o;
}

struct WaveLds {
    double *pnl, *nxt, *w, *y, *rn, *dinv, *acc_a, *acc_q, *racc, *yg;
    double *xn, *xc, *xg, *xs, *pn, *pc, *pg, *ps;
    int *misc;
};

template <int BP>
__device__ __forceinline__ WaveLds make_wave_lds(double *base)
{
    constexpr WaveLdsOff o = wave_lds_offsets<BP>();
    WaveLds L;
    L.pnl = base + o.pnl; L.nxt = base + o.nxt; L.w = base + o.w; L.y = base + o.y; L.rn = base + o.rn;
    L.dinv = base + o.dinv;
    L.acc_a = base + o.acc_a; L.acc_q = base + o.acc_q; L.racc = base + o.racc; L.yg = base + o.yg;
    L.xn = base + o.xn; L.xc = base + o.xc; L.xg = base + o.xg; L.xs = base + o.xs;
    L.pn = base + o.pn; L.pc = base + o.pc; L.pg = base + o.pg; L.ps = base + o.ps;
    L.misc = reinterpret_cast<int *>(base + o.misc);
    return L;
}

template <int NW>
__device__ __forceinline__ void gsync()
{
    if (NW == 1) wave_sync();
    else __syncthreads();
}

// Where the blocks of one stage of a chain come from.
//   Segment chain (RED = false), local stage i of segment k: natural stage
//   seg_first(k) + i.
//   Reduced chain (RED = true), stage t <-> separator sep_{t+2}: the partial
//   tilde A (Ld[s]) minus hat F hat F^T of the segment before it, the coupling
//   tilde H_{t+2} to the next separator, tilde Q (Lb[s]) minus hat G hat F^T, and
//   the partial tilde y (rhs[s]) plus -hat F hat y (Eqs. 7, 8c, 9d).
template <bool RED>
struct WChain {
    const Args &a;
    const SysDesc &sd;
    int k;
    __device__ __forceinline__ int stage(int i) const { return RED ? sep_of(sd, i + 2) : seg_first(sd, k) + i; }
    __device__ __forceinline__ int length() const { return RED ? sd.p - 1 : seg_len(sd, k); }
    __device__ __forceinline__ bool has_next(int i) const { return RED ? (i + 2 < sd.p) : (stage(i) + 1 < sd.N); }
    __device__ __forceinline__ double *scr(int seg) const { return a.F + sd.oScr + (long long)(seg - 1) * sd.scrStride; }
    // coupling block of local stage i (hat E / hat F_k in the Lc slot, hat H on the reduced chain)
    __device__ __forceinline__ long long coup_off(int i) const
    {
        const long long b2 = (long long)sd.b * sd.b;
        return RED ? sd.oH + (long long)i * b2 : sd.oLc + (long long)stage(i) * b2;
    }
    // fill block of local stage i of a segment k >= 2 (hat B^T_{ik})
    __device__ __forceinline__ long long fill_off(int i) const
    {
        const long long b2 = (long long)sd.b * sd.b;
        return i == 0 ? sd.oLc + (long long)sep_of(sd, k) * b2
                      : sd.oFill + ((long long)(k - 2) * (sd.Nk - 1) + (i - 1)) * b2;
    }
};

// Lane-contiguous element e of a rows x cols row-major block (e < 2^16, cols <= 64).
__device__ __forceinline__ void rc_of(int e, int cols, float invc, int &r, int &c)
{
    r = row_of(e, invc);
    c = e - r * cols;
}

// Rows [R0, R0 + rows) x [0, cols) of an LDS area (pitch P) to a row-major global
// block, optionally transposed (dst[r][c] = lds[c][r]) and scaled; every LDS read
// before the first store.
template <int NT, int MAXE, bool TR = false>
__device__ __forceinline__ void wstore(double *dst, const double *lds, int P, int rows, int cols, int t,
                                       double scale = 1.0)
{
    constexpr int M = (MAXE + NT - 1) / NT;
    const int n = rows * cols;
    const float invc = 1.0f / (float)cols;
    double v[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int e = t + m * NT;
        int r, c;
        rc_of(e < n ? e : 0, cols, invc, r, c);
        v[m] = scale * (TR ? lds[c * P + r] : lds[r * P + c]);
    }
    pin_row<M>(v);
    const GBlock g(dst, n);   // stores past the block's end are dropped
#pragma unroll
    for (int m = 0; m < M; ++m) g.st((t + m * NT) * 8, v[m]);
}

// rhs rows (rows x nr, global pitch nr) from LDS (pitch RP).
template <int NT, int MAXR>
__device__ __forceinline__ void wstore_rhs(double *dst, const double *lds, int rows, int nr, int t)
{
    constexpr int M = (MAXR * MAX_NRHS_DEV + NT - 1) / NT;
    const int n = rows * nr;
    const float invc = 1.0f / (float)nr;
    double v[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int e = t + m * NT;
        int r, j;
        rc_of(e < n ? e : 0, nr, invc, r, j);
        v[m] = lds[r * MAX_NRHS_DEV + j];
    }
    pin_row<M>(v);
    const GBlock g(dst, n);   // stores past the block's end are dropped
#pragma unroll
    for (int m = 0; m < M; ++m) g.st((int)(threadIdx.x + m * NT) * 8, v[m]);
}

// The thread index behind an opaque copy: values derived from it inside a loop
// are recomputed there instead of being hoisted out of the loop and kept live
// (as masks in scalar registers) across it.
__device__ __forceinline__ int opaque_tid()
{
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// ---------------------------------------------------------------- elimination
// Right-looking elimination of the rows held by one wave.  Lanes [0, W) hold the
// full (symmetric) rows of the working diagonal block; lanes with `panel` set hold
// panel rows; every other lane holds zeros.  Step c broadcasts the pivot and the
// rest of row c of the updated block from lane c (by symmetry, row c right of the
// pivot is column c below it), so lane l > c and every panel lane update their
// rows with one FMA per column; the broadcasts are taken eight at a time, each
// group right before its FMAs (a scheduling barrier per group keeps the
// broadcast values from piling up in scalar registers).  After the call lanes
// [0, W) hold the rows of L (entries right of the diagonal are stale) and panel
// lanes the rows of P L^{-T}.  A pivot that is not positive and finite leaves a
// NaN on the diagonal (the reciprocal square root of a value <= 0, 0 or infinity
// makes sqrt_rsqrt return NaN), which the callers test once after the sweep
// (testing every pivot here would keep all of them live to the end).
// Step c of the elimination, then the steps after it: the steps are expanded by
// template recursion, so every row index is a compile-time constant for any W
// (a loop over the columns is too large to unroll for the widest blocks, and a
// rolled loop would index the row at run time and force it out of registers).
template <int W, int c>
__device__ __forceinline__ void elim_step(double (&row)[W], bool panel, int lane)
{
    if constexpr (c < W) {
        const double dcc = readlane_d(row[c], c);
        double d, inv;
        sqrt_rsqrt(dcc, d, inv);
        const bool below = (lane < W && lane > c) || panel;
        const double v = row[c] * inv;
        const double f = below ? v * inv : 0.0;
        row[c] = (lane == c) ? d : (below ? v : row[c]);
#pragma unroll
        for (int m0 = 0; m0 < W; m0 += 8) {
            if (m0 + 8 <= c + 1) continue;
            double sv[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int m = m0 + q;
                if (m > c && m < W) sv[q] = readlane_d(row[m], c);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int m = m0 + q;
                if (m > c && m < W) row[m] = fma(-f, sv[q], row[m]);
            }
            if (W > 16) __builtin_amdgcn_sched_barrier(0);
        }
        elim_step<W, c + 1>(row, panel, lane);
    }
}

template <int W>
__device__ __forceinline__ void elim_wave(double (&row)[W], bool panel, int lane)
{
    elim_step<W, 0>(row, panel, lane);
}

// True on every lane of the wave if any lane with `mine` set holds a diagonal
// entry that is not positive and finite.
__device__ __forceinline__ bool any_bad_pivot(bool mine, double d)
{
    return __any(mine && !(d > 0.0 && isfinite(d)));
}

// Rows held by a wave other than the pivot wave: P <- P L^{-T} against L in LDS
// (rows of pitch P, 1 / L_cc in dinv).  Lanes without a row hold zeros and stay
// zero.  Column steps expanded by template recursion.
template <int W, int c>
__device__ __forceinline__ void trsm_step(double (&row)[W], const double *Lr, int P, const double *dinv)
{
    if constexpr (c < W) {
        const double v = row[c] * dinv[c];
        row[c] = v;
        // the column index behind an opaque copy that depends on this step's
        // multiplier: the reads of column c cannot be issued before the step
        // (their addresses are otherwise constants, and every column's reads would
        // be issued at once and spilled)
        int cc = c;
        asm volatile("" : "+v"(cc) : "v"(v));
#pragma unroll
        for (int m0 = 0; m0 < W; m0 += 8) {
            if (m0 + 8 <= c + 1) continue;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int m = m0 + q;
                if (m > c && m < W) row[m] = fma(-v, Lr[m * P + cc], row[m]);
            }
            if (W > 16) __builtin_amdgcn_sched_barrier(0);
        }
        trsm_step<W, c + 1>(row, Lr, P, dinv);
    }
}

template <int W>
__device__ __forceinline__ void trsm_wave(double (&row)[W], const double *Lr, int P, const double *dinv)
{
    trsm_step<W, 0>(row, Lr, P, dinv);
}

// Forward substitution with a factor already in place: lanes [0, W) hold the rows
// of L and dinv = 1 / L_rr, panel lanes their panel rows: lane c ends with
// y_c = w_c / L_cc, lanes l > c and panel lanes subtract L_lc y_c (P_lc y_c).
// Column steps expanded by template recursion (constant indices for any W).
template <int W, int c>
__device__ __forceinline__ void fsub_step(const double (&row)[W], double (&w)[MAX_NRHS_DEV], int nr, bool panel, int lane,
                                          double dinv)
{
    if constexpr (c < W) {
        const double ic = readlane_d(dinv, c);
        const bool below = (lane < W && lane > c) || panel;
#pragma unroll
        for (int j = 0; j < MAX_NRHS_DEV; ++j) {
            if (j < nr) {
                const double yc = readlane_d(w[j], c) * ic;
                w[j] = (lane == c) ? yc : (below ? fma(-row[c], yc, w[j]) : w[j]);
            }
        }
        fsub_step<W, c + 1>(row, w, nr, panel, lane, dinv);
    }
}

template <int W>
__device__ __forceinline__ void fsub_wave(const double (&row)[W], double (&w)[MAX_NRHS_DEV], int nr, bool panel, int lane,
                                          double dinv)
{
    fsub_step<W, 0>(row, w, nr, panel, lane, dinv);
}

// Forward substitution of rows held by a wave other than the pivot wave:
// w -= P y with y in LDS (pitch RP).
template <int W>
__device__ __forceinline__ void fsub_rows(const double (&row)[W], double (&w)[MAX_NRHS_DEV], int nr, const double *Y)
{
#pragma unroll
    for (int j = 0; j < MAX_NRHS_DEV; ++j) {
        if (j < nr) {
            double acc = w[j];
#pragma unroll
            for (int c = 0; c < W; ++c) {
                acc = fma(-row[c], Y[c * MAX_NRHS_DEV + j], acc);
                if (W > 16 && (c & 7) == 7) __builtin_amdgcn_sched_barrier(0);
            }
            w[j] = acc;
        }
    }
}

// Back substitution L^T x = acc on lanes [0, W) of one wave: lane c holds
// dcs[l] = L[l][c] / L[c][c] (l >= c meaningful, zeros above) and acc_c / L_cc in
// accs.  Returns x_c.  Steps expanded by template recursion.
template <int W, int c2>
__device__ __forceinline__ void bsub_step(const double (&dcs)[W], double &accs, double &xv, int lane)
{
    if constexpr (c2 >= 0) {
        const double x2 = readlane_d(accs, c2);
        if (lane == c2) xv = x2;
        accs = fma(-dcs[c2], x2, accs);
        bsub_step<W, c2 - 1>(dcs, accs, xv, lane);
    }
}

template <int W>
__device__ __forceinline__ double bsub_wave(const double (&dcs)[W], double accs, int lane)
{
    double xv = 0.0;
    bsub_step<W, W - 1>(dcs, accs, xv, lane);
    return xv;
}

// Four dots of a register row with rows [0, 4) of an LDS block (pitch P).  Wide
// rows are read eight columns at a time behind scheduling barriers, so that the
// broadcast reads are not all hoisted ahead of the FMAs (which would hold 4 W
// values in registers at once).
template <int W>
__device__ __forceinline__ void dot4(const double (&row)[W], const double *B, int P, double (&s)[4])
{
    double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
#pragma unroll
    for (int c0 = 0; c0 < W; c0 += 8) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int c = c0 + q;
            if (c < W) {
                t0 = fma(row[c], B[c], t0);
                t1 = fma(row[c], B[P + c], t1);
                t2 = fma(row[c], B[2 * P + c], t2);
                t3 = fma(row[c], B[3 * P + c], t3);
            }
        }
        if (W > 16) __builtin_amdgcn_sched_barrier(0);
    }
    s[0] = t0; s[1] = t1; s[2] = t2; s[3] = t3;
}

// The same with the own row read from LDS (own, contiguous), eight entries at a
// time: used by the widest class, whose row registers would otherwise stay live
// through the Gram.
template <int W>
__device__ __forceinline__ void dot4_lds(const double *own, const double *B, int P, double (&s)[4])
{
    double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
#pragma unroll
    for (int c0 = 0; c0 < W; c0 += 8) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int c = c0 + q;
            if (c < W) {
                const double o = own[c];
                t0 = fma(o, B[c], t0);
                t1 = fma(o, B[P + c], t1);
                t2 = fma(o, B[2 * P + c], t2);
                t3 = fma(o, B[3 * P + c], t3);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    s[0] = t0; s[1] = t1; s[2] = t2; s[3] = t3;
}

// ---------------------------------------------------------------- stage loads
// The blocks of one stage of a factor chain, fetched into registers with
// lane-contiguous, branch-free loads (element e = thread + NT m; entries past a
// block read as zero), then written to the next-row area of LDS.
template <int BP, bool RED>
struct FacLoad {
    using C = WC<BP>;
    static constexpr int NT = C::NT;
    static constexpr int MB = (BP * BP + NT - 1) / NT;
    static constexpr int MG = (NGM * BP + NT - 1) / NT;
    static constexpr int MR = (BP * MAX_NRHS_DEV + NT - 1) / NT;
    static constexpr int MB2 = RED ? MB : 1, MG2 = RED ? MG : 1, MR2 = RED ? MR : 1;
    double d[MB], c[MB], g[MG], r[MR];
    double d2[MB2], g2[MG2], r2[MR2];

    __device__ __forceinline__ void load(const WChain<RED> &ch, int j, bool fwd, int t)
    {
        const Args &a = ch.a;
        const SysDesc &sd = ch.sd;
        const int b = sd.b, ng = sd.ng, nr = a.nr, s = ch.stage(j);
        const int b2 = b * b, gb = ng * b, rb = b * nr;
        const bool hasE = ch.has_next(j);
        if constexpr (BP <= 32) {
            // the blocks are read through buffer resources: entries past a block's end
            // (and every entry of an absent block) read as zero
            const GBlock gD(RED ? a.F + sd.oLd + (long long)s * b2 : a.D + sd.oD + (long long)s * b2, b2);
            const GBlock gC(RED ? a.F + ch.coup_off(j) : a.C + sd.oC + (long long)s * b2, hasE ? b2 : 0);
            const GBlock gB(RED ? a.F + sd.oLb + (long long)s * gb : a.B + sd.oB + (long long)s * gb, gb);
            const GBlock gR(a.rhs + sd.oRhs + (long long)s * rb, fwd ? rb : 0);
            const double *sc = RED ? ch.scr(j + 1) : a.rhs;
            const GBlock gsD(sc + (RED ? scr_dA(b, ng, nr) : 0), RED ? b2 : 0);
            const GBlock gsQ(sc + (RED ? scr_dQ(b, ng, nr) : 0), RED ? gb : 0);
            const GBlock gsY(sc + (RED ? scr_dy(b, ng, nr) : 0), RED && fwd ? rb : 0);
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                const int e = (t + m * NT) * 8;
                d[m] = gD.ld(e);
                c[m] = gC.ld(e);
                if (RED) d2[m] = gsD.ld(e);
            }
#pragma unroll
            for (int m = 0; m < MG; ++m) {
                const int e = (t + m * NT) * 8;
                g[m] = gB.ld(e);
                if (RED) g2[m] = gsQ.ld(e);
            }
#pragma unroll
            for (int m = 0; m < MR; ++m) {
                const int e = (t + m * NT) * 8;
                r[m] = gR.ld(e);
                if (RED) r2[m] = gsY.ld(e);
            }
        } else {
            // (the 48-wide tiles keep 64-bit addresses: their per-load offsets would
            // add to registers that already spill)
            const double *Dp = RED ? a.F + sd.oLd + (long long)s * b2 : a.D + sd.oD + (long long)s * b2;
            const double *Cp = RED ? a.F + ch.coup_off(j) : a.C + sd.oC + (long long)s * b2;
            const double *Bp = RED ? a.F + sd.oLb + (long long)s * gb : a.B + sd.oB + (long long)s * gb;
            const double *Rp = a.rhs + sd.oRhs + (long long)s * rb;
            const double *sc = RED ? ch.scr(j + 1) : nullptr;
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                const int e = t + m * NT;
                d[m] = ld_or_zero(Dp, e, e < b2);
                c[m] = ld_or_zero(Cp, e, hasE && e < b2);
                if (RED) d2[m] = ld_or_zero(sc + scr_dA(b, ng, nr), e, e < b2);
            }
#pragma unroll
            for (int m = 0; m < MG; ++m) {
                const int e = t + m * NT;
                g[m] = ld_or_zero(Bp, e, e < gb);
                if (RED) g2[m] = ld_or_zero(sc + scr_dQ(b, ng, nr), e, e < gb);
            }
#pragma unroll
            for (int m = 0; m < MR; ++m) {
                const int e = t + m * NT;
                r[m] = ld_or_zero(Rp, e, fwd && e < rb);
                if (RED) r2[m] = ld_or_zero(sc + scr_dy(b, ng, nr), e, fwd && e < rb);
            }
        }
    }

    // Add the D rows (RED: minus hat F hat F^T) and G rows (RED: minus hat G hat F^T)
    // to what the Gram left in nxt, put the E rows (if the stage has a coupling),
    // and add the rhs (RED: plus -hat F y) to w.
    __device__ __forceinline__ void commit(double *nxt, double *w, const SysDesc &sd, int nr, bool hasE, bool fwd,
                                          int t) const
    {
        constexpr int P = C::P;
        const int b = sd.b, ng = sd.ng, b2 = b * b, gb = ng * b, rb = b * nr;
        const float invb = 1.0f / (float)b, invr = 1.0f / (float)nr;
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            const int e = t + m * NT;
            if (e < b2) {
                int rr, cc;
                rc_of(e, b, invb, rr, cc);
                nxt[(C::RD + rr) * P + cc] += RED ? d[m] - d2[m] : d[m];
                if (hasE) nxt[(C::RE + rr) * P + cc] = c[m];
            }
        }
#pragma unroll
        for (int m = 0; m < MG; ++m) {
            const int e = t + m * NT;
            if (e < gb) {
                int rr, cc;
                rc_of(e, b, invb, rr, cc);
                nxt[(C::RG + rr) * P + cc] += RED ? g[m] - g2[m] : g[m];
            }
        }
        if (fwd) {
#pragma unroll
            for (int m = 0; m < MR; ++m) {
                const int e = t + m * NT;
                if (e < rb) {
                    int rr, j;
                    rc_of(e, nr, invr, rr, j);
                    w[rr * C::RP + j] += RED ? r[m] + r2[m] : r[m];
                }
            }
        }
    }
};

// ---------------------------------------------------------------- factor sweep
// Factor (and with FWD forward-substitute) one chain: segment k of a system
// (Algorithm 1 parallel phase, with Algorithm 2 parallel phase fused), the whole
// system when p = 1, or (RED) the reduced separator chain (Algorithm 1 / 2
// sequential phases, without the corner).  Writes the factor blocks in the input
// pattern, y in place of the rhs, and the partials the next phase reads: for a
// segment k >= 2 hat A_k, hat Q_k and the separator rhs (separator slots); for a
// segment ending on hat F_k (k < p) hat F_k hat F_k^T, hat G hat F_k^T, -hat F_k y
// and tilde H_k = -hat F_k hat B (Eqs. 8a-8c, 9b-9d); the arrow partials
// -sum hat G hat G^T and -sum hat G y in the segment's scratch (RED: in LDS,
// for the corner).  Returns the 1-based natural index of the first stage whose
// pivot failed, 0 if none (meaningful in thread 0).
template <int BP, bool FWD, bool RED>
__device__ __forceinline__ int wave_factor(const Args &a, const SysDesc &sd, int k, const WaveLds &L)
{
    using C = WC<BP>;
    constexpr int NT = C::NT, P = C::P, NW = C::NW, RP = C::RP;
    const WChain<RED> ch{a, sd, k};
    const int b = sd.b, ng = sd.ng, nr = a.nr;
    const int b2 = b * b;
    double *F = a.F;
    const bool hasF = !RED && k > 1;
    const int len = ch.length();
    const int sep = hasF ? sep_of(sd, k) : 0;

    // ---- prologue.  The next-row area holds the identity on the padded diagonal
    // (rows b..BP-1) and zeros everywhere else, so rows read from it need no
    // padding logic and the blocks of the first stage can be added to it; then the
    // accumulators (Algorithm 1 init: hat R_k = 0, hat A_k = A_k = sym(D_sep),
    // hat Q_k = Q_k = B_sep), the first fill rows F_w = Psi_{sep_k, first(k)} = C_sep^T
    // and the separator rhs.
    {
        const int t = threadIdx.x;
        for (int e = t; e < (C::NROW + 2) * P; e += NT) {
            const int rr = e / P, cc = e - rr * P;
            L.nxt[e] = (rr < BP && rr == cc && rr >= b) ? 1.0 : 0.0;
        }
        for (int e = t; e < C::BPX * RP; e += NT) L.w[e] = 0.0;
        for (int e = t; e < NGM * (NGM + 1); e += NT) L.racc[e] = 0.0;
        if (hasF) {
            for (int e = t; e < BP * P; e += NT) L.acc_a[e] = 0.0;
            for (int e = t; e < NGM * P; e += NT) L.acc_q[e] = 0.0;
        }
    }
    FacLoad<BP, RED> pf;
    pf.load(ch, 0, FWD, threadIdx.x);
    gsync<NW>();
    if (hasF) {
        const int t = threadIdx.x;
        const double *Ds = a.D + sd.oD + (long long)sep * b2, *Cs = a.C + sd.oC + (long long)sep * b2;
        const double *Bs = a.B + sd.oB + (long long)sep * ng * b;
        const float invb = 1.0f / (float)b;
        for (int e = t; e < b2; e += NT) {
            int rr, cc;
            rc_of(e, b, invb, rr, cc);
            L.acc_a[rr * P + cc] = 0.5 * (Ds[e] + Ds[cc * b + rr]);
            L.nxt[(C::RF + cc) * P + rr] = Cs[e];
        }
        for (int e = t; e < ng * b; e += NT) {
            int rr, cc;
            rc_of(e, b, invb, rr, cc);
            L.acc_q[rr * P + cc] = Bs[e];
        }
    }
    pf.commit(L.nxt, L.w, sd, nr, ch.has_next(0), FWD, threadIdx.x);
    double w[MAX_NRHS_DEV];
    {
        const int t = threadIdx.x;
        const bool isF = hasF && t >= C::TF && t < C::TF + BP;
        const int r = t - C::TF;
#pragma unroll
        for (int j = 0; j < MAX_NRHS_DEV; ++j) {
            double v = 0.0;
            if (FWD && j < nr && isF && r < b) v = a.rhs[sd.oRhs + ((long long)sep * b + r) * nr + j];
            w[j] = v;
        }
    }
    gsync<NW>();

    int failed = 0;
    double row[BP];
    for (int i = 0; i < len; ++i) {
        const int gs = ch.stage(i);
        const bool hasE = ch.has_next(i);
        const bool last = i == len - 1;
        const bool endS = !RED && last && hasE;   // segment k < p ends on hat F_k
        const bool nextD = hasE && !endS;
        // per-thread roles, re-derived every stage (see opaque_tid)
        const int t = opaque_tid(), wave = t >> 6, lane = t & 63;
        const bool isD = t < BP;
        const bool isE = t >= C::TE && t < C::TE + BP;
        const bool isG = t >= C::TG && t < C::TG + NGM;
        const bool isF = hasF && t >= C::TF && t < C::TF + BP;
        const int r = isD ? t : isE ? t - C::TE : isG ? t - C::TG : isF ? t - C::TF : 0;
        const int prow = isD ? C::RD + r : isE ? C::RE + r : isG ? C::RG + r : isF ? C::RF + r : C::ZROW;
        const bool panel = isE || isG || isF;
        const bool w0 = NW == 1 || wave == 0;

        // ---- (1) own rows from the next-row area (diagonal rows symmetrized)
        {
            const double *src = L.nxt + prow * P, *col = L.nxt + C::RD * P + r;
            const bool zero = isE && !hasE;
#pragma unroll
            for (int m = 0; m < BP; ++m) {
                const double v = src[m];
                const double s2 = isD ? 0.5 * (v + col[m * P]) : v;
                row[m] = zero ? 0.0 : s2;
                if (BP > 16 && (m & 7) == 7) __builtin_amdgcn_sched_barrier(0);
            }
            if (FWD) {
#pragma unroll
                for (int j = 0; j < MAX_NRHS_DEV; ++j)
                    if (j < nr && (isD || isE)) w[j] = isD ? L.w[r * RP + j] : 0.0;
            }
        }
        gsync<NW>();
        // single-wave classes fetch the next stage now (it arrives during the
        // elimination); wider classes fetch it right before it is needed, to keep
        // registers free
        if (NW == 1 && !last) pf.load(ch, i + 1, FWD, t);

        // ---- (2) elimination: hat D, the panel rows, y (Algorithm 1 potrf / trsm, Algorithm 2)
        if (w0) {
            elim_wave<BP>(row, panel, lane);
            double *dst = L.pnl + prow * P;
            if (isD || isG || (NW == 1 && panel)) {
#pragma unroll
                for (int m = 0; m < BP; ++m) dst[m] = (isD && m > r) ? 0.0 : row[m];
            }
            wave_sync();
            // the diagonal entry read back from LDS (not by indexing a register array)
            const double dg = isD ? dst[r] : 1.0;
            if (any_bad_pivot(isD, dg) && !failed) failed = gs + 1;
            const double dinv = isD ? 1.0 / dg : 1.0;
            if (isD) L.dinv[r] = dinv;
            if (FWD) {
                // forward substitution (Algorithm 2): y = hat D^{-1} w on the D rows, and the
                // panel rows accumulate -hat E y, -hat G y, -hat B^T y
                fsub_wave<BP>(row, w, nr, panel, lane, dinv);
                if (isD) {
#pragma unroll
                    for (int j = 0; j < MAX_NRHS_DEV; ++j)
                        if (j < nr) L.y[r * RP + j] = w[j];
                }
            }
        }
        gsync<NW>();
        if (NW > 1) {
            // the E and F waves solve their rows against hat D from LDS
            if (!w0) {
                trsm_wave<BP>(row, L.pnl + C::RD * P, P, L.dinv);
                if (FWD) fsub_rows<BP>(row, w, nr, L.y);
                if (isE || isF) {
                    double *dst = L.pnl + prow * P;
#pragma unroll
                    for (int m = 0; m < BP; ++m) dst[m] = row[m];
                }
            }
            __syncthreads();
        }

        // ---- (3) factor blocks and y out (lane-contiguous stores from LDS)
        wstore<NT, BP * BP>(F + sd.oLd + (long long)gs * b2, L.pnl + C::RD * P, P, b, b, t);
        if (hasE) wstore<NT, BP * BP>(F + ch.coup_off(i), L.pnl + C::RE * P, P, b, b, t);
        if (ng) wstore<NT, NGM * BP>(F + sd.oLb + (long long)gs * ng * b, L.pnl + C::RG * P, P, ng, b, t);
        if (hasF) wstore<NT, BP * BP>(F + ch.fill_off(i), L.pnl + C::RF * P, P, b, b, t);
        if (FWD) wstore_rhs<NT, BP>(a.rhs + sd.oRhs + (long long)gs * b * nr, L.y, b, nr, t);

        // ---- (4) Gram of the panel rows (Eqs. 4, 6, 8a, 8b).  Every thread dots
        // its own row with broadcast rows; threads without an output write to the
        // sink row.  The widest class reads its own row back from LDS (OWN_LDS).
        constexpr bool OWN_LDS = BP > 32;
        const double *own = L.pnl + prow * P;
        gsync<NW>();
        if (hasE) {
            // with hat E (hat F_k at a segment end): E threads -hat E hat E^T (the next
            // diagonal block once D_{i+1} is added), G threads -hat G hat E^T (the next
            // arrow rows with B_{i+1}), F threads the next fill rows -hat B^T hat E^T;
            // at a segment end -hat F hat F^T, -hat G hat F^T and tilde H_k^T for the scratch
            const int orow = (isE && r < b) ? C::RD + r : (isG && r < ng) ? C::RG + r : (isF && r < b) ? C::RF + r : C::SROW;
            double *o = L.nxt + orow * P;
            const double *Eb = L.pnl + C::RE * P;
#pragma unroll 1
            for (int m0 = 0; m0 < BP; m0 += 4) {
                double s4[4];
                if (OWN_LDS) dot4_lds<BP>(own, Eb + m0 * P, P, s4);
                else dot4<BP>(row, Eb + m0 * P, P, s4);
#pragma unroll
                for (int q = 0; q < 4; ++q) o[m0 + q] = -s4[q];
            }
            if (FWD && isE && r < b) {
                // -hat E y: the next stage's rhs once r_{i+1} is added; at a segment end
                // -hat F_k y goes to the scratch
                if (nextD) {
#pragma unroll
                    for (int j = 0; j < MAX_NRHS_DEV; ++j)
                        if (j < nr) L.w[r * RP + j] = w[j];
                } else if (endS) {
                    double *dy = ch.scr(k) + scr_dy(b, ng, nr);
#pragma unroll
                    for (int j = 0; j < MAX_NRHS_DEV; ++j)
                        if (j < nr) dy[r * nr + j] = w[j];
                }
            }
        }
        if (w0 && ng > 0) {
            // G threads: hat R_k -= hat G hat G^T
            double *o = isG ? L.racc + r * (NGM + 1) : L.nxt + C::SROW * P;
            const double *Gb = L.pnl + C::RG * P;
#pragma unroll 1
            for (int q0 = 0; q0 < ng; q0 += 4) {
                double s4[4];
                if (OWN_LDS) dot4_lds<BP>(own, Gb + q0 * P, P, s4);
                else dot4<BP>(row, Gb + q0 * P, P, s4);
#pragma unroll
                for (int q = 0; q < 4; ++q) o[q0 + q] -= s4[q];
            }
        }
        if (hasF && (NW == 1 || wave == 0 || wave == C::WF)) {
            // F threads: hat A_k -= hat B^T hat B; G threads: hat Q_k -= hat G hat B
            double *o = isF ? L.acc_a + r * P : isG ? L.acc_q + r * P : L.nxt + C::SROW * P;
            const double *Fb = L.pnl + C::RF * P;
#pragma unroll 1
            for (int m0 = 0; m0 < BP; m0 += 4) {
                double s4[4];
                if (OWN_LDS) dot4_lds<BP>(own, Fb + m0 * P, P, s4);
                else dot4<BP>(row, Fb + m0 * P, P, s4);
#pragma unroll
                for (int q = 0; q < 4; ++q) o[m0 + q] -= s4[q];
            }
        }
        gsync<NW>();

        // ---- (5) the next stage's blocks added to the Gram's products
        if (!last) {
            if (NW > 1) pf.load(ch, i + 1, FWD, t);
            pf.commit(L.nxt, L.w, sd, nr, ch.has_next(i + 1), FWD, t);
        }
        gsync<NW>();
        if (endS) {
            // hat F_k hat F_k^T, hat G hat F_k^T (Eq. 8c) and tilde H_k = -hat F_k hat B (stored transposed)
            double *sc = ch.scr(k);
            wstore<NT, BP * BP>(sc + scr_dA(b, ng, nr), L.nxt + C::RD * P, P, b, b, t, -1.0);
            if (ng) wstore<NT, NGM * BP>(sc + scr_dQ(b, ng, nr), L.nxt + C::RG * P, P, ng, b, t, -1.0);
            if (hasF) wstore<NT, BP * BP, true>(F + sd.oH + (long long)(k - 2) * b2, L.nxt + C::RF * P, P, b, b, t);
        }
    }

    // ---- epilogue: separator partials (Eq. 8a, 9b) and the arrow partials (Eqs. 8b, 9c)
    const int t = threadIdx.x;
    const bool isG = t >= C::TG && t < C::TG + NGM;
    const bool isF = hasF && t >= C::TF && t < C::TF + BP;
    if (hasF) {
        wstore<NT, BP * BP>(F + sd.oLd + (long long)sep * b2, L.acc_a, P, b, b, t);
        if (ng) wstore<NT, NGM * BP>(F + sd.oLb + (long long)sep * ng * b, L.acc_q, P, ng, b, t);
        const int r = t - C::TF;
        if (FWD && isF && r < b) {
#pragma unroll
            for (int j = 0; j < MAX_NRHS_DEV; ++j)
                if (j < nr) a.rhs[sd.oRhs + ((long long)sep * b + r) * nr + j] = w[j];
        }
    }
    if (ng) {
        const int r = t - C::TG;
        if (!RED) {
            double *sc = ch.scr(k);
            wstore<NT, NGM * NGM>(sc + scr_Rk(b, ng, nr), L.racc, NGM + 1, ng, ng, t);
            if (FWD && isG && r < ng) {
#pragma unroll
                for (int j = 0; j < MAX_NRHS_DEV; ++j)
                    if (j < nr) sc[scr_yg(b, ng, nr) + r * nr + j] = w[j];
            }
        } else if (isG) {
#pragma unroll
            for (int j = 0; j < MAX_NRHS_DEV; ++j) L.yg[r * RP + j] = FWD ? w[j] : 0.0;
        }
    }
    gsync<NW>();
    return failed;
}

// The factor blocks of one stage of a chain (lane-contiguous, branch-free loads)
// and its right-hand-side rows (with PRIMAL also the primal solution rows, for
// the adjoint gradients).
template <int BP, bool RED>
struct SolveLoad {
    using C = WC<BP>;
    static constexpr int NT = C::NT;
    static constexpr int MB = (BP * BP + NT - 1) / NT;
    static constexpr int MG = (NGM * BP + NT - 1) / NT;
    static constexpr int MR = (BP * MAX_NRHS_DEV + NT - 1) / NT;
    double d[MB], e[MB], g[MG], f[MB], y[MR], px[MR];

    template <bool PRIMAL>
    __device__ __forceinline__ void load(const WChain<RED> &ch, int i, bool hasF, int t)
    {
        const Args &a = ch.a;
        const SysDesc &sd = ch.sd;
        const int b = sd.b, ng = sd.ng, nr = a.nr, s = ch.stage(i);
        const int b2 = b * b, gb = ng * b, rb = b * nr;
        const bool hasE = ch.has_next(i);
        if constexpr (BP <= 32) {
            // buffer resources: entries past a block's end (and absent blocks) read as zero
            const GBlock gLd(a.F + sd.oLd + (long long)s * b2, b2), gLe(a.F + ch.coup_off(i), hasE ? b2 : 0);
            const GBlock gLb(a.F + sd.oLb + (long long)s * gb, gb);
            const GBlock gLf(a.F + (hasF ? ch.fill_off(i) : 0), hasF ? b2 : 0);
            const GBlock gY(a.rhs + sd.oRhs + (long long)s * rb, rb);
            const GBlock gXP(PRIMAL ? a.xp + sd.oRhs + (long long)s * rb : a.rhs, PRIMAL ? rb : 0);
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                const int x = (t + m * NT) * 8;
                d[m] = gLd.ld(x);
                e[m] = gLe.ld(x);
                f[m] = gLf.ld(x);
            }
#pragma unroll
            for (int m = 0; m < MG; ++m) g[m] = gLb.ld((t + m * NT) * 8);
#pragma unroll
            for (int m = 0; m < MR; ++m) {
                const int x = (t + m * NT) * 8;
                y[m] = gY.ld(x);
                px[m] = PRIMAL ? gXP.ld(x) : 0.0;
            }
        } else {
            const double *Ld = a.F + sd.oLd + (long long)s * b2, *Le = a.F + ch.coup_off(i);
            const double *Lb = a.F + sd.oLb + (long long)s * gb;
            const double *Lf = a.F + (hasF ? ch.fill_off(i) : 0);
            const double *Y = a.rhs + sd.oRhs + (long long)s * rb;
            const double *XP = PRIMAL ? a.xp + sd.oRhs + (long long)s * rb : Y;
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                const int x = t + m * NT;
                d[m] = ld_or_zero(Ld, x, x < b2);
                e[m] = ld_or_zero(Le, x, hasE && x < b2);
                f[m] = ld_or_zero(Lf, x, hasF && x < b2);
            }
#pragma unroll
            for (int m = 0; m < MG; ++m) {
                const int x = t + m * NT;
                g[m] = ld_or_zero(Lb, x, x < gb);
            }
#pragma unroll
            for (int m = 0; m < MR; ++m) {
                const int x = t + m * NT;
                y[m] = ld_or_zero(Y, x, x < rb);
                px[m] = PRIMAL ? ld_or_zero(XP, x, x < rb) : 0.0;
            }
        }
    }

    // blocks into rows of pitch P at D / E / G / F rows of `area` (zeros outside the
    // blocks up to BP columns), y into Yl and the primal rows into Pl (pitch RP)
    template <bool PRIMAL>
    __device__ __forceinline__ void commit(double *area, double *Yl, double *Pl, const SysDesc &sd, int nr, int t) const
    {
        constexpr int P = C::P;
        const int b = sd.b, ng = sd.ng, b2 = b * b, gb = ng * b, rb = b * nr;
        const float invb = 1.0f / (float)b, invr = 1.0f / (float)nr;
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            const int x = t + m * NT;
            if (x < b2) {
                int rr, cc;
                rc_of(x, b, invb, rr, cc);
                area[(C::RD + rr) * P + cc] = d[m];
                area[(C::RE + rr) * P + cc] = e[m];
                area[(C::RF + rr) * P + cc] = f[m];
            }
        }
#pragma unroll
        for (int m = 0; m < MG; ++m) {
            const int x = t + m * NT;
            if (x < gb) {
                int rr, cc;
                rc_of(x, b, invb, rr, cc);
                area[(C::RG + rr) * P + cc] = g[m];
            }
        }
#pragma unroll
        for (int m = 0; m < MR; ++m) {
            const int x = t + m * NT;
            if (x < rb) {
                int rr, j;
                rc_of(x, nr, invr, rr, j);
                Yl[rr * C::RP + j] = y[m];
                if (PRIMAL) Pl[rr * C::RP + j] = px[m];
            }
        }
    }
};

// Staging rows (pitch P) of the four groups plus the zero and sink rows: the
// identity in the diagonal area and zeros elsewhere, so that entries outside the
// b x b (ng x b) blocks read as the padding in every later stage.
template <int BP>
__device__ __forceinline__ void init_rows(double *area, int nrows)
{
    using C = WC<BP>;
    for (int e = threadIdx.x; e < nrows * C::P; e += C::NT) {
        const int rr = e / C::P, cc = e - rr * C::P;
        area[e] = (rr < BP && rr == cc) ? 1.0 : 0.0;
    }
}

// ---------------------------------------------------------------- forward sweep
// Forward substitution of one chain with its factor in place (Algorithm 2,
// parallel phase for a segment, sequential phase for RED): y overwrites the
// rhs; for a segment k >= 2 the separator rhs partial, for a segment ending on
// hat F_k the product -hat F_k y, and the arrow partial -sum hat G y go where the
// factor sweep puts them.
template <int BP, bool RED>
__device__ __forceinline__ void wave_forward(const Args &a, const SysDesc &sd, int k, const WaveLds &L)
{
    using C = WC<BP>;
    constexpr int NT = C::NT, P = C::P, NW = C::NW, RP = C::RP;
    const WChain<RED> ch{a, sd, k};
    const int b = sd.b, ng = sd.ng, nr = a.nr;
    const bool hasF = !RED && k > 1;
    const int len = ch.length();
    const int sep = hasF ? sep_of(sd, k) : 0;
    double *area = L.nxt;   // factor rows of the current stage

    init_rows<BP>(area, C::NROW + 2);
    for (int e = threadIdx.x; e < C::BPX * RP; e += NT) L.w[e] = 0.0;
    gsync<NW>();
    // w of the first stage (RED: plus -hat F y of the segment before it)
    {
        const int s0 = ch.stage(0);
        const double *src = a.rhs + sd.oRhs + (long long)s0 * b * nr;
        const double *add = RED ? ch.scr(1) + scr_dy(b, ng, nr) : nullptr;
        for (int e = threadIdx.x; e < b * nr; e += NT) {
            const int rr = e / nr, j = e - rr * nr;
            L.w[rr * RP + j] = src[e] + (RED ? add[e] : 0.0);
        }
    }
    double w[MAX_NRHS_DEV];
    {
        const int t = threadIdx.x;
        const bool isF = hasF && t >= C::TF && t < C::TF + BP;
        const int r = t - C::TF;
#pragma unroll
        for (int j = 0; j < MAX_NRHS_DEV; ++j) {
            double v = 0.0;
            if (j < nr && isF && r < b) v = a.rhs[sd.oRhs + ((long long)sep * b + r) * nr + j];
            w[j] = v;
        }
    }
    SolveLoad<BP, RED> pf;
    if (NW == 1) pf.template load<false>(ch, 0, hasF, threadIdx.x);
    for (int i = 0; i < len; ++i) {
        const int gs = ch.stage(i);
        const bool hasE = ch.has_next(i);
        const bool last = i == len - 1;
        const bool endS = !RED && last && hasE;
        const int t = opaque_tid(), wave = t >> 6, lane = t & 63;
        const bool isD = t < BP;
        const bool isE = t >= C::TE && t < C::TE + BP;
        const bool isG = t >= C::TG && t < C::TG + NGM;
        const bool isF = hasF && t >= C::TF && t < C::TF + BP;
        const int r = isD ? t : isE ? t - C::TE : isG ? t - C::TG : isF ? t - C::TF : 0;
        const int prow = isD ? C::RD + r : isE ? C::RE + r : isG ? C::RG + r : isF ? C::RF + r : C::ZROW;
        const bool panel = isE || isG || isF;
        const bool w0 = NW == 1 || wave == 0;
        gsync<NW>();
        if (NW > 1) pf.template load<false>(ch, i, hasF, t);
        pf.template commit<false>(area, L.y, L.y, sd, nr, t);   // the y staging is unused: w is in L.w
        gsync<NW>();
        if (NW == 1 && !last) pf.template load<false>(ch, i + 1, hasF, t);
        double row[BP];
        {
            const double *src = area + prow * P;
#pragma unroll
            for (int m = 0; m < BP; ++m) {
                row[m] = src[m];
                if (BP > 16 && (m & 7) == 7) __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int j = 0; j < MAX_NRHS_DEV; ++j)
                if (j < nr && (isD || isE)) w[j] = isD ? L.w[r * RP + j] : 0.0;
        }
        const double dinv = isD ? 1.0 / area[prow * P + r] : 1.0;
        gsync<NW>();
        if (w0) {
            fsub_wave<BP>(row, w, nr, panel, lane, dinv);
            if (isD) {
#pragma unroll
                for (int j = 0; j < MAX_NRHS_DEV; ++j)
                    if (j < nr) L.y[r * RP + j] = w[j];
            }
        }
        gsync<NW>();
        if (NW > 1 && !w0) fsub_rows<BP>(row, w, nr, L.y);
        // y out; the next stage's w = r_{i+1} (RED: plus -hat F y) - hat E y
        wstore_rhs<NT, BP>(a.rhs + sd.oRhs + (long long)gs * b * nr, L.y, b, nr, t);
        if (isE && r < b) {
            if (hasE && !endS) {
                const int ns = ch.stage(i + 1);
                const double *src = a.rhs + sd.oRhs + (long long)ns * b * nr;
                const double *add = RED ? ch.scr(i + 2) + scr_dy(b, ng, nr) : nullptr;
#pragma unroll
                for (int j = 0; j < MAX_NRHS_DEV; ++j)
                    if (j < nr) L.w[r * RP + j] = src[r * nr + j] + (RED ? add[r * nr + j] : 0.0) + w[j];
            } else if (endS) {
                double *dy = ch.scr(k) + scr_dy(b, ng, nr);
#pragma unroll
                for (int j = 0; j < MAX_NRHS_DEV; ++j)
                    if (j < nr) dy[r * nr + j] = w[j];
            }
        }
    }
    gsync<NW>();
    const int t = threadIdx.x;
    const bool isG = t >= C::TG && t < C::TG + NGM;
    const bool isF = hasF && t >= C::TF && t < C::TF + BP;
    if (isF && t - C::TF < b) {
        const int r = t - C::TF;
#pragma unroll
        for (int j = 0; j < MAX_NRHS_DEV; ++j)
            if (j < nr) a.rhs[sd.oRhs + ((long long)sep * b + r) * nr + j] = w[j];
    }
    if (ng && isG) {
        const int r = t - C::TG;
        if (!RED) {
            double *yg = ch.scr(k) + scr_yg(b, ng, nr);
            if (r < ng) {
#pragma unroll
                for (int j = 0; j < MAX_NRHS_DEV; ++j)
                    if (j < nr) yg[r * nr + j] = w[j];
            }
        } else {
#pragma unroll
            for (int j = 0; j < MAX_NRHS_DEV; ++j) L.yg[r * RP + j] = w[j];
        }
    }
    gsync<NW>();
}

// ---------------------------------------------------------------- backward sweep
// Backward substitution of one chain (Algorithm 3, Eqs. 11, 12): for the chain's
// stages in reverse, x_i = hat D_i^{-T} (y_i - hat E_i^T x_next - hat G_i^T x_g
// [- hat B_i x_sep]); x_g, x at the separator of segment k and x after the chain
// are already in place.  The blocks of stage i - 1 are fetched while stage i is
// solved: lane c of wave 0 owns column c.  With ADJ the solution is lambda and
// the gradient blocks of the chain's stages are written (dD_i = -sym(lambda_i x_i^T),
// dB_i = -(lambda_g x_i^T + x_g lambda_i^T), dC_i = -(lambda_{i+1} x_i^T +
// x_{i+1} lambda_i^T) for the couplings of natural neighbours).
template <int BP, bool ADJ, bool RED>
__device__ __forceinline__ void wave_backward(const Args &a, const SysDesc &sd, int k, const WaveLds &L)
{
    using C = WC<BP>;
    constexpr int NT = C::NT, P = C::P, NW = C::NW, RP = C::RP, BPX = C::BPX;
    const WChain<RED> ch{a, sd, k};
    const int b = sd.b, ng = sd.ng, nr = a.nr, N = sd.N;
    const int b2 = b * b;
    const bool hasF = !RED && k > 1;
    const int len = ch.length();
    const int sep = hasF ? sep_of(sd, k) : 0;
    double *X = a.rhs + sd.oRhs;
    const double *XP = ADJ ? a.xp + sd.oRhs : X;
    double *xn = L.xn, *xc = L.xc, *pn = L.pn, *pc = L.pc;
    double *area = L.pnl;
    init_rows<BP>(area, C::NROW);
    {
        const int t = threadIdx.x;
        const long long og = (long long)N * b * nr;
        for (int e = t; e < NGM * RP; e += NT) {
            const int q = e / RP, j = e - q * RP;
            const bool in = q < ng && j < nr;
            L.xg[e] = in ? X[og + q * nr + j] : 0.0;
            if (ADJ) L.pg[e] = in ? XP[og + q * nr + j] : 0.0;
        }
        const bool after = !RED && ch.has_next(len - 1);
        const long long on = after ? (long long)(ch.stage(len - 1) + 1) * b * nr : 0;
        const long long os = (long long)sep * b * nr;
        for (int e = t; e < BPX * RP; e += NT) {
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
    SolveLoad<BP, RED> pf;
    if (NW == 1) pf.template load<ADJ>(ch, len - 1, hasF, threadIdx.x);
    gsync<NW>();
    for (int i = len - 1; i >= 0; --i) {
        const int gs = ch.stage(i);
        const bool hasE = ch.has_next(i);
        const int t = opaque_tid(), wave = t >> 6, lane = t & 63;
        const bool w0 = NW == 1 || wave == 0;
        if (NW > 1) pf.template load<ADJ>(ch, i, hasF, t);
        pf.template commit<ADJ>(area, xc, pc, sd, nr, t);   // y_i (lambda: the adjoint's y) into xc
        gsync<NW>();
        if (NW == 1 && i > 0) pf.template load<ADJ>(ch, i - 1, hasF, t);
        if (w0) {
            // lane c owns column c (lanes past BP compute on column 0 and store nothing)
            const int c = lane;
            const int cc = c < BP ? c : 0;
            double acc[MAX_NRHS_DEV];
#pragma unroll
            for (int j = 0; j < MAX_NRHS_DEV; ++j) acc[j] = (j < nr) ? xc[cc * RP + j] : 0.0;
            if (hasE) {
                // - coupling^T x_next (hat E^T, hat F_k^T, or hat H_k^T on the reduced chain)
                for (int rr = 0; rr < b; ++rr) {
                    const double e = area[(C::RE + rr) * P + cc];
#pragma unroll
                    for (int j = 0; j < MAX_NRHS_DEV; ++j)
                        if (j < nr) acc[j] = fma(-e, xn[rr * RP + j], acc[j]);
                }
            }
            for (int q = 0; q < ng; ++q) {
                // - hat G^T x_g (hat Q_k^T on the reduced chain)
                const double g = area[(C::RG + q) * P + cc];
#pragma unroll
                for (int j = 0; j < MAX_NRHS_DEV; ++j)
                    if (j < nr) acc[j] = fma(-g, L.xg[q * RP + j], acc[j]);
            }
            if (hasF) {
                // - hat B x_sep
                for (int rr = 0; rr < b; ++rr) {
                    const double f = area[(C::RF + rr) * P + cc];
#pragma unroll
                    for (int j = 0; j < MAX_NRHS_DEV; ++j)
                        if (j < nr) acc[j] = fma(-f, L.xs[rr * RP + j], acc[j]);
                }
            }
            // x = hat D^{-T} acc; column c of hat D (the identity outside the block)
            const double dinv = 1.0 / area[(C::RD + cc) * P + cc];
            double dcs[BP];
#pragma unroll
            for (int m = 0; m < BP; ++m) {
                dcs[m] = area[(C::RD + m) * P + cc] * dinv;
                if (BP > 16 && (m & 7) == 7) __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int j = 0; j < MAX_NRHS_DEV; ++j) {
                if (j < nr) {
                    const double xv = bsub_wave<BP>(dcs, acc[j] * dinv, lane);
                    if (c < BP) xc[c * RP + j] = xv;
                }
            }
        }
        gsync<NW>();
        if (ADJ && w0 && lane < b) {
            const int c = lane;
            // dD_i = -sym(lambda_i x_i^T), column c
            double *dD = a.dD + sd.oD + (long long)gs * b2;
            for (int rr = 0; rr < b; ++rr) {
                double s = 0.0;
                for (int j = 0; j < nr; ++j) s += xc[rr * RP + j] * pc[c * RP + j] + pc[rr * RP + j] * xc[c * RP + j];
                dD[rr * b + c] = -0.5 * s;
            }
            // dB_i = -(lambda_g x_i^T + x_g lambda_i^T)
            double *dB = a.dB + sd.oB + (long long)gs * ng * b;
            for (int q = 0; q < ng; ++q) {
                double s = 0.0;
                for (int j = 0; j < nr; ++j) s += L.xg[q * RP + j] * pc[c * RP + j] + L.pg[q * RP + j] * xc[c * RP + j];
                dB[q * b + c] = -s;
            }
            if (!RED && hasE) {
                // dC_i = -(lambda_{i+1} x_i^T + x_{i+1} lambda_i^T): C_i couples stage i with its natural successor
                double *dC = a.dC + sd.oC + (long long)gs * b2;
                for (int rr = 0; rr < b; ++rr) {
                    double s = 0.0;
                    for (int j = 0; j < nr; ++j) s += xn[rr * RP + j] * pc[c * RP + j] + pn[rr * RP + j] * xc[c * RP + j];
                    dC[rr * b + c] = -s;
                }
            }
            if (hasF && i == 0) {
                // C_{sep_k} = Psi_{first(k), sep_k}: rows of the first stage, columns of the separator
                double *dC = a.dC + sd.oC + (long long)sep * b2;
                for (int rr = 0; rr < b; ++rr) {
                    double s = 0.0;
                    for (int j = 0; j < nr; ++j) s += xc[rr * RP + j] * L.ps[c * RP + j] + pc[rr * RP + j] * L.xs[c * RP + j];
                    dC[rr * b + c] = -s;
                }
            }
        }
        wstore_rhs<NT, BP>(X + (long long)gs * b * nr, xc, b, nr, t);
        gsync<NW>();
        double *tmp = xn; xn = xc; xc = tmp;
        tmp = pn; pn = pc; pc = tmp;
    }
    gsync<NW>();
}

// sum_{k < p} src[k * stride], eight loads in flight (the partials of the p
// segments sit a scratch stride apart)
__device__ __forceinline__ double sum8(const double *src, long long stride, int p)
{
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int k = 0;
    for (; k + 8 <= p; k += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] += src[(long long)(k + u) * stride];
    }
    for (; k < p; ++k) acc[0] += src[(long long)k * stride];
    return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

// ---------------------------------------------------------------- corner
// tilde R = sym(corner) + sum_k tilde R_k (+ the reduced chain's part) and
// hat R = chol(tilde R) (Algorithm 1, last lines; Eq. 8d); with FWD also
// hat y_g = hat R^{-1} tilde y_g and x_g = hat R^{-T} hat y_g (Algorithms 2, 3).
// CR (>= 16 x 17 doubles) and CW (>= 16 x 8) are LDS work areas; Rred (pitch 17)
// and Yred (pitch 8) hold the reduced chain's arrow partials, or are null.
// Every thread of the workgroup (NT) calls it; returns true if a pivot failed.
// SEGS: a segmented system (many partials; their sums keep eight loads in flight).
template <int NT, bool FWD, bool SEGS = false>
__device__ __forceinline__ bool corner_factor_w(const Args &a, const SysDesc &sd, double *CR, double *CW,
                                                const double *Rred, const double *Yred)
{
    constexpr int PC = NGM + 1, RP = MAX_NRHS_DEV;
    const int ng = sd.ng, nr = a.nr, tid = threadIdx.x, b = sd.b, N = sd.N;
    if (ng == 0) return false;
    __syncthreads();   // the partials were stored by other threads: complete and visible
    const double *cor = a.corner + sd.oCorner;
    const double *sc0 = a.F + sd.oScr;
    for (int e = tid; e < ng * ng; e += NT) {
        const int q = e / ng, c = e - q * ng;
        double v = 0.5 * (cor[e] + cor[c * ng + q]);
        if (SEGS) {
            v += sum8(sc0 + scr_Rk(b, ng, nr) + e, sd.scrStride, sd.p);
        } else {
            for (int k = 0; k < sd.p; ++k) v += sc0[(long long)k * sd.scrStride + scr_Rk(b, ng, nr) + e];
        }
        if (Rred) v += Rred[q * PC + c];
        CR[q * PC + c] = v;
    }
    if (FWD) {
        const double *rg = a.rhs + sd.oRhs + (long long)N * b * nr;
        for (int e = tid; e < ng * nr; e += NT) {
            const int q = e / nr, j = e - q * nr;
            double v = rg[e];
            if (SEGS) {
                v += sum8(sc0 + scr_yg(b, ng, nr) + e, sd.scrStride, sd.p);
            } else {
                for (int k = 0; k < sd.p; ++k) v += sc0[(long long)k * sd.scrStride + scr_yg(b, ng, nr) + e];
            }
            if (Yred) v += Yred[q * RP + j];
            CW[q * RP + j] = v;
        }
    }
    __syncthreads();
    bool bad = false;
    if (tid < 64) {
        const int q = tid;
        double row[NGM], w[MAX_NRHS_DEV];
#pragma unroll
        for (int m = 0; m < NGM; ++m) row[m] = (q < ng) ? (m < ng ? CR[q * PC + m] : 0.0) : (m == q ? 1.0 : 0.0);
#pragma unroll
        for (int j = 0; j < MAX_NRHS_DEV; ++j) w[j] = (FWD && q < ng && j < nr) ? CW[q * RP + j] : 0.0;
        elim_wave<NGM>(row, false, q);
        double *Lg = a.F + sd.oLg;
        if (q < ng) {
#pragma unroll
            for (int m = 0; m < NGM; ++m)
                if (m < ng) Lg[q * ng + m] = (m <= q) ? row[m] : 0.0;
        }
        if (q < NGM) {
#pragma unroll
            for (int m = 0; m < NGM; ++m) CR[q * PC + m] = (m <= q) ? row[m] : 0.0;
        }
        wave_sync();
        bad = any_bad_pivot(q < ng, CR[(q < NGM ? q : 0) * PC + (q < NGM ? q : 0)]);
        if (FWD) {
            const double dq = (q < ng) ? 1.0 / CR[(q < NGM ? q : 0) * PC + (q < NGM ? q : 0)] : 1.0;
            fsub_wave<NGM>(row, w, nr, false, q, dq);
            const int c = q;
            const bool cv = c < ng;
            const int cc = c < NGM ? c : 0;
            const double dinv = cv ? 1.0 / CR[c * PC + c] : 1.0;
            double dcs[NGM];
#pragma unroll
            for (int m = 0; m < NGM; ++m) dcs[m] = cv ? CR[m * PC + cc] * dinv : (m == c ? 1.0 : 0.0);
            double *xg = a.rhs + sd.oRhs + (long long)N * b * nr;
#pragma unroll
            for (int j = 0; j < MAX_NRHS_DEV; ++j) {
                if (j < nr) {
                    const double xv = bsub_wave<NGM>(dcs, w[j] * dinv, q);
                    if (cv) xg[c * nr + j] = xv;
                }
            }
        }
    }
    __syncthreads();
    return bad;
}

// Corner solve with the factor in place: tilde y_g, hat y_g, x_g.
template <int NT, bool SEGS = false>
__device__ __forceinline__ void corner_solve_w(const Args &a, const SysDesc &sd, double *CR, double *CW,
                                               const double *Yred)
{
    constexpr int PC = NGM + 1, RP = MAX_NRHS_DEV;
    const int ng = sd.ng, nr = a.nr, tid = threadIdx.x, b = sd.b, N = sd.N;
    if (ng == 0) return;
    __syncthreads();   // the partials were stored by other threads: complete and visible
    const double *sc0 = a.F + sd.oScr;
    double *rg = a.rhs + sd.oRhs + (long long)N * b * nr;
    const double *Lg = a.F + sd.oLg;
    for (int e = tid; e < ng * nr; e += NT) {
        const int q = e / nr, j = e - q * nr;
        double v = rg[e];
        if (SEGS) {
            v += sum8(sc0 + scr_yg(b, ng, nr) + e, sd.scrStride, sd.p);
        } else {
            for (int k = 0; k < sd.p; ++k) v += sc0[(long long)k * sd.scrStride + scr_yg(b, ng, nr) + e];
        }
        if (Yred) v += Yred[q * RP + j];
        CW[q * RP + j] = v;
    }
    for (int e = tid; e < NGM * PC; e += NT) CR[e] = 0.0;
    __syncthreads();
    for (int e = tid; e < ng * ng; e += NT) {
        const int q = e / ng, c = e - q * ng;
        CR[q * PC + c] = (c <= q) ? Lg[e] : 0.0;
    }
    __syncthreads();
    if (tid < 64) {
        const int q = tid;
        double row[NGM], w[MAX_NRHS_DEV];
#pragma unroll
        for (int m = 0; m < NGM; ++m) row[m] = (q < ng) ? CR[q * PC + m] : (m == q ? 1.0 : 0.0);
        const double di = (q < ng) ? 1.0 / CR[q * PC + q] : 1.0;
#pragma unroll
        for (int j = 0; j < MAX_NRHS_DEV; ++j) w[j] = (q < ng && j < nr) ? CW[q * RP + j] : 0.0;
        fsub_wave<NGM>(row, w, nr, false, q, di);
        const int c = q;
        const bool cv = c < ng;
        const int cc = c < NGM ? c : 0;
        double dcs[NGM];
#pragma unroll
        for (int m = 0; m < NGM; ++m) dcs[m] = cv ? CR[m * PC + cc] * di : (m == c ? 1.0 : 0.0);
#pragma unroll
        for (int j = 0; j < MAX_NRHS_DEV; ++j) {
            if (j < nr) {
                const double xv = bsub_wave<NGM>(dcs, w[j] * di, q);
                if (cv) rg[c * nr + j] = xv;
            }
        }
    }
    __syncthreads();
}

// dcorner = -sym(lambda_g x_g^T) summed over the rhs columns.
template <int NT>
__device__ __forceinline__ void corner_grad_w(const Args &a, const SysDesc &sd)
{
    const int ng = sd.ng, nr = a.nr, tid = threadIdx.x, b = sd.b, N = sd.N;
    if (ng == 0) return;
    const long long og = sd.oRhs + (long long)N * b * nr;
    const double *lg = a.rhs + og, *xg = a.xp + og;
    double *dR = a.dcorner + sd.oCorner;
    for (int e = tid; e < ng * ng; e += NT) {
        const int q = e / ng, c = e - q * ng;
        double s = 0.0;
        for (int j = 0; j < nr; ++j) s += lg[q * nr + j] * xg[c * nr + j] + xg[q * nr + j] * lg[c * nr + j];
        dR[e] = -0.5 * s;
    }
    __syncthreads();
}

// A failed system's solution is NaN (natural stage range [s0, s1), plus g if withg).
template <int NT>
__device__ __forceinline__ void nan_fill(const Args &a, const SysDesc &sd, int s0, int s1, bool withg)
{
    const int nr = a.nr, b = sd.b;
    const double qnan = __longlong_as_double(0x7ff8000000000000LL);
    double *X = a.rhs + sd.oRhs;
    for (long long e = (long long)s0 * b * nr + threadIdx.x; e < (long long)s1 * b * nr; e += NT) X[e] = qnan;
    if (withg)
        for (int e = threadIdx.x; e < sd.ng * nr; e += NT) X[(long long)sd.N * b * nr + e] = qnan;
}

}  // namespace kkt_dev
