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

// Phase boundary: the scheduler may not move instructions across it, so the live
// ranges of consecutive phases of a stage do not overlap.
__device__ __forceinline__ void phase_fence() { __builtin_amdgcn_sched_barrier(0); }

// Four independent 4x4x4 FP64 products per instruction (lane layout probed on
// gfx950: with lane l = x + 4 blk + 16 y, A[blk][x][y], B[blk][y][x] and
// D[blk][y][x] are held by lane l).  Used for the arrow rows when there are at
// most four of them, where a 16-row tile would be mostly padding.
__device__ __forceinline__ double mfma44(double a, double b, double c)
{
    return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// Lane mapping of a tile with DB columns handled by one 64-lane wave: lane l holds
// column l % DB of the rows l / DB + (64 / DB) m, so every LDS offset is a
// compile-time immediate and each row of a row-major global block is one
// contiguous access.
template <int DB>
struct TileMap {
    static constexpr int RS = 64 / DB;   // rows per pass
    int c, r0;
    __device__ __forceinline__ explicit TileMap(int lane) : c(lane & (DB - 1)), r0(lane / DB) {}
    __device__ __forceinline__ int row(int m) const { return r0 + RS * m; }
};

// Rows [0, rows) x columns [0, cols) of an LDS tile of ROWS rows (pitch DB + 1) to
// the row-major block g of rows x cols: every read first, then the stores (rows
// at or past the end fall outside the block, columns past cols are sent there).
template <int DB, int ROWS>
__device__ __forceinline__ void store_tile(const GBlock &g, const double *lds, int cols, int lane)
{
    constexpr int PD = DB + 1, M = ROWS / TileMap<DB>::RS;
    const TileMap<DB> t(lane);
    double v[M];
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = lds[t.row(m) * PD + t.c];
    pin_row<M>(v);
    const int base = t.c < cols ? (t.r0 * cols + t.c) * 8 : GB_OUT;
#pragma unroll
    for (int m = 0; m < M; ++m) g.st(base + TileMap<DB>::RS * m * cols * 8, v[m]);
}

// acc[rt] += A B on the FP64 matrix cores for the 16-row tiles rt < RT of A
// (KD columns) and B = KD x nr (nr <= 16, row pitch nr, columns >= nr taken as
// zero): A[r][k] = A[r * pa + k], or A[k * pa + r] with TA.  With LOWER, A is
// lower triangular and the k-chunks right of a tile's last row are skipped.
// Element v of lane l of acc[rt] is row 16 rt + 4 v + l / 16, column l % 16.
template <int RT, int KD, bool TA, bool LOWER = false>
__device__ __forceinline__ void mm_rhs(const double *A, int pa, const double *B, int nr, dx4 (&acc)[RT], int li,
                                       int lk)
{
    // every operand is read before the first product, so the reads overlap
    constexpr int KS = KD / 4;
    double bv[KS], av[KS][RT];
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
        const int k = 4 * kk + lk;
        bv[kk] = B[k * nr + (li < nr ? li : 0)];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int r = 16 * rt + li;
            av[kk][rt] = TA ? A[k * pa + r] : A[r * pa + k];
        }
    }
#pragma unroll
    for (int kk = 0; kk < KS; ++kk)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            if (LOWER && 4 * kk > 16 * rt + 15) continue;
            acc[rt] = mfma4(av[kk][rt], li < nr ? bv[kk] : 0.0, acc[rt]);
        }
}

// sum over k < KD of A(row, k) B[k] for a single rhs on the vector units, one row
// per lane, A(row, k) = A[row pa + k], or A[k pa + row] with TA.  With one rhs a
// 16-column MFMA tile would spend 15 of its columns on nothing; here the row and
// the vector are read CH entries at a time (every lane reads the vector at the
// same address) and summed in four chains.
template <int KD, bool TA, int CH = 16>
__device__ __forceinline__ double row_dot1(const double *A, int pa, int row, const double *B)
{
    static_assert(KD % CH == 0 && CH % 4 == 0, "rows are read in chunks of CH");
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
    for (int k0 = 0; k0 < KD; k0 += CH) {
        double av[CH], bv[CH];
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            av[t] = TA ? A[(k0 + t) * pa + row] : A[row * pa + k0 + t];
            bv[t] = B[k0 + t];
        }
#pragma unroll
        for (int t = 0; t < CH; t += 4) {
            s0 = fma(av[t], bv[t], s0);
            s1 = fma(av[t + 1], bv[t + 1], s1);
            s2 = fma(av[t + 2], bv[t + 2], s2);
            s3 = fma(av[t + 3], bv[t + 3], s3);
        }
    }
    return (s0 + s1) + (s2 + s3);
}

// x[c] of T^T x = rhs for a lower triangular T, lane c holding accs = rhs[c] / T[c][c]
// and dcs[l] = T[l][c] / T[c][c] for l > c, zero for l <= c: with the scaling done
// beforehand the serial chain is one broadcast and one FMA per column.  Lane c's own
// step subtracts nothing, so its accs is x[c] from then on (the later steps subtract
// zeros), and the sweep ends with x on every lane: no per-lane select.
template <int DB>
__device__ __forceinline__ double back_subst_scaled(const double (&dcs)[DB], double accs)
{
#pragma unroll
    for (int c2 = DB - 1; c2 >= 0; --c2) accs = fma(-dcs[c2], readlane_d(accs, c2), accs);
    return accs;
}

// Dense LDS layout: a panel area of (2 DB + 16) rows with pitch DB + 1 (the
// backward sweep and the corner reuse it as their staging area), then the same
// small vectors as the general layout.  Regions the p = 1 path never touches
// (fill-row accumulators) alias the panel area.
__host__ __device__ __forceinline__ LdsOff lds_offsets_dense(int DB, int nr, bool seg = false)
{
    LdsOff o;
    const int PITCH = DB + 1;
    int t = 0;
    o.col = t; t += 2 * (DB > NGM ? DB : NGM) + 64;   // + one dummy slot per lane
    o.P = t;   t += (seg ? 4 * DB + 2 * NGM : 2 * DB + NGM) * PITCH;   // segments: + fill rows, hat A, hat Q
    o.A = o.P; o.Q = o.P; o.RP = o.P;
    o.R = t;   t += NGM * NGM;
    o.W = t;   t += (DB > NGM ? DB : NGM) * nr;
    o.Y = t;   t += (DB > NGM ? DB : NGM) * nr;
    o.XN = t;  t += DB * nr;
    o.XS = t;  t += seg ? DB * nr : 0;
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

__device__ __forceinline__ Lds make_lds_dense(double *base, int DB, int nr, bool seg = false)
{
    const LdsOff o = lds_offsets_dense(DB, nr, seg);
    Lds L;
    L.col = base + o.col; L.P = base + o.P; L.A = base + o.A; L.Q = base + o.Q; L.R = base + o.R;
    L.W = base + o.W; L.Y = base + o.Y; L.RP = base + o.RP; L.XN = base + o.XN; L.XS = base + o.XS;
    L.XC = base + o.XC; L.XG = base + o.XG; L.PN = base + o.PN; L.PS = base + o.PS; L.PC = base + o.PC;
    L.PG = base + o.PG; L.misc = reinterpret_cast<int *>(base + o.misc);
    return L;
}

// Factor (and with FWD forward-substitute) one chain with one wave: a whole
// system (SEG = false), or segment k of a segmented system (SEG = true; Algorithm 1
// parallel phase with the fill rows of k >= 2).  Writes the factor blocks, y in
// place of the rhs and, for segment k, the partials the sequential phase reads:
// hat A_k, hat Q_k and the separator rhs (k >= 2) in the separator's slots, and in
// the scratch of segment k the arrow partials (-sum hat G hat G^T, -sum hat G y)
// and, when the segment ends on a coupling block hat F_k (k < p), hat F_k hat F_k^T,
// hat G hat F_k^T, -hat F_k y and tilde H_k = -hat F_k hat B^T (Eqs. 8a-8c, 9b-9d).
// Returns the 1-based natural index of the first stage whose pivot is not
// positive and finite, 0 if none.
template <int DB, bool FWD, bool SEG = false>
__device__ __forceinline__ int dense_factor(const Args &a, const SysDesc &sd, const Lds &L, int k = 1)
{
    constexpr int PD = DB + 1, TB = DB / 16, KS = DB / 4, NTL = 64;
    static_assert(DB == 16 || DB == 32, "dense sweep tiles are 16 or 32 wide");
    const int lane = threadIdx.x;
    const int b = sd.b, ng = sd.ng, nr = a.nr, N = sd.N;
    const long long b2 = (long long)b * b;
    double *F = a.F;
    double *RA = L.P;                 // Dw -> L (store staging) -> hat E -> next Dw
    double *RB = L.P + DB * PD;       // L^{-T}: row j holds column j of L^{-1}
    double *RG = L.P + 2 * DB * PD;   // Gw -> hat G -> next Gw (16 rows)
    double *RF = RG + NGM * PD;       // SEG, k >= 2: fill rows Fw -> hat B^T -> next Fw
    double *RAA = RF + DB * PD;       //              hat A_k accumulator
    double *RQ = RAA + DB * PD;       //              hat Q_k accumulator (16 rows)
    double *buf0 = L.col, *buf1 = L.col + DB;
    const int s0 = SEG ? seg_first(sd, k) : 0;
    const int len = SEG ? seg_len(sd, k) : N;
    const bool hasF = SEG && k > 1;
    const int sep = hasF ? sep_of(sd, k) : 0;
    double *sc = F + sd.oScr + (long long)(k - 1) * sd.scrStride;

    // ---- prologue: Dw = D_s0 (sym is taken when it is read), Gw = B_s0, w = r_s0, y_g partial = 0; for k >= 2
    // hat A_k = sym(D_sep), hat Q_k = B_sep, Fw = C_sep^T, separator rhs = r_sep
    {
        const double *D0 = a.D + sd.oD + (long long)s0 * b2;
        for (int e = lane; e < DB * DB; e += NTL) {
            const int r = e / DB, c = e - r * DB;
            RA[r * PD + c] = (r < b && c < b) ? D0[r * b + c] : (r == c ? 1.0 : 0.0);   // symmetrized when read
        }
        const double *B0 = a.B + sd.oB + (long long)s0 * ng * b;
        for (int e = lane; e < NGM * DB; e += NTL) {
            const int q = e / DB, c = e - q * DB;
            RG[q * PD + c] = (q < ng && c < b) ? B0[q * b + c] : 0.0;
        }
        if (FWD) {
            const double *r0 = a.rhs + sd.oRhs + (long long)s0 * b * nr;
            for (int e = lane; e < DB * nr; e += NTL) L.W[e] = (e < b * nr) ? r0[e] : 0.0;
            for (int e = lane; e < NGM * nr; e += NTL) L.XG[e] = 0.0;
        }
        if (hasF) {
            const double *Ds = a.D + sd.oD + (long long)sep * b2, *Cs = a.C + sd.oC + (long long)sep * b2;
            const double *Bs = a.B + sd.oB + (long long)sep * ng * b;
            for (int e = lane; e < DB * DB; e += NTL) {
                const int r = e / DB, c = e - r * DB;
                const bool in = r < b && c < b;
                RAA[r * PD + c] = in ? 0.5 * (Ds[r * b + c] + Ds[c * b + r]) : 0.0;
                RF[r * PD + c] = in ? Cs[c * b + r] : 0.0;
            }
            for (int e = lane; e < NGM * DB; e += NTL) {
                const int q = e / DB, c = e - q * DB;
                RQ[q * PD + c] = (q < ng && c < b) ? Bs[q * b + c] : 0.0;
            }
            if (FWD) {
                const double *rs = a.rhs + sd.oRhs + (long long)sep * b * nr;
                for (int e = lane; e < DB * nr; e += NTL) L.XS[e] = (e < b * nr) ? rs[e] : 0.0;
            }
        }
    }
    wave_sync();

    dx4 accR = {0.0, 0.0, 0.0, 0.0};
    double accR4 = 0.0;                 // the same on 4x4 tiles (ng <= 4), partial per block
    // at most four arrow rows: hat G, hat G hat E^T and hat G hat G^T on 4x4 tiles
    const bool g4 = sd.ng > 0 && sd.ng <= 4;
    constexpr int T4 = DB / 16;         // 4x4x4 instructions per k-chunk (4 column blocks each)
    int failed = 0;
    for (int i = 0; i < len; ++i) {
        const int gs = s0 + i;
        const bool hasN = gs + 1 < N;
        // segment k < p ends on the coupling block hat F_k to the next separator
        const bool endS = SEG && i == len - 1 && hasN;
        const bool nextD = hasN && !endS;   // the chain continues with a diagonal block
        // lane-derived indices and masks are re-derived every stage: hoisting the
        // unrolled per-element addresses and predicates out of the stage loop would
        // keep hundreds of them live across it
        int lane_s = lane;
        asm volatile("" : "+v"(lane_s));
        const int li = lane_s & 15, lk = lane_s >> 4;
        const bool isP = lane_s < DB;
        const bool isI = lane_s >= DB && lane_s < 2 * DB;
        const int ri = isP ? lane_s : lane_s - DB;

        // ---- (0) r_{i+1} and C_i (MFMA operand layout), in flight during the factorization
        double rn[TB][4];   // r_{i+1} in product layout (row 16 rt + 4 v + lk, rhs li)
        if (FWD) {
            const double *rs = a.rhs + sd.oRhs + (long long)(gs + 1) * b * nr;
#pragma unroll
            for (int rt = 0; rt < TB; ++rt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * rt + 4 * v + lk;
                    rn[rt][v] = ld_or_zero(rs, r * nr + li, nextD && r < b && li < nr);
                }
        }
        // the same for a single rhs, row lane_s
        const double rn1 = FWD ? GBlock(a.rhs + sd.oRhs + (long long)(gs + 1) * b, nextD ? b : 0).ld(lane_s * 8) : 0.0;
        double cA[TB][KS];
        const GBlock gC(a.C + sd.oC + (long long)gs * b2, hasN ? b2 : 0);
#pragma unroll
        for (int rt = 0; rt < TB; ++rt)
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) {
                const int r = 16 * rt + li, c = 4 * kk + lk;
                cA[rt][kk] = gC.ld(c < b ? (r * b + c) * 8 : GB_OUT);   // rows past b: past the end
            }
        phase_fence();
        // ---- (1) L = chol(Dw) on the row lanes, L^{-1} on the column lanes
        double vec[DB];
        {
            // every lane reads both candidates (in bounds for all lanes) before any
            // select, so the reads issue together instead of one round trip each
            const double *rowp = RA + (isP ? ri : 0) * PD, *colp = RA + (isP ? ri : 0);
            double lo[DB], up[DB];
#pragma unroll
            for (int c = 0; c < DB; ++c) {
                lo[c] = rowp[c];
                up[c] = colp[c * PD];
            }
            pin_row<DB>(lo);
            pin_row<DB>(up);
            // Dw = sym of the block (the Gram term is symmetric already)
#pragma unroll
            for (int c = 0; c < DB; ++c)
                vec[c] = isP ? 0.5 * (lo[c] + up[c]) : ((isI && c == ri) ? 1.0 : 0.0);
        }
        bool bad = false;
        // Every lane applies every step unmasked.  A row lane at or above the pivot
        // then only changes entries right of its diagonal, which no later step reads
        // and the staging of L clears; an inverse lane right of the pivot holds an
        // exact zero in row c, so its multiplier and update are exact zeros.  Every
        // row lane writes its column entry each step (the slots above the pivot are
        // not read), the other lanes a slot of their own: the step stays one basic
        // block, so all its LDS reads are issued together ahead of their use.
        double *const dummy = L.col + 2 * DB + lane_s;
        *(isP ? buf0 + ri : dummy) = vec[0];
        double *const wr0 = isP ? buf0 + ri : dummy, *const wr1 = isP ? buf1 + ri : dummy;
        const int dkey = isP ? ri : -1;
        wave_sync();
        double col[DB];
#pragma unroll
        for (int l = 0; l < DB; ++l) col[l] = buf0[l];
        // the pivot's square root and its inverse, one step ahead
        double d, inv;
        bad |= !(col[0] > 0.0) || !isfinite(col[0]);
        sqrt_rsqrt(col[0], d, inv);
        static_for<0, DB>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            double *nxt = (c & 1) ? buf0 : buf1;
            // row lanes below the pivot scale their entry of column c to L[ri][c];
            // inverse lanes at or left of the pivot form X[c][ri] = acc[c] / L[c][c]
            const double v = vec[c] * inv;
            const double f = v * inv;
            vec[c] = (dkey == c) ? d : v;
            if constexpr (c + 1 < DB) {
                // the next pivot column first: it is written and read back (a wave's
                // LDS accesses complete in order) while the remaining updates of this
                // step run; the next pivot itself comes straight from its row lane,
                // so its square root does not wait for the LDS round trip
                vec[c + 1] = fma(-f, col[c + 1], vec[c + 1]);
                const double pn = readlane_d(vec[c + 1], c + 1);
                *((c & 1) ? wr0 : wr1) = vec[c + 1];
                wave_sync();
                double coln[DB];
#pragma unroll
                for (int l = c + 1; l < DB; ++l) coln[l] = nxt[l];
                __builtin_amdgcn_sched_barrier(0);
                bad |= !(pn > 0.0) || !isfinite(pn);
                // the stages of that square root depend on each other: the remaining
                // updates of this step fill the gaps between them
                RsqChain q{pn, 0.0, 0.0, 0.0};
                static_for<0, RSQ_STAGES>([&](auto ss) {
                    constexpr int st = decltype(ss)::value;
                    rsq_stage(st, q);
                    constexpr int l0 = c + 2 + 2 * st, l1 = (st + 1 == RSQ_STAGES) ? DB : c + 4 + 2 * st;
#pragma unroll
                    for (int l = l0; l < (l1 < DB ? l1 : DB); ++l) vec[l] = fma(-f, col[l], vec[l]);
                    __builtin_amdgcn_sched_barrier(0);
                });
                d = q.g;
                inv = q.h;
#pragma unroll
                for (int l = c + 1; l < DB; ++l) col[l] = coln[l];
            }
            pin_row<DB>(vec);
        });
        wave_sync();
        if (bad && !failed) failed = gs + 1;
        // C_i and r_{i+1} have long arrived: retire them here, before this stage's
        // first stores, so that no later use of them waits for outstanding stores
        vm_drain();

        phase_fence();
        // ---- (2) L rows and L^{-1} columns into LDS (both as rows: L^{-1} is staged
        // transposed, so the two halves of the wave write in the same instructions);
        // store L.  The row lanes clear what is right of their diagonal; the inverse
        // lanes hold exact zeros above theirs.
        if (isP || isI) {
            double *const dst = (isP ? RA : RB) + ri * PD;
            const int keep = isP ? ri : DB;
#pragma unroll
            for (int c = 0; c < DB; ++c) dst[c] = (c <= keep) ? vec[c] : 0.0;
        }
        wave_sync();

        phase_fence();
        // ---- (3) hat E = C L^{-T}, hat G = Gw L^{-T} (and hat B^T = Fw L^{-T})
        dx4 accE[TB][TB], accG[TB];
#pragma unroll
        for (int ct = 0; ct < TB; ++ct) {
            accG[ct] = dx4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int rt = 0; rt < TB; ++rt) accE[rt][ct] = dx4{0.0, 0.0, 0.0, 0.0};
        }
        // B operand: L^{-T}[k][j] as staged, upper triangular: k-chunks past
        // a tile's last column are zero and skipped.  All operands are read before
        // the first product.
        double bo[KS][TB], ga[KS];
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            ga[kk] = RG[li * PD + 4 * kk + lk];
#pragma unroll
            for (int ct = 0; ct < TB; ++ct) bo[kk][ct] = RB[(4 * kk + lk) * PD + 16 * ct + li];
        }
        if (hasN) {
#pragma unroll
            for (int kk = 0; kk < KS; ++kk)
#pragma unroll
                for (int ct = 0; ct < TB; ++ct) {
                    if (4 * kk > 16 * ct + 15) continue;
#pragma unroll
                    for (int rt = 0; rt < TB; ++rt) accE[rt][ct] = mfma4(cA[rt][kk], bo[kk][ct], accE[rt][ct]);
                }
        }
        const int x4 = lane_s & 3, k4 = (lane_s >> 2) & 3, y4 = lane_s >> 4;
        double accG4[T4];
#pragma unroll
        for (int t = 0; t < T4; ++t) accG4[t] = 0.0;
        if (g4) {
            // hat G[y4][4 (4 t + k4) + x4] per lane: A = Gw[x4][4 kc + y4], B = L^{-1} rows
            // (columns of the staged L^{-T})
            double av[KS], bv[KS][T4];
#pragma unroll
            for (int kc = 0; kc < KS; ++kc) {
                av[kc] = RG[x4 * PD + 4 * kc + y4];
#pragma unroll
                for (int t = 0; t < T4; ++t) bv[kc][t] = RB[(4 * kc + y4) * PD + 4 * (4 * t + k4) + x4];
            }
#pragma unroll
            for (int kc = 0; kc < KS; ++kc)
#pragma unroll
                for (int t = 0; t < T4; ++t) {
                    if (kc > 4 * t + 3) continue;   // L^{-T} is zero there for all four blocks
                    accG4[t] = mfma44(av[kc], bv[kc][t], accG4[t]);
                }
        } else if (ng) {
#pragma unroll
            for (int kk = 0; kk < KS; ++kk)
#pragma unroll
                for (int ct = 0; ct < TB; ++ct) {
                    if (4 * kk > 16 * ct + 15) continue;
                    accG[ct] = mfma4(ga[kk], bo[kk][ct], accG[ct]);
                }
        }
        // while the products run on the matrix cores: L goes out, and with one rhs
        // y = L^{-1} w is formed on the row lanes
        store_tile<DB, DB>(GBlock(F + sd.oLd + (long long)gs * b2, b2), RA, b, lane_s);
        if (FWD && nr == 1) {
            const double yv = row_dot1<DB, true>(RB, PD, lane_s < DB ? lane_s : 0, L.W);
            if (lane_s < DB) L.Y[lane_s] = yv;
        }
        wave_sync();
        // hat E and hat G go to the factor straight from the accumulators (each
        // element v of a tile is 4 rows of 16 consecutive entries)
        if (hasN) {
            const GBlock gE(F + sd.oLc + (long long)gs * b2, b2);
#pragma unroll
            for (int rt = 0; rt < TB; ++rt)
#pragma unroll
                for (int ct = 0; ct < TB; ++ct)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = 16 * rt + 4 * v + lk, c = 16 * ct + li;
                        gE.st(c < b ? (r * b + c) * 8 : GB_OUT, accE[rt][ct][v]);
                    }
        }
        if (g4) {
            const GBlock gG(F + sd.oLb + (long long)gs * ng * b, (long long)ng * b);
#pragma unroll
            for (int t = 0; t < T4; ++t) {
                const int c = 4 * (4 * t + k4) + x4;
                gG.st(c < b ? (y4 * b + c) * 8 : GB_OUT, accG4[t]);
            }
        } else if (ng) {
            const GBlock gG(F + sd.oLb + (long long)gs * ng * b, (long long)ng * b);
#pragma unroll
            for (int ct = 0; ct < TB; ++ct)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int q = 4 * v + lk, c = 16 * ct + li;
                    gG.st(c < b ? (q * b + c) * 8 : GB_OUT, accG[ct][v]);
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
            }
        if (g4) {
            // rows 0..3 of the arrow tile (the rows below stay zero)
#pragma unroll
            for (int t = 0; t < T4; ++t) RG[y4 * PD + 4 * (4 * t + k4) + x4] = accG4[t];
        } else {
#pragma unroll
            for (int ct = 0; ct < TB; ++ct)
#pragma unroll
                for (int v = 0; v < 4; ++v) RG[(4 * v + lk) * PD + 16 * ct + li] = accG[ct][v];
        }
        wave_sync();
        if (SEG && hasF) {
            dx4 accF[TB][TB];
#pragma unroll
            for (int rt = 0; rt < TB; ++rt)
#pragma unroll
                for (int ct = 0; ct < TB; ++ct) accF[rt][ct] = dx4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < KS; ++kk)
#pragma unroll
                for (int ct = 0; ct < TB; ++ct) {
                    if (4 * kk > 16 * ct + 15) continue;
#pragma unroll
                    for (int rt = 0; rt < TB; ++rt)
                        accF[rt][ct] = mfma4(RF[(16 * rt + li) * PD + 4 * kk + lk], bo[kk][ct], accF[rt][ct]);
                }
            wave_sync();
#pragma unroll
            for (int rt = 0; rt < TB; ++rt)
#pragma unroll
                for (int ct = 0; ct < TB; ++ct)
#pragma unroll
                    for (int v = 0; v < 4; ++v) RF[(16 * rt + 4 * v + lk) * PD + 16 * ct + li] = accF[rt][ct][v];
            wave_sync();
            // the first fill block sits in the coupling slot of the separator
            double *dst = (i == 0) ? F + sd.oLc + (long long)sep * b2
                                   : F + sd.oFill + ((long long)(k - 2) * (sd.Nk - 1) + (i - 1)) * b2;
            store_tile<DB, DB>(GBlock(dst, b2), RF, b, lane_s);
        }

        phase_fence();
        // ---- next stage's blocks, in flight during the forward substitution
        // D_{i+1} as stored (all tiles, in accumulator layout: coalesced rows); the
        // next factorization symmetrizes it when it reads the block
        double dn[TB][TB][4];
        const GBlock gD(a.D + sd.oD + (long long)(gs + 1) * b2, nextD ? b2 : 0);
#pragma unroll
        for (int rt = 0; rt < TB; ++rt)
#pragma unroll
            for (int ct = 0; ct < TB; ++ct)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * rt + 4 * v + lk, c = 16 * ct + li;
                    dn[rt][ct][v] = gD.ld(c < b ? (r * b + c) * 8 : GB_OUT);
                }
        double bn[TB][4];
        const GBlock gB(a.B + sd.oB + (long long)(gs + 1) * ng * b, nextD ? (long long)ng * b : 0);
#pragma unroll
        for (int ct = 0; ct < TB; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int q = 4 * v + lk, c = 16 * ct + li;
                bn[ct][v] = gB.ld(c < b ? (q * b + c) * 8 : GB_OUT);
            }
        double bn4[T4];
#pragma unroll
        for (int t = 0; t < T4; ++t) {
            const int c = 4 * (4 * t + k4) + x4;
            bn4[t] = gB.ld(g4 && c < b ? (y4 * b + c) * 8 : GB_OUT);
        }

        phase_fence();
        // ---- (4) forward substitution: y = L^{-1} w, w' = r_{i+1} - hat E y, y_g -= hat G y
        // (at a segment end the scratch gets -hat F_k y instead of w'; with fill rows
        // the separator rhs -= hat B^T y)
        if (FWD && nr == 1) {
            // one rhs (y = L^{-1} w is in LDS already): hat E y (or hat F_k y) and,
            // with fill rows, hat B^T y on the row lanes and hat G y on the next 16 lanes
            const int r = lane_s;
            const bool rowL = r < DB, gl = r >= DB && r < DB + NGM;
            const int q = r - DB;
            const double ev = row_dot1<DB, false>(rowL ? RA : RG, PD, rowL ? r : (gl ? q : 0), L.Y);
            const double sv = (SEG && hasF) ? row_dot1<DB, false>(RF, PD, rowL ? r : 0, L.Y) : 0.0;
            wave_sync();
            if (rowL) {
                if (endS) {
                    if (r < b) sc[scr_dy(b, ng, 1) + r] = -ev;
                } else {
                    L.W[r] = (r < b) ? rn1 - ev : 0.0;
                }
                if (SEG && hasF && r < b) L.XS[r] -= sv;
            } else if (gl && q < ng) {
                L.XG[q] -= ev;
            }
        } else if (FWD) {
            // y = L^{-1} w, then hat E y and hat G y, all rhs at once on the matrix cores
            dx4 accY[TB];
#pragma unroll
            for (int rt = 0; rt < TB; ++rt) accY[rt] = dx4{0.0, 0.0, 0.0, 0.0};
            mm_rhs<TB, DB, true, true>(RB, PD, L.W, nr, accY, li, lk);
            if (li < nr) {
#pragma unroll
                for (int rt = 0; rt < TB; ++rt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = 16 * rt + 4 * v + lk;
                        L.Y[r * nr + li] = accY[rt][v];
                    }
            }
            wave_sync();
            dx4 accW[TB], accG1[1], accS[TB];
#pragma unroll
            for (int rt = 0; rt < TB; ++rt) {
                accW[rt] = dx4{0.0, 0.0, 0.0, 0.0};
                accS[rt] = dx4{0.0, 0.0, 0.0, 0.0};
            }
            accG1[0] = dx4{0.0, 0.0, 0.0, 0.0};
            if (hasN) mm_rhs<TB, DB, false>(RA, PD, L.Y, nr, accW, li, lk);
            if (ng) mm_rhs<1, DB, false>(RG, PD, L.Y, nr, accG1, li, lk);
            if (SEG && hasF) mm_rhs<TB, DB, false>(RF, PD, L.Y, nr, accS, li, lk);
            wave_sync();
            if (li < nr) {
#pragma unroll
                for (int rt = 0; rt < TB; ++rt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = 16 * rt + 4 * v + lk;
                        if (endS) {
                            if (r < b) sc[scr_dy(b, ng, nr) + r * nr + li] = -accW[rt][v];
                        } else {
                            L.W[r * nr + li] = (r < b) ? rn[rt][v] - accW[rt][v] : 0.0;
                        }
                        if (SEG && hasF && r < b) L.XS[r * nr + li] -= accS[rt][v];
                    }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int q = 4 * v + lk;
                    if (q < ng) L.XG[q * nr + li] -= accG1[0][v];
                }
            }
                }

        phase_fence();
        // ---- (5) Gram: next Dw and Gw (or, at a segment end, the scratch products),
        // arrow accumulator, fill-row products
        dx4 accD[TB][TB], accB[TB];
#pragma unroll
        for (int rt = 0; rt < TB; ++rt)
#pragma unroll
            for (int ct = 0; ct < TB; ++ct)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * rt + 4 * v + lk, c = 16 * ct + li;
                    accD[rt][ct][v] = endS ? 0.0 : ((r < b && c < b) ? dn[rt][ct][v] : (r == c ? 1.0 : 0.0));
                }
#pragma unroll
        for (int ct = 0; ct < TB; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) accB[ct][v] = bn[ct][v];
        // every operand is read before the first product
        double ek[KS][TB], gk[KS];
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            gk[kk] = RG[li * PD + 4 * kk + lk];
#pragma unroll
            for (int t = 0; t < TB; ++t) ek[kk][t] = RA[(16 * t + li) * PD + 4 * kk + lk];
        }
        // Only the tiles on and below the diagonal carry the product into the next
        // factorization: it reads sym of the block, so the tiles below the diagonal
        // are written back as D - 2 hat E hat E^T and those above as D alone, whose
        // half-sum is sym(D) - hat E hat E^T.  A segment end keeps every tile.
        if (hasN) {
#pragma unroll
            for (int kk = 0; kk < KS; ++kk)
#pragma unroll
                for (int rt = 0; rt < TB; ++rt)
#pragma unroll
                    for (int ct = 0; ct <= rt; ++ct)
                        accD[rt][ct] = mfma4(-ek[kk][rt], ek[kk][ct], accD[rt][ct]);
            if (endS) {
#pragma unroll
                for (int kk = 0; kk < KS; ++kk)
#pragma unroll
                    for (int rt = 0; rt < TB; ++rt)
#pragma unroll
                        for (int ct = rt + 1; ct < TB; ++ct)
                            accD[rt][ct] = mfma4(-ek[kk][rt], ek[kk][ct], accD[rt][ct]);
            }
        }
        double accB4[T4];
#pragma unroll
        for (int t = 0; t < T4; ++t) accB4[t] = bn4[t];
        if (g4) {
            // A = hat G[x4][4 kc + y4]; next Gw -= hat G hat E^T (B = hat E rows), and
            // hat G hat G^T with k-chunk 4 s + k4 in block k4 (summed over the blocks
            // at the end of the sweep)
            double gv[KS], evv[KS][T4];
#pragma unroll
            for (int kc = 0; kc < KS; ++kc) {
                gv[kc] = RG[x4 * PD + 4 * kc + y4];
#pragma unroll
                for (int t = 0; t < T4; ++t) evv[kc][t] = RA[(4 * (4 * t + k4) + x4) * PD + 4 * kc + y4];
            }
            if (hasN) {
#pragma unroll
                for (int kc = 0; kc < KS; ++kc)
#pragma unroll
                    for (int t = 0; t < T4; ++t) accB4[t] = mfma44(-gv[kc], evv[kc][t], accB4[t]);
            }
#pragma unroll
            for (int sc4 = 0; sc4 < T4; ++sc4) {
                const double gr = RG[x4 * PD + 4 * (4 * sc4 + k4) + y4];
                accR4 = mfma44(-gr, gr, accR4);
            }
        } else if (ng) {
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) {
                if (hasN) {
#pragma unroll
                    for (int ct = 0; ct < TB; ++ct) accB[ct] = mfma4(-gk[kk], ek[kk][ct], accB[ct]);
                }
                accR = mfma4(-gk[kk], gk[kk], accR);
            }
        }
        if (SEG && hasF) {
            // hat A_k -= hat B^T hat B, hat Q_k -= hat G hat B, next Fw = -hat B^T hat E^T,
            // and at a segment end tilde H_k = -hat F_k hat B
            dx4 accA[TB][TB], accQ[TB];
#pragma unroll
            for (int rt = 0; rt < TB; ++rt)
#pragma unroll
                for (int ct = 0; ct < TB; ++ct)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        accA[rt][ct][v] = RAA[(16 * rt + 4 * v + lk) * PD + 16 * ct + li];
#pragma unroll
            for (int ct = 0; ct < TB; ++ct)
#pragma unroll
                for (int v = 0; v < 4; ++v) accQ[ct][v] = RQ[(4 * v + lk) * PD + 16 * ct + li];
            double fk[KS][TB];
#pragma unroll
            for (int kk = 0; kk < KS; ++kk)
#pragma unroll
                for (int t = 0; t < TB; ++t) fk[kk][t] = RF[(16 * t + li) * PD + 4 * kk + lk];
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) {
#pragma unroll
                for (int rt = 0; rt < TB; ++rt)
#pragma unroll
                    for (int ct = 0; ct < TB; ++ct) accA[rt][ct] = mfma4(-fk[kk][rt], fk[kk][ct], accA[rt][ct]);
                if (ng) {
#pragma unroll
                    for (int ct = 0; ct < TB; ++ct) accQ[ct] = mfma4(-gk[kk], fk[kk][ct], accQ[ct]);
                }
            }
            dx4 accN[TB][TB];   // -hat B^T hat E^T (next Fw), or -hat E hat B^T (tilde H_k)
#pragma unroll
            for (int rt = 0; rt < TB; ++rt)
#pragma unroll
                for (int ct = 0; ct < TB; ++ct) accN[rt][ct] = dx4{0.0, 0.0, 0.0, 0.0};
            if (hasN) {
#pragma unroll
                for (int kk = 0; kk < KS; ++kk) {
#pragma unroll
                    for (int rt = 0; rt < TB; ++rt)
#pragma unroll
                        for (int ct = 0; ct < TB; ++ct)
                            accN[rt][ct] = endS ? mfma4(-ek[kk][rt], fk[kk][ct], accN[rt][ct])
                                                : mfma4(-fk[kk][rt], ek[kk][ct], accN[rt][ct]);
                }
            }
            wave_sync();
#pragma unroll
            for (int rt = 0; rt < TB; ++rt)
#pragma unroll
                for (int ct = 0; ct < TB; ++ct)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = 16 * rt + 4 * v + lk, c = 16 * ct + li;
                        RAA[r * PD + c] = accA[rt][ct][v];
                        if (endS) {
                            if (r < b && c < b) F[sd.oH + (long long)(k - 2) * b2 + r * b + c] = accN[rt][ct][v];
                        } else {
                            RF[r * PD + c] = accN[rt][ct][v];
                        }
                    }
#pragma unroll
            for (int ct = 0; ct < TB; ++ct)
#pragma unroll
                for (int v = 0; v < 4; ++v) RQ[(4 * v + lk) * PD + 16 * ct + li] = accQ[ct][v];
        }
        // the next stage's blocks replace hat E and hat G only now: the fill-row
        // products above read them
        wave_sync();
        if (nextD) {
#pragma unroll
            for (int rt = 0; rt < TB; ++rt)
#pragma unroll
                for (int ct = 0; ct < TB; ++ct)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = 16 * rt + 4 * v + lk, c = 16 * ct + li;
                        double o = accD[rt][ct][v];
                        if (ct < rt) o = fma(2.0, o, -((r < b && c < b) ? dn[rt][ct][v] : 0.0));
                        RA[r * PD + c] = o;
                    }
            if (g4) {
#pragma unroll
                for (int t = 0; t < T4; ++t) RG[y4 * PD + 4 * (4 * t + k4) + x4] = accB4[t];
            } else {
#pragma unroll
                for (int ct = 0; ct < TB; ++ct)
#pragma unroll
                    for (int v = 0; v < 4; ++v) RG[(4 * v + lk) * PD + 16 * ct + li] = accB[ct][v];
            }
        } else if (SEG && endS) {
            // hat F_k hat F_k^T and hat G hat F_k^T (accumulated as negatives)
#pragma unroll
            for (int rt = 0; rt < TB; ++rt)
#pragma unroll
                for (int ct = 0; ct < TB; ++ct)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = 16 * rt + 4 * v + lk, c = 16 * ct + li;
                        if (r < b && c < b) sc[scr_dA(b, ng, nr) + r * b + c] = -accD[rt][ct][v];
                    }
            if (g4) {
#pragma unroll
                for (int t = 0; t < T4; ++t) {
                    const int c = 4 * (4 * t + k4) + x4;
                    if (y4 < ng && c < b) sc[scr_dQ(b, ng, nr) + y4 * b + c] = -accB4[t];
                }
            } else {
#pragma unroll
                for (int ct = 0; ct < TB; ++ct)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int q = 4 * v + lk, c = 16 * ct + li;
                        if (q < ng && c < b) sc[scr_dQ(b, ng, nr) + q * b + c] = -accB[ct][v];
                    }
            }
        }
        wave_sync();
        // y_i goes out only now: stored earlier, the wait for the next stage's blocks
        // in the Gram would also wait for these stores
        if (FWD) {
            // uniform trip count, stores past the block dropped: no divergent branch
            const GBlock gy(a.rhs + sd.oRhs + (long long)gs * b * nr, (long long)b * nr);
            for (int e0 = 0; e0 < b * nr; e0 += NTL) {
                const int e = e0 + lane_s;
                gy.st(e * 8, L.Y[e < DB * nr ? e : 0]);
            }
        }
    }

    // ---- epilogue: separator partials (k >= 2) and the arrow partials of segment k
    if (SEG && hasF) {
        store_block<NTL, DB * DB>(F + sd.oLd + (long long)sep * b2, RAA, PD, b, b);
        if (ng) store_block<NTL, NGM * DB>(F + sd.oLb + (long long)sep * ng * b, RQ, PD, ng, b);
        if (FWD)
            for (int e = lane; e < b * nr; e += NTL) a.rhs[sd.oRhs + (long long)sep * b * nr + e] = L.XS[e];
    }
    if (g4) {
        // the four blocks' partial sums of hat G hat G^T, through the (now free)
        // pivot-column buffer
        L.col[lane] = accR4;
        wave_sync();
        const int x = lane & 3, y = lane >> 4;
        if (((lane >> 2) & 3) == 0 && y < ng && x < ng)
            sc[scr_Rk(b, ng, nr) + y * ng + x] = L.col[lane] + L.col[lane + 4] + L.col[lane + 8] + L.col[lane + 12];
        wave_sync();
        if (FWD)
            for (int e = lane; e < ng * nr; e += NTL) sc[scr_yg(b, ng, nr) + e] = L.XG[e];
    } else if (ng) {
        const int li = lane & 15, lk = lane >> 4;
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

// Factor blocks and y of stage i, fetched into registers: the blocks in the tile
// mapping (entries outside a block fetched as zeros), the rhs rows as element
// e = lane + 64 m.
template <int DB>
struct BwdStage {
    static constexpr int NTL = 64, MD = DB * DB / NTL, MG = NGM * DB / NTL,
                         MY = (DB * MAX_NRHS_DEV + NTL - 1) / NTL;
    double d[MD], e[MD], g[MG], y[MY], px[MY], f[MD];

    // fill block of stage i of segment k >= 2 (local stage il)
    __device__ __forceinline__ void fetch_fill(const Args &a, const SysDesc &sd, int k, int il, int lane)
    {
        const int b = sd.b;
        const long long b2 = (long long)b * b;
        const double *src = (il == 0) ? a.F + sd.oLc + (long long)sep_of(sd, k) * b2
                                      : a.F + sd.oFill + ((long long)(k - 2) * (sd.Nk - 1) + (il - 1)) * b2;
        const TileMap<DB> t(lane);
        const GBlock gF(src, b2);
        const int base = t.c < b ? (t.r0 * b + t.c) * 8 : GB_OUT;   // rows past b: past the end
#pragma unroll
        for (int m = 0; m < MD; ++m) f[m] = gF.ld(base + TileMap<DB>::RS * m * b * 8);
    }

    __device__ __forceinline__ void stage_fill(const SysDesc &sd, double *stF, int lane) const
    {
        constexpr int PD = DB + 1;
        const TileMap<DB> t(lane);
#pragma unroll
        for (int m = 0; m < MD; ++m) stF[t.row(m) * PD + t.c] = f[m];   // zeros outside the block
    }

    // with PRIMAL, also the primal solution of stage i (adjoint gradients)
    template <bool PRIMAL = false>
    __device__ __forceinline__ void fetch(const Args &a, const SysDesc &sd, int i, int lane)
    {
        const int b = sd.b, ng = sd.ng, nr = a.nr;
        const long long b2 = (long long)b * b;
        const bool hasE = i + 1 < sd.N;
        const GBlock gLd(a.F + sd.oLd + (long long)i * b2, b2), gLc(a.F + sd.oLc + (long long)i * b2, hasE ? b2 : 0);
        const GBlock gLb(a.F + sd.oLb + (long long)i * ng * b, (long long)ng * b);
        const GBlock gY(a.rhs + sd.oRhs + (long long)i * b * nr, (long long)b * nr);
        const TileMap<DB> t(lane);
        // one lane offset for all three blocks (b columns each): rows past the
        // block's last fall past its end
        const int base = t.c < b ? (t.r0 * b + t.c) * 8 : GB_OUT;
#pragma unroll
        for (int m = 0; m < MD; ++m) {
            d[m] = gLd.ld(base + TileMap<DB>::RS * m * b * 8);
            e[m] = gLc.ld(base + TileMap<DB>::RS * m * b * 8);
        }
#pragma unroll
        for (int m = 0; m < MG; ++m) g[m] = gLb.ld(base + TileMap<DB>::RS * m * b * 8);
#pragma unroll
        for (int m = 0; m < MY; ++m) y[m] = gY.ld((lane + m * NTL) * 8);
        if (PRIMAL) {
            const GBlock gP(a.xp + sd.oRhs + (long long)i * b * nr, (long long)b * nr);
#pragma unroll
            for (int m = 0; m < MY; ++m) px[m] = gP.ld((lane + m * NTL) * 8);
        }
    }

    // into the staging area (rows of pitch DB + 1) and XC
    __device__ __forceinline__ void stage(const SysDesc &sd, int nr, double *stD, double *stE, double *stG, double *XC,
                                          int lane) const
    {
        constexpr int PD = DB + 1;
        const int b = sd.b;
        const TileMap<DB> t(lane);
        // whole tiles: the entries outside the blocks were fetched as zeros
#pragma unroll
        for (int m = 0; m < MD; ++m) {
            stD[t.row(m) * PD + t.c] = d[m];
            stE[t.row(m) * PD + t.c] = e[m];
        }
#pragma unroll
        for (int m = 0; m < MG; ++m) stG[t.row(m) * PD + t.c] = g[m];
#pragma unroll
        for (int m = 0; m < MY; ++m) {
            const int x = lane + m * NTL;
            if (x < b * nr) XC[x] = y[m];
        }
    }

    __device__ __forceinline__ void stage_primal(const SysDesc &sd, int nr, double *PC, int lane) const
    {
#pragma unroll
        for (int m = 0; m < MY; ++m) {
            const int x = lane + m * NTL;
            if (x < sd.b * nr) PC[x] = px[m];
        }
    }
};

// Forward substitution of a whole system with one wave and the factor in place
// (Algorithm 2 with p = 1): y_i = L_ii^{-1} w_i, w_{i+1} = r_{i+1} - hat E_i y_i,
// y_g partial -= hat G_i y_i; y overwrites the rhs, the y_g partial goes to the
// scratch of segment 1.  The blocks and rhs of stage i + 1 are in flight while
// stage i is solved.
template <int DB>
__device__ __forceinline__ void dense_forward(const Args &a, const SysDesc &sd, const Lds &L)
{
    constexpr int PD = DB + 1, NTL = 64, MY = BwdStage<DB>::MY;
    const int lane = threadIdx.x;
    const int b = sd.b, ng = sd.ng, nr = a.nr, N = sd.N;
    double *X = a.rhs + sd.oRhs;
    double *stD = L.P, *stE = L.P + DB * PD, *stG = L.P + 2 * DB * PD;
    for (int e = lane; e < DB * nr; e += NTL) L.W[e] = (e < b * nr) ? X[e] : 0.0;
    for (int e = lane; e < NGM * nr; e += NTL) L.XG[e] = 0.0;
    // the staging area outside the b x b (ng x b) blocks stays zero for the products
    for (int e = lane; e < (2 * DB + NGM) * PD; e += NTL) L.P[e] = 0.0;
    BwdStage<DB> pf;
    pf.fetch(a, sd, 0, lane);
    for (int i = 0; i < N; ++i) {
        int lane_s = lane;
        asm volatile("" : "+v"(lane_s));
        const int r = lane_s;
        const bool rv = r < b;
        const bool hasN = i + 1 < N;
        wave_sync();
        pf.stage(sd, nr, stD, stE, stG, L.XC, lane_s);   // XC receives r_i (unused; w_i is in W)
        wave_sync();
        // y of the previous stage goes out only now, after the wait for this stage's
        // blocks: stored earlier, that wait would also wait for the stores
        if (i > 0)
            for (int e = lane_s; e < b * nr; e += NTL) X[(long long)(i - 1) * b * nr + e] = L.Y[e];
        if (hasN) pf.fetch(a, sd, i + 1, lane_s);
        double drow[DB];
#pragma unroll
        for (int c = 0; c < DB; ++c) {
            const double v = stD[(rv ? r : 0) * PD + c];
            drow[c] = (rv && c < b) ? (c <= r ? v : 0.0) : (c == r ? 1.0 : 0.0);
        }
        const double dinv = rv ? 1.0 / stD[r * PD + r] : 1.0;
        for (int j = 0; j < nr; ++j) {
            const double w = rv ? L.W[r * nr + j] : 0.0;
            const double yv = fwd_subst<DB>(drow, w, dinv);
            wave_sync();
            if (rv) {
                L.Y[r * nr + j] = yv;
            } else if (r < DB) {
                L.Y[r * nr + j] = 0.0;
            }
            wave_sync();
        }
        if (nr == 1) {
            // one rhs: hat E y on the row lanes, hat G y on the next 16 lanes
            const bool rowL = r < DB, gl = r >= DB && r < DB + NGM;
            const int q = r - DB;
            const double ev = row_dot1<DB, false>(rowL ? stE : stG, PD, rowL ? r : (gl ? q : 0), L.Y);
            wave_sync();
            if (rowL) {
                if (hasN) L.XN[r] = ev;
            } else if (gl && q < ng) {
                L.XG[q] -= ev;
            }
            wave_sync();
        } else {
            // hat E y and hat G y for all rhs on the matrix cores
            const int li = lane_s & 15, lk = lane_s >> 4;
            constexpr int TB = DB / 16;
            dx4 accW[TB], accG1[1];
#pragma unroll
            for (int rt = 0; rt < TB; ++rt) accW[rt] = dx4{0.0, 0.0, 0.0, 0.0};
            accG1[0] = dx4{0.0, 0.0, 0.0, 0.0};
            if (hasN) mm_rhs<TB, DB, false>(stE, PD, L.Y, nr, accW, li, lk);
            if (ng) mm_rhs<1, DB, false>(stG, PD, L.Y, nr, accG1, li, lk);
            wave_sync();
            if (li < nr) {
                if (hasN) {
#pragma unroll
                    for (int rt = 0; rt < TB; ++rt)
#pragma unroll
                        for (int v = 0; v < 4; ++v) L.XN[(16 * rt + 4 * v + lk) * nr + li] = accW[rt][v];
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int q = 4 * v + lk;
                    if (q < ng) L.XG[q * nr + li] -= accG1[0][v];
                }
            }
            wave_sync();
        }
        // w_{i+1} = r_{i+1} - hat E y (r_{i+1} is in flight in pf.y)
        if (hasN) {
#pragma unroll
            for (int m = 0; m < MY; ++m) {
                const int e = lane_s + m * NTL;
                if (e < DB * nr) L.W[e] = (e < b * nr) ? pf.y[m] - L.XN[e] : 0.0;
            }
        }
    }
    wave_sync();
    for (int e = lane; e < b * nr; e += NTL) X[(long long)(N - 1) * b * nr + e] = L.Y[e];
    if (ng)
        for (int e = lane; e < ng * nr; e += NTL) a.F[sd.oScr + scr_yg(b, ng, nr) + e] = L.XG[e];
    wave_sync();
}

// Backward substitution with one wave (Algorithm 3): a whole system, or (SEG)
// segment k of a segmented system after the sequential phase has solved its
// separators.  x_i = L_ii^{-T} (y_i - hat E_i^T x_{i+1} - hat G_i^T x_g
// [- hat B_i x_sep]) for the chain's stages in reverse, with the blocks of the
// next stage in flight while a stage is solved; x_g (and x at the separators) is
// in place.  With ADJ (whole systems) the solution is lambda and the gradient
// blocks of every stage are written: dD_i = -sym(lambda_i x_i^T),
// dB_i = -(lambda_g x_i^T + x_g lambda_i^T), dC_i = -(lambda_{i+1} x_i^T + x_{i+1} lambda_i^T),
// summed over the rhs columns.
template <int DB, bool ADJ, bool SEG = false>
__device__ __forceinline__ void dense_backward(const Args &a, const SysDesc &sd, const Lds &L, int k = 1)
{
    static_assert(!(ADJ && SEG), "the adjoint runs on whole systems");
    constexpr int PD = DB + 1, NTL = 64;
    const int lane = threadIdx.x;
    const int b = sd.b, ng = sd.ng, nr = a.nr, N = sd.N;
    const long long b2 = (long long)b * b;
    double *X = a.rhs + sd.oRhs;
    double *stD = L.P, *stE = L.P + DB * PD, *stG = L.P + 2 * DB * PD, *stF = stG + NGM * PD;
    const int s0 = SEG ? seg_first(sd, k) : 0;
    const int len = SEG ? seg_len(sd, k) : N;
    const bool hasF = SEG && k > 1;
    const int nxt = s0 + len;   // the separator after the chain (segments k < p)
    for (int e = lane; e < NGM * nr; e += NTL) {
        L.XG[e] = (e < ng * nr) ? X[(long long)N * b * nr + e] : 0.0;
        if (ADJ) L.PG[e] = (e < ng * nr) ? a.xp[sd.oRhs + (long long)N * b * nr + e] : 0.0;
    }
    for (int e = lane; e < DB * nr; e += NTL) {
        L.XN[e] = (SEG && nxt < N && e < b * nr) ? X[(long long)nxt * b * nr + e] : 0.0;
        if (ADJ) L.PN[e] = 0.0;
        if (SEG) L.XS[e] = (hasF && e < b * nr) ? X[(long long)sep_of(sd, k) * b * nr + e] : 0.0;
    }
    // the staging area outside the b x b (ng x b) blocks stays zero for the products
    for (int e = lane; e < ((SEG ? 3 : 2) * DB + NGM) * PD; e += NTL) L.P[e] = 0.0;
    BwdStage<DB> pf;
    pf.template fetch<ADJ>(a, sd, s0 + len - 1, lane);
    if (hasF) pf.fetch_fill(a, sd, k, len - 1, lane);
    for (int i = len - 1; i >= 0; --i) {
        int lane_s = lane;
        asm volatile("" : "+v"(lane_s));
        const int gs = s0 + i;
        const int c = lane_s;
        const bool cv = c < b;
        const bool hasE = gs + 1 < N;
        wave_sync();
        pf.stage(sd, nr, stD, stE, stG, L.XC, lane_s);
        if (ADJ) pf.stage_primal(sd, nr, L.PC, lane_s);
        if (hasF) pf.stage_fill(sd, stF, lane_s);
        wave_sync();
        // x of the stage solved last goes out only now, after the wait for this
        // stage's blocks: stored earlier, that wait would also wait for the stores
        if (i < len - 1) {
            const GBlock gx(X + (long long)(gs + 1) * b * nr, (long long)b * nr);
            for (int e0 = 0; e0 < b * nr; e0 += NTL) {
                const int e = e0 + lane_s;
                gx.st(e * 8, L.XN[e < DB * nr ? e : 0]);
            }
        }
        if (i > 0) {
            pf.template fetch<ADJ>(a, sd, gs - 1, lane_s);
            if (hasF) pf.fetch_fill(a, sd, k, i - 1, lane_s);
        }
        double dcol[DB];
#pragma unroll
        for (int l = 0; l < DB; ++l) {
            const double v = stD[l * PD + (cv ? c : 0)];
            dcol[l] = (cv && l < b && l != c) ? v : 0.0;   // the diagonal is taken out
        }
        const double dinv = cv ? 1.0 / stD[c * PD + c] : 1.0;
        double dcs[DB];
#pragma unroll
        for (int l = 0; l < DB; ++l) dcs[l] = dcol[l] * dinv;
        if (nr == 1) {
            // one rhs: column c of each block on lane c, on the vector units
            const int cc = c < DB ? c : 0;
            double t = 0.0;
            // (short chunks: this sweep holds the next stage's blocks in registers)
            constexpr int CH = ADJ ? 4 : 8;
            if (hasE) t += row_dot1<DB, true, CH>(stE, PD, cc, L.XN);
            if (ng) t += row_dot1<NGM, true, CH>(stG, PD, cc, L.XG);
            if (SEG && hasF) t += row_dot1<DB, true, CH>(stF, PD, cc, L.XS);
            if (c < DB) L.Y[c] = t;
        } else {
            // hat E^T x_{i+1} + hat G^T x_g (+ hat B x_sep) for all rhs on the matrix cores, into Y
            const int li = lane_s & 15, lk = lane_s >> 4;
            constexpr int TB = DB / 16;
            dx4 accT[TB];
#pragma unroll
            for (int rt = 0; rt < TB; ++rt) accT[rt] = dx4{0.0, 0.0, 0.0, 0.0};
            if (hasE) mm_rhs<TB, DB, true>(stE, PD, L.XN, nr, accT, li, lk);
            if (ng) mm_rhs<TB, NGM, true>(stG, PD, L.XG, nr, accT, li, lk);
            if (SEG && hasF) mm_rhs<TB, DB, true>(stF, PD, L.XS, nr, accT, li, lk);
            if (li < nr) {
#pragma unroll
                for (int rt = 0; rt < TB; ++rt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) L.Y[(16 * rt + 4 * v + lk) * nr + li] = accT[rt][v];
            }
        }
        wave_sync();
        for (int j = 0; j < nr; ++j) {
            const double acc = cv ? L.XC[c * nr + j] - L.Y[c * nr + j] : 0.0;
            const double xv = back_subst_scaled<DB>(dcs, acc * dinv);
            wave_sync();
            if (cv) L.XC[c * nr + j] = xv;
            wave_sync();
        }
        if (ADJ && nr == 1) {
            // one rhs: the rows unrolled, so their reads from LDS issue together;
            // lane c forms column c of each block.  Rows at or past b land past the
            // block's end and lanes past b are moved there, so the stores are
            // dropped without a per-row mask.
            const int cc = cv ? c : 0, ce = cv ? c : (1 << 20);
            const double pcc = L.PC[cc], xcc = L.XC[cc];
            const GBlock gdD(a.dD + sd.oD + (long long)gs * b2, b2);
            const GBlock gdC(a.dC + sd.oC + (long long)gs * b2, hasE ? b2 : 0);
            const GBlock gdB(a.dB + sd.oB + (long long)gs * ng * b, (long long)ng * b);
#pragma unroll
            for (int r = 0; r < DB; ++r) {
                const int o = (r * b + ce) * 8;
                gdD.st(o, -0.5 * fma(L.XC[r], pcc, L.PC[r] * xcc));
                gdC.st(o, -fma(L.XN[r], pcc, L.PN[r] * xcc));
            }
#pragma unroll
            for (int q = 0; q < NGM; ++q) gdB.st((q * b + ce) * 8, -fma(L.XG[q], pcc, L.PG[q] * xcc));
        } else if (ADJ && cv) {
            double *dD = a.dD + sd.oD + (long long)gs * b2;
            for (int r = 0; r < b; ++r) {
                double s = 0.0;
                for (int j = 0; j < nr; ++j)
                    s += L.XC[r * nr + j] * L.PC[c * nr + j] + L.PC[r * nr + j] * L.XC[c * nr + j];
                dD[r * b + c] = -0.5 * s;
            }
            if (ng) {
                double *dB = a.dB + sd.oB + (long long)gs * ng * b;
                for (int q = 0; q < ng; ++q) {
                    double s = 0.0;
                    for (int j = 0; j < nr; ++j)
                        s += L.XG[q * nr + j] * L.PC[c * nr + j] + L.PG[q * nr + j] * L.XC[c * nr + j];
                    dB[q * b + c] = -s;
                }
            }
            if (hasE) {
                double *dC = a.dC + sd.oC + (long long)gs * b2;
                for (int r = 0; r < b; ++r) {
                    double s = 0.0;
                    for (int j = 0; j < nr; ++j)
                        s += L.XN[r * nr + j] * L.PC[c * nr + j] + L.PN[r * nr + j] * L.XC[c * nr + j];
                    dC[r * b + c] = -s;
                }
            }
        }
        wave_sync();
        if (cv)
            for (int j = 0; j < nr; ++j) {
                L.XN[c * nr + j] = L.XC[c * nr + j];
                if (ADJ) L.PN[c * nr + j] = L.PC[c * nr + j];
            }
    }
    wave_sync();
    for (int e = lane; e < b * nr; e += NTL) X[(long long)s0 * b * nr + e] = L.XN[e];
    wave_sync();
}

}  // namespace kkt_dev
