// Stage sweeps of the segmented block Cholesky (gfx950, FP64): the parallel
// phase of one segment and the sequential phase on the reduced chain.
#pragma once
#include "kkt_device.h"

namespace kkt_dev {

// Where the inputs of one stage of a chain come from.
//   Segment chain (RED = false), stage gs of segment k: D[gs], C[gs] (coupling
//   rows to stage gs+1), B[gs], rhs[gs].
//   Reduced chain (RED = true), stage t <-> separator s = sep_{t+2}: the partial
//   tilde A (Ld[s]) minus hat F hat F^T of the previous segment, tilde H_{t+2}
//   (coupling to the next separator), tilde Q (Lb[s]) minus hat G hat F^T, and
//   the partial tilde y (rhs[s]) plus -hat F hat y (Eqs. 7, 8c, 9d).
template <int BP, bool RED>
struct Chain {
    const Args &a;
    const SysDesc &sd;
    int k;  // segment (RED = false)

    __device__ __forceinline__ int stage(int i) const { return RED ? sep_of(sd, i + 2) : seg_first(sd, k) + i; }
    __device__ __forceinline__ int length() const { return RED ? sd.p - 1 : seg_len(sd, k); }
    __device__ __forceinline__ bool has_next(int i) const { return RED ? (i + 2 < sd.p) : (stage(i) + 1 < sd.N); }
    __device__ __forceinline__ const double *scr(int seg) const { return a.F + sd.oScr + (long long)(seg - 1) * sd.scrStride; }

    // Stage the blocks of stage i into LDS: diagonal at P rows [0, BP), coupling
    // rows at [BP, 2BP), arrow rows at [2BP, 2BP + 16); rhs into W.
    __device__ __forceinline__ void stage_factor_inputs(int i, const Lds &L, bool fwd) const
    {
        constexpr int NT = K<BP>::NT, P = K<BP>::PITCH;
        const int b = sd.b, ng = sd.ng, nr = a.nr, s = stage(i);
        const long long b2 = (long long)b * b;
        if (!RED) {
            load_block<NT, BP * BP>(L.P, P, a.D + sd.oD + s * b2, nullptr, b, b);
            if (has_next(i)) load_block<NT, BP * BP>(L.P + BP * P, P, a.C + sd.oC + s * b2, nullptr, b, b);
            if (ng) load_block<NT, NGM * BP>(L.P + 2 * BP * P, P, a.B + sd.oB + (long long)s * ng * b, nullptr, ng, b);
            if (fwd) load_rhs<NT, BP * 8>(L.W, a.rhs + sd.oRhs + (long long)s * b * nr, nullptr, b * nr);
        } else {
            const double *sc = scr(i + 1);
            load_block<NT, BP * BP>(L.P, P, a.F + sd.oLd + s * b2, sc + scr_dA(b, ng, nr), b, b);
            if (has_next(i)) load_block<NT, BP * BP>(L.P + BP * P, P, a.F + sd.oH + i * b2, nullptr, b, b);
            if (ng) load_block<NT, NGM * BP>(L.P + 2 * BP * P, P, a.F + sd.oLb + (long long)s * ng * b, sc + scr_dQ(b, ng, nr), ng, b);
            if (fwd) load_rhs<NT, BP * 8>(L.W, a.rhs + sd.oRhs + (long long)s * b * nr, sc + scr_dy(b, ng, nr), b * nr);
        }
    }
};

// Factor (and, with FWD, forward-substitute) one chain: a segment (Algorithm 1
// parallel phase with Algorithm 2 parallel phase fused) or the reduced chain
// (Algorithm 1 / 2 sequential phases, without the corner).  Returns the 1-based
// natural index of the first stage whose pivot failed, 0 if none.
template <int BP, bool FWD, bool RED>
__device__ __forceinline__ int sweep_factor(const Args &a, const SysDesc &sd, int k, const Lds &L)
{
    using KK = K<BP>;
    constexpr int NT = KK::NT, P = KK::PITCH, E0 = KK::E0, G0 = KK::G0, F0 = KK::F0, NROWS = KK::NROWS;
    const Chain<BP, RED> ch{a, sd, k};
    const int tid = threadIdx.x;
    const int b = sd.b, ng = sd.ng, nr = a.nr;
    const long long b2 = (long long)b * b;
    double *F = a.F;
    const bool hasF = !RED && k > 1;
    const int len = ch.length();
    const int er = tid - E0, gq = tid - G0, fr = tid - F0;
    const bool isD = tid < BP;
    const bool isE = er >= 0 && er < BP;
    const bool isG = gq >= 0 && gq < ng;
    const bool isF = hasF && fr >= 0 && fr < b;
    const int sep = hasF ? sep_of(sd, k) : -1;
    int failed = 0;
    double row[BP];
#pragma unroll
    for (int c = 0; c < BP; ++c) row[c] = 0.0;

    // ---- prologue: accumulators (Algorithm 1 init; hat R_k = 0, hat A_k = A_k, hat Q_k = Q_k)
    for (int e = tid; e < NGM * NGM; e += NT) L.R[e] = 0.0;
    if (FWD) {
        for (int e = tid; e < NROWS * nr; e += NT) L.RP[e] = 0.0;
        for (int e = tid; e < KK::BPX * nr; e += NT) L.W[e] = 0.0;
    }
    if (hasF) {
        const double *Ds = a.D + sd.oD + sep * b2;
        for (int e = tid; e < b * b; e += NT) {
            const int r = e / b, c = e - r * b;
            L.A[r * P + c] = 0.5 * (Ds[e] + Ds[c * b + r]);
        }
        if (ng) load_block<NT, NGM * BP>(L.Q, P, a.B + sd.oB + (long long)sep * ng * b, nullptr, ng, b);
    }
    __syncthreads();
    ch.stage_factor_inputs(0, L, FWD);
    __syncthreads();
    if (isF) {
        // first fill row: row r of Psi_{sep_k, first(k)} = column r of C_{sep_k}
        const double *Cs = a.C + sd.oC + sep * b2;
#pragma unroll
        for (int c = 0; c < BP; ++c) row[c] = (c < b) ? Cs[c * b + fr] : 0.0;
        if (FWD)
            for (int j = 0; j < nr; ++j) L.RP[tid * nr + j] = a.rhs[sd.oRhs + ((long long)sep * b + fr) * nr + j];
    } else if (isD) {
#pragma unroll
        for (int c = 0; c < BP; ++c)
            row[c] = (tid < b && c < b) ? 0.5 * (L.P[tid * P + c] + L.P[c * P + tid]) : (tid == c ? 1.0 : 0.0);
    } else if (isE) {
        const bool nx = ch.has_next(0);
#pragma unroll
        for (int c = 0; c < BP; ++c) row[c] = (nx && er < b && c < b) ? L.P[(BP + er) * P + c] : 0.0;
    } else if (isG) {
#pragma unroll
        for (int c = 0; c < BP; ++c) row[c] = (c < b) ? L.P[(2 * BP + gq) * P + c] : 0.0;
    }
    __syncthreads();

    for (int i = 0; i < len; ++i) {
        const int gs = ch.stage(i);
        const bool hasE = ch.has_next(i);
        const bool last = (i == len - 1);

        if (eliminate<BP>(row, L, nr, FWD) && !failed) failed = gs + 1;

        // all rows into LDS (hat D with its upper part zeroed), then coalesced stores
        if (tid < NROWS) {
#pragma unroll
            for (int c = 0; c < BP; ++c) L.P[tid * P + c] = (isD && c > tid) ? 0.0 : row[c];
        }
        __syncthreads();
        {
            double *o = F + sd.oLd + gs * b2;
            store_block<NT, BP * BP>(o, L.P, P, b, b);
        }
        if (FWD)
            for (int e = tid; e < b * nr; e += NT) a.rhs[sd.oRhs + (long long)gs * b * nr + e] = L.Y[e];
        if (hasE) {
            double *o = RED ? F + sd.oH + i * b2 : F + sd.oLc + gs * b2;
            store_block<NT, BP * BP>(o, L.P + E0 * P, P, b, b);
        }
        if (ng) {
            double *o = F + sd.oLb + (long long)gs * ng * b;
            store_block<NT, NGM * BP>(o, L.P + G0 * P, P, ng, b);
        }
        if (hasF) {
            double *o = (i == 0) ? F + sd.oLc + sep * b2
                                 : F + sd.oFill + ((long long)(k - 2) * (sd.Nk - 1) + (i - 1)) * b2;
            store_block<NT, BP * BP>(o, L.P + F0 * P, P, b, b);
        }

        // Gram of the panel rows (Eqs. 6, 8a, 8b).  D lanes take the coupling row of
        // their index and produce the next diagonal row; G and F lanes use their own.
        if (isD) {
#pragma unroll
            for (int c = 0; c < BP; ++c) row[c] = L.P[(E0 + tid) * P + c];
        }
        double tE[BP];
#pragma unroll
        for (int r = 0; r < BP; ++r) {
            tE[r] = hasE ? dot_row<BP>(row, L.P + (E0 + r) * P) : 0.0;
            if ((r & 3) == 3) asm volatile("" : "+v"(tE[r]), "+v"(tE[r - 1]), "+v"(tE[r - 2]), "+v"(tE[r - 3]));
        }
        if (hasF && (isG || isF)) {
            for (int c = 0; c < b; ++c) {
                const double s = dot_row<BP>(row, L.P + (F0 + c) * P);
                if (isG) L.Q[gq * P + c] -= s;
                else L.A[fr * P + c] -= s;
            }
        }
        if (isG) {
            for (int q = 0; q < ng; ++q) L.R[gq * NGM + q] -= dot_row<BP>(row, L.P + (G0 + q) * P);
        }
        if (FWD && (isE || isG || isF)) {
            for (int j = 0; j < nr; ++j) {
                const double s = dot_col<BP>(row, L.Y + j, nr);
                if (isE) L.RP[tid * nr + j] = -s;
                else L.RP[tid * nr + j] -= s;
            }
        }
        __syncthreads();

        if (!last) {
            ch.stage_factor_inputs(i + 1, L, FWD);
            __syncthreads();
            if (isD) {
#pragma unroll
                for (int c = 0; c < BP; ++c) {
                    const double dv = (tid < b && c < b) ? 0.5 * (L.P[tid * P + c] + L.P[c * P + tid]) : (tid == c ? 1.0 : 0.0);
                    row[c] = dv - tE[c];
                }
                if (FWD && tid < b)
                    for (int j = 0; j < nr; ++j) L.W[tid * nr + j] += L.RP[(E0 + tid) * nr + j];
            } else if (isE) {
                const bool nx = ch.has_next(i + 1);
#pragma unroll
                for (int c = 0; c < BP; ++c) row[c] = (nx && er < b && c < b) ? L.P[(BP + er) * P + c] : 0.0;
            } else if (isG) {
#pragma unroll
                for (int c = 0; c < BP; ++c) row[c] = ((c < b) ? L.P[(2 * BP + gq) * P + c] : 0.0) - tE[c];
            } else if (isF) {
#pragma unroll
                for (int c = 0; c < BP; ++c) row[c] = -tE[c];
            }
            __syncthreads();
        } else if (hasE) {
            // last stage of segment k < p: the coupling rows are hat F_k (Eqs. 8c, 9d, 8b)
            double *sc = F + sd.oScr + (long long)(k - 1) * sd.scrStride;
            if (isD && tid < b) {
#pragma unroll
                for (int c = 0; c < BP; ++c)
                    if (c < b) sc[scr_dA(b, ng, nr) + tid * b + c] = tE[c];
            } else if (isE && er < b) {
                if (FWD)
                    for (int j = 0; j < nr; ++j) sc[scr_dy(b, ng, nr) + er * nr + j] = L.RP[tid * nr + j];
            } else if (isG) {
#pragma unroll
                for (int c = 0; c < BP; ++c)
                    if (c < b) sc[scr_dQ(b, ng, nr) + gq * b + c] = tE[c];
            } else if (isF) {
                // tilde H_k = -hat F_k hat B_{N_k k}: lane fr holds its column fr
                double *H = F + sd.oH + (long long)(k - 2) * b2;
#pragma unroll
                for (int r = 0; r < BP; ++r)
                    if (r < b) H[r * b + fr] = -tE[r];
            }
        }
    }

    // ---- epilogue: separator accumulators (Eq. 8a) and partials (Eqs. 8b, 9b, 9c)
    if (hasF) {
        double *oA = F + sd.oLd + sep * b2;
        for (int e = tid; e < b * b; e += NT) { const int r = e / b; oA[e] = L.A[r * P + (e - r * b)]; }
        if (ng) {
            double *oQ = F + sd.oLb + (long long)sep * ng * b;
            for (int e = tid; e < ng * b; e += NT) { const int r = e / b; oQ[e] = L.Q[r * P + (e - r * b)]; }
        }
        if (FWD && isF)
            for (int j = 0; j < nr; ++j) a.rhs[sd.oRhs + ((long long)sep * b + fr) * nr + j] = L.RP[tid * nr + j];
    }
    if (!RED && ng) {
        double *sc = F + sd.oScr + (long long)(k - 1) * sd.scrStride;
        for (int e = tid; e < ng * ng; e += NT) { const int r = e / ng; sc[scr_Rk(b, ng, nr) + e] = L.R[r * NGM + (e - r * ng)]; }
        if (FWD && isG)
            for (int j = 0; j < nr; ++j) sc[scr_yg(b, ng, nr) + gq * nr + j] = L.RP[tid * nr + j];
    }
    __syncthreads();
    return failed;
}

// Forward substitution of one chain with a factor already in place
// (Algorithm 2, parallel phase for a segment, sequential phase for RED).
template <int BP, bool RED>
__device__ __forceinline__ void sweep_forward(const Args &a, const SysDesc &sd, int k, const Lds &L)
{
    using KK = K<BP>;
    constexpr int NT = KK::NT, P = KK::PITCH, E0 = KK::E0, G0 = KK::G0, F0 = KK::F0, NROWS = KK::NROWS;
    const Chain<BP, RED> ch{a, sd, k};
    const int tid = threadIdx.x;
    const int b = sd.b, ng = sd.ng, nr = a.nr;
    const long long b2 = (long long)b * b;
    const double *F = a.F;
    const bool hasF = !RED && k > 1;
    const int len = ch.length();
    const int er = tid - E0, gq = tid - G0, fr = tid - F0;
    const bool isE = er >= 0 && er < b;
    const bool isG = gq >= 0 && gq < ng;
    const bool isF = hasF && fr >= 0 && fr < b;
    const int sep = hasF ? sep_of(sd, k) : -1;
    double *stD = L.P, *stE = L.P + BP * P, *stG = L.P + 2 * BP * P, *stF = L.A;

    for (int e = tid; e < NROWS * nr; e += NT) L.RP[e] = 0.0;
    for (int e = tid; e < KK::BPX * nr; e += NT) L.W[e] = 0.0;
    __syncthreads();
    if (isF)
        for (int j = 0; j < nr; ++j) L.RP[tid * nr + j] = a.rhs[sd.oRhs + ((long long)sep * b + fr) * nr + j];
    {
        const int s0 = ch.stage(0);
        const double *add = RED ? ch.scr(1) + scr_dy(b, ng, nr) : nullptr;
        load_rhs<NT, BP * 8>(L.W, a.rhs + sd.oRhs + (long long)s0 * b * nr, add, b * nr);
    }
    for (int i = 0; i < len; ++i) {
        const int gs = ch.stage(i);
        const bool hasE = ch.has_next(i);
        load_block<NT, BP * BP>(stD, P, F + sd.oLd + gs * b2, nullptr, b, b);
        if (hasE) load_block<NT, BP * BP>(stE, P, RED ? F + sd.oH + i * b2 : F + sd.oLc + gs * b2, nullptr, b, b);
        if (ng) load_block<NT, NGM * BP>(stG, P, F + sd.oLb + (long long)gs * ng * b, nullptr, ng, b);
        if (hasF) {
            const double *src = (i == 0) ? F + sd.oLc + sep * b2
                                         : F + sd.oFill + ((long long)(k - 2) * (sd.Nk - 1) + (i - 1)) * b2;
            load_block<NT, BP * BP>(stF, P, src, nullptr, b, b);
        }
        __syncthreads();
        if (tid < 64) {
            double drow[BP];
#pragma unroll
            for (int c = 0; c < BP; ++c)
                drow[c] = (tid < b && c < b) ? (c <= tid ? stD[tid * P + c] : 0.0) : (tid == c ? 1.0 : 0.0);
            const double dinv = (tid < b) ? 1.0 / stD[tid * P + tid] : 1.0;
            for (int j = 0; j < nr; ++j) {
                const double w = (tid < b) ? L.W[tid * nr + j] : 0.0;
                const double y = fwd_subst<BP>(drow, w, dinv);
                if (tid < BP) L.Y[tid * nr + j] = y;
                if (tid < b) a.rhs[sd.oRhs + ((long long)gs * b + tid) * nr + j] = y;
            }
        }
        __syncthreads();
        double row[BP];
#pragma unroll
        for (int c = 0; c < BP; ++c) {
            double v = 0.0;
            if (c < b) {
                if (isE && hasE) v = stE[er * P + c];
                else if (isG) v = stG[gq * P + c];
                else if (isF) v = stF[fr * P + c];
            }
            row[c] = v;
        }
        if (isE || isG || isF) {
            for (int j = 0; j < nr; ++j) {
                const double s = dot_col<BP>(row, L.Y + j, nr);
                if (isE) L.RP[tid * nr + j] = s;
                else L.RP[tid * nr + j] -= s;
            }
        }
        __syncthreads();
        if (hasE && isE) {
            if (i + 1 < len) {
                const int ns = ch.stage(i + 1);
                const double *add = RED ? ch.scr(i + 2) + scr_dy(b, ng, nr) : nullptr;
                for (int j = 0; j < nr; ++j) {
                    double v = a.rhs[sd.oRhs + ((long long)ns * b + er) * nr + j];
                    if (add) v += add[er * nr + j];
                    L.W[er * nr + j] = v - L.RP[tid * nr + j];
                }
            } else {
                double *sc = a.F + sd.oScr + (long long)(k - 1) * sd.scrStride;
                for (int j = 0; j < nr; ++j) sc[scr_dy(b, ng, nr) + er * nr + j] = -L.RP[tid * nr + j];
            }
        }
        __syncthreads();
    }
    if (isF)
        for (int j = 0; j < nr; ++j) a.rhs[sd.oRhs + ((long long)sep * b + fr) * nr + j] = L.RP[tid * nr + j];
    if (!RED && isG) {
        double *sc = a.F + sd.oScr + (long long)(k - 1) * sd.scrStride;
        for (int j = 0; j < nr; ++j) sc[scr_yg(b, ng, nr) + gq * nr + j] = L.RP[tid * nr + j];
    }
    __syncthreads();
}

// Backward substitution of one chain (Algorithm 3, Eqs. 11, 12).  All threads
// stage each stage's blocks (hat D, coupling block, hat G, fill block) and its y
// rows into LDS with coalesced loads; wave 0 computes, lane c owning column c.
// The current solution (x, or lambda in the adjoint) is read from and written to
// rhs in place.  With ADJ the gradient blocks of the stages visited are written.
template <int BP, bool ADJ, bool RED, int NTT = K<BP>::NT>
__device__ __forceinline__ void sweep_backward(const Args &a, const SysDesc &sd, int k, const Lds &L)
{
    constexpr int NT = NTT, P = K<BP>::PITCH;
    const Chain<BP, RED> ch{a, sd, k};
    const int tid = threadIdx.x;
    const int b = sd.b, ng = sd.ng, nr = a.nr, N = sd.N;
    const long long b2 = (long long)b * b;
    const double *F = a.F;
    const bool hasF = !RED && k > 1;
    const int len = ch.length();
    const int sep = hasF ? sep_of(sd, k) : -1;
    const int c = tid;
    const bool cv = c < b;
    double *X = a.rhs + sd.oRhs;
    const double *xp = ADJ ? a.xp + sd.oRhs : nullptr;
    double *stD = L.P, *stE = L.P + BP * P, *stG = L.P + 2 * BP * P, *stF = L.A;

    // solution (and primal) at g, at the separator, and at the stage after the chain
    for (int e = tid; e < ng * nr; e += NT) {
        L.XG[e] = X[(long long)N * b * nr + e];
        if (ADJ) L.PG[e] = xp[(long long)N * b * nr + e];
    }
    if (hasF)
        for (int e = tid; e < b * nr; e += NT) {
            L.XS[e] = X[(long long)sep * b * nr + e];
            if (ADJ) L.PS[e] = xp[(long long)sep * b * nr + e];
        }
    if (!RED && ch.has_next(len - 1)) {
        const int nxt = ch.stage(len - 1) + 1;
        for (int e = tid; e < b * nr; e += NT) {
            L.XN[e] = X[(long long)nxt * b * nr + e];
            if (ADJ) L.PN[e] = xp[(long long)nxt * b * nr + e];
        }
    }

    for (int i = len - 1; i >= 0; --i) {
        const int gs = ch.stage(i);
        const bool hasE = ch.has_next(i);
        __syncthreads();   // previous stage done with the staging area and XC
        load_block<NT, BP * BP>(stD, P, F + sd.oLd + gs * b2, nullptr, b, b);
        if (hasE) load_block<NT, BP * BP>(stE, P, RED ? F + sd.oH + i * b2 : F + sd.oLc + gs * b2, nullptr, b, b);
        if (ng) load_block<NT, NGM * BP>(stG, P, F + sd.oLb + (long long)gs * ng * b, nullptr, ng, b);
        if (hasF) {
            const double *src = (i == 0) ? F + sd.oLc + sep * b2
                                         : F + sd.oFill + ((long long)(k - 2) * (sd.Nk - 1) + (i - 1)) * b2;
            load_block<NT, BP * BP>(stF, P, src, nullptr, b, b);
        }
        load_rhs<NT, BP * 8>(L.XC, X + (long long)gs * b * nr, nullptr, b * nr);   // y of this stage
        if (ADJ) load_rhs<NT, BP * 8>(L.PC, xp + (long long)gs * b * nr, nullptr, b * nr);
        __syncthreads();
        if (tid < 64) {
            double dcol[BP];
#pragma unroll
            for (int l = 0; l < BP; ++l) dcol[l] = (cv && l < b) ? stD[l * P + c] : (l == c ? 1.0 : 0.0);
            const double dinv = cv ? 1.0 / stD[c * P + c] : 1.0;
            for (int j = 0; j < nr; ++j) {
                double acc = cv ? L.XC[c * nr + j] : 0.0;
                if (hasE)
                    for (int r = 0; r < b; ++r) acc = fma(-(cv ? stE[r * P + c] : 0.0), L.XN[r * nr + j], acc);
                for (int q = 0; q < ng; ++q) acc = fma(-(cv ? stG[q * P + c] : 0.0), L.XG[q * nr + j], acc);
                if (hasF)
                    for (int r = 0; r < b; ++r) acc = fma(-(cv ? stF[r * P + c] : 0.0), L.XS[r * nr + j], acc);
                const double xv = back_subst<BP>(dcol, acc, dinv);
                wave_sync();
                if (cv) {
                    X[((long long)gs * b + c) * nr + j] = xv;
                    L.XC[c * nr + j] = xv;
                }
                wave_sync();
            }
            if (ADJ && cv) {
                // dD_gs = -sym(lambda x^T); dB_gs = -(lambda_g x^T + x_g lambda^T); dC_gs (stage couplings only)
                double *dD = a.dD + sd.oD + gs * b2;
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
                if (!RED && hasE) {
                    double *dC = a.dC + sd.oC + gs * b2;
                    for (int r = 0; r < b; ++r) {
                        double s = 0.0;
                        for (int j = 0; j < nr; ++j)
                            s += L.XN[r * nr + j] * L.PC[c * nr + j] + L.PN[r * nr + j] * L.XC[c * nr + j];
                        dC[r * b + c] = -s;
                    }
                }
                if (hasF && i == 0) {
                    // C_{sep_k} = Psi_{first(k), sep_k}: rows of the first stage, columns of the separator
                    double *dC = a.dC + sd.oC + sep * b2;
                    for (int r = 0; r < b; ++r) {
                        double s = 0.0;
                        for (int j = 0; j < nr; ++j)
                            s += L.XC[r * nr + j] * L.PS[c * nr + j] + L.PC[r * nr + j] * L.XS[c * nr + j];
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
            wave_sync();
        }
    }
    __syncthreads();
}

}  // namespace kkt_dev
