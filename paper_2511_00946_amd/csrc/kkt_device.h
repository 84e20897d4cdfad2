// Device-side building blocks of the segmented block Cholesky (gfx950, FP64).
//
// One workgroup processes one work item: a segment of one system (Algorithm 1,
// parallel phase; Algorithm 2 parallel phase; Algorithm 3 parallel phase) or the
// reduced separator/arrow chain of one system plus its corner block (Algorithm 1
// sequential phase, Eq. 7; Algorithms 2-3 sequential phases).
//
// Lane roles inside a workgroup of K<BP>::NT threads (BP = padded block size):
//   tid <  BP                   "D lane"  r = tid: row r of the working diagonal block
//   BP <= tid < 2 BP            "E lane"  r = tid - BP: row r of the coupling block to
//                               the next pivot (hat E, hat F_k, or hat H_k on the
//                               reduced chain)
//   2 BP <= tid < 2 BP + 16     "G lane"  q = tid - 2 BP: row q of the arrow block
//   2 BP + 16 <= tid < 3 BP + 16 "F lane" r = tid - 2 BP - 16: row r of the separator
//                               fill block hat B^T_{ik} (segments k >= 2 only)
// Every lane holds its one row in registers.  A stage step is one right-looking
// elimination of the tall matrix [D_w ; E ; G ; F] (b + b + ng + b rows, b
// columns): it produces hat D (potrf) and the panel hat P = P D^{-T} (the trsm of
// Eq. 5 / Algorithm 1) in one sweep over the b columns, with the right-hand side
// of the diagonal rows carried along (forward substitution, Algorithm 2).  The
// Gram matrix of the panel rows then gives every update of Eq. (6)/(8): the next
// diagonal block, the next arrow and fill rows, and the separator accumulators
// hat A_k, hat Q_k, hat R_k.
//
// Padding: a block of size b < BP is embedded in BP x BP with identity on the
// padded diagonal and zeros elsewhere; this is exact (the padded part factors to
// the identity and never mixes with the real part).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kkt_dev {

constexpr int NGM = 16;          // maximum global block size
constexpr int MAX_NRHS_DEV = 8;  // maximum right-hand sides per call

struct SysDesc {
    int N, b, ng, p, N1, Nk, cls, pad;
    long long oD, oC, oB, oCorner, oRhs;          // input pools (doubles)
    long long oLd, oLc, oLb, oLg, oFill, oH;      // factor region (doubles)
    long long oScr, scrStride;                    // per-segment scratch (doubles)
};

// Per-segment scratch (segment k at oScr + (k-1) * scrStride), written by the
// parallel phase of segment k and read by the reduced phase:
//   dA  [b, b]      hat F_k hat F_k^T       (subtracted from tilde A_{k+1}, Eq. 8c)
//   dQ  [ng, b]     hat G_{N_k k} hat F_k^T (subtracted from tilde Q_{k+1}, Eq. 8c)
//   dy  [b, nrhs]   -hat F_k hat y_{N_k k}  (added to tilde y_{k+1}, Eq. 9d)
//   Rk  [ng, ng]    tilde R_k = -sum hat G hat G^T (Eq. 8b)
//   ygk [ng, nrhs]  tilde y_{g,k} = -sum hat G hat y (Eq. 9c)
__host__ __device__ __forceinline__ long long scr_dA(int b, int ng, int nr) { return 0; }
__host__ __device__ __forceinline__ long long scr_dQ(int b, int ng, int nr) { return (long long)b * b; }
__host__ __device__ __forceinline__ long long scr_dy(int b, int ng, int nr) { return (long long)b * b + (long long)ng * b; }
__host__ __device__ __forceinline__ long long scr_Rk(int b, int ng, int nr) { return scr_dy(b, ng, nr) + (long long)b * nr; }
__host__ __device__ __forceinline__ long long scr_yg(int b, int ng, int nr) { return scr_Rk(b, ng, nr) + (long long)ng * ng; }
__host__ __device__ __forceinline__ long long scr_stride(int b, int ng, int nr) { return scr_yg(b, ng, nr) + (long long)ng * nr; }

enum Mode { M_FACTOR = 0, M_FACTOR_SOLVE = 1, M_SOLVE = 2, M_ADJOINT = 3 };

struct Args {
    const double *D, *C, *B, *corner;
    double *rhs;
    const double *xp;                   // adjoint: primal solution x
    double *dD, *dC, *dB, *dcorner;
    double *F;                          // factor region base
    const SysDesc *sys;
    const int2 *items;
    int n_items;
    int2 *s3_slot;
    int *s3_ready;
    int n_s3;
    int *ctr;                           // [0] item head, [1] s3 reserve, [2] s3 head, [3] error
    int *arrive;                        // per system
    int *failidx;                       // per system: first failing stage (1-based), INT_MAX = none
    int *status;                        // per system: final info of the last factorization
    int *info;                          // caller's info (factor modes), may be null
    const int *red;                     // systems of a segmented dense class (sequential phase)
    int n_red;
    int nr;
    int spin_limit;
};

template <int BP>
struct K {
    static constexpr int NROWS = 3 * BP + NGM;
    static constexpr int NT = ((NROWS + 63) / 64) * 64;
    static constexpr int PITCH = BP + 1;
    static constexpr int E0 = BP;
    static constexpr int G0 = 2 * BP;
    static constexpr int F0 = 2 * BP + NGM;
    static constexpr int BPX = BP > NGM ? BP : NGM;
};

struct LdsOff {
    int col, P, A, Q, R, W, Y, RP, XN, XS, XC, XG, PN, PS, PC, PG, misc, total;
};

// LDS layout in doubles for block class BP and nrhs right-hand sides.
__host__ __device__ __forceinline__ LdsOff lds_offsets(int BP, int nr)
{
    LdsOff o;
    const int BPX = BP > NGM ? BP : NGM;
    const int PITCH = BP + 1 > NGM + 1 ? BP + 1 : NGM + 1;
    const int NROWS = 3 * BP + NGM;
    int t = 0;
    o.col = t; t += 2 * BPX;
    o.P = t;   t += NROWS * PITCH;      // panel rows / staging of the next stage's blocks
    o.A = t;   t += BP * PITCH;         // hat A_k accumulator / fill staging in the solve
    o.Q = t;   t += NGM * PITCH;        // hat Q_k accumulator
    o.R = t;   t += NGM * NGM;          // hat R_k accumulator
    o.W = t;   t += BPX * nr;           // rhs of the diagonal rows
    o.Y = t;   t += BPX * nr;           // y of the current stage
    o.RP = t;  t += NROWS * nr;         // rhs of the panel rows
    o.XN = t;  t += BPX * nr;           // backward: solution at the next stage
    o.XS = t;  t += BPX * nr;           //           solution at the separator
    o.XC = t;  t += BPX * nr;           //           solution at the current stage
    o.XG = t;  t += NGM * nr;           //           solution at g
    o.PN = t;  t += BPX * nr;           // adjoint: primal x at the next stage
    o.PS = t;  t += BPX * nr;           //          primal x at the separator
    o.PC = t;  t += BPX * nr;           //          primal x at the current stage
    o.PG = t;  t += NGM * nr;           //          primal x at g
    o.misc = t; t += 8;
    o.total = t;
    return o;
}

struct Lds {
    double *col, *P, *A, *Q, *R, *W, *Y, *RP, *XN, *XS, *XC, *XG, *PN, *PS, *PC, *PG;
    int *misc;
};

__device__ __forceinline__ Lds make_lds(double *base, int BP, int nr)
{
    const LdsOff o = lds_offsets(BP, nr);
    Lds L;
    L.col = base + o.col; L.P = base + o.P; L.A = base + o.A; L.Q = base + o.Q; L.R = base + o.R;
    L.W = base + o.W; L.Y = base + o.Y; L.RP = base + o.RP; L.XN = base + o.XN; L.XS = base + o.XS;
    L.XC = base + o.XC; L.XG = base + o.XG; L.PN = base + o.PN; L.PS = base + o.PS; L.PC = base + o.PC;
    L.PG = base + o.PG; L.misc = reinterpret_cast<int *>(base + o.misc);
    return L;
}

// ---------------------------------------------------------------- small helpers
__device__ __forceinline__ int seg_first(const SysDesc &s, int k) { return k == 1 ? 0 : s.N1 + (k - 2) * (s.Nk + 1) + 1; }
__device__ __forceinline__ int seg_len(const SysDesc &s, int k) { return k == 1 ? s.N1 : s.Nk; }
__device__ __forceinline__ int sep_of(const SysDesc &s, int k) { return s.N1 + (k - 2) * (s.Nk + 1); }  // k >= 2

__device__ __forceinline__ double readlane_d(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
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

// Keeps the compiler from moving LDS accesses across this point; LDS operations of
// one wavefront execute in order, so lanes of the same wave then see each other's writes.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Wait for every outstanding vector memory operation of the wave.  Loads and
// stores share one counter here and may complete out of order with respect to
// each other, so a wait for a load issued while stores are pending waits for
// all of them; draining at a point where the loads are known to have arrived
// keeps later uses of their registers free of waits.
__device__ __forceinline__ void vm_drain()
{
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), expcnt(7), lgkmcnt(15)
}

// Opaque register use: values computed before this point cannot be sunk below it.
template <int BP>
__device__ __forceinline__ void pin_row(double (&v)[BP])
{
#pragma unroll
    for (int c = 0; c < BP; ++c) asm volatile("" : "+v"(v[c]));
}

template <int BP>
__device__ __forceinline__ double dot_row(const double (&v)[BP], const double *__restrict__ s)
{
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int c = 0; c < BP; c += 2) {
        a0 = fma(v[c], s[c], a0);
        if (c + 1 < BP) a1 = fma(v[c + 1], s[c + 1], a1);
    }
    return a0 + a1;
}

template <int BP>
__device__ __forceinline__ double dot_col(const double (&v)[BP], const double *__restrict__ s, int stride)
{
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int c = 0; c < BP; c += 2) {
        a0 = fma(v[c], s[c * stride], a0);
        if (c + 1 < BP) a1 = fma(v[c + 1], s[(c + 1) * stride], a1);
    }
    return a0 + a1;
}

// Row of a flat index e of a row-major block of width w (e < 2^16, w <= 64):
// (e + 0.5) / w in float is never within 0.5 / w of an integer, and its rounding
// error is far below that, so truncation gives floor(e / w) exactly.
__device__ __forceinline__ int row_of(int e, float invw) { return (int)(((float)e + 0.5f) * invw); }

// Copy a rows x cols row-major global block (rows * cols <= MAXE) into LDS with a
// row pitch, optionally subtracting a second block: every load is issued before
// the first LDS store, so the block costs one memory latency, not one per element.
template <int NT, int MAXE>
__device__ __forceinline__ void load_block(double *dst, int pitch, const double *src, const double *sub, int rows,
                                           int cols)
{
    constexpr int M = (MAXE + NT - 1) / NT;
    const int n = rows * cols;
    double v[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int e = threadIdx.x + m * NT;
        v[m] = 0.0;
        if (e < n) {
            v[m] = src[e];
            if (sub) v[m] -= sub[e];
        }
    }
    const float invc = 1.0f / (float)cols;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int e = threadIdx.x + m * NT;
        if (e < n) {
            const int r = row_of(e, invc);
            dst[r * pitch + (e - r * cols)] = v[m];
        }
    }
}

// rhs rows (n <= MAXE contiguous doubles) into LDS, optionally plus a second block.
template <int NT, int MAXE>
__device__ __forceinline__ void load_rhs(double *dst, const double *src, const double *add, int n)
{
    constexpr int M = (MAXE + NT - 1) / NT;
    double v[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int e = threadIdx.x + m * NT;
        v[m] = 0.0;
        if (e < n) {
            v[m] = src[e];
            if (add) v[m] += add[e];
        }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int e = threadIdx.x + m * NT;
        if (e < n) dst[e] = v[m];
    }
}

// Coalesced store of rows [0, rows) x [0, cols) of an LDS block with a row pitch
// to a row-major global block (rows * cols <= MAXE).
// Every thread reads all its elements first (indices past the block are clamped
// to element 0, so the reads need no branch) and only then stores: the block
// costs one LDS round trip, not one per element.
template <int NT, int MAXE>
__device__ __forceinline__ void store_block(double *dst, const double *lds, int pitch, int rows, int cols)
{
    constexpr int M = (MAXE + NT - 1) / NT;
    const int n = rows * cols;
    const float invc = 1.0f / (float)cols;
    double v[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int e = threadIdx.x + m * NT;
        const int ec = e < n ? e : 0;
        const int r = row_of(ec, invc);
        v[m] = lds[r * pitch + (ec - r * cols)];
    }
    pin_row<M>(v);
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int e = threadIdx.x + m * NT;
        if (e < n) dst[e] = v[m];
    }
}

// A word of zeros in device memory that nothing writes.
__device__ double zero_word[2];

// src[i] if ok, else 0, with neither a branch nor a select after the load: the
// address is chosen instead (the zero word when !ok), so the value can stay in
// flight until it is used.  src is not dereferenced when !ok.
__device__ __forceinline__ double ld_or_zero(const double *src, int i, bool ok)
{
    return *(ok ? src + i : zero_word);
}

// ---------------------------------------------------------------- elimination
// Right-looking column elimination of the tall matrix held one row per lane:
// D lanes (tid < BP) hold the working diagonal rows (lower part meaningful), all
// other lanes a panel row (zero rows are harmless).  After the call D lanes hold
// rows of hat D (lower) and panel lanes rows of hat P = P hat D^{-T}.  With fwd,
// W (rows of the diagonal, pitch nr) is eliminated along and Y = hat D^{-1} W.
// One barrier per column (the column buffer is double-buffered).  Returns true
// if a pivot was not positive and finite.
template <int BP>
__device__ __forceinline__ bool eliminate(double (&row)[BP], const Lds &L, int nr, bool fwd)
{
    const int tid = threadIdx.x;
    bool bad = false;
#pragma unroll
    for (int c = 0; c < BP; ++c) {
        double *buf = L.col + (c & 1) * BP;
        if (tid < BP && tid >= c) buf[tid] = row[c];
        __syncthreads();
        const double dcc = buf[c];
        bad |= !(dcc > 0.0) || !isfinite(dcc);
        double d, inv;
        sqrt_rsqrt(dcc, d, inv);
        const bool act = tid > c;                 // diagonal rows below the pivot, every panel row
        const double v = row[c] * inv;            // hat D[tid][c] or hat P[row][c]
        if (tid == c) row[c] = d;
        else if (act) row[c] = v;
        const double f = act ? v * inv : 0.0;
#pragma unroll
        for (int l = c + 1; l < BP; ++l) row[l] = fma(-f, buf[l], row[l]);
        if (fwd) {
            if (tid == c) {
                for (int j = 0; j < nr; ++j) L.Y[c * nr + j] = L.W[c * nr + j] * inv;
            } else if (act && tid < BP) {
                for (int j = 0; j < nr; ++j) L.W[tid * nr + j] = fma(-f, L.W[c * nr + j], L.W[tid * nr + j]);
            }
        }
        // materialise this column's updates here: without it the compiler sinks them
        // past the next barriers and keeps every loaded column value live across steps
        pin_row<BP>(row);
    }
    __syncthreads();
    return bad;
}

// Lane c of wave 0 holds acc = (rhs)[c] and dcol[l] = T[l][c] of a lower
// triangular T with dinv = 1 / T[c][c]; returns x[c] of T^T x = rhs.
template <int BP>
__device__ __forceinline__ double back_subst(const double (&dcol)[BP], double acc, double dinv)
{
    const int lane = threadIdx.x;
    double xv = 0.0;
#pragma unroll
    for (int c2 = BP - 1; c2 >= 0; --c2) {
        const double x2 = readlane_d(acc * dinv, c2);
        if (lane == c2) xv = x2;
        acc = fma(-dcol[c2], x2, acc);
    }
    return xv;
}

// Lane r of wave 0 holds acc = rhs[r] and drow[c] = T[r][c] of a lower triangular
// T with dinv = 1 / T[r][r]; returns y[r] of T y = rhs.
template <int BP>
__device__ __forceinline__ double fwd_subst(const double (&drow)[BP], double acc, double dinv)
{
    const int lane = threadIdx.x;
    double yv = 0.0;
#pragma unroll
    for (int c = 0; c < BP; ++c) {
        const double yc = readlane_d(acc * dinv, c);
        if (lane == c) yv = yc;
        acc = fma(-drow[c], yc, acc);
    }
    return yv;
}

}  // namespace kkt_dev
