// Device-side building blocks shared by the stage sweeps of the segmented block
// Cholesky (gfx950, FP64): system descriptors, the per-segment scratch layout,
// kernel arguments, and small load / store / broadcast helpers.
//
// Padding: a block of size b < BP is embedded in BP x BP with identity on the
// padded diagonal and zeros elsewhere; this is exact (the padded part factors to
// the identity and never mixes with the real part).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <climits>
#include <type_traits>

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
    const int2 *items;                  // phase-1 work list of the launch class: (system, segment)
    int n_items;
    const int *red;                     // segmented systems of the class (phase 2)
    int n_red;
    const int2 *s3;                     // segments of the segmented systems (phase 3)
    int n_s3;
    int *ctr;                           // queue heads [0] phase 1, [1] phase 2, [2] phase 3
    const int *abort;                   // nonzero: the workspace does not belong to this plan
    int *failidx;                       // per system: first failing stage (1-based), INT_MAX = none
    int *status;                        // per system: final info of the last factorization
    int *info;                          // caller's info (factor modes), may be null
    int nr;
};

__device__ __forceinline__ int load_status(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Next entry of a work list: thread 0 takes it from the queue counter (or, when
// the call was refused on the device, a value past every list), every thread of
// the workgroup gets it through LDS.
__device__ __forceinline__ int next_work(int *ctr, const int *abort, int *misc)
{
    if (threadIdx.x == 0) misc[0] = (*abort != 0) ? INT_MAX : atomicAdd(ctr, 1);
    __syncthreads();
    const int it = misc[0];
    __syncthreads();
    return it;
}

struct LdsOff {
    int col, P, A, Q, R, W, Y, RP, XN, XS, XC, XG, PN, PS, PC, PG, misc, total;
};

struct Lds {
    double *col, *P, *A, *Q, *R, *W, *Y, *RP, *XN, *XS, *XC, *XG, *PN, *PS, *PC, *PG;
    int *misc;
};

// ---------------------------------------------------------------- small helpers
__device__ __forceinline__ int seg_first(const SysDesc &s, int k) { return k == 1 ? 0 : s.N1 + (k - 2) * (s.Nk + 1) + 1; }
__device__ __forceinline__ int seg_len(const SysDesc &s, int k) { return k == 1 ? s.N1 : s.Nk; }
__device__ __forceinline__ int sep_of(const SysDesc &s, int k) { return s.N1 + (k - 2) * (s.Nk + 1); }  // k >= 2

// FP64 matrix-core product D = A B + C on 16 x 16 x 4 tiles (v_mfma_f64_16x16x4f64):
// A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k, D[4 v + lane / 16][lane % 16]
// in element v of lane `lane`.
typedef double dx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dx4 mfma4(double a, double b, dx4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Range-checked access through a buffer resource (raw, no stride): an element
// whose byte offset lies past the resource's byte count reads as zero and a store
// there is dropped; the hardware checks every access.  Dword 3 holds the 32-bit
// data format the gfx9 family expects for untyped buffer instructions.
typedef __amdgpu_buffer_rsrc_t brsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ brsrc_t brsrc(const double *p, long long n)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, (int)(n * 8), 0x00020000);
}

__device__ __forceinline__ double bload(brsrc_t r, int e)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, e * 8, 0, 0));
}

__device__ __forceinline__ void bstore(brsrc_t r, int e, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, e * 8, 0, 0);
}

__device__ __forceinline__ double readlane_d(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// f(std::integral_constant<int, I>) for I = I0 .. I1 - 1 in order: the index is a
// constant expression inside f, so arrays indexed by it stay in registers whatever
// the size of the body.
template <int I0, int I1, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I0 < I1) {
        f(std::integral_constant<int, I0>{});
        static_for<I0 + 1, I1>(f);
    }
}

// sqrt(x) and 1/sqrt(x) from the hardware reciprocal square root refined by two
// Goldschmidt iterations (g -> sqrt(x), h -> 1/(2 sqrt(x))); for x > 0 finite the
// result is within a few ulp of the correctly rounded values.  The iteration is
// split into its dependent stages so that a caller can place independent work
// between them; sqrt_rsqrt runs them back to back.
struct RsqChain {
    double x, g, h, r;
};
constexpr int RSQ_STAGES = 7;
__device__ __forceinline__ void rsq_stage(int s, RsqChain &q)
{
    switch (s) {
    case 0: q.h = __builtin_amdgcn_rsq(q.x); break;
    case 1: q.g = q.x * q.h; q.h = 0.5 * q.h; break;
    case 2: q.r = fma(-q.g, q.h, 0.5); break;
    case 3: q.g = fma(q.g, q.r, q.g); q.h = fma(q.h, q.r, q.h); break;
    case 4: q.r = fma(-q.g, q.h, 0.5); break;
    case 5: q.g = fma(q.g, q.r, q.g); q.h = fma(q.h, q.r, q.h); break;
    default: q.h = q.h + q.h; break;
    }
}
__device__ __forceinline__ void sqrt_rsqrt(double x, double &d, double &inv)
{
    RsqChain q{x, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < RSQ_STAGES; ++s) rsq_stage(s, q);
    d = q.g;
    inv = q.h;
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
static __device__ double zero_word[2];

// src[i] if ok, else 0, with neither a branch nor a select after the load: the
// address is chosen instead (the zero word when !ok), so the value can stay in
// flight until it is used.  src is not dereferenced when !ok.
__device__ __forceinline__ double ld_or_zero(const double *src, int i, bool ok)
{
    return *(ok ? src + i : zero_word);
}

// A block of n doubles in global memory addressed through a buffer resource with
// 32-bit byte offsets: a load past the end of the block returns zero and a store
// past it is dropped, so an edge predicate costs one offset select (or nothing,
// when the offset runs past the end by itself) instead of a branch or a 64-bit
// address select.  n = 0 makes every access fall outside.  p and n must be the
// same in every lane (the resource is a scalar operand; they are read from the
// first active lane).
constexpr int GB_OUT = 0x40000000;   // an offset past the end of every block
typedef unsigned int gb_u32x2 __attribute__((ext_vector_type(2)));
struct GBlock {
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ static double *uniform_ptr(const double *p)
    {
        const unsigned long long u = (unsigned long long)p;
        const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
        const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
        return (double *)(((unsigned long long)hi << 32) | lo);
    }
    __device__ __forceinline__ GBlock(const double *p, long long n)
        : r(__builtin_amdgcn_make_buffer_rsrc(uniform_ptr(p), (short)0,
                                              __builtin_amdgcn_readfirstlane((int)(n * 8)), 0x00020000))
    {
    }
    __device__ __forceinline__ double ld(int off) const
    {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    }
    __device__ __forceinline__ void st(int off, double v) const
    {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(gb_u32x2, v), r, off, 0, 0);
    }
};

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
