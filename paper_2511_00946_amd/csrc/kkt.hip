// MI355X (gfx950) segmented block Cholesky for block-tridiagonal-arrow KKT
// systems (arXiv 2511.00946): persistent kernels, host plan and the C ABI of
// include/kkt.h.
//
// Scheduling.  A plan splits every system into p segments (Eq. 13 or given) and
// lists one work item per (system, segment), longest first (LPT).  Systems are
// grouped by padded block size ("class"); each class gets one persistent launch
// whose workgroups pull items from an atomic queue:
//   phase 1  factor (+ forward) sweep of the segment               (Alg. 1/2 parallel)
//   arrival  the last segment of a system to finish runs phase 2:
//   phase 2  reduced chain + corner: factor, forward, backward      (Alg. 1/2/3 sequential)
//            then publishes the system's other segments for phase 3
//   phase 3  backward sweep of the segment (+ adjoint gradients)    (Alg. 3 parallel)
// Phase-3 items are taken only once the phase-1 queue is empty, so every item a
// worker waits for is already held by a running workgroup (no deadlock); the
// wait is bounded by a spin limit that raises an error flag instead of hanging.
// p = 1 systems run all three phases in one item with no synchronisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <unordered_set>
#include <vector>

#include "kkt.h"
#include "kkt_device.h"
#include "kkt_sweeps.h"
#include "kkt_dense.h"

using namespace kkt_dev;

namespace {

// ------------------------------------------------------------------ corner
template <int BP>
__device__ __forceinline__ const double *seg_scr(const Args &a, const SysDesc &sd, int k)
{
    return a.F + sd.oScr + (long long)(k - 1) * sd.scrStride;
}

// tilde R = sym(corner) + sum_k tilde R_k (+ reduced-chain part), then
// hat R = chol(tilde R) (Algorithm 1, last two lines; Eq. 8d).  With FWD also
// hat y_g = hat R^{-1} tilde y_g and x_g = hat R^{-T} hat y_g (Algorithms 2, 3).
template <int BP, bool FWD, int NTT = K<BP>::NT>
__device__ __forceinline__ bool corner_factor(const Args &a, const SysDesc &sd, const Lds &L, bool red)
{
    constexpr int NT = NTT, G0 = K<BP>::G0, PC = NGM + 1;
    static_assert(K<BP>::NROWS * (BP + 1) >= NGM * PC || BP >= NGM, "corner staging must fit");
    const int ng = sd.ng, nr = a.nr, tid = threadIdx.x, b = sd.b, N = sd.N;
    if (ng == 0) return false;
    double *St = L.P;
    const double *cor = a.corner + sd.oCorner;
    for (int e = tid; e < NGM * nr; e += NT) L.W[e] = 0.0;
    __syncthreads();
    for (int e = tid; e < ng * ng; e += NT) {
        const int q = e / ng, c = e - q * ng;
        double v = 0.5 * (cor[e] + cor[c * ng + q]);
        for (int k = 1; k <= sd.p; ++k) v += seg_scr<BP>(a, sd, k)[scr_Rk(b, ng, nr) + e];
        if (red) v += L.R[q * NGM + c];
        St[q * PC + c] = v;
    }
    if (FWD) {
        const double *rg = a.rhs + sd.oRhs + (long long)N * b * nr;
        for (int e = tid; e < ng * nr; e += NT) {
            const int q = e / nr, j = e - q * nr;
            double v = rg[e];
            for (int k = 1; k <= sd.p; ++k) v += seg_scr<BP>(a, sd, k)[scr_yg(b, ng, nr) + e];
            if (red) v += L.RP[(G0 + q) * nr + j];
            L.W[q * nr + j] = v;
        }
    }
    __syncthreads();
    double xr[NGM];
#pragma unroll
    for (int c = 0; c < NGM; ++c) {
        xr[c] = (tid < NGM) ? ((tid < ng && c < ng) ? St[tid * PC + c] : (tid == c ? 1.0 : 0.0)) : 0.0;
    }
    const bool bad = eliminate<NGM>(xr, L, nr, FWD);
    double *Lg = a.F + sd.oLg;
    if (tid < ng) {
#pragma unroll
        for (int c = 0; c < NGM; ++c)
            if (c < ng) Lg[tid * ng + c] = (c <= tid) ? xr[c] : 0.0;
    }
    if (tid < NGM) {
#pragma unroll
        for (int c = 0; c < NGM; ++c) St[tid * PC + c] = (c <= tid) ? xr[c] : 0.0;
    }
    __syncthreads();
    if (FWD && tid < 64) {
        double dcol[NGM];
#pragma unroll
        for (int l = 0; l < NGM; ++l) dcol[l] = (tid < NGM) ? St[l * PC + tid] : (l == tid ? 1.0 : 0.0);
        const double dinv = (tid < NGM) ? 1.0 / St[tid * PC + tid] : 1.0;
        double *xg = a.rhs + sd.oRhs + (long long)N * b * nr;
        for (int j = 0; j < nr; ++j) {
            const double acc = (tid < NGM) ? L.Y[tid * nr + j] : 0.0;
            const double x = back_subst<NGM>(dcol, acc, dinv);
            if (tid < ng) xg[tid * nr + j] = x;
        }
    }
    __syncthreads();
    return bad;
}

// Corner solve with the factor in place: tilde y_g, hat y_g, x_g.
template <int BP, int NTT = K<BP>::NT>
__device__ __forceinline__ void corner_solve(const Args &a, const SysDesc &sd, const Lds &L, bool red)
{
    constexpr int NT = NTT, G0 = K<BP>::G0;
    const int ng = sd.ng, nr = a.nr, tid = threadIdx.x, b = sd.b, N = sd.N;
    if (ng == 0) return;
    double *rg = a.rhs + sd.oRhs + (long long)N * b * nr;
    for (int e = tid; e < ng * nr; e += NT) {
        const int q = e / nr, j = e - q * nr;
        double v = rg[e];
        for (int k = 1; k <= sd.p; ++k) v += seg_scr<BP>(a, sd, k)[scr_yg(b, ng, nr) + e];
        if (red) v += L.RP[(G0 + q) * nr + j];
        L.W[q * nr + j] = v;
    }
    __syncthreads();
    if (tid < 64) {
        const double *Lg = a.F + sd.oLg;
        double drow[NGM], dcol[NGM];
        const bool v = tid < ng;
#pragma unroll
        for (int c = 0; c < NGM; ++c) {
            drow[c] = (v && c < ng) ? (c <= tid ? Lg[tid * ng + c] : 0.0) : (tid == c ? 1.0 : 0.0);
            dcol[c] = (v && c < ng) ? (c >= tid ? Lg[c * ng + tid] : 0.0) : (tid == c ? 1.0 : 0.0);
        }
        const double dinv = v ? 1.0 / Lg[tid * ng + tid] : 1.0;
        for (int j = 0; j < nr; ++j) {
            const double w = v ? L.W[tid * nr + j] : 0.0;
            const double y = fwd_subst<NGM>(drow, w, dinv);
            const double x = back_subst<NGM>(dcol, y, dinv);
            if (v) rg[tid * nr + j] = x;
        }
    }
    __syncthreads();
}

// dcorner = -sym(lambda_g x_g^T) summed over the rhs columns.
template <int BP>
__device__ __forceinline__ void corner_grad(const Args &a, const SysDesc &sd, const Lds &L)
{
    const int ng = sd.ng, nr = a.nr, tid = threadIdx.x, b = sd.b, N = sd.N;
    if (ng == 0) return;
    const long long og = sd.oRhs + (long long)N * b * nr;
    if (tid < 64) {
        for (int e = tid; e < ng * nr; e += 64) { L.XG[e] = a.rhs[og + e]; L.PG[e] = a.xp[og + e]; }
        wave_sync();
        if (tid < ng) {
            double *dR = a.dcorner + sd.oCorner;
            for (int q = 0; q < ng; ++q) {
                double s = 0.0;
                for (int j = 0; j < nr; ++j)
                    s += L.XG[q * nr + j] * L.PG[tid * nr + j] + L.PG[q * nr + j] * L.XG[tid * nr + j];
                dR[q * ng + tid] = -0.5 * s;
            }
        }
    }
    __syncthreads();
}

__device__ __forceinline__ int load_status(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A failed system's solution is NaN (natural stage range [s0, s1), plus g if withg).
template <int NT>
__device__ __forceinline__ void fill_nan(const Args &a, const SysDesc &sd, int s0, int s1, bool withg)
{
    const int nr = a.nr, b = sd.b;
    const double qnan = __longlong_as_double(0x7ff8000000000000LL);
    double *X = a.rhs + sd.oRhs;
    for (long long e = (long long)s0 * b * nr + threadIdx.x; e < (long long)s1 * b * nr; e += NT) X[e] = qnan;
    if (withg)
        for (int e = threadIdx.x; e < sd.ng * nr; e += NT) X[(long long)sd.N * b * nr + e] = qnan;
}

// ------------------------------------------------------------------ phases
template <int BP, int MODE>
__device__ __forceinline__ void phase1(const Args &a, const SysDesc &sd, int s, int k, const Lds &L)
{
    int f = 0;
    if (MODE == M_FACTOR) f = sweep_factor<BP, false, false>(a, sd, k, L);
    else if (MODE == M_FACTOR_SOLVE) f = sweep_factor<BP, true, false>(a, sd, k, L);
    else sweep_forward<BP, false>(a, sd, k, L);
    if (f && threadIdx.x == 0) atomicMin(&a.failidx[s], f);
}

template <int BP, int MODE>
__device__ __forceinline__ void phase2(const Args &a, const SysDesc &sd, int s, const Lds &L)
{
    constexpr int NT = K<BP>::NT;
    const bool red = sd.p > 1;
    const int tid = threadIdx.x;
    if (MODE == M_FACTOR || MODE == M_FACTOR_SOLVE) {
        constexpr bool FWD = MODE == M_FACTOR_SOLVE;
        int rf = 0;
        if (red) rf = sweep_factor<BP, FWD, true>(a, sd, 0, L);
        const bool cf = corner_factor<BP, FWD>(a, sd, L, red);
        if (tid == 0) {
            const int segf = load_status(&a.failidx[s]);
            const int info = segf != INT_MAX ? segf : (rf ? rf : (cf ? sd.N + 1 : 0));
            a.status[s] = info;
            if (a.info) a.info[s] = info;
            L.misc[2] = info;
        }
        __syncthreads();
        if (FWD && red) sweep_backward<BP, false, true>(a, sd, 0, L);
    } else {
        if (tid == 0) L.misc[2] = load_status(&a.status[s]);
        if (red) sweep_forward<BP, true>(a, sd, 0, L);
        corner_solve<BP>(a, sd, L, red);
        if (MODE == M_ADJOINT) corner_grad<BP>(a, sd, L);
        if (red) sweep_backward<BP, MODE == M_ADJOINT, true>(a, sd, 0, L);
    }
    __syncthreads();
    if (MODE != M_FACTOR && L.misc[2] != 0) {
        // NaN the separators and g (segments do their own stages in phase 3)
        for (int k = 2; k <= sd.p; ++k) {
            const int sp = sep_of(sd, k);
            fill_nan<NT>(a, sd, sp, sp + 1, false);
        }
        fill_nan<NT>(a, sd, 0, 0, true);
    }
    __syncthreads();
}

template <int BP, int MODE>
__device__ __forceinline__ void phase3(const Args &a, const SysDesc &sd, int s, int k, const Lds &L)
{
    constexpr int NT = K<BP>::NT;
    sweep_backward<BP, MODE == M_ADJOINT, false>(a, sd, k, L);
    __syncthreads();
    if (threadIdx.x == 0) L.misc[3] = load_status(&a.status[s]);
    __syncthreads();
    if (L.misc[3] != 0) {
        const int f = seg_first(sd, k);
        fill_nan<NT>(a, sd, f, f + seg_len(sd, k), false);
    }
    __syncthreads();
}

// ------------------------------------------------------------------ kernels
template <int BP, int MODE>
__global__ void __launch_bounds__(K<BP>::NT) kkt_persistent(Args a)
{
    extern __shared__ double lds_raw[];
    const Lds L = make_lds(lds_raw, BP, a.nr);
    int *sh = L.misc;
    const int tid = threadIdx.x;

    for (;;) {
        if (tid == 0) sh[0] = atomicAdd(&a.ctr[0], 1);
        __syncthreads();
        const int it = sh[0];
        __syncthreads();
        if (it >= a.n_items) break;
        const int2 w = a.items[it];
        const SysDesc sd = a.sys[w.x];
        phase1<BP, MODE>(a, sd, w.x, w.y, L);
        if (sd.p == 1) {
            phase2<BP, MODE>(a, sd, w.x, L);
            if (MODE != M_FACTOR) phase3<BP, MODE>(a, sd, w.x, 1, L);
            continue;
        }
        __threadfence();
        __syncthreads();
        if (tid == 0) sh[1] = (atomicAdd(&a.arrive[w.x], 1) == sd.p - 1) ? 1 : 0;
        __syncthreads();
        const bool lastArr = sh[1] != 0;
        __syncthreads();
        if (!lastArr) continue;
        __threadfence();
        phase2<BP, MODE>(a, sd, w.x, L);
        if (MODE == M_FACTOR) continue;
        __threadfence();
        __syncthreads();
        if (tid == 0) {
            const int base = atomicAdd(&a.ctr[1], sd.p - 1);
            int m = 0;
            for (int kk = 1; kk <= sd.p; ++kk)
                if (kk != w.y) a.s3_slot[base + m++] = make_int2(w.x, kk);
            __threadfence();
            for (m = 0; m < sd.p - 1; ++m)
                __hip_atomic_store(&a.s3_ready[base + m], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        phase3<BP, MODE>(a, sd, w.x, w.y, L);
    }
    if (MODE == M_FACTOR || a.n_s3 == 0) return;
    for (;;) {
        if (tid == 0) {
            int j = atomicAdd(&a.ctr[2], 1);
            if (j < a.n_s3) {
                int spins = 0;
                while (__hip_atomic_load(&a.s3_ready[j], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                    __builtin_amdgcn_s_sleep(8);
                    if (++spins > a.spin_limit) {
                        atomicOr(&a.ctr[3], 1);
                        j = INT_MAX;
                        break;
                    }
                }
            }
            sh[0] = j;
        }
        __syncthreads();
        const int j = sh[0];
        __syncthreads();
        if (j >= a.n_s3) break;
        __threadfence();
        int2 w;
        w.x = __hip_atomic_load(&a.s3_slot[j].x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        w.y = __hip_atomic_load(&a.s3_slot[j].y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const SysDesc sd = a.sys[w.x];
        phase3<BP, MODE>(a, sd, w.x, w.y, L);
    }
}

// Whole (p = 1) systems of the 16-, 24- and 32-wide classes: one wave per
// system, dense stage sweeps (factor on the matrix cores, forward and backward
// substitution with the next stage's blocks in flight), then the corner
// (Algorithms 1-3 with p = 1).
template <int DB, int MODE>
__global__ void __launch_bounds__(64, DB == 16 ? 2 : 1) kkt_dense(Args a)
{
    extern __shared__ double lds_raw[];
    const Lds L = make_lds_dense(lds_raw, DB, a.nr);
    int *sh = L.misc;
    const int tid = threadIdx.x;
    constexpr bool FACT = MODE == M_FACTOR || MODE == M_FACTOR_SOLVE;
    for (;;) {
        if (tid == 0) sh[0] = atomicAdd(&a.ctr[0], 1);
        __syncthreads();
        const int it = sh[0];
        __syncthreads();
        if (it >= a.n_items) break;
        const int2 w = a.items[it];
        const SysDesc sd = a.sys[w.x];
        if (FACT) {
            constexpr bool FWD = MODE == M_FACTOR_SOLVE;
            const int f = dense_factor<DB, FWD>(a, sd, L);
            const bool cf = corner_factor<DB, FWD, 64>(a, sd, L, false);
            if (tid == 0) {
                const int info = f ? f : (cf ? sd.N + 1 : 0);
                a.status[w.x] = info;
                if (a.info) a.info[w.x] = info;
                sh[2] = info;
            }
        } else {
            dense_forward<DB>(a, sd, L);
            corner_solve<DB, 64>(a, sd, L, false);
            if (MODE == M_ADJOINT) corner_grad<DB>(a, sd, L);
            if (tid == 0) sh[2] = load_status(&a.status[w.x]);
        }
        __syncthreads();
    }
}

// Backward substitution (and with ADJ the adjoint gradients) of the whole systems
// of a dense class, after kkt_dense has run the factor or forward sweep and the
// corner of every one of them; a launch of its own, so that each of the two
// sweeps gets the registers it needs.  Items come from the second queue counter.
template <int DB, bool ADJ>
__global__ void __launch_bounds__(64, 2) kkt_dense_bwd(Args a)
{
    extern __shared__ double lds_raw[];
    const Lds L = make_lds_dense(lds_raw, DB, a.nr);
    int *sh = L.misc;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) sh[0] = atomicAdd(&a.ctr[1], 1);
        __syncthreads();
        const int it = sh[0];
        __syncthreads();
        if (it >= a.n_items) break;
        const int2 w = a.items[it];
        const SysDesc sd = a.sys[w.x];
        dense_backward<DB, ADJ>(a, sd, L);
        if (tid == 0) sh[2] = load_status(&a.status[w.x]);
        __syncthreads();
        if (sh[2] != 0) fill_nan<64>(a, sd, 0, sd.N, true);
        __syncthreads();
    }
}

// Segmented systems of the 16-, 24- and 32-wide classes, factor modes: (1) every
// segment's factor (+ forward) sweep, one wave per segment (Algorithm 1/2
// parallel phase); (2) kkt_reduced: each system's reduced chain and corner
// (sequential phase); (3) every segment's backward sweep (Algorithm 3 parallel
// phase).  Three launches on one stream: each launch boundary is the
// synchronisation between the phases.
template <int DB, bool FWD>
__global__ void __launch_bounds__(64, DB == 16 ? 2 : 1) kkt_dense_seg(Args a)
{
    extern __shared__ double lds_raw[];
    const Lds L = make_lds_dense(lds_raw, DB, a.nr, true);
    int *sh = L.misc;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) sh[0] = atomicAdd(&a.ctr[0], 1);
        __syncthreads();
        const int it = sh[0];
        __syncthreads();
        if (it >= a.n_items) break;
        const int2 w = a.items[it];
        const SysDesc sd = a.sys[w.x];
        const int f = dense_factor<DB, FWD, true>(a, sd, L, w.y);
        if (tid == 0 && f) atomicMin(&a.failidx[w.x], f);
        __syncthreads();
    }
}

template <int BP, int MODE>
__global__ void __launch_bounds__(K<BP>::NT) kkt_reduced(Args a)
{
    extern __shared__ double lds_raw[];
    const Lds L = make_lds(lds_raw, BP, a.nr);
    int *sh = L.misc;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) sh[0] = atomicAdd(&a.ctr[1], 1);
        __syncthreads();
        const int it = sh[0];
        __syncthreads();
        if (it >= a.n_red) break;
        const int s = a.red[it];
        const SysDesc sd = a.sys[s];
        phase2<BP, MODE>(a, sd, s, L);
    }
}

template <int DB>
__global__ void __launch_bounds__(64, DB == 16 ? 2 : 1) kkt_dense_seg_bwd(Args a)
{
    extern __shared__ double lds_raw[];
    const Lds L = make_lds_dense(lds_raw, DB, a.nr, true);
    int *sh = L.misc;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) sh[0] = atomicAdd(&a.ctr[2], 1);
        __syncthreads();
        const int it = sh[0];
        __syncthreads();
        if (it >= a.n_items) break;
        const int2 w = a.items[it];
        const SysDesc sd = a.sys[w.x];
        dense_backward<DB, false, true>(a, sd, L, w.y);
        if (tid == 0) sh[2] = load_status(&a.status[w.x]);
        __syncthreads();
        if (sh[2] != 0) {
            const int f0 = seg_first(sd, w.y);
            fill_nan<64>(a, sd, f0, f0 + seg_len(sd, w.y), false);
        }
        __syncthreads();
    }
}

__global__ void kkt_reset(int *ctr, int nctr, int *arrive, int *failidx, int S, int *ready, int nready,
                          int *info)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x, st = gridDim.x * blockDim.x;
    for (int i = t; i < nctr; i += st) ctr[i] = 0;
    for (int i = t; i < S; i += st) {
        arrive[i] = 0;
        if (failidx) failidx[i] = INT_MAX;
        if (info) info[i] = 0;
    }
    for (int i = t; i < nready; i += st) ready[i] = 0;
}

// ------------------------------------------------------------------ host plan
constexpr int NCLS = 4;
constexpr int CLS_BP[NCLS] = {8, 16, 24, 32};

int class_of(int b)
{
    for (int c = 0; c < NCLS; ++c)
        if (b <= CLS_BP[c]) return c;
    return -1;
}

typedef void (*kfun_t)(Args);

template <int BP>
kfun_t kernel_for(int mode)
{
    switch (mode) {
    case M_FACTOR: return kkt_persistent<BP, M_FACTOR>;
    case M_FACTOR_SOLVE: return kkt_persistent<BP, M_FACTOR_SOLVE>;
    case M_SOLVE: return kkt_persistent<BP, M_SOLVE>;
    default: return kkt_persistent<BP, M_ADJOINT>;
    }
}

template <int DB>
kfun_t dense_kernel_for(int mode)
{
    switch (mode) {
    case M_FACTOR: return kkt_dense<DB, M_FACTOR>;
    case M_FACTOR_SOLVE: return kkt_dense<DB, M_FACTOR_SOLVE>;
    case M_SOLVE: return kkt_dense<DB, M_SOLVE>;
    default: return kkt_dense<DB, M_ADJOINT>;
    }
}

kfun_t dense_kernel_for(int bp, int mode)
{
    return bp <= 16 ? dense_kernel_for<16>(mode) : dense_kernel_for<32>(mode);
}

kfun_t dseg_kernel_for(int bp, int mode, int l)
{
    const bool w16 = bp <= 16;
    if (l == 0) {
        if (mode == M_FACTOR) return w16 ? kkt_dense_seg<16, false> : kkt_dense_seg<32, false>;
        return w16 ? kkt_dense_seg<16, true> : kkt_dense_seg<32, true>;
    }
    if (l == 2) return w16 ? kkt_dense_seg_bwd<16> : kkt_dense_seg_bwd<32>;
    const bool fs = mode == M_FACTOR_SOLVE;
    switch (bp) {
    case 16: return fs ? kkt_reduced<16, M_FACTOR_SOLVE> : kkt_reduced<16, M_FACTOR>;
    case 24: return fs ? kkt_reduced<24, M_FACTOR_SOLVE> : kkt_reduced<24, M_FACTOR>;
    default: return fs ? kkt_reduced<32, M_FACTOR_SOLVE> : kkt_reduced<32, M_FACTOR>;
    }
}

kfun_t dense_bwd_kernel_for(int bp, int mode)
{
    if (mode == M_ADJOINT) return bp <= 16 ? kkt_dense_bwd<16, true> : kkt_dense_bwd<32, true>;
    return bp <= 16 ? kkt_dense_bwd<16, false> : kkt_dense_bwd<32, false>;
}

int dense_width(int bp) { return bp <= 16 ? 16 : 32; }

kfun_t kernel_for_class(int cls, int mode)
{
    switch (CLS_BP[cls]) {
    case 8: return kernel_for<8>(mode);
    case 16: return kernel_for<16>(mode);
    case 24: return kernel_for<24>(mode);
    default: return kernel_for<32>(mode);
    }
}

int nt_of_class(int cls)
{
    const int bp = CLS_BP[cls];
    return ((3 * bp + NGM + 63) / 64) * 64;
}

// Eq. (13) with the (p - 1 + sigma) denominator, sigma = 19/7, ties to floor,
// N_1 >= 1 and N_k >= 1 enforced.  Exact rational comparisons (integers x21).
bool partition_eq13(int N, int p, int *N1, int *Nk)
{
    if (p == 1) { *N1 = N; *Nk = 0; return true; }
    // bar N_k = (N - p + 1) / (p - 1 + 19/7) = 7 (N - p + 1) / (7 p + 12)
    const long long num = 7LL * (N - p + 1), den = 7LL * p + 12;
    const long long fl = num / den, ce = (num + den - 1) / den;
    bool have = false;
    long long best = 0;
    int b1 = 0, bk = 0;
    const long long cand[2] = {fl, ce};
    for (int t = 0; t < 2; ++t) {
        const long long nk = cand[t];
        if (t == 1 && ce == fl) break;
        const long long n1 = N - (p - 1) - (p - 1) * nk;
        if (nk < 1 || n1 < 1) continue;
        const long long cost = std::max(7 * n1, 19 * nk);   // x3
        if (!have || cost < best) { have = true; best = cost; b1 = (int)n1; bk = (int)nk; }
    }
    if (!have) return false;
    *N1 = b1; *Nk = bk;
    return true;
}

// Segment lengths balancing a first segment at t1 per stage against the others at
// tk per stage (Eq. 13 with sigma = tk / t1); false if N < 2p - 1.
bool partition_sigma(int N, int p, double t1, double tk, int *N1, int *Nk)
{
    if (p == 1) { *N1 = N; *Nk = 0; return true; }
    const double sigma = tk / t1;
    const double nbar = (double)(N - p + 1) / ((double)(p - 1) + sigma);
    const long long cand[2] = {(long long)std::floor(nbar), (long long)std::ceil(nbar)};
    bool have = false;
    double best = 0;
    for (int t = 0; t < 2; ++t) {
        const long long nk = cand[t];
        if (t == 1 && cand[1] == cand[0]) break;
        const long long n1 = N - (p - 1) - (p - 1) * nk;
        if (nk < 1 || n1 < 1) continue;
        const double cost = std::max(n1 * t1, nk * tk);
        if (!have || cost < best) { have = true; best = cost; *N1 = (int)n1; *Nk = (int)nk; }
    }
    return have;
}

struct ItemEst {
    double longest, total;
};

// Estimated longest item and total work of one system split into p segments.
ItemEst estimate(int N, int p, int cls, const kkt_cost_model &m)
{
    int N1 = N, Nk = 0;
    if (p > 1 && !partition_sigma(N, p, m.t_first[cls], m.t_fill[cls], &N1, &Nk)) return {1e300, 1e300};
    const double seg1 = m.t_item[cls] + N1 * m.t_first[cls];
    const double segk = p > 1 ? m.t_item[cls] + Nk * m.t_fill[cls] : 0.0;
    const double red = (p - 1) * m.t_red[cls];
    return {std::max(seg1, segk) + red, seg1 + (p - 1) * segk + red};
}

// Items of class cls the device runs at once, for systems of p segments.
double pool(const kkt_cost_model &m, int cls, int p)
{
    const double w = (p > 1 && m.workers_seg[cls] > 0.0) ? m.workers_seg[cls] : m.workers[cls];
    return std::max(1.0, w);
}

// Choose p for the systems with dims[s].p == 0.  The classes of a batch run
// concurrently and share the device, so the step is modelled as
// max(sum over classes of total work / workers, longest item of any class).  For a
// bound T on the longest item every tuned system takes the fewest segments whose
// longest item stays within T; total work falls as T grows, so the best T sits
// where the summed work crosses T.  The candidate bounds are the longest-item
// values themselves, searched by bisection, and the two candidates around the
// crossing are compared.  Systems of one class and length always get equal p (a
// greedy split of one system at a time stalls on such ties).
void choose_segments(std::vector<kkt_dims> &dims, const std::vector<int> &cls_of, const kkt_cost_model &m)
{
    double fixed_work = 0.0, fixed_longest = 0.0;
    std::map<std::pair<int, int>, int> count;      // tuned systems per (class, N)
    for (size_t s = 0; s < dims.size(); ++s) {
        const int c = cls_of[s];
        if (dims[s].p == 0) {
            count[{c, dims[s].N}] += 1;
        } else {
            const ItemEst e = estimate(dims[s].N, dims[s].p, c, m);
            fixed_work += e.total / pool(m, c, dims[s].p);
            fixed_longest = std::max(fixed_longest, e.longest);
        }
    }
    if (count.empty()) return;
    struct Len {
        int cls, N, cnt;
        std::vector<ItemEst> est;                  // est[p - 1], p = 1 .. (N + 1) / 2
    };
    std::vector<Len> lens;
    std::vector<double> cand;
    for (const auto &kv : count) {
        const int c = kv.first.first, N = kv.first.second;
        Len L{c, N, kv.second, {}};
        const int pmax = std::max(1, std::min((N + 1) / 2, 256));
        for (int p = 1; p <= pmax; ++p) {
            L.est.push_back(estimate(N, p, c, m));
            if (L.est.back().longest < 1e299) cand.push_back(std::max(L.est.back().longest, fixed_longest));
        }
        lens.push_back(std::move(L));
    }
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    // fewest segments meeting T (the shortest longest item if none does), per length
    auto pick = [&](double T, std::vector<int> *ps, double *longest) {
        double work = fixed_work;
        *longest = fixed_longest;
        for (size_t i = 0; i < lens.size(); ++i) {
            const Len &L = lens[i];
            int best = 0;
            for (int q = 0; q < (int)L.est.size(); ++q) {
                if (L.est[q].longest <= T) { best = q; break; }
                if (L.est[q].longest < L.est[best].longest) best = q;
            }
            if (ps) (*ps)[i] = best + 1;
            work += L.cnt * L.est[best].total / pool(m, L.cls, best + 1);
            *longest = std::max(*longest, L.est[best].longest);
        }
        return work;
    };
    // smallest candidate T that the choice for T meets: summed work <= T, longest <= T
    double lg = 0.0;
    auto meets = [&](double T) { return std::max(pick(T, nullptr, &lg), lg) <= T; };
    size_t lo = 0, hi = cand.size() - 1;
    if (meets(cand[hi])) {
        while (lo < hi) {
            const size_t mid = (lo + hi) / 2;
            if (meets(cand[mid])) hi = mid; else lo = mid + 1;
        }
    } else {
        lo = hi;
    }
    double best_span = 1e300;
    std::vector<int> ps(lens.size()), best_ps(lens.size(), 1);
    for (size_t k = (lo > 0 ? lo - 1 : 0); k <= lo; ++k) {
        const double work = pick(cand[k], &ps, &lg);
        const double span = std::max(work, lg);
        if (span < best_span) { best_span = span; best_ps = ps; }
    }
    std::map<std::pair<int, int>, int> p_of;
    for (size_t i = 0; i < lens.size(); ++i) p_of[{lens[i].cls, lens[i].N}] = best_ps[i];
    // a tuned system is split with the balance the estimates assumed (Eq. 13 with
    // sigma = t_fill / t_first of the model) unless its first segment is given
    for (size_t s = 0; s < dims.size(); ++s) {
        if (dims[s].p != 0) continue;
        const int c = cls_of[s], p = p_of[{c, dims[s].N}];
        dims[s].p = p;
        int N1 = 0, Nk = 0;
        if (p > 1 && dims[s].N1 == 0 && partition_sigma(dims[s].N, p, m.t_first[c], m.t_fill[c], &N1, &Nk))
            dims[s].N1 = N1;
    }
}

kkt_cost_model default_cost_model()
{
    kkt_cost_model m;
    for (int c = 0; c < 4; ++c) {
        const double b3 = (double)CLS_BP[c] * CLS_BP[c] * CLS_BP[c];
        m.t_first[c] = 7.0 / 3.0 * b3;
        m.t_fill[c] = 19.0 / 3.0 * b3;
        m.t_red[c] = 10.0 / 3.0 * b3;
        m.t_item[c] = 0.0;
        m.workers[c] = 512.0;
        m.workers_seg[c] = 512.0;
    }
    return m;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct kkt_plan {
    int S = 0, nrhs = 1;
    std::vector<SysDesc> sys;
    std::vector<kkt_system_layout> lay;
    struct Cls {
        int cls = 0, bp = 0, nt = 0;
        int item_off = 0, item_cnt = 0, s3_off = 0, s3_cnt = 0;
        size_t lds = 0;
        bool dense = false;       // whole (p = 1) systems: dense single-wave sweeps
        bool dseg = false;        // segmented systems of the 16/24/32 classes: dense segment sweeps
        size_t lds_dense = 0;     // LDS of the dense launches
        int red_off = 0, red_cnt = 0;   // dseg: systems (sequential phase)
    };
    std::vector<Cls> cls;
    std::vector<int2> items;
    std::vector<int> red;
    size_t o_ctr = 0, o_sys = 0, o_items = 0, o_slot = 0, o_ready = 0, o_arrive = 0, o_fail = 0,
           o_status = 0, o_tag = 0, o_F = 0, o_red = 0, bytes = 0;
    long long nF = 0;
    kkt_plan_info info{};
    int spin_limit = 1 << 22;
    // Workspaces this plan has factored into (a host-side guard against solving
    // with no factor; kkt_workspace_init forgets a workspace again).
    mutable std::mutex factored_mu;
    mutable std::unordered_set<const void *> factored;
    void mark_factored(const void *ws) const { std::lock_guard<std::mutex> g(factored_mu); factored.insert(ws); }
    void forget(const void *ws) const { std::lock_guard<std::mutex> g(factored_mu); factored.erase(ws); }
    bool is_factored(const void *ws) const
    {
        std::lock_guard<std::mutex> g(factored_mu);
        return factored.count(ws) != 0;
    }
    // launch configuration per (class, mode), filled on first use so that later
    // calls (and graph capture) make no device queries
    static constexpr int MAXC = 8;
    mutable int grid[MAXC][12] = {{0}};   // per (mode, launch of the class)
    // optional per-class timing events (kkt_plan_set_class_events)
    hipEvent_t ev_start[MAXC] = {nullptr};
    hipEvent_t ev_stop[MAXC] = {nullptr};
    // With several classes, the first NSIDE classes run on streams of their own,
    // forked from and joined back into the caller's stream through events (created
    // on first use on the current device; the mutex keeps concurrent callers'
    // fork/join sequences from interleaving), and any further class runs on the
    // caller's stream itself.  HIP maps a process's streams onto 4 hardware queues
    // by default; a fourth side stream would share a queue with another side stream
    // and run only after that stream's work, while the caller's stream has a queue
    // of its own.
    static constexpr int NSIDE = 3;
    mutable std::mutex side_mu;
    mutable int side_dev = -1;
    mutable hipStream_t side[MAXC] = {nullptr};
    mutable hipEvent_t fork_ev = nullptr;
    mutable hipEvent_t join_ev[MAXC] = {nullptr};
    void release_side() const
    {
        // teardown: a failure to destroy leaves nothing to recover, so it is ignored
        for (int c = 0; c < MAXC; ++c) {
            if (side[c]) (void)hipStreamDestroy(side[c]);
            if (join_ev[c]) (void)hipEventDestroy(join_ev[c]);
            side[c] = nullptr;
            join_ev[c] = nullptr;
        }
        if (fork_ev) (void)hipEventDestroy(fork_ev);
        fork_ev = nullptr;
        side_dev = -1;
    }
    bool ensure_side(int dev) const
    {
        if (side_dev == dev) return true;
        release_side();
        if (hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming) != hipSuccess) return false;
        for (size_t c = 0; c < cls.size() && c < (size_t)NSIDE; ++c) {
            if (hipStreamCreateWithFlags(&side[c], hipStreamNonBlocking) != hipSuccess) return false;
            if (hipEventCreateWithFlags(&join_ev[c], hipEventDisableTiming) != hipSuccess) return false;
        }
        side_dev = dev;
        return true;
    }
    ~kkt_plan() { release_side(); }
};

namespace {

const long long PLAN_TAG = 0x6b6b742d67393530LL;   // written by kkt_workspace_init

bool valid_dims(const kkt_dims &d)
{
    if (d.N < 1 || d.b < 1 || d.b > KKT_MAX_B || d.ng < 0 || d.ng > KKT_MAX_NG) return false;
    if (d.p < 0) return false;
    if (d.p > 1 && d.N < 2 * d.p - 1) return false;
    return true;
}

// Cost of one (system, segment) item in stage-steps, weighted by block size:
// used for the LPT order only.
double item_cost(const SysDesc &s, int k)
{
    const double b = s.b < 8 ? 8.0 : (double)s.b;
    const int len = (k == 1) ? s.N1 : s.Nk;
    const double per = (k == 1) ? 1.0 : 2.5;
    return len * per * b * b * b + (s.p > 1 && k == s.p ? s.p * 3.0 * b * b * b : 0.0);
}

int launch_mode(const kkt_plan *plan, int mode, const Args &base, hipStream_t stream, int *info)
{
    const int nctr = 4 * (int)plan->cls.size();
    char *ws = (char *)0;
    (void)ws;
    hipLaunchKernelGGL(kkt_reset, dim3(std::max(1, std::min(1024, (plan->S + 255) / 256))), dim3(256), 0, stream,
                       base.ctr, nctr, base.arrive, (mode <= M_FACTOR_SOLVE) ? base.failidx : nullptr, plan->S,
                       base.s3_ready - 0, (int)plan->info.num_items, (mode <= M_FACTOR_SOLVE) ? info : nullptr);
    if (hipGetLastError() != hipSuccess) return KKT_ELAUNCH;
    int ncls = 0;
    for (const kkt_plan::Cls &c : plan->cls) ncls += c.item_cnt > 0;
    const bool fork = ncls > 1;
    std::unique_lock<std::mutex> side_lock(plan->side_mu, std::defer_lock);
    if (fork) {
        side_lock.lock();
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || !plan->ensure_side(dev)) return KKT_ELAUNCH;
        if (hipEventRecord(plan->fork_ev, stream) != hipSuccess) return KKT_ELAUNCH;
    }
    // active classes 0 .. NSIDE-1 on the side streams, the rest on the caller's stream
    int nside = 0;
    for (size_t ci = 0; ci < plan->cls.size(); ++ci) {
        const kkt_plan::Cls &c = plan->cls[ci];
        if (c.item_cnt == 0) continue;
        const bool on_side = fork && nside < kkt_plan::NSIDE;
        hipStream_t st = on_side ? plan->side[nside] : stream;
        if (on_side && hipStreamWaitEvent(st, plan->fork_ev, 0) != hipSuccess) return KKT_ELAUNCH;
        Args a = base;
        a.items = base.items + c.item_off;
        a.n_items = c.item_cnt;
        a.s3_slot = base.s3_slot + c.s3_off;
        a.s3_ready = base.s3_ready + c.s3_off;
        a.n_s3 = c.s3_cnt;
        a.ctr = base.ctr + 4 * ci;
        // launches of this class: a dense class runs its (factor or forward) sweep and
        // then its backward sweep; a segmented dense class in the factor modes runs the
        // segment sweeps, the sequential phase (general kernel) and the segment
        // backward sweeps; everything else is one general persistent launch
        const bool dseg = c.dseg && mode <= M_FACTOR_SOLVE;
        const int nlaunch = c.dense ? (mode != M_FACTOR ? 2 : 1) : dseg ? (mode == M_FACTOR ? 2 : 3) : 1;
        if (dseg) {
            a.red = base.red + c.red_off;
            a.n_red = c.red_cnt;
        }
        if (plan->ev_start[ci] && hipEventRecord(plan->ev_start[ci], st) != hipSuccess) return KKT_ELAUNCH;
        for (int l = 0; l < nlaunch; ++l) {
            kfun_t fn;
            int nt = 64, work = c.item_cnt;
            size_t lds = c.lds_dense;
            if (c.dense) {
                fn = l == 0 ? dense_kernel_for(c.bp, mode) : dense_bwd_kernel_for(c.bp, mode);
            } else if (dseg) {
                fn = dseg_kernel_for(c.bp, mode, l);
                if (l == 1) {
                    nt = c.nt;
                    lds = c.lds;
                    work = c.red_cnt;
                }
            } else {
                fn = kernel_for_class(c.cls, mode);
                nt = c.nt;
                lds = c.lds;
            }
            int &grid = plan->grid[ci][mode * 3 + l];
            if (grid == 0) {
                int dev = 0, ncu = 0, occ = 0;
                if (hipGetDevice(&dev) != hipSuccess) return KKT_ELAUNCH;
                if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
                    return KKT_ELAUNCH;
                if (lds > 65536 &&
                    hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
                        hipSuccess)
                    return KKT_ELAUNCH;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)fn, nt, lds) != hipSuccess ||
                    occ < 1)
                    occ = 1;
                grid = std::max(1, std::min(work, occ * ncu));
            }
            hipLaunchKernelGGL(fn, dim3(grid), dim3(nt), lds, st, a);
            if (hipGetLastError() != hipSuccess) return KKT_ELAUNCH;
        }
        if (plan->ev_stop[ci] && hipEventRecord(plan->ev_stop[ci], st) != hipSuccess) return KKT_ELAUNCH;
        if (on_side && hipEventRecord(plan->join_ev[nside++], st) != hipSuccess) return KKT_ELAUNCH;
    }
    // the caller's stream waits for the side streams only after its own classes are
    // queued, so that those run beside the side streams
    for (int j = 0; j < nside; ++j)
        if (hipStreamWaitEvent(stream, plan->join_ev[j], 0) != hipSuccess) return KKT_ELAUNCH;
    return KKT_OK;
}

Args base_args(const kkt_plan *plan, void *workspace)
{
    char *ws = (char *)workspace;
    Args a;
    std::memset(&a, 0, sizeof(a));
    a.F = (double *)(ws + plan->o_F);
    a.sys = (const SysDesc *)(ws + plan->o_sys);
    a.items = (const int2 *)(ws + plan->o_items);
    a.red = (const int *)(ws + plan->o_red);
    a.s3_slot = (int2 *)(ws + plan->o_slot);
    a.s3_ready = (int *)(ws + plan->o_ready);
    a.ctr = (int *)(ws + plan->o_ctr);
    a.arrive = (int *)(ws + plan->o_arrive);
    a.failidx = (int *)(ws + plan->o_fail);
    a.status = (int *)(ws + plan->o_status);
    a.nr = plan->nrhs;
    a.spin_limit = plan->spin_limit;
    return a;
}

bool aligned8(const void *p) { return ((uintptr_t)p & 7) == 0; }

}  // namespace

extern "C" {

int kkt_plan_create(kkt_plan **out, int32_t S, const kkt_dims *dims, int32_t nrhs)
{
    return kkt_plan_create_tuned(out, S, dims, nrhs, nullptr);
}

int kkt_plan_create_tuned(kkt_plan **out, int32_t S, const kkt_dims *dims_in, int32_t nrhs,
                          const kkt_cost_model *model)
{
    if (!out) return KKT_EPOINTER;
    *out = nullptr;
    if (S < 1 || !dims_in) return S < 1 ? KKT_EDIMS : KKT_EPOINTER;
    if (nrhs < 1 || nrhs > KKT_MAX_NRHS) return KKT_EDIMS;
    std::vector<kkt_dims> dims(dims_in, dims_in + S);
    {
        std::vector<int> cls0(S);
        for (int s = 0; s < S; ++s) {
            if (!valid_dims(dims[s])) return KKT_EDIMS;
            cls0[s] = class_of(dims[s].b);
        }
        const kkt_cost_model m = model ? *model : default_cost_model();
        choose_segments(dims, cls0, m);
    }
    kkt_plan *P = new (std::nothrow) kkt_plan;
    if (!P) return KKT_EINTERNAL;
    P->S = S;
    P->nrhs = nrhs;
    P->sys.resize(S);
    P->lay.resize(S);
    long long oD = 0, oC = 0, oB = 0, oCor = 0, oR = 0, oF = 0;
    double fflops = 0, sflops = 0;
    long long fwords = 0, iwords = 0;
    std::vector<int> cls_of(S);
    for (int s = 0; s < S; ++s) {
        kkt_dims d = dims[s];
        if (!valid_dims(d)) { delete P; return KKT_EDIMS; }
        const int p = d.p;
        int N1 = 0, Nk = 0;
        if (p == 1) {
            N1 = d.N;
        } else if (d.N1 > 0) {
            const int rest = d.N - d.N1 - (p - 1);
            if (rest < p - 1 || rest % (p - 1) != 0) { delete P; return KKT_EDIMS; }
            N1 = d.N1;
            Nk = rest / (p - 1);
        } else if (!partition_eq13(d.N, p, &N1, &Nk)) {
            delete P;
            return KKT_EDIMS;
        }
        const long long N = d.N, b = d.b, ng = d.ng, b2 = b * b;
        SysDesc &sd = P->sys[s];
        std::memset(&sd, 0, sizeof(sd));
        sd.N = d.N; sd.b = d.b; sd.ng = d.ng; sd.p = p; sd.N1 = N1; sd.Nk = Nk;
        sd.cls = class_of(d.b);
        cls_of[s] = sd.cls;
        sd.oD = oD; sd.oC = oC; sd.oB = oB; sd.oCorner = oCor; sd.oRhs = oR;
        oD += N * b2; oC += (N - 1) * b2; oB += N * ng * b; oCor += ng * ng; oR += (N * b + ng) * nrhs;
        const long long fill = (p >= 2) ? (long long)(p - 1) * (Nk - 1) * b2 : 0;
        const long long H = (p >= 3) ? (long long)(p - 2) * b2 : 0;
        sd.oLd = oF; oF += N * b2;
        sd.oLc = oF; oF += (N - 1) * b2;
        sd.oLb = oF; oF += N * ng * b;
        sd.oLg = oF; oF += ng * ng;
        sd.oFill = oF; oF += fill;
        sd.oH = oF; oF += H;
        sd.scrStride = scr_stride((int)b, (int)ng, nrhs);
        sd.oScr = oF; oF += (long long)p * sd.scrStride;
        oF = (oF + 31) & ~31LL;
        kkt_system_layout &L = P->lay[s];
        L.N = d.N; L.b = d.b; L.ng = d.ng; L.p = p; L.N1 = N1; L.Nk = Nk;
        L.off_D = sd.oD; L.off_C = sd.oC; L.off_B = sd.oB; L.off_corner = sd.oCorner; L.off_rhs = sd.oRhs;
        L.off_Ld = sd.oLd; L.off_Lc = sd.oLc; L.off_Lb = sd.oLb; L.off_Lg = sd.oLg; L.off_fill = sd.oFill;
        L.off_H = sd.oH;
        // standard flop counts of the sequential method (potrf n^3/3, trsm m n^2,
        // syrk/gemm 2 m n k) plus the fill-in work of the segmented order
        const double bb = (double)b, gg = (double)ng;
        double fseq = N * bb * bb * bb / 3 + (N - 1) * (bb * bb * bb + 2 * bb * bb * bb) +
                      N * (gg * bb * bb + 2 * gg * gg * bb) + (N - 1) * 2 * gg * bb * bb + gg * gg * gg / 3;
        if (p >= 2) {
            // per stage of segments k >= 2: trsm of b fill rows, their Gram with themselves,
            // with the next-stage rows and with the arrow rows
            const double extra_stage = bb * bb * bb + 2 * bb * bb * bb + 2 * bb * bb * bb + 2 * gg * bb * bb;
            fseq += (double)(p - 1) * Nk * extra_stage + (double)(p - 1) * 2 * bb * bb * bb;
        }
        fflops += fseq;
        sflops += nrhs * (2.0 * N * bb * bb + 4.0 * (N - 1) * bb * bb + 4.0 * N * gg * bb + 2 * gg * gg +
                          (p >= 2 ? 4.0 * (double)(p - 1) * Nk * bb * bb : 0.0));
        fwords += N * b2 + (N - 1) * b2 + N * ng * b + ng * ng + fill + H;
        iwords += N * b2 + (N - 1) * b2 + N * ng * b + ng * ng;
    }
    P->nF = oF;
    // items grouped by class, LPT (longest first) inside a class
    int nitems = 0, ns3 = 0;
    for (int cc = 0; cc < 2 * NCLS; ++cc) {
        // per block-size class: whole systems of the 16/24/32 classes first (dense
        // launch in the factor modes), then everything else
        const int c = cc >> 1;
        const bool dense = (cc & 1) == 0 && CLS_BP[c] >= 16;
        if ((cc & 1) == 0 && !dense) continue;
        std::vector<std::pair<double, int2>> its;
        int s3 = 0;
        for (int s = 0; s < S; ++s) {
            if (cls_of[s] != c) continue;
            const SysDesc &sd = P->sys[s];
            if (CLS_BP[c] >= 16 && (sd.p == 1) != dense) continue;
            for (int k = 1; k <= sd.p; ++k) its.push_back({item_cost(sd, k), make_int2(s, k)});
            if (sd.p > 1) s3 += sd.p - 1;
        }
        if (its.empty()) continue;
        std::stable_sort(its.begin(), its.end(), [](const std::pair<double, int2> &x, const std::pair<double, int2> &y) {
            return x.first > y.first;
        });
        kkt_plan::Cls C;
        C.cls = c;
        C.bp = CLS_BP[c];
        C.nt = nt_of_class(c);
        C.item_off = nitems;
        C.item_cnt = (int)its.size();
        C.s3_off = ns3;
        C.s3_cnt = s3;
        C.lds = (size_t)lds_offsets(C.bp, nrhs).total * sizeof(double);
        C.dense = dense;
        C.dseg = !dense && CLS_BP[c] >= 16;
        if (dense) C.lds_dense = (size_t)lds_offsets_dense(dense_width(C.bp), nrhs).total * sizeof(double);
        if (C.dseg) {
            C.lds_dense = (size_t)lds_offsets_dense(dense_width(C.bp), nrhs, true).total * sizeof(double);
            C.red_off = (int)P->red.size();
            for (int s = 0; s < S; ++s)
                if (cls_of[s] == c && P->sys[s].p > 1) P->red.push_back(s);
            C.red_cnt = (int)P->red.size() - C.red_off;
        }
        for (auto &x : its) P->items.push_back(x.second);
        nitems += C.item_cnt;
        ns3 += s3;
        P->cls.push_back(C);
    }
    // workspace layout
    size_t o = 0;
    P->o_tag = o; o = align256(o + 16);
    P->o_ctr = o; o = align256(o + sizeof(int) * 4 * P->cls.size());
    P->o_sys = o; o = align256(o + sizeof(SysDesc) * S);
    P->o_items = o; o = align256(o + sizeof(int2) * std::max(1, nitems));
    P->o_red = o; o = align256(o + sizeof(int) * std::max<size_t>(1, P->red.size()));
    P->o_slot = o; o = align256(o + sizeof(int2) * std::max(1, ns3));
    P->o_ready = o; o = align256(o + sizeof(int) * std::max(1, std::max(ns3, nitems)));
    P->o_arrive = o; o = align256(o + sizeof(int) * S);
    P->o_fail = o; o = align256(o + sizeof(int) * S);
    P->o_status = o; o = align256(o + sizeof(int) * S);
    P->o_F = o; o = align256(o + sizeof(double) * (size_t)oF);
    P->bytes = o;
    kkt_plan_info &I = P->info;
    I.num_systems = S;
    I.nrhs = nrhs;
    I.num_items = nitems;
    I.num_classes = (int)P->cls.size();
    I.D_len = oD; I.C_len = oC; I.B_len = oB; I.corner_len = oCor; I.rhs_len = oR;
    I.workspace_bytes = (int64_t)P->bytes;
    I.factor_flops = fflops;
    I.solve_flops = sflops;
    I.factor_words = fwords;
    I.input_words = iwords;
    *out = P;
    return KKT_OK;
}

int kkt_plan_destroy(kkt_plan *plan)
{
    delete plan;
    return KKT_OK;
}

int kkt_plan_get_info(const kkt_plan *plan, kkt_plan_info *info)
{
    if (!plan || !info) return KKT_EPOINTER;
    *info = plan->info;
    return KKT_OK;
}

int kkt_plan_system(const kkt_plan *plan, int32_t s, kkt_system_layout *out)
{
    if (!plan || !out) return KKT_EPOINTER;
    if (s < 0 || s >= plan->S) return KKT_EDIMS;
    *out = plan->lay[s];
    return KKT_OK;
}

int64_t kkt_plan_factor_offset(const kkt_plan *plan) { return plan ? (int64_t)plan->o_F : -1; }

int kkt_workspace_init(const kkt_plan *plan, void *workspace, hipStream_t stream)
{
    if (!plan || !workspace) return KKT_EPOINTER;
    if (((uintptr_t)workspace & 255) != 0) return KKT_EPOINTER;
    char *ws = (char *)workspace;
    if (hipMemcpyAsync(ws + plan->o_sys, plan->sys.data(), sizeof(SysDesc) * plan->S, hipMemcpyHostToDevice, stream) !=
        hipSuccess)
        return KKT_ELAUNCH;
    if (!plan->items.empty() &&
        hipMemcpyAsync(ws + plan->o_items, plan->items.data(), sizeof(int2) * plan->items.size(), hipMemcpyHostToDevice,
                       stream) != hipSuccess)
        return KKT_ELAUNCH;
    if (!plan->red.empty() &&
        hipMemcpyAsync(ws + plan->o_red, plan->red.data(), sizeof(int) * plan->red.size(), hipMemcpyHostToDevice,
                       stream) != hipSuccess)
        return KKT_ELAUNCH;
    std::vector<int> st(plan->S, 0);
    if (hipMemcpyAsync(ws + plan->o_status, st.data(), sizeof(int) * plan->S, hipMemcpyHostToDevice, stream) !=
        hipSuccess)
        return KKT_ELAUNCH;
    long long tag[2] = {PLAN_TAG, (long long)plan->bytes};
    if (hipMemcpyAsync(ws + plan->o_tag, tag, sizeof(tag), hipMemcpyHostToDevice, stream) != hipSuccess)
        return KKT_ELAUNCH;
    if (hipStreamSynchronize(stream) != hipSuccess) return KKT_ELAUNCH;
    plan->forget(workspace);
    return KKT_OK;
}

int kkt_factor(const kkt_plan *plan, const double *D, const double *C, const double *B, const double *corner,
               void *workspace, int32_t *info, hipStream_t stream)
{
    if (!plan || !workspace || !D || !info) return KKT_EPOINTER;
    if (plan->info.C_len && !C) return KKT_EPOINTER;
    if (plan->info.B_len && (!B || !corner)) return KKT_EPOINTER;
    if (((uintptr_t)workspace & 255) || !aligned8(D) || !aligned8(C) || !aligned8(B) || !aligned8(corner))
        return KKT_EPOINTER;
    Args a = base_args(plan, workspace);
    a.D = D; a.C = C; a.B = B; a.corner = corner; a.info = info;
    const int rc = launch_mode(plan, M_FACTOR, a, stream, info);
    if (rc == KKT_OK) plan->mark_factored(workspace);
    return rc;
}

int kkt_factor_solve(const kkt_plan *plan, const double *D, const double *C, const double *B, const double *corner,
                     void *workspace, double *rhs, int32_t *info, hipStream_t stream)
{
    if (!plan || !workspace || !D || !info || !rhs) return KKT_EPOINTER;
    if (plan->info.C_len && !C) return KKT_EPOINTER;
    if (plan->info.B_len && (!B || !corner)) return KKT_EPOINTER;
    if (((uintptr_t)workspace & 255) || !aligned8(D) || !aligned8(C) || !aligned8(B) || !aligned8(corner) ||
        !aligned8(rhs))
        return KKT_EPOINTER;
    Args a = base_args(plan, workspace);
    a.D = D; a.C = C; a.B = B; a.corner = corner; a.info = info; a.rhs = rhs;
    const int rc = launch_mode(plan, M_FACTOR_SOLVE, a, stream, info);
    if (rc == KKT_OK) plan->mark_factored(workspace);
    return rc;
}

int kkt_solve(const kkt_plan *plan, void *workspace, double *rhs, hipStream_t stream)
{
    if (!plan || !workspace || !rhs) return KKT_EPOINTER;
    if (((uintptr_t)workspace & 255) || !aligned8(rhs)) return KKT_EPOINTER;
    if (!plan->is_factored(workspace)) return KKT_ENOTFACTORED;
    Args a = base_args(plan, workspace);
    a.rhs = rhs;
    return launch_mode(plan, M_SOLVE, a, stream, nullptr);
}

int kkt_solve_adjoint(const kkt_plan *plan, void *workspace, const double *x, double *gx, double *dD, double *dC,
                      double *dB, double *dcorner, hipStream_t stream)
{
    if (!plan || !workspace || !x || !gx || !dD) return KKT_EPOINTER;
    if (plan->info.C_len && !dC) return KKT_EPOINTER;
    if (plan->info.B_len && (!dB || !dcorner)) return KKT_EPOINTER;
    if (((uintptr_t)workspace & 255) || !aligned8(x) || !aligned8(gx) || !aligned8(dD) || !aligned8(dC) ||
        !aligned8(dB) || !aligned8(dcorner))
        return KKT_EPOINTER;
    if (!plan->is_factored(workspace)) return KKT_ENOTFACTORED;
    Args a = base_args(plan, workspace);
    a.rhs = gx; a.xp = x; a.dD = dD; a.dC = dC; a.dB = dB; a.dcorner = dcorner;
    return launch_mode(plan, M_ADJOINT, a, stream, nullptr);
}

int kkt_workspace_error(const kkt_plan *plan, const void *workspace, hipStream_t stream, int32_t *flag)
{
    if (!plan || !workspace || !flag) return KKT_EPOINTER;
    std::vector<int> ctr(4 * plan->cls.size(), 0);
    if (ctr.empty()) { *flag = 0; return KKT_OK; }
    if (hipMemcpyAsync(ctr.data(), (const char *)workspace + plan->o_ctr, sizeof(int) * ctr.size(),
                       hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return KKT_ELAUNCH;
    int f = 0;
    for (size_t c = 0; c < plan->cls.size(); ++c) f |= ctr[4 * c + 3];
    *flag = f;
    return KKT_OK;
}

int kkt_plan_set_spin_limit(kkt_plan *plan, int32_t limit)
{
    if (!plan) return KKT_EPOINTER;
    if (limit < 1) return KKT_EDIMS;
    plan->spin_limit = limit;
    return KKT_OK;
}

int kkt_plan_class_info(const kkt_plan *plan, int32_t c, int32_t *block_pad, int32_t *num_items,
                        int32_t *threads, int64_t *lds_bytes, int32_t *grid)
{
    if (grid && plan && c >= 0 && c < (int)plan->cls.size()) {
        // the item sweeps: the first launch of the factor modes
        *grid = std::max(plan->grid[c][M_FACTOR * 3], plan->grid[c][M_FACTOR_SOLVE * 3]);
    }
    if (!plan) return KKT_EPOINTER;
    if (c < 0 || c >= (int)plan->cls.size()) return KKT_EDIMS;
    const kkt_plan::Cls &C = plan->cls[c];
    if (block_pad) *block_pad = C.bp;
    if (num_items) *num_items = C.item_cnt;
    if (threads) *threads = (C.dense || C.dseg) ? 64 : C.nt;
    if (lds_bytes) *lds_bytes = (int64_t)((C.dense || C.dseg) ? C.lds_dense : C.lds);
    return KKT_OK;
}

int kkt_plan_class_kind(const kkt_plan *plan, int32_t c, int32_t *kind)
{
    if (!plan || !kind) return KKT_EPOINTER;
    if (c < 0 || c >= (int)plan->cls.size()) return KKT_EDIMS;
    const kkt_plan::Cls &C = plan->cls[c];
    *kind = C.dense ? KKT_CLASS_DENSE : C.dseg ? KKT_CLASS_DENSE_SEGMENTED : KKT_CLASS_GENERAL;
    return KKT_OK;
}

int kkt_plan_set_class_events(kkt_plan *plan, int32_t c, hipEvent_t start, hipEvent_t stop)
{
    if (!plan) return KKT_EPOINTER;
    if (c < 0 || c >= (int)plan->cls.size()) return KKT_EDIMS;
    plan->ev_start[c] = start;
    plan->ev_stop[c] = stop;
    return KKT_OK;
}

const char *kkt_status_string(int status)
{
    switch (status) {
    case KKT_OK: return "ok";
    case KKT_EDIMS: return "unsupported dimensions";
    case KKT_EPOINTER: return "null or misaligned pointer";
    case KKT_EWORKSPACE: return "workspace too small or not initialised";
    case KKT_ELAUNCH: return "HIP launch error";
    case KKT_ENOTFACTORED: return "solve before factorization in this workspace";
    case KKT_EINTERNAL: return "internal error";
    default: return "unknown status";
    }
}

}  // extern "C"
