// Row-lane kernels: three launches per mode (phase 1: every item; phase 2: the
// reduced chain and the corner of segmented systems; phase 3: the backward sweeps
// of their segments).  Padded block sizes 8 and 16 run the single-wave sweeps
// (kkt_lane.h), wider blocks the multi-wave sweeps (kkt_wave.h).  NR: the
// right-hand-side count of the single-wave instance (1, 4 or 8).
#pragma once
#include "kkt_lane.h"

namespace kkt_dev {

template <int BP, int NR, bool FWD, bool RED>
__device__ __forceinline__ int any_factor(const Args &a, const SysDesc &sd, int k, const WaveLds &L)
{
    if constexpr (WC<BP>::NW == 1) return lane_factor<BP, NR, FWD, RED>(a, sd, k, L);
    else return wave_factor<BP, FWD, RED>(a, sd, k, L);
}

template <int BP, int NR, bool RED>
__device__ __forceinline__ void any_forward(const Args &a, const SysDesc &sd, int k, const WaveLds &L)
{
    if constexpr (WC<BP>::NW == 1) lane_forward<BP, NR, RED>(a, sd, k, L);
    else wave_forward<BP, RED>(a, sd, k, L);
}

template <int BP, int NR, bool ADJ, bool RED>
__device__ __forceinline__ void any_backward(const Args &a, const SysDesc &sd, int k, const WaveLds &L)
{
    if constexpr (WC<BP>::NW == 1) lane_backward<BP, NR, ADJ, RED>(a, sd, k, L);
    else wave_backward<BP, ADJ, RED>(a, sd, k, L);
}

// ---------------------------------------------------------------- kernels
// Phase 1: every item of the class's first list.  A whole system (p = 1) runs
// all phases: factor (+ forward) sweep, corner, backward sweep (Algorithms 1-3
// with p = 1); a segment of a segmented system runs its parallel-phase factor
// (+ forward) sweep (factor modes) or its forward sweep (solve modes).
template <int BP, int MODE, int NR>
__global__ void __launch_bounds__(WC<BP>::NT) kkt_wave_p1(Args a)
{
    using C = WC<BP>;
    constexpr int NT = C::NT;
    constexpr bool FACT = MODE == M_FACTOR || MODE == M_FACTOR_SOLVE, FWD = MODE == M_FACTOR_SOLVE;
    extern __shared__ double lds_raw[];
    const WaveLds L = make_wave_lds<BP>(lds_raw);
    for (;;) {
        const int it = next_work(a.ctr + 0, a.abort, L.misc);
        if (it >= a.n_items) break;
        const int2 w = a.items[it];
        const SysDesc sd = a.sys[w.x];
        const bool whole = sd.p == 1;
        // one instance of each sweep serves whole systems (segment 1 of 1) and segments
        int f = 0;
        if (FACT) {
            f = any_factor<BP, NR, FWD, false>(a, sd, whole ? 1 : w.y, L);
            if (threadIdx.x == 0) {
                if (!whole && f) atomicMin(&a.failidx[w.x], f);
                L.misc[1] = f;
            }
        } else {
            if (threadIdx.x == 0) L.misc[1] = load_status(&a.status[w.x]);
            any_forward<BP, NR, false>(a, sd, whole ? 1 : w.y, L);
        }
        __syncthreads();
        if (whole) {
            int info = L.misc[1];
            if (FACT) {
                const bool cf = corner_factor_w<NT, FWD>(a, sd, L.nxt, L.nxt + NGM * (NGM + 1), nullptr, nullptr);
                if (threadIdx.x == 0) {
                    info = info ? info : (cf ? sd.N + 1 : 0);
                    a.status[w.x] = info;
                    if (a.info) a.info[w.x] = info;
                    L.misc[1] = info;
                }
                __syncthreads();
                info = L.misc[1];
            } else {
                corner_solve_w<NT>(a, sd, L.nxt, L.nxt + NGM * (NGM + 1), nullptr);
                if (MODE == M_ADJOINT) corner_grad_w<NT>(a, sd);
            }
            __syncthreads();
            if (MODE != M_FACTOR) {
                any_backward<BP, NR, MODE == M_ADJOINT, false>(a, sd, 1, L);
                if (info != 0) nan_fill<NT>(a, sd, 0, sd.N, true);
            }
        }
        __syncthreads();
    }
}

// Phase 2 of a segmented system (after every segment's phase 1): the reduced
// separator chain and the corner (Algorithm 1, 2 and 3 sequential phases).
template <int BP, int MODE, int NR>
__global__ void __launch_bounds__(WC<BP>::NT) kkt_wave_p2(Args a)
{
    using C = WC<BP>;
    constexpr int NT = C::NT;
    constexpr bool FACT = MODE == M_FACTOR || MODE == M_FACTOR_SOLVE, FWD = MODE == M_FACTOR_SOLVE;
    extern __shared__ double lds_raw[];
    const WaveLds L = make_wave_lds<BP>(lds_raw);
    for (;;) {
        const int it = next_work(a.ctr + 1, a.abort, L.misc);
        if (it >= a.n_red) break;
        const int s = a.red[it];
        const SysDesc sd = a.sys[s];
        int info;
        if (FACT) {
            const int rf = any_factor<BP, NR, FWD, true>(a, sd, 0, L);
            __syncthreads();
            const bool cf = corner_factor_w<NT, FWD, true>(a, sd, L.nxt, L.nxt + NGM * (NGM + 1), L.racc, L.yg);
            if (threadIdx.x == 0) {
                const int segf = load_status(&a.failidx[s]);
                const int v = segf != INT_MAX ? segf : (rf ? rf : (cf ? sd.N + 1 : 0));
                a.status[s] = v;
                if (a.info) a.info[s] = v;
                L.misc[1] = v;
            }
            __syncthreads();
            info = L.misc[1];
            if (FWD) any_backward<BP, NR, false, true>(a, sd, 0, L);
        } else {
            if (threadIdx.x == 0) L.misc[1] = load_status(&a.status[s]);
            any_forward<BP, NR, true>(a, sd, 0, L);
            __syncthreads();
            info = L.misc[1];
            corner_solve_w<NT, true>(a, sd, L.nxt, L.nxt + NGM * (NGM + 1), L.yg);
            if (MODE == M_ADJOINT) corner_grad_w<NT>(a, sd);
            __syncthreads();
            any_backward<BP, NR, MODE == M_ADJOINT, true>(a, sd, 0, L);
        }
        if (MODE != M_FACTOR && info != 0) {
            // NaN the separators and g (the segments do their own stages in phase 3)
            for (int k = 2; k <= sd.p; ++k) {
                const int sp = sep_of(sd, k);
                nan_fill<NT>(a, sd, sp, sp + 1, false);
            }
            nan_fill<NT>(a, sd, 0, 0, true);
        }
        __syncthreads();
    }
}

// Phase 3 of a segmented system (after its phase 2): the backward sweep of one
// segment (Algorithm 3, parallel phase; with the adjoint, its gradients).
template <int BP, int MODE, int NR>
__global__ void __launch_bounds__(WC<BP>::NT) kkt_wave_p3(Args a)
{
    using C = WC<BP>;
    constexpr int NT = C::NT;
    extern __shared__ double lds_raw[];
    const WaveLds L = make_wave_lds<BP>(lds_raw);
    for (;;) {
        const int it = next_work(a.ctr + 2, a.abort, L.misc);
        if (it >= a.n_s3) break;
        const int2 w = a.s3[it];
        const SysDesc sd = a.sys[w.x];
        any_backward<BP, NR, MODE == M_ADJOINT, false>(a, sd, w.y, L);
        if (threadIdx.x == 0) L.misc[1] = load_status(&a.status[w.x]);
        __syncthreads();
        if (L.misc[1] != 0) {
            const int f = seg_first(sd, w.y);
            nan_fill<NT>(a, sd, f, f + seg_len(sd, w.y), false);
        }
        __syncthreads();
    }
}

}  // namespace kkt_dev
