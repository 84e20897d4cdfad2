// MI355X (gfx950) segmented block Cholesky for block-tridiagonal-arrow KKT
// systems (arXiv 2511.00946): dense single-wave kernels, host plan and the C ABI
// of include/kkt.h.
//
// Scheduling.  A plan splits every system into p segments (Eq. 13 or given) and
// lists one work item per (system, segment), longest first (LPT).  Systems are
// grouped by padded block size into launch classes; each class runs up to three
// persistent launches whose workgroups pull work from atomic queues:
//   phase 1  every item: a whole system (p = 1) runs Algorithms 1-3 end to end;
//            a segment runs its factor (+ forward) sweep or its forward sweep
//            (Algorithms 1/2, parallel phase)
//   phase 2  each segmented system: the reduced separator chain and the corner
//            (Algorithms 1-3, sequential phases)
//   phase 3  each segment of a segmented system: its backward sweep (+ adjoint
//            gradients) (Algorithm 3, parallel phase)
// The launch boundaries order the phases, so no workgroup ever waits on another.
// Whole systems of the 16/24/32 classes run on the dense single-wave sweeps
// (kkt_dense.h), their segments' phases 1 and 3 on the dense segment sweeps;
// everything else runs on the row-lane sweeps (kkt_wave.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "kkt.h"

#include "kkt_device.h"
#include "kkt_internal.h"
#include "kkt_wave.h"
#include "kkt_dense.h"

using namespace kkt_dev;

namespace kkt_dev {

kfun_t wave_kernel(int bp, int mode, int phase, int nr)
{
    // the single-wave classes have instances for 1, 4 and 8 right-hand sides
    const int c = nr <= 1 ? 1 : (nr <= 4 ? 4 : 8);
    switch (bp) {
    case 8: return c == 1 ? wave_kernel_8_1(mode, phase) : (c == 4 ? wave_kernel_8_4(mode, phase) : wave_kernel_8_8(mode, phase));
    case 16:
        return c == 1 ? wave_kernel_16_1(mode, phase) : (c == 4 ? wave_kernel_16_4(mode, phase) : wave_kernel_16_8(mode, phase));
    case 24: return wave_kernel_24_8(mode, phase);
    case 32: return wave_kernel_32_8(mode, phase);
    default: return wave_kernel_48_8(mode, phase);
    }
}

int wave_threads(int bp)
{
    switch (bp) {
    case 8: return wave_threads_8();
    case 16: return wave_threads_16();
    case 24: return wave_threads_24();
    case 32: return wave_threads_32();
    default: return wave_threads_48();
    }
}

size_t wave_lds_bytes(int bp)
{
    switch (bp) {
    case 8: return wave_lds_bytes_8();
    case 16: return wave_lds_bytes_16();
    case 24: return wave_lds_bytes_24();
    case 32: return wave_lds_bytes_32();
    default: return wave_lds_bytes_48();
    }
}

}  // namespace kkt_dev

namespace {

// ------------------------------------------------------------------ dense kernels
// Whole (p = 1) systems of the 16-, 24- and 32-wide classes: one wave per
// system, dense stage sweeps (factor on the matrix cores, forward and backward
// substitution with the next stage's blocks in flight), then the corner
// (Algorithms 1-3 with p = 1).
template <int DB, int MODE>
__global__ void __launch_bounds__(64, DB == 16 ? 2 : 1) kkt_dense(Args a)
{
    extern __shared__ double lds_raw[];
    const Lds L = make_lds_dense(lds_raw, DB, a.nr);
    double *CR = L.P, *CW = L.P + NGM * (NGM + 1);
    constexpr bool FACT = MODE == M_FACTOR || MODE == M_FACTOR_SOLVE;
    for (;;) {
        const int it = next_work(a.ctr + 0, a.abort, L.misc);
        if (it >= a.n_items) break;
        const int2 w = a.items[it];
        const SysDesc sd = a.sys[w.x];
        if (FACT) {
            constexpr bool FWD = MODE == M_FACTOR_SOLVE;
            const int f = dense_factor<DB, FWD>(a, sd, L);
            const bool cf = corner_factor_w<64, FWD>(a, sd, CR, CW, nullptr, nullptr);
            if (threadIdx.x == 0) {
                const int info = f ? f : (cf ? sd.N + 1 : 0);
                a.status[w.x] = info;
                if (a.info) a.info[w.x] = info;
            }
        } else {
            dense_forward<DB>(a, sd, L);
            corner_solve_w<64>(a, sd, CR, CW, nullptr);
            if (MODE == M_ADJOINT) corner_grad_w<64>(a, sd);
        }
        __syncthreads();
    }
}

// Backward substitution (and with ADJ the adjoint gradients) of the whole systems
// of a dense class, after kkt_dense has run the factor or forward sweep and the
// corner of every one of them; a launch of its own, so that each of the two
// sweeps gets the registers it needs.  Items come from the second queue.
template <int DB, bool ADJ>
__global__ void __launch_bounds__(64, 2) kkt_dense_bwd(Args a)
{
    extern __shared__ double lds_raw[];
    const Lds L = make_lds_dense(lds_raw, DB, a.nr);
    for (;;) {
        const int it = next_work(a.ctr + 1, a.abort, L.misc);
        if (it >= a.n_items) break;
        const int2 w = a.items[it];
        const SysDesc sd = a.sys[w.x];
        dense_backward<DB, ADJ>(a, sd, L);
        if (threadIdx.x == 0) L.misc[2] = load_status(&a.status[w.x]);
        __syncthreads();
        if (L.misc[2] != 0) nan_fill<64>(a, sd, 0, sd.N, true);
        __syncthreads();
    }
}

// Segmented systems of the 16-, 24- and 32-wide classes, factor modes, phase 1:
// every segment's factor (+ forward) sweep, one wave per segment.
template <int DB, bool FWD>
__global__ void __launch_bounds__(64, DB == 16 ? 2 : 1) kkt_dense_seg(Args a)
{
    extern __shared__ double lds_raw[];
    const Lds L = make_lds_dense(lds_raw, DB, a.nr, true);
    for (;;) {
        const int it = next_work(a.ctr + 0, a.abort, L.misc);
        if (it >= a.n_items) break;
        const int2 w = a.items[it];
        const SysDesc sd = a.sys[w.x];
        const int f = dense_factor<DB, FWD, true>(a, sd, L, w.y);
        if (threadIdx.x == 0 && f) atomicMin(&a.failidx[w.x], f);
        __syncthreads();
    }
}

// ... phase 3: every segment's backward sweep, the separators already solved.
template <int DB>
__global__ void __launch_bounds__(64, DB == 16 ? 2 : 1) kkt_dense_seg_bwd(Args a)
{
    extern __shared__ double lds_raw[];
    const Lds L = make_lds_dense(lds_raw, DB, a.nr, true);
    for (;;) {
        const int it = next_work(a.ctr + 2, a.abort, L.misc);
        if (it >= a.n_s3) break;
        const int2 w = a.s3[it];
        const SysDesc sd = a.sys[w.x];
        dense_backward<DB, false, true>(a, sd, L, w.y);
        if (threadIdx.x == 0) L.misc[2] = load_status(&a.status[w.x]);
        __syncthreads();
        if (L.misc[2] != 0) {
            const int f0 = seg_first(sd, w.y);
            nan_fill<64>(a, sd, f0, f0 + seg_len(sd, w.y), false);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ recursive segmentation
// A nested system's reduced chain is handed to the child plan as an ordinary
// system: after phase 1, stage j of the chain (separator k = j + 2) has
//   D'_j = hat A_k partial (factor slot of the separator) - hat F_{k-1} hat F_{k-1}^T
//   B'_j = hat Q_k partial - hat G_{N_{k-1}, k-1} hat F_{k-1}^T
//   r'_j = separator rhs partial + (-hat F_{k-1} hat y_{N_{k-1}, k-1})
// (Eqs. 8c, 9d), the couplings hat H_k where phase 1 left them (read in place),
// corner' = sym(corner) + sum_k tilde R_k and r'_g = r_g + sum_k tilde y_{g,k}
// (Eqs. 8b, 9c, 10).  The child's solution is the separators' and g's part of x.
struct NestArgs {
    const int2 *pairs;     // (system, child system)
    const int2 *units;     // (pair, separator j; -1: corner and arrow rhs)
    const SysDesc *csys;   // child systems
    const int *cstatus;    // child per-system status
    double *cD, *cB, *cCor, *cR;
    // the child call's start (what its reset kernel would do): tag check, queue
    // heads, failure indices
    const long long *ctag;
    long long cexpect;
    int *cabort, *cctr, *cfail;
    int cnctr, cS;
};

// In thread t < E of a 256-thread workgroup: sum_{k < p} src[k * stride + t]
// (E <= 256).  Each element's k range is cut into 256 / E slices, each slice
// keeps eight loads in flight, and the slices meet in LDS.  Every thread calls it.
__device__ __forceinline__ double strided_sum(const double *src, long long stride, int p, int E, double *lds)
{
    if (E <= 0) return 0.0;
    const int t = threadIdx.x, KS = 256 / E, e = t % E, ks = t / E;
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (ks < KS) {
        int k = ks;
        for (; k + 7 * KS < p; k += 8 * KS) {
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] += src[(long long)(k + u * KS) * stride + e];
        }
        for (; k < p; k += KS) acc[0] += src[(long long)k * stride + e];
    }
    __syncthreads();
    lds[t] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    __syncthreads();
    double w = 0.0;
    if (t < E)
        for (int q = 0; q < KS; ++q) w += lds[q * E + t];
    __syncthreads();
    return w;
}

template <int MODE>
__global__ void __launch_bounds__(256) kkt_nest_gather(Args a, NestArgs na)
{
    constexpr bool FACT = MODE == M_FACTOR || MODE == M_FACTOR_SOLVE, RHS = MODE != M_FACTOR;
    __shared__ double red[256];
    if (blockIdx.x == 0) {
        // the start of the child's call (its reset kernel's work)
        const bool ok = na.ctag[0] == na.cexpect && *a.abort == 0;
        if (threadIdx.x == 0) *na.cabort = ok ? 0 : 1;
        if (ok) {
            for (int i = threadIdx.x; i < na.cnctr; i += 256) na.cctr[i] = 0;
            if (FACT)
                for (int i = threadIdx.x; i < na.cS; i += 256) na.cfail[i] = INT_MAX;
        }
    }
    if (*a.abort) return;
    const int2 u = na.units[blockIdx.x];
    const int2 pr = na.pairs[u.x];
    const SysDesc sd = a.sys[pr.x];
    const SysDesc cd = na.csys[pr.y];
    const int b = sd.b, ng = sd.ng, nr = a.nr, t = threadIdx.x;
    const long long b2 = (long long)b * b, gb = (long long)ng * b, rb = (long long)b * nr;
    const double *F = a.F;
    if (u.y >= 0) {
        const int j = u.y, sep = sep_of(sd, j + 2);
        const double *sc = F + sd.oScr + (long long)j * sd.scrStride;   // segment j + 1 ends on separator j + 2
        if (FACT) {
            const double *As = F + sd.oLd + sep * b2, *Qs = F + sd.oLb + sep * gb;
            double *Dc = na.cD + cd.oD + j * b2, *Bc = na.cB + cd.oB + j * gb;
            for (int e = t; e < b2; e += 256) Dc[e] = As[e] - sc[scr_dA(b, ng, nr) + e];
            for (int e = t; e < gb; e += 256) Bc[e] = Qs[e] - sc[scr_dQ(b, ng, nr) + e];
        }
        if (RHS) {
            const double *rs = a.rhs + sd.oRhs + sep * rb;
            double *Rc = na.cR + cd.oRhs + j * rb;
            for (int e = t; e < rb; e += 256) Rc[e] = rs[e] + sc[scr_dy(b, ng, nr) + e];
        }
    } else {
        const double *sc0 = F + sd.oScr;
        if (FACT) {
            const double *cor = a.corner + sd.oCorner;
            const double v = strided_sum(sc0 + scr_Rk(b, ng, nr), sd.scrStride, sd.p, ng * ng, red);
            if (t < ng * ng) {
                const int q = t / ng, c = t - q * ng;
                na.cCor[cd.oCorner + t] = 0.5 * (cor[t] + cor[c * ng + q]) + v;
            }
        }
        if (RHS) {
            const double *rg = a.rhs + sd.oRhs + (long long)sd.N * rb;
            double *Rc = na.cR + cd.oRhs + (long long)cd.N * rb;
            const double v = strided_sum(sc0 + scr_yg(b, ng, nr), sd.scrStride, sd.p, ng * nr, red);
            if (t < ng * nr) Rc[t] = rg[t] + v;
        }
    }
}

// After the child's call: the nested system's info (factor modes: its segments'
// first failure, else the child's failure mapped to the separator or corner it
// names), then (solve modes) the separators' and g's solution, NaN if the system
// failed, and with the adjoint their gradient blocks (dD, dB of the separators,
// dcorner) as the sequential sweep would write them.  One workgroup per system.
template <int MODE>
__global__ void __launch_bounds__(256) kkt_nest_finish(Args a, NestArgs na)
{
    constexpr bool FACT = MODE == M_FACTOR || MODE == M_FACTOR_SOLVE;
    if (*a.abort) return;
    const int2 pr = na.pairs[blockIdx.x];
    const SysDesc sd = a.sys[pr.x];
    const SysDesc cd = na.csys[pr.y];
    const int b = sd.b, ng = sd.ng, nr = a.nr, t = threadIdx.x, M = cd.N;
    const long long rb = (long long)b * nr;
    __shared__ int st;
    if (t == 0) {
        if (FACT) {
            const int segf = load_status(&a.failidx[pr.x]);
            const int c = load_status(&na.cstatus[pr.y]);
            const int v = segf != INT_MAX ? segf : (c == 0 ? 0 : (c <= M ? sep_of(sd, c + 1) + 1 : sd.N + 1));
            a.status[pr.x] = v;
            if (a.info) a.info[pr.x] = v;
            st = v;
        } else {
            st = load_status(&a.status[pr.x]);
        }
    }
    __syncthreads();
    if (MODE == M_FACTOR) return;
    const bool bad = st != 0;
    const double qnan = __longlong_as_double(0x7ff8000000000000LL);
    double *X = a.rhs + sd.oRhs;
    const double *Xc = na.cR + cd.oRhs;
    // every (separator, entry) pair at once: the loads are independent
    for (long long e = t; e < (long long)M * rb; e += 256) {
        const int j = (int)(e / rb);
        const long long r = e - (long long)j * rb;
        X[(long long)sep_of(sd, j + 2) * rb + r] = bad ? qnan : Xc[e];
    }
    const long long og = (long long)sd.N * rb, ocg = (long long)M * rb;
    for (int e = t; e < ng * nr; e += 256) X[og + e] = bad ? qnan : Xc[ocg + e];
    if (MODE != M_ADJOINT) return;
    // lambda (read from the child's solution) and the primal x
    const double *XP = a.xp + sd.oRhs;
    auto lam = [&](long long o) { return bad ? qnan : Xc[o]; };
    const long long b2 = (long long)b * b, gb = (long long)ng * b;
    for (long long e = t; e < (long long)M * b2; e += 256) {
        const int j = (int)(e / b2);
        const int rc = (int)(e - (long long)j * b2), r = rc / b, c = rc - r * b;
        const int sep = sep_of(sd, j + 2);
        const long long os = (long long)sep * rb, oc = (long long)j * rb;
        double v = 0.0;
        for (int q = 0; q < nr; ++q)
            v += lam(oc + r * nr + q) * XP[os + c * nr + q] + XP[os + r * nr + q] * lam(oc + c * nr + q);
        a.dD[sd.oD + sep * b2 + rc] = -0.5 * v;
    }
    for (long long e = t; e < (long long)M * gb; e += 256) {
        const int j = (int)(e / gb);
        const int gc = (int)(e - (long long)j * gb), g = gc / b, c = gc - g * b;
        const int sep = sep_of(sd, j + 2);
        const long long os = (long long)sep * rb, oc = (long long)j * rb;
        double v = 0.0;
        for (int q = 0; q < nr; ++q)
            v += lam(ocg + g * nr + q) * XP[os + c * nr + q] + XP[og + g * nr + q] * lam(oc + c * nr + q);
        a.dB[sd.oB + sep * gb + gc] = -v;
    }
    double *dR = a.dcorner + sd.oCorner;
    for (int e = t; e < ng * ng; e += 256) {
        const int g = e / ng, c = e - g * ng;
        double v = 0.0;
        for (int q = 0; q < nr; ++q)
            v += lam(ocg + g * nr + q) * XP[og + c * nr + q] + XP[og + g * nr + q] * lam(ocg + c * nr + q);
        dR[e] = -0.5 * v;
    }
}

typedef void (*nfun_t)(Args, NestArgs);

nfun_t nest_kernel(int mode, bool finish)
{
    switch (mode) {
    case M_FACTOR: return finish ? kkt_nest_finish<M_FACTOR> : kkt_nest_gather<M_FACTOR>;
    case M_FACTOR_SOLVE: return finish ? kkt_nest_finish<M_FACTOR_SOLVE> : kkt_nest_gather<M_FACTOR_SOLVE>;
    case M_SOLVE: return finish ? kkt_nest_finish<M_SOLVE> : kkt_nest_gather<M_SOLVE>;
    default: return finish ? kkt_nest_finish<M_ADJOINT> : kkt_nest_gather<M_ADJOINT>;
    }
}

// Start of every call: check that the workspace holds this plan's tables (a
// mismatch makes every later kernel of the call return at once and is reported
// by kkt_workspace_error), then clear the queue heads and the per-system failure
// indices of the call.  A kernel, not a memset, so the call can be captured.
__global__ void kkt_reset(const long long *tag, long long expect, int *abort, int *ctr, int nctr, int *failidx, int S,
                          int *info)
{
    const bool ok = tag[0] == expect;
    const int t = blockIdx.x * blockDim.x + threadIdx.x, st = gridDim.x * blockDim.x;
    if (t == 0) *abort = ok ? 0 : 1;
    if (!ok) return;
    for (int i = t; i < nctr; i += st) ctr[i] = 0;
    for (int i = t; i < S; i += st) {
        if (failidx) failidx[i] = INT_MAX;
        if (info) info[i] = 0;
    }
}

// ------------------------------------------------------------------ host plan
constexpr int NCLS = 5;
constexpr int CLS_BP[NCLS] = {8, 16, 24, 32, 48};

int class_of(int b)
{
    for (int c = 0; c < NCLS; ++c)
        if (b <= CLS_BP[c]) return c;
    return -1;
}

// Padded sizes 24 and 32 run the dense single-wave sweeps on 32-wide tiles; 8 and
// 16 the single-wave row-lane sweeps (measured faster for 16), 48 the multi-wave
// row-lane sweeps.
bool dense_capable(int bp) { return bp == 24 || bp == 32; }

template <int DB>
kfun_t dense_for(int mode)
{
    switch (mode) {
    case M_FACTOR: return kkt_dense<DB, M_FACTOR>;
    case M_FACTOR_SOLVE: return kkt_dense<DB, M_FACTOR_SOLVE>;
    case M_SOLVE: return kkt_dense<DB, M_SOLVE>;
    default: return kkt_dense<DB, M_ADJOINT>;
    }
}

// The launches of one class in one mode: kernel, threads, LDS bytes, and which
// work list sizes its grid (0 items, 1 reduced systems, 2 phase-3 segments).
struct Launch {
    kfun_t fn;
    int nt;
    size_t lds;
    int list;
};

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

// The reduced chain of M separators, swept sequentially (M t_red) or segmented
// recursively: at each level q segments balanced by Eq. 13 with the model's
// sigma, then the chain of their q - 1 separators, t_level per extra level.  The
// estimate keeps the shortest longest path; p[] holds the segment counts per
// level that reach it (0: sequential).
struct ChainEst {
    double longest = 0.0, total = 0.0;
    int p[KKT_MAX_LEVELS] = {};
};

struct ChainModel {
    const kkt_cost_model &m;
    int cls;
    std::map<std::pair<int, int>, ChainEst> memo;

    ChainModel(const kkt_cost_model &model, int c) : m(model), cls(c) {}

    ChainEst best(int M, int depth)
    {
        ChainEst serial;
        serial.longest = serial.total = M * m.t_red[cls];
        if (depth <= 0 || M < 3) return serial;
        const auto key = std::make_pair(M, depth);
        const auto it = memo.find(key);
        if (it != memo.end()) return it->second;
        ChainEst b = serial;
        for (int q = 2; 2 * q - 1 <= M; ++q) {
            int N1 = 0, Nk = 0;
            if (!partition_sigma(M, q, m.t_first[cls], m.t_fill[cls], &N1, &Nk)) continue;
            const double seg1 = m.t_item[cls] + N1 * m.t_first[cls], segk = m.t_item[cls] + Nk * m.t_fill[cls];
            const ChainEst sub = best(q - 1, depth - 1);
            const double lg = std::max(seg1, segk) + sub.longest + m.t_level[cls];
            if (lg < b.longest) {
                b.longest = lg;
                b.total = seg1 + (q - 1) * segk + sub.total + m.t_level[cls];
                b.p[0] = q;
                for (int l = 1; l < KKT_MAX_LEVELS; ++l) b.p[l] = sub.p[l - 1];
            }
        }
        memo[key] = b;
        return b;
    }
};

// Estimated longest item and total work of one system split into p segments,
// its reduced chain as cm chooses (sequential if cm is null); *nest receives the
// chain's segment counts.
ItemEst estimate(int N, int p, int cls, const kkt_cost_model &m, ChainModel *cm = nullptr, kkt_nest *nest = nullptr)
{
    int N1 = N, Nk = 0;
    if (p > 1 && !partition_sigma(N, p, m.t_first[cls], m.t_fill[cls], &N1, &Nk)) return {1e300, 1e300};
    const double seg1 = m.t_item[cls] + N1 * m.t_first[cls];
    const double segk = p > 1 ? m.t_item[cls] + Nk * m.t_fill[cls] : 0.0;
    ChainEst red;
    red.longest = red.total = (p - 1) * m.t_red[cls];
    if (cm && p > 1) red = cm->best(p - 1, KKT_MAX_LEVELS);
    if (nest)
        for (int l = 0; l < KKT_MAX_LEVELS; ++l) nest->p[l] = red.p[l];
    return {std::max(seg1, segk) + red.longest, seg1 + (p - 1) * segk + red.total};
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
void choose_segments(std::vector<kkt_dims> &dims, std::vector<kkt_nest> &nest, const std::vector<int> &cls_of,
                     const kkt_cost_model &m)
{
    std::vector<ChainModel> chains;
    for (int c = 0; c < NCLS; ++c) chains.emplace_back(m, c);
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
        const int pmax = std::max(1, std::min((N + 1) / 2, 1024));
        for (int p = 1; p <= pmax; ++p) {
            L.est.push_back(estimate(N, p, c, m, &chains[c]));
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
        estimate(dims[s].N, p, c, m, &chains[c], &nest[s]);
        // every level of the recursion is split with the balance the estimate assumed
        for (int l = 0, M = p - 1; l < KKT_MAX_LEVELS && nest[s].p[l] >= 2; M = nest[s].p[l] - 1, ++l) {
            int N1 = 0, Nk = 0;
            nest[s].N1[l] = partition_sigma(M, nest[s].p[l], m.t_first[c], m.t_fill[c], &N1, &Nk) ? N1 : 0;
        }
        int N1 = 0, Nk = 0;
        if (p > 1 && dims[s].N1 == 0 && partition_sigma(dims[s].N, p, m.t_first[c], m.t_fill[c], &N1, &Nk))
            dims[s].N1 = N1;
    }
}

kkt_cost_model default_cost_model()
{
    kkt_cost_model m;
    for (int c = 0; c < NCLS; ++c) {
        const double b3 = (double)CLS_BP[c] * CLS_BP[c] * CLS_BP[c];
        m.t_first[c] = 7.0 / 3.0 * b3;
        m.t_fill[c] = 19.0 / 3.0 * b3;
        m.t_red[c] = 10.0 / 3.0 * b3;
        m.t_item[c] = 0.0;
        m.workers[c] = 512.0;
        m.workers_seg[c] = 512.0;
        m.t_level[c] = 64.0 * m.t_first[c];
        m.family[c] = 0.0;
    }
    return m;
}

// Standard flop counts (potrf n^3/3, trsm m n^2, syrk n^2 k, gemm 2 m n k, matrix
// additions m n per term) of the operations of Algorithm 1 for one system with
// segment lengths N1, Nk (p segments): the parallel phase of every segment, then
// the sequential phase on the separators and the corner (seq false: without the
// sequential phase and the corner factor, which a segmented reduced chain counts).
double factor_flops_std(int N1, int Nk, int p, double b, double g, bool seq = true)
{
    const double potrf = b * b * b / 3.0, trsm = b * b * b, syrk = b * b * b, gemm = 2.0 * b * b * b;
    const double trsm_g = g * b * b, syrk_g = g * g * b, gemm_g = 2.0 * g * b * b;
    double f = 0.0;
    for (int k = 1; k <= p; ++k) {
        const int nk = k == 1 ? N1 : Nk;
        const double n = nk, inner = nk - 1;
        f += n * potrf + inner * (trsm + syrk);
        if (g > 0) f += n * (trsm_g + syrk_g) + inner * gemm_g;
        if (k > 1) {
            f += n * (trsm + syrk) + inner * gemm;
            if (g > 0) f += n * gemm_g;
        }
        if (k < p) f += trsm;
        if (k > 1 && k < p) f += gemm;
    }
    if (!seq) return f + (g > 0 ? g * g * p : 0.0);
    for (int k = 2; k <= p; ++k) {
        f += syrk + potrf;
        if (k < p) f += trsm + syrk;
        if (g > 0) {
            f += gemm_g + trsm_g + syrk_g;
            if (k < p) f += gemm_g;
        }
    }
    if (g > 0) f += g * g * p + g * g * g / 3.0;
    return f;
}

// The same for one solve with one right-hand side (trsv n^2, gemv 2 m n), Algorithms 2 and 3.
double solve_flops_std(int N1, int Nk, int p, double b, double g, bool seq = true)
{
    const double trsv = b * b, gemv = 2.0 * b * b, gemv_g = 2.0 * g * b;
    double f = 0.0;
    for (int k = 1; k <= p; ++k) {
        const double n = k == 1 ? N1 : Nk;
        // forward: trsv per stage, hat E y between stages, fill rows, arrow rows
        f += n * trsv + (n - 1) * gemv + (k > 1 ? n * gemv : 0.0) + (g > 0 ? n * gemv_g : 0.0);
        // backward: the same products transposed, and hat F_k^T x_{k+1}
        f += n * trsv + (n - 1) * gemv + (k > 1 ? n * gemv : 0.0) + (g > 0 ? n * gemv_g : 0.0) + (k < p ? gemv : 0.0);
    }
    if (!seq) return f + (g > 0 ? g * p : 0.0);
    for (int k = 2; k <= p; ++k) {
        f += gemv + 2 * trsv + (k < p ? 2 * gemv : 0.0) + (g > 0 ? 2 * gemv_g : 0.0);
    }
    if (g > 0) f += g * p + 2.0 * g * g;
    return f;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

std::atomic<long long> g_tag_counter{0};

long long new_plan_tag()
{
    static const long long seed =
        (long long)std::chrono::steady_clock::now().time_since_epoch().count() * 0x9E3779B97F4A7C15LL;
    const long long t = seed + (g_tag_counter.fetch_add(1) + 1) * 0x632BE59BD9B4E019LL;
    return t == 0 ? 1 : t;
}

}  // namespace

struct kkt_plan {
    enum { K_WAVE = 0, K_DENSE = 1, K_DSEG = 2 };
    int S = 0, nrhs = 1;
    std::vector<SysDesc> sys;
    std::vector<kkt_system_layout> lay;
    struct Cls {
        int cls = 0, bp = 0, kind = K_WAVE;
        int item_off = 0, item_cnt = 0, red_off = 0, red_cnt = 0, s3_off = 0, s3_cnt = 0;
    };
    std::vector<Cls> cls;
    std::vector<int2> items, s3;
    std::vector<int> red;
    size_t o_tag = 0, o_ctr = 0, o_sys = 0, o_items = 0, o_red = 0, o_s3 = 0, o_fail = 0, o_status = 0, o_F = 0,
           bytes = 0;
    // Recursive segmentation: the reduced chains of the nested systems form the
    // systems of a child plan, whose input pools (D, B, corner, rhs; C is read in
    // this plan's factor region) and workspace sit at the end of this workspace.
    kkt_plan *child = nullptr;
    std::vector<int2> npairs;   // (system, child system) per nested system
    std::vector<int2> nunits;   // gather units: (pair, separator j along the chain; -1 the corner)
    std::vector<int> child_of;  // per system: its child system or -1
    size_t o_npairs = 0, o_nunits = 0, o_cD = 0, o_cB = 0, o_cCor = 0, o_cR = 0, o_child = 0;
    long long nF = 0;
    long long tag = 0;
    kkt_plan_info info{};
    static constexpr int MAXC = 8, NSIDE = 3;
    // The launch state of one device, made by kkt_workspace_init so that factor
    // and solve calls make no device queries and create nothing (they can be
    // captured in a graph, first call included).  With several classes, the first
    // NSIDE active classes of a call run on streams of their own, forked from and
    // joined back into the caller's stream through events, and any further class
    // runs on the caller's stream itself.  HIP maps a process's streams onto 4
    // hardware queues by default; a fourth side stream would share a queue with
    // another side stream and run only after that stream's work, while the
    // caller's stream has a queue of its own.
    struct Dev {
        int dev = -1;
        bool needs_streams = false;   // several active classes; side streams made when fork is set
        hipStream_t side[NSIDE] = {};
        hipEvent_t fork = nullptr, join[NSIDE] = {};
        int grid[MAXC][4][3] = {};
    };
    // Host-side registry, guarded by mu (every call and kkt_workspace_init hold
    // the lock while they enqueue): the per-device launch state, the workspaces
    // initialised for this plan and their device, the workspaces holding a factor.
    mutable std::mutex mu;
    mutable std::vector<Dev> devs;
    mutable std::unordered_map<const void *, int> ws_dev;
    mutable std::unordered_set<const void *> factored;
    hipEvent_t ev_start[MAXC] = {}, ev_stop[MAXC] = {};

    const Dev *dev_state(int d) const
    {
        for (const Dev &x : devs)
            if (x.dev == d) return &x;
        return nullptr;
    }
    ~kkt_plan()
    {
        delete child;
        // teardown: a failure to destroy leaves nothing to recover, so it is ignored
        for (Dev &d : devs) {
            for (int j = 0; j < NSIDE; ++j) {
                if (d.side[j]) (void)hipStreamDestroy(d.side[j]);
                if (d.join[j]) (void)hipEventDestroy(d.join[j]);
            }
            if (d.fork) (void)hipEventDestroy(d.fork);
        }
    }
};

namespace {

bool valid_dims(const kkt_dims &d)
{
    if (d.N < 1 || d.b < 1 || d.b > KKT_MAX_B || d.ng < 0 || d.ng > KKT_MAX_NG) return false;
    if (d.p < 0) return false;
    if (d.p > 1 && d.N < 2 * d.p - 1) return false;
    return true;
}

// The recursion of a system of p segments: each level's chain long enough for
// its segment count (a count <= 1 ends it).
bool valid_nest(int p, const kkt_nest &n)
{
    int M = p - 1;
    for (int l = 0; l < KKT_MAX_LEVELS; ++l) {
        const int q = n.p[l];
        if (q < 0 || n.N1[l] < 0) return false;
        if (q <= 1) return true;
        if (M < 2 * q - 1) return false;
        if (n.N1[l] > 0) {
            const int rest = M - n.N1[l] - (q - 1);
            if (rest < q - 1 || rest % (q - 1) != 0) return false;
        }
        M = q - 1;
    }
    return true;
}

// Cost of one (system, segment) item in stage-steps weighted by block size: the
// LPT order only.
double item_cost(const SysDesc &s, int k)
{
    const double b = s.b < 8 ? 8.0 : (double)s.b;
    const int len = (k == 1) ? s.N1 : s.Nk;
    const double per = (k == 1) ? 1.0 : 2.5;
    return len * per * b * b * b + (s.p > 1 && k == s.p ? s.p * 3.0 * b * b * b : 0.0);
}

// The launches of one class in one mode (at most three).
int launches_of(const kkt_plan::Cls &c, int mode, int nr, Launch *out)
{
    const bool fact = mode == M_FACTOR || mode == M_FACTOR_SOLVE, fwd = mode == M_FACTOR_SOLVE;
    int n = 0;
    if (c.kind == kkt_plan::K_DENSE) {
        const size_t lds = (size_t)lds_offsets_dense(32, nr).total * sizeof(double);
        out[n++] = {dense_for<32>(mode), 64, lds, 0};
        if (mode != M_FACTOR) out[n++] = {mode == M_ADJOINT ? kkt_dense_bwd<32, true> : kkt_dense_bwd<32, false>, 64, lds, 0};
        return n;
    }
    const int wnt = wave_threads(c.bp);
    const size_t wl = wave_lds_bytes(c.bp);
    if (c.kind == kkt_plan::K_DSEG && fact) {
        const size_t lds = (size_t)lds_offsets_dense(32, nr, true).total * sizeof(double);
        out[n++] = {fwd ? kkt_dense_seg<32, true> : kkt_dense_seg<32, false>, 64, lds, 0};
        if (c.red_cnt > 0) out[n++] = {wave_kernel(c.bp, mode, 1, nr), wnt, wl, 1};
        if (fwd) out[n++] = {kkt_dense_seg_bwd<32>, 64, lds, 2};
        return n;
    }
    out[n++] = {wave_kernel(c.bp, mode, 0, nr), wnt, wl, 0};
    if (c.red_cnt > 0) out[n++] = {wave_kernel(c.bp, mode, 1, nr), wnt, wl, 1};
    if (c.s3_cnt > 0 && mode != M_FACTOR) out[n++] = {wave_kernel(c.bp, mode, 2, nr), wnt, wl, 2};
    return n;
}

int work_of(const kkt_plan::Cls &c, int list) { return list == 0 ? c.item_cnt : list == 1 ? c.red_cnt : c.s3_cnt; }

// The launch state of the current device: side streams and events, dynamic LDS
// limits and the grid of every launch (as many workgroups as fit on the device
// at once, at most one per work entry).  Called with the plan's lock held.
int ensure_device_one(const kkt_plan *plan, int dev, bool streams);

int ensure_device(const kkt_plan *plan, int dev, bool streams = true)
{
    int rc = ensure_device_one(plan, dev, streams);
    if (rc == KKT_OK && plan->child) rc = ensure_device(plan->child, dev, streams);
    return rc;
}

int ensure_device_one(const kkt_plan *plan, int dev, bool streams)
{
    if (const kkt_plan::Dev *have = plan->dev_state(dev)) {
        if (!streams || have->fork || !have->needs_streams) return KKT_OK;
        // made without side streams (by the no-allocation entry point): rebuild it with them
        for (size_t i = 0; i < plan->devs.size(); ++i)
            if (plan->devs[i].dev == dev) { plan->devs.erase(plan->devs.begin() + i); break; }
    }
    kkt_plan::Dev d;
    d.dev = dev;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
        return KKT_ELAUNCH;
    int nact = 0;
    for (const kkt_plan::Cls &c : plan->cls) nact += c.item_cnt > 0;
    bool ok = true;
    d.needs_streams = nact > 1;
    if (nact > 1 && streams) {
        ok = hipEventCreateWithFlags(&d.fork, hipEventDisableTiming) == hipSuccess;
        for (int j = 0; ok && j < kkt_plan::NSIDE && j < nact; ++j) {
            ok = hipStreamCreateWithFlags(&d.side[j], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&d.join[j], hipEventDisableTiming) == hipSuccess;
        }
    }
    for (size_t ci = 0; ok && ci < plan->cls.size(); ++ci) {
        for (int mode = 0; ok && mode < 4; ++mode) {
            Launch L[3];
            const int n = launches_of(plan->cls[ci], mode, plan->nrhs, L);
            for (int l = 0; ok && l < n; ++l) {
                if (L[l].lds > 65536 && hipFuncSetAttribute((const void *)L[l].fn,
                                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                                            (int)L[l].lds) != hipSuccess) {
                    ok = false;
                    break;
                }
                int occ = 0;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)L[l].fn, L[l].nt, L[l].lds) !=
                        hipSuccess ||
                    occ < 1)
                    occ = 1;
                d.grid[ci][mode][l] = std::max(1, std::min(work_of(plan->cls[ci], L[l].list), occ * ncu));
            }
        }
    }
    if (!ok) {
        for (int j = 0; j < kkt_plan::NSIDE; ++j) {
            if (d.side[j]) (void)hipStreamDestroy(d.side[j]);
            if (d.join[j]) (void)hipEventDestroy(d.join[j]);
        }
        if (d.fork) (void)hipEventDestroy(d.fork);
        return KKT_ELAUNCH;
    }
    plan->devs.push_back(d);
    return KKT_OK;
}

// ------------------------------------------------------------------ no-allocation entry point
// Device memory of the no-allocation entry point: one array per device, held
// until the process ends.  In host code `scratch` names a host-side stand-in; the
// device address comes from hipGetSymbolAddress, once per device, and only that
// address is ever passed to kernels or copies.
constexpr size_t NOALLOC_BYTES = (size_t)KKT_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAXDEV = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[NOALLOC_MAXDEV] = {};
long long g_noalloc_owner[NOALLOC_MAXDEV] = {};   // tag of the plan whose tables the array holds

// The array's device address on device dev (the current device); null on failure.
void *noalloc_scratch(int dev)
{
    if (dev < 0 || dev >= NOALLOC_MAXDEV) return nullptr;
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_noalloc_ptr[dev] = ptr;
    }
    return g_noalloc_ptr[dev];
}

// Copy a plan's tables (and its child's, into its sub-workspace) into a
// workspace; with zero_status also clear the per-system status words.
bool put_tables(const kkt_plan *plan, char *ws, hipStream_t stream, bool zero_status)
{
    auto put = [&](size_t off, const void *src, size_t n) {
        return n == 0 || hipMemcpyAsync(ws + off, src, n, hipMemcpyHostToDevice, stream) == hipSuccess;
    };
    const long long tag[3] = {plan->tag, (long long)plan->bytes, 0};
    if (!put(plan->o_sys, plan->sys.data(), sizeof(SysDesc) * plan->S) ||
        !put(plan->o_items, plan->items.data(), sizeof(int2) * plan->items.size()) ||
        !put(plan->o_red, plan->red.data(), sizeof(int) * plan->red.size()) ||
        !put(plan->o_s3, plan->s3.data(), sizeof(int2) * plan->s3.size()) || !put(plan->o_tag, tag, sizeof(tag)))
        return false;
    if (zero_status) {
        std::vector<int> st(plan->S, 0);
        if (!put(plan->o_status, st.data(), sizeof(int) * plan->S)) return false;
        // the copy must not outlive st
        if (hipStreamSynchronize(stream) != hipSuccess) return false;
    }
    if (plan->child) {
        if (!put(plan->o_npairs, plan->npairs.data(), sizeof(int2) * plan->npairs.size()) ||
            !put(plan->o_nunits, plan->nunits.data(), sizeof(int2) * plan->nunits.size()))
            return false;
        return put_tables(plan->child, ws + plan->o_child, stream, zero_status);
    }
    return true;
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
    a.s3 = (const int2 *)(ws + plan->o_s3);
    a.ctr = (int *)(ws + plan->o_ctr);
    a.abort = (const int *)(ws + plan->o_tag + 16);
    a.failidx = (int *)(ws + plan->o_fail);
    a.status = (int *)(ws + plan->o_status);
    a.nr = plan->nrhs;
    return a;
}

// Enqueue one call: the reset kernel, then every class's launches (classes on
// forked streams when there are several).  On an error after the fork, the side
// streams used so far are still joined back into the caller's stream.
int launch_locked(const kkt_plan *plan, const kkt_plan::Dev *d, int mode, const Args &base, const void *ws,
                  hipStream_t stream, int *info, bool allow_fork, bool reset = true);

int launch_mode(const kkt_plan *plan, int mode, const Args &base, const void *ws, hipStream_t stream, int *info,
                bool need_factor)
{
    std::lock_guard<std::mutex> guard(plan->mu);
    const auto wit = plan->ws_dev.find(ws);
    if (wit == plan->ws_dev.end()) return KKT_EWORKSPACE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return KKT_ELAUNCH;
    if (wit->second != dev) return KKT_EWORKSPACE;
    if (need_factor && plan->factored.count(ws) == 0) return KKT_ENOTFACTORED;
    const kkt_plan::Dev *d = plan->dev_state(dev);
    if (!d) return KKT_EWORKSPACE;
    return launch_locked(plan, d, mode, base, ws, stream, info, true);
}

// The launches of every class whose work list is in lists (bit l: list l), the
// classes on forked streams when there are several, joined back into stream.  On
// an error after the fork, the side streams used so far are still joined.
int enqueue_classes(const kkt_plan *plan, const kkt_plan::Dev *d, int mode, const Args &base, hipStream_t stream,
                    bool allow_fork, int lists, bool rec_start, bool rec_stop)
{
    Launch L[kkt_plan::MAXC][3];
    int n[kkt_plan::MAXC] = {}, nact = 0;
    for (size_t ci = 0; ci < plan->cls.size(); ++ci) {
        const kkt_plan::Cls &c = plan->cls[ci];
        n[ci] = c.item_cnt > 0 ? launches_of(c, mode, plan->nrhs, L[ci]) : 0;
        bool any = false;
        for (int l = 0; l < n[ci]; ++l) any |= ((lists >> L[ci][l].list) & 1) != 0;
        if (!any) n[ci] = 0;
        nact += n[ci] > 0;
    }
    const bool fork = allow_fork && nact > 1 && d->fork;
    if (fork && hipEventRecord(d->fork, stream) != hipSuccess) return KKT_ELAUNCH;
    int rc = KKT_OK, nside = 0;
    for (size_t ci = 0; ci < plan->cls.size() && rc == KKT_OK; ++ci) {
        const kkt_plan::Cls &c = plan->cls[ci];
        if (n[ci] == 0) continue;
        const bool on_side = fork && nside < kkt_plan::NSIDE;
        hipStream_t st = on_side ? d->side[nside] : stream;
        if (on_side && hipStreamWaitEvent(st, d->fork, 0) != hipSuccess) {
            rc = KKT_ELAUNCH;
            break;
        }
        Args a = base;
        a.items = base.items + c.item_off;
        a.n_items = c.item_cnt;
        a.red = base.red + c.red_off;
        a.n_red = c.red_cnt;
        a.s3 = base.s3 + c.s3_off;
        a.n_s3 = c.s3_cnt;
        a.ctr = base.ctr + 4 * ci;
        if (rec_start && plan->ev_start[ci] && hipEventRecord(plan->ev_start[ci], st) != hipSuccess) rc = KKT_ELAUNCH;
        for (int l = 0; l < n[ci] && rc == KKT_OK; ++l) {
            if (((lists >> L[ci][l].list) & 1) == 0) continue;
            hipLaunchKernelGGL(L[ci][l].fn, dim3(d->grid[ci][mode][l]), dim3(L[ci][l].nt), L[ci][l].lds, st, a);
            if (hipGetLastError() != hipSuccess) rc = KKT_ELAUNCH;
        }
        if (rc == KKT_OK && rec_stop && plan->ev_stop[ci] && hipEventRecord(plan->ev_stop[ci], st) != hipSuccess)
            rc = KKT_ELAUNCH;
        if (on_side) {
            if (hipEventRecord(d->join[nside], st) != hipSuccess) rc = KKT_ELAUNCH;
            ++nside;
        }
    }
    // the caller's stream waits for the side streams only after its own classes are
    // queued, so that those run beside the side streams
    for (int j = 0; j < nside; ++j)
        if (hipStreamWaitEvent(stream, d->join[j], 0) != hipSuccess) rc = KKT_ELAUNCH;
    return rc;
}

// Enqueue one call with the plan's lock held and its launch state d of the current
// device.  Without reduced chains to segment, each class runs its phases back to
// back on its stream.  Otherwise every class runs phases 1 and 2, then on the
// caller's stream the nested systems' chains are gathered, the child plan makes
// its own call (recursively) and the results are scattered back, and then every
// class runs phase 3.
int launch_locked(const kkt_plan *plan, const kkt_plan::Dev *d, int mode, const Args &base, const void *ws,
                  hipStream_t stream, int *info, bool allow_fork, bool reset)
{
    const bool fact = mode == M_FACTOR || mode == M_FACTOR_SOLVE;
    const char *w = (const char *)ws;
    if (reset) {
        hipLaunchKernelGGL(kkt_reset, dim3(std::max(1, std::min(1024, (plan->S + 255) / 256))), dim3(256), 0, stream,
                           (const long long *)(w + plan->o_tag), plan->tag, (int *)(w + plan->o_tag + 16), base.ctr,
                           4 * (int)plan->cls.size(), fact ? base.failidx : nullptr, plan->S, fact ? info : nullptr);
        if (hipGetLastError() != hipSuccess) return KKT_ELAUNCH;
    }
    if (!plan->child) return enqueue_classes(plan, d, mode, base, stream, allow_fork, 7, true, true);
    int rc = enqueue_classes(plan, d, mode, base, stream, allow_fork, 3, true, false);
    if (rc != KKT_OK) return rc;
    const kkt_plan *ch = plan->child;
    const kkt_plan::Dev *cdv = ch->dev_state(d->dev);
    if (!cdv) return KKT_EWORKSPACE;
    char *cw = (char *)ws + plan->o_child;
    NestArgs na;
    na.pairs = (const int2 *)(w + plan->o_npairs);
    na.units = (const int2 *)(w + plan->o_nunits);
    na.csys = (const SysDesc *)(cw + ch->o_sys);
    na.cstatus = (const int *)(cw + ch->o_status);
    na.cD = (double *)(w + plan->o_cD);
    na.cB = (double *)(w + plan->o_cB);
    na.cCor = (double *)(w + plan->o_cCor);
    na.cR = (double *)(w + plan->o_cR);
    na.ctag = (const long long *)(cw + ch->o_tag);
    na.cexpect = ch->tag;
    na.cabort = (int *)(cw + ch->o_tag + 16);
    na.cctr = (int *)(cw + ch->o_ctr);
    na.cnctr = 4 * (int)ch->cls.size();
    na.cfail = (int *)(cw + ch->o_fail);
    na.cS = ch->S;
    hipLaunchKernelGGL(nest_kernel(mode, false), dim3((unsigned)plan->nunits.size()), dim3(256), 0, stream, base, na);
    if (hipGetLastError() != hipSuccess) return KKT_ELAUNCH;
    Args ca = base_args(ch, cw);
    ca.D = na.cD;
    ca.C = base.F;   // the couplings hat H_k, in place (child offsets point there)
    ca.B = na.cB;
    ca.corner = na.cCor;
    ca.rhs = mode != M_FACTOR ? na.cR : nullptr;
    // the gather kernel has done the child's reset
    rc = launch_locked(ch, cdv, mode == M_ADJOINT ? M_SOLVE : mode, ca, cw, stream, nullptr, allow_fork, false);
    if (rc != KKT_OK) return rc;
    hipLaunchKernelGGL(nest_kernel(mode, true), dim3((unsigned)plan->npairs.size()), dim3(256), 0, stream, base, na);
    if (hipGetLastError() != hipSuccess) return KKT_ELAUNCH;
    return enqueue_classes(plan, d, mode, base, stream, allow_fork, 4, false, true);
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
    return kkt_plan_create_nested(out, S, dims_in, nullptr, nrhs, model);
}

int kkt_plan_create_nested(kkt_plan **out, int32_t S, const kkt_dims *dims_in, const kkt_nest *nest_in,
                           int32_t nrhs, const kkt_cost_model *model)
{
    if (!out) return KKT_EPOINTER;
    *out = nullptr;
    if (S < 1 || !dims_in) return S < 1 ? KKT_EDIMS : KKT_EPOINTER;
    if (nrhs < 1 || nrhs > KKT_MAX_NRHS) return KKT_EDIMS;
    std::vector<kkt_dims> dims(dims_in, dims_in + S);
    std::vector<kkt_nest> nest(S);
    std::memset(nest.data(), 0, sizeof(kkt_nest) * S);
    const kkt_cost_model m = model ? *model : default_cost_model();
    {
        std::vector<int> cls0(S);
        for (int s = 0; s < S; ++s) {
            if (!valid_dims(dims[s])) return KKT_EDIMS;
            cls0[s] = class_of(dims[s].b);
            if (dims[s].p != 0 && nest_in) {
                nest[s] = nest_in[s];
                if (!valid_nest(dims[s].p, nest[s])) return KKT_EDIMS;
            }
        }
        choose_segments(dims, nest, cls0, m);
    }
    kkt_plan *P = new (std::nothrow) kkt_plan;
    if (!P) return KKT_EINTERNAL;
    P->S = S;
    P->nrhs = nrhs;
    P->tag = new_plan_tag();
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
        const bool seq = !(p >= 2 && nest[s].p[0] >= 2);
        fflops += factor_flops_std(N1, Nk, p, (double)b, (double)ng, seq);
        sflops += nrhs * solve_flops_std(N1, Nk, p, (double)b, (double)ng, seq);
        fwords += N * b2 + (N - 1) * b2 + N * ng * b + ng * ng + fill + H;
        iwords += N * b2 + (N - 1) * b2 + N * ng * b + ng * ng;
    }
    P->nF = oF;
    // classes: per block-size class the whole systems of the 16/24/32 groups (dense
    // sweeps), then everything else (segmented dense-group systems; all systems of
    // the 8 and 48 groups); items longest first (LPT) inside a class
    // the sweep family of each class: the dense sweeps where they exist, unless the
    // cost model chose the row-lane sweeps (family 2)
    bool dense_ok[NCLS];
    for (int c = 0; c < NCLS; ++c) dense_ok[c] = dense_capable(CLS_BP[c]) && m.family[c] != 2.0;
    for (int cc = 0; cc < 2 * NCLS; ++cc) {
        const int c = cc >> 1, bp = CLS_BP[c];
        const bool dense = (cc & 1) == 0;
        if (dense && !dense_ok[c]) continue;
        std::vector<std::pair<double, int2>> its;
        std::vector<int> reds;
        for (int s = 0; s < S; ++s) {
            if (cls_of[s] != c) continue;
            const SysDesc &sd = P->sys[s];
            if (dense_ok[c] && (sd.p == 1) != dense) continue;
            for (int k = 1; k <= sd.p; ++k) its.push_back({item_cost(sd, k), make_int2(s, k)});
            if (sd.p > 1 && nest[s].p[0] < 2) reds.push_back(s);
        }
        if (its.empty()) continue;
        std::stable_sort(its.begin(), its.end(), [](const std::pair<double, int2> &x, const std::pair<double, int2> &y) {
            return x.first > y.first;
        });
        kkt_plan::Cls C;
        C.cls = c;
        C.bp = bp;
        C.kind = dense ? kkt_plan::K_DENSE : (dense_ok[c] ? kkt_plan::K_DSEG : kkt_plan::K_WAVE);
        C.item_off = (int)P->items.size();
        C.item_cnt = (int)its.size();
        C.red_off = (int)P->red.size();
        C.red_cnt = (int)reds.size();
        C.s3_off = (int)P->s3.size();
        for (auto &x : its) {
            P->items.push_back(x.second);
            if (P->sys[x.second.x].p > 1) P->s3.push_back(x.second);
        }
        C.s3_cnt = (int)P->s3.size() - C.s3_off;
        for (int s : reds) P->red.push_back(s);
        if ((int)P->cls.size() >= kkt_plan::MAXC) { delete P; return KKT_EINTERNAL; }
        P->cls.push_back(C);
    }
    // the reduced chains of the nested systems: the child plan (recursively)
    P->child_of.assign(S, -1);
    {
        std::vector<kkt_dims> cdims;
        std::vector<kkt_nest> cnest;
        for (int s = 0; s < S; ++s) {
            const SysDesc &sd = P->sys[s];
            if (sd.p < 2 || nest[s].p[0] < 2) continue;
            kkt_dims cd;
            cd.N = sd.p - 1; cd.b = sd.b; cd.ng = sd.ng; cd.p = nest[s].p[0]; cd.N1 = nest[s].N1[0];
            kkt_nest cn;
            std::memset(&cn, 0, sizeof(cn));
            for (int l = 1; l < KKT_MAX_LEVELS; ++l) {
                cn.p[l - 1] = nest[s].p[l];
                cn.N1[l - 1] = nest[s].N1[l];
            }
            P->child_of[s] = (int)cdims.size();
            P->npairs.push_back(make_int2(s, (int)cdims.size()));
            cdims.push_back(cd);
            cnest.push_back(cn);
        }
        if (!cdims.empty()) {
            kkt_plan *ch = nullptr;
            const int rc = kkt_plan_create_nested(&ch, (int)cdims.size(), cdims.data(), cnest.data(), nrhs, model);
            if (rc != KKT_OK) { delete P; return rc; }
            P->child = ch;
            for (size_t i = 0; i < P->npairs.size(); ++i) {
                const int2 pr = P->npairs[i];
                // the chain's couplings hat H_k are read where phase 1 leaves them
                ch->sys[pr.y].oC = P->sys[pr.x].oH;
                ch->lay[pr.y].off_C = P->sys[pr.x].oH;
                for (int j = 0; j < P->sys[pr.x].p - 1; ++j) P->nunits.push_back(make_int2((int)i, j));
                P->nunits.push_back(make_int2((int)i, -1));
            }
            fflops += ch->info.factor_flops;
            sflops += ch->info.solve_flops;
            fwords += ch->info.factor_words;
        }
    }
    // workspace layout: tag (plan tag, size, refusal word), queue heads, tables, factor
    size_t o = 0;
    P->o_tag = o; o = align256(o + 24);
    P->o_ctr = o; o = align256(o + sizeof(int) * 4 * P->cls.size());
    P->o_sys = o; o = align256(o + sizeof(SysDesc) * S);
    P->o_items = o; o = align256(o + sizeof(int2) * std::max<size_t>(1, P->items.size()));
    P->o_red = o; o = align256(o + sizeof(int) * std::max<size_t>(1, P->red.size()));
    P->o_s3 = o; o = align256(o + sizeof(int2) * std::max<size_t>(1, P->s3.size()));
    P->o_fail = o; o = align256(o + sizeof(int) * S);
    P->o_status = o; o = align256(o + sizeof(int) * S);
    P->o_F = o; o = align256(o + sizeof(double) * (size_t)oF);
    if (P->child) {
        const kkt_plan *ch = P->child;
        P->o_npairs = o; o = align256(o + sizeof(int2) * P->npairs.size());
        P->o_nunits = o; o = align256(o + sizeof(int2) * P->nunits.size());
        P->o_cD = o; o = align256(o + sizeof(double) * (size_t)ch->info.D_len);
        P->o_cB = o; o = align256(o + sizeof(double) * (size_t)ch->info.B_len);
        P->o_cCor = o; o = align256(o + sizeof(double) * (size_t)ch->info.corner_len);
        P->o_cR = o; o = align256(o + sizeof(double) * (size_t)ch->info.rhs_len);
        P->o_child = o; o = align256(o + ch->bytes);
    }
    P->bytes = o;
    kkt_plan_info &I = P->info;
    I.num_systems = S;
    I.nrhs = nrhs;
    I.num_items = (int)P->items.size();
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

int kkt_plan_reduced(const kkt_plan *plan, int32_t s, const kkt_plan **child, int32_t *child_system,
                     int64_t *workspace_offset)
{
    if (!plan || !child || !child_system || !workspace_offset) return KKT_EPOINTER;
    if (s < 0 || s >= plan->S) return KKT_EDIMS;
    const int cs = plan->child_of[s];
    *child = cs >= 0 ? plan->child : nullptr;
    *child_system = cs;
    *workspace_offset = cs >= 0 ? (int64_t)plan->o_child : -1;
    return KKT_OK;
}

int64_t kkt_plan_factor_offset(const kkt_plan *plan) { return plan ? (int64_t)plan->o_F : -1; }

int kkt_workspace_init(const kkt_plan *plan, void *workspace, hipStream_t stream)
{
    if (!plan || !workspace) return KKT_EPOINTER;
    if (((uintptr_t)workspace & 255) != 0) return KKT_EPOINTER;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return KKT_ELAUNCH;
    std::lock_guard<std::mutex> guard(plan->mu);
    const int rc = ensure_device(plan, dev);
    if (rc != KKT_OK) return rc;
    if (!put_tables(plan, (char *)workspace, stream, true) || hipStreamSynchronize(stream) != hipSuccess)
        return KKT_ELAUNCH;
    plan->ws_dev[workspace] = dev;
    plan->factored.erase(workspace);
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
    const int rc = launch_mode(plan, M_FACTOR, a, workspace, stream, info, false);
    if (rc == KKT_OK) {
        std::lock_guard<std::mutex> guard(plan->mu);
        plan->factored.insert(workspace);
    }
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
    const int rc = launch_mode(plan, M_FACTOR_SOLVE, a, workspace, stream, info, false);
    if (rc == KKT_OK) {
        std::lock_guard<std::mutex> guard(plan->mu);
        plan->factored.insert(workspace);
    }
    return rc;
}

int kkt_factor_solve_noalloc(const kkt_plan *plan, const double *D, const double *C, const double *B,
                             const double *corner, double *rhs, int32_t *info, hipStream_t stream)
{
    if (!plan || !D || !info || !rhs) return KKT_EPOINTER;
    if (plan->info.C_len && !C) return KKT_EPOINTER;
    if (plan->info.B_len && (!B || !corner)) return KKT_EPOINTER;
    if (!aligned8(D) || !aligned8(C) || !aligned8(B) || !aligned8(corner) || !aligned8(rhs)) return KKT_EPOINTER;
    if (plan->bytes > NOALLOC_BYTES) return KKT_EWORKSPACE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return KKT_ELAUNCH;
    std::lock_guard<std::mutex> nguard(g_noalloc_mu);
    void *ws = noalloc_scratch(dev);
    if (!ws) return KKT_ELAUNCH;
    std::lock_guard<std::mutex> guard(plan->mu);
    int rc = ensure_device(plan, dev, false);
    if (rc != KKT_OK) return rc;
    if (g_noalloc_owner[dev] != plan->tag) {
        // the array last held another plan's tables (or none): copy this plan's in
        if (!put_tables(plan, (char *)ws, stream, false)) return KKT_ELAUNCH;
        g_noalloc_owner[dev] = plan->tag;
    }
    Args a = base_args(plan, ws);
    a.D = D; a.C = C; a.B = B; a.corner = corner; a.info = info; a.rhs = rhs;
    return launch_locked(plan, plan->dev_state(dev), M_FACTOR_SOLVE, a, ws, stream, info, false);
}

int kkt_solve(const kkt_plan *plan, void *workspace, double *rhs, hipStream_t stream)
{
    if (!plan || !workspace || !rhs) return KKT_EPOINTER;
    if (((uintptr_t)workspace & 255) || !aligned8(rhs)) return KKT_EPOINTER;
    Args a = base_args(plan, workspace);
    a.rhs = rhs;
    return launch_mode(plan, M_SOLVE, a, workspace, stream, nullptr, true);
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
    Args a = base_args(plan, workspace);
    a.rhs = gx; a.xp = x; a.dD = dD; a.dC = dC; a.dB = dB; a.dcorner = dcorner;
    return launch_mode(plan, M_ADJOINT, a, workspace, stream, nullptr, true);
}

int kkt_workspace_error(const kkt_plan *plan, const void *workspace, hipStream_t stream, int32_t *flag)
{
    if (!plan || !workspace || !flag) return KKT_EPOINTER;
    int refused = 0;
    if (hipMemcpyAsync(&refused, (const char *)workspace + plan->o_tag + 16, sizeof(int), hipMemcpyDeviceToHost,
                       stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return KKT_ELAUNCH;
    *flag = refused ? KKT_WS_FOREIGN : 0;
    return KKT_OK;
}

int kkt_plan_class_info(const kkt_plan *plan, int32_t c, int32_t *block_pad, int32_t *num_items,
                        int32_t *threads, int64_t *lds_bytes, int32_t *grid)
{
    if (!plan) return KKT_EPOINTER;
    if (c < 0 || c >= (int)plan->cls.size()) return KKT_EDIMS;
    const kkt_plan::Cls &C = plan->cls[c];
    Launch L[3];
    launches_of(C, M_FACTOR_SOLVE, plan->nrhs, L);
    if (block_pad) *block_pad = C.bp;
    if (num_items) *num_items = C.item_cnt;
    if (threads) *threads = L[0].nt;
    if (lds_bytes) *lds_bytes = (int64_t)L[0].lds;
    if (grid) {
        std::lock_guard<std::mutex> guard(plan->mu);
        int dev = 0;
        const kkt_plan::Dev *d = hipGetDevice(&dev) == hipSuccess ? plan->dev_state(dev) : nullptr;
        *grid = d ? d->grid[c][M_FACTOR_SOLVE][0] : 0;
    }
    return KKT_OK;
}

int kkt_plan_class_kind(const kkt_plan *plan, int32_t c, int32_t *kind)
{
    if (!plan || !kind) return KKT_EPOINTER;
    if (c < 0 || c >= (int)plan->cls.size()) return KKT_EDIMS;
    const kkt_plan::Cls &C = plan->cls[c];
    *kind = C.kind == kkt_plan::K_DENSE ? KKT_CLASS_DENSE
                                        : C.kind == kkt_plan::K_DSEG ? KKT_CLASS_DENSE_SEGMENTED : KKT_CLASS_ROWLANE;
    return KKT_OK;
}

int kkt_plan_set_class_events(kkt_plan *plan, int32_t c, hipEvent_t start, hipEvent_t stop)
{
    if (!plan) return KKT_EPOINTER;
    if (c < 0 || c >= (int)plan->cls.size()) return KKT_EDIMS;
    std::lock_guard<std::mutex> guard(plan->mu);
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
    case KKT_EWORKSPACE: return "workspace not initialised for this plan on this device";
    case KKT_ELAUNCH: return "HIP launch error";
    case KKT_ENOTFACTORED: return "solve before factorization in this workspace";
    case KKT_EINTERNAL: return "internal error";
    default: return "unknown status";
    }
}

}  // extern "C"
