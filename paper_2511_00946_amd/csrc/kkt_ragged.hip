// Non-uniform stage sizes (paper Sec. 2, Eqs. 1 and 3: stage i has its own size
// n_i) on top of the uniform-block path: every stage is embedded in the plan's
// padded block size b >= n_i with the identity on the padded diagonal and zeros
// in the padded rows and columns of the coupling and arrow blocks.  The padded
// variables are then decoupled from the rest of the system, their solution is
// zero, and the real entries of the padded solution are the solution of the
// non-uniform system: the padding is exact.  Built on the public C ABI only (the
// plan's layouts); one workgroup per stage copies its blocks.
#include <hip/hip_runtime.h>

#include <new>
#include <vector>

#include "kkt.h"

namespace {

// One stage of one system: offsets (doubles) of its blocks in the non-uniform
// pools (r*) and in the plan's padded pools (p*); the first stage of a system
// also carries its corner and the arrow part of the rhs (rco >= 0).
struct RagUnit {
    long long rD, rC, rB, rR, pD, pC, pB, pR;
    long long rco, pco, rg, pg;
    int n, nn, b, ng;
};

__global__ void __launch_bounds__(256) kkt_ragged_pad_k(const RagUnit *U, int nr, const double *D, const double *C,
                                                        const double *B, const double *corner, const double *rhs,
                                                        double *Dp, double *Cp, double *Bp, double *cornerp,
                                                        double *rhsp)
{
    const RagUnit u = U[blockIdx.x];
    const int t = threadIdx.x, b = u.b, n = u.n, nn = u.nn, ng = u.ng;
    for (int e = t; e < b * b; e += 256) {
        const int r = e / b, c = e - r * b;
        const bool in = r < n && c < n;
        Dp[u.pD + e] = in ? D[u.rD + r * n + c] : (r == c ? 1.0 : 0.0);
        if (nn > 0) {
            const bool ic = r < nn && c < n;   // C_i is n_{i+1} x n_i
            Cp[u.pC + e] = ic ? C[u.rC + r * n + c] : 0.0;
        }
    }
    for (int e = t; e < ng * b; e += 256) {
        const int q = e / b, c = e - q * b;
        Bp[u.pB + e] = c < n ? B[u.rB + q * n + c] : 0.0;
    }
    for (int e = t; e < b * nr; e += 256) rhsp[u.pR + e] = e < n * nr ? rhs[u.rR + e] : 0.0;
    if (u.rco >= 0) {
        for (int e = t; e < ng * ng; e += 256) cornerp[u.pco + e] = corner[u.rco + e];
        for (int e = t; e < ng * nr; e += 256) rhsp[u.pg + e] = rhs[u.rg + e];
    }
}

__global__ void __launch_bounds__(256) kkt_ragged_unpad_k(const RagUnit *U, int nr, const double *xp, double *x)
{
    const RagUnit u = U[blockIdx.x];
    const int t = threadIdx.x;
    for (int e = t; e < u.n * nr; e += 256) x[u.rR + e] = xp[u.pR + e];
    if (u.rco >= 0)
        for (int e = t; e < u.ng * nr; e += 256) x[u.rg + e] = xp[u.pg + e];
}

bool aligned8(const void *p) { return ((uintptr_t)p & 7) == 0; }

}  // namespace

struct kkt_ragged {
    int units = 0, nrhs = 0;
    RagUnit *dU = nullptr;
    long long len[5] = {};   // non-uniform pools: D, C, B, corner, rhs (doubles)
    ~kkt_ragged()
    {
        if (dU) (void)hipFree(dU);   // teardown: nothing to recover from a failure
    }
};

extern "C" {

int kkt_ragged_create(const kkt_plan *plan, const int32_t *stage_sizes, kkt_ragged **out)
{
    if (!plan || !stage_sizes || !out) return KKT_EPOINTER;
    *out = nullptr;
    kkt_plan_info info;
    int rc = kkt_plan_get_info(plan, &info);
    if (rc != KKT_OK) return rc;
    const int nr = info.nrhs;
    std::vector<RagUnit> U;
    long long oD = 0, oC = 0, oB = 0, oCo = 0, oR = 0;
    size_t k = 0;
    for (int s = 0; s < info.num_systems; ++s) {
        kkt_system_layout L;
        rc = kkt_plan_system(plan, s, &L);
        if (rc != KKT_OK) return rc;
        const int N = L.N, b = L.b, ng = L.ng;
        const int32_t *n = stage_sizes + k;
        k += (size_t)N;
        for (int i = 0; i < N; ++i)
            if (n[i] < 1 || n[i] > b) return KKT_EDIMS;
        const size_t first = U.size();
        for (int i = 0; i < N; ++i) {
            RagUnit u;
            u.n = n[i];
            u.nn = i + 1 < N ? n[i + 1] : 0;
            u.b = b;
            u.ng = ng;
            u.rD = oD; oD += (long long)n[i] * n[i];
            u.pD = L.off_D + (long long)i * b * b;
            u.rC = oC; u.pC = L.off_C + (long long)i * b * b;
            if (i + 1 < N) oC += (long long)n[i + 1] * n[i];
            u.rB = oB; oB += (long long)ng * n[i];
            u.pB = L.off_B + (long long)i * ng * b;
            u.rR = oR; oR += (long long)n[i] * nr;
            u.pR = L.off_rhs + (long long)i * b * nr;
            u.rco = u.pco = u.rg = u.pg = -1;
            U.push_back(u);
        }
        RagUnit &u0 = U[first];
        u0.rco = oCo; u0.pco = L.off_corner; oCo += (long long)ng * ng;
        u0.rg = oR; u0.pg = L.off_rhs + (long long)N * b * nr; oR += (long long)ng * nr;
    }
    kkt_ragged *r = new (std::nothrow) kkt_ragged;
    if (!r) return KKT_EINTERNAL;
    r->units = (int)U.size();
    r->nrhs = nr;
    r->len[0] = oD; r->len[1] = oC; r->len[2] = oB; r->len[3] = oCo; r->len[4] = oR;
    if (!U.empty()) {
        if (hipMalloc((void **)&r->dU, sizeof(RagUnit) * U.size()) != hipSuccess) {
            r->dU = nullptr;
            delete r;
            return KKT_ELAUNCH;
        }
        if (hipMemcpy(r->dU, U.data(), sizeof(RagUnit) * U.size(), hipMemcpyHostToDevice) != hipSuccess) {
            delete r;
            return KKT_ELAUNCH;
        }
    }
    *out = r;
    return KKT_OK;
}

int kkt_ragged_destroy(kkt_ragged *r)
{
    delete r;
    return KKT_OK;
}

int kkt_ragged_lengths(const kkt_ragged *r, int64_t *D_len, int64_t *C_len, int64_t *B_len, int64_t *corner_len,
                       int64_t *rhs_len)
{
    if (!r) return KKT_EPOINTER;
    if (D_len) *D_len = r->len[0];
    if (C_len) *C_len = r->len[1];
    if (B_len) *B_len = r->len[2];
    if (corner_len) *corner_len = r->len[3];
    if (rhs_len) *rhs_len = r->len[4];
    return KKT_OK;
}

int kkt_ragged_pad(const kkt_ragged *r, const double *D, const double *C, const double *B, const double *corner,
                   const double *rhs, double *Dp, double *Cp, double *Bp, double *cornerp, double *rhsp,
                   hipStream_t stream)
{
    if (!r || !D || !rhs || !Dp || !rhsp) return KKT_EPOINTER;
    if ((r->len[1] && (!C || !Cp)) || (r->len[2] && (!B || !Bp)) || (r->len[3] && (!corner || !cornerp)))
        return KKT_EPOINTER;
    const void *ps[] = {D, C, B, corner, rhs, Dp, Cp, Bp, cornerp, rhsp};
    for (const void *p : ps)
        if (!aligned8(p)) return KKT_EPOINTER;
    if (r->units == 0) return KKT_OK;
    kkt_ragged_pad_k<<<r->units, 256, 0, stream>>>(r->dU, r->nrhs, D, C, B, corner, rhs, Dp, Cp, Bp, cornerp, rhsp);
    return hipGetLastError() == hipSuccess ? KKT_OK : KKT_ELAUNCH;
}

int kkt_ragged_unpad(const kkt_ragged *r, const double *xp, double *x, hipStream_t stream)
{
    if (!r || !xp || !x) return KKT_EPOINTER;
    if (!aligned8(xp) || !aligned8(x)) return KKT_EPOINTER;
    if (r->units == 0) return KKT_OK;
    kkt_ragged_unpad_k<<<r->units, 256, 0, stream>>>(r->dU, r->nrhs, xp, x);
    return hipGetLastError() == hipSuccess ? KKT_OK : KKT_ELAUNCH;
}

}  // extern "C"
