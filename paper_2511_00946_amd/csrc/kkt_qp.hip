// KKT systems of a multistage QP (Sec. 2, Eq. 1) on top of the plan's layouts:
// assembly of Psi = P + rho I + A^T A / delta + G^T W G into the plan's D, C, B and
// corner pools, the reduced right-hand side rx + A^T ry / delta + G^T W rz, and the
// recovery of dy = (A dx - ry) / delta and dz = W (G dx - rz) -- the block
// elimination of the proximal interior-point Newton system (the reading documented
// in kkt.h).  Built on the public C ABI only (the plan's layouts).
//
// Stage i of a system touches constraint groups i (on x_i, x_{i+1}, g) and i - 1
// (on x_{i-1}, x_i, g).  One 256-thread workgroup per (system, stage) stages the
// rows of both groups in LDS and forms every output entry of its stage as a dot
// product over those rows; the sums over all groups (the corner, the g rows of the
// rhs) go through per-stage partials that a second kernel adds up per system.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "kkt.h"

namespace {

struct QpSys {
    long long oD, oC, oB, oCor, oR;                        // the plan's pools (doubles)
    long long oEL, oER, oEG, oIL, oIR, oIG, ow, oy, oz;    // QP pools (doubles)
    long long oPart;                                       // scratch partials
    int N, b, ng, pe, me, nr;
};

struct QpPtr {
    const double *Q, *S, *T, *Qg, *EL, *ER, *EG, *IL, *IR, *IG, *w;
};

// Largest block shapes of the plan: they size the LDS areas.
struct QpMax {
    int P, M, B, G, R;   // rows of a group (equality, inequality), b, ng, rhs columns
};

// LDS areas of one stage: group i (EL, ER, EG, IL, IR, IG, w) and group i - 1
// (ERp, EGp, IRp, IGp, wp), the rows of ry and rz of both groups, and the three
// parts of dx (x_i, x_{i+1}, g).
struct StageLds {
    double *EL, *ER, *EG, *IL, *IR, *IG, *w, *ERp, *EGp, *IRp, *IGp, *wp;
    double *ry, *ryp, *rz, *rzp, *xi, *xn, *xg;
};

__host__ __device__ inline size_t stage_lds_doubles(const QpMax &m)
{
    const size_t PB = (size_t)m.P * m.B, PG = (size_t)m.P * m.G, MB = (size_t)m.M * m.B, MG = (size_t)m.M * m.G;
    return 3 * PB + 2 * PG + 3 * MB + 2 * MG + 2 * (size_t)m.M + 2 * (size_t)m.P * m.R + 2 * (size_t)m.M * m.R +
           2 * (size_t)m.B * m.R + (size_t)m.G * m.R;
}

__device__ inline StageLds carve(double *p, const QpMax &m)
{
    StageLds L;
    const int PB = m.P * m.B, PG = m.P * m.G, MB = m.M * m.B, MG = m.M * m.G;
    L.EL = p; p += PB;
    L.ER = p; p += PB;
    L.ERp = p; p += PB;
    L.EG = p; p += PG;
    L.EGp = p; p += PG;
    L.IL = p; p += MB;
    L.IR = p; p += MB;
    L.IRp = p; p += MB;
    L.IG = p; p += MG;
    L.IGp = p; p += MG;
    L.w = p; p += m.M;
    L.wp = p; p += m.M;
    L.ry = p; p += m.P * m.R;
    L.ryp = p; p += m.P * m.R;
    L.rz = p; p += m.M * m.R;
    L.rzp = p; p += m.M * m.R;
    L.xi = p; p += m.B * m.R;
    L.xn = p; p += m.B * m.R;
    L.xg = p;
    return L;
}

// n doubles from src into dst (zeros when the block does not exist: src is then
// never read).
__device__ inline void stage(double *dst, const double *src, int n, bool have)
{
    for (int e = threadIdx.x; e < n; e += 256) dst[e] = have ? src[e] : 0.0;
}

// The constraint rows of group i on x_i and g (and their weights), with nextg its
// rows on x_{i+1}, with prevg group i - 1's rows on x_i and g, into LDS.
__device__ inline void stage_rows(const StageLds &L, const QpPtr &d, const QpSys &q, int i, bool nextg, bool prevg)
{
    const int b = q.b, ng = q.ng, pe = q.pe, me = q.me;
    const bool nx = i + 1 < q.N, pv = i > 0;
    const long long pb = (long long)pe * b, pg = (long long)pe * ng, mb = (long long)me * b, mg = (long long)me * ng;
    stage(L.EL, d.EL + q.oEL + i * pb, pe * b, true);
    stage(L.EG, d.EG + q.oEG + i * pg, pe * ng, true);
    stage(L.IL, d.IL + q.oIL + i * mb, me * b, true);
    stage(L.IG, d.IG + q.oIG + i * mg, me * ng, true);
    stage(L.w, d.w + q.ow + (long long)i * me, me, true);
    if (nextg) {
        stage(L.ER, d.ER + q.oER + i * pb, pe * b, nx);
        stage(L.IR, d.IR + q.oIR + i * mb, me * b, nx);
    }
    if (prevg) {
        stage(L.ERp, d.ER + q.oER + (i - 1) * pb, pe * b, pv);
        stage(L.EGp, d.EG + q.oEG + (i - 1) * pg, pe * ng, pv);
        stage(L.IRp, d.IR + q.oIR + (i - 1) * mb, me * b, pv);
        stage(L.IGp, d.IG + q.oIG + (i - 1) * mg, me * ng, pv);
        stage(L.wp, d.w + q.ow + (long long)(i - 1) * me, me, pv);
    }
}

// Psi's blocks of stage i: D_i, C_i (i < N - 1), B_i, and group i's part of the corner.
__global__ void __launch_bounds__(256) qp_assemble_k(const QpSys *sys, const int2 *units, QpPtr d, QpMax mx,
                                                     double rho, double rdelta, double *D, double *C, double *B,
                                                     double *part)
{
    extern __shared__ double lds[];
    const StageLds L = carve(lds, mx);
    const int2 u = units[blockIdx.x];
    const QpSys q = sys[u.x];
    const int i = u.y, b = q.b, ng = q.ng, pe = q.pe, me = q.me, t = threadIdx.x;
    stage_rows(L, d, q, i, true, true);
    __syncthreads();
    const long long b2 = (long long)b * b;
    for (int e = t; e < b * b; e += 256) {
        const int r = e / b, c = e - r * b;
        double se = 0.0, si = 0.0;
        for (int k = 0; k < pe; ++k) se += L.EL[k * b + r] * L.EL[k * b + c] + L.ERp[k * b + r] * L.ERp[k * b + c];
        for (int k = 0; k < me; ++k)
            si += L.w[k] * L.IL[k * b + r] * L.IL[k * b + c] + L.wp[k] * L.IRp[k * b + r] * L.IRp[k * b + c];
        const long long o = q.oD + i * b2 + e;
        D[o] = d.Q[o] + (r == c ? rho : 0.0) + se * rdelta + si;
    }
    if (i + 1 < q.N) {
        for (int e = t; e < b * b; e += 256) {
            const int r = e / b, c = e - r * b;   // r: a variable of stage i + 1, c: of stage i
            double se = 0.0, si = 0.0;
            for (int k = 0; k < pe; ++k) se += L.ER[k * b + r] * L.EL[k * b + c];
            for (int k = 0; k < me; ++k) si += L.w[k] * L.IR[k * b + r] * L.IL[k * b + c];
            const long long o = q.oC + i * b2 + e;
            C[o] = d.S[o] + se * rdelta + si;
        }
    }
    for (int e = t; e < ng * b; e += 256) {
        const int g = e / b, c = e - g * b;
        double se = 0.0, si = 0.0;
        for (int k = 0; k < pe; ++k) se += L.EG[k * ng + g] * L.EL[k * b + c] + L.EGp[k * ng + g] * L.ERp[k * b + c];
        for (int k = 0; k < me; ++k)
            si += L.w[k] * L.IG[k * ng + g] * L.IL[k * b + c] + L.wp[k] * L.IGp[k * ng + g] * L.IRp[k * b + c];
        const long long o = q.oB + (long long)i * ng * b + e;
        B[o] = d.T[o] + se * rdelta + si;
    }
    for (int e = t; e < ng * ng; e += 256) {
        const int g1 = e / ng, g2 = e - g1 * ng;
        double se = 0.0, si = 0.0;
        for (int k = 0; k < pe; ++k) se += L.EG[k * ng + g1] * L.EG[k * ng + g2];
        for (int k = 0; k < me; ++k) si += L.w[k] * L.IG[k * ng + g1] * L.IG[k * ng + g2];
        part[q.oPart + (long long)i * ng * ng + e] = se * rdelta + si;
    }
}

// In thread t < E of a 256-thread workgroup: sum_{k < n} src[k * stride + t] (E <=
// 256), the k range split over 256 / E slices with eight loads in flight each.
__device__ inline double slice_sum(const double *src, long long stride, int n, int E, double *red)
{
    const int t = threadIdx.x, KS = 256 / E, e = t % E, ks = t / E;
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (ks < KS) {
        int k = ks;
        for (; k + 7 * KS < n; k += 8 * KS) {
#pragma unroll
            for (int v = 0; v < 8; ++v) acc[v] += src[(long long)(k + v * KS) * stride + e];
        }
        for (; k < n; k += KS) acc[0] += src[(long long)k * stride + e];
    }
    red[t] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    __syncthreads();
    double s = 0.0;
    if (t < E)
        for (int v = 0; v < KS; ++v) s += red[v * E + t];
    return s;
}

// corner = Qg + rho I + sum of the groups' partials (one workgroup per system).
__global__ void __launch_bounds__(256) qp_corner_k(const QpSys *sys, QpPtr d, double rho, double *corner,
                                                   const double *part)
{
    __shared__ double red[256];
    const QpSys q = sys[blockIdx.x];
    const int ng = q.ng, E = ng * ng, t = threadIdx.x;
    if (E == 0) return;
    const double s = slice_sum(part + q.oPart, E, q.N, E, red);
    if (t < E) {
        const long long o = q.oCor + t;
        corner[o] = d.Qg[o] + ((t / ng) == (t % ng) ? rho : 0.0) + s;
    }
}

// The reduced rhs of stage i, and group i's part of its g rows.
__global__ void __launch_bounds__(256) qp_rhs_k(const QpSys *sys, const int2 *units, QpPtr d, QpMax mx, double rdelta,
                                                const double *rx, const double *ry, const double *rz, double *rhs,
                                                double *part)
{
    extern __shared__ double lds[];
    const StageLds L = carve(lds, mx);
    const int2 u = units[blockIdx.x];
    const QpSys q = sys[u.x];
    const int i = u.y, b = q.b, ng = q.ng, pe = q.pe, me = q.me, nr = q.nr, t = threadIdx.x;
    const bool pv = i > 0;
    stage_rows(L, d, q, i, false, true);
    stage(L.ry, ry + q.oy + (long long)i * pe * nr, pe * nr, true);
    stage(L.rz, rz + q.oz + (long long)i * me * nr, me * nr, true);
    stage(L.ryp, ry + q.oy + (long long)(i - 1) * pe * nr, pe * nr, pv);
    stage(L.rzp, rz + q.oz + (long long)(i - 1) * me * nr, me * nr, pv);
    __syncthreads();
    for (int e = t; e < b * nr; e += 256) {
        const int r = e / nr, j = e - r * nr;
        double se = 0.0, si = 0.0;
        for (int k = 0; k < pe; ++k) se += L.EL[k * b + r] * L.ry[k * nr + j] + L.ERp[k * b + r] * L.ryp[k * nr + j];
        for (int k = 0; k < me; ++k)
            si += L.IL[k * b + r] * L.w[k] * L.rz[k * nr + j] + L.IRp[k * b + r] * L.wp[k] * L.rzp[k * nr + j];
        const long long o = q.oR + (long long)i * b * nr + e;
        rhs[o] = rx[o] + se * rdelta + si;
    }
    for (int e = t; e < ng * nr; e += 256) {
        const int g = e / nr, j = e - g * nr;
        double se = 0.0, si = 0.0;
        for (int k = 0; k < pe; ++k) se += L.EG[k * ng + g] * L.ry[k * nr + j];
        for (int k = 0; k < me; ++k) si += L.IG[k * ng + g] * L.w[k] * L.rz[k * nr + j];
        part[q.oPart + (long long)i * ng * nr + e] = se * rdelta + si;
    }
}

// The g rows of the reduced rhs (one workgroup per system).
__global__ void __launch_bounds__(256) qp_rhs_g_k(const QpSys *sys, const double *rx, double *rhs, const double *part)
{
    __shared__ double red[256];
    const QpSys q = sys[blockIdx.x];
    const int E = q.ng * q.nr, t = threadIdx.x;
    if (E == 0) return;
    const double s = slice_sum(part + q.oPart, E, q.N, E, red);
    if (t < E) {
        const long long o = q.oR + (long long)q.N * q.b * q.nr + t;
        rhs[o] = rx[o] + s;
    }
}

// dy and dz of constraint group i.
__global__ void __launch_bounds__(256) qp_recover_k(const QpSys *sys, const int2 *units, QpPtr d, QpMax mx,
                                                    double rdelta, const double *dx, const double *ry,
                                                    const double *rz, double *dy, double *dz)
{
    extern __shared__ double lds[];
    const StageLds L = carve(lds, mx);
    const int2 u = units[blockIdx.x];
    const QpSys q = sys[u.x];
    const int i = u.y, b = q.b, ng = q.ng, pe = q.pe, me = q.me, nr = q.nr, t = threadIdx.x;
    const bool nx = i + 1 < q.N;
    stage_rows(L, d, q, i, true, false);
    const long long rb = (long long)b * nr;
    stage(L.xi, dx + q.oR + i * rb, b * nr, true);
    stage(L.xn, dx + q.oR + (i + 1) * rb, b * nr, nx);
    stage(L.xg, dx + q.oR + (long long)q.N * rb, ng * nr, true);
    __syncthreads();
    for (int e = t; e < pe * nr; e += 256) {
        const int k = e / nr, j = e - k * nr;
        double s = 0.0;
        for (int c = 0; c < b; ++c) s += L.EL[k * b + c] * L.xi[c * nr + j] + L.ER[k * b + c] * L.xn[c * nr + j];
        for (int g = 0; g < ng; ++g) s += L.EG[k * ng + g] * L.xg[g * nr + j];
        const long long o = q.oy + (long long)i * pe * nr + e;
        dy[o] = (s - ry[o]) * rdelta;
    }
    for (int e = t; e < me * nr; e += 256) {
        const int k = e / nr, j = e - k * nr;
        double s = 0.0;
        for (int c = 0; c < b; ++c) s += L.IL[k * b + c] * L.xi[c * nr + j] + L.IR[k * b + c] * L.xn[c * nr + j];
        for (int g = 0; g < ng; ++g) s += L.IG[k * ng + g] * L.xg[g * nr + j];
        const long long o = q.oz + (long long)i * me * nr + e;
        dz[o] = L.w[k] * (s - rz[o]);
    }
}

bool aligned8(const void *p) { return ((uintptr_t)p & 7) == 0; }

}  // namespace

struct kkt_qp {
    int S = 0, nunits = 0;
    QpSys *dsys = nullptr;
    int2 *dunits = nullptr;
    double *dpart = nullptr;
    std::vector<QpSys> hsys;
    long long len[9] = {};
    QpMax mx{0, 0, 0, 0, 0};
    size_t lds = 0;
    ~kkt_qp()
    {
        // teardown: nothing to recover from a failure
        if (dsys) (void)hipFree(dsys);
        if (dunits) (void)hipFree(dunits);
        if (dpart) (void)hipFree(dpart);
    }
};

namespace {

QpPtr ptrs(const kkt_qp_data *d)
{
    return QpPtr{d->Q, d->S, d->T, d->Qg, d->EL, d->ER, d->EG, d->IL, d->IR, d->IG, d->w};
}

// The data pointers a call needs: the cost pools only for the assembly; every
// non-empty pool must be given and 8-byte aligned.
bool data_ok(const kkt_qp *qp, const kkt_qp_data *d, bool cost, long long Dlen, long long Clen, long long Blen,
             long long Corlen)
{
    if (!d) return false;
    const void *need[] = {d->EL, d->ER, d->EG, d->IL, d->IR, d->IG, d->w};
    const long long lens[] = {qp->len[0], qp->len[1], qp->len[2], qp->len[3], qp->len[4], qp->len[5], qp->len[6]};
    for (int k = 0; k < 7; ++k)
        if ((lens[k] && !need[k]) || !aligned8(need[k])) return false;
    if (cost) {
        const void *c[] = {d->Q, d->S, d->T, d->Qg};
        const long long cl[] = {Dlen, Clen, Blen, Corlen};
        for (int k = 0; k < 4; ++k)
            if ((cl[k] && !c[k]) || !aligned8(c[k])) return false;
    }
    return true;
}

int set_lds(const void *fn, size_t lds)
{
    if (lds > 65536 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return KKT_ELAUNCH;
    return KKT_OK;
}

}  // namespace

extern "C" {

int kkt_qp_create(const kkt_plan *plan, const int32_t *n_eq, const int32_t *n_in, kkt_qp **out)
{
    if (!plan || !n_eq || !n_in || !out) return KKT_EPOINTER;
    *out = nullptr;
    kkt_plan_info info;
    int rc = kkt_plan_get_info(plan, &info);
    if (rc != KKT_OK) return rc;
    const int S = info.num_systems, nr = info.nrhs;
    for (int s = 0; s < S; ++s)
        if (n_eq[s] < 0 || n_eq[s] > KKT_QP_MAX_ROWS || n_in[s] < 0 || n_in[s] > KKT_QP_MAX_ROWS) return KKT_EDIMS;
    std::vector<QpSys> sys(S);
    std::vector<int2> units;
    long long o[9] = {}, oP = 0;
    QpMax mx{1, 1, 1, 1, nr};
    for (int s = 0; s < S; ++s) {
        kkt_system_layout L;
        rc = kkt_plan_system(plan, s, &L);
        if (rc != KKT_OK) return rc;
        QpSys &q = sys[s];
        const long long N = L.N, b = L.b, ng = L.ng, pe = n_eq[s], me = n_in[s];
        q.N = L.N; q.b = L.b; q.ng = L.ng; q.pe = n_eq[s]; q.me = n_in[s]; q.nr = nr;
        q.oD = L.off_D; q.oC = L.off_C; q.oB = L.off_B; q.oCor = L.off_corner; q.oR = L.off_rhs;
        q.oEL = o[0]; o[0] += N * pe * b;
        q.oER = o[1]; o[1] += (N - 1) * pe * b;
        q.oEG = o[2]; o[2] += N * pe * ng;
        q.oIL = o[3]; o[3] += N * me * b;
        q.oIR = o[4]; o[4] += (N - 1) * me * b;
        q.oIG = o[5]; o[5] += N * me * ng;
        q.ow = o[6]; o[6] += N * me;
        q.oy = o[7]; o[7] += N * pe * nr;
        q.oz = o[8]; o[8] += N * me * nr;
        q.oPart = oP; oP += N * std::max(ng * ng, ng * (long long)nr);
        for (int i = 0; i < L.N; ++i) units.push_back(make_int2(s, i));
        mx.P = std::max(mx.P, q.pe); mx.M = std::max(mx.M, q.me);
        mx.B = std::max(mx.B, q.b); mx.G = std::max(mx.G, q.ng);
    }
    kkt_qp *qp = new (std::nothrow) kkt_qp;
    if (!qp) return KKT_EINTERNAL;
    qp->S = S;
    qp->nunits = (int)units.size();
    qp->hsys = sys;
    for (int k = 0; k < 9; ++k) qp->len[k] = o[k];
    qp->mx = mx;
    qp->lds = stage_lds_doubles(mx) * sizeof(double);
    if (qp->lds > 160 * 1024) { delete qp; return KKT_EDIMS; }
    const bool ok = hipMalloc((void **)&qp->dsys, sizeof(QpSys) * S) == hipSuccess &&
                    hipMalloc((void **)&qp->dunits, sizeof(int2) * units.size()) == hipSuccess &&
                    hipMalloc((void **)&qp->dpart, sizeof(double) * std::max(1LL, oP)) == hipSuccess &&
                    hipMemcpy(qp->dsys, sys.data(), sizeof(QpSys) * S, hipMemcpyHostToDevice) == hipSuccess &&
                    hipMemcpy(qp->dunits, units.data(), sizeof(int2) * units.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok || set_lds((const void *)qp_assemble_k, qp->lds) != KKT_OK ||
        set_lds((const void *)qp_rhs_k, qp->lds) != KKT_OK || set_lds((const void *)qp_recover_k, qp->lds) != KKT_OK) {
        delete qp;
        return KKT_ELAUNCH;
    }
    *out = qp;
    return KKT_OK;
}

int kkt_qp_destroy(kkt_qp *qp)
{
    delete qp;
    return KKT_OK;
}

int kkt_qp_lengths(const kkt_qp *qp, int64_t *EL_len, int64_t *ER_len, int64_t *EG_len, int64_t *IL_len,
                   int64_t *IR_len, int64_t *IG_len, int64_t *w_len, int64_t *ry_len, int64_t *rz_len)
{
    if (!qp) return KKT_EPOINTER;
    int64_t *outs[9] = {EL_len, ER_len, EG_len, IL_len, IR_len, IG_len, w_len, ry_len, rz_len};
    for (int k = 0; k < 9; ++k)
        if (outs[k]) *outs[k] = qp->len[k];
    return KKT_OK;
}

int kkt_qp_offsets(const kkt_qp *qp, int32_t s, int64_t offsets[9])
{
    if (!qp || !offsets) return KKT_EPOINTER;
    if (s < 0 || s >= qp->S) return KKT_EDIMS;
    const QpSys &q = qp->hsys[s];
    const long long v[9] = {q.oEL, q.oER, q.oEG, q.oIL, q.oIR, q.oIG, q.ow, q.oy, q.oz};
    for (int k = 0; k < 9; ++k) offsets[k] = v[k];
    return KKT_OK;
}

int kkt_qp_assemble(const kkt_qp *qp, const kkt_qp_data *data, double rho, double delta, double *D, double *C,
                    double *B, double *corner, hipStream_t stream)
{
    if (!qp || !D) return KKT_EPOINTER;
    if (!(delta > 0.0) || !(rho >= 0.0)) return KKT_EDIMS;
    long long Dl = 0, Cl = 0, Bl = 0, Col = 0;
    for (const QpSys &q : qp->hsys) {
        Dl += (long long)q.N * q.b * q.b;
        Cl += (long long)(q.N - 1) * q.b * q.b;
        Bl += (long long)q.N * q.ng * q.b;
        Col += (long long)q.ng * q.ng;
    }
    if (!data_ok(qp, data, true, Dl, Cl, Bl, Col)) return KKT_EPOINTER;
    if ((Cl && !C) || (Bl && !B) || (Col && !corner) || !aligned8(D) || !aligned8(C) || !aligned8(B) ||
        !aligned8(corner))
        return KKT_EPOINTER;
    if (qp->nunits == 0) return KKT_OK;
    const QpPtr d = ptrs(data);
    hipLaunchKernelGGL(qp_assemble_k, dim3(qp->nunits), dim3(256), qp->lds, stream, qp->dsys, qp->dunits, d, qp->mx,
                       rho, 1.0 / delta, D, C, B, qp->dpart);
    if (hipGetLastError() != hipSuccess) return KKT_ELAUNCH;
    if (Col) {
        hipLaunchKernelGGL(qp_corner_k, dim3(qp->S), dim3(256), 0, stream, qp->dsys, d, rho, corner, qp->dpart);
        if (hipGetLastError() != hipSuccess) return KKT_ELAUNCH;
    }
    return KKT_OK;
}

int kkt_qp_reduce_rhs(const kkt_qp *qp, const kkt_qp_data *data, double delta, const double *rx, const double *ry,
                      const double *rz, double *rhs, hipStream_t stream)
{
    if (!qp || !rx || !rhs) return KKT_EPOINTER;
    if (!(delta > 0.0)) return KKT_EDIMS;
    if (!data_ok(qp, data, false, 0, 0, 0, 0)) return KKT_EPOINTER;
    if ((qp->len[7] && !ry) || (qp->len[8] && !rz) || !aligned8(rx) || !aligned8(ry) || !aligned8(rz) ||
        !aligned8(rhs))
        return KKT_EPOINTER;
    if (qp->nunits == 0) return KKT_OK;
    const QpPtr d = ptrs(data);
    hipLaunchKernelGGL(qp_rhs_k, dim3(qp->nunits), dim3(256), qp->lds, stream, qp->dsys, qp->dunits, d, qp->mx,
                       1.0 / delta, rx, ry, rz, rhs, qp->dpart);
    if (hipGetLastError() != hipSuccess) return KKT_ELAUNCH;
    hipLaunchKernelGGL(qp_rhs_g_k, dim3(qp->S), dim3(256), 0, stream, qp->dsys, rx, rhs, qp->dpart);
    return hipGetLastError() == hipSuccess ? KKT_OK : KKT_ELAUNCH;
}

int kkt_qp_recover(const kkt_qp *qp, const kkt_qp_data *data, double delta, const double *dx, const double *ry,
                   const double *rz, double *dy, double *dz, hipStream_t stream)
{
    if (!qp || !dx) return KKT_EPOINTER;
    if (!(delta > 0.0)) return KKT_EDIMS;
    if (!data_ok(qp, data, false, 0, 0, 0, 0)) return KKT_EPOINTER;
    if ((qp->len[7] && (!ry || !dy)) || (qp->len[8] && (!rz || !dz)) || !aligned8(dx) || !aligned8(ry) ||
        !aligned8(rz) || !aligned8(dy) || !aligned8(dz))
        return KKT_EPOINTER;
    if (qp->nunits == 0) return KKT_OK;
    hipLaunchKernelGGL(qp_recover_k, dim3(qp->nunits), dim3(256), qp->lds, stream, qp->dsys, qp->dunits, ptrs(data),
                       qp->mx, 1.0 / delta, dx, ry, rz, dy, dz);
    return hipGetLastError() == hipSuccess ? KKT_OK : KKT_ELAUNCH;
}

}  // extern "C"
