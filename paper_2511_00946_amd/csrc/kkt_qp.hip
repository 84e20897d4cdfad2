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
#include <cmath>
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
    double *ry, *ryp, *rz, *rzp, *xi, *xn, *xg, *xp;
};

__host__ __device__ inline size_t stage_lds_doubles(const QpMax &m)
{
    const size_t PB = (size_t)m.P * m.B, PG = (size_t)m.P * m.G, MB = (size_t)m.M * m.B, MG = (size_t)m.M * m.G;
    return 3 * PB + 2 * PG + 3 * MB + 2 * MG + 2 * (size_t)m.M + 2 * (size_t)m.P * m.R + 2 * (size_t)m.M * m.R +
           3 * (size_t)m.B * m.R + (size_t)m.G * m.R;
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
    L.xp = p; p += m.B * m.R;
    L.xg = p;
    return L;
}

// n doubles from src into dst (zeros when the block does not exist: src is then
// never read).
template <int NT>
__device__ inline void stage(double *dst, const double *src, int n, bool have)
{
    for (int e = threadIdx.x; e < n; e += NT) dst[e] = have ? src[e] : 0.0;
}

// The constraint rows of group i on x_i and g (and their weights), with nextg its
// rows on x_{i+1}, with prevg group i - 1's rows on x_i and g, into LDS.
template <int NT>
__device__ inline void stage_rows(const StageLds &L, const QpPtr &d, const QpSys &q, int i, bool nextg, bool prevg)
{
    const int b = q.b, ng = q.ng, pe = q.pe, me = q.me;
    const bool nx = i + 1 < q.N, pv = i > 0;
    const long long pb = (long long)pe * b, pg = (long long)pe * ng, mb = (long long)me * b, mg = (long long)me * ng;
    stage<NT>(L.EL, d.EL + q.oEL + i * pb, pe * b, true);
    stage<NT>(L.EG, d.EG + q.oEG + i * pg, pe * ng, true);
    stage<NT>(L.IL, d.IL + q.oIL + i * mb, me * b, true);
    stage<NT>(L.IG, d.IG + q.oIG + i * mg, me * ng, true);
    stage<NT>(L.w, d.w + q.ow + (long long)i * me, me, true);
    if (nextg) {
        stage<NT>(L.ER, d.ER + q.oER + i * pb, pe * b, nx);
        stage<NT>(L.IR, d.IR + q.oIR + i * mb, me * b, nx);
    }
    if (prevg) {
        stage<NT>(L.ERp, d.ER + q.oER + (i - 1) * pb, pe * b, pv);
        stage<NT>(L.EGp, d.EG + q.oEG + (i - 1) * pg, pe * ng, pv);
        stage<NT>(L.IRp, d.IR + q.oIR + (i - 1) * mb, me * b, pv);
        stage<NT>(L.IGp, d.IG + q.oIG + (i - 1) * mg, me * ng, pv);
        stage<NT>(L.wp, d.w + q.ow + (long long)(i - 1) * me, me, pv);
    }
}

// Psi's blocks of stage i: D_i, C_i (i < N - 1), B_i, and group i's part of the corner.
template <int NT>
__global__ void __launch_bounds__(NT) qp_assemble_k(const QpSys *sys, const int2 *units, QpPtr d, QpMax mx,
                                                     double rho, double rdelta, double *D, double *C, double *B,
                                                     double *part)
{
    extern __shared__ double lds[];
    const StageLds L = carve(lds, mx);
    const int2 u = units[blockIdx.x];
    const QpSys q = sys[u.x];
    const int i = u.y, b = q.b, ng = q.ng, pe = q.pe, me = q.me, t = threadIdx.x;
    stage_rows<NT>(L, d, q, i, true, true);
    __syncthreads();
    const long long b2 = (long long)b * b;
    for (int e = t; e < b * b; e += NT) {
        const int r = e / b, c = e - r * b;
        double se = 0.0, si = 0.0;
        for (int k = 0; k < pe; ++k) se += L.EL[k * b + r] * L.EL[k * b + c] + L.ERp[k * b + r] * L.ERp[k * b + c];
        for (int k = 0; k < me; ++k)
            si += L.w[k] * L.IL[k * b + r] * L.IL[k * b + c] + L.wp[k] * L.IRp[k * b + r] * L.IRp[k * b + c];
        const long long o = q.oD + i * b2 + e;
        D[o] = d.Q[o] + (r == c ? rho : 0.0) + se * rdelta + si;
    }
    if (i + 1 < q.N) {
        for (int e = t; e < b * b; e += NT) {
            const int r = e / b, c = e - r * b;   // r: a variable of stage i + 1, c: of stage i
            double se = 0.0, si = 0.0;
            for (int k = 0; k < pe; ++k) se += L.ER[k * b + r] * L.EL[k * b + c];
            for (int k = 0; k < me; ++k) si += L.w[k] * L.IR[k * b + r] * L.IL[k * b + c];
            const long long o = q.oC + i * b2 + e;
            C[o] = d.S[o] + se * rdelta + si;
        }
    }
    for (int e = t; e < ng * b; e += NT) {
        const int g = e / b, c = e - g * b;
        double se = 0.0, si = 0.0;
        for (int k = 0; k < pe; ++k) se += L.EG[k * ng + g] * L.EL[k * b + c] + L.EGp[k * ng + g] * L.ERp[k * b + c];
        for (int k = 0; k < me; ++k)
            si += L.w[k] * L.IG[k * ng + g] * L.IL[k * b + c] + L.wp[k] * L.IGp[k * ng + g] * L.IRp[k * b + c];
        const long long o = q.oB + (long long)i * ng * b + e;
        B[o] = d.T[o] + se * rdelta + si;
    }
    for (int e = t; e < ng * ng; e += NT) {
        const int g1 = e / ng, g2 = e - g1 * ng;
        double se = 0.0, si = 0.0;
        for (int k = 0; k < pe; ++k) se += L.EG[k * ng + g1] * L.EG[k * ng + g2];
        for (int k = 0; k < me; ++k) si += L.w[k] * L.IG[k * ng + g1] * L.IG[k * ng + g2];
        part[q.oPart + (long long)i * ng * ng + e] = se * rdelta + si;
    }
}

// In thread t < E of a 256-thread workgroup: sum_{k < n} src[k * stride + t] (E <=
// 256), the k range split over 256 / E slices with eight loads in flight each.
template <int NT>
__device__ inline double slice_sum(const double *src, long long stride, int n, int E, double *red)
{
    const int t = threadIdx.x, KS = NT / E, e = t % E, ks = t / E;
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

// The sums over a system's stages below run in one workgroup per system: 1024
// threads when some horizon is long (NT / E threads per entry read the stage
// partials in few rounds), 256 otherwise.
constexpr int SUM_NT_LONG = 1024, SUM_NT_SHORT = 256, SUM_LONG_N = 512;
// The kernels with one workgroup per (system, stage): 256 threads, or 64 when a
// plan has many stages (small stages then keep more workgroups in flight).
constexpr int UNIT_NT = 256, UNIT_NT_SMALL = 64, UNIT_MANY = 8192;

// corner = Qg + rho I + sum of the groups' partials (one workgroup per system).
template <int NT>
__global__ void __launch_bounds__(NT) qp_corner_k(const QpSys *sys, QpPtr d, double rho, double *corner,
                                                  const double *part)
{
    __shared__ double red[NT];
    const QpSys q = sys[blockIdx.x];
    const int ng = q.ng, E = ng * ng, t = threadIdx.x;
    if (E == 0) return;
    const double s = slice_sum<NT>(part + q.oPart, E, q.N, E, red);
    if (t < E) {
        const long long o = q.oCor + t;
        corner[o] = d.Qg[o] + ((t / ng) == (t % ng) ? rho : 0.0) + s;
    }
}

// The reduced rhs of stage i, and group i's part of its g rows.
template <int NT>
__global__ void __launch_bounds__(NT) qp_rhs_k(const QpSys *sys, const int2 *units, QpPtr d, QpMax mx, double rdelta,
                                                const double *rx, const double *ry, const double *rz, double *rhs,
                                                double *part)
{
    extern __shared__ double lds[];
    const StageLds L = carve(lds, mx);
    const int2 u = units[blockIdx.x];
    const QpSys q = sys[u.x];
    const int i = u.y, b = q.b, ng = q.ng, pe = q.pe, me = q.me, nr = q.nr, t = threadIdx.x;
    const bool pv = i > 0;
    stage_rows<NT>(L, d, q, i, false, true);
    stage<NT>(L.ry, ry + q.oy + (long long)i * pe * nr, pe * nr, true);
    stage<NT>(L.rz, rz + q.oz + (long long)i * me * nr, me * nr, true);
    stage<NT>(L.ryp, ry + q.oy + (long long)(i - 1) * pe * nr, pe * nr, pv);
    stage<NT>(L.rzp, rz + q.oz + (long long)(i - 1) * me * nr, me * nr, pv);
    __syncthreads();
    for (int e = t; e < b * nr; e += NT) {
        const int r = e / nr, j = e - r * nr;
        double se = 0.0, si = 0.0;
        for (int k = 0; k < pe; ++k) se += L.EL[k * b + r] * L.ry[k * nr + j] + L.ERp[k * b + r] * L.ryp[k * nr + j];
        for (int k = 0; k < me; ++k)
            si += L.IL[k * b + r] * L.w[k] * L.rz[k * nr + j] + L.IRp[k * b + r] * L.wp[k] * L.rzp[k * nr + j];
        const long long o = q.oR + (long long)i * b * nr + e;
        rhs[o] = rx[o] + se * rdelta + si;
    }
    for (int e = t; e < ng * nr; e += NT) {
        const int g = e / nr, j = e - g * nr;
        double se = 0.0, si = 0.0;
        for (int k = 0; k < pe; ++k) se += L.EG[k * ng + g] * L.ry[k * nr + j];
        for (int k = 0; k < me; ++k) si += L.IG[k * ng + g] * L.w[k] * L.rz[k * nr + j];
        part[q.oPart + (long long)i * ng * nr + e] = se * rdelta + si;
    }
}

// The g rows of the reduced rhs (one workgroup per system).
template <int NT>
__global__ void __launch_bounds__(NT) qp_rhs_g_k(const QpSys *sys, const double *rx, double *rhs, const double *part)
{
    __shared__ double red[NT];
    const QpSys q = sys[blockIdx.x];
    const int E = q.ng * q.nr, t = threadIdx.x;
    if (E == 0) return;
    const double s = slice_sum<NT>(part + q.oPart, E, q.N, E, red);
    if (t < E) {
        const long long o = q.oR + (long long)q.N * q.b * q.nr + t;
        rhs[o] = rx[o] + s;
    }
}

// dy and dz of constraint group i.
template <int NT>
__global__ void __launch_bounds__(NT) qp_recover_k(const QpSys *sys, const int2 *units, QpPtr d, QpMax mx,
                                                    double rdelta, const double *dx, const double *ry,
                                                    const double *rz, double *dy, double *dz)
{
    extern __shared__ double lds[];
    const StageLds L = carve(lds, mx);
    const int2 u = units[blockIdx.x];
    const QpSys q = sys[u.x];
    const int i = u.y, b = q.b, ng = q.ng, pe = q.pe, me = q.me, nr = q.nr, t = threadIdx.x;
    const bool nx = i + 1 < q.N;
    stage_rows<NT>(L, d, q, i, true, false);
    const long long rb = (long long)b * nr;
    stage<NT>(L.xi, dx + q.oR + i * rb, b * nr, true);
    stage<NT>(L.xn, dx + q.oR + (i + 1) * rb, b * nr, nx);
    stage<NT>(L.xg, dx + q.oR + (long long)q.N * rb, ng * nr, true);
    __syncthreads();
    for (int e = t; e < pe * nr; e += NT) {
        const int k = e / nr, j = e - k * nr;
        double s = 0.0;
        for (int c = 0; c < b; ++c) s += L.EL[k * b + c] * L.xi[c * nr + j] + L.ER[k * b + c] * L.xn[c * nr + j];
        for (int g = 0; g < ng; ++g) s += L.EG[k * ng + g] * L.xg[g * nr + j];
        const long long o = q.oy + (long long)i * pe * nr + e;
        dy[o] = (s - ry[o]) * rdelta;
    }
    for (int e = t; e < me * nr; e += NT) {
        const int k = e / nr, j = e - k * nr;
        double s = 0.0;
        for (int c = 0; c < b; ++c) s += L.IL[k * b + c] * L.xi[c * nr + j] + L.IR[k * b + c] * L.xn[c * nr + j];
        for (int g = 0; g < ng; ++g) s += L.IG[k * ng + g] * L.xg[g * nr + j];
        const long long o = q.oz + (long long)i * me * nr + e;
        dz[o] = L.w[k] * (s - rz[o]);
    }
}

// ------------------------------------------------------------------ interior-point loop
// Residuals of the KKT conditions at (x, y, z, s), one rhs column:
//   r_d = P x + c + A^T y + G^T z,  r_p = A x - beq,  r_s = G x + s - h.
// Stage i's rows of r_d (and group i's part of its g rows), and group i's rows of
// r_p and r_s.  P's blocks are read from the Q, S, T pools where they are used.
template <int NT>
__global__ void __launch_bounds__(NT) ipm_resid_k(const QpSys *sys, const int2 *units, QpPtr d, QpMax mx,
                                                   const double *x, const double *y, const double *z,
                                                   const double *s, const double *c, const double *beq,
                                                   const double *h, double *rd, double *rp, double *rs, double *part)
{
    extern __shared__ double lds[];
    const StageLds L = carve(lds, mx);
    const int2 u = units[blockIdx.x];
    const QpSys q = sys[u.x];
    const int i = u.y, b = q.b, ng = q.ng, pe = q.pe, me = q.me, N = q.N, t = threadIdx.x;
    const bool nx = i + 1 < N, pv = i > 0;
    stage_rows<NT>(L, d, q, i, true, true);
    stage<NT>(L.xi, x + q.oR + (long long)i * b, b, true);
    stage<NT>(L.xn, x + q.oR + (long long)(i + 1) * b, b, nx);
    stage<NT>(L.xp, x + q.oR + (long long)(i - 1) * b, b, pv);
    stage<NT>(L.xg, x + q.oR + (long long)N * b, ng, true);
    stage<NT>(L.ry, y + q.oy + (long long)i * pe, pe, true);
    stage<NT>(L.ryp, y + q.oy + (long long)(i - 1) * pe, pe, pv);
    stage<NT>(L.rz, z + q.oz + (long long)i * me, me, true);
    stage<NT>(L.rzp, z + q.oz + (long long)(i - 1) * me, me, pv);
    __syncthreads();
    const long long b2 = (long long)b * b;
    const double *Qi = d.Q + q.oD + i * b2, *Si = d.S + q.oC + i * b2, *Sp = d.S + q.oC + (i - 1) * b2;
    const double *Ti = d.T + q.oB + (long long)i * ng * b;
    for (int r = t; r < b; r += NT) {
        double v = c[q.oR + (long long)i * b + r];
        for (int cc = 0; cc < b; ++cc) v += Qi[r * b + cc] * L.xi[cc];
        if (nx)
            for (int cc = 0; cc < b; ++cc) v += Si[cc * b + r] * L.xn[cc];
        if (pv)
            for (int cc = 0; cc < b; ++cc) v += Sp[r * b + cc] * L.xp[cc];
        for (int g = 0; g < ng; ++g) v += Ti[g * b + r] * L.xg[g];
        for (int k = 0; k < pe; ++k) v += L.EL[k * b + r] * L.ry[k] + L.ERp[k * b + r] * L.ryp[k];
        for (int k = 0; k < me; ++k) v += L.IL[k * b + r] * L.rz[k] + L.IRp[k * b + r] * L.rzp[k];
        rd[q.oR + (long long)i * b + r] = v;
    }
    for (int g = t; g < ng; g += NT) {
        double v = 0.0;
        for (int cc = 0; cc < b; ++cc) v += Ti[g * b + cc] * L.xi[cc];
        for (int k = 0; k < pe; ++k) v += L.EG[k * ng + g] * L.ry[k];
        for (int k = 0; k < me; ++k) v += L.IG[k * ng + g] * L.rz[k];
        part[q.oPart + (long long)i * ng + g] = v;
    }
    for (int k = t; k < pe; k += NT) {
        double v = -beq[q.oy + (long long)i * pe + k];
        for (int cc = 0; cc < b; ++cc) v += L.EL[k * b + cc] * L.xi[cc] + L.ER[k * b + cc] * L.xn[cc];
        for (int g = 0; g < ng; ++g) v += L.EG[k * ng + g] * L.xg[g];
        rp[q.oy + (long long)i * pe + k] = v;
    }
    for (int k = t; k < me; k += NT) {
        const long long o = q.oz + (long long)i * me + k;
        double v = s[o] - h[o];
        for (int cc = 0; cc < b; ++cc) v += L.IL[k * b + cc] * L.xi[cc] + L.IR[k * b + cc] * L.xn[cc];
        for (int g = 0; g < ng; ++g) v += L.IG[k * ng + g] * L.xg[g];
        rs[o] = v;
    }
}

// The g rows of r_d: c_g + Qg x_g + the stages' parts (one workgroup per system).
template <int NT>
__global__ void __launch_bounds__(NT) ipm_resid_g_k(const QpSys *sys, QpPtr d, const double *x, const double *c,
                                                    double *rd, const double *part)
{
    __shared__ double red[NT];
    const QpSys q = sys[blockIdx.x];
    const int ng = q.ng, t = threadIdx.x;
    if (ng == 0) return;
    const double sum = slice_sum<NT>(part + q.oPart, ng, q.N, ng, red);
    if (t < ng) {
        const long long og = q.oR + (long long)q.N * q.b;
        double v = c[og + t] + sum;
        for (int g = 0; g < ng; ++g) v += d.Qg[q.oCor + t * ng + g] * x[og + g];
        rd[og + t] = v;
    }
}

struct IpmState {
    double mu;
    int status;   // 0 running, 1 converged, -1 a factorization failed
    int iters;
};

struct IpmVec {
    double *x, *y, *z, *s, *w;
    const double *rd, *rp, *rs;
    double *RX, *RY, *RZ, *X, *DY, *DZ, *DS;
    const int *info;
};

// Block-wide reductions over the NT threads (every thread calls them).
template <int NT>
__device__ inline double block_reduce(double v, double *red, int op)   // 0 sum, 1 max, 2 min
{
    const int t = threadIdx.x;
    __syncthreads();
    red[t] = v;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if (t < h) {
            const double a = red[t], bb = red[t + h];
            red[t] = op == 0 ? a + bb : (op == 1 ? fmax(a, bb) : fmin(a, bb));
        }
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Largest step in (0, 1] keeping v + a dv >= 0 over one thread's share (min-reduced afterwards).
__device__ inline double ratio(double v, double dv) { return dv < 0.0 ? -v / dv : 1.0; }

// The vector work of one iteration for one system (one workgroup per system):
//   PH 0 (after the residuals; PH 4 the same without counting an iteration): mu,
//        the residual norm, the convergence test; for a
//        running system the weights w = z / (s + delta z) and the predictor rhs
//        (rx, ry, rz) = (-r_d, -r_p, -r_s + s); a finished one gets w = 1 and a zero rhs.
//   PH 1 (after the predictor's solve): ds, the affine step, sigma = (mu_aff / mu)^3
//        and the corrector's rz = -r_s - (-s z + sigma mu - ds dz) / z.
//   PH 2 (after the corrector's solve): ds, the step 0.99 * (largest step keeping s,
//        z >= 0) capped at 1, and the update of x, y, z, s.
//   PH 3 (the starting point, after a predictor solve from x = 0, s = z = 1): the
//        full step, then s and z moved into the interior by Mehrotra's heuristic:
//        s += max(-1.5 min s, 0), z += max(-1.5 min z, 0), and with t = s^T z,
//        s += t / (2 sum z), z += t / (2 sum s).  Systems without inequality rows
//        start the loop at x = 0.
template <int PH, int NT>
__global__ void __launch_bounds__(NT) ipm_vec_k(const QpSys *sys, IpmState *state, int *active, IpmVec v,
                                                double delta, double tol)
{
    __shared__ double red[NT];
    const QpSys q = sys[blockIdx.x];
    const int t = threadIdx.x;
    IpmState st = state[blockIdx.x];
    const long long nx = (long long)q.N * q.b + q.ng, ny = (long long)q.N * q.pe, nz = (long long)q.N * q.me;
    double *x = v.x + q.oR, *X = v.X + q.oR, *RX = v.RX + q.oR;
    const double *rd = v.rd + q.oR;
    double *y = v.y + q.oy, *DY = v.DY + q.oy, *RY = v.RY + q.oy;
    const double *rp = v.rp + q.oy;
    double *z = v.z + q.oz, *s = v.s + q.oz, *w = v.w + q.ow, *RZ = v.RZ + q.oz, *DZ = v.DZ + q.oz,
           *DS = v.DS + q.oz;
    const double *rs = v.rs + q.oz;
    if (PH == 0 || PH == 4) {
        double res = 0.0, sz = 0.0;
        for (long long e = t; e < nx; e += NT) res = fmax(res, fabs(rd[e]));
        for (long long e = t; e < ny; e += NT) res = fmax(res, fabs(rp[e]));
        for (long long e = t; e < nz; e += NT) {
            res = fmax(res, fabs(rs[e]));
            sz += s[e] * z[e];
        }
        res = block_reduce<NT>(res, red, 1);
        sz = block_reduce<NT>(sz, red, 0);
        const double mu = nz > 0 ? sz / (double)nz : 0.0;
        bool run = st.status == 0;
        if (run && res <= tol && mu <= tol) {
            run = false;
            if (t == 0) state[blockIdx.x].status = 1;
        }
        for (long long e = t; e < nx; e += NT) RX[e] = run ? -rd[e] : 0.0;
        for (long long e = t; e < ny; e += NT) RY[e] = run ? -rp[e] : 0.0;
        for (long long e = t; e < nz; e += NT) {
            w[e] = run ? z[e] / (s[e] + delta * z[e]) : 1.0;
            RZ[e] = run ? -rs[e] + s[e] : 0.0;
        }
        if (t == 0 && run) {
            state[blockIdx.x].mu = mu;
            if (PH == 0) state[blockIdx.x].iters = st.iters + 1;
            atomicAdd(active, 1);
        }
        return;
    }
    if (st.status != 0) return;
    if (v.info[blockIdx.x] != 0) {
        if (PH == 2 && t == 0) state[blockIdx.x].status = -1;
        return;
    }
    if (PH == 3) {
        if (nz == 0) return;
        double smin = 1e300, zmin = 1e300;
        for (long long e = t; e < nx; e += NT) x[e] += X[e];
        for (long long e = t; e < ny; e += NT) y[e] += DY[e];
        for (long long e = t; e < nz; e += NT) {
            s[e] += -rs[e] - RZ[e] - DZ[e] / w[e];
            z[e] += DZ[e];
            smin = fmin(smin, s[e]);
            zmin = fmin(zmin, z[e]);
        }
        smin = block_reduce<NT>(smin, red, 2);
        zmin = block_reduce<NT>(zmin, red, 2);
        const double ps = fmax(-1.5 * smin, 0.0), pz = fmax(-1.5 * zmin, 0.0);
        double tsz = 0.0, ss = 0.0, sumz = 0.0;
        for (long long e = t; e < nz; e += NT) {
            s[e] += ps;
            z[e] += pz;
            tsz += s[e] * z[e];
            ss += s[e];
            sumz += z[e];
        }
        tsz = block_reduce<NT>(tsz, red, 0);
        ss = block_reduce<NT>(ss, red, 0);
        sumz = block_reduce<NT>(sumz, red, 0);
        const double hs = 0.5 * tsz / sumz, hz = 0.5 * tsz / ss;
        for (long long e = t; e < nz; e += NT) {
            s[e] += hs;
            z[e] += hz;
        }
        return;
    }
    double amax = 1.0;
    for (long long e = t; e < nz; e += NT) {
        const double ds = -rs[e] - RZ[e] - DZ[e] / w[e];
        DS[e] = ds;
        amax = fmin(amax, fmin(ratio(s[e], ds), ratio(z[e], DZ[e])));
    }
    amax = block_reduce<NT>(amax, red, 2);
    if (PH == 1) {
        if (nz == 0) return;
        double sz = 0.0;
        for (long long e = t; e < nz; e += NT) sz += (s[e] + amax * DS[e]) * (z[e] + amax * DZ[e]);
        sz = block_reduce<NT>(sz, red, 0);
        const double mu_aff = sz / (double)nz;
        const double sg = mu_aff / st.mu, sigma = sg * sg * sg;
        for (long long e = t; e < nz; e += NT) {
            const double rc = -s[e] * z[e] + sigma * st.mu - DS[e] * DZ[e];
            RZ[e] = -rs[e] - rc / z[e];
        }
        return;
    }
    const double alpha = nz > 0 ? fmin(1.0, 0.99 * amax) : 1.0;
    for (long long e = t; e < nx; e += NT) x[e] += alpha * X[e];
    for (long long e = t; e < ny; e += NT) y[e] += alpha * DY[e];
    for (long long e = t; e < nz; e += NT) {
        z[e] += alpha * DZ[e];
        s[e] += alpha * DS[e];
    }
}

// The starting point x = 0, y = 0, s = z = 1 and a fresh state.
__global__ void __launch_bounds__(256) ipm_init_k(const QpSys *sys, IpmState *state, double *x, double *y,
                                                  double *z, double *s)
{
    const QpSys q = sys[blockIdx.x];
    const int t = threadIdx.x;
    const long long nx = (long long)q.N * q.b + q.ng, ny = (long long)q.N * q.pe, nz = (long long)q.N * q.me;
    for (long long e = t; e < nx; e += 256) x[q.oR + e] = 0.0;
    for (long long e = t; e < ny; e += 256) y[q.oy + e] = 0.0;
    for (long long e = t; e < nz; e += 256) {
        z[q.oz + e] = 1.0;
        s[q.oz + e] = 1.0;
    }
    if (t == 0) state[blockIdx.x] = IpmState{0.0, 0, 0};
}

__global__ void ipm_clear_k(int *active)
{
    if (threadIdx.x == 0) *active = 0;
}

// Per system: iterations to convergence, -1 (a factorization failed) or -2 (not
// converged within the iteration limit).
__global__ void __launch_bounds__(256) ipm_status_k(const IpmState *state, int S, int32_t *out)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < S) out[i] = state[i].status == 1 ? state[i].iters : (state[i].status == -1 ? -1 : -2);
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
    bool long_n = false;   // some horizon of SUM_LONG_N stages or more
    int unit_nt = UNIT_NT; // threads per (system, stage) workgroup
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

// One vector phase for every system: 1024 threads per system once a horizon is
// long, 256 otherwise.
template <int PH>
void launch_vec(const kkt_qp *qp, int S, hipStream_t stream, IpmState *state, int *active, const IpmVec &v,
                double delta, double tol)
{
    if (qp->long_n)
        hipLaunchKernelGGL((ipm_vec_k<PH, SUM_NT_LONG>), dim3(S), dim3(SUM_NT_LONG), 0, stream, qp->dsys, state,
                           active, v,
                           delta, tol);
    else
        hipLaunchKernelGGL((ipm_vec_k<PH, SUM_NT_SHORT>), dim3(S), dim3(SUM_NT_SHORT), 0, stream, qp->dsys, state,
                           active,
                           v, delta, tol);
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
    bool long_n = false;
    for (int s = 0; s < S; ++s) {
        kkt_system_layout L;
        rc = kkt_plan_system(plan, s, &L);
        if (rc != KKT_OK) return rc;
        QpSys &q = sys[s];
        const long long N = L.N, b = L.b, ng = L.ng, pe = n_eq[s], me = n_in[s];
        q.N = L.N; q.b = L.b; q.ng = L.ng; q.pe = n_eq[s]; q.me = n_in[s]; q.nr = nr;
        if (L.N >= SUM_LONG_N) long_n = true;
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
    qp->long_n = long_n;
    qp->unit_nt = units.size() >= (size_t)UNIT_MANY ? UNIT_NT_SMALL : UNIT_NT;
    qp->lds = stage_lds_doubles(mx) * sizeof(double);
    if (qp->lds > 160 * 1024) { delete qp; return KKT_EDIMS; }
    const bool ok = hipMalloc((void **)&qp->dsys, sizeof(QpSys) * S) == hipSuccess &&
                    hipMalloc((void **)&qp->dunits, sizeof(int2) * units.size()) == hipSuccess &&
                    hipMalloc((void **)&qp->dpart, sizeof(double) * std::max(1LL, oP)) == hipSuccess &&
                    hipMemcpy(qp->dsys, sys.data(), sizeof(QpSys) * S, hipMemcpyHostToDevice) == hipSuccess &&
                    hipMemcpy(qp->dunits, units.data(), sizeof(int2) * units.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok || set_lds((const void *)qp_assemble_k<UNIT_NT>, qp->lds) != KKT_OK ||
        set_lds((const void *)qp_assemble_k<UNIT_NT_SMALL>, qp->lds) != KKT_OK ||
        set_lds((const void *)qp_rhs_k<UNIT_NT>, qp->lds) != KKT_OK ||
        set_lds((const void *)qp_rhs_k<UNIT_NT_SMALL>, qp->lds) != KKT_OK ||
        set_lds((const void *)qp_recover_k<UNIT_NT>, qp->lds) != KKT_OK ||
        set_lds((const void *)qp_recover_k<UNIT_NT_SMALL>, qp->lds) != KKT_OK) {
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
    if (qp->unit_nt == UNIT_NT_SMALL)
        hipLaunchKernelGGL(qp_assemble_k<UNIT_NT_SMALL>, dim3(qp->nunits), dim3(UNIT_NT_SMALL), qp->lds, stream,
                           qp->dsys, qp->dunits, d, qp->mx, rho, 1.0 / delta, D, C, B, qp->dpart);
    else
        hipLaunchKernelGGL(qp_assemble_k<UNIT_NT>, dim3(qp->nunits), dim3(UNIT_NT), qp->lds, stream, qp->dsys,
                           qp->dunits, d, qp->mx, rho, 1.0 / delta, D, C, B, qp->dpart);
    if (hipGetLastError() != hipSuccess) return KKT_ELAUNCH;
    if (Col) {
        if (qp->long_n)
            hipLaunchKernelGGL(qp_corner_k<SUM_NT_LONG>, dim3(qp->S), dim3(SUM_NT_LONG), 0, stream, qp->dsys, d, rho,
                               corner, qp->dpart);
        else
            hipLaunchKernelGGL(qp_corner_k<SUM_NT_SHORT>, dim3(qp->S), dim3(SUM_NT_SHORT), 0, stream, qp->dsys, d, rho,
                               corner, qp->dpart);
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
    if (qp->unit_nt == UNIT_NT_SMALL)
        hipLaunchKernelGGL(qp_rhs_k<UNIT_NT_SMALL>, dim3(qp->nunits), dim3(UNIT_NT_SMALL), qp->lds, stream, qp->dsys,
                           qp->dunits, d, qp->mx, 1.0 / delta, rx, ry, rz, rhs, qp->dpart);
    else
        hipLaunchKernelGGL(qp_rhs_k<UNIT_NT>, dim3(qp->nunits), dim3(UNIT_NT), qp->lds, stream, qp->dsys, qp->dunits,
                           d, qp->mx, 1.0 / delta, rx, ry, rz, rhs, qp->dpart);
    if (hipGetLastError() != hipSuccess) return KKT_ELAUNCH;
    if (qp->long_n)
        hipLaunchKernelGGL(qp_rhs_g_k<SUM_NT_LONG>, dim3(qp->S), dim3(SUM_NT_LONG), 0, stream, qp->dsys, rx, rhs,
                           qp->dpart);
    else
        hipLaunchKernelGGL(qp_rhs_g_k<SUM_NT_SHORT>, dim3(qp->S), dim3(SUM_NT_SHORT), 0, stream, qp->dsys, rx, rhs,
                           qp->dpart);
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
    if (qp->unit_nt == UNIT_NT_SMALL)
        hipLaunchKernelGGL(qp_recover_k<UNIT_NT_SMALL>, dim3(qp->nunits), dim3(UNIT_NT_SMALL), qp->lds, stream,
                           qp->dsys, qp->dunits, ptrs(data), qp->mx, 1.0 / delta, dx, ry, rz, dy, dz);
    else
        hipLaunchKernelGGL(qp_recover_k<UNIT_NT>, dim3(qp->nunits), dim3(UNIT_NT), qp->lds, stream, qp->dsys,
                           qp->dunits, ptrs(data), qp->mx, 1.0 / delta, dx, ry, rz, dy, dz);
    return hipGetLastError() == hipSuccess ? KKT_OK : KKT_ELAUNCH;
}

}  // extern "C"

struct kkt_ipm {
    const kkt_plan *plan = nullptr;
    const kkt_qp *qp = nullptr;
    long long nx = 0, ny = 0, nz = 0, nD = 0, nC = 0, nB = 0, nCor = 0;
    double *buf = nullptr;
    IpmState *state = nullptr;
    int *active = nullptr, *info = nullptr, *h_active = nullptr;
    ~kkt_ipm()
    {
        // teardown: nothing to recover from a failure
        if (buf) (void)hipFree(buf);
        if (state) (void)hipFree(state);
        if (active) (void)hipFree(active);
        if (info) (void)hipFree(info);
        if (h_active) (void)hipHostFree(h_active);
    }
};

extern "C" {

int kkt_ipm_create(const kkt_plan *plan, const kkt_qp *qp, kkt_ipm **out)
{
    if (!plan || !qp || !out) return KKT_EPOINTER;
    *out = nullptr;
    kkt_plan_info info;
    int rc = kkt_plan_get_info(plan, &info);
    if (rc != KKT_OK) return rc;
    if (info.nrhs != 1 || info.num_systems != qp->S) return KKT_EDIMS;
    kkt_ipm *m = new (std::nothrow) kkt_ipm;
    if (!m) return KKT_EINTERNAL;
    m->plan = plan;
    m->qp = qp;
    m->nx = info.rhs_len; m->ny = qp->len[7]; m->nz = qp->len[8];
    m->nD = info.D_len; m->nC = info.C_len; m->nB = info.B_len; m->nCor = info.corner_len;
    const long long total = 3 * m->nx + 3 * m->ny + 5 * m->nz + m->nD + m->nC + m->nB + m->nCor;
    const bool ok = hipMalloc((void **)&m->buf, sizeof(double) * std::max(1LL, total)) == hipSuccess &&
                    hipMalloc((void **)&m->state, sizeof(IpmState) * std::max(1, qp->S)) == hipSuccess &&
                    hipMalloc((void **)&m->active, sizeof(int)) == hipSuccess &&
                    hipMalloc((void **)&m->info, sizeof(int) * std::max(1, qp->S)) == hipSuccess &&
                    hipHostMalloc((void **)&m->h_active, sizeof(int), hipHostMallocDefault) == hipSuccess &&
                    set_lds((const void *)ipm_resid_k<UNIT_NT>, qp->lds) == KKT_OK &&
                    set_lds((const void *)ipm_resid_k<UNIT_NT_SMALL>, qp->lds) == KKT_OK;
    if (!ok) {
        delete m;
        return KKT_ELAUNCH;
    }
    *out = m;
    return KKT_OK;
}

int kkt_ipm_destroy(kkt_ipm *ipm)
{
    delete ipm;
    return KKT_OK;
}

int kkt_ipm_solve(kkt_ipm *ipm, void *workspace, const kkt_qp_data *data, const double *c, const double *beq,
                  const double *h, double rho, double delta, double tol, int32_t max_iter, double *x, double *y,
                  double *z, double *s, int32_t *status, hipStream_t stream)
{
    if (!ipm || !workspace || !data || !c || !x || !status) return KKT_EPOINTER;
    const kkt_qp *qp = ipm->qp;
    if ((ipm->ny && (!beq || !y)) || (ipm->nz && (!h || !z || !s))) return KKT_EPOINTER;
    if (!(delta > 0.0) || !(rho >= 0.0) || !(tol > 0.0) || max_iter < 0) return KKT_EDIMS;
    const void *ps[] = {c, beq, h, x, y, z, s};
    for (const void *p : ps)
        if (!aligned8(p)) return KKT_EPOINTER;
    if (qp->nunits == 0) return KKT_OK;
    // work vectors: r_d, rx, dx (rhs layout); r_p, ry, dy; r_s, rz, dz, ds, w; Psi's pools
    double *p = ipm->buf;
    double *rd = p; p += ipm->nx;
    double *RX = p; p += ipm->nx;
    double *X = p; p += ipm->nx;
    double *rp = p; p += ipm->ny;
    double *RY = p; p += ipm->ny;
    double *DY = p; p += ipm->ny;
    double *rs = p; p += ipm->nz;
    double *RZ = p; p += ipm->nz;
    double *DZ = p; p += ipm->nz;
    double *DS = p; p += ipm->nz;
    double *w = p; p += ipm->nz;
    double *D = p; p += ipm->nD;
    double *C = p; p += ipm->nC;
    double *B = p; p += ipm->nB;
    double *Cor = p;
    kkt_qp_data dw = *data;
    dw.w = w;   // the iteration's own weights
    const QpPtr d = ptrs(&dw);
    if (!data_ok(qp, &dw, true, ipm->nD, ipm->nC, ipm->nB, ipm->nCor)) return KKT_EPOINTER;
    const int S = qp->S;
    IpmVec v{x, y, z, s, w, rd, rp, rs, RX, RY, RZ, X, DY, DZ, DS, ipm->info};
    hipLaunchKernelGGL(ipm_init_k, dim3(S), dim3(256), 0, stream, qp->dsys, ipm->state, x, y, z, s);
    if (hipGetLastError() != hipSuccess) return KKT_ELAUNCH;
    int rc = KKT_OK;
    // the starting point: a predictor solve from x = 0, s = z = 1, then the shift
    if (ipm->nz > 0) {
        if (qp->unit_nt == UNIT_NT_SMALL)
            hipLaunchKernelGGL(ipm_resid_k<UNIT_NT_SMALL>, dim3(qp->nunits), dim3(UNIT_NT_SMALL), qp->lds, stream,
                               qp->dsys, qp->dunits, d, qp->mx, (const double *)x, (const double *)y,
                               (const double *)z, (const double *)s, c, beq, h, rd, rp, rs, qp->dpart);
        else
            hipLaunchKernelGGL(ipm_resid_k<UNIT_NT>, dim3(qp->nunits), dim3(UNIT_NT), qp->lds, stream, qp->dsys,
                               qp->dunits, d, qp->mx, (const double *)x, (const double *)y, (const double *)z,
                               (const double *)s, c, beq, h, rd, rp, rs, qp->dpart);
        if (qp->long_n)
            hipLaunchKernelGGL(ipm_resid_g_k<SUM_NT_LONG>, dim3(S), dim3(SUM_NT_LONG), 0, stream, qp->dsys, d,
                               (const double *)x, c, rd, (const double *)qp->dpart);
        else
            hipLaunchKernelGGL(ipm_resid_g_k<SUM_NT_SHORT>, dim3(S), dim3(SUM_NT_SHORT), 0, stream, qp->dsys, d,
                               (const double *)x, c, rd, (const double *)qp->dpart);
        launch_vec<4>(qp, S, stream, ipm->state, ipm->active, v, delta, tol);
        if (hipGetLastError() != hipSuccess) return KKT_ELAUNCH;
        rc = kkt_qp_assemble(qp, &dw, rho, delta, D, C, B, Cor, stream);
        if (rc == KKT_OK) rc = kkt_factor(ipm->plan, D, C, B, Cor, workspace, ipm->info, stream);
        if (rc == KKT_OK) rc = kkt_qp_reduce_rhs(qp, &dw, delta, RX, RY, RZ, X, stream);
        if (rc == KKT_OK) rc = kkt_solve(ipm->plan, workspace, X, stream);
        if (rc == KKT_OK) rc = kkt_qp_recover(qp, &dw, delta, X, RY, RZ, DY, DZ, stream);
        if (rc != KKT_OK) return rc;
        launch_vec<3>(qp, S, stream, ipm->state, ipm->active, v, delta, tol);
        if (hipGetLastError() != hipSuccess) return KKT_ELAUNCH;
    }
    for (int it = 0; it <= max_iter && rc == KKT_OK; ++it) {
        // the regularisation falls tenfold per iteration, to 1e-4 of its start
        const double f = std::max(1e-4, std::pow(10.0, -(double)(it + 1)));
        const double rk = rho * f, dk = delta * f;
        hipLaunchKernelGGL(ipm_clear_k, dim3(1), dim3(64), 0, stream, ipm->active);
        if (qp->unit_nt == UNIT_NT_SMALL)
            hipLaunchKernelGGL(ipm_resid_k<UNIT_NT_SMALL>, dim3(qp->nunits), dim3(UNIT_NT_SMALL), qp->lds, stream,
                               qp->dsys, qp->dunits, d, qp->mx, (const double *)x, (const double *)y,
                               (const double *)z, (const double *)s, c, beq, h, rd, rp, rs, qp->dpart);
        else
            hipLaunchKernelGGL(ipm_resid_k<UNIT_NT>, dim3(qp->nunits), dim3(UNIT_NT), qp->lds, stream, qp->dsys,
                               qp->dunits, d, qp->mx, (const double *)x, (const double *)y, (const double *)z,
                               (const double *)s, c, beq, h, rd, rp, rs, qp->dpart);
        if (qp->long_n)
            hipLaunchKernelGGL(ipm_resid_g_k<SUM_NT_LONG>, dim3(S), dim3(SUM_NT_LONG), 0, stream, qp->dsys, d,
                               (const double *)x, c, rd, (const double *)qp->dpart);
        else
            hipLaunchKernelGGL(ipm_resid_g_k<SUM_NT_SHORT>, dim3(S), dim3(SUM_NT_SHORT), 0, stream, qp->dsys, d,
                               (const double *)x, c, rd, (const double *)qp->dpart);
        launch_vec<0>(qp, S, stream, ipm->state, ipm->active, v, dk, tol);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(ipm->h_active, ipm->active, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess) {
            rc = KKT_ELAUNCH;
            break;
        }
        if (*ipm->h_active == 0 || it == max_iter) break;
        // one factorization, two solves (predictor, corrector)
        rc = kkt_qp_assemble(qp, &dw, rk, dk, D, C, B, Cor, stream);
        if (rc == KKT_OK) rc = kkt_factor(ipm->plan, D, C, B, Cor, workspace, ipm->info, stream);
        for (int ph = 1; ph <= 2 && rc == KKT_OK; ++ph) {
            rc = kkt_qp_reduce_rhs(qp, &dw, dk, RX, RY, RZ, X, stream);
            if (rc == KKT_OK) rc = kkt_solve(ipm->plan, workspace, X, stream);
            if (rc == KKT_OK) rc = kkt_qp_recover(qp, &dw, dk, X, RY, RZ, DY, DZ, stream);
            if (rc == KKT_OK) {
                if (ph == 1)
                    launch_vec<1>(qp, S, stream, ipm->state, ipm->active, v, dk, tol);
                else
                    launch_vec<2>(qp, S, stream, ipm->state, ipm->active, v, dk, tol);
                if (hipGetLastError() != hipSuccess) rc = KKT_ELAUNCH;
            }
        }
    }
    if (rc != KKT_OK) return rc;
    hipLaunchKernelGGL(ipm_status_k, dim3((S + 255) / 256), dim3(256), 0, stream, ipm->state, S, status);
    return hipGetLastError() == hipSuccess ? KKT_OK : KKT_ELAUNCH;
}

}  // extern "C"
