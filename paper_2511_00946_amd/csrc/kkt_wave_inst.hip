// Instances of the row-lane kernels for one padded block size, KKT_WAVE_BP, and
// one right-hand-side count, KKT_WAVE_NR (compiled once per pair so they build in
// parallel).  The single-wave classes (8, 16) have instances for 1, 4 and 8
// right-hand sides; the wider classes one for every count (KKT_WAVE_NR = 8).
#include <hip/hip_runtime.h>

#include "kkt_internal.h"
#include "kkt_kernels.h"

#ifndef KKT_WAVE_BP
#error "KKT_WAVE_BP must be defined (8, 16, 24, 32 or 48)"
#endif

#ifndef KKT_WAVE_NR
#define KKT_WAVE_NR 8
#endif

#define KKT_CAT4(a, b, c, d) a##b##c##d
#define KKT_CAT(a, b, c, d) KKT_CAT4(a, b, c, d)
#define KKT_CAT2(a, b) a##b
#define KKT_CATB(a, b) KKT_CAT2(a, b)

namespace kkt_dev {

namespace {

template <int BP, int NR>
kfun_t pick(int mode, int phase)
{
    if (phase == 0) {
        switch (mode) {
        case M_FACTOR: return kkt_wave_p1<BP, M_FACTOR, NR>;
        case M_FACTOR_SOLVE: return kkt_wave_p1<BP, M_FACTOR_SOLVE, NR>;
        case M_SOLVE: return kkt_wave_p1<BP, M_SOLVE, NR>;
        default: return kkt_wave_p1<BP, M_ADJOINT, NR>;
        }
    }
    if (phase == 1) {
        switch (mode) {
        case M_FACTOR: return kkt_wave_p2<BP, M_FACTOR, NR>;
        case M_FACTOR_SOLVE: return kkt_wave_p2<BP, M_FACTOR_SOLVE, NR>;
        case M_SOLVE: return kkt_wave_p2<BP, M_SOLVE, NR>;
        default: return kkt_wave_p2<BP, M_ADJOINT, NR>;
        }
    }
    // the backward sweep is the same for the factor-solve and solve modes
    return mode == M_ADJOINT ? kkt_wave_p3<BP, M_ADJOINT, NR> : kkt_wave_p3<BP, M_SOLVE, NR>;
}

}  // namespace

kfun_t KKT_CAT(wave_kernel_, KKT_WAVE_BP, _, KKT_WAVE_NR)(int mode, int phase)
{
    return pick<KKT_WAVE_BP, KKT_WAVE_NR>(mode, phase);
}

#if KKT_WAVE_NR == 8
int KKT_CATB(wave_threads_, KKT_WAVE_BP)() { return WC<KKT_WAVE_BP>::NT; }

size_t KKT_CATB(wave_lds_bytes_, KKT_WAVE_BP)()
{
    return (size_t)wave_lds_offsets<KKT_WAVE_BP>().total * sizeof(double);
}
#endif

}  // namespace kkt_dev
