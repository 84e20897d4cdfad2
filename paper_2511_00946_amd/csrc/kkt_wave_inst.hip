// Instances of the row-lane kernels (kkt_wave.h) for one padded block size,
// KKT_WAVE_BP (compiled once per block class so the classes build in parallel).
#include <hip/hip_runtime.h>

#include "kkt_internal.h"
#include "kkt_wave.h"

#ifndef KKT_WAVE_BP
#error "KKT_WAVE_BP must be defined (8, 16, 24, 32 or 48)"
#endif

#define KKT_CAT2(a, b) a##b
#define KKT_CAT(a, b) KKT_CAT2(a, b)

namespace kkt_dev {

kfun_t KKT_CAT(wave_kernel_, KKT_WAVE_BP)(int mode, int phase)
{
    constexpr int BP = KKT_WAVE_BP;
    if (phase == 0) {
        switch (mode) {
        case M_FACTOR: return kkt_wave_p1<BP, M_FACTOR>;
        case M_FACTOR_SOLVE: return kkt_wave_p1<BP, M_FACTOR_SOLVE>;
        case M_SOLVE: return kkt_wave_p1<BP, M_SOLVE>;
        default: return kkt_wave_p1<BP, M_ADJOINT>;
        }
    }
    if (phase == 1) {
        switch (mode) {
        case M_FACTOR: return kkt_wave_p2<BP, M_FACTOR>;
        case M_FACTOR_SOLVE: return kkt_wave_p2<BP, M_FACTOR_SOLVE>;
        case M_SOLVE: return kkt_wave_p2<BP, M_SOLVE>;
        default: return kkt_wave_p2<BP, M_ADJOINT>;
        }
    }
    // the backward sweep is the same for the factor-solve and solve modes
    return mode == M_ADJOINT ? kkt_wave_p3<BP, M_ADJOINT> : kkt_wave_p3<BP, M_SOLVE>;
}

int KKT_CAT(wave_threads_, KKT_WAVE_BP)() { return WC<KKT_WAVE_BP>::NT; }

size_t KKT_CAT(wave_lds_bytes_, KKT_WAVE_BP)()
{
    return (size_t)wave_lds_offsets<KKT_WAVE_BP>().total * sizeof(double);
}

}  // namespace kkt_dev
