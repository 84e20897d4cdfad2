// Internal interface between the host plan (kkt.hip) and the translation units
// that instantiate the row-lane kernels (kkt_wave_inst.hip, one per block class).
#pragma once
#include <stddef.h>
#include "kkt_device.h"

namespace kkt_dev {

typedef void (*kfun_t)(Args);

// Row-lane kernel of padded block size bp (8, 16, 24, 32, 48) for a mode, a phase
// (0: every item, 1: reduced chain + corner, 2: segment backward sweeps) and the
// call's right-hand-side count.
kfun_t wave_kernel(int bp, int mode, int phase, int nr);
int wave_threads(int bp);
size_t wave_lds_bytes(int bp);

// per-class instances (kkt_wave_inst.hip compiled once per class and rhs count)
#define KKT_WAVE_DECL(BP)                                  \
    kfun_t wave_kernel_##BP##_8(int mode, int phase);      \
    int wave_threads_##BP();                               \
    size_t wave_lds_bytes_##BP();
KKT_WAVE_DECL(8)
KKT_WAVE_DECL(16)
KKT_WAVE_DECL(24)
KKT_WAVE_DECL(32)
KKT_WAVE_DECL(48)
kfun_t wave_kernel_8_1(int mode, int phase);
kfun_t wave_kernel_8_4(int mode, int phase);
kfun_t wave_kernel_16_1(int mode, int phase);
kfun_t wave_kernel_16_4(int mode, int phase);
#undef KKT_WAVE_DECL

}  // namespace kkt_dev
