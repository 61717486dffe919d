// kern_nd_fix.hip -- fixed-shape instances of the separable d-D axis pass:
// axis lengths 2^7 .. 2^10, padded-row (axis 0) or interleaved (strided axes)
// LDS layout, drift-only or closing x-phase passes.  Same arithmetic as the
// runtime-shaped instances (the twiddles come from the same table), with every
// LDS address a per-thread base plus a compile-time offset.
#include <hip/hip_runtime.h>

#include "nd_pass.hpp"

namespace hfgpe {

template <typename Store, int MODE, int TPB, int LOGN>
static hipError_t launch_fix_layout(const LaunchND &L)
{
    // the closing x-phase falls on the last axis, never on axis 0 (d >= 2)
    if (L.axis == 0) {
        if constexpr (MODE == 0) return launch_pass_tpb<Store, 8, 1, MODE, TPB, kPassSep, 2 * LOGN>(L);
        return hipErrorInvalidValue;
    }
    return launch_pass_tpb<Store, 8, 1, MODE, TPB, kPassSep, 2 * LOGN + 1>(L);
}

template <typename Store, int MODE, int TPB>
static hipError_t launch_fix_n(const LaunchND &L)
{
    switch (L.n[L.axis]) {
    case 128: return launch_fix_layout<Store, MODE, TPB, 7>(L);
    case 256: return launch_fix_layout<Store, MODE, TPB, 8>(L);
    case 512: return launch_fix_layout<Store, MODE, TPB, 9>(L);
    case 1024: return launch_fix_layout<Store, MODE, TPB, 10>(L);
    default: return hipErrorInvalidValue;
    }
}

template <typename Store, int MODE>
static hipError_t launch_fix_tpb(const LaunchND &L)
{
    if constexpr (sizeof(Store) == 8) {
        // 512-thread groups only for c64 strided axes with short rows
        if (nd_pass_threads(L) == 512) {
            if (L.axis == 0) return hipErrorInvalidValue;
            switch (L.n[L.axis]) {
            case 128: return launch_pass_tpb<Store, 8, 1, MODE, 512, kPassSep, 2 * 7 + 1>(L);
            case 256: return launch_pass_tpb<Store, 8, 1, MODE, 512, kPassSep, 2 * 8 + 1>(L);
            case 512: return launch_pass_tpb<Store, 8, 1, MODE, 512, kPassSep, 2 * 9 + 1>(L);
            case 1024: return launch_pass_tpb<Store, 8, 1, MODE, 512, kPassSep, 2 * 10 + 1>(L);
            default: return hipErrorInvalidValue;
            }
        }
    }
    return launch_fix_n<Store, MODE, kThreadsND>(L);
}

hipError_t launch_nd_pass_fixed(const LaunchND &L)
{
    if (L.kind != kPassSep || L.apply_open || !nd_fixed_shape(L.n, L.axis, nd_pass_threads(L)))
        return hipErrorInvalidValue;
    if (L.c64) return L.apply_close ? launch_fix_tpb<float2, 1>(L) : launch_fix_tpb<float2, 0>(L);
    return L.apply_close ? launch_fix_tpb<double2, 1>(L) : launch_fix_tpb<double2, 0>(L);
}

}  // namespace hfgpe
