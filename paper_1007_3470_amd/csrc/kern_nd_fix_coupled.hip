// kern_nd_fix_coupled.hip -- fixed-shape instances of the coupled-trap axis
// passes (forward transform, forward + whole drift + inverse, inverse
// transform) for axes of 2^7 .. 2^10 points, 256-thread groups.  The passes
// that occur: forward along axes 0 .. d-2 and inverse along d-2 .. 0 (padded
// rows on axis 0, interleaved pencils on axis 1), the whole drift on the last
// axis (interleaved), and the closing x-phase only on the last inverse pass,
// along axis 0.
#include <hip/hip_runtime.h>

#include "nd_pass.hpp"

namespace hfgpe {

template <typename Store, int LOGN>
static hipError_t launch_coupled_n(const LaunchND &L)
{
    constexpr int ROW = 2 * LOGN, STR = 2 * LOGN + 1;
    const bool row = L.axis == 0;
    switch (L.kind) {
    case kPassFwd:
        if (L.apply_close) return hipErrorInvalidValue;
        return row ? launch_pass_tpb<Store, 8, 1, 0, kThreadsND, kPassFwd, ROW>(L)
                   : launch_pass_tpb<Store, 8, 1, 0, kThreadsND, kPassFwd, STR>(L);
    case kPassMid:
        if (L.apply_close || row) return hipErrorInvalidValue;
        return launch_pass_tpb<Store, 8, 1, 0, kThreadsND, kPassMid, STR>(L);
    case kPassInv:
        if (row) {
            return L.apply_close ? launch_pass_tpb<Store, 8, 1, 1, kThreadsND, kPassInv, ROW>(L)
                                 : launch_pass_tpb<Store, 8, 1, 0, kThreadsND, kPassInv, ROW>(L);
        }
        if (L.apply_close) return hipErrorInvalidValue;
        return launch_pass_tpb<Store, 8, 1, 0, kThreadsND, kPassInv, STR>(L);
    default: return hipErrorInvalidValue;
    }
}

template <typename Store>
static hipError_t launch_coupled_store(const LaunchND &L)
{
    switch (L.n[L.axis]) {
    case 128: return launch_coupled_n<Store, 7>(L);
    case 256: return launch_coupled_n<Store, 8>(L);
    case 512: return launch_coupled_n<Store, 9>(L);
    case 1024: return launch_coupled_n<Store, 10>(L);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_nd_pass_fixed_coupled(const LaunchND &L)
{
    if (L.kind == kPassSep || L.apply_open || !nd_fixed_shape(L.n, L.axis, kThreadsND)) return hipErrorInvalidValue;
    return L.c64 ? launch_coupled_store<float2>(L) : launch_coupled_store<double2>(L);
}

}  // namespace hfgpe
