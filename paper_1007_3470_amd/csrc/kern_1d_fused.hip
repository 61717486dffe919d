// kern_1d_fused.hip -- the fixed-shape resident 1-D step kernel with the
// stage records evaluated inside the kernel (hf1d_fixed.hpp), one instance
// per HO rule and storage type.
#include <hip/hip_runtime.h>

#include "hf1d_fixed.hpp"

namespace hfgpe {

template <typename Store>
static hipError_t launch_fused_rule(const Launch1D &L)
{
    switch (L.coef_rule) {
    case 0: return launch_hf1d_fixed<Store, 0>(L);
    case 1: return launch_hf1d_fixed<Store, 1>(L);
    case 2: return launch_hf1d_fixed<Store, 2>(L);
    case 3: return launch_hf1d_fixed<Store, 3>(L);
    case 4: return launch_hf1d_fixed<Store, 4>(L);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_hf1d_fused(const Launch1D &L)
{
    if (L.n_items <= 0) return hipSuccess;
    if (!L.fixed || L.P != 8 || !L.scheme || !L.err) return hipErrorInvalidValue;
    if (L.c64) return launch_fused_rule<float2>(L);
    return launch_fused_rule<double2>(L);
}

}  // namespace hfgpe
