// Coefficient kernels for n = 8 guidance channels (all compiled radii, both
// regularisation forms, float32 and bfloat16 cost).
#include "coef.hpp"

namespace hgf {
hipError_t launch_coef_n8(const CoefLaunch& a, hipStream_t s) { return coef_launch_n<8>(a, s); }
}  // namespace hgf
