// Coefficient kernels for n = 9 guidance channels (all compiled radii, both
// regularisation forms, float32 and bfloat16 cost).
#include "coef.hpp"

namespace hgf {
hipError_t launch_coef_n9(const CoefLaunch& a, hipStream_t s) { return coef_launch_n<9>(a, s); }
}  // namespace hgf
