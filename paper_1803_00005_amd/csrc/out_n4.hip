// Output kernels for n = 4 guidance channels (all compiled radii).
#include "out.hpp"

namespace hgf {
hipError_t launch_out_n4(const OutLaunch& a, hipStream_t s) { return out_launch_n<4>(a, s); }
}  // namespace hgf
