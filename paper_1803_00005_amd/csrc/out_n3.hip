// Output kernels for n = 3 guidance channels (all compiled radii).
#include "out.hpp"

namespace hgf {
hipError_t launch_out_n3(const OutLaunch& a, hipStream_t s) { return out_launch_n<3>(a, s); }
}  // namespace hgf
