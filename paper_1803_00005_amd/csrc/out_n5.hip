// Output kernels for n = 5 guidance channels (all compiled radii).
#include "out.hpp"

namespace hgf {
hipError_t launch_out_n5(const OutLaunch& a, hipStream_t s) { return out_launch_n<5>(a, s); }
}  // namespace hgf
