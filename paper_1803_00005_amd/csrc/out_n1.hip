// Output kernels for n = 1 guidance channels (all compiled radii).
#include "out.hpp"

namespace hgf {
hipError_t launch_out_n1(const OutLaunch& a, hipStream_t s) { return out_launch_n<1>(a, s); }
}  // namespace hgf
