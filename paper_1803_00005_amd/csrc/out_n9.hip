// Output kernels for n = 9 guidance channels (all compiled radii).
#include "out.hpp"

namespace hgf {
hipError_t launch_out_n9(const OutLaunch& a, hipStream_t s) { return out_launch_n<9>(a, s); }
}  // namespace hgf
