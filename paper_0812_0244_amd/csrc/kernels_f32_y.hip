// Axis-2 passes of the FP32 evaluation, every length class and radix order (see
// kernels.hpp).
#include "kernels.hpp"

namespace vdwnl {

hipError_t launch_y_f32(int kind, int lc, int var, const LaunchArgs &a) {
    VDWNL_LC_VARIANTS(launch_y_lc, float, kind, lc, var, a)
}

}  // namespace vdwnl
