// The kernels of the FP32 evaluation (see kernels.hpp).
#include "kernels.hpp"

namespace vdwnl {

hipError_t launch_kind_f32(int kind, int lc, const LaunchArgs &a) { return launch_kind_t<float>(kind, lc, a); }

hipError_t launch_probe_f32(int probe, int lc, const LaunchArgs &a, void *dst, int target) {
    return launch_probe_t<float>(probe, lc, a, dst, target);
}

}  // namespace vdwnl
