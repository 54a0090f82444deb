// Device launchers for the host-only sanitizer build (test infrastructure):
// a context on device -1 never launches, so each returns an error.
#include "../../paper_0812_0244_amd/csrc/common.hpp"

namespace vdwnl {
hipError_t launch_kind(int, int, int, const LaunchArgs &) { return hipErrorNoDevice; }
hipError_t launch_probe(int, int, int, const LaunchArgs &, void *, int) { return hipErrorNoDevice; }
hipError_t launch_reduce(const InstDev *, int, double *, hipStream_t) { return hipErrorNoDevice; }
}  // namespace vdwnl
