// Host-only stand-ins for the device launchers of lbm_kernels.hip, for the sanitizer
// build of the library's host code (validation, derived constants, thermodynamics,
// batch bookkeeping).  Every launcher reports that no device is present; the size
// queries return the real sizes of the types they describe.
#include <hip/hip_runtime.h>

#include "lbm_internal.hpp"

namespace lbm_dev {

hipError_t launch_init(int, const void*, void*, const double*, const double*, const double*, const double*, int,
                       hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_step_ab(int, const void*, const void*, void*, LaunchShape, bool, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_step_aa(int, const void*, void*, double*, int, LaunchShape, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_density(int, const void*, const void*, int, double*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_moments(int, const void*, const void*, int, const double*, double*, double*, double*,
                          hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_invariants(int, const void*, const void*, int, const double*, double*, double*, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_step_ab_batch(int, const void*, const int32_t*, unsigned*, uint32_t*, int, int, int, BatchLaunch,
                                bool, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_step_bounded(int, const void*, const void*, void*, void*, int, int, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_moments_bounded(int, const void*, const void*, const void*, double*, double*, double*, double*,
                                  hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_invariants_bounded(int, const void*, const void*, const void*, double*, hipStream_t) {
    return hipErrorNoDevice;
}
int batch_blocks_per_cu(int, int, int, bool) { return 1; }
size_t batch_desc_size(int prec) { return prec == kF64 ? sizeof(BatchDesc<double>) : sizeof(BatchDesc<float>); }
size_t consts_size(int prec) { return prec == kF64 ? sizeof(Consts<double>) : sizeof(Consts<float>); }
size_t storage_bytes(int prec) { return prec == kF64 ? 8 : (prec == kF32 ? 4 : 2); }

}  // namespace lbm_dev
