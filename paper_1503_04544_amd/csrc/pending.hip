// Entry points whose device implementation is not part of this library build
// yet: they report an error instead of computing anything.
#include <hip/hip_runtime.h>

#include "ccdvm_impl.h"

namespace ccdvm {

bool regular_supported_3d(int) { return false; }
hipError_t build_geometry_3d(cc_ctx*) { return hipErrorNotSupported; }
hipError_t launch_init_maxwellian_3d(cc_ctx*) { return hipErrorNotSupported; }
hipError_t launch_load_state_3d(cc_ctx*, const double*) { return hipErrorNotSupported; }
hipError_t launch_store_state_3d(const cc_ctx*, double*) { return hipErrorNotSupported; }
hipError_t launch_merge_3d(cc_ctx*) { return hipErrorNotSupported; }
hipError_t launch_moments_all_3d(cc_ctx*) { return hipErrorNotSupported; }
hipError_t launch_step_3d(cc_ctx*, double*, double*) { return hipErrorNotSupported; }
hipError_t launch_mass_3d(cc_ctx*, double*) { return hipErrorNotSupported; }
hipError_t launch_moments_out_3d(cc_ctx*, double*) { return hipErrorNotSupported; }
hipError_t launch_force_only_3d(cc_ctx*, double*) { return hipErrorNotSupported; }

}  // namespace ccdvm
