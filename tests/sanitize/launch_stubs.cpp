// Host-only stand-ins for the kernel launchers (kernels.hip) and the device scratch lookup
// (noalloc_scratch.hip), so that the host driver links without device code.  None is reached by
// host_driver.cpp, whose calls all return before any launch; each would report that no device
// code is present.
#include "kernels.h"

namespace fh {

hipError_t launch_xfwd(int, int, const XFwdArgs&, int, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_xinv(int, const XInvArgs&, int, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_mid(int, const AxisArgs&, int, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_outer(int, const AxisArgs&, int, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_cg_reduce(int, CgState*, const double*, int, int, hipStream_t, const int*) { return hipErrorNoBinaryForGpu; }
hipError_t launch_cg_finish(double*, const double*, const CgState*, const Geom&, int, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_init_reference(double*, const Geom&, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_shift(double*, const double*, const Geom&, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_update(double*, const double*, double*, int, const Geom&, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_homogenize(int, const double*, MatParams, double*, int, const Geom&, CgState*, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_tangent_matrix(int, const double*, const double*, const double*, MatParams, double*, int, const Geom&, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_reduce_slots(const double*, int, int, double*, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_store_tangent(int, const double*, MatParams, double*, const Geom&, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_expand(const double*, double*, const Geom&, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_pack(const double*, double*, const Geom&, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_stress_field(int, const double*, MatParams, double*, double*, const Geom&, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_simp_scale(const double*, double, double*, long long, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_plan_tables(AxisPlan*, double2*, hipStream_t, bool) { return hipErrorNoBinaryForGpu; }
hipError_t launch_check_phase(const uint8_t*, long long, int, int*, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_debug_constitutive(int, const double*, const double*, double*, double*, double*, MatParams, const Geom&, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_simp_gradient(int, const double*, const double*, MatParams, const double*, double, const double*, double, double*, const Geom&, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_j2_commit(int, const double*, MatParams, double*, const Geom&, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_j2_plastic(int, const double*, MatParams, double*, const Geom&, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t set_smem_limits(const Geom&, int, size_t) { return hipErrorNoBinaryForGpu; }
hipError_t noalloc_scratch_address(void**) { return hipErrorNoBinaryForGpu; }

}  // namespace fh
