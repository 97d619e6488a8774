// The pass kernels instantiated with the chirp-z (Bluestein) FFT, for axes whose plan carries a
// convolution length m > 0 (lengths with large prime factors).  A translation unit of its own so
// that it compiles beside kernels.hip; the launchers there route chirp-z plans here.
#include "pass_kernels.h"

namespace fh {

hipError_t launch_xfwd_chirp(int prod, int mat, const XFwdArgs& a, dim3 grid, size_t sm, hipStream_t s) {
  return dispatch_xfwd<kChirp>(prod, mat, a, grid, sm, s);
}
hipError_t launch_xinv_chirp(int cons, const XInvArgs& a, dim3 grid, size_t sm, hipStream_t s) {
  return dispatch_xinv<kChirp>(cons, a, grid, sm, s);
}
hipError_t launch_mid_chirp(int dir, bool rows, const AxisArgs& a, dim3 grid, size_t sm, hipStream_t s) {
  return dispatch_mid<kChirp>(dir, rows, a, grid, sm, s);
}
hipError_t launch_outer_chirp(int mode, bool rows, const AxisArgs& a, dim3 grid, size_t sm, hipStream_t s) {
  return dispatch_outer<kChirp>(mode, rows, a, grid, sm, s);
}
hipError_t set_smem_limits_chirp(const Geom& g, int mat, size_t bytes) { return pass_smem_limits<kChirp>(g, mat, bytes); }

}  // namespace fh
