// Launch geometry of the CG passes: LDS bytes, sequences per FFT call, tile limits and
// register-staging capacity for a launch shape.  Host-only C++ (no device code): the host driver
// sizes and validates launch shapes with it, the kernel launchers use the same functions.
#include <algorithm>
#include <cstddef>

#include "kernels.h"

namespace fh {

size_t xfwd_smem(const Geom& g, int R, int inplace) {
  const int P = (g.c * R + 1) / 2;
  const size_t fft = (inplace ? 1ull : 2ull) * g.nx * P * sizeof(double2);
  const size_t stage = (size_t)R * g.nx * g.c * sizeof(double);
  return fft + stage;
}
size_t xinv_smem(const Geom& g, int R, int inplace) {
  const int P = (g.c * R + 1) / 2;
  const size_t a = (size_t)g.nx * P;
  size_t bsz = inplace ? 0 : (size_t)g.nx * P;
  const size_t h = (size_t)g.nxh * g.c * R;
  if (h > bsz) bsz = h;
  return (a + bsz) * sizeof(double2);
}
int mid_sequences(const Geom& g, int TX, int ZB, int proj) {
  (void)proj;  // the row-wise finite-strain y pass transforms one component tile at a time
  return kx_tile_max(g.nxh, TX) * ZB;
}
bool mid_fits(const Geom& g, int TX, int ZB, int proj) {
  return !(proj && finite_rows(g)) || (long long)g.ny * kx_tile_max(g.nxh, TX) * ZB <= (long long)kFrowHeld * kThreads;
}
size_t mid_smem(const Geom& g, int TX, int inplace, int ZB, int proj) {
  return (inplace ? 1ull : 2ull) * g.ny * mid_sequences(g, TX, ZB, proj) * sizeof(double2);
}
int mid_planes(const Geom& g, const AxisPlan& pl, int TX, int inplace, long long B, int proj) {
  if (g.ndim != 3 || kx_tiles(g.nxh, TX) > 1) return 1;
  constexpr size_t kLdsPlanes = 32 * 1024;
  constexpr long long kBlocks = 512;
  const int per_rhs = proj && finite_rows(g) ? 3 : g.c;
  int zb = 1;
  for (int z = 2; z <= std::min(8, g.nz); ++z) {
    if (mid_smem(g, TX, inplace, z, proj) > kLdsPlanes || !mid_fits(g, TX, z, proj)) break;
    if (inplace && !inplace_ok(pl, mid_sequences(g, TX, z, proj))) break;
    if ((long long)((g.nz + z - 1) / z) * per_rhs * B < kBlocks) break;
    zb = z;
  }
  return zb;
}
// Projection: small strain couples all Mandel components of a wavevector; finite strain projects
// each row of F on its own -- in 3D the row arrives as two components (see k_outer_frow), in 2D
// as its two entries.  Plain transforms (debug FFTs) take whole rows (finite) or all components.
int outer_group(const Geom& g, int mode) {
  if (g.small) return g.c;
  return (mode == OUTER_PROJECT && g.ndim == 3) ? 2 : g.ndim;
}
int outer_groups_per_rhs(const Geom& g, int mode) {
  (void)mode;  // rows of F (finite strain) or one group of all components (small strain)
  return g.small ? 1 : g.ndim;
}
size_t outer_smem(const Geom& g, int TX, int inplace, int mode) {
  return (size_t)(outer_group(g, mode) * (inplace ? 1 : 2)) * g.n_outer * kx_tile_max(g.nxh, TX) * sizeof(double2);
}
bool outer_inplace_ok(const Geom& g, const AxisPlan& pl, int TX, int mode) {
  return inplace_ok(pl, outer_group(g, mode) * kx_tile_max(g.nxh, TX));
}
bool inplace_ok(const AxisPlan& pl, int nseq) {
  for (int st = 0; st < pl.nstages; ++st) {
    const int R = pl.radix[st];
    if (R != 2 && R != 3 && R != 4 && R != 5 && R != 8 && R != 16) return false;
    const long long total = (long long)nseq * (pl.n / R);
    const long long per_thread = (total + kThreads - 1) / kThreads;
    if (per_thread > kInplaceElems / R) return false;
  }
  return true;
}

}  // namespace fh
