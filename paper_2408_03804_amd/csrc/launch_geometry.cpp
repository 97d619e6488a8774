// Launch geometry of the CG passes: LDS bytes, sequences per FFT call, tile limits and
// register-staging capacity for a launch shape.  Host-only C++ (no device code): the host driver
// sizes and validates launch shapes with it, the kernel launchers use the same functions.
#include <algorithm>
#include <cstddef>
#include <initializer_list>

#include "kernels.h"

namespace fh {

size_t xfwd_smem(const Geom& g, int R, int inplace) {
  const int P = (g.c * R + 1) / 2;
  const size_t fft = (inplace ? 1ull : 2ull) * g.lx * P * sizeof(double2);
  const size_t stage = (size_t)R * g.nx * g.c * sizeof(double);
  return fft + stage;
}
size_t xinv_smem(const Geom& g, int R, int inplace) {
  const int P = (g.c * R + 1) / 2;
  const size_t a = (size_t)g.lx * P;
  size_t bsz = inplace ? 0 : (size_t)g.lx * P;
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
  return (inplace ? 1ull : 2ull) * g.lm * mid_sequences(g, TX, ZB, proj) * sizeof(double2);
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
  return (size_t)(outer_group(g, mode) * (inplace ? 1 : 2)) * g.lo * kx_tile_max(g.nxh, TX) * sizeof(double2);
}
bool outer_inplace_ok(const Geom& g, const AxisPlan& pl, int TX, int mode) {
  return inplace_ok(pl, outer_group(g, mode) * kx_tile_max(g.nxh, TX));
}
bool inplace_ok(const AxisPlan& pl, int nseq) {
  for (int st = 0; st < pl.nstages; ++st) {
    const int R = pl.radix[st];
    if (R != 2 && R != 3 && R != 4 && R != 5 && R != 8 && R != 16) return false;
    const long long total = (long long)nseq * (lds_len(pl) / R);
    const long long per_thread = (total + kThreads - 1) / kThreads;
    if (per_thread > kInplaceElems / R) return false;
  }
  return true;
}


// Factor n into Stockham radices: the compiled schedule for its length, else 8, 4, 2 for the
// power of two, then 3, 5 and any remaining prime factor (direct DFT stage).
bool factorize(int n, int* radix, int* nst) {
  if (fixed_nstages(n) > 0) {
    *nst = fixed_nstages(n);
    for (int st = 0; st < *nst; ++st) radix[st] = fixed_radix(n, st);
    return true;
  }
  int k = 0;
  int m = n;
  while (m % 8 == 0 && k < kMaxStages) { radix[k++] = 8; m /= 8; }
  while (m % 4 == 0 && k < kMaxStages) { radix[k++] = 4; m /= 4; }
  while (m % 2 == 0 && k < kMaxStages) { radix[k++] = 2; m /= 2; }
  for (int p = 3; m > 1 && k < kMaxStages; p += 2) {
    while (m % p == 0 && k < kMaxStages) { radix[k++] = p; m /= p; }
  }
  *nst = k;
  return m == 1;
}

// smallest length >= 2n - 1 whose only prime factors are 2, 3 and 5
static int chirp_len(int n) {
  for (int m = 2 * n - 1;; ++m) {
    int q = m;
    for (int p : {2, 3, 5})
      while (q % p == 0) q /= p;
    if (q == 1) return m;
  }
}
constexpr int kMaxChirpLen = 2048;

bool make_plan(int n, AxisPlan* pl, int chirp_above) {
  pl->n = n;
  pl->m = 0;
  pl->tw = pl->chirp = pl->filt = nullptr;
  int rad[kMaxStages], ns = 0;
  const bool ok = factorize(n, rad, &ns);
  int direct = ok ? 0 : 1 << 30;  // sum of the direct stages' prime lengths
  for (int st = 0; st < ns; ++st)
    if (rad[st] != 2 && rad[st] != 3 && rad[st] != 4 && rad[st] != 5 && rad[st] != 8 && rad[st] != 16) direct += rad[st];
  if (chirp_above > 0 && direct > chirp_above) {
    const int m = chirp_len(n);
    int mrad[kMaxStages], mns = 0;
    if (m <= kMaxChirpLen && factorize(m, mrad, &mns)) {
      pl->m = m;
      pl->nstages = mns;
      for (int st = 0; st < mns; ++st) pl->radix[st] = mrad[st];
      return true;
    }
  }
  if (!ok) return false;
  pl->nstages = ns;
  for (int st = 0; st < ns; ++st) pl->radix[st] = rad[st];
  return true;
}

size_t plan_table_elems(const AxisPlan& pl) { return (size_t)lds_len(pl) + (pl.m > 0 ? (size_t)pl.n + pl.m : 0); }

void set_lds_lens(Geom* g, const AxisPlan* pl) {
  g->lx = lds_len(pl[0]);
  g->lm = g->ndim == 3 ? lds_len(pl[1]) : 1;
  g->lo = lds_len(pl[g->ndim - 1]);
}

}  // namespace fh
