// Host driver of the C ABI declared in include/fft_homog.h.
//
// Owns no device memory: every buffer is a slice of the caller's workspace.
// All kernels run on the stream given at create time; the host reads back only
// the small per-right-hand-side CG records (every few CG iterations) and the
// reduced scalars of the Newton loop.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fft_homog.h"
#include "common.h"
#include "kernels.h"

using namespace fh;


namespace {

constexpr size_t kAlign = 256;
constexpr int kResults = 128;
constexpr int kChunk = 8;          // CG iterations enqueued between host checks
constexpr int kTimedLaunches = 7;  // launches of one CG iteration (kernel timing)
constexpr size_t kLdsFft = 48 * 1024;
constexpr size_t kLdsOuter = 64 * 1024;
constexpr size_t kLdsMax = 160 * 1024;
constexpr int kOuterTileMax = 4;   // kx bins per outer-pass block (measured best at 128^3)
constexpr long long kBlocksTarget = 512;  // blocks per pass the default tiles aim for (2 per CU)

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
// work-vector stagger candidates and the room reserved for them (stagger s moves x, r, p and the
// half spectrum by s, 2 s, 3 s and 4 s bytes)
constexpr size_t kPlaceSlack = 16u << 20;
constexpr size_t kStaggers[] = {0, 256, 16u << 10, 256u << 10, 2u << 20, 4u << 20};

int ncomp_of(int kin, int ndim) { return kin == FFT_HOMOG_SMALL_STRAIN ? (ndim == 3 ? 6 : 3) : ndim * ndim; }

struct Layout {
  size_t F, x, r, p, spec, kst, phase, density, scale, table, hist, tw[3], partials, state, active, results, flags,
      total;
  size_t slack;  // bytes behind the spectrum that the work vectors may be staggered into
  int cells;  // independent cells (microstructures) of this grid held by the handle
  int B, R, TXm, TXo, nblk_x, nblk_vox;
  size_t n_results;
  int in_x, in_m, in_o;  // in-place (register-staged) FFT per pass
  size_t n_partials, smem_max;
  bool chirp;  // axes with large prime factors use the chirp-z transform (else direct stages)
};

// Chirp-z thresholds (sum of the direct stages' prime lengths above 5, see make_plan), measured per
// pass from CG-iteration kernel times on MI355X with both forms, lengths 31 to 511 in 2D and 3D:
// the outer pass (G-hat between a forward and an inverse transform) gains from 80 (511 = 7 * 73)
// and 97 on and loses at 61 and at 36 (299 = 13 * 23); the x passes break even at 127 and gain
// at 199, the y pass loses at 97.  The x and y passes hold more sequences per block, which the
// chirp-z buffers (about twice the axis length) crowd out.
constexpr int kChirpOuter = 70;
constexpr int kChirpRows = 150;

// FFT plans of the axes of d (pl[2] = pl[1] in 2D) and the LDS lengths of g that follow from them.
bool make_plans(const fft_homog_desc* d, bool chirp, AxisPlan* pl, Geom* g) {
  for (int a = 0; a < 3; ++a) {
    const int lim = !chirp ? 0 : a == d->ndim - 1 ? kChirpOuter : kChirpRows;
    if (!make_plan(a < d->ndim ? d->n[a] : 1, &pl[a], lim)) return false;
  }
  if (d->ndim == 2) pl[2] = pl[1];
  set_lds_lens(g, pl);
  return true;
}

bool make_geom(const fft_homog_desc* d, Geom* g) {
  g->ndim = d->ndim;
  g->c = ncomp_of(d->kinematics, d->ndim);
  g->nx = d->n[0];
  g->ny = d->n[1];
  g->nz = d->ndim == 3 ? d->n[2] : 1;
  g->nxh = g->nx / 2 + 1;
  g->nxp = g->nxh >= 8 ? (g->nxh + 7) / 8 * 8 : g->nxh;
  g->lx = g->nx;  // direct stages until make_plans sets the plans' LDS lengths
  g->lm = d->ndim == 3 ? g->ny : 1;
  g->lo = d->ndim == 3 ? g->nz : g->ny;
  g->n_outer = d->ndim == 3 ? g->nz : g->ny;
  g->n_mid = d->ndim == 3 ? g->ny : 1;
  g->N = (long long)g->nx * g->ny * g->nz;
  g->Nh = (long long)g->nxp * g->ny * g->nz;
  const double twopi = 6.283185307179586476925286766559;
  for (int a = 0; a < 3; ++a) g->ks[a] = (a < d->ndim) ? twopi / d->len[a] : 0.0;
  g->small = d->kinematics == FFT_HOMOG_SMALL_STRAIN;
  return true;
}

// kernel material code: 2 * material + (ndim - 2); Neo-Hookean and J2 under plane stress have laws
// of their own (8, 9), linear elasticity and St. Venant-Kirchhoff under plane stress are their 2D
// laws with a reduced first Lame parameter (set_material converts the table)
static int material_code(const fft_homog_desc* d) {
  if ((d->flags & FFT_HOMOG_FLAG_PLANE_STRESS) && d->material == FFT_HOMOG_NEO_HOOKEAN) return 8;
  if ((d->flags & FFT_HOMOG_FLAG_PLANE_STRESS) && d->material == FFT_HOMOG_J2_PLASTIC) return 9;
  return 2 * d->material + (d->ndim - 2);
}

int validate_desc(const fft_homog_desc* d) {
  if (!d) return FFT_HOMOG_EINVAL;
  if (d->ndim != 2 && d->ndim != 3) return FFT_HOMOG_EINVAL;
  for (int a = 0; a < d->ndim; ++a) {
    if (d->n[a] < 1) return FFT_HOMOG_EINVAL;
    if (!(d->len[a] > 0.0) || !std::isfinite(d->len[a])) return FFT_HOMOG_EINVAL;
    if (d->n[a] > kMaxAxis) return FFT_HOMOG_EUNSUPPORTED;
  }
  if (d->kinematics != FFT_HOMOG_SMALL_STRAIN && d->kinematics != FFT_HOMOG_FINITE_STRAIN) return FFT_HOMOG_EINVAL;
  if (d->kinematics == FFT_HOMOG_SMALL_STRAIN && d->material != FFT_HOMOG_LINEAR_ELASTIC &&
      d->material != FFT_HOMOG_J2_PLASTIC)
    return FFT_HOMOG_EINVAL;
  if (d->material == FFT_HOMOG_J2_PLASTIC && (d->batch > 1 || (d->flags & FFT_HOMOG_FLAG_DENSITY)))
    return FFT_HOMOG_EINVAL;
  if (d->kinematics == FFT_HOMOG_FINITE_STRAIN && d->material != FFT_HOMOG_NEO_HOOKEAN &&
      d->material != FFT_HOMOG_STVK)
    return FFT_HOMOG_EINVAL;
  if (d->nphase < 1 || d->nphase > kMaxPhase) return FFT_HOMOG_EINVAL;
  if (!(d->tol_newton > 0.0) || !(d->tol_cg > 0.0)) return FFT_HOMOG_EINVAL;
  if (d->max_newton < 0 || d->max_cg < 0) return FFT_HOMOG_EINVAL;
  if (d->k_mode != FFT_HOMOG_K_RECOMPUTE && d->k_mode != FFT_HOMOG_K_STORED) return FFT_HOMOG_EINVAL;
  if (d->batch < 0) return FFT_HOMOG_EINVAL;
  if (d->flags & ~(FFT_HOMOG_FLAG_TANGENT | FFT_HOMOG_FLAG_DENSITY | FFT_HOMOG_FLAG_GRAPH | FFT_HOMOG_FLAG_PLANE_STRESS))
    return FFT_HOMOG_EINVAL;
  if ((d->flags & FFT_HOMOG_FLAG_PLANE_STRESS) && d->ndim != 2) return FFT_HOMOG_EINVAL;
  if (d->batch > 1) {
    // a multi-cell handle runs the tangent solves of every cell at the reference state
    if (!(d->flags & FFT_HOMOG_FLAG_TANGENT)) return FFT_HOMOG_EINVAL;
    if (d->flags & FFT_HOMOG_FLAG_DENSITY) return FFT_HOMOG_EINVAL;
    if (d->k_mode != FFT_HOMOG_K_RECOMPUTE) return FFT_HOMOG_EINVAL;
    const long long C = ncomp_of(d->kinematics, d->ndim);
    // grid limits of the batched launches (B * c blocks along z of the spectral passes)
    if ((long long)d->batch * C * C > 65535) return FFT_HOMOG_EUNSUPPORTED;
  }
  return FFT_HOMOG_OK;
}

// Largest dynamic LDS of any pass at the launch shape of L: the projection chain's y and outer
// kernels, and the plain transforms of the stage-level FFT entry points (which may carry more
// components per block and fall back to the ping-pong buffer).
size_t smem_needed(const Geom& g, const AxisPlan* pl, const Layout& L) {
  size_t m = std::max(xfwd_smem(g, L.R, L.in_x), xinv_smem(g, L.R, L.in_x));
  if (g.ndim == 3) {
    m = std::max(m, mid_smem(g, L.TXm, L.in_m, mid_planes(g, pl[1], L.TXm, L.in_m, L.B, 1), 1));
    m = std::max(m, mid_smem(g, L.TXm, L.in_m, mid_planes(g, pl[1], L.TXm, L.in_m, L.B, 0), 0));
  }
  m = std::max(m, outer_smem(g, L.TXo, L.in_o, OUTER_PROJECT));
  // plain transforms narrow their tile to 64 KiB of LDS, down to one bin
  m = std::max(m, std::min(outer_smem(g, L.TXo, 0, OUTER_FWD), std::max((size_t)64 * 1024, outer_smem(g, 1, 0, OUTER_FWD))));
  return m;
}

int make_layout_with(const fft_homog_desc* d, Layout* L, bool chirp) {
  Geom g;
  make_geom(d, &g);
  const int C = g.c;
  AxisPlan pl[3];
  if (!make_plans(d, chirp, pl, &g)) return FFT_HOMOG_EUNSUPPORTED;
  L->chirp = chirp;
  L->cells = d->batch > 1 ? d->batch : 1;
  L->B = (d->flags & FFT_HOMOG_FLAG_TANGENT) ? C * L->cells : 1;
  const AxisPlan& pouter = pl[d->ndim - 1];
  const int rows = g.ny * g.nz;
  // Default tiles: as large as the LDS budget allows, but small enough that each pass still
  // launches about kBlocksTarget blocks at the handle's typical batch (one right-hand side, or
  // all of a multi-cell handle's) -- small grids otherwise leave most of the 256 CUs idle.
  const long long Bd = L->cells > 1 ? L->B : 1;
  auto par_cap = [&](long long work_per_unit, int hi) {
    return (int)std::max(1LL, std::min((long long)hi, work_per_unit * Bd / kBlocksTarget));
  };
  // x pass: rows per block, aiming at one or two voxels per thread
  int rmax = std::max(1, std::min(16, (2 * kThreads + g.nx - 1) / g.nx));
  rmax = std::min(rmax, par_cap(rows, rmax));
  int R = 0, inx = 0;
  for (int r = rmax; r >= 1; --r) {
    if (r > rows && r > 1) continue;
    const int P = (C * r + 1) / 2;
    const int ip = inplace_ok(pl[0], P) ? 1 : 0;
    if (xfwd_smem(g, r, ip) <= kLdsFft && xinv_smem(g, r, ip) <= kLdsFft) { R = r; inx = ip; break; }
  }
  if (R == 0) {
    const int P = (C + 1) / 2;
    inx = inplace_ok(pl[0], P) ? 1 : 0;
    if (xfwd_smem(g, 1, inx) <= kLdsMax && xinv_smem(g, 1, inx) <= kLdsMax) R = 1;
    else return FFT_HOMOG_EUNSUPPORTED;
  }
  L->R = R;
  L->in_x = inx;
  // y pass: sized for the projection chain's kernel (row-wise for finite strain 3D: three
  // components per block)
  const int ypr = finite_rows(g) ? 3 : C;
  int TXm = 0, inm = 0;
  for (int t = par_cap((long long)g.nxh * g.nz * ypr, 16); t >= 1; --t) {
    if (t > g.nxh && t > 1) continue;
    const int ip = inplace_ok(pl[1], mid_sequences(g, t, 1, 1)) ? 1 : 0;
    if (mid_smem(g, t, ip, 1, 1) <= kLdsFft && mid_fits(g, t, 1, 1)) { TXm = t; inm = ip; break; }
  }
  if (TXm == 0) {
    TXm = 1;
    inm = inplace_ok(pl[1], mid_sequences(g, 1, 1, 1)) ? 1 : 0;
    if (mid_smem(g, 1, inm, 1, 1) > kLdsMax || !mid_fits(g, 1, 1, 1)) return FFT_HOMOG_EUNSUPPORTED;
  }
  L->TXm = TXm;
  L->in_m = inm;
  // outer tile: the finite-strain row-wise projection moves two components per block and takes
  // whole 128-byte lines (8 bins); the other outer passes take 4 bins
  const int otmax = finite_rows(g) ? 2 * kOuterTileMax : kOuterTileMax;
  int TXo = 0, ino = 0;
  for (int t = par_cap((long long)g.nxh * g.n_mid * outer_groups_per_rhs(g), otmax); t >= 1; --t) {
    if (t > g.nxh && t > 1) continue;
    const int ip = outer_inplace_ok(g, pouter, t) ? 1 : 0;
    if (t <= otmax && outer_smem(g, t, ip) <= kLdsOuter) { TXo = t; ino = ip; break; }
  }
  if (TXo == 0) {
    TXo = 1;
    ino = outer_inplace_ok(g, pouter, 1) ? 1 : 0;
    if (outer_smem(g, 1, ino) > kLdsMax) return FFT_HOMOG_EUNSUPPORTED;
  }
  L->TXo = TXo;
  L->in_o = ino;
  L->smem_max = smem_needed(g, pl, *L);
  L->nblk_x = (rows + R - 1) / R;
  L->nblk_vox = (int)((g.N + kThreads - 1) / kThreads);

  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const size_t fld = (size_t)C * g.N * sizeof(double);
  L->F = take(fld);
  L->x = take(fld * L->B);
  L->r = take(fld * L->B);
  L->p = take(fld * L->B);
  L->spec = take((size_t)L->B * C * g.Nh * sizeof(double2));
  // On large grids the work vectors get room to be staggered (fft_homog_tune_placement): F, x, r
  // and p sit at multiples of the component size from one another, and their relative placement
  // moves the x pass's time (measured: 180-232 us at 128^3 for the same kernels)
  L->slack = fld >= (64u << 20) ? kPlaceSlack : 0;
  take(L->slack);
  L->kst = take(d->k_mode == FFT_HOMOG_K_STORED ? (size_t)C * (C + 1) / 2 * g.N * sizeof(double) : 0);
  L->phase = take((size_t)L->cells * g.N);
  L->density = take((d->flags & FFT_HOMOG_FLAG_DENSITY) ? (size_t)g.N * sizeof(double) : 0);
  L->scale = take((d->flags & FFT_HOMOG_FLAG_DENSITY) ? (size_t)g.N * sizeof(double) : 0);
  const bool j2 = d->material == FFT_HOMOG_J2_PLASTIC;
  L->table = take((size_t)L->cells * (j2 ? 4 : 2) * kMaxPhase * sizeof(double));
  L->hist = take(j2 ? (size_t)(C + 1) * g.N * sizeof(double) : 0);
  for (int a = 0; a < 3; ++a) L->tw[a] = take(a < d->ndim ? plan_table_elems(pl[a]) * sizeof(double2) : 0);
  // room for one partial per row, so that any x-pass block height fits (launch-shape tuning)
  size_t np = (size_t)L->B * rows;
  np = std::max(np, (size_t)C * C * L->nblk_vox);
  np = std::max(np, (size_t)(C + 1) * L->nblk_vox);
  L->n_partials = np;
  L->partials = take(np * sizeof(double));
  L->state = take((size_t)L->B * sizeof(CgState));
  L->active = take((size_t)L->B * sizeof(int));
  L->n_results = std::max((size_t)kResults, (size_t)L->cells * C * C);
  L->results = take(L->n_results * sizeof(double));
  L->flags = take(16 * sizeof(int));
  L->total = off;
  return FFT_HOMOG_OK;
}

// Chirp-z plans where they cost less; the direct stages if the chirp-z buffers do not fit LDS.
int make_layout(const fft_homog_desc* d, Layout* L) {
  const int rc = validate_desc(d);
  if (rc) return rc;
  if (make_layout_with(d, L, true) == FFT_HOMOG_OK) return FFT_HOMOG_OK;
  return make_layout_with(d, L, false);
}

// out = G*in for `batch` packed fields: the x pass (real-to-complex), the y pass, the outer pass
// with G-hat and its inverse, the inverse y pass and the complex-to-real x pass, with the launch
// shape of L, the grid g (g.nxp: the spectrum pitch in use) and `spec` as the half spectrum.
// Enqueue only.  Shared by the handle's debug_project and the allocation-free projection.
hipError_t enqueue_projection(const Geom& g, const AxisPlan* pl, const Layout& L, int matcode, const double* in,
                              double* out, double2* spec, int batch, hipStream_t s) {
  XFwdArgs a;
  memset(&a, 0, sizeof(a));
  a.g = g;
  a.px = pl[0];
  a.R = L.R;
  a.nblocks = (g.ny * g.nz + L.R - 1) / L.R;
  a.inplace = L.in_x;
  a.in = in;
  a.spec = spec;
  hipError_t e = launch_xfwd(PROD_IDENT, matcode, a, batch, s);
  auto axis = [&](int ax, int TX, int inplace) {
    AxisArgs x;
    memset(&x, 0, sizeof(x));
    x.g = g;
    x.pl = pl[ax];
    x.TX = TX;
    x.inplace = inplace;
    x.proj = 1;
    x.ZB = (ax == 1 && g.ndim == 3) ? mid_planes(g, pl[1], TX, inplace, L.B, 1) : 1;
    x.spec = spec;
    return x;
  };
  const AxisArgs am = axis(1, L.TXm, L.in_m);
  const AxisArgs ao = axis(g.ndim - 1, L.TXo, L.in_o);
  if (e == hipSuccess && g.ndim == 3) e = launch_mid(-1, am, batch, s);
  if (e == hipSuccess) e = launch_outer(OUTER_PROJECT, ao, batch, s);
  if (e == hipSuccess && g.ndim == 3) e = launch_mid(1, am, batch, s);
  if (e == hipSuccess) {
    XInvArgs ai;
    memset(&ai, 0, sizeof(ai));
    ai.g = g;
    ai.px = pl[0];
    ai.R = L.R;
    ai.nblocks = a.nblocks;
    ai.inplace = L.in_x;
    ai.spec = spec;
    ai.out = out;
    ai.scale = 1.0 / (double)g.N;
    e = launch_xinv(CONS_IDENT, ai, batch, s);
  }
  return e;
}

}  // namespace

struct fft_homog {
  fft_homog_desc desc;
  Geom g;
  Layout L;
  int matcode;
  hipStream_t stream;
  char* ws;
  double *F, *x, *r, *p, *kst, *partials, *results, *table, *density, *scale, *hist;
  bool j2_pending;  // J2: the last converged load step is not yet committed to the history
  double simp_p;
  double2* spec;
  size_t stagger;  // work-vector placement (fft_homog_tune_placement)
  uint8_t* phase;
  int* flags;
  int* active;  // right-hand sides still running, for compacted launches
  CgState* st;
  AxisPlan plan[3];
  MatParams mat;
  double macro_cur[kMaxC];
  bool solved_ok;
  // pinned host mirror of the device records
  CgState* h_st;
  double* h_results;
  int* h_flags;
  int* h_active;
  hipEvent_t ev0, ev1;
  // replayable chunks of CG iterations (FLAG_GRAPH): [0] one right-hand side, [1] the batch
  hipStream_t cap;
  hipGraphExec_t gexec[2];
  int gB[2];
  // sampled kernel timing inside the CG loop (fft_homog_set_kernel_timing): event groups of
  // kTimedLaunches + 1 events recorded since the last host check, and the running sums
  long long host_checks;  // CG-record read-backs of the current call (stats.host_checks)
  int time_every;
  long long time_count;  // CG iterations enqueued eagerly since timing was switched on
  std::vector<hipEvent_t> tev;
  int tev_used;
  double time_acc[kTimedLaunches];
  long long time_samples;
  std::string err;
};

namespace {

// message of the last failed handle-free call on this thread (fft_homog_create, the
// allocation-free projection): no handle exists to hold it; a fixed buffer, so that setting it
// allocates nothing
thread_local char g_create_err[256];

int fail(fft_homog_t* h, int code, const char* msg) {
  if (h) h->err = msg ? msg : "";
  return code;
}

int create_fail(int code, const char* what, hipError_t e) {
  if (e != hipSuccess) snprintf(g_create_err, sizeof(g_create_err), "%s: %s", what, hipGetErrorString(e));
  else snprintf(g_create_err, sizeof(g_create_err), "%s", what);
  return code;
}

#define FH_CK(expr)                                                               \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) return fail(h, FFT_HOMOG_EDEVICE, hipGetErrorString(e_)); \
  } while (0)

XFwdArgs xfwd_args(fft_homog_t* h) {
  XFwdArgs a;
  memset(&a, 0, sizeof(a));
  a.g = h->g;
  a.px = h->plan[0];
  a.R = h->L.R;
  a.nblocks = h->L.nblk_x;
  a.inplace = h->L.in_x;
  a.x = h->x;
  a.F = h->F;
  a.Kst = h->kst;
  a.spec = h->spec;
  a.mat = h->mat;
  a.per_inst = h->L.cells > 1 ? h->g.c : 0;
  a.st = h->st;
  a.partials = h->partials;
  return a;
}

XInvArgs xinv_args(fft_homog_t* h) {
  XInvArgs a;
  memset(&a, 0, sizeof(a));
  a.g = h->g;
  a.px = h->plan[0];
  a.R = h->L.R;
  a.nblocks = h->L.nblk_x;
  a.inplace = h->L.in_x;
  a.spec = h->spec;
  a.x = h->x;
  a.r = h->r;
  a.st = h->st;
  a.partials = h->partials;
  a.scale = 1.0 / (double)h->g.N;
  return a;
}

// proj: the pass belongs to a projection chain (y pass: the row-wise finite-strain kernels)
AxisArgs axis_args(fft_homog_t* h, int axis, int TX, const CgState* st, int inplace = -1, int proj = 1) {
  AxisArgs a;
  a.g = h->g;
  a.pl = h->plan[axis];
  a.TX = TX;
  a.inplace = inplace >= 0 ? inplace : (axis == 1 && h->g.ndim == 3) ? h->L.in_m : h->L.in_o;
  a.proj = proj;
  a.ZB = (axis == 1 && h->g.ndim == 3) ? mid_planes(h->g, h->plan[1], TX, a.inplace, h->L.B, proj) : 1;
  a.spec = h->spec;
  a.st = st;
  a.active = nullptr;
  a.pq_st = nullptr;
  a.pq_partials = nullptr;
  a.pq_nblocks = 0;
  return a;
}

// spectral part shared by every operator application: y, outer (+G-hat), y^-1
hipError_t enqueue_spectral(fft_homog_t* h, int mode, int B, const CgState* st, hipStream_t s,
                            const int* active = nullptr) {
  hipError_t e = hipSuccess;
  AxisArgs am = axis_args(h, 1, h->L.TXm, st, -1, mode == OUTER_PROJECT);
  AxisArgs ao = axis_args(h, h->g.ndim - 1, h->L.TXo, st);
  am.active = ao.active = active;
  if (h->g.ndim == 3 && mode != OUTER_INV) e = launch_mid(-1, am, B, s);
  if (e == hipSuccess) e = launch_outer(mode, ao, B, s);
  if (e == hipSuccess && h->g.ndim == 3 && mode != OUTER_FWD) e = launch_mid(1, am, B, s);
  return e;
}

int spectral_middle(fft_homog_t* h, int mode, int B, const CgState* st) {
  FH_CK(enqueue_spectral(h, mode, B, st, h->stream));
  return FFT_HOMOG_OK;
}

// Next group of kTimedLaunches + 1 events for a sampled CG iteration (created on first use).
hipError_t timing_events(fft_homog_t* h, hipEvent_t** out) {
  const size_t need = (size_t)(h->tev_used + 1) * (kTimedLaunches + 1);
  while (h->tev.size() < need) {
    hipEvent_t ev = nullptr;
    const hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) return e;
    h->tev.push_back(ev);
  }
  *out = h->tev.data() + (size_t)h->tev_used * (kTimedLaunches + 1);
  ++h->tev_used;
  return hipSuccess;
}

// Add the sampled iterations recorded since the last host check to the running sums; the
// stream has been synchronised.
int harvest_timing(fft_homog_t* h) {
  for (int gi = 0; gi < h->tev_used; ++gi) {
    const hipEvent_t* ev = h->tev.data() + (size_t)gi * (kTimedLaunches + 1);
    for (int k = 0; k < kTimedLaunches; ++k) {
      float t = 0.f;
      FH_CK(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
      h->time_acc[k] += t;
    }
    ++h->time_samples;
  }
  h->tev_used = 0;
  return FFT_HOMOG_OK;
}

// Work vectors at stagger s (a multiple of 256 bytes with 4 s within the layout's slack).
void place_work_vectors(fft_homog_t* h, size_t s) {
  h->x = (double*)(h->ws + h->L.x + s);
  h->r = (double*)(h->ws + h->L.r + 2 * s);
  h->p = (double*)(h->ws + h->L.p + 3 * s);
  h->spec = (double2*)(h->ws + h->L.spec + 4 * s);
  h->stagger = s;
}

// m CG iterations, enqueued on stream s, over B launch slots: slot i is right-hand side
// active[i] (active == nullptr: i).  Right-hand sides that stop inside the chunk make
// their blocks return at once.  With kernel timing on (and s the handle's own stream, not a
// graph capture), every time_every-th iteration gets an event before its first launch and
// after each launch.
hipError_t enqueue_cg_iters(fft_homog_t* h, int B, int m, hipStream_t s, const int* active = nullptr) {
  const int prod = h->desc.k_mode == FFT_HOMOG_K_STORED ? PROD_CGOP_STORED : PROD_CGOP;
  XFwdArgs a = xfwd_args(h);
  a.in = h->r;
  a.p = h->p;
  a.active = active;
  XInvArgs ai = xinv_args(h);
  ai.active = active;
  AxisArgs am = axis_args(h, 1, h->L.TXm, h->st);
  AxisArgs ao = axis_args(h, h->g.ndim - 1, h->L.TXo, h->st);
  am.active = ao.active = active;
  ao.pq_st = h->st;
  ao.pq_partials = h->partials;
  ao.pq_nblocks = h->L.nblk_x;
  const bool three = h->g.ndim == 3;
  const bool timing = h->time_every > 0 && s == h->stream;
  hipError_t e = hipSuccess;
  for (int i = 0; i < m && e == hipSuccess; ++i) {
    hipEvent_t* ev = nullptr;
    if (timing && h->time_count++ % h->time_every == 0) e = timing_events(h, &ev);
    int k = 0;
    auto mark = [&]() {
      if (ev && e == hipSuccess) e = hipEventRecord(ev[k++], s);
    };
    mark();
    if (e == hipSuccess) e = launch_xfwd(prod, h->matcode, a, B, s);
    mark();
    mark();  // <p, K:p> is reduced inside the outer pass
    if (e == hipSuccess && three) e = launch_mid(-1, am, B, s);
    mark();
    if (e == hipSuccess) e = launch_outer(OUTER_PROJECT, ao, B, s);
    mark();
    if (e == hipSuccess && three) e = launch_mid(1, am, B, s);
    mark();
    if (e == hipSuccess) e = launch_xinv(CONS_CGUPD, ai, B, s);
    mark();
    if (e == hipSuccess) e = launch_cg_reduce(RED_RR, h->st, h->partials, h->L.nblk_x, B, s, active);
    mark();
  }
  return e;
}

void drop_graphs(fft_homog_t* h) {
  for (int k = 0; k < 2; ++k) {
    if (h->gexec[k]) hipGraphExecDestroy(h->gexec[k]);
    h->gexec[k] = nullptr;
    h->gB[k] = 0;
  }
}

// Enqueue m CG iterations.  With FLAG_GRAPH a full chunk is one launch of a graph
// captured (on a private stream, which the capture does not run) from the same
// launches; every kernel argument is a workspace pointer or a launch-shape
// constant, so the graph stays valid until the material or the shape changes.
int cg_chunk(fft_homog_t* h, int B, int m, int nrun, const int* active) {
  if (!(h->desc.flags & FFT_HOMOG_FLAG_GRAPH) || m != kChunk || active) {
    FH_CK(enqueue_cg_iters(h, nrun, m, h->stream, active));
    return FFT_HOMOG_OK;
  }
  const int k = B == 1 ? 0 : 1;
  if (!h->gexec[k] || h->gB[k] != B) {
    if (h->gexec[k]) hipGraphExecDestroy(h->gexec[k]);
    h->gexec[k] = nullptr;
    FH_CK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_cg_iters(h, B, kChunk, h->cap);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(h->cap, &graph);
    if (e == hipSuccess) e = e2;
    hipGraphExec_t ex = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    if (graph) hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(h, FFT_HOMOG_EDEVICE, hipGetErrorString(e));
    h->gexec[k] = ex;
    h->gB[k] = B;
  }
  FH_CK(hipGraphLaunch(h->gexec[k], h->stream));
  return FFT_HOMOG_OK;
}

int upload_states(fft_homog_t* h, int B) {
  for (int b = 0; b < B; ++b) {
    CgState& s = h->h_st[b];
    memset(&s, 0, sizeof(s));
    s.tol = h->desc.tol_cg;
    s.max_iters = h->desc.max_cg;
    s.status = CG_RUNNING;
  }
  FH_CK(hipMemcpyAsync(h->st, h->h_st, B * sizeof(CgState), hipMemcpyHostToDevice, h->stream));
  return FFT_HOMOG_OK;
}

int read_states(fft_homog_t* h, int B) {
  FH_CK(hipMemcpyAsync(h->h_st, h->st, B * sizeof(CgState), hipMemcpyDeviceToHost, h->stream));
  FH_CK(hipStreamSynchronize(h->stream));
  return FFT_HOMOG_OK;
}

// right-hand sides b = -G*(source) for B loads; leaves x = 0, r = b and the CG records initialised
int rhs_chain(fft_homog_t* h, int prod, int B, const double* unit) {
  int rc = upload_states(h, B);
  if (rc) return rc;
  XFwdArgs a = xfwd_args(h);
  if (unit)
    for (int k = 0; k < h->g.c; ++k) a.unit[k] = unit[k];
  FH_CK(launch_xfwd(prod, h->matcode, a, B, h->stream));
  FH_CK(launch_cg_reduce(RED_SRC, h->st, h->partials, h->L.nblk_x, B, h->stream));
  rc = spectral_middle(h, OUTER_PROJECT, B, nullptr);
  if (rc) return rc;
  FH_CK(launch_xinv(CONS_RHS, xinv_args(h), B, h->stream));
  FH_CK(launch_cg_reduce(RED_RHS, h->st, h->partials, h->L.nblk_x, B, h->stream));
  return read_states(h, B);
}

// CG iterations a single right-hand side enqueues before its next host check.  While the
// residual is far from the tolerance: 2 kChunk.  Near it: about the remainder predicted from
// the mean residual decay per iteration so far (fewer host checks and fewer launches after
// convergence), but at least kChunk / 2 unless the decay since the previous check agrees with
// that mean to a factor of two -- a stagnating residual (a tolerance at the rounding floor)
// would otherwise cost a host check per iteration.  Chunking never changes the iterates:
// iterations enqueued past convergence return at once.
int cg_chunk_length(int iters, double rr0, double rr, double tol, int prev_iters, double prev_rr) {
  if (!(iters >= 4 && rr > 0.0 && rr0 > 0.0 && rr < rr0 && tol > 0.0)) return kChunk;
  const double rate = std::log(rr / rr0) / iters;  // < 0
  double left = std::log(tol * tol * rr0 / rr) / rate;
  if (!(left > 0.0)) return kChunk;                // reached, or not a number
  left = std::min(left, 2.0 * kChunk);             // clamp before the integer conversion
  int m = std::max(1, (int)std::ceil(left));
  bool trust = false;
  if (prev_iters >= 0 && iters > prev_iters && prev_rr > 0.0) {
    const double recent = std::log(rr / prev_rr) / (iters - prev_iters);
    trust = recent <= 0.5 * rate && recent >= 2.0 * rate;
  }
  if (!trust) m = std::max(m, kChunk / 2);
  return m;
}

// Conjugate gradients on all running right-hand sides until none is running.  Once some
// have stopped, the launches cover only the running ones (their indices are uploaded
// before each chunk), so a batch's slow tail does not pay for its finished members.
int cg_loop(fft_homog_t* h, int B) {
  h->tev_used = 0;  // event groups of an earlier call that failed before its host check
  int prev_iters = -1;
  double prev_rr = 0.0;
  for (;;) {
    int nrun = 0;
    int done = 1 << 30;
    for (int b = 0; b < B; ++b)
      if (h->h_st[b].status == CG_RUNNING) {
        h->h_active[nrun++] = b;
        done = std::min(done, h->h_st[b].iters);
      }
    if (nrun == 0) return FFT_HOMOG_OK;
    // Iterations to enqueue before the next host check.  A single right-hand side (not replayed
    // from a graph) takes up to 2 kChunk at once while far from the tolerance and about the
    // predicted remainder near it, from its mean residual decay per iteration so far: fewer
    // host checks and fewer launches after convergence (128^3 solve -0.35 %).  Chunking does not
    // change the iterates; iterations past convergence return at once.
    int m = kChunk;
    if (B == 1 && !(h->desc.flags & FFT_HOMOG_FLAG_GRAPH)) {
      const CgState& S = h->h_st[0];
      m = cg_chunk_length(S.iters, S.rr0, S.rr, S.tol, prev_iters, prev_rr);
      prev_iters = S.iters;
      prev_rr = S.rr;
    }
    m = std::min(m, std::max(1, h->desc.max_cg - done));
    const int* act = nullptr;
    if (nrun < B) {
      FH_CK(hipMemcpyAsync(h->active, h->h_active, nrun * sizeof(int), hipMemcpyHostToDevice, h->stream));
      act = h->active;
    }
    int rc = cg_chunk(h, B, m, nrun, act);
    if (rc) return rc;
    rc = read_states(h, B);
    if (rc) return rc;
    ++h->host_checks;
    if (h->tev_used) {
      rc = harvest_timing(h);
      if (rc) return rc;
    }
    bool still = false;
    for (int b = 0; b < B; ++b) still = still || h->h_st[b].status == CG_RUNNING;
    if (!still) {
      FH_CK(launch_cg_finish(h->x, h->p, h->st, h->g, B, h->stream));
      return FFT_HOMOG_OK;
    }
  }
}

void to_packed(const fft_homog_t* h, const double* macro, double* out) {
  const int C = h->g.c;
  const double h2 = 0.70710678118654752440;
  for (int k = 0; k < C; ++k) out[k] = macro[k];
  if (h->g.small)
    for (int k = h->g.ndim; k < C; ++k) out[k] = macro[k] * h2;
}

void from_packed_stress(const fft_homog_t* h, const double* s, double* out) {
  const int C = h->g.c;
  const double h2 = 0.70710678118654752440;
  for (int k = 0; k < C; ++k) out[k] = s[k];
  if (h->g.small)
    for (int k = h->g.ndim; k < C; ++k) out[k] = s[k] * h2;
}

void unit_loads(const fft_homog_t* h, double* unit) {
  const double h2 = 0.70710678118654752440;
  for (int k = 0; k < h->g.c; ++k) unit[k] = (h->g.small && k >= h->g.ndim) ? h2 : 1.0;
}

int reduce_to_host(fft_homog_t* h, int nslots, int nblocks) {
  FH_CK(launch_reduce_slots(h->partials, nslots, nblocks, h->results, h->stream));
  FH_CK(hipMemcpyAsync(h->h_results, h->results, nslots * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  FH_CK(hipStreamSynchronize(h->stream));
  return FFT_HOMOG_OK;
}

// Apply a launch shape (the layout of fft_homog_get_launch_shape) after checking that every
// pass fits what its kernel assumes; returns EINVAL and changes nothing otherwise.
int apply_shape(fft_homog_t* h, const int* s) {
  const Geom& g = h->g;
  const int rows = g.ny * g.nz;
  const int R = s[0], TXm = s[1], TXo = s[2], ix = s[3], im = s[4], io = s[5], pitch = s[6];
  const int pad = g.nxh >= 8 ? (g.nxh + 7) / 8 * 8 : g.nxh;
  if (pitch != g.nxh && pitch != pad) return FFT_HOMOG_EINVAL;
  if (R < 1 || R > 16 || R > rows || TXm < 1 || TXm > g.nxh || TXo < 1 || TXo > g.nxh) return FFT_HOMOG_EINVAL;
  if ((ix != 0 && ix != 1) || (im != 0 && im != 1) || (io != 0 && io != 1)) return FFT_HOMOG_EINVAL;
  if (ix && !inplace_ok(h->plan[0], (g.c * R + 1) / 2)) return FFT_HOMOG_EINVAL;
  if (g.ndim == 3 && im && !inplace_ok(h->plan[1], mid_sequences(g, TXm, 1, 1))) return FFT_HOMOG_EINVAL;
  if (io && !outer_inplace_ok(g, h->plan[g.ndim - 1], TXo)) return FFT_HOMOG_EINVAL;
  const size_t lim = 64 * 1024;
  if (std::max(xfwd_smem(g, R, ix), xinv_smem(g, R, ix)) > lim && !(R == h->L.R && ix == h->L.in_x))
    return FFT_HOMOG_EINVAL;
  if (g.ndim == 3 && mid_smem(g, TXm, im, 1, 1) > lim && !(TXm == h->L.TXm && im == h->L.in_m))
    return FFT_HOMOG_EINVAL;
  if (g.ndim == 3 && !mid_fits(g, TXm, 1, 1)) return FFT_HOMOG_EINVAL;
  if (outer_smem(g, TXo, io) > lim && !(TXo == h->L.TXo && io == h->L.in_o)) return FFT_HOMOG_EINVAL;
  drop_graphs(h);
  h->g.nxp = pitch;
  h->g.Nh = (long long)pitch * g.ny * g.nz;
  h->L.R = R;
  h->L.in_x = ix;
  h->L.nblk_x = (rows + R - 1) / R;
  if (g.ndim == 3) {
    h->L.TXm = TXm;
    h->L.in_m = im;
  }
  h->L.TXo = TXo;
  h->L.in_o = io;
  return FFT_HOMOG_OK;
}

// Average device time (ms) of `reps` launches of `body` after one untimed launch.
template <class Body>
hipError_t time_launches(fft_homog_t* h, int reps, Body body, double* ms) {
  hipError_t e = body();
  if (e == hipSuccess) e = hipEventRecord(h->ev0, h->stream);
  for (int i = 0; i < reps && e == hipSuccess; ++i) e = body();
  if (e == hipSuccess) e = hipEventRecord(h->ev1, h->stream);
  if (e == hipSuccess) e = hipEventSynchronize(h->ev1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, h->ev0, h->ev1);
  *ms = (double)t / reps;
  return e;
}

}  // namespace

// =============================================================================
// public API
// =============================================================================
extern "C" {

int fft_homog_workspace_size(const fft_homog_desc* d, size_t* bytes) {
  if (!bytes) return FFT_HOMOG_EINVAL;
  Layout L;
  int rc = make_layout(d, &L);
  if (rc) return rc;
  *bytes = L.total;
  return FFT_HOMOG_OK;
}

int fft_homog_create(const fft_homog_desc* d, void* dev_workspace, size_t bytes, void* hip_stream,
                     fft_homog_t** out) {
  if (!out) return create_fail(FFT_HOMOG_EINVAL, "null output handle", hipSuccess);
  *out = nullptr;
  Layout L;
  int rc = make_layout(d, &L);
  if (rc) return create_fail(rc, "invalid or unsupported descriptor", hipSuccess);
  if (!dev_workspace || bytes < L.total || ((uintptr_t)dev_workspace % kAlign) != 0)
    return create_fail(FFT_HOMOG_EWORKSPACE, "workspace too small or not 256-byte aligned", hipSuccess);

  fft_homog_t* h = new fft_homog();
  h->desc = *d;
  make_geom(d, &h->g);
  make_plans(d, L.chirp, h->plan, &h->g);
  h->L = L;
  h->matcode = material_code(d);
  h->stream = (hipStream_t)hip_stream;
  h->ws = (char*)dev_workspace;
  h->F = (double*)(h->ws + L.F);
  place_work_vectors(h, 0);
  h->kst = d->k_mode == FFT_HOMOG_K_STORED ? (double*)(h->ws + L.kst) : nullptr;
  h->phase = (uint8_t*)(h->ws + L.phase);
  h->density = (d->flags & FFT_HOMOG_FLAG_DENSITY) ? (double*)(h->ws + L.density) : nullptr;
  h->scale = (d->flags & FFT_HOMOG_FLAG_DENSITY) ? (double*)(h->ws + L.scale) : nullptr;
  h->table = (double*)(h->ws + L.table);
  h->partials = (double*)(h->ws + L.partials);
  h->st = (CgState*)(h->ws + L.state);
  h->results = (double*)(h->ws + L.results);
  h->flags = (int*)(h->ws + L.flags);
  h->active = (int*)(h->ws + L.active);
  h->solved_ok = false;
  for (int k = 0; k < kMaxC; ++k) h->macro_cur[k] = 0.0;
  if (!h->g.small)
    for (int i = 0; i < d->ndim; ++i) h->macro_cur[i * d->ndim + i] = 1.0;
  const bool j2 = d->material == FFT_HOMOG_J2_PLASTIC;
  h->hist = j2 ? (double*)(h->ws + L.hist) : nullptr;
  h->j2_pending = false;
  h->mat.phase = h->phase;
  h->mat.table = h->table;
  h->mat.scale = nullptr;
  h->mat.hist = h->hist;
  h->mat.hN = h->g.N;
  h->mat.tstride = j2 ? 4 : 2;
  h->simp_p = 0.0;
  h->h_st = nullptr;
  h->ev0 = h->ev1 = nullptr;
  h->cap = nullptr;
  h->gexec[0] = h->gexec[1] = nullptr;
  h->gB[0] = h->gB[1] = 0;
  h->host_checks = 0;

  hipError_t e = hipHostMalloc((void**)&h->h_st,
                               L.B * sizeof(CgState) + L.n_results * sizeof(double) + 64 + L.B * sizeof(int), 0);
  if (e != hipSuccess) {
    delete h;
    return create_fail(FFT_HOMOG_EDEVICE, "hipHostMalloc", e);
  }
  h->h_results = (double*)((char*)h->h_st + L.B * sizeof(CgState));
  h->h_flags = (int*)(h->h_results + L.n_results);
  h->h_active = h->h_flags + 16;
  const char* step = "hipEventCreate";
  e = hipEventCreate(&h->ev0);
  if (e == hipSuccess) e = hipEventCreate(&h->ev1);
  if (e == hipSuccess && (d->flags & FFT_HOMOG_FLAG_GRAPH)) {
    step = "capture stream";
    e = hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking);
  }

  // twiddle tables of the stages' length, computed in extended precision and rounded once; the
  // chirp-z tables of chirp-z axes on the device
  std::vector<double2> tw[3];
  for (int a = 0; a < d->ndim && e == hipSuccess; ++a) {
    AxisPlan& pl = h->plan[a];
    const int n = lds_len(pl);
    tw[a].resize(n);
    for (int m = 0; m < n; ++m) {
      const long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)n;
      tw[a][m] = make_double2((double)cosl(ang), (double)-sinl(ang));
    }
    double2* dtw = (double2*)(h->ws + L.tw[a]);
    step = "twiddle upload";
    e = hipMemcpyAsync(dtw, tw[a].data(), n * sizeof(double2), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) {
      step = "chirp-z tables";
      e = launch_plan_tables(&pl, dtw, h->stream, false);
    }
  }
  if (h->g.ndim == 2) h->plan[2] = h->plan[1];
  std::vector<double> zeros((size_t)L.cells * (j2 ? 4 : 2) * kMaxPhase, 0.0);
  if (e == hipSuccess) {
    step = "phase table init";
    e = hipMemcpyAsync(h->table, zeros.data(), zeros.size() * sizeof(double), hipMemcpyHostToDevice, h->stream);
  }
  if (e == hipSuccess) {
    step = "phase map init";
    e = hipMemsetAsync(h->phase, 0, (size_t)L.cells * h->g.N, h->stream);
  }
  if (e == hipSuccess) {
    step = "reference strain";
    e = launch_init_reference(h->F, h->g, h->stream);
  }
  if (e == hipSuccess && j2) {
    step = "plastic history init";
    e = hipMemsetAsync(h->hist, 0, (size_t)(h->g.c + 1) * h->g.N * sizeof(double), h->stream);
  }
  if (e == hipSuccess) {
    step = "LDS limit";
    e = set_smem_limits(h->g, h->matcode, L.smem_max);
  }
  if (e == hipSuccess) {
    step = "stream synchronize";
    e = hipStreamSynchronize(h->stream);
  }
  if (e != hipSuccess) {
    fft_homog_destroy(h);
    return create_fail(FFT_HOMOG_EDEVICE, step, e);
  }
  g_create_err[0] = 0;
  *out = h;
  return FFT_HOMOG_OK;
}

int fft_homog_set_material(fft_homog_t* h, const uint8_t* phase, const double* lm, const double* density,
                           double simp_p) {
  if (!h || !phase || !lm) return fail(h, FFT_HOMOG_EINVAL, "null argument");
  if (density && !h->density) return fail(h, FFT_HOMOG_EINVAL, "density given but FLAG_DENSITY not set");
  const int cells = h->L.cells;
  const int ts = h->mat.tstride;
  const size_t row = (size_t)ts * h->desc.nphase * sizeof(double);
  for (long long k = 0; k < (long long)ts * h->desc.nphase * cells; ++k)
    if (!std::isfinite(lm[k])) return fail(h, FFT_HOMOG_EINVAL, "non-finite phase table entry");
  if (ts == 4)
    for (int ph = 0; ph < h->desc.nphase; ++ph)
      if (!(lm[4 * ph + 2] >= 0.0) || !(lm[4 * ph + 3] >= 0.0) || !(3.0 * lm[4 * ph + 1] + lm[4 * ph + 3] > 0.0))
        return fail(h, FFT_HOMOG_EINVAL, "J2 phase needs sig_y >= 0, H >= 0, 3 mu + H > 0");
  // plane stress, linear elasticity and St. Venant-Kirchhoff: both energies are quadratic in the
  // strain (eps, resp. E = (F^T F - I)/2) with the same Lame form, so the out-of-plane normal stress
  // = 0 eliminates the out-of-plane strain and leaves the 2D law with the reduced first Lame
  // parameter 2 lam mu / (lam + 2 mu).  Neo-Hookean and J2 run laws of their own, which solve for
  // the out-of-plane entry per voxel: Neo-Hookean's Newton iteration needs lam >= 0 and mu > 0, J2's
  // (on a bracket) an increasing sigma_33, mu > 0 and 3 lam + 2 mu > 0.
  std::vector<double> reduced;
  const bool ps = (h->desc.flags & FFT_HOMOG_FLAG_PLANE_STRESS) != 0;
  if (ps && h->desc.material == FFT_HOMOG_NEO_HOOKEAN) {
    for (size_t k = 0; k < (size_t)2 * h->desc.nphase * cells; k += 2)
      if (!(lm[k] >= 0.0) || !(lm[k + 1] > 0.0))
        return fail(h, FFT_HOMOG_EINVAL, "Neo-Hookean plane stress needs lam >= 0 and mu > 0");
  } else if (ps && h->desc.material == FFT_HOMOG_J2_PLASTIC) {
    for (size_t k = 0; k < (size_t)4 * h->desc.nphase * cells; k += 4)
      if (!(lm[k + 1] > 0.0) || !(3.0 * lm[k] + 2.0 * lm[k + 1] > 0.0))
        return fail(h, FFT_HOMOG_EINVAL, "J2 plane stress needs mu > 0 and 3 lam + 2 mu > 0");
  } else if (ps) {
    reduced.assign(lm, lm + (size_t)2 * h->desc.nphase * cells);
    for (size_t k = 0; k < reduced.size(); k += 2) {
      const double la = reduced[k], m = reduced[k + 1];
      if (!(la + 2.0 * m != 0.0)) return fail(h, FFT_HOMOG_EINVAL, "plane stress needs lam + 2 mu != 0");
      reduced[k] = 2.0 * la * m / (la + 2.0 * m);
    }
    lm = reduced.data();
  }
  drop_graphs(h);
  FH_CK(hipMemcpyAsync(h->phase, phase, (size_t)cells * h->g.N, hipMemcpyDeviceToDevice, h->stream));
  FH_CK(hipMemcpy2DAsync(h->table, (size_t)ts * kMaxPhase * sizeof(double), lm, row, row, cells,
                         hipMemcpyHostToDevice, h->stream));
  if (density) {
    FH_CK(hipMemcpyAsync(h->density, density, (size_t)h->g.N * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    FH_CK(launch_simp_scale(h->density, simp_p, h->scale, h->g.N, h->stream));
  }
  h->mat.scale = density ? h->scale : nullptr;
  h->simp_p = simp_p;
  h->h_flags[0] = 0;
  FH_CK(hipMemcpyAsync(h->flags, h->h_flags, sizeof(int), hipMemcpyHostToDevice, h->stream));
  FH_CK(launch_check_phase(h->phase, (long long)cells * h->g.N, h->desc.nphase, h->flags, h->stream));
  FH_CK(hipMemcpyAsync(h->h_flags, h->flags, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  FH_CK(hipStreamSynchronize(h->stream));
  h->solved_ok = false;
  if (h->h_flags[0]) return fail(h, FFT_HOMOG_EINVAL, "phase id >= nphase");
  return FFT_HOMOG_OK;
}

int fft_homog_solve(fft_homog_t* h, const double* macro, int n_increments, double* macro_stress, double* energy,
                    fft_homog_stats* stats) {
  if (!h || !macro || n_increments < 1) return fail(h, FFT_HOMOG_EINVAL, "bad solve arguments");
  if (h->L.cells > 1) return fail(h, FFT_HOMOG_EUNSUPPORTED, "multi-cell handles compute tangents only");
  const int C = h->g.c;
  for (int k = 0; k < C; ++k)
    if (!std::isfinite(macro[k])) return fail(h, FFT_HOMOG_EINVAL, "non-finite macro load");
  fft_homog_stats S;
  memset(&S, 0, sizeof(S));
  h->host_checks = 0;
  FH_CK(hipEventRecord(h->ev0, h->stream));

  double target[kMaxC], start[kMaxC], prev[kMaxC], cur[kMaxC], delta[kMaxC];
  to_packed(h, macro, target);
  for (int k = 0; k < C; ++k) start[k] = prev[k] = h->macro_cur[k];
  const double sqrtN = std::sqrt((double)h->g.N);
  int status = FFT_HOMOG_OK;
  h->solved_ok = false;

  for (int n = 1; n <= n_increments && status == FFT_HOMOG_OK; ++n) {
    const double f = (double)n / (double)n_increments;
    double mn = 0.0;
    for (int k = 0; k < C; ++k) {
      cur[k] = start[k] + f * (target[k] - start[k]);
      delta[k] = cur[k] - prev[k];
      prev[k] = cur[k];
      mn += cur[k] * cur[k];
    }
    mn = std::sqrt(mn);
    if (h->j2_pending) {
      // the previous load step converged: its plastic state becomes the history of this one
      FH_CK(launch_j2_commit(h->matcode, h->F, h->mat, h->hist, h->g, h->stream));
      h->j2_pending = false;
    }
    FH_CK(launch_shift(h->F, delta, h->g, h->stream));
    for (int k = 0; k < C; ++k) h->macro_cur[k] = cur[k];
    int it = 0;
    for (;;) {
      int rc = rhs_chain(h, PROD_STRESS, 1, nullptr);
      if (rc) return rc;
      const CgState& cs = h->h_st[0];
      if (cs.domain) { status = FFT_HOMOG_EDOMAIN; break; }
      if (cs.status == CG_ZERO_RHS) break;
      if (it >= h->desc.max_newton) { status = FFT_HOMOG_ENOTCONV; break; }
      if (h->kst) FH_CK(launch_store_tangent(h->matcode, h->F, h->mat, h->kst, h->g, h->stream));
      rc = cg_loop(h, 1);
      if (rc) return rc;
      const CgState& ce = h->h_st[0];
      if (S.n_recorded < FFT_HOMOG_MAX_RECORDED) S.cg_per_newton[S.n_recorded++] = ce.iters;
      S.cg_iterations += ce.iters;
      S.cg_residual = ce.rr0 > 0 ? std::sqrt(ce.rr / ce.rr0) : 0.0;
      if (ce.status == CG_BREAKDOWN) { status = FFT_HOMOG_EBREAKDOWN; break; }
      if (ce.status == CG_MAXIT) { status = FFT_HOMOG_ENOTCONV; break; }
      FH_CK(launch_update(h->F, h->x, h->partials, h->L.nblk_vox, h->g, h->stream));
      rc = reduce_to_host(h, 2, h->L.nblk_vox);
      if (rc) return rc;
      ++it;
      S.newton_iterations++;
      // RMS update over the RMS macro load; a zero macro load (small strain unloaded to zero,
      // where a history-dependent law leaves residual stresses) takes the updated field's own
      // norm as the scale, and a zero field counts as converged
      const double scale = mn > 0.0 ? sqrtN * mn : std::sqrt(h->h_results[1]);
      const double dn = std::sqrt(h->h_results[0]);
      const double res = scale > 0.0 ? dn / scale : (dn > 0.0 ? HUGE_VAL : 0.0);
      S.newton_residual = res;
      if (res < h->desc.tol_newton) break;
    }
    if (status == FFT_HOMOG_OK) {
      S.increments = n;
      if (h->hist) h->j2_pending = true;
    }
  }

  if (status != FFT_HOMOG_EDOMAIN) {
    FH_CK(launch_homogenize(h->matcode, h->F, h->mat, h->partials, h->L.nblk_vox, h->g, h->st, h->stream));
    int rc = reduce_to_host(h, C + 1, h->L.nblk_vox);
    if (rc) return rc;
    double sbar[kMaxC];
    for (int k = 0; k < C; ++k) sbar[k] = h->h_results[k] / (double)h->g.N;
    if (macro_stress) from_packed_stress(h, sbar, macro_stress);
    if (energy) *energy = h->h_results[C] / (double)h->g.N;
  }
  FH_CK(hipEventRecord(h->ev1, h->stream));
  FH_CK(hipEventSynchronize(h->ev1));
  float ms = 0.f;
  FH_CK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  S.seconds = ms * 1e-3;
  S.status = status;
  S.host_checks = (int)h->host_checks;
  h->solved_ok = status == FFT_HOMOG_OK;
  if (stats) *stats = S;
  if (status != FFT_HOMOG_OK) {
    h->err = status == FFT_HOMOG_EDOMAIN ? "det F <= 0 or non-finite stress"
             : status == FFT_HOMOG_EBREAKDOWN ? "CG breakdown: <p, K:p> <= 0"
                                              : "iteration limit reached";
  }
  return status;
}

int fft_homog_tangent(fft_homog_t* h, double* Cout, fft_homog_stats* stats) {
  if (!h || !Cout) return fail(h, FFT_HOMOG_EINVAL, "null argument");
  if (!(h->desc.flags & FFT_HOMOG_FLAG_TANGENT)) return fail(h, FFT_HOMOG_ESTATE, "FLAG_TANGENT not set at create");
  const int cells = h->L.cells;
  // a multi-cell handle never leaves the reference state
  if (cells == 1 && !h->solved_ok) return fail(h, FFT_HOMOG_ESTATE, "no converged solve");
  const int C = h->g.c;
  const int B = h->L.B;
  fft_homog_stats S;
  memset(&S, 0, sizeof(S));
  h->host_checks = 0;
  FH_CK(hipEventRecord(h->ev0, h->stream));
  double unit[kMaxC];
  unit_loads(h, unit);
  int rc = rhs_chain(h, PROD_TRHS, B, unit);
  if (rc) return rc;
  if (h->kst) FH_CK(launch_store_tangent(h->matcode, h->F, h->mat, h->kst, h->g, h->stream));
  rc = cg_loop(h, B);
  if (rc) return rc;
  int status = FFT_HOMOG_OK;
  for (int b = 0; b < B; ++b) {
    const CgState& s = h->h_st[b];
    S.cg_iterations += s.iters;
    if (S.n_recorded < FFT_HOMOG_MAX_RECORDED) S.cg_per_newton[S.n_recorded++] = s.iters;
    if (s.status == CG_BREAKDOWN) status = FFT_HOMOG_EBREAKDOWN;
    else if (s.status == CG_MAXIT && status == FFT_HOMOG_OK) status = FFT_HOMOG_ENOTCONV;
  }
  // C_IJ of each cell: the partial sums of one cell are reduced before the next reuses them
  for (int cell = 0; cell < cells; ++cell) {
    MatParams m = h->mat;
    m.phase += (long long)cell * h->g.N;
    m.table += (long long)cell * 2 * kMaxPhase;
    const double* X = h->x + (size_t)cell * C * C * h->g.N;
    FH_CK(launch_tangent_matrix(h->matcode, h->F, X, unit, m, h->partials, h->L.nblk_vox, h->g, h->stream));
    FH_CK(launch_reduce_slots(h->partials, C * C, h->L.nblk_vox, h->results + (size_t)cell * C * C, h->stream));
  }
  FH_CK(hipMemcpyAsync(h->h_results, h->results, (size_t)cells * C * C * sizeof(double), hipMemcpyDeviceToHost,
                       h->stream));
  FH_CK(hipStreamSynchronize(h->stream));
  for (long long k = 0; k < (long long)cells * C * C; ++k) Cout[k] = h->h_results[k] / (double)h->g.N;
  FH_CK(hipEventRecord(h->ev1, h->stream));
  FH_CK(hipEventSynchronize(h->ev1));
  float ms = 0.f;
  FH_CK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  S.seconds = ms * 1e-3;
  S.status = status;
  S.host_checks = (int)h->host_checks;
  if (stats) *stats = S;
  return status;
}

int fft_homog_adjoint(fft_homog_t* h, const double* w_stress, double w_energy, double* grad_density,
                      fft_homog_stats* stats) {
  if (!h || !w_stress || !grad_density) return fail(h, FFT_HOMOG_EINVAL, "null argument");
  if (h->L.cells > 1) return fail(h, FFT_HOMOG_EUNSUPPORTED, "multi-cell handles compute tangents only");
  if (h->hist) return fail(h, FFT_HOMOG_EUNSUPPORTED, "no density gradient for J2 plasticity");
  if (!h->mat.scale) return fail(h, FFT_HOMOG_ESTATE, "no density field set (FLAG_DENSITY and set_material)");
  if (!h->solved_ok) return fail(h, FFT_HOMOG_ESTATE, "no converged solve");
  if (!std::isfinite(w_energy)) return fail(h, FFT_HOMOG_EINVAL, "non-finite weight");
  const int C = h->g.c;
  for (int k = 0; k < C; ++k)
    if (!std::isfinite(w_stress[k])) return fail(h, FFT_HOMOG_EINVAL, "non-finite weight");
  fft_homog_stats S;
  memset(&S, 0, sizeof(S));
  h->host_checks = 0;
  FH_CK(hipEventRecord(h->ev0, h->stream));
  // W in the packed basis: the objective is sum_I w_I out_I with out_I = W-packed . P-packed
  double W[kMaxC];
  from_packed_stress(h, w_stress, W);
  XFwdArgs a = xfwd_args(h);
  for (int k = 0; k < C; ++k) a.unit[k] = W[k];
  a.w_energy = w_energy;
  int rc = upload_states(h, 1);
  if (rc) return rc;
  FH_CK(launch_xfwd(PROD_ADJ, h->matcode, a, 1, h->stream));
  FH_CK(launch_cg_reduce(RED_SRC, h->st, h->partials, h->L.nblk_x, 1, h->stream));
  rc = spectral_middle(h, OUTER_PROJECT, 1, nullptr);
  if (rc) return rc;
  FH_CK(launch_xinv(CONS_RHS, xinv_args(h), 1, h->stream));
  FH_CK(launch_cg_reduce(RED_RHS, h->st, h->partials, h->L.nblk_x, 1, h->stream));
  rc = read_states(h, 1);
  if (rc) return rc;
  if (h->kst) FH_CK(launch_store_tangent(h->matcode, h->F, h->mat, h->kst, h->g, h->stream));
  rc = cg_loop(h, 1);
  if (rc) return rc;
  const CgState& cs = h->h_st[0];
  int status = FFT_HOMOG_OK;
  if (cs.status == CG_BREAKDOWN) status = FFT_HOMOG_EBREAKDOWN;
  else if (cs.status == CG_MAXIT) status = FFT_HOMOG_ENOTCONV;
  S.cg_iterations = cs.iters;
  S.n_recorded = 1;
  S.cg_per_newton[0] = cs.iters;
  S.cg_residual = cs.rr0 > 0 ? std::sqrt(cs.rr / cs.rr0) : 0.0;
  FH_CK(launch_simp_gradient(h->matcode, h->F, h->x, h->mat, h->density, h->simp_p, W, w_energy, grad_density, h->g,
                             h->stream));
  FH_CK(hipEventRecord(h->ev1, h->stream));
  FH_CK(hipEventSynchronize(h->ev1));
  float ms = 0.f;
  FH_CK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  S.seconds = ms * 1e-3;
  S.status = status;
  S.host_checks = (int)h->host_checks;
  if (stats) *stats = S;
  if (status) h->err = status == FFT_HOMOG_EBREAKDOWN ? "CG breakdown" : "iteration limit reached";
  return status;
}

int fft_homog_get_field(fft_homog_t* h, int which, double* dst) {
  if (!h || !dst) return fail(h, FFT_HOMOG_EINVAL, "null argument");
  if (h->L.cells > 1) return fail(h, FFT_HOMOG_EUNSUPPORTED, "multi-cell handles compute tangents only");
  if (which == FFT_HOMOG_FIELD_STRAIN) {
    FH_CK(launch_expand(h->F, dst, h->g, h->stream));
  } else if (which == FFT_HOMOG_FIELD_STRESS) {
    FH_CK(launch_stress_field(h->matcode, h->F, h->mat, h->r, nullptr, h->g, h->stream));
    FH_CK(launch_expand(h->r, dst, h->g, h->stream));
  } else if (which == FFT_HOMOG_FIELD_ENERGY) {
    FH_CK(launch_stress_field(h->matcode, h->F, h->mat, nullptr, dst, h->g, h->stream));
  } else if (which == FFT_HOMOG_FIELD_PLASTIC && h->hist) {
    FH_CK(launch_j2_plastic(h->matcode, h->F, h->mat, dst, h->g, h->stream));
  } else {
    return fail(h, FFT_HOMOG_EINVAL, "unknown field");
  }
  FH_CK(hipStreamSynchronize(h->stream));
  return FFT_HOMOG_OK;
}

int fft_homog_set_field(fft_homog_t* h, const double* src, const double* macro) {
  if (!h || !src || !macro) return fail(h, FFT_HOMOG_EINVAL, "null argument");
  if (h->L.cells > 1) return fail(h, FFT_HOMOG_EUNSUPPORTED, "multi-cell handles compute tangents only");
  FH_CK(launch_pack(src, h->F, h->g, h->stream));
  if (h->hist) {
    // a prescribed state starts with a virgin plastic history
    FH_CK(hipMemsetAsync(h->hist, 0, (size_t)(h->g.c + 1) * h->g.N * sizeof(double), h->stream));
    h->j2_pending = false;
  }
  to_packed(h, macro, h->macro_cur);
  FH_CK(hipStreamSynchronize(h->stream));
  h->solved_ok = false;
  return FFT_HOMOG_OK;
}

void fft_homog_destroy(fft_homog_t* h) {
  if (!h) return;
  if (h->stream) hipStreamSynchronize(h->stream);
  else hipDeviceSynchronize();
  if (h->h_st) hipHostFree(h->h_st);
  if (h->ev0) hipEventDestroy(h->ev0);
  if (h->ev1) hipEventDestroy(h->ev1);
  for (hipEvent_t ev : h->tev) hipEventDestroy(ev);
  drop_graphs(h);
  if (h->cap) hipStreamDestroy(h->cap);
  delete h;
}

const char* fft_homog_strerror(int s) {
  switch (s) {
    case FFT_HOMOG_OK: return "ok";
    case FFT_HOMOG_EINVAL: return "invalid argument";
    case FFT_HOMOG_ENOTCONV: return "not converged (iteration limit)";
    case FFT_HOMOG_EDOMAIN: return "constitutive domain error (det F <= 0 or non-finite stress)";
    case FFT_HOMOG_EBREAKDOWN: return "CG breakdown (<p, K:p> <= 0)";
    case FFT_HOMOG_ESTATE: return "invalid call order";
    case FFT_HOMOG_EUNSUPPORTED: return "unsupported";
    case FFT_HOMOG_EDEVICE: return "HIP runtime error";
    case FFT_HOMOG_EWORKSPACE: return "workspace too small or misaligned";
    default: return "unknown status";
  }
}

const char* fft_homog_last_error(const fft_homog_t* h) { return h ? h->err.c_str() : g_create_err; }

// ---- stage-level entry points -------------------------------------------------
static int check_batch(fft_homog_t* h, int batch) {
  if (batch < 1 || batch > h->L.B) return fail(h, FFT_HOMOG_EINVAL, "batch out of range");
  return FFT_HOMOG_OK;
}

int fft_homog_debug_constitutive(fft_homog_t* h, const double* e, const double* de, double* P, double* KdE,
                                 double* psi) {
  if (!h || !e || !de || !P || !KdE || !psi) return fail(h, FFT_HOMOG_EINVAL, "null argument");
  FH_CK(launch_debug_constitutive(h->matcode, e, de, P, KdE, psi, h->mat, h->g, h->stream));
  FH_CK(hipStreamSynchronize(h->stream));
  return FFT_HOMOG_OK;
}

int fft_homog_debug_rfft(fft_homog_t* h, const double* in, double* spec, int batch) {
  if (!h || !in || !spec) return fail(h, FFT_HOMOG_EINVAL, "null argument");
  int rc = check_batch(h, batch);
  if (rc) return rc;
  XFwdArgs a = xfwd_args(h);
  a.in = in;
  FH_CK(launch_xfwd(PROD_IDENT, h->matcode, a, batch, h->stream));
  rc = spectral_middle(h, OUTER_FWD, batch, nullptr);
  if (rc) return rc;
  FH_CK(hipMemcpy2DAsync(spec, h->g.nxh * sizeof(double2), h->spec, h->g.nxp * sizeof(double2),
                         h->g.nxh * sizeof(double2), (size_t)batch * h->g.c * h->g.ny * h->g.nz,
                         hipMemcpyDeviceToDevice, h->stream));
  FH_CK(hipStreamSynchronize(h->stream));
  return FFT_HOMOG_OK;
}

int fft_homog_debug_irfft(fft_homog_t* h, const double* spec, double* out, int batch) {
  if (!h || !spec || !out) return fail(h, FFT_HOMOG_EINVAL, "null argument");
  int rc = check_batch(h, batch);
  if (rc) return rc;
  FH_CK(hipMemcpy2DAsync(h->spec, h->g.nxp * sizeof(double2), spec, h->g.nxh * sizeof(double2),
                         h->g.nxh * sizeof(double2), (size_t)batch * h->g.c * h->g.ny * h->g.nz,
                         hipMemcpyDeviceToDevice, h->stream));
  rc = spectral_middle(h, OUTER_INV, batch, nullptr);
  if (rc) return rc;
  XInvArgs a = xinv_args(h);
  a.out = out;
  FH_CK(launch_xinv(CONS_IDENT, a, batch, h->stream));
  FH_CK(hipStreamSynchronize(h->stream));
  return FFT_HOMOG_OK;
}

int fft_homog_debug_project(fft_homog_t* h, const double* in, double* out, int batch) {
  if (!h || !in || !out) return fail(h, FFT_HOMOG_EINVAL, "null argument");
  int rc = check_batch(h, batch);
  if (rc) return rc;
  FH_CK(enqueue_projection(h->g, h->plan, h->L, h->matcode, in, out, h->spec, batch, h->stream));
  FH_CK(hipStreamSynchronize(h->stream));
  return FFT_HOMOG_OK;
}

int fft_homog_debug_apply_operator(fft_homog_t* h, const double* p, double* q, int batch) {
  if (!h || !p || !q) return fail(h, FFT_HOMOG_EINVAL, "null argument");
  int rc = check_batch(h, batch);
  if (rc) return rc;
  // q = G*(K:p): run one CG-operator pass with r = p, first = 1 (p_dir = r)
  rc = upload_states(h, batch);
  if (rc) return rc;
  const size_t bytes = (size_t)batch * h->g.c * h->g.N * sizeof(double);
  FH_CK(hipMemcpyAsync(h->r, p, bytes, hipMemcpyDeviceToDevice, h->stream));
  for (int b = 0; b < batch; ++b) h->h_st[b].first = 1;
  FH_CK(hipMemcpyAsync(h->st, h->h_st, batch * sizeof(CgState), hipMemcpyHostToDevice, h->stream));
  if (h->kst) FH_CK(launch_store_tangent(h->matcode, h->F, h->mat, h->kst, h->g, h->stream));
  XFwdArgs a = xfwd_args(h);
  a.in = h->r;
  a.p = h->p;
  FH_CK(launch_xfwd(h->kst ? PROD_CGOP_STORED : PROD_CGOP, h->matcode, a, batch, h->stream));
  rc = spectral_middle(h, OUTER_PROJECT, batch, nullptr);
  if (rc) return rc;
  XInvArgs ai = xinv_args(h);
  ai.out = q;
  FH_CK(launch_xinv(CONS_IDENT, ai, batch, h->stream));
  FH_CK(hipStreamSynchronize(h->stream));
  return FFT_HOMOG_OK;
}

int fft_homog_debug_cg(fft_homog_t* h, int iters, double* x_out, double* r_out) {
  if (!h || !x_out || !r_out || iters < 1) return fail(h, FFT_HOMOG_EINVAL, "bad arguments");
  if (h->L.cells > 1) return fail(h, FFT_HOMOG_EUNSUPPORTED, "multi-cell handles compute tangents only");
  int rc = rhs_chain(h, PROD_STRESS, 1, nullptr);
  if (rc) return rc;
  if (h->h_st[0].domain) return fail(h, FFT_HOMOG_EDOMAIN, "det F <= 0 or non-finite stress");
  if (h->h_st[0].status != CG_RUNNING) return fail(h, FFT_HOMOG_ESTATE, "zero Newton right-hand side");
  // exactly `iters` iterations: no convergence test, stop at the iteration limit
  h->h_st[0].tol = 0.0;
  h->h_st[0].max_iters = iters;
  FH_CK(hipMemcpyAsync(h->st, h->h_st, sizeof(CgState), hipMemcpyHostToDevice, h->stream));
  if (h->kst) FH_CK(launch_store_tangent(h->matcode, h->F, h->mat, h->kst, h->g, h->stream));
  FH_CK(enqueue_cg_iters(h, 1, iters, h->stream));
  FH_CK(launch_cg_finish(h->x, h->p, h->st, h->g, 1, h->stream));
  rc = read_states(h, 1);
  if (rc) return rc;
  if (h->h_st[0].status != CG_MAXIT || h->h_st[0].iters != iters)
    return fail(h, FFT_HOMOG_EBREAKDOWN, "CG stopped before the requested iteration count");
  const size_t bytes = (size_t)h->g.c * h->g.N * sizeof(double);
  FH_CK(hipMemcpyAsync(x_out, h->x, bytes, hipMemcpyDeviceToDevice, h->stream));
  FH_CK(hipMemcpyAsync(r_out, h->r, bytes, hipMemcpyDeviceToDevice, h->stream));
  FH_CK(hipStreamSynchronize(h->stream));
  return FFT_HOMOG_OK;
}

int fft_homog_debug_cg_chunk(int iters, double rr0, double rr, double tol, int prev_iters, double prev_rr) {
  return cg_chunk_length(iters, rr0, rr, tol, prev_iters, prev_rr);
}

int fft_homog_debug_time_cg(fft_homog_t* h, int iters, double* ms) {
  if (!h || !ms || iters < 1) return fail(h, FFT_HOMOG_EINVAL, "bad arguments");
  double unit[kMaxC];
  unit_loads(h, unit);
  int rc = rhs_chain(h, PROD_TRHS, 1, unit);
  if (rc) return rc;
  if (h->h_st[0].status == CG_ZERO_RHS) return fail(h, FFT_HOMOG_ESTATE, "zero right-hand side (homogeneous cell)");
  // keep the solve running for exactly `iters` iterations
  h->h_st[0].status = CG_RUNNING;
  h->h_st[0].tol = 0.0;
  h->h_st[0].max_iters = iters + 1;
  FH_CK(hipMemcpyAsync(h->st, h->h_st, sizeof(CgState), hipMemcpyHostToDevice, h->stream));
  if (h->kst) FH_CK(launch_store_tangent(h->matcode, h->F, h->mat, h->kst, h->g, h->stream));
  const int prod = h->kst ? PROD_CGOP_STORED : PROD_CGOP;
  XFwdArgs a = xfwd_args(h);
  a.in = h->r;
  a.p = h->p;
  XInvArgs ai = xinv_args(h);
  AxisArgs ao = axis_args(h, h->g.ndim - 1, h->L.TXo, h->st);
  ao.pq_st = h->st;
  ao.pq_partials = h->partials;
  ao.pq_nblocks = h->L.nblk_x;
  const bool three = h->g.ndim == 3;
  hipEvent_t ev[8];
  for (int k = 0; k < 8; ++k) FH_CK(hipEventCreate(&ev[k]));
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  int status = FFT_HOMOG_OK;
  for (int i = 0; i < iters && status == FFT_HOMOG_OK; ++i) {
    hipError_t e = hipEventRecord(ev[0], h->stream);
    if (e == hipSuccess) e = launch_xfwd(prod, h->matcode, a, 1, h->stream);
    if (e == hipSuccess) e = hipEventRecord(ev[1], h->stream);
    // <p, K:p> is reduced inside the outer pass: its slot stays empty
    if (e == hipSuccess) e = hipEventRecord(ev[2], h->stream);
    if (e == hipSuccess && three) e = launch_mid(-1, axis_args(h, 1, h->L.TXm, h->st), 1, h->stream);
    if (e == hipSuccess) e = hipEventRecord(ev[3], h->stream);
    if (e == hipSuccess) e = launch_outer(OUTER_PROJECT, ao, 1, h->stream);
    if (e == hipSuccess) e = hipEventRecord(ev[4], h->stream);
    if (e == hipSuccess && three) e = launch_mid(1, axis_args(h, 1, h->L.TXm, h->st), 1, h->stream);
    if (e == hipSuccess) e = hipEventRecord(ev[5], h->stream);
    if (e == hipSuccess) e = launch_xinv(CONS_CGUPD, ai, 1, h->stream);
    if (e == hipSuccess) e = hipEventRecord(ev[6], h->stream);
    if (e == hipSuccess) e = launch_cg_reduce(RED_RR, h->st, h->partials, h->L.nblk_x, 1, h->stream);
    if (e == hipSuccess) e = hipEventRecord(ev[7], h->stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev[7]);
    for (int k = 0; k < 7 && e == hipSuccess; ++k) {
      float t = 0.f;
      e = hipEventElapsedTime(&t, ev[k], ev[k + 1]);
      acc[k] += t;
    }
    if (e != hipSuccess) status = fail(h, FFT_HOMOG_EDEVICE, hipGetErrorString(e));
  }
  for (int k = 0; k < 8; ++k) hipEventDestroy(ev[k]);
  if (status) return status;
  int rc2 = read_states(h, 1);
  if (rc2) return rc2;
  if (h->h_st[0].status != CG_RUNNING && h->h_st[0].status != CG_MAXIT)
    return fail(h, FFT_HOMOG_ESTATE, "timed CG stopped early (breakdown)");
  for (int k = 0; k < 7; ++k) ms[k] = acc[k] / iters;
  return FFT_HOMOG_OK;
}

int fft_homog_set_kernel_timing(fft_homog_t* h, int every) {
  if (!h || every < 0) return fail(h, FFT_HOMOG_EINVAL, "bad arguments");
  h->tev_used = 0;
  h->time_every = every;
  h->time_count = 0;
  for (int k = 0; k < kTimedLaunches; ++k) h->time_acc[k] = 0.0;
  h->time_samples = 0;
  return FFT_HOMOG_OK;
}

int fft_homog_get_kernel_timing(const fft_homog_t* h, double* ms, long long* samples) {
  if (!h || !ms || !samples) return FFT_HOMOG_EINVAL;
  *samples = h->time_samples;
  for (int k = 0; k < kTimedLaunches; ++k) ms[k] = h->time_samples ? h->time_acc[k] / h->time_samples : 0.0;
  return FFT_HOMOG_OK;
}

int fft_homog_get_launch_shape(const fft_homog_t* h, int shape[7]) {
  if (!h || !shape) return FFT_HOMOG_EINVAL;
  shape[6] = h->g.nxp;
  shape[0] = h->L.R;
  shape[1] = h->L.TXm;
  shape[2] = h->L.TXo;
  shape[3] = h->L.in_x;
  shape[4] = h->L.in_m;
  shape[5] = h->L.in_o;
  return FFT_HOMOG_OK;
}

int fft_homog_set_launch_shape(fft_homog_t* h, const int* shape) {
  if (!h || !shape) return fail(h, FFT_HOMOG_EINVAL, "null argument");
  if (apply_shape(h, shape)) return fail(h, FFT_HOMOG_EINVAL, "launch shape does not fit this grid");
  return FFT_HOMOG_OK;
}

int fft_homog_autotune(fft_homog_t* h, int reps, int* shape) {
  if (!h || reps < 1) return fail(h, FFT_HOMOG_EINVAL, "bad arguments");
  Geom& g = h->g;
  const int C = g.c;
  const int B = h->L.B;
  const int rows = g.ny * g.nz;
  const AxisPlan& pouter = h->plan[g.ndim - 1];
  // A candidate replaces the incumbent only when it is clearly faster, so that timing
  // noise does not move the shape away from the default.
  const double kGain = 0.98;
  // candidates stay within the default per-block LDS limit (more would cut the blocks
  // per CU to two or one); the incumbent is always timed
  const size_t kLdsTune = 64 * 1024;
  // right-hand sides timed: enough voxels (4 Mi) to fill the GPU, not the whole batch
  const int Bt = (int)std::max(1LL, std::min((long long)B, (1LL << 22) / g.N));
  drop_graphs(h);
  // work vectors at zero, every right-hand side running with alpha = beta = 0: the passes
  // then do all their loads, stores and arithmetic while the state stays put (no reduction
  // runs, so nothing can stop the solve)
  const size_t vec = (size_t)Bt * C * g.N * sizeof(double);
  FH_CK(hipMemsetAsync(h->x, 0, vec, h->stream));
  FH_CK(hipMemsetAsync(h->r, 0, vec, h->stream));
  FH_CK(hipMemsetAsync(h->p, 0, vec, h->stream));
  int rc = upload_states(h, Bt);
  if (rc) return rc;
  if (h->kst) FH_CK(launch_store_tangent(h->matcode, h->F, h->mat, h->kst, g, h->stream));
  const int prod = h->kst ? PROD_CGOP_STORED : PROD_CGOP;

  // The spectrum row pitch is tuned with the rest: the default pads rows to 8 bins (whole
  // 128-byte lines for the y and outer tiles); unpadded rows move fewer bytes, which pays on
  // small grids where the padding is a large share.  Per pitch, each pass is tuned on its own.
  struct Shape { int nxp, R, in_x, TXm, in_m, TXo, in_o; double t; };
  const Shape def{g.nxp, h->L.R, h->L.in_x, h->L.TXm, h->L.in_m, h->L.TXo, h->L.in_o, 0.0};
  Shape best = def;
  bool have_best = false;
  const int pitches[2] = {def.nxp, g.nxh};
  for (int pi = 0; pi < 2; ++pi) {
    if (pi == 1 && pitches[1] == pitches[0]) break;
    g.nxp = pitches[pi];
    g.Nh = (long long)g.nxp * g.ny * g.nz;
    Shape cur = def;
    cur.nxp = g.nxp;
    double total = 0.0;
    // x passes: block height and register staging (forward and inverse together)
    {
      double bt = 0.0;
      const int rmax = std::min(16, rows);
      for (int pass = 0; pass < 2; ++pass)
        for (int r = rmax; r >= 1; --r)
          for (int ip = 1; ip >= 0; --ip) {
            const bool incumbent = (r == def.R && ip == def.in_x);
            if ((pass == 0) != incumbent) continue;  // time the incumbent first
            if (ip && !inplace_ok(h->plan[0], (C * r + 1) / 2)) continue;
            if (!incumbent && std::max(xfwd_smem(g, r, ip), xinv_smem(g, r, ip)) > kLdsTune) continue;
            XFwdArgs a = xfwd_args(h);
            a.in = h->r;
            a.p = h->p;
            a.R = r;
            a.nblocks = (rows + r - 1) / r;
            a.inplace = ip;
            XInvArgs ai = xinv_args(h);
            ai.R = r;
            ai.nblocks = a.nblocks;
            ai.inplace = ip;
            double ms = 0.0;
            FH_CK(time_launches(h, reps, [&]() {
              hipError_t e = launch_xfwd(prod, h->matcode, a, Bt, h->stream);
              return e == hipSuccess ? launch_xinv(CONS_CGUPD, ai, Bt, h->stream) : e;
            }, &ms));
            if (incumbent) bt = ms;
            else if (ms < kGain * bt) { bt = ms; cur.R = r; cur.in_x = ip; }
          }
      total += bt;
    }
    // y passes (3D): kx bins per block, forward and inverse together
    if (g.ndim == 3) {
      double bt = 0.0;
      for (int pass = 0; pass < 2; ++pass)
        for (int t = std::min(32, g.nxh); t >= 1; --t)
          for (int ip = 1; ip >= 0; --ip) {
            const bool incumbent = (t == def.TXm && ip == def.in_m);
            if ((pass == 0) != incumbent) continue;
            if (ip && !inplace_ok(h->plan[1], mid_sequences(g, t, 1, 1))) continue;
            if (!incumbent && (mid_smem(g, t, ip, 1, 1) > kLdsTune || !mid_fits(g, t, 1, 1))) continue;
            const AxisArgs a = axis_args(h, 1, t, h->st, ip);
            double ms = 0.0;
            FH_CK(time_launches(h, reps, [&]() {
              hipError_t e = launch_mid(-1, a, Bt, h->stream);
              return e == hipSuccess ? launch_mid(1, a, Bt, h->stream) : e;
            }, &ms));
            if (incumbent) bt = ms;
            else if (ms < kGain * bt) { bt = ms; cur.TXm = t; cur.in_m = ip; }
          }
      total += bt;
    }
    // outer pass: kx bins per block
    {
      double bt = 0.0;
      for (int pass = 0; pass < 2; ++pass)
        for (int t = std::min(32, g.nxh); t >= 1; --t)
          for (int ip = 1; ip >= 0; --ip) {
            const bool incumbent = (t == def.TXo && ip == def.in_o);
            if ((pass == 0) != incumbent) continue;
            if (ip && !outer_inplace_ok(g, pouter, t)) continue;
            if (!incumbent && outer_smem(g, t, ip) > kLdsTune) continue;
            const AxisArgs a = axis_args(h, g.ndim - 1, t, h->st, ip);
            double ms = 0.0;
            FH_CK(time_launches(h, reps, [&]() { return launch_outer(OUTER_PROJECT, a, Bt, h->stream); }, &ms));
            if (incumbent) bt = ms;
            else if (ms < kGain * bt) { bt = ms; cur.TXo = t; cur.in_o = ip; }
          }
      total += bt;
    }
    cur.t = total;
    if (!have_best || total < kGain * best.t) {
      best = cur;
      have_best = true;
    }
  }
  g.nxp = best.nxp;
  g.Nh = (long long)g.nxp * g.ny * g.nz;
  h->L.R = best.R;
  h->L.in_x = best.in_x;
  h->L.nblk_x = (rows + best.R - 1) / best.R;
  h->L.TXm = best.TXm;
  h->L.in_m = best.in_m;
  h->L.TXo = best.TXo;
  h->L.in_o = best.in_o;
  h->L.smem_max = smem_needed(g, h->plan, h->L);
  if (shape) fft_homog_get_launch_shape(h, shape);
  return FFT_HOMOG_OK;
}

int fft_homog_set_placement(fft_homog_t* h, size_t stagger) {
  if (!h) return FFT_HOMOG_EINVAL;
  if (stagger % kAlign != 0 || 4 * stagger > h->L.slack)
    return fail(h, FFT_HOMOG_EINVAL, "stagger not a multiple of 256 or beyond the layout's slack");
  drop_graphs(h);
  place_work_vectors(h, stagger);
  return FFT_HOMOG_OK;
}

int fft_homog_tune_placement(fft_homog_t* h, int reps, size_t* stagger) {
  if (!h || reps < 1) return fail(h, FFT_HOMOG_EINVAL, "bad arguments");
  if (h->L.slack == 0) {  // no room to stagger: the only placement is the current one
    if (stagger) *stagger = h->stagger;
    return FFT_HOMOG_OK;
  }
  const Geom& g = h->g;
  const int B = h->L.B;
  const int Bt = (int)std::max(1LL, std::min((long long)B, (1LL << 22) / g.N));
  const double kGain = 0.98;  // a new placement must be clearly faster than the incumbent
  drop_graphs(h);
  const int prod = h->kst ? PROD_CGOP_STORED : PROD_CGOP;
  const size_t vec = (size_t)Bt * g.c * g.N * sizeof(double);
  const size_t inc = h->stagger;
  size_t best = inc;
  double best_t = 0.0;
  for (int pass = 0; pass < 2; ++pass)
    for (const size_t s : kStaggers) {
      const bool incumbent = s == inc;
      if ((pass == 0) != incumbent || 4 * s > h->L.slack) continue;  // the incumbent first
      place_work_vectors(h, s);
      // zero work vectors, every right-hand side running with alpha = beta = 0 (as in the
      // launch-shape autotuner): the x passes do all their loads and stores, the state stays put
      FH_CK(hipMemsetAsync(h->x, 0, vec, h->stream));
      FH_CK(hipMemsetAsync(h->r, 0, vec, h->stream));
      FH_CK(hipMemsetAsync(h->p, 0, vec, h->stream));
      const int rc = upload_states(h, Bt);
      if (rc) return rc;
      XFwdArgs a = xfwd_args(h);
      a.in = h->r;
      a.p = h->p;
      XInvArgs ai = xinv_args(h);
      double ms = 0.0;
      FH_CK(time_launches(h, reps, [&]() {
        hipError_t e = launch_xfwd(prod, h->matcode, a, Bt, h->stream);
        return e == hipSuccess ? launch_xinv(CONS_CGUPD, ai, Bt, h->stream) : e;
      }, &ms));
      if (incumbent) best_t = ms;
      else if (ms < kGain * best_t) {
        best_t = ms;
        best = s;
      }
    }
  place_work_vectors(h, best);
  if (stagger) *stagger = best;
  return FFT_HOMOG_OK;
}

int fft_homog_project_noalloc(const fft_homog_desc* d, const double* in, double* out, int batch, void* hip_stream) {
  if (!in || !out || batch < 1) return create_fail(FFT_HOMOG_EINVAL, "null field or batch < 1", hipSuccess);
  Layout L;
  const int rc = make_layout(d, &L);
  if (rc) return create_fail(rc, "invalid or unsupported descriptor", hipSuccess);
  Geom g;
  make_geom(d, &g);
  AxisPlan pl[3];
  make_plans(d, L.chirp, pl, &g);
  // scratch: FFT tables of the axes, then the half spectrum [batch][c][z][y][pitch]
  size_t off = 0;
  size_t tw_off[3] = {0, 0, 0};
  for (int a = 0; a < d->ndim; ++a) {
    tw_off[a] = off;
    off = align_up(off + plan_table_elems(pl[a]) * sizeof(double2));
  }
  const size_t spec_off = off;
  const size_t need = spec_off + (size_t)batch * g.c * g.Nh * sizeof(double2);
  if (need > kNoAllocScratchBytes) {
    char msg[160];
    snprintf(msg, sizeof(msg), "needs %zu bytes of scratch; the allocation-free projection has %zu per device",
             need, kNoAllocScratchBytes);
    return create_fail(FFT_HOMOG_EWORKSPACE, msg, hipSuccess);
  }
  char* base = nullptr;
  hipError_t e = noalloc_scratch_address((void**)&base);
  if (e != hipSuccess) return create_fail(FFT_HOMOG_EDEVICE, "hipGetSymbolAddress(scratch)", e);
  const hipStream_t s = (hipStream_t)hip_stream;
  for (int a = 0; a < d->ndim && e == hipSuccess; ++a) e = launch_plan_tables(&pl[a], (double2*)(base + tw_off[a]), s, true);
  if (d->ndim == 2) pl[2] = pl[1];
  const int matcode = material_code(d);
  if (e == hipSuccess) e = set_smem_limits(g, matcode, L.smem_max);
  if (e == hipSuccess) e = enqueue_projection(g, pl, L, matcode, in, out, (double2*)(base + spec_off), batch, s);
  if (e != hipSuccess) return create_fail(FFT_HOMOG_EDEVICE, "projection launch", e);
  g_create_err[0] = 0;
  return FFT_HOMOG_OK;
}

}  // extern "C"
