// Kernel launchers used by the host driver (all enqueue on the given stream).
#pragma once

#include "common.h"

namespace fh {

enum Producer { PROD_IDENT = 0, PROD_STRESS = 1, PROD_CGOP = 2, PROD_TRHS = 3, PROD_CGOP_STORED = 4, PROD_ADJ = 5 };
enum Consumer { CONS_IDENT = 0, CONS_RHS = 1, CONS_CGUPD = 2 };
enum OuterMode { OUTER_PROJECT = 0, OUTER_FWD = 1, OUTER_INV = 2 };
enum Reduce { RED_SRC = 0, RED_RHS = 1, RED_PQ = 2, RED_RR = 3 };

// x-axis forward pass: per-voxel producer, then real-to-complex FFT along x.
struct XFwdArgs {
  Geom g;
  AxisPlan px;
  int R;                 // rows (y,z lines) per block
  int nblocks;           // blocks per right-hand side
  int inplace;           // FFT stages staged through registers (one LDS buffer)
  const double* in;      // IDENT: field [B][c][N]; CGOP: residual r [B][c][N]
  double* p;             // CGOP: search direction, updated in place
  double* x;             // CGOP: CG solution, receives the previous iteration's alpha p
  const double* F;       // linearisation point / strain [c][N]
  const double* Kst;     // stored tangent [c(c+1)/2][N]
  double2* spec;         // [B][c][Nh]
  MatParams mat;          // cell 0; cell i has its phase map at phase + i N, its table at table + i 2 kMaxPhase
  int per_inst;          // right-hand sides per cell of a multi-cell batch (0: one cell, every b uses cell 0)
  const int* active;     // nullable: right-hand side of launch index blockIdx.y (the running ones)
  CgState* st;           // per right-hand side
  double* partials;      // [B][nblocks]
  double unit[kMaxC];    // TRHS: load l of a cell is unit[l] * e_l in the packed basis; ADJ: packed W
  double w_energy;       // ADJ: weight of the energy in the objective
};

// x-axis inverse pass: complex-to-real FFT along x, then per-voxel consumer.
struct XInvArgs {
  Geom g;
  AxisPlan px;
  int R;
  int nblocks;
  int inplace;
  const double2* spec;
  double* out;           // IDENT output [B][c][N]
  double* x;             // RHS: CG solution [B][c][N], set to zero
  double* r;             // CG residual [B][c][N]
  const int* active;     // nullable: right-hand side of launch index blockIdx.y
  CgState* st;
  double* partials;
  double scale;          // 1 / N
};

// y (3D) or outer-axis pass over the half spectrum.
struct AxisArgs {
  Geom g;
  AxisPlan pl;
  int TX;                // kx bins per block
  int ZB;                // y pass: consecutive z planes per block (1 for the other passes)
  int inplace;
  int proj;              // y pass inside the projection chain (finite strain 3D: the row-wise
                         // y passes that carry two components per row to the outer pass)
  double2* spec;
  const CgState* st;     // nullable: skip right-hand sides whose CG is not running
  const int* active;     // nullable: right-hand side of each launch-index group
  // nullable (outer pass of a CG iteration): one block per right-hand side also sums the x
  // pass's <p, K:p> block partials and sets alpha, in place of a separate reduction launch
  CgState* pq_st;
  const double* pq_partials;
  int pq_nblocks;
};

// dynamic LDS bytes of each pass; `inplace` drops the ping-pong buffer
size_t xfwd_smem(const Geom& g, int R, int inplace);
size_t xinv_smem(const Geom& g, int R, int inplace);
// y pass; proj != 0: the projection chain's y pass (three tiles per block for finite strain 3D)
size_t mid_smem(const Geom& g, int TX, int inplace, int ZB = 1, int proj = 0);
// sequences of one FFT call of a y-pass block of TX bins and ZB planes
int mid_sequences(const Geom& g, int TX, int ZB, int proj);
// the row-wise finite-strain y pass holds kFrowHeld elements per thread: ny * TX * ZB must fit
constexpr int kFrowHeld = 8;
bool mid_fits(const Geom& g, int TX, int ZB, int proj);
// z planes per y-pass block for a tile of TX bins: 1 unless the tile spans the whole stored row,
// then as many as fit 32 KiB of LDS while the pass keeps about 512 blocks over B right-hand sides
int mid_planes(const Geom& g, const AxisPlan& pl, int TX, int inplace, long long B, int proj = 0);
// outer pass: LDS bytes, components per block and blocks per right-hand side along z of the
// grid, for the projection (mode OUTER_PROJECT) or a plain transform (OUTER_FWD / OUTER_INV)
size_t outer_smem(const Geom& g, int TX, int inplace, int mode = OUTER_PROJECT);
int outer_group(const Geom& g, int mode = OUTER_PROJECT);
int outer_groups_per_rhs(const Geom& g, int mode = OUTER_PROJECT);
// register staging possible for an outer-pass block of TX bins (widest tile)
bool outer_inplace_ok(const Geom& g, const AxisPlan& pl, int TX, int mode = OUTER_PROJECT);
// true if the y pass of the projection chain uses the row-wise finite-strain kernels
inline bool finite_rows(const Geom& g) { return !g.small && g.ndim == 3; }
// true if an in-place transform of nseq sequences of this plan fits the register staging
bool inplace_ok(const AxisPlan& pl, int nseq);

// FFT plan of an axis of length n: the direct stages, or the chirp-z form with its convolution
// length when the direct stages' prime lengths other than 2, 3 and 5 sum to more than chirp_above
// (0: never); table pointers left null.  False if n has no factorisation within kMaxStages stages.
bool make_plan(int n, AxisPlan* pl, int chirp_above);
// LDS rows per sequence of the x, mid and outer transforms of the plans pl[0..ndim-1]
void set_lds_lens(Geom* g, const AxisPlan* pl);
// the stages of length n (radices 16/8/4/2/3/5 and remaining primes); false if more than kMaxStages
bool factorize(int n, int* radix, int* nst);
// complex entries of an axis plan's device tables: twiddles of lds_len, then chirp (n) and filter (m)
size_t plan_table_elems(const AxisPlan& pl);
// set the table pointers of pl into `base` (plan_table_elems entries, device memory) and fill the
// tables: the twiddles (exp(-2 pi i j / L) by sincospi of exact rational arguments) unless the
// caller wrote them there, the chirp-z tables of a chirp-z plan
hipError_t launch_plan_tables(AxisPlan* pl, double2* base, hipStream_t s, bool twiddles);

hipError_t launch_xfwd(int prod, int mat, const XFwdArgs& a, int B, hipStream_t s);
hipError_t launch_xinv(int cons, const XInvArgs& a, int B, hipStream_t s);
hipError_t launch_mid(int dir, const AxisArgs& a, int B, hipStream_t s);
hipError_t launch_outer(int mode, const AxisArgs& a, int B, hipStream_t s);
// B blocks; block i reduces right-hand side active[i] (active nullable: i)
hipError_t launch_cg_reduce(int what, CgState* st, const double* partials, int nblocks, int B, hipStream_t s,
                            const int* active = nullptr);
// x += alpha p for every right-hand side whose CG stopped after at least one full iteration
hipError_t launch_cg_finish(double* x, const double* p, const CgState* st, const Geom& g, int B, hipStream_t s);

// Newton-level and post-processing kernels.
hipError_t launch_init_reference(double* F, const Geom& g, hipStream_t s);
hipError_t launch_shift(double* F, const double* delta, const Geom& g, hipStream_t s);
hipError_t launch_update(double* F, const double* x, double* partials, int nblocks, const Geom& g,
                         hipStream_t s);
hipError_t launch_homogenize(int mat, const double* F, MatParams m, double* partials, int nblocks,
                             const Geom& g, CgState* st, hipStream_t s);
hipError_t launch_tangent_matrix(int mat, const double* F, const double* X, const double* unit, MatParams m,
                                 double* partials, int nblocks, const Geom& g, hipStream_t s);
hipError_t launch_reduce_slots(const double* partials, int nslots, int nblocks, double* out, hipStream_t s);
hipError_t launch_store_tangent(int mat, const double* F, MatParams m, double* Kst, const Geom& g,
                                hipStream_t s);
hipError_t launch_expand(const double* packed, double* full, const Geom& g, hipStream_t s);
hipError_t launch_pack(const double* full, double* packed, const Geom& g, hipStream_t s);
hipError_t launch_stress_field(int mat, const double* F, MatParams m, double* full_out, double* energy_out,
                               const Geom& g, hipStream_t s);
hipError_t launch_simp_scale(const double* density, double p, double* scale, long long N, hipStream_t s);
hipError_t launch_check_phase(const uint8_t* phase, long long N, int nphase, int* flag, hipStream_t s);
hipError_t launch_debug_constitutive(int mat, const double* e, const double* de, double* P, double* KdE,
                                     double* psi, MatParams m, const Geom& g, hipStream_t s);
// dJ/drho_v = p / (N rho_v) [ w_e psi_v + (W + x_v) : P_v ]  (adjoint density gradient)
hipError_t launch_simp_gradient(int mat, const double* F, const double* x, MatParams m, const double* density,
                                double p, const double* W, double w_energy, double* grad, const Geom& g,
                                hipStream_t s);
// J2 plasticity: commit the history at the converged strain F (in place), and the
// cumulative plastic strain of the state at F
hipError_t launch_j2_commit(int mat, const double* F, MatParams m, double* hist, const Geom& g, hipStream_t s);
hipError_t launch_j2_plastic(int mat, const double* F, MatParams m, double* out, const Geom& g, hipStream_t s);
hipError_t set_smem_limits(const Geom& g, int mat, size_t bytes);
// the pass kernels with the chirp-z transform (kernels_chirp.hip), for plans with m > 0
hipError_t launch_xfwd_chirp(int prod, int mat, const XFwdArgs& a, dim3 grid, size_t sm, hipStream_t s);
hipError_t launch_xinv_chirp(int cons, const XInvArgs& a, dim3 grid, size_t sm, hipStream_t s);
hipError_t launch_mid_chirp(int dir, bool rows, const AxisArgs& a, dim3 grid, size_t sm, hipStream_t s);
hipError_t launch_outer_chirp(int mode, bool rows, const AxisArgs& a, dim3 grid, size_t sm, hipStream_t s);
hipError_t set_smem_limits_chirp(const Geom& g, int mat, size_t bytes);
// the CG-loop pass kernels for single axis lengths with compiled schedules (kernels_fixed.hip):
// lengths that have them; each launcher sets *done when it launched (else the caller launches the
// generic kernel)
bool fixed_len_kernels(int n);
hipError_t launch_xfwd_fixed(int prod, int mat, const XFwdArgs& a, dim3 grid, size_t sm, hipStream_t s, bool* done);
hipError_t launch_xinv_fixed(int cons, const XInvArgs& a, dim3 grid, size_t sm, hipStream_t s, bool* done);
hipError_t launch_mid_fixed(int dir, bool rows, const AxisArgs& a, dim3 grid, size_t sm, hipStream_t s, bool* done);
hipError_t launch_outer_fixed(int mode, bool rows, const AxisArgs& a, dim3 grid, size_t sm, hipStream_t s, bool* done);
hipError_t set_smem_limits_fixed(const Geom& g, int mat, size_t bytes);

// Scratch of the allocation-free projection: a file-scope device array of this many bytes per
// device (noalloc_scratch.hip); its address on the current device.
constexpr size_t kNoAllocScratchBytes = 64ull << 20;
hipError_t noalloc_scratch_address(void** out);

}  // namespace fh
