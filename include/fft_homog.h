/*
 * fft_homog.h -- C ABI of the MI355X (gfx950) Fourier-Galerkin homogenization library.
 *
 * The library solves the periodic cell problem of Pundir & Kammer,
 * "Simplifying FFT-based methods for solid mechanics with automatic
 * differentiation" (arXiv:2408.03804):
 *
 *   section 3, Fourier-Galerkin equilibrium:  IFFT( G-hat(xi) : FFT(sigma(eps)) ) = 0
 *   Appendix A, Algorithm 1:                  Newton outer loop, conjugate-gradient inner loop
 *   section 3.1 / 3.2:                        stress = d psi / d eps and the incremental stress
 *                                             K : d eps obtained by differentiating the energy
 *                                             (here: forward-mode dual numbers inside the kernels)
 *   section 3.3:                              homogenized stress (voxel average) and homogenized
 *                                             tangent C = d sigma-bar / d eps-bar
 *
 * All compute runs on one HIP device in FP64.  Every function returns an
 * fft_homog_status code; nothing throws across the ABI.  The library never
 * allocates device memory: the caller passes one device workspace whose size
 * fft_homog_workspace_size() reports.
 *
 * Conventions
 *   grid        n[0], n[1], n[2] points along x, y, z (2D: n[2] is ignored, taken as 1);
 *               device fields are stored component-major [comp][z][y][x], x fastest.
 *   macro load  small strain: Voigt order [11,22,33,23,13,12] with engineering shear
 *               strains (2D plane strain: [11,22,12]);
 *               finite strain: the deformation gradient F-bar, row-major 3x3 (2D: 2x2).
 *   macro out   stress in the same order without factors (small) / first Piola-Kirchhoff
 *               stress row-major (finite); tangent C_IJ = d out_I / d macro_J, row-major.
 *   ncomp       number of macro components: 3 / 6 (small, 2D / 3D), 4 / 9 (finite).
 *
 * Fixed behaviour (no descriptor switch):
 *   Nyquist     on an even axis the Nyquist index k = n/2 gets a zero wavevector component
 *               (the spectral derivative of the real trigonometric interpolant has no Nyquist
 *               part); the projection stays an exact, Hermitian-consistent per-mode projection.
 *               The paper only uses odd grids, where the rule never applies.
 *   determinism every reduction (CG dot products, Newton norms, homogenized averages) sums in a
 *               fixed order (wavefront shuffles, then fixed wave and block order; no atomics), so
 *               a repeated call on the same inputs and launch shape is bitwise identical.
 *   2D          plane strain unless FFT_HOMOG_FLAG_PLANE_STRESS.
 */
#ifndef FFT_HOMOG_H
#define FFT_HOMOG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fft_homog_status {
  FFT_HOMOG_OK = 0,
  FFT_HOMOG_EINVAL = 1,       /* invalid argument or descriptor */
  FFT_HOMOG_ENOTCONV = 2,     /* max_newton or max_cg reached; results and stats still written */
  FFT_HOMOG_EDOMAIN = 3,      /* det F <= 0 or a non-finite stress in the constitutive law */
  FFT_HOMOG_EBREAKDOWN = 4,   /* CG found <p, K:p> <= 0 (operator not positive definite) */
  FFT_HOMOG_ESTATE = 5,       /* call order violated (e.g. tangent before a successful solve) */
  FFT_HOMOG_EUNSUPPORTED = 6, /* grid size or option not supported by this build */
  FFT_HOMOG_EDEVICE = 7,      /* HIP runtime error; see fft_homog_last_error() */
  FFT_HOMOG_EWORKSPACE = 8    /* workspace too small or not 256-byte aligned */
} fft_homog_status;

enum { FFT_HOMOG_SMALL_STRAIN = 0, FFT_HOMOG_FINITE_STRAIN = 1 };

/* Constitutive laws (energy densities; lam, mu per phase):
 *   LINEAR_ELASTIC (small strain)   psi = lam/2 tr(eps)^2 + mu eps:eps
 *   NEO_HOOKEAN    (finite strain)  psi = mu/2 (tr(F^T F) - 3) - mu ln J + lam/2 (ln J)^2
 *   STVK           (finite strain)  psi = lam/2 tr(E)^2 + mu E:E,  E = (F^T F - I)/2
 *   J2_PLASTIC     (small strain)   von Mises plasticity with linear isotropic hardening
 *                                   (section 4.1.2, Appendix B): per phase lam, mu, yield
 *                                   stress sig_y and hardening modulus H; the stress is the
 *                                   predictor-corrector return mapping from the plastic
 *                                   history of the last load step (flow direction
 *                                   3/2 s/sig_eq), K : d_eps its forward-mode derivative.
 *                                   The history of a converged load step is committed when
 *                                   the next load step starts; the energy output is the
 *                                   stored elastic energy.
 * 2D is plane strain (eps_33 = 0, F_33 = 1). */
enum { FFT_HOMOG_LINEAR_ELASTIC = 0, FFT_HOMOG_NEO_HOOKEAN = 1, FFT_HOMOG_STVK = 2, FFT_HOMOG_J2_PLASTIC = 3 };

/* How the CG operator obtains K : p (section 3.2):
 *   RECOMPUTE  forward-over-forward dual-number JVP of the stress at every CG iteration
 *              (the paper's jvp variant; reads only the linearisation point)
 *   STORED     K materialised once per Newton iteration (the linearize / stored-tangent
 *              variant; ncomp(ncomp+1)/2 doubles per voxel) */
enum { FFT_HOMOG_K_RECOMPUTE = 0, FFT_HOMOG_K_STORED = 1 };

/* flags */
#define FFT_HOMOG_FLAG_TANGENT 1u  /* size the workspace for the ncomp-RHS tangent solve */
#define FFT_HOMOG_FLAG_DENSITY 2u  /* reserve a per-voxel density field (SIMP scaling) */
#define FFT_HOMOG_FLAG_PLANE_STRESS 8u /* 2D plane stress instead of plane strain: the out-of-plane
                                          normal stress of the 3D law vanishes at every voxel.
                                          Linear elasticity and St. Venant-Kirchhoff become their 2D
                                          laws with the reduced first Lame parameter
                                          2 lam mu / (lam + 2 mu); Neo-Hookean solves for F33 and
                                          J2 for eps_33 per voxel (set_material then needs lam >= 0,
                                          mu > 0, resp. mu > 0, 3 lam + 2 mu > 0), with the tangent
                                          condensed on the out-of-plane entry.  EINVAL for 3D */
#define FFT_HOMOG_FLAG_GRAPH 4u    /* enqueue full chunks of CG iterations by replaying a captured
                                      HIP graph (built on first use, rebuilt after set_material or
                                      autotune); results are bitwise those of direct launches */

enum { FFT_HOMOG_FIELD_STRAIN = 0, FFT_HOMOG_FIELD_STRESS = 1, FFT_HOMOG_FIELD_ENERGY = 2,
       FFT_HOMOG_FIELD_PLASTIC = 3 /* J2: cumulative plastic strain */ };

typedef struct fft_homog_desc {
  int ndim;          /* 2 or 3 */
  int n[3];          /* grid points along x, y, z; each 1..1024.  Factors 2, 3, 5 run radix stages;
                        other prime factors run a direct DFT stage of that length, or, when those
                        lengths add up to more than 70 (outer axis) or 150 (x and y axes), the axis
                        runs the chirp-z (Bluestein) transform through cyclic convolutions of a
                        length m >= 2n - 1 with factors 2, 3, 5 (more LDS per sequence; if its
                        buffers do not fit, every axis keeps the direct stages) */
  double len[3];     /* cell edge lengths along x, y, z (> 0); wavevector xi = 2 pi k / len */
  int kinematics;    /* FFT_HOMOG_SMALL_STRAIN or FFT_HOMOG_FINITE_STRAIN */
  int material;      /* LINEAR_ELASTIC or J2_PLASTIC (small), NEO_HOOKEAN or STVK (finite); J2
                        takes no FLAG_DENSITY and no batch > 1 */
  int nphase;        /* 1..256 */
  double tol_newton; /* Newton stop: ||dF||_2 / (sqrt(N) ||F-bar||_F) < tol_newton (RMS update over the
                        RMS macro load, section 4 / Appendix A); for a zero macro load (small
                        strain unloaded to zero) the scale is the updated field's norm ||F||_2 */
  double tol_cg;     /* CG stop: ||r|| <= tol_cg ||b|| */
  int max_newton;    /* per load increment */
  int max_cg;        /* per linear solve */
  int k_mode;        /* FFT_HOMOG_K_RECOMPUTE or FFT_HOMOG_K_STORED */
  unsigned flags;    /* FFT_HOMOG_FLAG_* */
  int batch;         /* independent cells of this grid held by the handle (0 or 1: one cell).
                        batch > 1 makes a multi-cell handle: it needs FLAG_TANGENT and
                        K_RECOMPUTE, takes no FLAG_DENSITY, and computes the homogenized tangent
                        of every cell at the reference state (eps = 0, F = I) with all
                        batch * ncomp linear solves in the same launches; solve, adjoint,
                        get_field and set_field return EUNSUPPORTED on it.  batch * ncomp^2
                        must not exceed 65535 (EUNSUPPORTED). */
} fft_homog_desc;

#define FFT_HOMOG_MAX_RECORDED 256

typedef struct fft_homog_stats {
  int status;                 /* fft_homog_status of the call */
  int increments;             /* load increments completed */
  int newton_iterations;      /* Newton iterations (linear solves) performed */
  int cg_iterations;          /* CG iterations summed over all linear solves */
  double newton_residual;     /* last ||dF||_2 / (sqrt(N) ||F-bar||_F) */
  double cg_residual;         /* last ||r|| / ||b|| of the last linear solve */
  double seconds;             /* device time of the call (HIP events on the stream) */
  int n_recorded;             /* entries of cg_per_newton written */
  int cg_per_newton[FFT_HOMOG_MAX_RECORDED]; /* CG iterations of each Newton iteration */
  int host_checks;            /* times the host read back the CG records during the call (each
                                 costs a stream synchronisation of some tens of microseconds) */
} fft_homog_stats;

typedef struct fft_homog fft_homog_t;

/* Size in bytes of the device workspace that fft_homog_create() needs for *d.
 * Pure host call.  EINVAL for an invalid descriptor, EUNSUPPORTED for a grid
 * size this build cannot transform. */
int fft_homog_workspace_size(const fft_homog_desc* d, size_t* bytes);

/* Create a solver instance.
 *   dev_workspace  device pointer, 256-byte aligned, >= workspace_size bytes; owned by the
 *                  caller, must outlive the handle and is not freed by fft_homog_destroy().
 *   hip_stream     hipStream_t on which every kernel of this handle is enqueued (NULL = the
 *                  default stream).
 * The strain field starts at the reference state (eps = 0, F = I); the
 * material starts as phase 0 everywhere with lam = mu = 0 until
 * fft_homog_set_material() is called. */
int fft_homog_create(const fft_homog_desc* d, void* dev_workspace, size_t bytes, void* hip_stream,
                     fft_homog_t** out);

/* Microstructure (the two-phase RVEs of section 4: per-phase Lame parameters).
 *   phase            device u8[N], layout [z][y][x]; copied into the workspace.
 *                    Multi-cell handle: u8[batch][N], the cells back to back.
 *   phase_lambda_mu  host f64[nphase][2] = (lam, mu) per phase; J2_PLASTIC: f64[nphase][4] =
 *                    (lam, mu, sig_y, H) with sig_y >= 0, H >= 0, 3 mu + H > 0.
 *                    Multi-cell handle: f64[batch][nphase][2], one table per cell.
 *   density          device f64[N] or NULL; when given (requires FLAG_DENSITY), lam and mu of
 *                    voxel v are scaled by density[v]^simp_p.
 * EINVAL if a phase id is >= nphase (checked on the device before returning). */
int fft_homog_set_material(fft_homog_t* h, const uint8_t* phase, const double* phase_lambda_mu,
                           const double* density, double simp_p);

/* Newton-CG solve (Appendix A, Algorithm 1) from the current state to the macro load
 * `macro` (host f64[ncomp]) in n_increments equal load steps; each step starts from the
 * previous converged field shifted by the uniform macro increment.
 * Outputs (host, each nullable): macro_stress f64[ncomp] = voxel average of the stress,
 * energy = voxel average of psi, stats.  Synchronous.  Returns OK, ENOTCONV,
 * EDOMAIN or EBREAKDOWN; on ENOTCONV the state and outputs are those reached. */
int fft_homog_solve(fft_homog_t* h, const double* macro, int n_increments, double* macro_stress,
                    double* energy, fft_homog_stats* st);

/* Homogenized tangent at the last converged state (section 3.3): host f64[ncomp][ncomp],
 * C_IJ = < (E_I + x_I) : K : (E_J + x_J) > with x_I solving G*(K:x_I) = -G*(K:E_I) for the
 * unit macro loads E_I; all ncomp linear solves run batched in the same launches.
 * Requires FLAG_TANGENT and a prior solve that returned OK (else ESTATE).
 * Multi-cell handle (desc.batch > 1): C is host f64[batch][ncomp][ncomp], each cell's tangent
 * at the reference state; no prior solve is needed.  stats.cg_per_newton lists the CG
 * iterations of the first 256 linear solves (cell-major, load index fastest). */
int fft_homog_tangent(fft_homog_t* h, double* C, fft_homog_stats* st);

/* Sensitivity of a homogenized objective to the per-voxel density (the paper's section 4.4.2
 * microstructure-optimisation use case), by the adjoint of the converged Fourier-Galerkin problem:
 *   J = w_energy * psi-bar + sum_I w_stress[I] * out_I     (out as returned by fft_homog_solve)
 *   solve G*(K : x) = -G*(w_energy P + K : W)              (one more CG solve, same operator)
 *   grad_density[v] = dJ/drho_v = p / (N rho_v) * (w_energy psi_v + (W + x_v) : P_v)
 * with W the macro tensor of the weights and lam, mu scaled by rho^p (set_material).
 * w_stress: host f64[ncomp]; grad_density: device f64[N], layout [z][y][x].  A pure energy
 * objective needs no CG (its right-hand side vanishes at equilibrium).  Requires a density
 * field (FLAG_DENSITY + set_material) and a prior solve that returned OK, else ESTATE. */
int fft_homog_adjoint(fft_homog_t* h, const double* w_stress, double w_energy, double* grad_density,
                      fft_homog_stats* st);

/* Copy a field of the current state to device memory dst:
 *   STRAIN / STRESS: f64[d*d][N], full row-major tensor components (small strain expanded from
 *                    the packed storage); ENERGY: f64[N]; PLASTIC (J2 only, else EINVAL): f64[N]
 *                    cumulative plastic strain of the current state. */
int fft_homog_get_field(fft_homog_t* h, int which, double* dst);

/* Restart from a given state: src device f64[d*d][N] full tensors, macro host f64[ncomp] the
 * macro load that state belongs to (its voxel average).  Small strain takes the symmetric part.
 * J2: the plastic history restarts virgin (zero). */
int fft_homog_set_field(fft_homog_t* h, const double* src, const double* macro);

/* Launch shape of the CG passes: shape[0] lines per x-pass block, shape[1] kx bins per
 * y-pass block, shape[2] kx bins per outer-pass block, shape[3..5] 1 if the x, y and outer
 * FFT stages are staged through registers (one LDS buffer) rather than ping-ponged,
 * shape[6] the row pitch of the stored half spectrum in bins (nx/2+1 rounded up to a
 * multiple of 8 by default, or unpadded). */
int fft_homog_get_launch_shape(const fft_homog_t* h, int shape[7]);

/* Set the launch shape (layout of fft_homog_get_launch_shape), e.g. one that
 * fft_homog_autotune chose for another handle of the same grid and batch.  EINVAL, with
 * nothing changed, unless: the pitch is nx/2+1 or its default padding; 1 <= shape[0] <= 16 and
 * <= ny*nz; 1 <= shape[1], shape[2] <= nx/2+1; register staging only where the FFT plan allows
 * it; every pass within 64 KiB of LDS (or the shape create chose).  Takes effect from the next
 * call; results agree with other shapes to rounding. */
int fft_homog_set_launch_shape(fft_homog_t* h, const int shape[7]);

/* Time every candidate launch shape of the CG passes on this handle's grid (each pass over
 * `reps` launches after one warm-up, HIP events on the handle's stream, over as many
 * right-hand sides of the batch as make up 4 Mi voxels) and keep the fastest; the chosen
 * shape is written to shape[7] (nullable) in the layout of fft_homog_get_launch_shape.
 * Candidates: both row pitches of the half spectrum; per pitch, x-pass block heights 1..16
 * and 1..32 kx bins per y- and outer-pass block, each with and without register staging,
 * within the default 64 KiB per-block LDS limit; a candidate must beat the default by 2 %.
 * The CG work vectors are overwritten; the strain state, the material and the last tangent's
 * inputs are kept, so it may be called between any two calls.  Results of later solves agree
 * with those of the default shape to rounding (the block height changes the order of the
 * partial sums). */
int fft_homog_autotune(fft_homog_t* h, int reps, int shape[7]);

/* Choose where the CG work vectors sit in the workspace.  F and the work vectors x, r, p lie at
 * multiples of the component size from one another; on large grids (one right-hand side of
 * 64 MiB or more) the layout keeps 16 MiB behind the half spectrum, and a stagger s moves x, r, p
 * and the spectrum by s, 2 s, 3 s and 4 s bytes.  How the x passes' streams spread over the HBM
 * channels depends on that placement and on the physical pages behind the workspace, so the
 * candidates {0, 256 B, 16 KiB, 256 KiB, 2 MiB, 4 MiB} are timed on this handle (reps launches of
 * the forward and inverse x passes each, work vectors zeroed) and the fastest is kept if it beats
 * the current one by 2 %.  Results do not depend on the placement (same kernels, same reduction
 * order): only the time does.  *stagger (may be NULL) receives the chosen s.  On smaller grids
 * the only candidate is 0.  Call it between solves, not during one (the work vectors are
 * overwritten); captured graphs are dropped.  EINVAL for reps < 1. */
int fft_homog_tune_placement(fft_homog_t* h, int reps, size_t* stagger);

/* Apply a work-vector stagger chosen elsewhere (see fft_homog_tune_placement): a multiple of 256
 * bytes with 4 * stagger within the layout's slack (16 MiB on large grids, else 0), else EINVAL.
 * Between solves only; the work vectors' contents are not moved. */
int fft_homog_set_placement(fft_homog_t* h, size_t stagger);

void fft_homog_destroy(fft_homog_t* h);
const char* fft_homog_strerror(int status);
/* Message of the last failure on handle h; with h == NULL, of the last failed
 * fft_homog_create on the calling thread. */
const char* fft_homog_last_error(const fft_homog_t* h);

/* For callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, hosts that forbid hipMalloc.  out = G*in, the compatibility projection of the
 * Fourier-Galerkin method (the same launches and results as fft_homog_debug_project on a handle
 * of descriptor *d, which needs a workspace), without a handle or a workspace:
 *   d          grid, kinematics and material as for fft_homog_create (material only selects the
 *              component count: 3 / 6 small strain, 4 / 9 finite strain); flags, tolerances and
 *              phases are ignored
 *   in, out    device f64[batch][c][z][y][x], packed layout of the stage-level entry points
 *              below; caller-owned; may not overlap
 *   batch      >= 1 fields
 *   hip_stream stream of the current device on which the work is enqueued (NULL = default).
 * Enqueue only: nothing is synchronised and nothing is allocated; out is complete when the stream
 * reaches this point.  Scratch (twiddle tables and the half spectrum, about
 * batch * c * Ny * Nz * (Nx/2+1 rounded up to 8) * 16 bytes) lives in a 64 MiB device array that
 * each device holds from library load to process end; larger requests return EWORKSPACE before
 * touching the device.  Every call on a device shares that device's array: calls that overlap in
 * time on one device (different streams, or different host threads) race and give wrong results.
 * Errors: EINVAL / EUNSUPPORTED (descriptor, null pointers, batch < 1), EWORKSPACE, EDEVICE;
 * fft_homog_last_error(NULL) describes the last failure on the calling thread. */
int fft_homog_project_noalloc(const fft_homog_desc* d, const double* in, double* out, int batch,
                              void* hip_stream);

/* ---- stage-level entry points (tests) --------------------------------------------------
 * Device arrays in the internal packed layout [batch][c][z][y][x]: c = ncomp, small strain
 * packed as Mandel components [11,22,33,sqrt2*23,sqrt2*13,sqrt2*12] (2D [11,22,sqrt2*12]),
 * finite strain F row-major.  Half spectra are complex f64 pairs [batch][c][z][y][nx/2+1].
 * batch <= ncomp when FLAG_TANGENT is set, else 1. */

/* Per voxel at strain e: P = d psi/de, K:de and psi by dual numbers (section 3.1, 3.2). */
int fft_homog_debug_constitutive(fft_homog_t* h, const double* e, const double* de, double* P,
                                 double* KdE, double* psi);
/* Unnormalised forward real-to-complex 3D (2D) DFT of each component. */
int fft_homog_debug_rfft(fft_homog_t* h, const double* in, double* spec, int batch);
/* Inverse of debug_rfft including the 1/N scaling. */
int fft_homog_debug_irfft(fft_homog_t* h, const double* spec, double* out, int batch);
/* out = G*in = IFFT(G-hat : FFT(in)) (section 3, projection operator). */
int fft_homog_debug_project(fft_homog_t* h, const double* in, double* out, int batch);
/* q = G*(K(eps_current) : p), the CG operator at the current state. */
int fft_homog_debug_apply_operator(fft_homog_t* h, const double* p, double* q, int batch);

/* Exactly `iters` CG iterations (Appendix A, the linear solve of one Newton iteration) on the
 * Newton system at the current state, G*(K:x) = -G*(P), from x = 0, with the handle's launch
 * shape and the solver's own kernels; no convergence test.  x_out and r_out (device, packed
 * layout, f64[c][N], caller-owned) receive the iterate x_iters and the residual r_iters.  The
 * strain state is unchanged.  ESTATE if the right-hand side is zero to rounding (nothing to
 * iterate), EBREAKDOWN if <p, K:p> <= 0 before `iters`, EUNSUPPORTED on multi-cell handles. */
int fft_homog_debug_cg(fft_homog_t* h, int iters, double* x_out, double* r_out);

/* Pure host function: the number of CG iterations the solver enqueues before its next host
 * check for a single right-hand side that has run `iters` iterations with residual norms
 * rr0 = <b,b>, rr = <r,r> and relative tolerance tol, given the iteration count and <r,r> at
 * the previous check (prev_iters < 0: none).  Between 1 and 16; at least 4 unless the decay
 * since the previous check agrees with the mean decay to a factor of two. */
int fft_homog_debug_cg_chunk(int iters, double rr0, double rr, double tol, int prev_iters, double prev_rr);

/* Average device time (ms, HIP events on the handle's stream) of each kernel of one CG
 * iteration (section 3 operator, Appendix A linear solve), measured over `iters` iterations
 * of the linear solve G*(K:x) = -G*(K:E_1) at the current state, batch 1, with the
 * convergence test disabled.  ms[7] receives, in launch order: x-pass forward (CG vector
 * update, K:p, x-FFT, partial <p,K:p>), a slot for a separate <p,K:p> reduction (0: one block
 * of the outer pass sums <p,K:p> and sets alpha), y-pass forward, outer pass (outer-axis FFT,
 * G-hat, inverse FFT), y-pass inverse, x-pass inverse (inverse x-FFT, residual update, partial
 * <r,r>), <r,r> reduction, beta and the convergence test; 2D grids report 0 for the y passes.
 * Leaves the strain state unchanged. */
int fft_homog_debug_time_cg(fft_homog_t* h, int iters, double* ms);

/* Sampled kernel timing inside the solver's own CG loops (solve, tangent and adjoint calls):
 * with every > 0, each every-th CG iteration enqueued on the handle's stream gets a HIP event
 * before its first launch and after each of its seven launches; every = 0 switches sampling
 * off.  Either call clears the accumulated samples.  Chunks replayed from a HIP graph
 * (FLAG_GRAPH) are not sampled.  The events add a few microseconds to each sampled iteration.
 * EINVAL for every < 0. */
int fft_homog_set_kernel_timing(fft_homog_t* h, int every);
/* Average device time (ms) of each launch of the sampled CG iterations since the last
 * fft_homog_set_kernel_timing, in the launch order and layout of fft_homog_debug_time_cg's
 * ms[7]: the time from the previous launch's end event to this launch's end event, so it
 * includes the launch's dispatch.  *samples receives the number of sampled iterations (ms is
 * all zero when it is 0). */
int fft_homog_get_kernel_timing(const fft_homog_t* h, double* ms, long long* samples);

#ifdef __cplusplus
}
#endif

#endif /* FFT_HOMOG_H */
