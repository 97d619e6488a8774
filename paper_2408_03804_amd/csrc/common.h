// Types shared by the host driver and the kernels (host-compilable: no device-only code).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fh {

constexpr int kMaxStages = 20;
constexpr int kMaxC = 9;
constexpr int kMaxAxis = 1024;
constexpr int kThreads = 256;
constexpr int kMaxPhase = 256;  // phase-table rows reserved per cell

// Radix schedules compiled into the FFT engine for the common axis lengths; the
// host factorisation returns the same schedule for these lengths.
__host__ __device__ constexpr int fixed_nstages(int n) {
  return n == 256 ? 2 : n == 192 ? 3 : n == 160 ? 3 : n == 128 ? 2 : n == 96 ? 3 : n == 80 ? 2 : n == 64 ? 2
       : n == 48 ? 2 : n == 32 ? 2 : n == 16 ? 1 : n == 8 ? 1 : 0;
}
__host__ __device__ constexpr int fixed_radix(int n, int st) {
  return n == 256 ? 16
       : n == 192 ? (st == 0 ? 16 : st == 1 ? 4 : 3)
       : n == 160 ? (st == 0 ? 16 : st == 1 ? 5 : 2)
       : n == 128 ? (st == 0 ? 16 : 8)
       : n == 96 ? (st == 0 ? 8 : st == 1 ? 4 : 3)
       : n == 80 ? (st == 0 ? 16 : 5)
       : n == 64 ? 8
       : n == 48 ? (st == 0 ? 16 : 3)
       : n == 32 ? (st == 0 ? 8 : 4)
       : n == 16 ? 16
       : 8;
}

// Exact w / d for w * d < 2^32 with a precomputed multiplier m = floor(2^32 / d) + 1
// (d = 1 has no 32-bit multiplier and is passed through).
struct FastDiv {
  unsigned d;
  unsigned m;
};
__host__ __device__ inline FastDiv make_fastdiv(unsigned d) { return FastDiv{d, d > 1 ? 0xFFFFFFFFu / d + 1u : 0u}; }

// register-staged FFT stages hold at most this many elements per thread
constexpr int kInplaceElems = 16;

// Tiles of kx bins of the y and outer passes: nxh bins in tiles of TX, tile b starting at bin b * TX.
__host__ __device__ inline int kx_tiles(int nxh, int TX) { return (nxh + TX - 1) / TX; }
__host__ __device__ inline int kx_tile_width(int nxh, int TX, int b) { return b * TX + TX <= nxh ? TX : nxh - b * TX; }
__host__ __device__ inline int kx_tile_max(int nxh, int TX) { return TX < nxh ? TX : nxh; }

// Factorisation of one FFT axis into Stockham stages and its twiddle table
// tw[j] = exp(-2 pi i j / L), j < L, of the transform length L the stages run on (device memory,
// computed on the device from exact rational arguments).
// Chirp-z axes (m > 0): a length n whose direct prime stages would cost more than the chirp-z
// (Bluestein) form runs as a cyclic convolution of length m >= 2n - 1 (factors 2, 3 and 5): the
// stages (nstages, radix, tw) are those of length m; chirp[j] = exp(-i pi j^2 / n), j < n, and
// filt = FFT_m(h) / m with h_j = h_(m-j) = conj(chirp[j]) for j < n and zero between.
struct AxisPlan {
  int n;
  int m;         // chirp-z convolution length, 0: the stages run on n itself
  int nstages;
  int radix[kMaxStages];
  const double2* tw;
  const double2* chirp;  // chirp-z axes only
  const double2* filt;   // chirp-z axes only
};

// Rows per sequence that a transform of this axis occupies in LDS.
__host__ __device__ inline int lds_len(const AxisPlan& p) { return p.m > 0 ? p.m : p.n; }

// Grid geometry.  2D grids are stored with nz = 1; the "outer" axis is the
// slowest non-trivial one (z in 3D, y in 2D) and the "mid" axis is y in 3D.
struct Geom {
  int ndim;
  int c;       // packed components per voxel
  int nx, ny, nz;
  int nxh;     // nx/2 + 1 half-spectrum bins along x
  int nxp;     // row pitch of the stored half spectrum (nxh rounded up to 8 bins = 128 bytes)
  int lx, lm, lo;  // LDS rows per sequence of the x, mid and outer transforms (lds_len of their plans)
  int n_outer, n_mid;
  long long N;   // voxels
  long long Nh;  // stored half-spectrum entries per component (nxp * ny * nz)
  double ks[3];  // 2 pi / L along x, y, z
  int small;     // small strain (Mandel packing) or finite strain
};

// Per-voxel material parameters: row table[tstride * phase[v]] holds (lam, mu) and,
// for J2 plasticity, (sig_y, H); lam and mu are multiplied by scale[v] = density^p,
// precomputed once per set_material (nullable: 1).  J2 also reads the plastic history
// of the voxel: hist[k * hN + v], k < c (packed plastic strain) and k = c (cumulative
// plastic strain).
struct MatParams {
  const uint8_t* phase;
  const double* table;    // [nphase][tstride]
  const double* scale;    // nullable
  const double* hist;     // J2 only: [c + 1][N]
  long long hN;           // voxels (history stride)
  int tstride;            // 2, or 4 for J2
};

// CG bookkeeping of one right-hand side, kept on the device so alpha and beta
// never leave it.  status: see CgStatus.
struct CgState {
  double rr;        // current <r, r>
  double rr0;       // <b, b>
  double pq;        // <p, K:p>
  double alpha;
  double beta;
  double src2;      // squared norm of the field whose projection is the right-hand side
  double tol;       // relative CG tolerance
  double pad0;
  int iters;
  int status;
  int first;        // next CG iteration starts with p = r
  int max_iters;
  int domain;       // constitutive domain error raised (det F <= 0 or non-finite stress)
  int pq_fail;      // this iteration's <p, K:p> was not positive; the <r, r> step stops the CG
  int pad1[2];
};

enum CgStatus { CG_RUNNING = 0, CG_CONVERGED = 1, CG_ZERO_RHS = 2, CG_BREAKDOWN = 3, CG_MAXIT = 4 };

}  // namespace fh
