// HIP kernels of the Fourier-Galerkin Newton-CG solve for gfx950 (FP64): the pass kernels with
// the direct FFT stages and their launchers, the reductions, the Newton-level and
// post-processing kernels.  The pass kernels themselves are in pass_kernels.h.
#include "pass_kernels.h"

namespace fh {

// x += alpha p after the last CG iteration of each right-hand side (the
// iteration-k update is otherwise folded into the next x-forward pass)
__global__ void __launch_bounds__(kThreads) k_cg_finish(double* x, const double* p, const CgState* st, Geom g) {
  const int b = blockIdx.y;
  const CgState& S = st[b];
  if (S.iters < 1 || (S.status != CG_CONVERGED && S.status != CG_MAXIT)) return;
  const double alpha = S.alpha;
  const long long tot = (long long)g.c * g.N;
  const long long off = (long long)b * tot;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < tot; i += (long long)gridDim.x * blockDim.x)
    x[off + i] += alpha * p[off + i];
}

// ============================================================================
// reductions of block partial sums (one block per right-hand side, fixed order)
// ============================================================================
// One block per right-hand side sums the block partials in a fixed order.
constexpr int kReduceThreads = 1024;

template <int WHAT>
__global__ void __launch_bounds__(kReduceThreads) k_cg_reduce(CgState* st, const double* partials, int nblocks,
                                                                const int* active) {
  __shared__ double red[kReduceThreads / 64];
  const int b = active ? active[blockIdx.x] : (int)blockIdx.x;
  CgState& S = st[b];
  if (WHAT == RED_RR && S.status != CG_RUNNING) return;
  const double s = block_sum(strided_sum<8, kReduceThreads>(partials + (long long)b * nblocks, nblocks), red);
  if (threadIdx.x == 0) cg_finalize<WHAT>(S, s);
}

__global__ void __launch_bounds__(kThreads) k_reduce_slots(const double* partials, int nblocks, double* out) {
  __shared__ double red[kThreads / 64];
  const int sl = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) acc += partials[(long long)sl * nblocks + i];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) out[sl] = s;
}

// ============================================================================
// Newton-level and post-processing kernels (one voxel per thread)
// ============================================================================
struct Small9 {
  double v[kMaxC];
};

__global__ void k_init_reference(double* F, Geom g) {
  const long long N = g.N;
  const long long tot = N * g.c;
  const int d = g.ndim;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < tot;
       i += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(i / N);
    F[i] = (!g.small && (j / d) == (j % d)) ? 1.0 : 0.0;
  }
}

__global__ void k_shift(double* F, Small9 delta, Geom g) {
  const long long N = g.N;
  const long long tot = N * g.c;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < tot;
       i += (long long)gridDim.x * blockDim.x)
    F[i] += delta.v[i / N];
}

// F += x; block partials of ||x||^2 (slot 0) and of the updated ||F||^2 (slot 1)
__global__ void __launch_bounds__(kThreads) k_update(double* F, const double* x, double* partials, Geom g) {
  __shared__ double red[kThreads / 64];
  const long long N = g.N;
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  double acc = 0.0, accf = 0.0;
  if (v < N) {
    for (int j = 0; j < g.c; ++j) {
      const double dx = x[j * N + v];
      const double f = F[j * N + v] + dx;
      F[j * N + v] = f;
      acc += dx * dx;
      accf += f * f;
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
  const double sf = block_sum(accf, red);
  if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = sf;
}

// per-block sums of m values per thread, written to partials[slot][block]
__device__ __forceinline__ void block_sum_many(const double* vals, int m, double* sh, double* partials,
                                               int nblocks) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  for (int k = 0; k < m; ++k) {
    const double w = wave_sum(vals[k]);
    if (lane == 0) sh[k * nw + wid] = w;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < m; k += blockDim.x) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += sh[k * nw + w];
    partials[(long long)k * nblocks + blockIdx.x] = s;
  }
}

template <int MAT, int NDIM>
__global__ void __launch_bounds__(kThreads) k_homogenize(const double* F, MatParams m, double* partials,
                                                         int nblocks, Geom g, CgState* st) {
  constexpr int C = MatTraits<MAT, NDIM>::C;
  __shared__ double sh[(C + 1) * (kThreads / 64)];
  const long long N = g.N;
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  double vals[C + 1];
#pragma unroll
  for (int k = 0; k <= C; ++k) vals[k] = 0.0;
  if (v < N) {
    double e[C];
    Local L;
#pragma unroll
    for (int j = 0; j < C; ++j) e[j] = F[j * N + v];
    load_local<MAT, NDIM>(m, v, L);
    if (finite_mat(MAT)) {
      const double J = det_packed<NDIM>(e);
      if (!(finite_bits(J) && J > 0.0)) st[0].domain = 1;
    }
    vals[C] = stress_ad<MAT, NDIM>(e, L, vals);
  }
  block_sum_many(vals, C + 1, sh, partials, nblocks);
}

// C_IJ partial sums: (E_I + x_I) . K : (E_J + x_J) per voxel
template <int MAT, int NDIM>
__global__ void __launch_bounds__(kThreads) k_tangent_matrix(const double* F, const double* X, Small9 unit,
                                                             MatParams m, double* partials, int nblocks, Geom g) {
  constexpr int C = MatTraits<MAT, NDIM>::C;
  __shared__ double sh[C * C * (kThreads / 64)];
  const long long N = g.N;
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  double vals[C * C];
#pragma unroll
  for (int k = 0; k < C * C; ++k) vals[k] = 0.0;
  if (v < N) {
    double e[C];
    Local L;
    const bool need_e = MAT != MAT_LE;
#pragma unroll
    for (int j = 0; j < C; ++j) e[j] = need_e ? F[j * N + v] : 0.0;
    load_local<MAT, NDIM>(m, v, L);
    for (int J = 0; J < C; ++J) {
      double tJ[C], w[C];
#pragma unroll
      for (int j = 0; j < C; ++j) tJ[j] = X[((long long)J * C + j) * N + v] + (j == J ? unit.v[J] : 0.0);
      tangent_jvp_ad<MAT, NDIM>(e, tJ, L, w);
      for (int I = 0; I < C; ++I) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < C; ++j) s += (X[((long long)I * C + j) * N + v] + (j == I ? unit.v[I] : 0.0)) * w[j];
        vals[I * C + J] = s;
      }
    }
  }
  block_sum_many(vals, C * C, sh, partials, nblocks);
}

template <int MAT, int NDIM>
__global__ void __launch_bounds__(kThreads) k_store_tangent(const double* F, MatParams m, double* Kst, Geom g) {
  constexpr int C = MatTraits<MAT, NDIM>::C;
  const long long N = g.N;
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (v >= N) return;
  double e[C];
  Local L;
#pragma unroll
  for (int j = 0; j < C; ++j) e[j] = F[j * N + v];
  load_local<MAT, NDIM>(m, v, L);
  int idx = 0;
  for (int i = 0; i < C; ++i) {
    double de[C], col[C];
#pragma unroll
    for (int j = 0; j < C; ++j) de[j] = (j == i) ? 1.0 : 0.0;
    tangent_jvp_ad<MAT, NDIM>(e, de, L, col);  // column i = row i (K symmetric)
    for (int j = i; j < C; ++j) {
      Kst[(long long)idx * N + v] = col[j];
      ++idx;
    }
  }
}

// packed (Mandel / row-major F) -> full row-major d x d components
__global__ void k_expand(const double* packed, double* full, Geom g) {
  const long long N = g.N;
  const int d = g.ndim;
  const double h2 = 0.70710678118654752440;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N; v += (long long)gridDim.x * blockDim.x) {
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        double val;
        if (!g.small) {
          val = packed[(i * d + j) * N + v];
        } else if (i == j) {
          val = packed[i * N + v];
        } else {
          int k;
          if (d == 2) k = 2;
          else k = (i + j == 3) ? 3 : (i + j == 2 ? 4 : 5);  // (1,2)->3, (0,2)->4, (0,1)->5
          val = h2 * packed[k * N + v];
        }
        full[(i * d + j) * N + v] = val;
      }
  }
}

__global__ void k_pack(const double* full, double* packed, Geom g) {
  const long long N = g.N;
  const int d = g.ndim;
  const double r2 = 1.41421356237309504880;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N; v += (long long)gridDim.x * blockDim.x) {
    if (!g.small) {
      for (int k = 0; k < d * d; ++k) packed[k * N + v] = full[k * N + v];
    } else {
      for (int i = 0; i < d; ++i) packed[i * N + v] = full[(i * d + i) * N + v];
      auto sym = [&](int i, int j) { return 0.5 * (full[(i * d + j) * N + v] + full[(j * d + i) * N + v]); };
      if (d == 2) {
        packed[2 * N + v] = r2 * sym(0, 1);
      } else {
        packed[3 * N + v] = r2 * sym(1, 2);
        packed[4 * N + v] = r2 * sym(0, 2);
        packed[5 * N + v] = r2 * sym(0, 1);
      }
    }
  }
}

// J2 (MAT_J2, or MAT_J2_PS under plane stress): history of the converged state at F of the step
template <int MAT, int NDIM>
__device__ inline void j2_commit_any(const double* e, const Local& L, double* h) {
  if constexpr (MAT == MAT_J2_PS) j2_ps_commit(e, L, h);
  else j2_commit<NDIM>(e, L, h);
}

// J2: move the plastic history to the converged state at F (one load step ends)
template <int MAT, int NDIM>
__global__ void __launch_bounds__(kThreads) k_j2_commit(const double* F, MatParams m, double* hist, Geom g) {
  constexpr int C = MatTraits<MAT, NDIM>::C;
  const long long N = g.N;
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (v >= N) return;
  double e[C], h[C + 1];
  Local L;
#pragma unroll
  for (int j = 0; j < C; ++j) e[j] = F[j * N + v];
  load_local<MAT, NDIM>(m, v, L);
  j2_commit_any<MAT, NDIM>(e, L, h);
#pragma unroll
  for (int k = 0; k <= C; ++k) hist[k * N + v] = h[k];
}

// J2: cumulative plastic strain of the state at F (history plus this step's increment)
template <int MAT, int NDIM>
__global__ void __launch_bounds__(kThreads) k_j2_plastic(const double* F, MatParams m, double* out, Geom g) {
  constexpr int C = MatTraits<MAT, NDIM>::C;
  const long long N = g.N;
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (v >= N) return;
  double e[C], h[C + 1];
  Local L;
#pragma unroll
  for (int j = 0; j < C; ++j) e[j] = F[j * N + v];
  load_local<MAT, NDIM>(m, v, L);
  j2_commit_any<MAT, NDIM>(e, L, h);
  out[v] = h[C];
}

template <int MAT, int NDIM>
__global__ void __launch_bounds__(kThreads) k_stress_field(const double* F, MatParams m, double* packed_out,
                                                           double* energy_out, Geom g) {
  constexpr int C = MatTraits<MAT, NDIM>::C;
  const long long N = g.N;
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (v >= N) return;
  double e[C], P[C];
  Local L;
#pragma unroll
  for (int j = 0; j < C; ++j) e[j] = F[j * N + v];
  load_local<MAT, NDIM>(m, v, L);
  const double psi = stress_ad<MAT, NDIM>(e, L, P);
  if (packed_out != nullptr) {
#pragma unroll
    for (int j = 0; j < C; ++j) packed_out[j * N + v] = P[j];
  }
  if (energy_out != nullptr) energy_out[v] = psi;
}

// Adjoint density gradient.  With lam, mu scaled by rho^p, d psi/d rho = (p/rho) psi and
// d P/d rho = (p/rho) P at fixed strain; x solves G*(K:x) = -G*(w_e P + K:W).
template <int MAT, int NDIM>
__global__ void __launch_bounds__(kThreads) k_simp_gradient(const double* F, const double* x, MatParams m,
                                                            const double* density, double p, Small9 W,
                                                            double w_energy, double* grad, Geom g) {
  constexpr int C = MatTraits<MAT, NDIM>::C;
  const long long N = g.N;
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (v >= N) return;
  double e[C], P[C];
  Local L;
#pragma unroll
  for (int j = 0; j < C; ++j) e[j] = F[j * N + v];
  load_local<MAT, NDIM>(m, v, L);
  const double psi = stress_ad<MAT, NDIM>(e, L, P);
  double wp = w_energy * psi;
#pragma unroll
  for (int j = 0; j < C; ++j) wp += (W.v[j] + x[j * N + v]) * P[j];
  grad[v] = p / ((double)N * density[v]) * wp;
}

// scale[v] = density[v]^p (SIMP interpolation of the Lame parameters)
// tw[m] = exp(-2 pi i m / n), m < n (twiddle table of one FFT axis computed on the device)
__global__ void k_twiddles(double2* tw, int n) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < n) {
    double sn, cs;
    sincospi(2.0 * (double)m / (double)n, &sn, &cs);
    tw[m] = make_double2(cs, -sn);
  }
}

// Chirp-z tables of an axis of length n with convolution length m (one block per filter bin k):
//   chirp[j] = exp(-i pi j^2 / n), j < n;
//   filt[k] = (1/m) sum_j h_j exp(-2 pi i j k / m), h_j = h_(m-j) = conj(chirp[j]) for j < n, 0 between.
// Every angle is reduced exactly in integers (j^2 mod 2n, j k mod m) before sincospi; the sum
// runs in a fixed order.
__global__ void __launch_bounds__(kThreads) k_chirp_tables(double2* chirp, double2* filt, int n, int m) {
  __shared__ double red[kThreads / 64];
  const int k = blockIdx.x;
  if (k == 0) {
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      double sn, cs;
      sincospi((double)(((long long)j * j) % (2LL * n)) / (double)n, &sn, &cs);
      chirp[j] = make_double2(cs, -sn);
    }
  }
  double re = 0.0, im = 0.0;
  for (int t = threadIdx.x; t < 2 * n - 1; t += blockDim.x) {
    const int r = t < n ? t : t - n + 1;     // chirp index |j|
    const int j = t < n ? t : m - r;         // position in the length-m sequence
    double hs, hc, es, ec;
    sincospi((double)(((long long)r * r) % (2LL * n)) / (double)n, &hs, &hc);          // h_j = exp(+i pi r^2 / n)
    sincospi(2.0 * (double)(((long long)j * k) % m) / (double)m, &es, &ec);          // exp(+2 pi i j k / m)
    // h_j * exp(-2 pi i j k / m)
    re += hc * ec + hs * es;
    im += hs * ec - hc * es;
  }
  re = block_sum(re, red);
  im = block_sum(im, red);
  if (threadIdx.x == 0) filt[k] = make_double2(re / m, im / m);
}

__global__ void k_simp_scale(const double* density, double p, double* scale, long long N) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N; v += (long long)gridDim.x * blockDim.x)
    scale[v] = pow(density[v], p);
}

__global__ void k_check_phase(const uint8_t* phase, long long N, int nphase, int* flag) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N; v += (long long)gridDim.x * blockDim.x)
    if (phase[v] >= nphase) flag[0] = 1;
}

template <int MAT, int NDIM>
__global__ void __launch_bounds__(kThreads) k_debug_constitutive(const double* e_in, const double* de_in, double* P,
                                                                 double* KdE, double* psi, MatParams m, Geom g) {
  constexpr int C = MatTraits<MAT, NDIM>::C;
  const long long N = g.N;
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (v >= N) return;
  double e[C], de[C], p[C], k[C];
  Local L;
#pragma unroll
  for (int j = 0; j < C; ++j) {
    e[j] = e_in[j * N + v];
    de[j] = de_in[j * N + v];
  }
  load_local<MAT, NDIM>(m, v, L);
  const double ps = stress_and_jvp_ad<MAT, NDIM>(e, de, L, p, k);
#pragma unroll
  for (int j = 0; j < C; ++j) {
    P[j * N + v] = p[j];
    KdE[j * N + v] = k[j];
  }
  psi[v] = ps;
}

// ============================================================================
// host launchers
// ============================================================================
static inline int nblk_rows(const Geom& g, int R) { return (g.ny * g.nz + R - 1) / R; }

// x passes whose rows hold the benchmark's length in 3D: the CG-loop kernels specialised for it
static inline bool x_fixed128(const Geom& g, const AxisPlan& px, int R, int inplace) {
  return inplace && g.ndim == 3 && px.n == 128 && fixed_one_ok(128, (g.c * R + 1) / 2);
}

hipError_t launch_xfwd(int prod, int mat, const XFwdArgs& a, int B, hipStream_t s) {
  dim3 grid(nblk_rows(a.g, a.R), B);
  const size_t sm = xfwd_smem(a.g, a.R, a.inplace);
  if (a.px.m > 0) return launch_xfwd_chirp(prod, mat, a, grid, sm, s);
  if (a.inplace && a.g.ndim == 3 && fixed_len_kernels(a.px.n)) {
    bool done = false;
    const hipError_t e = launch_xfwd_fixed(prod, mat, a, grid, sm, s, &done);
    if (done) return e;
  }
  if (prod == PROD_CGOP && x_fixed128(a.g, a.px, a.R, a.inplace)) {
#define FH_C(M, D) hipLaunchKernelGGL((k_xfwd<PROD_CGOP, M, D, (D == 3 ? 128 : 0)>), grid, dim3(kThreads), sm, s, a);
    FH_DISPATCH_MAT(mat, FH_C)
#undef FH_C
    return hipGetLastError();
  }
  return dispatch_xfwd<0>(prod, mat, a, grid, sm, s);
}

hipError_t launch_xinv(int cons, const XInvArgs& a, int B, hipStream_t s) {
  dim3 grid(nblk_rows(a.g, a.R), B);
  const size_t sm = xinv_smem(a.g, a.R, a.inplace);
  if (a.px.m > 0) return launch_xinv_chirp(cons, a, grid, sm, s);
  if (a.inplace && a.g.ndim == 3 && fixed_len_kernels(a.px.n)) {
    bool done = false;
    const hipError_t e = launch_xinv_fixed(cons, a, grid, sm, s, &done);
    if (done) return e;
  }
  if (cons == CONS_CGUPD && x_fixed128(a.g, a.px, a.R, a.inplace) && (a.g.c == 9 || a.g.c == 6)) {
    if (a.g.c == 9) hipLaunchKernelGGL((k_xinv<CONS_CGUPD, 9, 128>), grid, dim3(kThreads), sm, s, a);
    else hipLaunchKernelGGL((k_xinv<CONS_CGUPD, 6, 128>), grid, dim3(kThreads), sm, s, a);
    return hipGetLastError();
  }
  return dispatch_xinv<0>(cons, a, grid, sm, s);
}

hipError_t launch_mid(int dir, const AxisArgs& a, int B, hipStream_t s) {
  const bool rows = a.proj && finite_rows(a.g);
  dim3 grid(kx_tiles(a.g.nxh, a.TX), (a.g.nz + a.ZB - 1) / a.ZB, B * (rows ? 3 : a.g.c));
  const size_t sm = mid_smem(a.g, a.TX, a.inplace, a.ZB, a.proj);
  if (a.pl.m > 0) return launch_mid_chirp(dir, rows, a, grid, sm, s);
  if (a.inplace && fixed_len_kernels(a.pl.n)) {
    bool done = false;
    const hipError_t e = launch_mid_fixed(dir, rows, a, grid, sm, s, &done);
    if (done) return e;
  }
  // the benchmark's axis length gets its own kernels when every stage keeps one butterfly per thread
  if (rows && a.inplace && a.pl.n == 128 && fixed_one_ok(128, mid_sequences(a.g, a.TX, a.ZB, a.proj))) {
    if (dir < 0) hipLaunchKernelGGL((k_mid_frow<-1, 128>), grid, dim3(kThreads), sm, s, a);
    else hipLaunchKernelGGL((k_mid_frow<1, 128>), grid, dim3(kThreads), sm, s, a);
    return hipGetLastError();
  }
  return dispatch_mid<0>(dir, rows, a, grid, sm, s);
}

hipError_t launch_outer(int mode, const AxisArgs& a_in, int B, hipStream_t s) {
  AxisArgs a = a_in;
  const int G = outer_group(a.g, mode);
  // a plain transform may carry more sequences per block than the projection the shape was
  // chosen for: stage through the ping-pong buffer when they exceed the register staging, and
  // narrow the tile while that needs more than 64 KiB of LDS (the grid follows the tile)
  if (a.inplace && !outer_inplace_ok(a.g, a.pl, a.TX, mode)) a.inplace = 0;
  if (mode != OUTER_PROJECT) {
    while (a.TX > 1 && outer_smem(a.g, a.TX, a.inplace, mode) > 64 * 1024) {
      a.TX = (a.TX + 1) / 2;
      a.inplace = a_in.inplace && outer_inplace_ok(a.g, a.pl, a.TX, mode) ? 1 : 0;
    }
  }
  dim3 grid(kx_tiles(a.g.nxh, a.TX), a.g.n_mid, B * outer_groups_per_rhs(a.g, mode));
  const size_t sm = outer_smem(a.g, a.TX, a.inplace, mode);
  const bool rows = mode == OUTER_PROJECT && finite_rows(a.g);
  if (a.pl.m > 0) return launch_outer_chirp(mode, rows, a, grid, sm, s);
  if (a.inplace && fixed_len_kernels(a.pl.n)) {
    bool done = false;
    const hipError_t e = launch_outer_fixed(mode, rows, a, grid, sm, s, &done);
    if (done) return e;
  }
  if (rows && a.inplace && a.pl.n == 128 && fixed_one_ok(128, G * kx_tile_max(a.g.nxh, a.TX))) {
    hipLaunchKernelGGL((k_outer_frow<128>), grid, dim3(kThreads), sm, s, a);
    return hipGetLastError();
  }
  return dispatch_outer<0>(mode, rows, a, grid, sm, s);
}

hipError_t launch_cg_reduce(int what, CgState* st, const double* partials, int nblocks, int B, hipStream_t s,
                            const int* active) {
  switch (what) {
    case RED_SRC: hipLaunchKernelGGL((k_cg_reduce<RED_SRC>), dim3(B), dim3(kReduceThreads), 0, s, st, partials, nblocks, active); break;
    case RED_RHS: hipLaunchKernelGGL((k_cg_reduce<RED_RHS>), dim3(B), dim3(kReduceThreads), 0, s, st, partials, nblocks, active); break;
    case RED_RR: hipLaunchKernelGGL((k_cg_reduce<RED_RR>), dim3(B), dim3(kReduceThreads), 0, s, st, partials, nblocks, active); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cg_finish(double* x, const double* p, const CgState* st, const Geom& g, int B, hipStream_t s) {
  long long blk = ((long long)g.c * g.N + kThreads - 1) / kThreads;
  if (blk > 4096) blk = 4096;
  hipLaunchKernelGGL(k_cg_finish, dim3((unsigned)blk, B), dim3(kThreads), 0, s, x, p, st, g);
  return hipGetLastError();
}

static inline dim3 vox_grid(const Geom& g) { return dim3((unsigned)((g.N + kThreads - 1) / kThreads)); }
static inline dim3 stride_grid(long long work) {
  long long b = (work + kThreads - 1) / kThreads;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

hipError_t launch_init_reference(double* F, const Geom& g, hipStream_t s) {
  hipLaunchKernelGGL(k_init_reference, stride_grid(g.N * g.c), dim3(kThreads), 0, s, F, g);
  return hipGetLastError();
}

hipError_t launch_shift(double* F, const double* delta, const Geom& g, hipStream_t s) {
  Small9 d;
  for (int k = 0; k < kMaxC; ++k) d.v[k] = k < g.c ? delta[k] : 0.0;
  hipLaunchKernelGGL(k_shift, stride_grid(g.N * g.c), dim3(kThreads), 0, s, F, d, g);
  return hipGetLastError();
}

hipError_t launch_update(double* F, const double* x, double* partials, int nblocks, const Geom& g, hipStream_t s) {
  (void)nblocks;
  hipLaunchKernelGGL(k_update, vox_grid(g), dim3(kThreads), 0, s, F, x, partials, g);
  return hipGetLastError();
}

hipError_t launch_homogenize(int mat, const double* F, MatParams m, double* partials, int nblocks, const Geom& g,
                             CgState* st, hipStream_t s) {
#define FH_L(M, D) hipLaunchKernelGGL((k_homogenize<M, D>), vox_grid(g), dim3(kThreads), 0, s, F, m, partials, nblocks, g, st)
  FH_DISPATCH_MAT(mat, FH_L)
#undef FH_L
  return hipGetLastError();
}

hipError_t launch_tangent_matrix(int mat, const double* F, const double* X, const double* unit, MatParams m,
                                 double* partials, int nblocks, const Geom& g, hipStream_t s) {
  Small9 u;
  for (int k = 0; k < kMaxC; ++k) u.v[k] = k < g.c ? unit[k] : 0.0;
#define FH_L(M, D) \
  hipLaunchKernelGGL((k_tangent_matrix<M, D>), vox_grid(g), dim3(kThreads), 0, s, F, X, u, m, partials, nblocks, g)
  FH_DISPATCH_MAT(mat, FH_L)
#undef FH_L
  return hipGetLastError();
}

hipError_t launch_reduce_slots(const double* partials, int nslots, int nblocks, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_slots, dim3(nslots), dim3(kThreads), 0, s, partials, nblocks, out);
  return hipGetLastError();
}

hipError_t launch_store_tangent(int mat, const double* F, MatParams m, double* Kst, const Geom& g, hipStream_t s) {
#define FH_L(M, D) hipLaunchKernelGGL((k_store_tangent<M, D>), vox_grid(g), dim3(kThreads), 0, s, F, m, Kst, g)
  FH_DISPATCH_MAT(mat, FH_L)
#undef FH_L
  return hipGetLastError();
}

hipError_t launch_expand(const double* packed, double* full, const Geom& g, hipStream_t s) {
  hipLaunchKernelGGL(k_expand, stride_grid(g.N), dim3(kThreads), 0, s, packed, full, g);
  return hipGetLastError();
}

hipError_t launch_pack(const double* full, double* packed, const Geom& g, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, stride_grid(g.N), dim3(kThreads), 0, s, full, packed, g);
  return hipGetLastError();
}

hipError_t launch_j2_commit(int mat, const double* F, MatParams m, double* hist, const Geom& g, hipStream_t s) {
  if (mat == 6) hipLaunchKernelGGL((k_j2_commit<MAT_J2, 2>), vox_grid(g), dim3(kThreads), 0, s, F, m, hist, g);
  else if (mat == 7) hipLaunchKernelGGL((k_j2_commit<MAT_J2, 3>), vox_grid(g), dim3(kThreads), 0, s, F, m, hist, g);
  else if (mat == 9) hipLaunchKernelGGL((k_j2_commit<MAT_J2_PS, 2>), vox_grid(g), dim3(kThreads), 0, s, F, m, hist, g);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_j2_plastic(int mat, const double* F, MatParams m, double* out, const Geom& g, hipStream_t s) {
  if (mat == 6) hipLaunchKernelGGL((k_j2_plastic<MAT_J2, 2>), vox_grid(g), dim3(kThreads), 0, s, F, m, out, g);
  else if (mat == 7) hipLaunchKernelGGL((k_j2_plastic<MAT_J2, 3>), vox_grid(g), dim3(kThreads), 0, s, F, m, out, g);
  else if (mat == 9) hipLaunchKernelGGL((k_j2_plastic<MAT_J2_PS, 2>), vox_grid(g), dim3(kThreads), 0, s, F, m, out, g);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_stress_field(int mat, const double* F, MatParams m, double* packed_out, double* energy_out,
                               const Geom& g, hipStream_t s) {
#define FH_L(M, D) \
  hipLaunchKernelGGL((k_stress_field<M, D>), vox_grid(g), dim3(kThreads), 0, s, F, m, packed_out, energy_out, g)
  FH_DISPATCH_MAT(mat, FH_L)
#undef FH_L
  return hipGetLastError();
}

hipError_t launch_simp_gradient(int mat, const double* F, const double* x, MatParams m, const double* density,
                                double p, const double* W, double w_energy, double* grad, const Geom& g,
                                hipStream_t s) {
  Small9 w;
  for (int k = 0; k < kMaxC; ++k) w.v[k] = k < g.c ? W[k] : 0.0;
#define FH_L(M, D)                                                                                          \
  hipLaunchKernelGGL((k_simp_gradient<M, D>), vox_grid(g), dim3(kThreads), 0, s, F, x, m, density, p, w, \
                     w_energy, grad, g)
  FH_DISPATCH_MAT(mat, FH_L)
#undef FH_L
  return hipGetLastError();
}

hipError_t launch_plan_tables(AxisPlan* pl, double2* base, hipStream_t s, bool twiddles) {
  const int L = lds_len(*pl);
  pl->tw = base;
  pl->chirp = pl->m > 0 ? base + L : nullptr;
  pl->filt = pl->m > 0 ? base + L + pl->n : nullptr;
  hipError_t e = hipSuccess;
  if (twiddles) {
    hipLaunchKernelGGL(k_twiddles, dim3((unsigned)((L + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, base, L);
    e = hipGetLastError();
  }
  if (e == hipSuccess && pl->m > 0) {
    hipLaunchKernelGGL(k_chirp_tables, dim3((unsigned)pl->m), dim3(kThreads), 0, s, base + L, base + L + pl->n, pl->n,
                       pl->m);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_simp_scale(const double* density, double p, double* scale, long long N, hipStream_t s) {
  hipLaunchKernelGGL(k_simp_scale, stride_grid(N), dim3(kThreads), 0, s, density, p, scale, N);
  return hipGetLastError();
}

hipError_t launch_check_phase(const uint8_t* phase, long long N, int nphase, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_check_phase, stride_grid(N), dim3(kThreads), 0, s, phase, N, nphase, flag);
  return hipGetLastError();
}

hipError_t launch_debug_constitutive(int mat, const double* e, const double* de, double* P, double* KdE, double* psi,
                                     MatParams m, const Geom& g, hipStream_t s) {
#define FH_L(M, D) \
  hipLaunchKernelGGL((k_debug_constitutive<M, D>), vox_grid(g), dim3(kThreads), 0, s, e, de, P, KdE, psi, m, g)
  FH_DISPATCH_MAT(mat, FH_L)
#undef FH_L
  return hipGetLastError();
}

// Raise the dynamic-LDS limit of the FFT kernels when a plan needs more than 64 KiB.
hipError_t set_smem_limits(const Geom& g, int mat, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  hipError_t e = pass_smem_limits<0>(g, mat, bytes);
  const int attr = (int)hipFuncAttributeMaxDynamicSharedMemorySize;
#define FH_SET(fn) \
  if (e == hipSuccess) e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn), (hipFuncAttribute)attr, (int)bytes)
#define FH_L(M, D) FH_SET((k_xfwd<PROD_CGOP, M, D, (D == 3 ? 128 : 0)>));
  FH_DISPATCH_MAT(mat, FH_L)
#undef FH_L
  if (g.c == 6) FH_SET((k_xinv<CONS_CGUPD, 6, 128>));
  if (g.c == 9) FH_SET((k_xinv<CONS_CGUPD, 9, 128>));
  FH_SET((k_mid_frow<-1, 128>));
  FH_SET((k_mid_frow<1, 128>));
  FH_SET((k_outer_frow<128>));
#undef FH_SET
  if (e == hipSuccess && (g.lx != g.nx || g.lo != g.n_outer || (g.ndim == 3 && g.lm != g.ny)))
    e = set_smem_limits_chirp(g, mat, bytes);
  if (e == hipSuccess) e = set_smem_limits_fixed(g, mat, bytes);
  return e;
}

}  // namespace fh
