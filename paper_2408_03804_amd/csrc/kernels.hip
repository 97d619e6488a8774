// HIP kernels of the Fourier-Galerkin Newton-CG solve for gfx950 (FP64).
//
// One CG iteration (section 3 equilibrium operator, section 3.2 incremental
// stress, Appendix A linear solve) is five passes over the data:
//
//   xfwd   per voxel: x += alpha_prev p, p = r + beta p, tau = K(F) : p by dual
//          numbers, partial <p, tau>; real-to-complex FFT of tau along x
//   mid    complex FFT along y of the half spectrum            (3D only)
//   outer  FFT along the outer axis, G-hat(xi) : tau-hat on each wavevector,
//          inverse FFT along the outer axis
//   mid    inverse FFT along y                                 (3D only)
//   xinv   complex-to-real FFT along x, r -= alpha q, partial <r, r>
//
// plus two one-block reductions that turn the partial sums into alpha and beta
// on the device.  <p, q> is taken as <p, K:p>: p lies in the range of the
// projection G (it is built from projected residuals) and G is self-adjoint, so
// <p, G(K:p)> = <G p, K:p> = <p, K:p> in exact arithmetic; q is therefore never
// stored.  The update x += alpha p of iteration k is applied by the xfwd pass of
// iteration k+1, which reads p anyway (k_cg_finish applies the last one).
#include "common.h"
#include "fft_lds.h"
#include "kernels.h"
#include "materials.h"

namespace fh {

// matcode = 2 * material + (ndim - 2)
#define FH_DISPATCH_MAT(matcode, MACRO) \
  switch (matcode) {                    \
    case 0: MACRO(MAT_LE, 2); break;    \
    case 1: MACRO(MAT_LE, 3); break;    \
    case 2: MACRO(MAT_NH, 2); break;    \
    case 3: MACRO(MAT_NH, 3); break;    \
    case 4: MACRO(MAT_STVK, 2); break;  \
    case 5: MACRO(MAT_STVK, 3); break;  \
    case 6: MACRO(MAT_J2, 2); break;    \
    case 7: MACRO(MAT_J2, 3); break;    \
    default: return hipErrorInvalidValue; \
  }

// Parameters (and for J2 the plastic history) of voxel v.
template <int MAT, int NDIM>
__device__ __forceinline__ void load_local(const MatParams& m, long long v, Local& L) {
  const int ph = m.phase[v];
  const double* row = m.table + (long long)m.tstride * ph;
  L.lam = row[0];
  L.mu = row[1];
  if (m.scale != nullptr) {
    const double s = m.scale[v];
    L.lam *= s;
    L.mu *= s;
  }
  if constexpr (MAT == MAT_J2) {
    constexpr int C = MatTraits<MAT_J2, NDIM>::C;
    L.sy = row[2];
    L.H = row[3];
#pragma unroll
    for (int k = 0; k <= C; ++k) L.hist[k] = m.hist[k * m.hN + v];
  }
}

__device__ __forceinline__ int ceil_div(int a, int b) { return (a + b - 1) / b; }

// FFT of a pass.  NF > 0: a kernel specialised for axis length NF with one butterfly per thread per
// stage -- only that length's code and a butterfly's registers (the launchers check fixed_one_ok);
// NF = 0: any length, with the register staging or the ping-pong buffer the host chose.
template <int D, int NF>
__device__ __forceinline__ void pass_fft(double2* A, double2* Bf, int nseq, const AxisPlan& pl, int inplace) {
  if constexpr (NF > 0) fft_fixed_one<NF, D>(A, nseq, pl.tw);
  else fft_lds_any<D>(A, Bf, nseq, pl, inplace);
}

// Streaming access for the CG vectors and the linearisation point: each is touched once
// per CG iteration, so keeping them out of the caches leaves room for the half spectrum
// that the FFT passes hand to each other.
__device__ __forceinline__ double ld_stream(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_stream(double* p, double v) { __builtin_nontemporal_store(v, p); }

// ============================================================================
// CG scalar bookkeeping from a reduced sum (fixed-order two-stage sums)
// ============================================================================
template <int WHAT>
__device__ __forceinline__ void cg_finalize(CgState& S, double s) {
  if (WHAT == RED_SRC) {
    S.src2 = s;
  } else if (WHAT == RED_RHS) {
    S.rr0 = s;
    S.rr = s;
    S.iters = 0;
    S.first = 1;
    S.beta = 0.0;
    if (!finite_bits(s)) S.status = CG_BREAKDOWN;
    else if (sqrt(s) <= 1e-13 * sqrt(S.src2)) S.status = CG_ZERO_RHS;
    else if (sqrt(s) <= S.tol * sqrt(s)) S.status = CG_CONVERGED;
    else if (S.max_iters <= 0) S.status = CG_MAXIT;
    else S.status = CG_RUNNING;
  } else if (WHAT == RED_PQ) {
    // runs inside the outer pass, whose other blocks read the status: a breakdown is only
    // flagged here and becomes the status at the <r, r> step
    S.pq = s;
    if (!(finite_bits(s) && s > 0.0)) S.pq_fail = 1;
    else S.alpha = S.rr / s;
  } else {  // RED_RR
    if (S.pq_fail) {
      S.status = CG_BREAKDOWN;
      return;
    }
    S.beta = s / S.rr;
    S.rr = s;
    S.iters += 1;
    S.first = 0;
    if (!finite_bits(s)) S.status = CG_BREAKDOWN;
    else if (sqrt(s) <= S.tol * sqrt(S.rr0)) S.status = CG_CONVERGED;
    else if (S.iters >= S.max_iters) S.status = CG_MAXIT;
  }
}

// ============================================================================
// x-axis forward pass
// ============================================================================
template <int PROD, int MAT, int NDIM, int NF = 0>
__global__ void __launch_bounds__(kThreads) k_xfwd(XFwdArgs a) {
  constexpr int C = MatTraits<MAT, NDIM>::C;
  constexpr bool CGOP = (PROD == PROD_CGOP || PROD == PROD_CGOP_STORED);
  const int b = a.active ? a.active[blockIdx.y] : (int)blockIdx.y;
  if (CGOP) {
    if (a.st[b].status != CG_RUNNING) return;
  }
  const Geom& g = a.g;
  // cell of this right-hand side and its load index within the cell
  MatParams mat = a.mat;
  int lb = b;
  if (a.per_inst > 0) {
    const int cell = b / a.per_inst;
    lb = b - cell * a.per_inst;
    mat.phase += (long long)cell * g.N;
    mat.table += (long long)cell * 2 * kMaxPhase;
  }
  const int nx = g.nx;
  const int rows = g.ny * g.nz;
  const int row0 = blockIdx.x * a.R;
  const int nr = min(a.R, rows - row0);
  const int nseq = C * nr;
  const int P = (nseq + 1) >> 1;
  extern __shared__ double2 smem[];
  double2* A = smem;
  // CG operator: strain staged by phase A (after the FFT buffers)
  const int nv = nr * nx;
  double* E = reinterpret_cast<double*>(smem + (size_t)(a.inplace ? 1 : 2) * nx * P);
  double2* Bf = smem + (size_t)nx * P;  // ping-pong partner (unused in place)
  __shared__ double red[kThreads / 64];

  double beta = 0.0, alpha_prev = 0.0;
  int first = 1;
  if (CGOP) {
    beta = a.st[b].beta;
    alpha_prev = a.st[b].alpha;
    first = a.st[b].first;
  }
  const long long N = g.N;
  double acc = 0.0;
  int bad = 0;

  // LDS slot of component j of row r at column x (two real rows per complex sequence)
  auto slot = [&](int j, int r, int x) -> double* {
    const int qr = j * nr + r;
    return reinterpret_cast<double*>(&A[x * P + (qr >> 1)]) + (qr & 1);
  };

  if (CGOP) {
    // phase A: every global load of the voxel in flight together.
    //   x += alpha_prev p_old ; p = r + beta p_old   (p staged in the FFT slots)
    //   strain staged for phase B
    for (int t = threadIdx.x; t < nv; t += blockDim.x) {
      const int r = t / nx;
      const int x = t - r * nx;
      const long long vox = (long long)(row0 + r) * nx + x;
      if (PROD == PROD_CGOP && MAT != MAT_LE) {
#pragma unroll
        for (int j = 0; j < C; ++j) E[j * nv + t] = ld_stream(a.F + j * N + vox);
      }
      if (MAT != MAT_J2) {
        Local L;
        load_local<MAT, NDIM>(mat, vox, L);  // brings the phase id and table line into cache
        (void)L;
      }
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const long long idx = ((long long)b * C + j) * N + vox;
        const double rj = ld_stream(a.in + idx);
        double pj;
        if (first) {
          pj = rj;
        } else {
          const double po = ld_stream(a.p + idx);
          st_stream(a.x + idx, ld_stream(a.x + idx) + alpha_prev * po);
          pj = rj + beta * po;
        }
        st_stream(a.p + idx, pj);
        *slot(j, r, x) = pj;
      }
    }
  }

  // phase B (or the only phase): per-voxel producer, result into the LDS slots
#pragma unroll 1
  for (int t = threadIdx.x; t < nr * nx; t += blockDim.x) {
    const int r = t / nx;
    const int x = t - r * nx;
    const long long vox = (long long)(row0 + r) * nx + x;
    double v[C];
    if (PROD == PROD_IDENT) {
#pragma unroll
      for (int j = 0; j < C; ++j) v[j] = a.in[((long long)b * C + j) * N + vox];
    } else {
      Local L;
      double e[C];
      // the linear elastic energy is quadratic: K does not depend on the strain,
      // so the tangent passes do not read it
      // (lam, mu) are re-read here (cache hits): staging them in LDS as well
      // raises the register count of the fused kernel by a third
      load_local<MAT, NDIM>(mat, vox, L);
      if (CGOP) {
#pragma unroll
        for (int j = 0; j < C; ++j) e[j] = (PROD == PROD_CGOP && MAT != MAT_LE) ? E[j * nv + t] : 0.0;
      } else {
        const bool need_e = (PROD == PROD_STRESS) || (PROD == PROD_ADJ) || (MAT != MAT_LE);
#pragma unroll
        for (int j = 0; j < C; ++j) e[j] = need_e ? a.F[j * N + vox] : 0.0;
      }
      if (PROD == PROD_STRESS) {
        if (MAT == MAT_NH || MAT == MAT_STVK) {
          const double J = det_packed<NDIM>(e);
          if (!(finite_bits(J) && J > 0.0)) bad = 1;
        }
        stress_ad<MAT, NDIM>(e, L, v);
#pragma unroll
        for (int j = 0; j < C; ++j) {
          acc += v[j] * v[j];
          if (!finite_bits(v[j])) bad = 1;
        }
      } else if (PROD == PROD_ADJ) {
        // objective gradient with respect to the strain: g = w_e P + K : W
        double P[C], W[C];
#pragma unroll
        for (int j = 0; j < C; ++j) W[j] = a.unit[j];
        stress_and_jvp_ad<MAT, NDIM>(e, W, L, P, v);
#pragma unroll
        for (int j = 0; j < C; ++j) {
          v[j] += a.w_energy * P[j];
          acc += v[j] * v[j];
        }
      } else if (PROD == PROD_TRHS) {
        double de[C];
#pragma unroll
        for (int j = 0; j < C; ++j) de[j] = (j == lb) ? a.unit[lb] : 0.0;
        tangent_jvp_ad<MAT, NDIM>(e, de, L, v);
#pragma unroll
        for (int j = 0; j < C; ++j) acc += v[j] * v[j];
      } else {  // CG operator: v = K : p with p from phase A
        double pv[C];
#pragma unroll
        for (int j = 0; j < C; ++j) pv[j] = *slot(j, r, x);
        if (PROD == PROD_CGOP) {
          tangent_jvp_ad<MAT, NDIM>(e, pv, L, v);
        } else {
          // stored symmetric tangent, upper triangle row by row
#pragma unroll
          for (int i = 0; i < C; ++i) v[i] = 0.0;
          int idx = 0;
#pragma unroll
          for (int i = 0; i < C; ++i) {
#pragma unroll
            for (int j = i; j < C; ++j) {
              const double k = a.Kst[(long long)idx * N + vox];
              v[i] += k * pv[j];
              if (j != i) v[j] += k * pv[i];
              ++idx;
            }
          }
        }
#pragma unroll
        for (int j = 0; j < C; ++j) acc += pv[j] * v[j];
      }
    }
#pragma unroll
    for (int j = 0; j < C; ++j) *slot(j, r, x) = v[j];
  }
  if (nseq & 1) {
    for (int x = threadIdx.x; x < nx; x += blockDim.x) A[x * P + P - 1].y = 0.0;
  }
  if (PROD == PROD_STRESS && bad) a.st[b].domain = 1;
  __syncthreads();

  pass_fft<-1, NF>(A, Bf, P, a.px, a.inplace);
  const double2* res = A;

  // separate the two real rows packed in each complex sequence
  const int nxh = g.nxh;
  const FastDiv fdh = make_fastdiv((unsigned)nxh);
  for (int t = threadIdx.x; t < P * nxh; t += blockDim.x) {
    const int q = (int)fdiv((unsigned)t, fdh);
    const int k = t - q * nxh;
    const double2 zk = res[k * P + q];
    const double2 zm = res[(k == 0 ? 0 : nx - k) * P + q];
    const int qa = 2 * q;
    const int ja = qa / nr;
    const int ra = qa - ja * nr;
    a.spec[((long long)b * C + ja) * g.Nh + (long long)(row0 + ra) * g.nxp + k] =
        make_double2(0.5 * (zk.x + zm.x), 0.5 * (zk.y - zm.y));
    if (qa + 1 < nseq) {
      const int jb = (qa + 1) / nr;
      const int rb = (qa + 1) - jb * nr;
      a.spec[((long long)b * C + jb) * g.Nh + (long long)(row0 + rb) * g.nxp + k] =
          make_double2(0.5 * (zk.y + zm.y), 0.5 * (zm.x - zk.x));
    }
  }

  if (PROD != PROD_IDENT) {
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) a.partials[(long long)b * a.nblocks + blockIdx.x] = s;
  }
}

// ============================================================================
// x-axis inverse pass
// ============================================================================
template <int CONS, int C, int NF = 0>
// 4 waves per SIMD (at most 128 VGPRs): measured 5 % faster at 128^3 than the unconstrained 166
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) k_xinv(XInvArgs a) {
  const int b = a.active ? a.active[blockIdx.y] : (int)blockIdx.y;
  if (CONS == CONS_CGUPD) {
    if (a.st[b].status != CG_RUNNING) return;
  }
  const Geom& g = a.g;
  const int nx = g.nx;
  const int nxh = g.nxh;
  const int rows = g.ny * g.nz;
  const int row0 = blockIdx.x * a.R;
  const int nr = min(a.R, rows - row0);
  const int nseq = C * nr;
  const int P = (nseq + 1) >> 1;
  extern __shared__ double2 smem[];
  double2* A = smem;
  double2* H = smem + (size_t)nx * P;  // loaded half rows, then the ping-pong partner
  __shared__ double red[kThreads / 64];
  const long long N = g.N;

  // the residual of this thread's voxel is loaded before the transform so that
  // its latency hides behind the FFT (one voxel per thread)
  const bool pre = (CONS == CONS_CGUPD) && (nr * nx <= (int)blockDim.x);
  double rpre[C];
  if (pre && (int)threadIdx.x < nr * nx) {
    const int r = threadIdx.x / nx;
    const int x = threadIdx.x - r * nx;
    const long long vox = (long long)(row0 + r) * nx + x;
#pragma unroll
    for (int j = 0; j < C; ++j) rpre[j] = ld_stream(a.r + ((long long)b * C + j) * N + vox);
  }

  const FastDiv fdh = make_fastdiv((unsigned)nxh);
  const FastDiv fdp = make_fastdiv((unsigned)P);
  for (int t = threadIdx.x; t < nseq * nxh; t += blockDim.x) {
    const int qr = (int)fdiv((unsigned)t, fdh);
    const int k = t - qr * nxh;
    const int j = qr / nr;
    const int r = qr - j * nr;
    H[k * nseq + qr] = a.spec[((long long)b * C + j) * g.Nh + (long long)(row0 + r) * g.nxp + k];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < P * nx; t += blockDim.x) {
    const int k = (int)fdiv((unsigned)t, fdp);
    const int q = t - k * P;
    const int qa = 2 * q;
    const bool hb = qa + 1 < nseq;
    double2 z;
    if (k < nxh) {
      double2 ha = H[k * nseq + qa];
      double2 hv = hb ? H[k * nseq + qa + 1] : make_double2(0.0, 0.0);
      if (k == 0 || 2 * k == nx) {
        ha.y = 0.0;
        hv.y = 0.0;
      }
      z = make_double2(ha.x - hv.y, ha.y + hv.x);
    } else {
      const int m = nx - k;
      const double2 ha = H[m * nseq + qa];
      const double2 hv = hb ? H[m * nseq + qa + 1] : make_double2(0.0, 0.0);
      z = make_double2(ha.x + hv.y, hv.x - ha.y);
    }
    A[k * P + q] = z;
  }
  __syncthreads();

  pass_fft<1, NF>(A, H, P, a.px, a.inplace);
  const double2* res = A;

  double alpha = 0.0;
  if (CONS == CONS_CGUPD) alpha = a.st[b].alpha;
  double acc = 0.0;
  for (int t = threadIdx.x; t < nr * nx; t += blockDim.x) {
    const int r = t / nx;
    const int x = t - r * nx;
    const long long vox = (long long)(row0 + r) * nx + x;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int qr = j * nr + r;
      const double* d = reinterpret_cast<const double*>(&res[x * P + (qr >> 1)]);
      const double u = d[qr & 1] * a.scale;
      const long long idx = ((long long)b * C + j) * N + vox;
      if (CONS == CONS_IDENT) {
        a.out[idx] = u;
      } else if (CONS == CONS_RHS) {
        a.r[idx] = -u;
        a.x[idx] = 0.0;
        acc += u * u;
      } else {
        const double rn = (pre ? rpre[j] : ld_stream(a.r + idx)) - alpha * u;
        st_stream(a.r + idx, rn);
        acc += rn * rn;
      }
    }
  }
  if (CONS != CONS_IDENT) {
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) a.partials[(long long)b * a.nblocks + blockIdx.x] = s;
  }
}

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
// y-axis pass (3D): complex FFT of the half spectrum along y, in place
// ============================================================================
// A block transforms the tw bins kx0.. of ZB consecutive z planes (contiguous in memory when
// the tile spans the whole row); sequence q = zz * tw + s, element y at A[y * nseq + q].
template <int DIR>
__global__ void __launch_bounds__(kThreads) k_mid(AxisArgs a) {
  const Geom& g = a.g;
  const int vb = blockIdx.z / g.c;
  const int comp = blockIdx.z - vb * g.c;
  const int b = a.active ? a.active[vb] : vb;
  if (a.st != nullptr && a.st[b].status != CG_RUNNING) return;
  const int kx0 = blockIdx.x * a.TX;
  const int tw = kx_tile_width(g.nxh, a.TX, blockIdx.x);
  const int ny = g.ny;
  const int z0 = blockIdx.y * a.ZB;
  const int nseq = min(a.ZB, g.nz - z0) * tw;
  extern __shared__ double2 smem[];
  double2* A = smem;
  double2* Bf = smem + (size_t)ny * nseq;
  const long long base = ((long long)b * g.c + comp) * g.Nh + (long long)z0 * ny * g.nxp + kx0;
  const FastDiv fdq = make_fastdiv((unsigned)nseq);
  const FastDiv fdt = make_fastdiv((unsigned)tw);
  for (int t = threadIdx.x; t < ny * nseq; t += blockDim.x) {
    const int y = (int)fdiv((unsigned)t, fdq);
    const int q = t - y * nseq;
    const int zz = (int)fdiv((unsigned)q, fdt);
    const int s = q - zz * tw;
    A[t] = a.spec[base + (long long)(zz * ny + y) * g.nxp + s];
  }
  __syncthreads();
  fft_lds_any<DIR>(A, Bf, nseq, a.pl, a.inplace);
  for (int t = threadIdx.x; t < ny * nseq; t += blockDim.x) {
    const int y = (int)fdiv((unsigned)t, fdq);
    const int q = t - y * nseq;
    const int zz = (int)fdiv((unsigned)q, fdt);
    const int s = q - zz * tw;
    a.spec[base + (long long)(zz * ny + y) * g.nxp + s] = A[t];
  }
}

// Consecutive blocks are dealt round-robin to the 8 XCDs, each with its own L2.  Re-index the
// grid so that the blocks one XCD receives are consecutive in (x, y, z): neighbouring kx tiles of
// a spectrum row, which share 128-byte lines when a tile is not a whole number of lines, then run
// on the same XCD close in time and meet in its L2.
__device__ __forceinline__ void xcd_blocks(unsigned* bx, unsigned* by, unsigned* bz) {
  *bx = blockIdx.x;
  *by = blockIdx.y;
  *bz = blockIdx.z;
  const unsigned tot = gridDim.x * gridDim.y * gridDim.z;
  if ((tot & 7u) == 0u) {
    const unsigned lin = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const unsigned l2 = (lin & 7u) * (tot >> 3) + (lin >> 3);
    *bx = l2 % gridDim.x;
    *by = (l2 / gridDim.x) % gridDim.y;
    *bz = l2 / (gridDim.x * gridDim.y);
  }
}

// ============================================================================
// outer-axis pass with the projection G-hat (section 3)
// ============================================================================
__device__ __forceinline__ double signed_freq(int k, int n, double scale) {
  if (2 * k < n) return k * scale;
  if (2 * k == n) return 0.0;  // Nyquist: zero wavevector component
  return (k - n) * scale;
}

// finite strain: A -> (A n) (x) n on row-major d x d tensors
template <int D>
__device__ __forceinline__ void project_finite(double2* v, const double* nv) {
  double2 an[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    an[i] = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      an[i].x += v[i * D + j].x * nv[j];
      an[i].y += v[i * D + j].y * nv[j];
    }
  }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) v[i * D + j] = make_double2(an[i].x * nv[j], an[i].y * nv[j]);
}

// small strain, Mandel packed: A -> n (x) (A n) + (A n) (x) n - (n.A.n) n (x) n
template <int D>
__device__ __forceinline__ void project_small(double2* v, const double* nv) {
  const double r2 = 1.41421356237309504880;
  const double h2 = 0.70710678118654752440;
  double2 T[D][D];
  if (D == 3) {
    T[0][0] = v[0]; T[1][1] = v[1]; T[2][2] = v[2];
    T[1][2] = T[2][1] = make_double2(h2 * v[3].x, h2 * v[3].y);
    T[0][2] = T[2][0] = make_double2(h2 * v[4].x, h2 * v[4].y);
    T[0][1] = T[1][0] = make_double2(h2 * v[5].x, h2 * v[5].y);
  } else {
    T[0][0] = v[0]; T[1][1] = v[1];
    T[0][1] = T[1][0] = make_double2(h2 * v[2].x, h2 * v[2].y);
  }
  double2 an[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    an[i] = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      an[i].x += T[i][j].x * nv[j];
      an[i].y += T[i][j].y * nv[j];
    }
  }
  double2 s = make_double2(0.0, 0.0);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    s.x += nv[i] * an[i].x;
    s.y += nv[i] * an[i].y;
  }
  auto o = [&](int i, int j) {
    return make_double2(an[i].x * nv[j] + nv[i] * an[j].x - s.x * nv[i] * nv[j],
                        an[i].y * nv[j] + nv[i] * an[j].y - s.y * nv[i] * nv[j]);
  };
  if (D == 3) {
    v[0] = o(0, 0); v[1] = o(1, 1); v[2] = o(2, 2);
    double2 t;
    t = o(1, 2); v[3] = make_double2(r2 * t.x, r2 * t.y);
    t = o(0, 2); v[4] = make_double2(r2 * t.x, r2 * t.y);
    t = o(0, 1); v[5] = make_double2(r2 * t.x, r2 * t.y);
  } else {
    v[0] = o(0, 0); v[1] = o(1, 1);
    const double2 t = o(0, 1);
    v[2] = make_double2(r2 * t.x, r2 * t.y);
  }
}

// Finite strain projects each row of F on its own ((A n)_i n_j involves only
// row i), so a block transforms the NDIM components of one row; small strain
// couples all C Mandel components.  LDS layout: element o of sequence (jj, s)
// at D[o * nseq + jj * tw + s], nseq = G * tw, one FFT call for all of them.
template <int MODE, int SMALL, int NDIM>
// uncapped: a 5-wave cap spilled 87 VGPRs in the small-strain projection (256-cell job 2 % slower)
__global__ void __launch_bounds__(kThreads) k_outer(AxisArgs a) {
  constexpr int C = SMALL ? (NDIM == 3 ? 6 : 3) : (NDIM == 3 ? 9 : 4);
  constexpr int G = SMALL ? C : NDIM;
  constexpr int NGRP = C / G;
  const Geom& g = a.g;
  unsigned bx, by, bz;
  xcd_blocks(&bx, &by, &bz);
  const int vb = bz / NGRP;
  const int grp = bz - vb * NGRP;
  const int b = a.active ? a.active[vb] : vb;
  if (a.st != nullptr && a.st[b].status != CG_RUNNING) return;
  if (MODE == OUTER_PROJECT && a.pq_st != nullptr && bx == 0 && by == 0 && grp == 0) {
    // <p, K:p> and alpha of right-hand side b, summed in a fixed order; nothing in this
    // pass reads them (the inverse x pass does)
    __shared__ double red[kThreads / 64];
    const double* pp = a.pq_partials + (long long)b * a.pq_nblocks;
    double acc = 0.0;
    for (int i = threadIdx.x; i < a.pq_nblocks; i += blockDim.x) acc += pp[i];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) cg_finalize<RED_PQ>(a.pq_st[b], s);
  }
  const int kx0 = bx * a.TX;
  const int tw = kx_tile_width(g.nxh, a.TX, (int)bx);
  const int mid = by;
  const int n = g.n_outer;
  const int nseq = G * tw;
  const int cnt = n * nseq;
  extern __shared__ double2 smem[];
  double2* D = smem;
  double2* pong = smem + (size_t)cnt;
  const long long ostride = (long long)g.n_mid * g.nxp;
  const long long base0 = (long long)mid * g.nxp + kx0;
  const long long cbase = ((long long)b * C + grp * G) * g.Nh;

  const FastDiv fdq = make_fastdiv((unsigned)nseq);
  const FastDiv fdt = make_fastdiv((unsigned)tw);
  for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
    const int o = (int)fdiv((unsigned)t, fdq);
    const int rem = t - o * nseq;
    const int jj = (int)fdiv((unsigned)rem, fdt);
    const int s = rem - jj * tw;
    D[t] = a.spec[cbase + (long long)jj * g.Nh + base0 + o * ostride + s];
  }
  __syncthreads();

  if (MODE != OUTER_INV) fft_lds_any<-1>(D, pong, nseq, a.pl, a.inplace);

  if (MODE == OUTER_PROJECT) {
    for (int t = threadIdx.x; t < n * tw; t += blockDim.x) {
      const int o = (int)fdiv((unsigned)t, fdt);
      const int s = t - o * tw;
      double xi[NDIM];
      xi[0] = signed_freq(kx0 + s, g.nx, g.ks[0]);
      if (NDIM == 3) {
        xi[1] = signed_freq(mid, g.ny, g.ks[1]);
        xi[NDIM - 1] = signed_freq(o, g.nz, g.ks[2]);
      } else {
        xi[1] = signed_freq(o, g.ny, g.ks[1]);
      }
      double nrm2 = 0.0;
#pragma unroll
      for (int i = 0; i < NDIM; ++i) nrm2 += xi[i] * xi[i];
      double2 v[G];
      const int e0 = o * nseq + s;
      if (nrm2 > 0.0) {
        const double inv = 1.0 / sqrt(nrm2);
        double nv[NDIM];
#pragma unroll
        for (int i = 0; i < NDIM; ++i) nv[i] = xi[i] * inv;
#pragma unroll
        for (int jj = 0; jj < G; ++jj) v[jj] = D[e0 + jj * tw];
        if (SMALL) {
          project_small<NDIM>(v, nv);
        } else {
          // one row of F: (sum_j A_j n_j) n
          double2 an = make_double2(0.0, 0.0);
#pragma unroll
          for (int jj = 0; jj < G; ++jj) {
            an.x += v[jj].x * nv[jj];
            an.y += v[jj].y * nv[jj];
          }
#pragma unroll
          for (int jj = 0; jj < G; ++jj) v[jj] = make_double2(an.x * nv[jj], an.y * nv[jj]);
        }
      } else {
#pragma unroll
        for (int jj = 0; jj < G; ++jj) v[jj] = make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int jj = 0; jj < G; ++jj) D[e0 + jj * tw] = v[jj];
    }
    __syncthreads();
  }

  if (MODE != OUTER_FWD) fft_lds_any<+1>(D, pong, nseq, a.pl, a.inplace);

  for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
    const int o = (int)fdiv((unsigned)t, fdq);
    const int rem = t - o * nseq;
    const int jj = (int)fdiv((unsigned)rem, fdt);
    const int s = rem - jj * tw;
    a.spec[cbase + (long long)jj * g.Nh + base0 + o * ostride + s] = D[t];
  }
}

// ============================================================================
// finite strain, 3D: the projection chain row by row
// ============================================================================
// G-hat maps a row a_i = (a_i0, a_i1, a_i2) of A-hat to s_i xi with s_i = (a_i . xi) / |xi|^2
// ((A n) (x) n with n = xi / |xi|).  xi_x depends only on kx and xi_y only on ky, so both factors
// commute with the transforms along the other axes: the forward y pass already combines
// v_i = xi_x a_i0 + xi_y a_i1 (w_i = a_i2 stays), the outer pass reads two components per row,
// forms s_i = (v_i + xi_z w_i) / |xi|^2 and writes back s_i and xi_z s_i, and the inverse y pass
// expands them to xi_x s_i, xi_y s_i, xi_z s_i.  The y and outer passes then move 15 + 12 + 15
// instead of 18 + 18 + 18 component transfers per wavevector, and the outer pass transforms
// 2 instead of 3 columns per row.  Slots: (i,0) carries v_i / s_i, (i,2) carries w_i / xi_z s_i.

// y pass of row i = blockIdx.z mod 3 over a tile of TX bins and ZB planes, one component tile in
// LDS at a time (the LDS and occupancy of a plain y pass); what the next phase combines is held in
// registers, at most kFrowHeld elements per thread (the host keeps ny * TX * ZB <= kFrowHeld * 256).
// Element y of sequence q = zz * tw + s at A[y * nseq + q]; thread t owns elements t + e * 256.
//   DIR = -1: Y a_i0 -> held = xi_x Y a_i0;  Y a_i1 -> slot (i,0) = held + xi_y Y a_i1;
//             Y a_i2 -> slot (i,2)
//   DIR = +1: slot (i,0) = u -> held = xi_y u, Y^-1 u -> slot (i,0) = xi_x Y^-1 u;
//             Y^-1 held -> slot (i,1);  slot (i,2) = w -> Y^-1 w -> slot (i,2)

template <int DIR, int NF>
// 4 waves per SIMD (at most 128 VGPRs; 157 unconstrained): measured 15 % faster at 128^3
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) k_mid_frow(AxisArgs a) {
  const Geom& g = a.g;
  unsigned bx, by, bz;
  xcd_blocks(&bx, &by, &bz);
  const int vb = bz / 3;
  const int row = bz - vb * 3;
  const int b = a.active ? a.active[vb] : vb;
  if (a.st != nullptr && a.st[b].status != CG_RUNNING) return;
  const int kx0 = bx * a.TX;
  const int tw = kx_tile_width(g.nxh, a.TX, bx);
  const int ny = g.ny;
  const int z0 = by * a.ZB;
  const int nseq = min(a.ZB, g.nz - z0) * tw;
  const int cnt = ny * nseq;
  extern __shared__ double2 smem[];
  double2* A = smem;
  double2* Bf = smem + (size_t)cnt;
  const long long cbase = ((long long)b * 9 + row * 3) * g.Nh + (long long)z0 * ny * g.nxp + kx0;
  const FastDiv fdq = make_fastdiv((unsigned)nseq);
  const FastDiv fdt = make_fastdiv((unsigned)tw);
  // global offset (within a component) and wavevector components of element t
  auto where = [&](int t, long long* off, double* xx, double* xy) {
    const int y = (int)fdiv((unsigned)t, fdq);
    const int q = t - y * nseq;
    const int zz = (int)fdiv((unsigned)q, fdt);
    const int sx = q - zz * tw;
    *off = (long long)(zz * ny + y) * g.nxp + sx;
    *xx = signed_freq(kx0 + sx, g.nx, g.ks[0]);
    *xy = signed_freq(y, ny, g.ks[1]);
  };
  auto load = [&](int slot) {
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
      long long off;
      double xx, xy;
      where(t, &off, &xx, &xy);
      A[t] = a.spec[cbase + slot * g.Nh + off];
    }
  };
  auto store = [&](int slot) {
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
      long long off;
      double xx, xy;
      where(t, &off, &xx, &xy);
      a.spec[cbase + slot * g.Nh + off] = A[t];
    }
  };
  double2 held[kFrowHeld];
  if (DIR < 0) {
    load(0);
    __syncthreads();
    pass_fft<-1, NF>(A, Bf, nseq, a.pl, a.inplace);
#pragma unroll
    for (int e = 0; e < kFrowHeld; ++e) {
      const int t = threadIdx.x + e * blockDim.x;
      if (t < cnt) {
        long long off;
        double xx, xy;
        where(t, &off, &xx, &xy);
        held[e] = make_double2(xx * A[t].x, xx * A[t].y);
      }
    }
    __syncthreads();
    load(1);
    __syncthreads();
    pass_fft<-1, NF>(A, Bf, nseq, a.pl, a.inplace);
#pragma unroll
    for (int e = 0; e < kFrowHeld; ++e) {
      const int t = threadIdx.x + e * blockDim.x;
      if (t < cnt) {
        long long off;
        double xx, xy;
        where(t, &off, &xx, &xy);
        const double2 v = A[t];
        a.spec[cbase + off] = make_double2(held[e].x + xy * v.x, held[e].y + xy * v.y);
      }
    }
    __syncthreads();
    load(2);
    __syncthreads();
    pass_fft<-1, NF>(A, Bf, nseq, a.pl, a.inplace);
    store(2);
  } else {
#pragma unroll
    for (int e = 0; e < kFrowHeld; ++e) {
      const int t = threadIdx.x + e * blockDim.x;
      if (t < cnt) {
        long long off;
        double xx, xy;
        where(t, &off, &xx, &xy);
        const double2 u = a.spec[cbase + off];
        A[t] = u;
        held[e] = make_double2(xy * u.x, xy * u.y);
      }
    }
    __syncthreads();
    pass_fft<1, NF>(A, Bf, nseq, a.pl, a.inplace);
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
      long long off;
      double xx, xy;
      where(t, &off, &xx, &xy);
      a.spec[cbase + off] = make_double2(xx * A[t].x, xx * A[t].y);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kFrowHeld; ++e) {
      const int t = threadIdx.x + e * blockDim.x;
      if (t < cnt) A[t] = held[e];
    }
    __syncthreads();
    pass_fft<1, NF>(A, Bf, nseq, a.pl, a.inplace);
    store(1);
    __syncthreads();
    load(2);
    __syncthreads();
    pass_fft<1, NF>(A, Bf, nseq, a.pl, a.inplace);
    store(2);
  }
}

// Outer (z) pass of the row-wise projection: row i = blockIdx.z mod 3 (after the XCD-aware
// re-indexing), slots (i,0) = v and (i,2) = w of TX bins at one ky.  LDS: element o of sequence
// (jj, s) at D[o * 2 tw + jj * tw + s].
template <int NF>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(5, 8))) k_outer_frow(AxisArgs a) {
  const Geom& g = a.g;
  unsigned bx, by, bz;
  xcd_blocks(&bx, &by, &bz);
  const int vb = bz / 3;
  const int row = bz - vb * 3;
  const int b = a.active ? a.active[vb] : vb;
  if (a.st != nullptr && a.st[b].status != CG_RUNNING) return;
  if (a.pq_st != nullptr && bx == 0 && by == 0 && row == 0) {
    // <p, K:p> and alpha of right-hand side b, summed in a fixed order (read by the inverse x pass)
    __shared__ double red[kThreads / 64];
    const double* pp = a.pq_partials + (long long)b * a.pq_nblocks;
    double acc = 0.0;
    for (int i = threadIdx.x; i < a.pq_nblocks; i += blockDim.x) acc += pp[i];
    const double sum = block_sum(acc, red);
    if (threadIdx.x == 0) cg_finalize<RED_PQ>(a.pq_st[b], sum);
  }
  const int kx0 = bx * a.TX;
  const int tw = kx_tile_width(g.nxh, a.TX, (int)bx);
  const int mid = by;
  const int n = g.nz;
  const int nseq = 2 * tw;
  const int cnt = n * nseq;
  extern __shared__ double2 smem[];
  double2* D = smem;
  double2* pong = smem + (size_t)cnt;
  const long long ostride = (long long)g.ny * g.nxp;
  const long long cbase = ((long long)b * 9 + row * 3) * g.Nh + (long long)mid * g.nxp + kx0;
  const FastDiv fdq = make_fastdiv((unsigned)nseq);
  const FastDiv fdt = make_fastdiv((unsigned)tw);
  for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
    const int o = (int)fdiv((unsigned)t, fdq);
    const int rem = t - o * nseq;
    const int jj = (int)fdiv((unsigned)rem, fdt);
    const int sx = rem - jj * tw;
    D[t] = a.spec[cbase + 2 * jj * g.Nh + o * ostride + sx];
  }
  __syncthreads();
  pass_fft<-1, NF>(D, pong, nseq, a.pl, a.inplace);
  const double xy = signed_freq(mid, g.ny, g.ks[1]);
  for (int t = threadIdx.x; t < n * tw; t += blockDim.x) {
    const int o = (int)fdiv((unsigned)t, fdt);
    const int sx = t - o * tw;
    const double xx = signed_freq(kx0 + sx, g.nx, g.ks[0]);
    const double xz = signed_freq(o, n, g.ks[2]);
    const double nrm2 = xx * xx + xy * xy + xz * xz;
    const int e0 = o * nseq + sx;
    double2 sv = make_double2(0.0, 0.0);
    if (nrm2 > 0.0) {
      const double inv = 1.0 / nrm2;
      const double2 v = D[e0];
      const double2 w = D[e0 + tw];
      sv = make_double2((v.x + xz * w.x) * inv, (v.y + xz * w.y) * inv);
    }
    D[e0] = sv;
    D[e0 + tw] = make_double2(xz * sv.x, xz * sv.y);
  }
  __syncthreads();
  pass_fft<1, NF>(D, pong, nseq, a.pl, a.inplace);
  for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
    const int o = (int)fdiv((unsigned)t, fdq);
    const int rem = t - o * nseq;
    const int jj = (int)fdiv((unsigned)rem, fdt);
    const int sx = rem - jj * tw;
    a.spec[cbase + 2 * jj * g.Nh + o * ostride + sx] = D[t];
  }
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
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) acc += partials[(long long)b * nblocks + i];
  const double s = block_sum(acc, red);
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
    if (MAT == MAT_NH || MAT == MAT_STVK) {
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

// J2: move the plastic history to the converged state at F (one load step ends)
template <int NDIM>
__global__ void __launch_bounds__(kThreads) k_j2_commit(const double* F, MatParams m, double* hist, Geom g) {
  constexpr int C = MatTraits<MAT_J2, NDIM>::C;
  const long long N = g.N;
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (v >= N) return;
  double e[C], h[C + 1];
  Local L;
#pragma unroll
  for (int j = 0; j < C; ++j) e[j] = F[j * N + v];
  load_local<MAT_J2, NDIM>(m, v, L);
  j2_commit<NDIM>(e, L, h);
#pragma unroll
  for (int k = 0; k <= C; ++k) hist[k * N + v] = h[k];
}

// J2: cumulative plastic strain of the state at F (history plus this step's increment)
template <int NDIM>
__global__ void __launch_bounds__(kThreads) k_j2_plastic(const double* F, MatParams m, double* out, Geom g) {
  constexpr int C = MatTraits<MAT_J2, NDIM>::C;
  const long long N = g.N;
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (v >= N) return;
  double e[C], h[C + 1];
  Local L;
#pragma unroll
  for (int j = 0; j < C; ++j) e[j] = F[j * N + v];
  load_local<MAT_J2, NDIM>(m, v, L);
  j2_commit<NDIM>(e, L, h);
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
  if (prod == PROD_CGOP && x_fixed128(a.g, a.px, a.R, a.inplace)) {
#define FH_C(M, D) hipLaunchKernelGGL((k_xfwd<PROD_CGOP, M, D, (D == 3 ? 128 : 0)>), grid, dim3(kThreads), sm, s, a);
    FH_DISPATCH_MAT(mat, FH_C)
#undef FH_C
    return hipGetLastError();
  }
#define FH_L(M, D)                                                                                       \
  switch (prod) {                                                                                        \
    case PROD_IDENT: hipLaunchKernelGGL((k_xfwd<PROD_IDENT, M, D>), grid, dim3(kThreads), sm, s, a); break;   \
    case PROD_STRESS: hipLaunchKernelGGL((k_xfwd<PROD_STRESS, M, D>), grid, dim3(kThreads), sm, s, a); break; \
    case PROD_CGOP: hipLaunchKernelGGL((k_xfwd<PROD_CGOP, M, D>), grid, dim3(kThreads), sm, s, a); break;     \
    case PROD_TRHS: hipLaunchKernelGGL((k_xfwd<PROD_TRHS, M, D>), grid, dim3(kThreads), sm, s, a); break;     \
    case PROD_CGOP_STORED:                                                                               \
      hipLaunchKernelGGL((k_xfwd<PROD_CGOP_STORED, M, D>), grid, dim3(kThreads), sm, s, a); break;       \
    case PROD_ADJ: hipLaunchKernelGGL((k_xfwd<PROD_ADJ, M, D>), grid, dim3(kThreads), sm, s, a); break;       \
    default: return hipErrorInvalidValue;                                                                \
  }
  FH_DISPATCH_MAT(mat, FH_L)
#undef FH_L
  return hipGetLastError();
}

hipError_t launch_xinv(int cons, const XInvArgs& a, int B, hipStream_t s) {
  dim3 grid(nblk_rows(a.g, a.R), B);
  const size_t sm = xinv_smem(a.g, a.R, a.inplace);
  if (cons == CONS_CGUPD && x_fixed128(a.g, a.px, a.R, a.inplace) && (a.g.c == 9 || a.g.c == 6)) {
    if (a.g.c == 9) hipLaunchKernelGGL((k_xinv<CONS_CGUPD, 9, 128>), grid, dim3(kThreads), sm, s, a);
    else hipLaunchKernelGGL((k_xinv<CONS_CGUPD, 6, 128>), grid, dim3(kThreads), sm, s, a);
    return hipGetLastError();
  }
#define FH_L(CC)                                                                                        \
  switch (cons) {                                                                                       \
    case CONS_IDENT: hipLaunchKernelGGL((k_xinv<CONS_IDENT, CC>), grid, dim3(kThreads), sm, s, a); break; \
    case CONS_RHS: hipLaunchKernelGGL((k_xinv<CONS_RHS, CC>), grid, dim3(kThreads), sm, s, a); break;     \
    case CONS_CGUPD: hipLaunchKernelGGL((k_xinv<CONS_CGUPD, CC>), grid, dim3(kThreads), sm, s, a); break; \
    default: return hipErrorInvalidValue;                                                               \
  }
  switch (a.g.c) {
    case 3: FH_L(3); break;
    case 4: FH_L(4); break;
    case 6: FH_L(6); break;
    case 9: FH_L(9); break;
    default: return hipErrorInvalidValue;
  }
#undef FH_L
  return hipGetLastError();
}

hipError_t launch_mid(int dir, const AxisArgs& a, int B, hipStream_t s) {
  const bool rows = a.proj && finite_rows(a.g);
  dim3 grid(kx_tiles(a.g.nxh, a.TX), (a.g.nz + a.ZB - 1) / a.ZB, B * (rows ? 3 : a.g.c));
  const size_t sm = mid_smem(a.g, a.TX, a.inplace, a.ZB, a.proj);
  if (rows) {
    // the benchmark's axis length gets its own kernels when every stage keeps one butterfly per thread
    const bool f128 = a.inplace && a.pl.n == 128 && fixed_one_ok(128, mid_sequences(a.g, a.TX, a.ZB, a.proj));
    if (dir < 0) {
      if (f128) hipLaunchKernelGGL((k_mid_frow<-1, 128>), grid, dim3(kThreads), sm, s, a);
      else hipLaunchKernelGGL((k_mid_frow<-1, 0>), grid, dim3(kThreads), sm, s, a);
    } else {
      if (f128) hipLaunchKernelGGL((k_mid_frow<1, 128>), grid, dim3(kThreads), sm, s, a);
      else hipLaunchKernelGGL((k_mid_frow<1, 0>), grid, dim3(kThreads), sm, s, a);
    }
  } else {
    if (dir < 0) hipLaunchKernelGGL((k_mid<-1>), grid, dim3(kThreads), sm, s, a);
    else hipLaunchKernelGGL((k_mid<1>), grid, dim3(kThreads), sm, s, a);
  }
  return hipGetLastError();
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
  if (mode == OUTER_PROJECT && finite_rows(a.g)) {
    if (a.inplace && a.pl.n == 128 && fixed_one_ok(128, G * kx_tile_max(a.g.nxh, a.TX)))
      hipLaunchKernelGGL((k_outer_frow<128>), grid, dim3(kThreads), sm, s, a);
    else
      hipLaunchKernelGGL((k_outer_frow<0>), grid, dim3(kThreads), sm, s, a);
    return hipGetLastError();
  }
#define FH_L(SM, D)                                                                                          \
  switch (mode) {                                                                                            \
    case OUTER_PROJECT: hipLaunchKernelGGL((k_outer<OUTER_PROJECT, SM, D>), grid, dim3(kThreads), sm, s, a); break; \
    case OUTER_FWD: hipLaunchKernelGGL((k_outer<OUTER_FWD, SM, D>), grid, dim3(kThreads), sm, s, a); break;         \
    case OUTER_INV: hipLaunchKernelGGL((k_outer<OUTER_INV, SM, D>), grid, dim3(kThreads), sm, s, a); break;         \
    default: return hipErrorInvalidValue;                                                                    \
  }
  if (a.g.small) {
    if (a.g.ndim == 3) { FH_L(1, 3) } else { FH_L(1, 2) }
  } else {
    if (a.g.ndim == 3) { FH_L(0, 3) } else { FH_L(0, 2) }
  }
#undef FH_L
  return hipGetLastError();
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
  if (mat == 6) hipLaunchKernelGGL((k_j2_commit<2>), vox_grid(g), dim3(kThreads), 0, s, F, m, hist, g);
  else if (mat == 7) hipLaunchKernelGGL((k_j2_commit<3>), vox_grid(g), dim3(kThreads), 0, s, F, m, hist, g);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_j2_plastic(int mat, const double* F, MatParams m, double* out, const Geom& g, hipStream_t s) {
  if (mat == 6) hipLaunchKernelGGL((k_j2_plastic<2>), vox_grid(g), dim3(kThreads), 0, s, F, m, out, g);
  else if (mat == 7) hipLaunchKernelGGL((k_j2_plastic<3>), vox_grid(g), dim3(kThreads), 0, s, F, m, out, g);
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

hipError_t launch_twiddles(double2* tw, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_twiddles, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, tw, n);
  return hipGetLastError();
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
  const int attr = (int)hipFuncAttributeMaxDynamicSharedMemorySize;
  hipError_t e = hipSuccess;
#define FH_SET(fn) \
  if (e == hipSuccess) e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn), (hipFuncAttribute)attr, (int)bytes)
#define FH_L(M, D)                                  \
  FH_SET((k_xfwd<PROD_IDENT, M, D>));               \
  FH_SET((k_xfwd<PROD_STRESS, M, D>));              \
  FH_SET((k_xfwd<PROD_CGOP, M, D>));                \
  FH_SET((k_xfwd<PROD_TRHS, M, D>));                \
  FH_SET((k_xfwd<PROD_CGOP_STORED, M, D>));         \
  FH_SET((k_xfwd<PROD_ADJ, M, D>));                \
  FH_SET((k_xfwd<PROD_CGOP, M, D, (D == 3 ? 128 : 0)>));
  FH_DISPATCH_MAT(mat, FH_L)
#undef FH_L
#define FH_X(CC) FH_SET((k_xinv<CONS_IDENT, CC>)); FH_SET((k_xinv<CONS_RHS, CC>)); FH_SET((k_xinv<CONS_CGUPD, CC>));
  switch (g.c) {
    case 3: FH_X(3); break;
    case 4: FH_X(4); break;
    case 6: FH_X(6); FH_SET((k_xinv<CONS_CGUPD, 6, 128>)); break;
    case 9: FH_X(9); FH_SET((k_xinv<CONS_CGUPD, 9, 128>)); break;
    default: break;
  }
#undef FH_X
  FH_SET((k_mid<-1>));
  FH_SET((k_mid<1>));
  FH_SET((k_mid_frow<-1, 0>));
  FH_SET((k_mid_frow<1, 0>));
  FH_SET((k_mid_frow<-1, 128>));
  FH_SET((k_mid_frow<1, 128>));
  FH_SET((k_outer_frow<0>));
  FH_SET((k_outer_frow<128>));
#define FH_O(SM, D) FH_SET((k_outer<OUTER_PROJECT, SM, D>)); FH_SET((k_outer<OUTER_FWD, SM, D>)); FH_SET((k_outer<OUTER_INV, SM, D>));
  if (g.small) {
    if (g.ndim == 3) { FH_O(1, 3) } else { FH_O(1, 2) }
  } else {
    if (g.ndim == 3) { FH_O(0, 3) } else { FH_O(0, 2) }
  }
#undef FH_O
#undef FH_SET
  return e;
}

}  // namespace fh
