// The pass kernels of the Fourier-Galerkin Newton-CG solve for gfx950 (FP64), as templates:
// kernels.hip instantiates them with the direct FFT stages (and the kernels specialised for
// 128-point axes), kernels_fixed.hip for 96-, 64-, 48- and 32-point axes, kernels_chirp.hip with
// the chirp-z transform.
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
#pragma once

#include "common.h"
#include "fft_lds.h"
#include "kernels.h"
#include "materials.h"

namespace fh {

// matcode = 2 * material + (ndim - 2); 8, 9: Neo-Hookean, J2 under plane stress (2D)
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
    case 8: MACRO(MAT_NH_PS, 2); break; \
    case 9: MACRO(MAT_J2_PS, 2); break; \
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
  if constexpr (j2_mat(MAT)) {
    constexpr int C = MatTraits<MAT, NDIM>::C;
    L.sy = row[2];
    L.H = row[3];
#pragma unroll
    for (int k = 0; k <= C; ++k) L.hist[k] = m.hist[k * m.hN + v];
  }
}

__device__ __forceinline__ int ceil_div(int a, int b) { return (a + b - 1) / b; }

// FFT variant of a pass kernel (template parameter NF):
//   0              any length with direct stages, with the register staging or the ping-pong
//                  buffer the host chose;
//   kChirp         the chirp-z transform (plans with m > 0; kernels_chirp.hip);
//   L, 0 < L < kStaged   length L only, one butterfly per thread per stage (the launchers check
//                  fixed_one_ok): only that length's code and a butterfly's registers;
//   kStaged + L    length L only (a compiled schedule), register staging of up to kInplaceElems
//                  elements per thread (the host chose in-place stages; kernels_fixed.hip).
// The generic kernels hold every compiled schedule, and their registers follow the longest one;
// the length-specific kernels hold one.  The buffers hold lds_len(pl) rows per sequence.
constexpr int kChirp = -1;
constexpr int kStaged = 1 << 12;
template <int D, int NF>
__device__ __forceinline__ void pass_fft(double2* A, double2* Bf, int nseq, const AxisPlan& pl, int inplace) {
  if constexpr (NF > kStaged) fixed_stages<NF - kStaged, D, 0, 1>(A, nseq, make_fastdiv((unsigned)nseq), pl.tw);
  else if constexpr (NF > 0) fft_fixed_one<NF, D>(A, nseq, pl.tw);
  else if constexpr (NF == kChirp) fft_chirp<D>(A, Bf, nseq, pl, inplace);
  else fft_lds_any<D>(A, Bf, nseq, pl, inplace);
}

// Streaming access for the CG vectors and the linearisation point: each is touched once
// per CG iteration, so keeping them out of the caches leaves room for the half spectrum
// that the FFT passes hand to each other.
__device__ __forceinline__ double ld_stream(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_stream(double* p, double v) { __builtin_nontemporal_store(v, p); }

// Sum of x[tid], x[tid + kThreads], x[tid + 2 kThreads], ... (i < n) in that order, with up to S of
// the thread's loads in flight together; bitwise the strided loop's sum.
template <int S, int BD>
__device__ __forceinline__ double strided_sum(const double* __restrict__ x, int n) {
  double acc = 0.0;
  for (int base = 0; base < n; base += S * BD) {
    double v[S];
#pragma unroll
    for (int e = 0; e < S; ++e) {
      const int i = base + (int)threadIdx.x + e * BD;
      v[e] = i < n ? x[i] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < S; ++e) acc += v[e];
  }
  return acc;
}

// Gather n complex entries into LDS: dst[i] = v for (v, i) = src(t), t < n.  Each thread issues up
// to S global loads before its first LDS write, so that S of its loads are in flight together (in
// a plain load-then-write loop each load waits for the previous one).  Used where it measured
// faster: the inverse x pass and the plain y pass; the row-wise y and outer passes, which run at
// their register caps, were slower with it.
template <int S, typename Src>
__device__ __forceinline__ void gather_staged(double2* dst, int n, Src src) {
  for (int base = 0; base < n; base += S * kThreads) {
    double2 v[S];
    int di[S];
#pragma unroll
    for (int e = 0; e < S; ++e) {
      const int t = base + (int)threadIdx.x + e * kThreads;
      di[e] = -1;
      if (t < n) v[e] = src(t, &di[e]);
    }
#pragma unroll
    for (int e = 0; e < S; ++e)
      if (di[e] >= 0) dst[di[e]] = v[e];
  }
}

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
  double* E = reinterpret_cast<double*>(smem + (size_t)(a.inplace ? 1 : 2) * g.lx * P);
  double2* Bf = smem + (size_t)g.lx * P;  // ping-pong partner (unused in place)
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
      if (!j2_mat(MAT)) {
        Local L;
        load_local<MAT, NDIM>(mat, vox, L);  // brings the phase id and table line into cache
        (void)L;
      }
      // r, p and x are distinct buffers: every load is issued before the first store (without the
      // restrict qualifiers the compiler must order each component's loads after the previous
      // component's stores, one memory round trip per component)
      const double* __restrict__ rin = a.in + (long long)b * C * N + vox;
      double* __restrict__ pio = a.p + (long long)b * C * N + vox;
      double* __restrict__ xio = a.x + (long long)b * C * N + vox;
      double rv[C], pv[C], xv[C];
#pragma unroll
      for (int j = 0; j < C; ++j) rv[j] = ld_stream(rin + j * N);
      if (!first) {
#pragma unroll
        for (int j = 0; j < C; ++j) {
          pv[j] = ld_stream(pio + j * N);
          xv[j] = ld_stream(xio + j * N);
        }
      }
#pragma unroll
      for (int j = 0; j < C; ++j) {
        double pj = rv[j];
        if (!first) {
          st_stream(xio + j * N, xv[j] + alpha_prev * pv[j]);
          pj = rv[j] + beta * pv[j];
        }
        st_stream(pio + j * N, pj);
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
        if (finite_mat(MAT)) {
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
  double2* H = smem + (size_t)g.lx * P;  // loaded half rows, then the ping-pong partner
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
  gather_staged<8>(H, nseq * nxh, [&](int t, int* di) {
    const int qr = (int)fdiv((unsigned)t, fdh);
    const int k = t - qr * nxh;
    const int j = qr / nr;
    const int r = qr - j * nr;
    *di = k * nseq + qr;
    return a.spec[((long long)b * C + j) * g.Nh + (long long)(row0 + r) * g.nxp + k];
  });
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
    // the residual's components are all loaded before the first store (restrict: no component's
    // store has to wait for the next one's load)
    double* __restrict__ rio = a.r + (long long)b * C * N + vox;
    double rv[C];
    if (CONS == CONS_CGUPD) {
#pragma unroll
      for (int j = 0; j < C; ++j) rv[j] = pre ? rpre[j] : ld_stream(rio + j * N);
    }
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
        const double rn = rv[j] - alpha * u;
        st_stream(rio + j * N, rn);
        acc += rn * rn;
      }
    }
  }
  if (CONS != CONS_IDENT) {
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) a.partials[(long long)b * a.nblocks + blockIdx.x] = s;
  }
}

// ============================================================================
// y-axis pass (3D): complex FFT of the half spectrum along y, in place
// ============================================================================
// A block transforms the tw bins kx0.. of ZB consecutive z planes (contiguous in memory when
// the tile spans the whole row); sequence q = zz * tw + s, element y at A[y * nseq + q].
template <int DIR, int NF = 0>
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
  double2* Bf = smem + (size_t)g.lm * nseq;
  const long long base = ((long long)b * g.c + comp) * g.Nh + (long long)z0 * ny * g.nxp + kx0;
  const FastDiv fdq = make_fastdiv((unsigned)nseq);
  const FastDiv fdt = make_fastdiv((unsigned)tw);
  gather_staged<8>(A, ny * nseq, [&](int t, int* di) {
    const int y = (int)fdiv((unsigned)t, fdq);
    const int q = t - y * nseq;
    const int zz = (int)fdiv((unsigned)q, fdt);
    const int s = q - zz * tw;
    *di = t;
    return a.spec[base + (long long)(zz * ny + y) * g.nxp + s];
  });
  __syncthreads();
  pass_fft<DIR, NF>(A, Bf, nseq, a.pl, a.inplace);
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
template <int MODE, int SMALL, int NDIM, int NF = 0>
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
    const double s = block_sum(strided_sum<8, kThreads>(a.pq_partials + (long long)b * a.pq_nblocks, a.pq_nblocks), red);
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
  double2* pong = smem + (size_t)g.lo * nseq;
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

  if (MODE != OUTER_INV) pass_fft<-1, NF>(D, pong, nseq, a.pl, a.inplace);

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

  if (MODE != OUTER_FWD) pass_fft<+1, NF>(D, pong, nseq, a.pl, a.inplace);

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
  double2* Bf = smem + (size_t)g.lm * nseq;
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
    const double sum = block_sum(strided_sum<8, kThreads>(a.pq_partials + (long long)b * a.pq_nblocks, a.pq_nblocks), red);
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
  double2* pong = smem + (size_t)g.lo * nseq;
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
// launches of the pass kernels with FFT variant NF (grid and LDS bytes from the caller)
// ============================================================================
template <int NF>
hipError_t dispatch_xfwd(int prod, int mat, const XFwdArgs& a, dim3 grid, size_t sm, hipStream_t s) {
#define FH_L(M, D)                                                                                             \
  switch (prod) {                                                                                              \
    case PROD_IDENT: hipLaunchKernelGGL((k_xfwd<PROD_IDENT, M, D, NF>), grid, dim3(kThreads), sm, s, a); break;   \
    case PROD_STRESS: hipLaunchKernelGGL((k_xfwd<PROD_STRESS, M, D, NF>), grid, dim3(kThreads), sm, s, a); break; \
    case PROD_CGOP: hipLaunchKernelGGL((k_xfwd<PROD_CGOP, M, D, NF>), grid, dim3(kThreads), sm, s, a); break;     \
    case PROD_TRHS: hipLaunchKernelGGL((k_xfwd<PROD_TRHS, M, D, NF>), grid, dim3(kThreads), sm, s, a); break;     \
    case PROD_CGOP_STORED:                                                                                     \
      hipLaunchKernelGGL((k_xfwd<PROD_CGOP_STORED, M, D, NF>), grid, dim3(kThreads), sm, s, a); break;         \
    case PROD_ADJ: hipLaunchKernelGGL((k_xfwd<PROD_ADJ, M, D, NF>), grid, dim3(kThreads), sm, s, a); break;       \
    default: return hipErrorInvalidValue;                                                                      \
  }
  FH_DISPATCH_MAT(mat, FH_L)
#undef FH_L
  return hipGetLastError();
}

template <int NF>
hipError_t dispatch_xinv(int cons, const XInvArgs& a, dim3 grid, size_t sm, hipStream_t s) {
#define FH_L(CC)                                                                                              \
  switch (cons) {                                                                                             \
    case CONS_IDENT: hipLaunchKernelGGL((k_xinv<CONS_IDENT, CC, NF>), grid, dim3(kThreads), sm, s, a); break; \
    case CONS_RHS: hipLaunchKernelGGL((k_xinv<CONS_RHS, CC, NF>), grid, dim3(kThreads), sm, s, a); break;     \
    case CONS_CGUPD: hipLaunchKernelGGL((k_xinv<CONS_CGUPD, CC, NF>), grid, dim3(kThreads), sm, s, a); break; \
    default: return hipErrorInvalidValue;                                                                     \
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

// rows: the row-wise finite-strain y pass of the projection chain
template <int NF>
hipError_t dispatch_mid(int dir, bool rows, const AxisArgs& a, dim3 grid, size_t sm, hipStream_t s) {
  if (rows) {
    if (dir < 0) hipLaunchKernelGGL((k_mid_frow<-1, NF>), grid, dim3(kThreads), sm, s, a);
    else hipLaunchKernelGGL((k_mid_frow<1, NF>), grid, dim3(kThreads), sm, s, a);
  } else {
    if (dir < 0) hipLaunchKernelGGL((k_mid<-1, NF>), grid, dim3(kThreads), sm, s, a);
    else hipLaunchKernelGGL((k_mid<1, NF>), grid, dim3(kThreads), sm, s, a);
  }
  return hipGetLastError();
}

// rows: the row-wise finite-strain projection (3D)
template <int NF>
hipError_t dispatch_outer(int mode, bool rows, const AxisArgs& a, dim3 grid, size_t sm, hipStream_t s) {
  if (rows) {
    hipLaunchKernelGGL((k_outer_frow<NF>), grid, dim3(kThreads), sm, s, a);
    return hipGetLastError();
  }
#define FH_L(SM, D)                                                                                                  \
  switch (mode) {                                                                                                    \
    case OUTER_PROJECT: hipLaunchKernelGGL((k_outer<OUTER_PROJECT, SM, D, NF>), grid, dim3(kThreads), sm, s, a); break; \
    case OUTER_FWD: hipLaunchKernelGGL((k_outer<OUTER_FWD, SM, D, NF>), grid, dim3(kThreads), sm, s, a); break;         \
    case OUTER_INV: hipLaunchKernelGGL((k_outer<OUTER_INV, SM, D, NF>), grid, dim3(kThreads), sm, s, a); break;         \
    default: return hipErrorInvalidValue;                                                                            \
  }
  if (a.g.small) {
    if (a.g.ndim == 3) { FH_L(1, 3) } else { FH_L(1, 2) }
  } else {
    if (a.g.ndim == 3) { FH_L(0, 3) } else { FH_L(0, 2) }
  }
#undef FH_L
  return hipGetLastError();
}

// Dynamic-LDS limit of every pass kernel of variant NF that a grid of this kind launches.
template <int NF>
hipError_t pass_smem_limits(const Geom& g, int mat, size_t bytes) {
  const int attr = (int)hipFuncAttributeMaxDynamicSharedMemorySize;
  hipError_t e = hipSuccess;
#define FH_SET(fn) \
  if (e == hipSuccess) e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn), (hipFuncAttribute)attr, (int)bytes)
#define FH_L(M, D)                          \
  FH_SET((k_xfwd<PROD_IDENT, M, D, NF>));   \
  FH_SET((k_xfwd<PROD_STRESS, M, D, NF>));  \
  FH_SET((k_xfwd<PROD_CGOP, M, D, NF>));    \
  FH_SET((k_xfwd<PROD_TRHS, M, D, NF>));    \
  FH_SET((k_xfwd<PROD_CGOP_STORED, M, D, NF>)); \
  FH_SET((k_xfwd<PROD_ADJ, M, D, NF>));
  FH_DISPATCH_MAT(mat, FH_L)
#undef FH_L
#define FH_X(CC) FH_SET((k_xinv<CONS_IDENT, CC, NF>)); FH_SET((k_xinv<CONS_RHS, CC, NF>)); FH_SET((k_xinv<CONS_CGUPD, CC, NF>));
  switch (g.c) {
    case 3: FH_X(3); break;
    case 4: FH_X(4); break;
    case 6: FH_X(6); break;
    case 9: FH_X(9); break;
    default: break;
  }
#undef FH_X
  FH_SET((k_mid<-1, NF>));
  FH_SET((k_mid<1, NF>));
  FH_SET((k_mid_frow<-1, NF>));
  FH_SET((k_mid_frow<1, NF>));
  FH_SET((k_outer_frow<NF>));
#define FH_O(SM, D) FH_SET((k_outer<OUTER_PROJECT, SM, D, NF>)); FH_SET((k_outer<OUTER_FWD, SM, D, NF>)); FH_SET((k_outer<OUTER_INV, SM, D, NF>));
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
