// Batched complex FFT of many short sequences held in LDS (Stockham autosort,
// mixed radix 2/3/4/5/8/16 plus a direct DFT for any other prime factor, or the
// chirp-z form for lengths whose prime factors make the direct stages costly).
//
// Layout: `nseq` sequences of length n interleaved element-major, element i of
// sequence s at buf[i * nseq + s].  Consecutive threads work on consecutive
// sequences, so LDS reads and writes of a stage are contiguous across a wave
// and the tiles loaded from HBM (kx fastest) need no transpose.
//
// Each stage reads one buffer and writes the other (ping-pong); the function
// returns the buffer that holds the result.  Forward transforms use
// exp(-2 pi i jk/n), inverse exp(+2 pi i jk/n), both unnormalised.
#pragma once

#include "common.h"

namespace fh {

// x is neither NaN nor +-Inf, decided on the exponent bits: the CG kernels are compiled with
// finite-math assumptions (see build.py), under which a floating-point isfinite() or NaN
// comparison may be folded away; integer tests are not.
__device__ __forceinline__ bool finite_bits(double x) {
  return (__double_as_longlong(x) & 0x7ff0000000000000LL) != 0x7ff0000000000000LL;
}

__device__ __forceinline__ unsigned fdiv(unsigned w, FastDiv f) { return f.d > 1 ? __umulhi(w, f.m) : w; }

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// multiply by DIR * i  (DIR = -1 forward, +1 inverse)
template <int DIR>
__device__ __forceinline__ double2 mul_i(double2 a) {
  return DIR > 0 ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}
template <int DIR>
__device__ __forceinline__ double2 twiddle(const double2* tw, int idx) {
  double2 w = tw[idx];
  return DIR > 0 ? make_double2(w.x, -w.y) : w;
}

template <int DIR>
__device__ __forceinline__ void dft2(double2* v) {
  double2 a = v[0];
  v[0] = cadd(a, v[1]);
  v[1] = csub(a, v[1]);
}

template <int DIR>
__device__ __forceinline__ void dft3(double2* v) {
  const double h = 0.86602540378443864676;  // sqrt(3)/2
  double2 s = cadd(v[1], v[2]);
  double2 d = csub(v[1], v[2]);
  double2 m = make_double2(v[0].x - 0.5 * s.x, v[0].y - 0.5 * s.y);
  double2 t = mul_i<DIR>(cscale(d, h));
  v[0] = cadd(v[0], s);
  v[1] = cadd(m, t);
  v[2] = csub(m, t);
}

template <int DIR>
__device__ __forceinline__ void dft4(double2* v) {
  double2 t0 = cadd(v[0], v[2]);
  double2 t1 = csub(v[0], v[2]);
  double2 t2 = cadd(v[1], v[3]);
  double2 t3 = mul_i<DIR>(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <int DIR>
__device__ __forceinline__ void dft5(double2* v) {
  const double c1 = 0.30901699437494742410;   // cos(2 pi/5)
  const double c2 = -0.80901699437494742410;  // cos(4 pi/5)
  const double s1 = 0.95105651629515357212;   // sin(2 pi/5)
  const double s2 = 0.58778525229247312917;   // sin(4 pi/5)
  double2 b1 = cadd(v[1], v[4]), d1 = csub(v[1], v[4]);
  double2 b2 = cadd(v[2], v[3]), d2 = csub(v[2], v[3]);
  double2 a0 = v[0];
  double2 m1 = make_double2(a0.x + c1 * b1.x + c2 * b2.x, a0.y + c1 * b1.y + c2 * b2.y);
  double2 m2 = make_double2(a0.x + c2 * b1.x + c1 * b2.x, a0.y + c2 * b1.y + c1 * b2.y);
  double2 n1 = mul_i<DIR>(make_double2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y));
  double2 n2 = mul_i<DIR>(make_double2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y));
  v[0] = cadd(a0, cadd(b1, b2));
  v[1] = cadd(m1, n1);
  v[4] = csub(m1, n1);
  v[2] = cadd(m2, n2);
  v[3] = csub(m2, n2);
}

template <int DIR>
__device__ __forceinline__ void dft8(double2* v) {
  const double r = 0.70710678118654752440;
  double2 b[4], c[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    b[t] = cadd(v[t], v[t + 4]);
    c[t] = csub(v[t], v[t + 4]);
  }
  // c[t] *= w8^t, w8 = exp(DIR 2 pi i / 8)
  c[1] = make_double2(r * (c[1].x - DIR * c[1].y), r * (c[1].y + DIR * c[1].x));
  c[2] = mul_i<DIR>(c[2]);
  c[3] = make_double2(r * (-c[3].x - DIR * c[3].y), r * (-c[3].y + DIR * c[3].x));
  dft4<DIR>(b);
  dft4<DIR>(c);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    v[2 * t] = b[t];
    v[2 * t + 1] = c[t];
  }
}

// 16-point DFT as 4 x 4: DFTs over n1 of x[4 n1 + n2], twiddle by w16^(n2 k1),
// DFTs over n2; output k1 + 4 k2.  Twiddles are compile-time constants.
template <int DIR>
__device__ __forceinline__ void dft16(double2* v) {
  constexpr double C16[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                              0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                              -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
                              0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
  double2 y[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    double2 t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
    dft4<DIR>(t);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      const int m = (n2 * k1) & 15;
      const double c = C16[m];
      const double sn = DIR * C16[(m + 12) & 15];  // sin(2 pi m / 16) = cos(2 pi (m - 4) / 16)
      y[n2][k1] = (m == 0) ? t[k1] : make_double2(t[k1].x * c - t[k1].y * sn, t[k1].x * sn + t[k1].y * c);
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    double2 t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
    dft4<DIR>(t);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
  }
}

template <int R, int DIR>
__device__ __forceinline__ void dft_small(double2* v) {
  if constexpr (R == 2) dft2<DIR>(v);
  else if constexpr (R == 3) dft3<DIR>(v);
  else if constexpr (R == 4) dft4<DIR>(v);
  else if constexpr (R == 5) dft5<DIR>(v);
  else if constexpr (R == 8) dft8<DIR>(v);
  else if constexpr (R == 16) dft16<DIR>(v);
}

// One Stockham stage of radix R for all sequences.
//   Ns: product of the radices already applied; stride = n / (Ns R).
//   Butterfly j (0 <= j < n/R) of a sequence: inputs x[j + t n/R], twiddled by
//   w_n^(t k stride) with k = j mod Ns, output to (j - k) R + k + t Ns.
template <int R, int DIR>
__device__ __forceinline__ void stage_small(const double2* __restrict__ src, double2* __restrict__ dst,
                                            int nseq, int n, int Ns, const double2* __restrict__ tw) {
  const int nb = n / R;
  const int stride = n / (Ns * R);
  const int total = nb * nseq;
  for (int w = threadIdx.x; w < total; w += blockDim.x) {
    const int j = w / nseq;
    const int s = w - j * nseq;
    const int k = j % Ns;
    double2 v[R];
#pragma unroll
    for (int t = 0; t < R; ++t) v[t] = src[(j + t * nb) * nseq + s];
    if (Ns > 1) {
#pragma unroll
      for (int t = 1; t < R; ++t) v[t] = cmul(v[t], twiddle<DIR>(tw, t * k * stride));
    }
    dft_small<R, DIR>(v);
    const int base = (j - k) * R + k;
#pragma unroll
    for (int t = 0; t < R; ++t) dst[(base + t * Ns) * nseq + s] = v[t];
  }
}

// Generic radix (any factor, used for primes > 5): direct DFT reading the
// untouched source buffer; w_R^q = tw[(q mod R) * n / R].
template <int DIR>
__device__ __forceinline__ void stage_generic(const double2* __restrict__ src, double2* __restrict__ dst,
                                              int nseq, int n, int Ns, int R, const double2* __restrict__ tw) {
  const int nb = n / R;
  const int stride = n / (Ns * R);
  const int rstep = n / R;
  const int total = nb * R * nseq;  // one thread per output element
  for (int w = threadIdx.x; w < total; w += blockDim.x) {
    const int s = w % nseq;
    const int jm = w / nseq;
    const int m = jm % R;   // output index within the butterfly
    const int j = jm / R;   // butterfly
    const int k = j % Ns;
    double2 acc = make_double2(0.0, 0.0);
    int q = 0;  // (t * m) mod R
    for (int t = 0; t < R; ++t) {
      double2 x = src[(j + t * nb) * nseq + s];
      if (Ns > 1 && t > 0) x = cmul(x, twiddle<DIR>(tw, t * k * stride));
      acc = cadd(acc, cmul(x, twiddle<DIR>(tw, q * rstep)));
      q += m;
      if (q >= R) q -= R;
    }
    const int base = (j - k) * R + k;
    dst[(base + m * Ns) * nseq + s] = acc;
  }
}

// Full transform of `nseq` interleaved sequences of length L with the stages (nst, radix, tw);
// returns the buffer holding the result (a or b).  Must be called by every thread of the block.
template <int DIR>
__device__ double2* fft_stages_pp(double2* a, double2* b, int nseq, int L, int nst, const int* radix,
                                  const double2* tw) {
  double2* src = a;
  double2* dst = b;
  int Ns = 1;
  for (int st = 0; st < nst; ++st) {
    const int R = radix[st];
    switch (R) {
      case 2: stage_small<2, DIR>(src, dst, nseq, L, Ns, tw); break;
      case 3: stage_small<3, DIR>(src, dst, nseq, L, Ns, tw); break;
      case 4: stage_small<4, DIR>(src, dst, nseq, L, Ns, tw); break;
      case 5: stage_small<5, DIR>(src, dst, nseq, L, Ns, tw); break;
      case 8: stage_small<8, DIR>(src, dst, nseq, L, Ns, tw); break;
      case 16: stage_small<16, DIR>(src, dst, nseq, L, Ns, tw); break;
      default: stage_generic<DIR>(src, dst, nseq, L, Ns, R, tw); break;
    }
    __syncthreads();
    double2* t = src;
    src = dst;
    dst = t;
    Ns *= R;
  }
  return src;
}

template <int DIR>
__device__ double2* fft_lds(double2* a, double2* b, int nseq, const AxisPlan& pl) {
  return fft_stages_pp<DIR>(a, b, nseq, pl.n, pl.nstages, pl.radix, pl.tw);
}

// ---- in-place variant: register-staged stages, one LDS buffer ---------------
// Every stage first loads all butterfly inputs of the thread into registers and computes its
// butterflies, synchronises, then writes the outputs to their Stockham positions in the same
// buffer.  Usable when all radices are 2/3/4/5/8 and no thread owns more than
// kInplaceElems elements in a stage (checked by the host: inplace_ok()).

// (Run-time length and stage position; the divisions by nseq and Ns are magic multiplies.)
template <int R, int DIR>
__device__ __forceinline__ void stage_inplace(double2* __restrict__ buf, int nseq, FastDiv fdq, int n, int Ns,
                                              const double2* __restrict__ tw) {
  constexpr int MB = kInplaceElems / R;
  const int nb = n / R;
  const int stride = n / (Ns * R);
  const int total = nb * nseq;
  const FastDiv fdn = make_fastdiv((unsigned)Ns);
  double2 v[MB][R];
  int ov[MB], sv[MB];
  // butterflies in registers before the barrier, which only guards the in-place write
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int w = threadIdx.x + i * blockDim.x;
    ov[i] = 0;
    sv[i] = 0;
    if (w < total) {
      const int j = (int)fdiv((unsigned)w, fdq);
      const int s = w - j * nseq;
      const int k = j - (int)fdiv((unsigned)j, fdn) * Ns;
#pragma unroll
      for (int t = 0; t < R; ++t) v[i][t] = buf[(j + t * nb) * nseq + s];
      if (Ns > 1) {
#pragma unroll
        for (int t = 1; t < R; ++t) v[i][t] = cmul(v[i][t], twiddle<DIR>(tw, t * k * stride));
      }
      dft_small<R, DIR>(v[i]);
      ov[i] = (j - k) * R + k;
      sv[i] = s;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int w = threadIdx.x + i * blockDim.x;
    if (w < total) {
#pragma unroll
      for (int t = 0; t < R; ++t) buf[(ov[i] + t * Ns) * nseq + sv[i]] = v[i][t];
    }
  }
  __syncthreads();
}

// Same stage with the length, radix and stage position known at compile time
// (no integer division except one magic multiply per element).
// MB: butterflies per thread (the host guarantees nseq * N / R <= MB * blockDim); MB = 1 keeps
// one butterfly's values and twiddles live, which the kernels specialised for one length use.
template <int R, int NS, int N, int DIR, int MB = kInplaceElems / R>
__device__ __forceinline__ void stage_fixed(double2* __restrict__ buf, int nseq, FastDiv fd,
                                            const double2* __restrict__ tw) {
  constexpr int NB = N / R;
  constexpr int STRIDE = N / (NS * R);
  const int total = NB * nseq;
  double2 v[MB][R];
  int ov[MB], sv[MB];
  // each thread's butterflies are computed in registers before the barrier (their twiddle loads
  // and arithmetic overlap the other waves' LDS reads); the barrier only guards the in-place write
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int w = threadIdx.x + i * blockDim.x;
    ov[i] = 0;
    sv[i] = 0;
    if (w < total) {
      const int j = (int)fdiv((unsigned)w, fd);
      const int s = w - j * nseq;
      const int k = j % NS;
#pragma unroll
      for (int t = 0; t < R; ++t) v[i][t] = buf[(j + t * NB) * nseq + s];
      if (NS > 1) {
#pragma unroll
        for (int t = 1; t < R; ++t) v[i][t] = cmul(v[i][t], twiddle<DIR>(tw, t * k * STRIDE));
      }
      dft_small<R, DIR>(v[i]);
      ov[i] = (j - k) * R + k;
      sv[i] = s;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int w = threadIdx.x + i * blockDim.x;
    if (w < total) {
#pragma unroll
      for (int t = 0; t < R; ++t) buf[(ov[i] + t * NS) * nseq + sv[i]] = v[i][t];
    }
  }
  __syncthreads();
}

template <int N, int DIR, int ST, int NS, bool ONE = false>
__device__ __forceinline__ void fixed_stages(double2* buf, int nseq, FastDiv fd, const double2* tw) {
  if constexpr (ST < fixed_nstages(N)) {
    constexpr int R = fixed_radix(N, ST);
    stage_fixed<R, NS, N, DIR, ONE ? 1 : kInplaceElems / R>(buf, nseq, fd, tw);
    fixed_stages<N, DIR, ST + 1, NS * R, ONE>(buf, nseq, fd, tw);
  }
}

// In-place transform of length N (a compiled schedule) with one butterfly per thread per stage:
// only that length's code and registers.  The caller guarantees fixed_one_ok(N, nseq).
template <int N, int DIR>
__device__ __forceinline__ void fft_fixed_one(double2* buf, int nseq, const double2* tw) {
  fixed_stages<N, DIR, 0, 1, true>(buf, nseq, make_fastdiv((unsigned)nseq), tw);
}
__host__ __device__ inline bool fixed_one_ok(int n, int nseq) {
  if (fixed_nstages(n) == 0) return false;
  for (int st = 0; st < fixed_nstages(n); ++st)
    if ((long long)nseq * (n / fixed_radix(n, st)) > kThreads) return false;
  return true;
}

template <int DIR>
__device__ void fft_stages_ip(double2* buf, int nseq, int L, int nst, const int* radix, const double2* tw) {
  const FastDiv fd = make_fastdiv((unsigned)nseq);
  switch (L) {
    case 256: fixed_stages<256, DIR, 0, 1>(buf, nseq, fd, tw); return;
    case 192: fixed_stages<192, DIR, 0, 1>(buf, nseq, fd, tw); return;
    case 160: fixed_stages<160, DIR, 0, 1>(buf, nseq, fd, tw); return;
    case 128: fixed_stages<128, DIR, 0, 1>(buf, nseq, fd, tw); return;
    case 96: fixed_stages<96, DIR, 0, 1>(buf, nseq, fd, tw); return;
    case 80: fixed_stages<80, DIR, 0, 1>(buf, nseq, fd, tw); return;
    case 64: fixed_stages<64, DIR, 0, 1>(buf, nseq, fd, tw); return;
    case 48: fixed_stages<48, DIR, 0, 1>(buf, nseq, fd, tw); return;
    case 32: fixed_stages<32, DIR, 0, 1>(buf, nseq, fd, tw); return;
    case 16: fixed_stages<16, DIR, 0, 1>(buf, nseq, fd, tw); return;
    case 8: fixed_stages<8, DIR, 0, 1>(buf, nseq, fd, tw); return;
    default: break;
  }
  int Ns = 1;
  for (int st = 0; st < nst; ++st) {
    const int R = radix[st];
    switch (R) {
      case 2: stage_inplace<2, DIR>(buf, nseq, fd, L, Ns, tw); break;
      case 3: stage_inplace<3, DIR>(buf, nseq, fd, L, Ns, tw); break;
      case 4: stage_inplace<4, DIR>(buf, nseq, fd, L, Ns, tw); break;
      case 5: stage_inplace<5, DIR>(buf, nseq, fd, L, Ns, tw); break;
      case 16: stage_inplace<16, DIR>(buf, nseq, fd, L, Ns, tw); break;
      default: stage_inplace<8, DIR>(buf, nseq, fd, L, Ns, tw); break;
    }
    Ns *= R;
  }
}

template <int DIR>
__device__ void fft_lds_inplace(double2* buf, int nseq, const AxisPlan& pl) {
  fft_stages_ip<DIR>(buf, nseq, pl.n, pl.nstages, pl.radix, pl.tw);
}

// Transform in place when the plan allows it (inplace != 0), else ping-pong
// through `pong` and copy back.  Result always in `buf`.
template <int DIR>
__device__ __forceinline__ void fft_lds_any(double2* buf, double2* pong, int nseq, const AxisPlan& pl, int inplace) {
  if (inplace) {
    fft_lds_inplace<DIR>(buf, nseq, pl);
  } else {
    double2* res = fft_lds<DIR>(buf, pong, nseq, pl);
    if (res != buf) {
      const int cnt = pl.n * nseq;
      for (int t = threadIdx.x; t < cnt; t += blockDim.x) buf[t] = res[t];
      __syncthreads();
    }
  }
}

// ---- chirp-z (Bluestein) transform for axes with large prime factors ----------
// With c_j = exp(DIR i pi j^2 / n) (pl.chirp for DIR = -1, its conjugate for DIR = +1),
// j k = (j^2 + k^2 - (k - j)^2) / 2 turns the length-n DFT into
//   X_k = c_k sum_j (x_j c_j) conj(c_(k-j)),
// a linear convolution with the even sequence conj(c_j), |j| < n.  Zero-padded to m >= 2n - 1
// it is a cyclic convolution of length m: a forward length-m FFT, a product with the filter
// f = FFT_m(h) / m (pl.filt; h is even, so the DIR = +1 filter is conj(f)), an inverse length-m
// FFT.  The LDS buffer holds m rows per sequence; the result is left in rows 0..n-1.  The
// length-m stages run in place when the host allowed it (inplace), else through `pong`.
// one length-m transform of the chirp-z convolution, result in buf
template <int D>
__device__ __forceinline__ void chirp_conv_fft(double2* buf, double2* pong, int nseq, const AxisPlan& pl, int inplace) {
  if (inplace) {
    fft_stages_ip<D>(buf, nseq, pl.m, pl.nstages, pl.radix, pl.tw);
  } else {
    double2* res = fft_stages_pp<D>(buf, pong, nseq, pl.m, pl.nstages, pl.radix, pl.tw);
    if (res != buf) {
      for (int t = threadIdx.x; t < pl.m * nseq; t += blockDim.x) buf[t] = res[t];
      __syncthreads();
    }
  }
}

template <int DIR>
__device__ void fft_chirp(double2* buf, double2* pong, int nseq, const AxisPlan& pl, int inplace) {
  const int n = pl.n;
  const int m = pl.m;
  const FastDiv fd = make_fastdiv((unsigned)nseq);
  for (int t = threadIdx.x; t < m * nseq; t += blockDim.x) {
    const int j = (int)fdiv((unsigned)t, fd);
    double2 v = make_double2(0.0, 0.0);
    if (j < n) v = cmul(buf[t], twiddle<DIR>(pl.chirp, j));
    buf[t] = v;
  }
  __syncthreads();
  chirp_conv_fft<-1>(buf, pong, nseq, pl, inplace);
  for (int t = threadIdx.x; t < m * nseq; t += blockDim.x) {
    const int j = (int)fdiv((unsigned)t, fd);
    buf[t] = cmul(buf[t], twiddle<DIR>(pl.filt, j));
  }
  __syncthreads();
  chirp_conv_fft<1>(buf, pong, nseq, pl, inplace);
  for (int t = threadIdx.x; t < n * nseq; t += blockDim.x) {
    const int j = (int)fdiv((unsigned)t, fd);
    buf[t] = cmul(buf[t], twiddle<DIR>(pl.chirp, j));
  }
  __syncthreads();
}

// ---- deterministic block reduction (wave64 shuffles, fixed order) ------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Sum over the block; the result is valid in thread 0.  `sh` needs blockDim/64 doubles.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) s += sh[w];
  }
  __syncthreads();
  return s;
}

}  // namespace fh
