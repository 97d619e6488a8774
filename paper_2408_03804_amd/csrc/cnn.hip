// Voxel-CNN stiffness surrogate on the gfx950 matrix cores.
//
// Every layer is a bf16 x bf16 -> fp32 GEMM on gfx950 MFMA 16x16x32 tiles:
//   conv forward      pre[m][co]   = col[m][k] . W[co][k]            (col = periodic stride-2 im2col)
//   conv weight grad  dW[co][k]    = sum_m dpre[m][co] col[m][k]      (split over m, fixed-order sum)
//   conv input grad   dcol[m][k]   = sum_co dpre[m][co] W[co][k], then a gather back to the voxels
// col is never stored for blocks 2-4: their GEMM tile loaders gather it from the previous
// block's activations (implicit GEMM); block 1 (one input channel, the u8 phase map) expands it.
//   dense layers      the same three products with m = sample
// around small element-wise kernels (bias + gelu, pooling, loss, Adam).  All sums that
// cross blocks go through partial buffers reduced in a fixed order, so a training step is
// bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fft_homog.h"
#include "fft_homog_cnn.h"

namespace cnn {

typedef uint16_t bf16;
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kT = 256;
constexpr int BM = 64, BN = 64, BK = 32, LDT = BK + 8;  // GEMM tile; LDS row pitch in bf16
constexpr int kMaxSplits = 1024;
constexpr int kColRows = 256;  // rows per block of the bias-gradient column sums

// fp32 -> bf16, round to nearest even (NaN stays NaN)
__host__ __device__ inline bf16 to_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (bf16)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16)(u >> 16);
}
__device__ inline float from_bf16(bf16 b) { return __uint_as_float((uint32_t)b << 16); }

__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// ---------------------------------------------------------------------------
// GEMM: C[z][m][n] = sum_{k in split z} A(m,k) B(n,k)
// ---------------------------------------------------------------------------
// Implicit im2col operand of a conv block: element (row, k) of col, row = ((b m + oz) m + oy) m + ox
// over the m^3 outputs of each sample, k = t Ci + ci with tap t = 9 tz + 3 ty + tx < 27, is
// src[b, (2 oz + tz - 1) mod n, (2 oy + ty - 1) mod n, (2 ox + tx - 1) mod n, ci]  (n = 2 m), and
// zero for k >= 27 Ci.  Ci % 8 == 0, so 8 consecutive k share a tap (one 16-byte load).
struct ConvOperand {
  const bf16* src;  // [b][z][y][x][Ci] activations of the previous block
  int n, m, Ci;
};

struct GemmArgs {
  int M, N, K, kchunk;
  const bf16* A;
  long long sam, sak;
  const bf16* B;
  long long sbn, sbk;
  float* C;
  ConvOperand cv;  // the implicit operand (A for CONV = 1, B for CONV = 2)
};

// periodic input coordinate of output coordinate o and tap component t (0..2)
__device__ inline int tap_coord(int o, int t, int n) {
  int i = 2 * o + t - 1;
  if (i < 0) i += n;
  if (i >= n) i -= n;
  return i;
}

// The 8 col entries (row, k..k+7) of the implicit operand (zero past 27 Ci); (b, oz, oy, ox) is row.
__device__ inline uint4 conv_gather(const ConvOperand& c, long long b, int oz, int oy, int ox, int k) {
  const int tap = k / c.Ci;
  if (tap >= 27) return make_uint4(0u, 0u, 0u, 0u);
  const int ci = k - tap * c.Ci;
  const int tz = tap / 9, ty = (tap / 3) % 3, tx = tap % 3;
  const long long vox = ((b * c.n + tap_coord(oz, tz, c.n)) * c.n + tap_coord(oy, ty, c.n)) * c.n + tap_coord(ox, tx, c.n);
  return *reinterpret_cast<const uint4*>(c.src + vox * c.Ci + ci);
}

// output row -> (sample, oz, oy, ox); rows are below 2^31 (max_batch m^3 outputs per block)
__device__ inline void conv_row(const ConvOperand& c, int row, long long* b, int* oz, int* oy, int* ox) {
  const unsigned m = (unsigned)c.m;
  unsigned r = (unsigned)row;
  unsigned q = r / m;
  *ox = (int)(r - q * m);
  r = q;
  q = r / m;
  *oy = (int)(r - q * m);
  r = q;
  q = r / m;
  *oz = (int)(r - q * m);
  *b = q;
}

// Stage a 64 x 32 (rows x k) operand tile into LDS, zero outside [0,nrows) x [k0,kend).
// KC: the operand is contiguous along k (else along rows).
template <bool KC>
__device__ inline void load_tile(bf16 (*T)[LDT], const bf16* P, long long s_row, long long s_k, int row0, int nrows,
                                 int k0, int kend) {
  const int t = threadIdx.x;
  bf16 v[8];
  if (KC) {
    const int r = t >> 2;
    const int kk = (t & 3) * 8;
    const int row = row0 + r;
    const int k = k0 + kk;
    const bf16* src = P + (long long)row * s_row + (long long)k * s_k;
    if (row < nrows && k + 8 <= kend && ((reinterpret_cast<uintptr_t>(src) & 15u) == 0)) {
      const uint4 q = *reinterpret_cast<const uint4*>(src);
      memcpy(v, &q, 16);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = (row < nrows && k + i < kend) ? P[(long long)row * s_row + (long long)(k + i) * s_k] : 0;
    }
    uint4 q;
    memcpy(&q, v, 16);
    *reinterpret_cast<uint4*>(&T[r][kk]) = q;
  } else {
    const int kk = t >> 3;
    const int rr = (t & 7) * 8;
    const int k = k0 + kk;
    const int row = row0 + rr;
    const bf16* src = P + (long long)row * s_row + (long long)k * s_k;
    if (k < kend && row + 8 <= nrows && ((reinterpret_cast<uintptr_t>(src) & 15u) == 0)) {
      const uint4 q = *reinterpret_cast<const uint4*>(src);
      memcpy(v, &q, 16);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = (k < kend && row + i < nrows) ? P[(long long)(row + i) * s_row + (long long)k * s_k] : 0;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) T[rr + i][kk] = v[i];
  }
}

// 256 threads = 4 waves in a 2 x 2 arrangement, each wave a 32 x 32 block of 2 x 2 MFMA tiles.
// gfx950 MFMA 16x16x32 bf16 (v_mfma_f32_16x16x32_bf16, one instruction per 32-deep k step of a tile):
// lane l holds rows/cols (l mod 16) at k = 8 (l / 16) + 0..7 (one 16-byte LDS read per operand);
// the accumulator holds column (l mod 16), rows 4 (l / 16) + 0..3.
// CONV = 1: A is the implicit im2col operand g.cv (rows = outputs, contiguous along k);
// CONV = 2: B is (B rows = col k, GEMM k = outputs).  The other operand is read from memory.
template <bool AK, bool BK_, int CONV = 0>
__global__ void __launch_bounds__(kT) k_gemm(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) bf16 As[BM][LDT];
  __shared__ __attribute__((aligned(16))) bf16 Bs[BN][LDT];
  const int m0 = blockIdx.x * BM;
  const int n0 = blockIdx.y * BN;
  const int kbeg = blockIdx.z * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int wm = (w >> 1) * 32;
  const int wn = (w & 1) * 32;
  const int lr = lane & 15;
  const int lk = 4 * (lane >> 4);   // accumulator rows
  const int lk8 = 8 * (lane >> 4);  // operand k offset
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  // CONV = 1: this thread's A row of every k tile (row r = t / 4, k offset 8 (t mod 4))
  long long cb = 0;
  int coz = 0, coy = 0, cox = 0;
  const int crow = m0 + (threadIdx.x >> 2);
  if (CONV == 1 && crow < g.M) conv_row(g.cv, crow, &cb, &coz, &coy, &cox);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    if constexpr (CONV == 1) {
      const int kk = (threadIdx.x & 3) * 8;
      uint4 q = make_uint4(0u, 0u, 0u, 0u);
      if (crow < g.M && k0 + kk < kend) q = conv_gather(g.cv, cb, coz, coy, cox, k0 + kk);
      *reinterpret_cast<uint4*>(&As[threadIdx.x >> 2][kk]) = q;
    } else {
      load_tile<AK>(As, g.A, g.sam, g.sak, m0, g.M, k0, kend);
    }
    if constexpr (CONV == 2) {
      // GEMM k = output row k0 + t / 8, B rows (col k) n0 + 8 (t mod 8) .. + 7, stored transposed
      const int kk = threadIdx.x >> 3;
      const int rr = (threadIdx.x & 7) * 8;
      uint4 q = make_uint4(0u, 0u, 0u, 0u);
      if (k0 + kk < kend && n0 + rr < g.N) {
        long long b;
        int oz, oy, ox;
        conv_row(g.cv, k0 + kk, &b, &oz, &oy, &ox);
        q = conv_gather(g.cv, b, oz, oy, ox, n0 + rr);
      }
      bf16 v[8];
      memcpy(v, &q, 16);
#pragma unroll
      for (int i = 0; i < 8; ++i) Bs[rr + i][kk] = v[i];
    } else {
      load_tile<BK_>(Bs, g.B, g.sbn, g.sbk, n0, g.N, k0, kend);
    }
    __syncthreads();
    static_assert(BK == 32, "one 16x16x32 MFMA per k tile");
    {
      v8bf a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = *reinterpret_cast<const v8bf*>(&As[wm + 16 * i + lr][lk8]);
        b[i] = *reinterpret_cast<const v8bf*>(&Bs[wn + 16 * i + lr][lk8]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  float* C = g.C + (long long)blockIdx.z * g.M * g.N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = m0 + wm + 16 * i + lk + e;
        const int col = n0 + wn + 16 * j + lr;
        if (row < g.M && col < g.N) C[(long long)row * g.N + col] = acc[i][j][e];
      }
}

hipError_t gemm(int M, int N, int K, const bf16* A, long long sam, long long sak, const bf16* B, long long sbn,
                long long sbk, float* C, int splits, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  GemmArgs g;
  g.M = M;
  g.N = N;
  g.K = K;
  splits = std::max(1, std::min(splits, kMaxSplits));
  int chunk = (K + splits - 1) / splits;
  chunk = (chunk + BK - 1) / BK * BK;
  splits = (K + chunk - 1) / chunk;
  g.kchunk = chunk;
  g.A = A;
  g.sam = sam;
  g.sak = sak;
  g.B = B;
  g.sbn = sbn;
  g.sbk = sbk;
  g.C = C;
  dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN, splits);
  const bool ak = sak == 1, bk = sbk == 1;
  if (ak && bk) hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(kT), 0, s, g);
  else if (ak) hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(kT), 0, s, g);
  else if (bk) hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(kT), 0, s, g);
  else hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(kT), 0, s, g);
  return hipGetLastError();
}

// The two conv products with the implicit im2col operand cv (Kp = 32-padded 27 Ci):
//   forward      pre[M][N] = col[M][Kp] . W[N][Kp]                    (CONV = 1)
//   weight grad  dW[z][co][Kp] = sum_{m in split z} dpre[m][co] col[m][Kp]   (CONV = 2; A = dpre, [M][co])
hipError_t gemm_conv_forward(int M, int N, int Kp, const ConvOperand& cv, const bf16* W, float* C, hipStream_t s) {
  if (M <= 0 || N <= 0 || Kp <= 0) return hipSuccess;
  GemmArgs g{};
  g.M = M;
  g.N = N;
  g.K = Kp;
  g.kchunk = Kp;
  g.B = W;
  g.sbn = Kp;
  g.sbk = 1;
  g.C = C;
  g.cv = cv;
  hipLaunchKernelGGL((k_gemm<true, true, 1>), dim3((M + BM - 1) / BM, (N + BN - 1) / BN, 1), dim3(kT), 0, s, g);
  return hipGetLastError();
}
hipError_t gemm_conv_wgrad(int Co, int Kp, int M, const bf16* dpre, const ConvOperand& cv, float* C, int splits,
                           hipStream_t s) {
  if (M <= 0 || Co <= 0 || Kp <= 0) return hipSuccess;
  GemmArgs g{};
  g.M = Co;
  g.N = Kp;
  g.K = M;
  splits = std::max(1, std::min(splits, kMaxSplits));
  int chunk = (M + splits - 1) / splits;
  chunk = (chunk + BK - 1) / BK * BK;
  splits = (M + chunk - 1) / chunk;
  g.kchunk = chunk;
  g.A = dpre;
  g.sam = 1;
  g.sak = Co;
  g.C = C;
  g.cv = cv;
  hipLaunchKernelGGL((k_gemm<false, false, 2>), dim3((Co + BM - 1) / BM, (Kp + BN - 1) / BN, splits), dim3(kT), 0, s, g);
  return hipGetLastError();
}

// number of k-splits that gives each split about `rows` reduction steps
int splits_for(int K, int rows) { return std::max(1, std::min(kMaxSplits, (K + rows - 1) / rows)); }

// ---------------------------------------------------------------------------
// element-wise and gather kernels
// ---------------------------------------------------------------------------
inline unsigned blocks(long long n) { return (unsigned)std::min<long long>((n + kT - 1) / kT, 1 << 20); }

// im2col of a periodic stride-2 3x3x3 window: col[(b,o)][t * Ci + ci] = a[b, (2 o + t - 1) mod n, ci]
// (zero for k >= 27 Ci).  One thread per (output row, tap) copies the tap's Ci channels, 16 bytes
// at a time when Ci is a multiple of 8 (rows of src and col are then 16-byte aligned).
__global__ void k_im2col(const bf16* src, int B, int n, int Ci, int Kp, bf16* col) {
  const int m = n / 2;
  const long long rows = (long long)B * m * m * m;
  const long long tot = rows * 27;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const long long row = e / 27;
    const int t = (int)(e - row * 27);
    const int tz = t / 9, ty = (t / 3) % 3, tx = t % 3;
    long long r = row;
    const int ox = (int)(r % m);
    r /= m;
    const int oy = (int)(r % m);
    r /= m;
    const int oz = (int)(r % m);
    const long long b = r / m;
    const int iz = (2 * oz + tz - 1 + n) % n, iy = (2 * oy + ty - 1 + n) % n, ix = (2 * ox + tx - 1 + n) % n;
    const bf16* sp = src + (((b * n + iz) * n + iy) * n + ix) * Ci;
    bf16* dp = col + row * Kp + (long long)t * Ci;
    if ((Ci & 7) == 0) {
      for (int c = 0; c < Ci; c += 8) *reinterpret_cast<uint4*>(dp + c) = *reinterpret_cast<const uint4*>(sp + c);
    } else {
      for (int c = 0; c < Ci; ++c) dp[c] = sp[c];
    }
    if (t == 26)
      for (int k = 27 * Ci; k < Kp; ++k) col[row * Kp + k] = 0;
  }
}

// First block: the input is the u8 phase map (one channel); one thread per output row writes
// its Kp entries (27 taps, then zeros).  Ids above 1 raise *bad.
__global__ void k_im2col_phase(const uint8_t* phase, int B, int n, int Kp, bf16* col, int* bad) {
  const int m = n / 2;
  const long long rows = (long long)B * m * m * m;
  for (long long row = blockIdx.x * (long long)blockDim.x + threadIdx.x; row < rows;
       row += (long long)gridDim.x * blockDim.x) {
    long long r = row;
    const int ox = (int)(r % m);
    r /= m;
    const int oy = (int)(r % m);
    r /= m;
    const int oz = (int)(r % m);
    const long long b = r / m;
    const uint8_t* pb = phase + b * n * n * n;
    bf16* dp = col + row * Kp;
    // the 27 taps as bits, then 16-byte stores of the bf16 row (Kp is a multiple of 32)
    uint32_t bits = 0;
    int t = 0;
    for (int tz = 0; tz < 3; ++tz) {
      const int iz = (2 * oz + tz - 1 + n) % n;
      for (int ty = 0; ty < 3; ++ty) {
        const int iy = (2 * oy + ty - 1 + n) % n;
        for (int tx = 0; tx < 3; ++tx, ++t) {
          const int ix = (2 * ox + tx - 1 + n) % n;
          const uint8_t p = pb[((long long)iz * n + iy) * n + ix];
          if (p > 1) *bad = 1;
          bits |= (p ? 1u : 0u) << t;
        }
      }
    }
    for (int k0 = 0; k0 < Kp; k0 += 8) {
      uint32_t wv[4];
      for (int q = 0; q < 4; ++q) {
        const int k = k0 + 2 * q;
        const uint32_t lo = (k < 27 && ((bits >> k) & 1u)) ? 0x3f80u : 0u;
        const uint32_t hi = (k + 1 < 27 && ((bits >> (k + 1)) & 1u)) ? 0x3f80u : 0u;
        wv[q] = lo | (hi << 16);
      }
      *reinterpret_cast<uint4*>(dp + k0) = make_uint4(wv[0], wv[1], wv[2], wv[3]);
    }
  }
}

// pre[m][n] += bias[n]; act[m][n] = bf16(gelu(pre))   (act may be null).  A block covers
// kT / N rows (N <= kT) or one row in chunks (N > kT); no per-element division.
__global__ void k_bias_gelu(float* pre, const float* bias, long long M, int N, bf16* act) {
  const int rpb = N <= kT ? kT / N : 1;
  const int c0 = N <= kT ? (int)threadIdx.x % N : (int)threadIdx.x;
  const int rr = N <= kT ? (int)threadIdx.x / N : 0;
  if (rr >= rpb) return;
  for (long long r = (long long)blockIdx.x * rpb + rr; r < M; r += (long long)gridDim.x * rpb)
    for (int c = c0; c < N; c += (N <= kT ? N : kT)) {
      const long long e = r * N + c;
      const float x = pre[e] + bias[c];
      pre[e] = x;
      if (act) act[e] = to_bf16(gelu(x));
    }
}

// x5[b][:] = [bf16(mean over V voxels of gelu(pre4[b])), bf16(feat[b]), 0 ...]
__global__ void k_pool_concat(const float* pre4, int B, int V, int C, const float* feat, int nf, int Kp, bf16* x5) {
  const long long tot = (long long)B * Kp;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(e / Kp);
    const int k = (int)(e - (long long)b * Kp);
    float v = 0.f;
    if (k < C) {
      for (int i = 0; i < V; ++i) v += gelu(pre4[((long long)b * V + i) * C + k]);
      v /= (float)V;
    } else if (k < C + nf) {
      v = feat[(long long)b * nf + (k - C)];
    }
    x5[e] = to_bf16(v);
  }
}

// y[b][o] = (C[b][o] + bias[o]) * scale[b]
// y = offset + scale (C + bias) per sample (offset, scale nullable)
__global__ void k_output(const float* C, const float* bias, const float* scale, const float* offset, int B, int O,
                         float* y) {
  const long long tot = (long long)B * O;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(e / O);
    const int o = (int)(e - (long long)b * O);
    float v = C[e] + bias[o];
    if (scale) v *= scale[b];
    if (offset) v += offset[e];
    y[e] = v;
  }
}

// loss = mean (y - t)^2 over B*O (one block, fixed order); dy = 2 (y - t) / (B O)
__global__ void k_loss(const float* y, const float* t, long long n, float* loss, float* dy32, bf16* dyb) {
  __shared__ double red[1024];
  double acc = 0.0;
  const float inv = 2.0f / (float)n;
  for (long long e = threadIdx.x; e < n; e += blockDim.x) {
    const float d = y[e] - t[e];
    acc += (double)d * d;
    dy32[e] = d * inv;
    dyb[e] = to_bf16(d * inv);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(red[0] / (double)n);
}

// column sums of X [M][C] (fp32): partial[blk][c] over the block's row range, fixed order
__global__ void k_colsum_partial(const float* X, long long M, int C, long long rows_per_blk, float* partial) {
  __shared__ float red[kT];
  const long long r0 = blockIdx.x * rows_per_blk;
  const long long r1 = std::min(M, r0 + rows_per_blk);
  for (int c0 = 0; c0 < C; c0 += kT) {
    // thread layout: column c0 + (tid mod cw), row group tid / cw
    const int cw = std::min(kT, C - c0);
    const int groups = kT / cw;
    const int tid = threadIdx.x;
    const int c = c0 + tid % cw;
    const int grp = tid / cw;
    float acc = 0.f;
    if (grp < groups)
      for (long long r = r0 + grp; r < r1; r += groups) acc += X[r * C + c];
    red[tid] = (grp < groups) ? acc : 0.f;
    __syncthreads();
    if (tid < cw) {
      float s = 0.f;
      for (int gi = 0; gi < groups; ++gi) s += red[gi * cw + tid];
      partial[(long long)blockIdx.x * C + c0 + tid] = s;
    }
    __syncthreads();
  }
}

// dst[c] = sum over blocks of partial[blk][c]: one block per column, thread-strided partial sums
// combined by a fixed tree
__global__ void k_colsum_final(const float* partial, int nb, int C, float* dst) {
  __shared__ float red[kT];
  const int c = blockIdx.x;
  float acc = 0.f;
  for (int i = threadIdx.x; i < nb; i += kT) acc += partial[(long long)i * C + c];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) dst[c] = red[0];
}

// out[n] = sum_s P[s][n] in order (n < N); with `rows`>1, P is [S][rows][N] and out [rows][ldo]
__global__ void k_sum_splits(const float* P, int S, long long rows, int N, int Nvalid, float* out, int ldo, int accumulate) {
  const long long tot = rows * Nvalid;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const long long r = e / Nvalid;
    const int n = (int)(e - r * Nvalid);
    float s = 0.f;
    for (int z = 0; z < S; ++z) s += P[((long long)z * rows + r) * N + n];
    float* dst = out + r * ldo + n;
    *dst = accumulate ? *dst + s : s;
  }
}

// dpre = dA * gelu'(pre), fp32 and bf16 copies; dA read as src[r*lds + c]
__global__ void k_gelu_back(const float* src, int lds, const float* pre, long long M, int C, float scale, float* d32,
                            bf16* db) {
  const long long tot = M * C;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const long long r = e / C;
    const int c = (int)(e - r * C);
    const float v = src[r * lds + c] * scale * gelu_grad(pre[e]);
    d32[e] = v;
    db[e] = to_bf16(v);
  }
}

// pooled features back to the voxels of the last conv block: da4[b][v][c] = dx5[b][c] / V
__global__ void k_unpool_back(const float* dx5, int ldx, const float* pre4, int B, int V, int C, float* d32, bf16* db) {
  const long long tot = (long long)B * V * C;
  const float inv = 1.0f / (float)V;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const long long b = e / ((long long)V * C);
    const float v = dx5[b * ldx + c] * inv * gelu_grad(pre4[e]);
    d32[e] = v;
    db[e] = to_bf16(v);
  }
}

// Gather of dcol back to the input voxels of a stride-2 periodic layer, times gelu'(pre_in):
// voxel i of an axis of length n is tap t of output o when 2 o + t - 1 = i (mod n), i.e. t = 1
// (o = i/2) for even i and t = 0 (o = (i+1)/2 mod n/2) or t = 2 (o = (i-1)/2) for odd i.
// One thread per (input voxel, group of 4 channels; 1 channel when Ci is not a multiple of 4):
// consecutive threads read consecutive channels of the same dcol rows.
__global__ void k_col2im_gelu(const float* dcol, int B, int n, int Ci, int Kp, const float* pre_in, float* d32,
                              bf16* db) {
  const int m = n / 2;
  const int w = (Ci & 3) == 0 ? 4 : 1;
  const int groups = Ci / w;
  const long long tot = (long long)B * n * n * n * groups;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const long long vox = e / groups;
    const int ci = (int)(e - vox * groups) * w;
    long long r = vox;
    const int ix = (int)(r % n);
    r /= n;
    const int iy = (int)(r % n);
    r /= n;
    const int iz = (int)(r % n);
    const long long b = r / n;
    int tz[2], oz[2], ty[2], oy[2], tx[2], ox[2];
    int nzc, nyc, nxc;
    auto taps = [&](int i, int* t, int* o, int& cnt) {
      if ((i & 1) == 0) {
        t[0] = 1;
        o[0] = i / 2;
        cnt = 1;
      } else {
        t[0] = 0;
        o[0] = ((i + 1) / 2) % m;
        t[1] = 2;
        o[1] = (i - 1) / 2;
        cnt = 2;
      }
    };
    taps(iz, tz, oz, nzc);
    taps(iy, ty, oy, nyc);
    taps(ix, tx, ox, nxc);
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int a = 0; a < nzc; ++a)
      for (int c = 0; c < nyc; ++c)
        for (int d = 0; d < nxc; ++d) {
          const long long orow = ((b * m + oz[a]) * m + oy[c]) * m + ox[d];
          const int t = (tz[a] * 3 + ty[c]) * 3 + tx[d];
          const float* src = dcol + orow * Kp + (long long)t * Ci + ci;
          if (w == 4) {
            const float4 v = *reinterpret_cast<const float4*>(src);
            s.x += v.x;
            s.y += v.y;
            s.z += v.z;
            s.w += v.w;
          } else {
            s.x += src[0];
          }
        }
    const long long base = vox * Ci + ci;
    if (w == 4) {
      const float4 pr = *reinterpret_cast<const float4*>(pre_in + base);
      const float o0 = s.x * gelu_grad(pr.x), o1 = s.y * gelu_grad(pr.y), o2 = s.z * gelu_grad(pr.z),
                  o3 = s.w * gelu_grad(pr.w);
      *reinterpret_cast<float4*>(d32 + base) = make_float4(o0, o1, o2, o3);
      const uint2 packed = make_uint2((uint32_t)to_bf16(o0) | ((uint32_t)to_bf16(o1) << 16),
                                      (uint32_t)to_bf16(o2) | ((uint32_t)to_bf16(o3) << 16));
      *reinterpret_cast<uint2*>(db + base) = packed;
    } else {
      const float v = s.x * gelu_grad(pre_in[base]);
      d32[base] = v;
      db[base] = to_bf16(v);
    }
  }
}

// W [rows][K] fp32 (flat parameter block) -> Wb [rows][Kp] bf16 with zero padding
__global__ void k_pack(const float* W, int rows, int K, int Kp, bf16* Wb) {
  const long long tot = (long long)rows * Kp;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const long long r = e / Kp;
    const int k = (int)(e - r * Kp);
    Wb[e] = k < K ? to_bf16(W[r * K + k]) : (bf16)0;
  }
}

__global__ void k_adam(float* p, float* m, float* v, const float* g, long long n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

// positive definiteness of a symmetric 6x6 by Cholesky (double)
__device__ bool spd6(const double (*A)[6]) {
  double L[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = A[i][j];
      for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
      if (i == j) {
        if (!(s > 0.0)) return false;
        L[i][i] = sqrt(s);
      } else {
        L[i][j] = s / L[j][j];
      }
    }
  return true;
}

__device__ void iso6(double lam, double mu, double (*C)[6]) {
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) C[i][j] = 0.0;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) C[i][j] = lam;
    C[i][i] = lam + 2.0 * mu;
    C[i + 3][i + 3] = mu;
  }
}

// one block per sample: volume fraction, Voigt / Reuss bounds, Cholesky tests, feature range
__global__ void k_check(const uint8_t* phase, long long Nv, const float* lm, const float* feat, int nf, float* C21,
                        const float* C2, float tol, float lo, float hi, float max_spread, int* ok, float* spread_out) {
  __shared__ double red[kT];
  const int b = blockIdx.x;
  double cnt = 0.0;
  for (long long v = threadIdx.x; v < Nv; v += blockDim.x) cnt += phase[(long long)b * Nv + v] ? 1.0 : 0.0;
  red[threadIdx.x] = cnt;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double f1 = red[0] / (double)Nv, f0 = 1.0 - f1;
  const double l0 = lm[4 * b + 0], m0 = lm[4 * b + 1], l1 = lm[4 * b + 2], m1 = lm[4 * b + 3];
  // Voigt: arithmetic means of lam, mu; Reuss (isotropic phases): harmonic means of bulk and shear moduli
  const double lv = f0 * l0 + f1 * l1, mv = f0 * m0 + f1 * m1;
  const double k0 = l0 + 2.0 * m0 / 3.0, k1 = l1 + 2.0 * m1 / 3.0;
  const double kr = 1.0 / (f0 / k0 + f1 / k1), mr = 1.0 / (f0 / m0 + f1 / m1);
  const double lr = kr - 2.0 * mr / 3.0;
  double Cv[6][6], Cr[6][6], Cp[6][6], A[6][6];
  iso6(lv, mv, Cv);
  iso6(lr, mr, Cr);
  // with a second ensemble member: the prediction becomes the mean of the two, and their
  // spread (2-norm of the difference of the 21 components over that of the mean) is tested
  double d2 = 0.0, n2 = 0.0;
  int k = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) {
      double c = C21[(long long)b * 21 + k];
      if (C2) {
        const double c2 = C2[(long long)b * 21 + k];
        d2 += (c - c2) * (c - c2);
        c = 0.5 * (c + c2);
        n2 += c * c;
        C21[(long long)b * 21 + k] = (float)c;
      }
      Cp[i][j] = Cp[j][i] = c;
      ++k;
    }
  bool good = spd6(Cp);
  if (C2) good = good && (sqrt(d2) <= (double)max_spread * sqrt(n2));
  if (spread_out) spread_out[b] = C2 ? (float)(sqrt(d2) / fmax(sqrt(n2), 1e-300)) : 0.0f;
  // bounds with a slack of tol |C_Voigt|_F in every direction (prediction errors are measured
  // in that norm; a per-direction relative slack would reject small errors in the soft
  // shear directions)
  double fro = 0.0;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) fro += Cv[i][j] * Cv[i][j];
  const double slack = (double)tol * sqrt(fro);
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) A[i][j] = Cv[i][j] - Cp[i][j] + (i == j ? slack : 0.0);
  good = good && spd6(A);
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) A[i][j] = Cp[i][j] - Cr[i][j] + (i == j ? slack : 0.0);
  good = good && spd6(A);
  if (nf > 0) {
    const float x = feat[(long long)b * nf];
    good = good && (x >= lo) && (x <= hi);
  }
  ok[b] = good ? 1 : 0;
}

}  // namespace cnn

using namespace cnn;

struct fft_homog_cnn {
  fft_homog_cnn_desc d;
  hipStream_t s;
  char* ws;
  size_t P;
  // parameter blocks: offsets into the flat vector
  size_t offW[7], offB[7];
  int Kc[7], Kp[7], rows[7];  // per layer 1..6: K of the GEMM, padded K, output width
  int edge[5];                // cell edge at the input of conv block l (edge[0] = n), edge[4] = after block 4
  float *p, *m, *v, *g;
  bf16* Wb[7];
  bf16* col[5];
  float* pre[5];
  bf16* act[5];
  bf16 *x5, *h, *dyb, *dAb, *dBb;
  float *pre5, *y, *dy32, *dA, *dB, *dcol, *scratch, *colpart, *lossd;
  int* flag;
  size_t scratch_floats, colpart_floats;
  int step;
  float *h_loss;
  int* h_flag;
  hipEvent_t e0, e1;
  double fwd_ms, train_ms;
};

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int round32(int k) { return (k + 31) / 32 * 32; }

int validate(const fft_homog_cnn_desc* d) {
  if (!d) return FFT_HOMOG_EINVAL;
  if (d->n < 16 || d->n > 128 || d->n % 16 != 0) return FFT_HOMOG_EINVAL;
  if (d->channels[0] != 1) return FFT_HOMOG_EINVAL;
  for (int l = 1; l < 5; ++l)
    if (d->channels[l] < 1 || d->channels[l] > 1024) return FFT_HOMOG_EINVAL;
  if (d->hidden < 1 || d->hidden > 4096 || d->n_feat < 0 || d->n_feat > 32 || d->n_out < 1 || d->n_out > 4096)
    return FFT_HOMOG_EINVAL;
  if (d->max_batch < 1) return FFT_HOMOG_EINVAL;
  // GEMM rows (outputs of block 1 over the batch) are 32-bit
  const long long m1 = d->n / 2;
  if ((long long)d->max_batch * m1 * m1 * m1 > 0x7fffffffLL) return FFT_HOMOG_EINVAL;
  return FFT_HOMOG_OK;
}

struct Plan {
  size_t P, offW[7], offB[7];
  int Kc[7], Kp[7], rows[7], edge[5];
  size_t o_p, o_m, o_v, o_g, o_Wb[7], o_col[5], o_pre[5], o_act[5], o_x5, o_pre5, o_h, o_y, o_dy32, o_dyb, o_dA,
      o_dAb, o_dB, o_dBb, o_dcol, o_scratch, o_colpart, o_loss, o_flag, total;
  size_t scratch_floats, colpart_floats;
};

void plan(const fft_homog_cnn_desc* d, Plan* L) {
  const int* ch = d->channels;
  const long long Bm = d->max_batch;
  size_t k = 0;
  for (int l = 1; l <= 4; ++l) {
    L->rows[l] = ch[l];
    L->Kc[l] = 27 * ch[l - 1];
    L->Kp[l] = round32(L->Kc[l]);
    L->offW[l] = k;
    k += (size_t)ch[l] * L->Kc[l];
    L->offB[l] = k;
    k += ch[l];
  }
  L->rows[5] = d->hidden;
  L->Kc[5] = ch[4] + d->n_feat;
  L->Kp[5] = round32(L->Kc[5]);
  L->offW[5] = k;
  k += (size_t)d->hidden * L->Kc[5];
  L->offB[5] = k;
  k += d->hidden;
  L->rows[6] = d->n_out;
  L->Kc[6] = d->hidden;
  L->Kp[6] = round32(d->hidden);
  L->offW[6] = k;
  k += (size_t)d->n_out * d->hidden;
  L->offB[6] = k;
  k += d->n_out;
  L->P = k;
  L->edge[0] = d->n;
  for (int l = 1; l <= 4; ++l) L->edge[l] = L->edge[l - 1] / 2;

  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L->o_p = take(L->P * 4);
  L->o_m = take(L->P * 4);
  L->o_v = take(L->P * 4);
  L->o_g = take(L->P * 4);
  for (int l = 1; l <= 6; ++l) L->o_Wb[l] = take((size_t)L->rows[l] * L->Kp[l] * 2);
  size_t maxact = 0, maxcol = 0;
  for (int l = 1; l <= 4; ++l) {
    const long long Ml = Bm * (long long)L->edge[l] * L->edge[l] * L->edge[l];
    // block 1 always expands its operand; blocks 2-4 only when their input channels are not a
    // multiple of 8 (else the GEMMs gather it, implicit_conv)
    const bool expand = l == 1 || ch[l - 1] % 8 != 0;
    L->o_col[l] = take(expand ? (size_t)Ml * L->Kp[l] * 2 : 0);
    L->o_pre[l] = take((size_t)Ml * ch[l] * 4);
    L->o_act[l] = take((size_t)Ml * ch[l] * 2);
    maxact = std::max(maxact, (size_t)Ml * ch[l]);
    if (l >= 2) maxcol = std::max(maxcol, (size_t)Ml * L->Kp[l]);
  }
  maxact = std::max(maxact, (size_t)Bm * std::max(d->hidden, L->Kp[5]));
  L->o_x5 = take((size_t)Bm * L->Kp[5] * 2);
  L->o_pre5 = take((size_t)Bm * d->hidden * 4);
  L->o_h = take((size_t)Bm * d->hidden * 2);
  L->o_y = take((size_t)Bm * d->n_out * 4);
  L->o_dy32 = take((size_t)Bm * d->n_out * 4);
  L->o_dyb = take((size_t)Bm * d->n_out * 2);
  L->o_dA = take(maxact * 4);
  L->o_dAb = take(maxact * 2);
  L->o_dB = take(maxact * 4);
  L->o_dBb = take(maxact * 2);
  L->o_dcol = take(std::max<size_t>(maxcol, 1) * 4);
  // split-K partials of the weight gradients and the dense-layer products
  size_t sc = 0;
  for (int l = 1; l <= 4; ++l) {
    const long long Ml = Bm * (long long)L->edge[l] * L->edge[l] * L->edge[l];
    sc = std::max(sc, (size_t)splits_for((int)Ml, 4096) * L->rows[l] * L->Kp[l]);
  }
  sc = std::max(sc, (size_t)splits_for((int)Bm, 4096) * d->hidden * L->Kp[5]);
  sc = std::max(sc, (size_t)splits_for((int)Bm, 4096) * d->n_out * d->hidden);
  sc = std::max(sc, (size_t)Bm * std::max(L->Kp[5], std::max(d->hidden, d->n_out)));
  L->scratch_floats = sc;
  L->o_scratch = take(sc * 4);
  const long long M1 = Bm * (long long)L->edge[1] * L->edge[1] * L->edge[1];
  L->colpart_floats = (size_t)((M1 + kColRows - 1) / kColRows + 1) * std::max(std::max(1024, d->n_out), d->hidden);
  L->o_colpart = take(L->colpart_floats * 4);
  L->o_loss = take(64);
  L->o_flag = take(64);
  L->total = off;
}

#define CK(expr)                                        \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return FFT_HOMOG_EDEVICE;     \
  } while (0)

// bias gradient: column sums of X [M][C] into dst[C], two fixed-order stages
hipError_t colsum(fft_homog_cnn_t* h, const float* X, long long M, int C, float* dst) {
  const long long rpb = kColRows;
  const long long nb = (M + rpb - 1) / rpb;
  hipLaunchKernelGGL(k_colsum_partial, dim3((unsigned)nb), dim3(kT), 0, h->s, X, M, C, rpb, h->colpart);
  hipLaunchKernelGGL(k_colsum_final, dim3(C), dim3(kT), 0, h->s, h->colpart, (int)nb, C, dst);
  return hipGetLastError();
}

int check_batch(fft_homog_cnn_t* h, int B) { return (B >= 1 && B <= h->d.max_batch) ? FFT_HOMOG_OK : FFT_HOMOG_EINVAL; }

// conv block l > 1 gathers its im2col operand inside the GEMM when its input channels allow
// 16-byte loads of 8 channels
bool implicit_conv(const fft_homog_cnn_t* h, int l) { return l > 1 && h->d.channels[l - 1] % 8 == 0; }
ConvOperand conv_operand(const fft_homog_cnn_t* h, int l) {
  return ConvOperand{h->act[l - 1], h->edge[l - 1], h->edge[l], h->d.channels[l - 1]};
}

// forward pass of B samples into h->y (before output scaling is applied by the caller path)
int forward(fft_homog_cnn_t* h, const uint8_t* phase, const float* feat, int B) {
  const int* ch = h->d.channels;
  CK(hipMemsetAsync(h->flag, 0, sizeof(int), h->s));
  for (int l = 1; l <= 4; ++l) {
    const int n = h->edge[l - 1];
    const long long Ml = (long long)B * h->edge[l] * h->edge[l] * h->edge[l];
    if (l == 1 || !implicit_conv(h, l)) {
      if (l == 1)
        hipLaunchKernelGGL(k_im2col_phase, dim3(blocks(Ml)), dim3(kT), 0, h->s, phase, B, n, h->Kp[1], h->col[1], h->flag);
      else
        hipLaunchKernelGGL(k_im2col, dim3(blocks(Ml * 27)), dim3(kT), 0, h->s, h->act[l - 1], B, n, ch[l - 1], h->Kp[l],
                           h->col[l]);
      CK(hipGetLastError());
      CK(gemm((int)Ml, ch[l], h->Kp[l], h->col[l], h->Kp[l], 1, h->Wb[l], h->Kp[l], 1, h->pre[l], 1, h->s));
    } else {
      CK(gemm_conv_forward((int)Ml, ch[l], h->Kp[l], conv_operand(h, l), h->Wb[l], h->pre[l], h->s));
    }
    hipLaunchKernelGGL(k_bias_gelu, dim3(blocks(Ml * ch[l])), dim3(kT), 0, h->s, h->pre[l], h->p + h->offB[l], Ml, ch[l],
                       h->act[l]);
    CK(hipGetLastError());
  }
  const int V = h->edge[4] * h->edge[4] * h->edge[4];
  hipLaunchKernelGGL(k_pool_concat, dim3(blocks((long long)B * h->Kp[5])), dim3(kT), 0, h->s, h->pre[4], B, V, ch[4], feat,
                     h->d.n_feat, h->Kp[5], h->x5);
  CK(hipGetLastError());
  CK(gemm(B, h->d.hidden, h->Kp[5], h->x5, h->Kp[5], 1, h->Wb[5], h->Kp[5], 1, h->pre5, 1, h->s));
  hipLaunchKernelGGL(k_bias_gelu, dim3(blocks((long long)B * h->d.hidden)), dim3(kT), 0, h->s, h->pre5, h->p + h->offB[5],
                     (long long)B, h->d.hidden, h->h);
  CK(hipGetLastError());
  CK(gemm(B, h->d.n_out, h->d.hidden, h->h, h->d.hidden, 1, h->Wb[6], h->Kp[6], 1, h->scratch, 1, h->s));
  return FFT_HOMOG_OK;
}

int refresh_weights(fft_homog_cnn_t* h) {
  for (int l = 1; l <= 6; ++l) {
    hipLaunchKernelGGL(k_pack, dim3(blocks((long long)h->rows[l] * h->Kp[l])), dim3(kT), 0, h->s, h->p + h->offW[l],
                       h->rows[l], h->Kc[l], h->Kp[l], h->Wb[l]);
    CK(hipGetLastError());
  }
  return FFT_HOMOG_OK;
}

int read_flag(fft_homog_cnn_t* h) {
  CK(hipMemcpyAsync(h->h_flag, h->flag, sizeof(int), hipMemcpyDeviceToHost, h->s));
  CK(hipStreamSynchronize(h->s));
  return *h->h_flag ? FFT_HOMOG_EINVAL : FFT_HOMOG_OK;
}

}  // namespace

extern "C" {

int fft_homog_cnn_param_count(const fft_homog_cnn_desc* d, size_t* count) {
  if (!count) return FFT_HOMOG_EINVAL;
  int rc = validate(d);
  if (rc) return rc;
  Plan L;
  plan(d, &L);
  *count = L.P;
  return FFT_HOMOG_OK;
}

int fft_homog_cnn_workspace_size(const fft_homog_cnn_desc* d, size_t* bytes) {
  if (!bytes) return FFT_HOMOG_EINVAL;
  int rc = validate(d);
  if (rc) return rc;
  Plan L;
  plan(d, &L);
  *bytes = L.total;
  return FFT_HOMOG_OK;
}

int fft_homog_cnn_create(const fft_homog_cnn_desc* d, void* ws, size_t bytes, void* stream, fft_homog_cnn_t** out) {
  if (!out) return FFT_HOMOG_EINVAL;
  *out = nullptr;
  int rc = validate(d);
  if (rc) return rc;
  Plan L;
  plan(d, &L);
  if (!ws || bytes < L.total || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return FFT_HOMOG_EWORKSPACE;
  fft_homog_cnn_t* h = new fft_homog_cnn();
  h->d = *d;
  h->s = (hipStream_t)stream;
  h->ws = (char*)ws;
  h->P = L.P;
  for (int l = 1; l <= 6; ++l) {
    h->offW[l] = L.offW[l];
    h->offB[l] = L.offB[l];
    h->Kc[l] = L.Kc[l];
    h->Kp[l] = L.Kp[l];
    h->rows[l] = L.rows[l];
    h->Wb[l] = (bf16*)(h->ws + L.o_Wb[l]);
  }
  for (int l = 0; l < 5; ++l) h->edge[l] = L.edge[l];
  h->p = (float*)(h->ws + L.o_p);
  h->m = (float*)(h->ws + L.o_m);
  h->v = (float*)(h->ws + L.o_v);
  h->g = (float*)(h->ws + L.o_g);
  for (int l = 1; l <= 4; ++l) {
    h->col[l] = (bf16*)(h->ws + L.o_col[l]);
    h->pre[l] = (float*)(h->ws + L.o_pre[l]);
    h->act[l] = (bf16*)(h->ws + L.o_act[l]);
  }
  h->x5 = (bf16*)(h->ws + L.o_x5);
  h->pre5 = (float*)(h->ws + L.o_pre5);
  h->h = (bf16*)(h->ws + L.o_h);
  h->y = (float*)(h->ws + L.o_y);
  h->dy32 = (float*)(h->ws + L.o_dy32);
  h->dyb = (bf16*)(h->ws + L.o_dyb);
  h->dA = (float*)(h->ws + L.o_dA);
  h->dAb = (bf16*)(h->ws + L.o_dAb);
  h->dB = (float*)(h->ws + L.o_dB);
  h->dBb = (bf16*)(h->ws + L.o_dBb);
  h->dcol = (float*)(h->ws + L.o_dcol);
  h->scratch = (float*)(h->ws + L.o_scratch);
  h->colpart = (float*)(h->ws + L.o_colpart);
  h->lossd = (float*)(h->ws + L.o_loss);
  h->flag = (int*)(h->ws + L.o_flag);
  h->scratch_floats = L.scratch_floats;
  h->colpart_floats = L.colpart_floats;
  h->step = 0;
  h->fwd_ms = h->train_ms = 0.0;
  h->h_loss = nullptr;
  h->e0 = h->e1 = nullptr;
  hipError_t e = hipHostMalloc((void**)&h->h_loss, 64, 0);
  if (e == hipSuccess) {
    h->h_flag = (int*)(h->h_loss + 4);
    e = hipEventCreate(&h->e0);
  }
  if (e == hipSuccess) e = hipEventCreate(&h->e1);
  if (e == hipSuccess) e = hipMemsetAsync(h->ws, 0, L.o_Wb[1], h->s);  // parameters, moments, gradient
  if (e == hipSuccess) e = hipStreamSynchronize(h->s);
  if (e != hipSuccess) {
    fft_homog_cnn_destroy(h);
    return FFT_HOMOG_EDEVICE;
  }
  if (refresh_weights(h)) {
    fft_homog_cnn_destroy(h);
    return FFT_HOMOG_EDEVICE;
  }
  *out = h;
  return FFT_HOMOG_OK;
}

int fft_homog_cnn_set_params(fft_homog_cnn_t* h, const float* params) {
  if (!h || !params) return FFT_HOMOG_EINVAL;
  CK(hipMemcpyAsync(h->p, params, h->P * 4, hipMemcpyDeviceToDevice, h->s));
  CK(hipMemsetAsync(h->m, 0, h->P * 4, h->s));
  CK(hipMemsetAsync(h->v, 0, h->P * 4, h->s));
  h->step = 0;
  int rc = refresh_weights(h);
  if (rc) return rc;
  CK(hipStreamSynchronize(h->s));
  return FFT_HOMOG_OK;
}

int fft_homog_cnn_get_params(fft_homog_cnn_t* h, float* params) {
  if (!h || !params) return FFT_HOMOG_EINVAL;
  CK(hipMemcpyAsync(params, h->p, h->P * 4, hipMemcpyDeviceToDevice, h->s));
  CK(hipStreamSynchronize(h->s));
  return FFT_HOMOG_OK;
}

int fft_homog_cnn_forward(fft_homog_cnn_t* h, const uint8_t* phase, const float* feat, const float* out_scale,
                          const float* out_offset, float* out,
                          int batch) {
  if (!h || !phase || !out || (h->d.n_feat > 0 && !feat)) return FFT_HOMOG_EINVAL;
  if (check_batch(h, batch)) return FFT_HOMOG_EINVAL;
  CK(hipEventRecord(h->e0, h->s));
  int rc = forward(h, phase, feat, batch);
  if (rc) return rc;
  hipLaunchKernelGGL(k_output, dim3(blocks((long long)batch * h->d.n_out)), dim3(kT), 0, h->s, h->scratch,
                     h->p + h->offB[6], out_scale, out_offset, batch, h->d.n_out, out);
  CK(hipGetLastError());
  CK(hipEventRecord(h->e1, h->s));
  rc = read_flag(h);
  float ms = 0.f;
  CK(hipEventElapsedTime(&ms, h->e0, h->e1));
  h->fwd_ms = ms;
  return rc;
}

int fft_homog_cnn_loss_grad(fft_homog_cnn_t* h, const uint8_t* phase, const float* feat, const float* target, int B,
                            float* loss, float* grad) {
  if (!h || !phase || !target || !loss || (h->d.n_feat > 0 && !feat)) return FFT_HOMOG_EINVAL;
  if (check_batch(h, B)) return FFT_HOMOG_EINVAL;
  const int* ch = h->d.channels;
  const int O = h->d.n_out, H = h->d.hidden;
  CK(hipEventRecord(h->e0, h->s));
  int rc = forward(h, phase, feat, B);
  if (rc) return rc;
  hipLaunchKernelGGL(k_output, dim3(blocks((long long)B * O)), dim3(kT), 0, h->s, h->scratch, h->p + h->offB[6],
                     nullptr, nullptr, B, O, h->y);
  hipLaunchKernelGGL(k_loss, dim3(1), dim3(1024), 0, h->s, h->y, target, (long long)B * O, h->lossd, h->dy32, h->dyb);
  CK(hipGetLastError());
  // dense output layer: dW6 = dy^T h, db6 = sum dy, dh = dy W6
  CK(gemm(O, H, B, h->dyb, 1, O, h->h, 1, H, h->scratch, 1, h->s));
  hipLaunchKernelGGL(k_sum_splits, dim3(blocks((long long)O * H)), dim3(kT), 0, h->s, h->scratch, 1, (long long)O, H, H,
                     h->g + h->offW[6], H, 0);
  CK(colsum(h, h->dy32, B, O, h->g + h->offB[6]));
  CK(gemm(B, H, O, h->dyb, O, 1, h->Wb[6], 1, h->Kp[6], h->scratch, 1, h->s));
  hipLaunchKernelGGL(k_gelu_back, dim3(blocks((long long)B * H)), dim3(kT), 0, h->s, h->scratch, H, h->pre5, (long long)B,
                     H, 1.0f, h->dA, h->dAb);
  CK(hipGetLastError());
  // hidden layer: dW5 = dpre5^T x5, db5, dx5 = dpre5 W5
  const int K5 = h->Kc[5], Kp5 = h->Kp[5];
  CK(gemm(H, Kp5, B, h->dAb, 1, H, h->x5, 1, Kp5, h->scratch, 1, h->s));
  hipLaunchKernelGGL(k_sum_splits, dim3(blocks((long long)H * K5)), dim3(kT), 0, h->s, h->scratch, 1, (long long)H, Kp5, K5,
                     h->g + h->offW[5], K5, 0);
  CK(colsum(h, h->dA, B, H, h->g + h->offB[5]));
  CK(gemm(B, ch[4], H, h->dAb, H, 1, h->Wb[5], 1, Kp5, h->scratch, 1, h->s));
  const int V = h->edge[4] * h->edge[4] * h->edge[4];
  hipLaunchKernelGGL(k_unpool_back, dim3(blocks((long long)B * V * ch[4])), dim3(kT), 0, h->s, h->scratch, ch[4],
                     h->pre[4], B, V, ch[4], h->dB, h->dBb);
  CK(hipGetLastError());
  // conv blocks, last to first; dB/dBb hold dpre of block l
  float* d32 = h->dB;
  bf16* db = h->dBb;
  float* n32 = h->dA;
  bf16* nb = h->dAb;
  for (int l = 4; l >= 1; --l) {
    const long long Ml = (long long)B * h->edge[l] * h->edge[l] * h->edge[l];
    const int S = splits_for((int)Ml, 4096);
    if (l > 1 && implicit_conv(h, l))
      CK(gemm_conv_wgrad(ch[l], h->Kp[l], (int)Ml, db, conv_operand(h, l), h->scratch, S, h->s));
    else
      CK(gemm(ch[l], h->Kp[l], (int)Ml, db, 1, ch[l], h->col[l], 1, h->Kp[l], h->scratch, S, h->s));
    int Sused;
    {
      int chunk = ((int)Ml + S - 1) / S;
      chunk = (chunk + BK - 1) / BK * BK;
      Sused = ((int)Ml + chunk - 1) / chunk;
    }
    hipLaunchKernelGGL(k_sum_splits, dim3(blocks((long long)ch[l] * h->Kc[l])), dim3(kT), 0, h->s, h->scratch, Sused,
                       (long long)ch[l], h->Kp[l], h->Kc[l], h->g + h->offW[l], h->Kc[l], 0);
    CK(colsum(h, d32, Ml, ch[l], h->g + h->offB[l]));
    if (l > 1) {
      CK(gemm((int)Ml, h->Kp[l], ch[l], db, ch[l], 1, h->Wb[l], 1, h->Kp[l], h->dcol, 1, h->s));
      const int nin = h->edge[l - 1];
      const long long Min = (long long)B * nin * nin * nin;
      hipLaunchKernelGGL(k_col2im_gelu, dim3(blocks(Min * ch[l - 1])), dim3(kT), 0, h->s, h->dcol, B, nin, ch[l - 1],
                         h->Kp[l], h->pre[l - 1], n32, nb);
      CK(hipGetLastError());
      std::swap(d32, n32);
      std::swap(db, nb);
    }
  }
  if (grad) CK(hipMemcpyAsync(grad, h->g, h->P * 4, hipMemcpyDeviceToDevice, h->s));
  CK(hipMemcpyAsync(h->h_loss, h->lossd, 4, hipMemcpyDeviceToHost, h->s));
  CK(hipEventRecord(h->e1, h->s));
  rc = read_flag(h);
  *loss = h->h_loss[0];
  float ms = 0.f;
  CK(hipEventElapsedTime(&ms, h->e0, h->e1));
  h->train_ms = ms;
  return rc;
}

int fft_homog_cnn_adam_step(fft_homog_cnn_t* h, float lr, float beta1, float beta2, float eps) {
  if (!h || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return FFT_HOMOG_EINVAL;
  h->step += 1;
  const float bc1 = 1.0f - powf(beta1, (float)h->step);
  const float bc2 = 1.0f - powf(beta2, (float)h->step);
  hipLaunchKernelGGL(k_adam, dim3(blocks((long long)h->P)), dim3(kT), 0, h->s, h->p, h->m, h->v, h->g, (long long)h->P, lr,
                     beta1, beta2, eps, bc1, bc2);
  CK(hipGetLastError());
  int rc = refresh_weights(h);
  if (rc) return rc;
  CK(hipStreamSynchronize(h->s));
  return FFT_HOMOG_OK;
}

int fft_homog_cnn_check(fft_homog_cnn_t* h, const uint8_t* phase, const float* lam_mu, const float* feat, float* C,
                        const float* C2, int batch, float tol, float lo, float hi, float max_spread, int* ok,
                        float* spread_out) {
  if (!h || !phase || !lam_mu || !C || !ok || (h->d.n_feat > 0 && !feat)) return FFT_HOMOG_EINVAL;
  if (h->d.n_out != 21) return FFT_HOMOG_EINVAL;
  if (batch < 1) return FFT_HOMOG_EINVAL;
  const long long Nv = (long long)h->d.n * h->d.n * h->d.n;
  hipLaunchKernelGGL(k_check, dim3(batch), dim3(kT), 0, h->s, phase, Nv, lam_mu, feat, h->d.n_feat, C, C2, tol, lo, hi,
                     max_spread, ok, spread_out);
  CK(hipGetLastError());
  CK(hipStreamSynchronize(h->s));
  return FFT_HOMOG_OK;
}

int fft_homog_cnn_last_ms(const fft_homog_cnn_t* h, double* fwd, double* train) {
  if (!h) return FFT_HOMOG_EINVAL;
  if (fwd) *fwd = h->fwd_ms;
  if (train) *train = h->train_ms;
  return FFT_HOMOG_OK;
}

void fft_homog_cnn_destroy(fft_homog_cnn_t* h) {
  if (!h) return;
  if (h->s) (void)hipStreamSynchronize(h->s);
  else (void)hipDeviceSynchronize();
  if (h->h_loss) (void)hipHostFree(h->h_loss);
  if (h->e0) (void)hipEventDestroy(h->e0);
  if (h->e1) (void)hipEventDestroy(h->e1);
  delete h;
}

int fft_homog_cnn_debug_gemm(fft_homog_cnn_t* h, int M, int N, int K, const uint16_t* A, long long sam, long long sak,
                             const uint16_t* B, long long sbn, long long sbk, float* C, int splits) {
  if (!h || !A || !B || !C || M < 1 || N < 1 || K < 1 || splits < 1 || splits > kMaxSplits) return FFT_HOMOG_EINVAL;
  if (!(sak == 1 || sam == 1) || !(sbk == 1 || sbn == 1)) return FFT_HOMOG_EINVAL;
  CK(gemm(M, N, K, A, sam, sak, B, sbn, sbk, C, splits, h->s));
  CK(hipStreamSynchronize(h->s));
  return FFT_HOMOG_OK;
}

}  // extern "C"
