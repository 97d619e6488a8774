// Host-only exercise of the C ABI's host logic under AddressSanitizer and UndefinedBehaviorSanitizer:
// descriptor validation and workspace layout over many grids, the FFT plans (direct stages and the
// chirp-z form) of every axis length, the CG chunk policy, status strings and the argument checks
// that every entry point makes before it touches a device.  Built from
// the library's own sources with host-only compilation (no device code, no GPU needed) by
// tests/test_host_sanitized.py; exits non-zero if an expectation fails.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>

#include "fft_homog.h"
#include "kernels.h"

static int failures = 0;
#define EXPECT(cond)                                                        \
  do {                                                                      \
    if (!(cond)) {                                                          \
      std::fprintf(stderr, "expectation failed: %s (line %d)\n", #cond, __LINE__); \
      ++failures;                                                           \
    }                                                                       \
  } while (0)

static fft_homog_desc make(int ndim, int nx, int ny, int nz, int kin, int mat) {
  fft_homog_desc d;
  std::memset(&d, 0, sizeof(d));
  d.ndim = ndim;
  d.n[0] = nx;
  d.n[1] = ny;
  d.n[2] = nz;
  d.len[0] = d.len[1] = d.len[2] = 1.0;
  d.kinematics = kin;
  d.material = mat;
  d.nphase = 2;
  d.tol_newton = 1e-10;
  d.tol_cg = 1e-10;
  d.max_newton = 50;
  d.max_cg = 1000;
  d.k_mode = FFT_HOMOG_K_RECOMPUTE;
  d.flags = 0;
  d.batch = 1;
  return d;
}

int main() {
  // workspace sizes over grids with every radix path: powers of two, 3, 5, large primes, ragged
  const int sizes[] = {1, 2, 3, 5, 7, 8, 12, 13, 16, 17, 31, 32, 33, 48, 64, 80, 96, 97, 128, 160, 192, 199, 256, 299};
  const int kins[2] = {FFT_HOMOG_SMALL_STRAIN, FFT_HOMOG_FINITE_STRAIN};
  const int mats[2][2] = {{FFT_HOMOG_LINEAR_ELASTIC, FFT_HOMOG_J2_PLASTIC}, {FFT_HOMOG_NEO_HOOKEAN, FFT_HOMOG_STVK}};
  long long checked = 0;
  for (int ndim = 2; ndim <= 3; ++ndim)
    for (int k = 0; k < 2; ++k)
      for (int m = 0; m < 2; ++m)
        for (int a : sizes)
          for (int b : {1, 7, 32, 33}) {
            for (int flags : {0, (int)FFT_HOMOG_FLAG_TANGENT}) {
              fft_homog_desc d = make(ndim, a, b, ndim == 3 ? (a % 5) + 1 : 1, kins[k], mats[k][m]);
              d.flags = (unsigned)flags;
              size_t bytes = 0;
              const int rc = fft_homog_workspace_size(&d, &bytes);
              EXPECT(rc == FFT_HOMOG_OK);
              if (rc == FFT_HOMOG_OK) {
                const long long N = (long long)a * b * (ndim == 3 ? (a % 5) + 1 : 1);
                const int c = kins[k] == FFT_HOMOG_SMALL_STRAIN ? (ndim == 3 ? 6 : 3) : ndim * ndim;
                EXPECT(bytes >= (size_t)(8 * c * N * 4));
              }
              ++checked;
            }
          }
  // multi-cell handles
  for (int cells : {2, 16, 1000}) {
    fft_homog_desc d = make(3, 32, 32, 32, FFT_HOMOG_SMALL_STRAIN, FFT_HOMOG_LINEAR_ELASTIC);
    d.flags = FFT_HOMOG_FLAG_TANGENT;
    d.batch = cells;
    size_t bytes = 0;
    EXPECT(fft_homog_workspace_size(&d, &bytes) == FFT_HOMOG_OK);
  }
  // invalid descriptors are rejected on the host
  {
    fft_homog_desc d = make(3, 8, 8, 8, FFT_HOMOG_SMALL_STRAIN, FFT_HOMOG_LINEAR_ELASTIC);
    size_t bytes = 0;
    fft_homog_desc e = d; e.ndim = 4; EXPECT(fft_homog_workspace_size(&e, &bytes) == FFT_HOMOG_EINVAL);
    e = d; e.n[1] = 0; EXPECT(fft_homog_workspace_size(&e, &bytes) == FFT_HOMOG_EINVAL);
    e = d; e.n[0] = 5000; EXPECT(fft_homog_workspace_size(&e, &bytes) == FFT_HOMOG_EUNSUPPORTED);
    e = d; e.len[2] = NAN; EXPECT(fft_homog_workspace_size(&e, &bytes) == FFT_HOMOG_EINVAL);
    e = d; e.tol_cg = -1.0; EXPECT(fft_homog_workspace_size(&e, &bytes) == FFT_HOMOG_EINVAL);
    e = d; e.nphase = 300; EXPECT(fft_homog_workspace_size(&e, &bytes) == FFT_HOMOG_EINVAL);
    e = d; e.flags = 1u << 9; EXPECT(fft_homog_workspace_size(&e, &bytes) == FFT_HOMOG_EINVAL);
    e = d; e.batch = 4; EXPECT(fft_homog_workspace_size(&e, &bytes) == FFT_HOMOG_EINVAL);
    e = d; e.batch = 2000; e.flags = FFT_HOMOG_FLAG_TANGENT; EXPECT(fft_homog_workspace_size(&e, &bytes) == FFT_HOMOG_EUNSUPPORTED);
    EXPECT(fft_homog_workspace_size(nullptr, &bytes) == FFT_HOMOG_EINVAL);
    EXPECT(fft_homog_workspace_size(&d, nullptr) == FFT_HOMOG_EINVAL);
    // create refuses a missing or short workspace before any device call
    fft_homog_t* h = nullptr;
    EXPECT(fft_homog_create(&d, nullptr, 0, nullptr, &h) == FFT_HOMOG_EWORKSPACE && h == nullptr);
    EXPECT(std::strlen(fft_homog_last_error(nullptr)) > 0);
    EXPECT(fft_homog_create(&d, (void*)256, 16, nullptr, &h) == FFT_HOMOG_EWORKSPACE);
    EXPECT(fft_homog_create(&e, nullptr, 0, nullptr, &h) != FFT_HOMOG_OK);
    EXPECT(fft_homog_create(&d, nullptr, 0, nullptr, nullptr) == FFT_HOMOG_EINVAL);
    // the allocation-free projection refuses bad arguments and oversize requests before any launch
    double dummy[4];
    EXPECT(fft_homog_project_noalloc(&d, nullptr, dummy, 1, nullptr) == FFT_HOMOG_EINVAL);
    EXPECT(fft_homog_project_noalloc(&d, dummy, dummy, 0, nullptr) == FFT_HOMOG_EINVAL);
    EXPECT(fft_homog_project_noalloc(&e, dummy, dummy, 1, nullptr) != FFT_HOMOG_OK);
    fft_homog_desc big = make(3, 128, 128, 128, FFT_HOMOG_FINITE_STRAIN, FFT_HOMOG_NEO_HOOKEAN);
    EXPECT(fft_homog_project_noalloc(&big, dummy, dummy, 1, nullptr) == FFT_HOMOG_EWORKSPACE);
    EXPECT(std::strstr(fft_homog_last_error(nullptr), "scratch") != nullptr);
    // null handles
    EXPECT(fft_homog_solve(nullptr, nullptr, 1, nullptr, nullptr, nullptr) == FFT_HOMOG_EINVAL);
    EXPECT(fft_homog_tangent(nullptr, nullptr, nullptr) == FFT_HOMOG_EINVAL);
    EXPECT(fft_homog_get_launch_shape(nullptr, nullptr) == FFT_HOMOG_EINVAL);
    EXPECT(fft_homog_tune_placement(nullptr, 1, nullptr) == FFT_HOMOG_EINVAL);
    EXPECT(fft_homog_set_placement(nullptr, 0) == FFT_HOMOG_EINVAL);
    fft_homog_destroy(nullptr);
    // plane stress: every law in 2D, none in 3D
    for (int kin = 0; kin < 2; ++kin)
      for (int m = 0; m < 2; ++m) {
        fft_homog_desc ps = make(2, 31, 31, 1, kins[kin], mats[kin][m]);
        ps.flags = FFT_HOMOG_FLAG_PLANE_STRESS;
        EXPECT(fft_homog_workspace_size(&ps, &bytes) == FFT_HOMOG_OK);
        fft_homog_desc ps3 = make(3, 8, 8, 8, kins[kin], mats[kin][m]);
        ps3.flags = FFT_HOMOG_FLAG_PLANE_STRESS;
        EXPECT(fft_homog_workspace_size(&ps3, &bytes) == FFT_HOMOG_EINVAL);
      }
    // large grids keep 16 MiB of placement slack behind the spectrum: the 128^3 finite-strain
    // workspace exceeds its buffers' sum (F, x, r, p: 4 x 144 MiB; spectrum 9 x 65 x 128^2 x 16 B)
    {
      fft_homog_desc nh = make(3, 128, 128, 128, FFT_HOMOG_FINITE_STRAIN, FFT_HOMOG_NEO_HOOKEAN);
      EXPECT(fft_homog_workspace_size(&nh, &bytes) == FFT_HOMOG_OK);
      const size_t vecs = 4 * (size_t)9 * 128 * 128 * 128 * 8 + (size_t)9 * 72 * 128 * 128 * 16;
      EXPECT(bytes >= vecs + (16u << 20));
    }
  }
  // status strings
  for (int s = 0; s < 12; ++s) EXPECT(fft_homog_strerror(s) != nullptr);
  // CG chunk policy: always 1..16 iterations, for any residual history (including NaN and Inf)
  const double vals[] = {0.0, 1e-300, 1e-30, 1e-12, 0.5, 1.0, 2.0, 1e30, INFINITY, NAN, -1.0};
  for (int it : {0, 1, 4, 5, 100, 1000000})
    for (double rr0 : vals)
      for (double rr : vals)
        for (double tol : {1e-16, 1e-10, 0.5, 0.0})
          for (int prev : {-1, 0, 3, it})
            for (double prr : vals) {
              const int m = fft_homog_debug_cg_chunk(it, rr0, rr, tol, prev, prr);
              EXPECT(m >= 1 && m <= 16);
            }
  // FFT plans of every axis length: the stages multiply out to the length they run on; a chirp-z
  // plan has a convolution length m >= 2n - 1 with factors 2, 3, 5 only and register-stageable
  // radices, and is chosen only when the direct prime stages add up to more than the threshold
  for (int lim : {0, 70, 150}) {
    for (int n = 1; n <= 1024; ++n) {
      fh::AxisPlan pl;
      EXPECT(fh::make_plan(n, &pl, lim));
      const int L = fh::lds_len(pl);
      long long prod = 1;
      int primes = 0;
      EXPECT(pl.nstages >= 0 && pl.nstages <= fh::kMaxStages);
      for (int st = 0; st < pl.nstages; ++st) prod *= pl.radix[st];
      EXPECT(prod == L || (n == 1 && L == 1));
      int q = n;
      for (int p = 2; q > 1; ++p)
        while (q % p == 0) {
          if (p > 5) primes += p;
          q /= p;
        }
      if (pl.m > 0) {
        EXPECT(lim > 0 && primes > lim);
        EXPECT(pl.m >= 2 * n - 1 && pl.m <= 2048);
        int r = pl.m;
        for (int p : {2, 3, 5})
          while (r % p == 0) r /= p;
        EXPECT(r == 1);
        for (int st = 0; st < pl.nstages; ++st) EXPECT(pl.radix[st] <= 16 && pl.radix[st] != 7);
        EXPECT(fh::plan_table_elems(pl) == (size_t)(pl.m + n + pl.m));
      } else {
        EXPECT(lim == 0 || primes <= lim || 2 * n - 1 > 2048);
        EXPECT(fh::plan_table_elems(pl) == (size_t)n);
      }
    }
  }
  {
    fh::AxisPlan pl;
    fh::make_plan(199, &pl, 150);
    EXPECT(pl.m == 400);
    fh::make_plan(97, &pl, 70);
    EXPECT(pl.m == 200);
    fh::make_plan(97, &pl, 150);
    EXPECT(pl.m == 0 && pl.nstages == 1 && pl.radix[0] == 97);
    fh::make_plan(299, &pl, 70);
    EXPECT(pl.m == 0);  // 13 + 23 = 36
    fh::make_plan(511, &pl, 70);
    EXPECT(pl.m == 1024);  // 7 + 73 = 80
    fh::make_plan(1021, &pl, 150);
    EXPECT(pl.m == 2048);
    fh::make_plan(128, &pl, 70);
    EXPECT(pl.m == 0 && pl.nstages == 2 && pl.radix[0] == 16 && pl.radix[1] == 8);
  }
  std::printf("host checks: %lld descriptors, %d failures\n", checked, failures);
  return failures == 0 ? 0 : 1;
}
