// The CG-loop pass kernels instantiated for single axis lengths with compiled radix schedules
// (96, 64, 48 and 32 points; 128 has its one-butterfly kernels in kernels.hip): each holds only
// that length's schedule, so its registers do not follow the longest schedule of the generic
// kernels.  The launchers in kernels.hip route here when the axis has one of these lengths and its
// transform runs register-staged in place; the arithmetic is that of the generic kernels.
#include <initializer_list>

#include "pass_kernels.h"

namespace fh {

namespace {

template <int L>
hipError_t xfwd_len(int prod, int mat, const XFwdArgs& a, dim3 grid, size_t sm, hipStream_t s, bool* done) {
  *done = prod == PROD_CGOP && (mat == 1 || mat == 3 || mat == 5 || mat == 7);
  if (!*done) return hipSuccess;
  switch (mat) {
    case 1: hipLaunchKernelGGL((k_xfwd<PROD_CGOP, MAT_LE, 3, kStaged + L>), grid, dim3(kThreads), sm, s, a); break;
    case 3: hipLaunchKernelGGL((k_xfwd<PROD_CGOP, MAT_NH, 3, kStaged + L>), grid, dim3(kThreads), sm, s, a); break;
    case 5: hipLaunchKernelGGL((k_xfwd<PROD_CGOP, MAT_STVK, 3, kStaged + L>), grid, dim3(kThreads), sm, s, a); break;
    default: hipLaunchKernelGGL((k_xfwd<PROD_CGOP, MAT_J2, 3, kStaged + L>), grid, dim3(kThreads), sm, s, a); break;
  }
  return hipGetLastError();
}

template <int L>
hipError_t xinv_len(int cons, const XInvArgs& a, dim3 grid, size_t sm, hipStream_t s, bool* done) {
  *done = cons == CONS_CGUPD && (a.g.c == 6 || a.g.c == 9);
  if (!*done) return hipSuccess;
  if (a.g.c == 6) hipLaunchKernelGGL((k_xinv<CONS_CGUPD, 6, kStaged + L>), grid, dim3(kThreads), sm, s, a);
  else hipLaunchKernelGGL((k_xinv<CONS_CGUPD, 9, kStaged + L>), grid, dim3(kThreads), sm, s, a);
  return hipGetLastError();
}

template <int L>
hipError_t mid_len(int dir, bool rows, const AxisArgs& a, dim3 grid, size_t sm, hipStream_t s) {
  return dispatch_mid<kStaged + L>(dir, rows, a, grid, sm, s);
}

template <int L>
hipError_t outer_len(int mode, bool rows, const AxisArgs& a, dim3 grid, size_t sm, hipStream_t s, bool* done) {
  *done = rows || (mode == OUTER_PROJECT && a.g.small && a.g.ndim == 3);
  if (!*done) return hipSuccess;
  if (rows) hipLaunchKernelGGL((k_outer_frow<kStaged + L>), grid, dim3(kThreads), sm, s, a);
  else hipLaunchKernelGGL((k_outer<OUTER_PROJECT, 1, 3, kStaged + L>), grid, dim3(kThreads), sm, s, a);
  return hipGetLastError();
}

template <int L>
hipError_t limits_len(int mat, size_t bytes) {
  const int attr = (int)hipFuncAttributeMaxDynamicSharedMemorySize;
  hipError_t e = hipSuccess;
#define FH_SET(fn) \
  if (e == hipSuccess) e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn), (hipFuncAttribute)attr, (int)bytes)
  switch (mat) {
    case 1: FH_SET((k_xfwd<PROD_CGOP, MAT_LE, 3, kStaged + L>)); break;
    case 3: FH_SET((k_xfwd<PROD_CGOP, MAT_NH, 3, kStaged + L>)); break;
    case 5: FH_SET((k_xfwd<PROD_CGOP, MAT_STVK, 3, kStaged + L>)); break;
    case 7: FH_SET((k_xfwd<PROD_CGOP, MAT_J2, 3, kStaged + L>)); break;
    default: break;
  }
  FH_SET((k_xinv<CONS_CGUPD, 6, kStaged + L>));
  FH_SET((k_xinv<CONS_CGUPD, 9, kStaged + L>));
  FH_SET((k_mid<-1, kStaged + L>));
  FH_SET((k_mid<1, kStaged + L>));
  FH_SET((k_mid_frow<-1, kStaged + L>));
  FH_SET((k_mid_frow<1, kStaged + L>));
  FH_SET((k_outer_frow<kStaged + L>));
  FH_SET((k_outer<OUTER_PROJECT, 1, 3, kStaged + L>));
#undef FH_SET
  return e;
}

}  // namespace

bool fixed_len_kernels(int n) { return n == 96 || n == 64 || n == 48 || n == 32; }

#define FH_LEN_SWITCH(n, CALL) \
  switch (n) {                 \
    case 96: CALL(96);         \
    case 64: CALL(64);         \
    case 48: CALL(48);         \
    case 32: CALL(32);         \
    default: break;            \
  }

hipError_t launch_xfwd_fixed(int prod, int mat, const XFwdArgs& a, dim3 grid, size_t sm, hipStream_t s, bool* done) {
  *done = false;
#define FH_C(L) return xfwd_len<L>(prod, mat, a, grid, sm, s, done);
  FH_LEN_SWITCH(a.px.n, FH_C)
#undef FH_C
  return hipSuccess;
}
hipError_t launch_xinv_fixed(int cons, const XInvArgs& a, dim3 grid, size_t sm, hipStream_t s, bool* done) {
  *done = false;
#define FH_C(L) return xinv_len<L>(cons, a, grid, sm, s, done);
  FH_LEN_SWITCH(a.px.n, FH_C)
#undef FH_C
  return hipSuccess;
}
hipError_t launch_mid_fixed(int dir, bool rows, const AxisArgs& a, dim3 grid, size_t sm, hipStream_t s, bool* done) {
  *done = true;
#define FH_C(L) return mid_len<L>(dir, rows, a, grid, sm, s);
  FH_LEN_SWITCH(a.pl.n, FH_C)
#undef FH_C
  *done = false;
  return hipSuccess;
}
hipError_t launch_outer_fixed(int mode, bool rows, const AxisArgs& a, dim3 grid, size_t sm, hipStream_t s, bool* done) {
  *done = false;
#define FH_C(L) return outer_len<L>(mode, rows, a, grid, sm, s, done);
  FH_LEN_SWITCH(a.pl.n, FH_C)
#undef FH_C
  return hipSuccess;
}
hipError_t set_smem_limits_fixed(const Geom& g, int mat, size_t bytes) {
  hipError_t e = hipSuccess;
  for (int n : {g.nx, g.ny, g.nz}) {
    if (e != hipSuccess || !fixed_len_kernels(n)) continue;
#define FH_C(L) e = limits_len<L>(mat, bytes); break;
    FH_LEN_SWITCH(n, FH_C)
#undef FH_C
  }
  return e;
}

}  // namespace fh
