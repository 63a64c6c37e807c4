// Batched z-tridiagonal solves of the EigT preconditioner (Sec. 4.1, eq. Indep_precond_system), zeta_z = 1:
//   (gz + b) u_1 + u_2 = r_1,   u_{l-1} + b u_l + u_{l+1} = r_l,   u_{N-1} + (gz + b) u_N = r_N,
// one system per transformed line (i, j), with b = a_x d_x,i + a_y d_y,j + h_z^2 k0^2 - 2(a_x + a_y + 1)
// (eq. DIAGprec) built on the fly from the 1D eigenvalues, and r = h_z^2 * (transformed data), so that the
// system solved is A_p u = h_z^2 y, i.e. M u = y.
//
// Thomas elimination without pivoting: the eigenvalues of Lambda-bar lie in Im >= 0 for Im gamma >= 0, so
// every pivot stays in the upper half plane and away from zero. One thread owns one line; consecutive
// threads own consecutive i, so every access of a wavefront at a given l is one contiguous 64-element run.
// The forward sweep reads the right-hand side from `in` (which may be r itself), writes the eliminated
// right-hand side to r and the reciprocal pivots to `cp`; the backward sweep reads both and overwrites r with
// the solution. Loads are issued UNR levels ahead of use.
#include "tridiag_dev.h"

namespace helm {

namespace {

template <typename T>
__global__ __launch_bounds__(64) void k_tridiag(const typename c2<T>::t *in, typename c2<T>::t *r,
                                                typename c2<T>::t *__restrict__ cp, const double2 *__restrict__ dx,
                                                const double2 *__restrict__ dy, int nx, int ny, int nz, double ax,
                                                double ay, double c0, double2 gz, double scale) {
    const long long line = (long long)blockIdx.x * 64 + threadIdx.x;
    if (line >= (long long)nx * ny) return;
    tridiag_line<T>(in, r, cp, dx, dy, nx, ny, nz, ax, ay, c0, gz, scale, line);
}

}  // namespace

hipError_t launch_tridiag_z64(const double2 *in, double2 *r, double2 *cp, const double2 *dx, const double2 *dy, int nx,
                              int ny, int nz, double ax, double ay, double c0, double2 gz, double scale, hipStream_t s) {
    long long lines = (long long)nx * ny;
    hipLaunchKernelGGL(k_tridiag<double>, dim3((unsigned)((lines + 63) / 64)), dim3(64), 0, s, in, r, cp, dx, dy, nx,
                       ny, nz, ax, ay, c0, gz, scale);
    return hipGetLastError();
}

hipError_t launch_tridiag_z32(const float2 *in, float2 *r, float2 *cp, const double2 *dx, const double2 *dy, int nx,
                              int ny, int nz, double ax, double ay, double c0, double2 gz, double scale, hipStream_t s) {
    long long lines = (long long)nx * ny;
    hipLaunchKernelGGL(k_tridiag<float>, dim3((unsigned)((lines + 63) / 64)), dim3(64), 0, s, in, r, cp, dx, dy, nx,
                       ny, nz, ax, ay, c0, gz, scale);
    return hipGetLastError();
}

}  // namespace helm
