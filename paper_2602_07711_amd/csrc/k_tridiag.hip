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
#include "helm_internal.h"

namespace helm {

namespace {

template <typename T> struct c2;
template <> struct c2<double> { typedef double2 t; };
template <> struct c2<float> { typedef float2 t; };

template <typename T, typename CT> __device__ __forceinline__ CT mk(T a, T b) {
    CT r;
    r.x = a;
    r.y = b;
    return r;
}
template <typename CT> __device__ __forceinline__ CT cm(CT a, CT b) {
    CT r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename CT> __device__ __forceinline__ CT crecip(CT a) {
    auto s = a.x * a.x + a.y * a.y;
    CT r;
    r.x = a.x / s;
    r.y = -a.y / s;
    return r;
}

constexpr int UNR = 8;

template <typename T>
__global__ __launch_bounds__(64) void k_tridiag(const typename c2<T>::t *in, typename c2<T>::t *r, typename c2<T>::t *__restrict__ cp,
                                                const double2 *__restrict__ dx, const double2 *__restrict__ dy, int nx,
                                                int ny, int nz, double ax, double ay, double c0, double2 gz,
                                                double scale) {
    typedef typename c2<T>::t CT;
    const long long lines = (long long)nx * ny;
    const long long line = (long long)blockIdx.x * 64 + threadIdx.x;
    if (line >= lines) return;
    const int i = (int)(line % nx), j = (int)(line / nx);
    const double2 ex = dx[i], ey = dy[j];
    const CT b = mk<T, CT>((T)(ax * ex.x + ay * ey.x + c0), (T)(ax * ex.y + ay * ey.y));
    const CT g = mk<T, CT>((T)gz.x, (T)gz.y);
    const T sc = (T)scale;
    CT *rl = r + line;
    const CT *il = in + line;
    CT *cl = cp + line;

    CT inv = mk<T, CT>(0, 0), dprev = mk<T, CT>(0, 0);
    for (int l0 = 0; l0 < nz; l0 += UNR) {
        CT v[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u)
            if (l0 + u < nz) v[u] = il[(long long)(l0 + u) * lines];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int l = l0 + u;
            if (l >= nz) break;
            CT diag = b;
            if (l == 0 || l == nz - 1) { diag.x += g.x; diag.y += g.y; }
            if (l > 0) { diag.x -= inv.x; diag.y -= inv.y; }
            inv = crecip(diag);
            CT rhs = mk<T, CT>(sc * v[u].x - dprev.x, sc * v[u].y - dprev.y);
            dprev = cm(rhs, inv);
            rl[(long long)l * lines] = dprev;
            cl[(long long)l * lines] = inv;
        }
    }
    CT unext = dprev;   // u_N = d'_N, already stored
    for (int l1 = nz - 2; l1 >= 0; l1 -= UNR) {
        CT dv[UNR], cv[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u)
            if (l1 - u >= 0) {
                dv[u] = rl[(long long)(l1 - u) * lines];
                cv[u] = cl[(long long)(l1 - u) * lines];
            }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int l = l1 - u;
            if (l < 0) break;
            CT t = cm(cv[u], unext);
            unext = mk<T, CT>(dv[u].x - t.x, dv[u].y - t.y);
            rl[(long long)l * lines] = unext;
        }
    }
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
