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
// the solution.
//
// Partitioned form (k_tridiag_chunk): each line's rows are split into chunks of TL rows, one thread per chunk,
// with the chunk held in registers. The reciprocal pivots depend only on the line's shift b, so the pivot
// entering each chunk is computed once per context (k_tri_pivots) and each thread restarts the pivot recurrence
// from it. With zero incoming values each chunk's forward sweep gives d'_e = A d'_{s-1} + B and its backward
// sweep u_s = A u_{e+1} + D (A = prod of -1/pivot over the chunk); these affine maps are composed along the line
// in LDS, and a last pass adds the incoming contributions. The result equals Thomas elimination up to the
// order of rounding; HBM traffic is one read and one write per unknown (plus one pivot per chunk).
#include "tridiag_dev.h"

namespace helm {

namespace {

// reciprocal pivot entering each chunk: piv[k * lines + line] = 1/pivot_{k TL - 1} (k >= 1), 0 for k = 0; piv32 (if
// given) receives the same table rounded to complex64 for the FP32 z-solve
__global__ void k_tri_pivots(const double2 *__restrict__ dx, const double2 *__restrict__ dy, int nx, int ny, int nz,
                             double ax, double ay, double c0, double2 g, double zi, double2 *__restrict__ piv,
                             float2 *__restrict__ piv32) {
    const long long lines = (long long)nx * ny;
    const long long line = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (line >= lines) return;
    const int i = (int)(line % nx), j = (int)(line / nx);
    const double2 ex = dx[i], ey = dy[j];
    const double2 b = make_double2(ax * ex.x + ay * ey.x + c0, ax * ex.y + ay * ey.y);
    double2 inv = make_double2(0.0, 0.0);
    piv[line] = inv;
    if (piv32) piv32[line] = make_float2(0.f, 0.f);
    for (int l = 0; l < nz; ++l) {
        double2 d = b;
        if (l == 0 || l == nz - 1) { d.x = (d.x + g.x) * zi; d.y = (d.y + g.y) * zi; }
        if (l > 0) { d.x -= inv.x; d.y -= inv.y; }
        inv = crecip(d);
        if ((l + 1) % TL == 0 && l + 1 < nz) {
            const long long o = (long long)((l + 1) / TL) * lines + line;
            piv[o] = inv;
            if (piv32) piv32[o] = make_float2((float)inv.x, (float)inv.y);
        }
    }
}

template <typename T, typename PT>
__global__ __launch_bounds__(1024) void k_tridiag_chunk(const typename c2<T>::t *in, typename c2<T>::t *out,
                                                        const PT *__restrict__ piv,
                                                        const double2 *__restrict__ dx, const double2 *__restrict__ dy,
                                                        int nx, int ny, int nz, int P, int LX, double ax, double ay,
                                                        double c0, double2 gz, double scale, double zi) {
    extern __shared__ unsigned char smraw[];
    tri_chunk_block<T, PT>(in, out, piv, dx, dy, nx, ny, nz, P, LX, ax, ay, c0, gz, scale, blockIdx.x, smraw, zi);
}

template <typename T, typename PT>
hipError_t launch_chunk(const typename c2<T>::t *in, typename c2<T>::t *out, const PT *piv, const double2 *dx,
                        const double2 *dy, int nx, int ny, int nz, double ax, double ay, double c0, double2 gz,
                        double scale, hipStream_t s, double zi) {
    const int P = (nz + TL - 1) / TL;
    if (P > 1024) return hipErrorInvalidValue;
    // 16 lines per block (256 B per row access) for complex128, 32 for complex64 (measured 10% faster at 256^3)
    int LX = sizeof(T) == 4 ? 32 : 16;
    while (LX > 1 && LX * P > 1024) LX /= 2;
    const long long lines = (long long)nx * ny;
    const unsigned grid = (unsigned)((lines + LX - 1) / LX);
    const size_t sm = 2 * sizeof(typename c2<T>::t) * (size_t)P * LX;
    hipLaunchKernelGGL((k_tridiag_chunk<T, PT>), dim3(grid), dim3(LX * P), sm, s, in, out, piv, dx, dy, nx, ny, nz, P,
                       LX, ax, ay, c0, gz, scale, zi);
    return hipGetLastError();
}

}  // namespace

int tri_chunks(int nz) { return (nz + TL - 1) / TL; }

hipError_t launch_tri_pivots(const double2 *dx, const double2 *dy, int nx, int ny, int nz, double ax, double ay,
                             double c0, double2 gz, double2 *piv, float2 *piv32, hipStream_t s, double zi) {
    const long long lines = (long long)nx * ny;
    hipLaunchKernelGGL(k_tri_pivots, dim3((unsigned)((lines + 255) / 256)), dim3(256), 0, s, dx, dy, nx, ny, nz, ax,
                       ay, c0, gz, zi, piv, piv32);
    return hipGetLastError();
}

hipError_t launch_tridiag_chunk_z64(const double2 *in, double2 *out, const double2 *piv, const double2 *dx,
                                    const double2 *dy, int nx, int ny, int nz, double ax, double ay, double c0,
                                    double2 gz, double scale, hipStream_t s, double zi) {
    return launch_chunk<double, double2>(in, out, piv, dx, dy, nx, ny, nz, ax, ay, c0, gz, scale, s, zi);
}

hipError_t launch_tridiag_chunk_z32(const float2 *in, float2 *out, const float2 *piv, const double2 *dx,
                                    const double2 *dy, int nx, int ny, int nz, double ax, double ay, double c0,
                                    double2 gz, double scale, hipStream_t s, double zi) {
    return launch_chunk<float, float2>(in, out, piv, dx, dy, nx, ny, nz, ax, ay, c0, gz, scale, s, zi);
}

}  // namespace helm
