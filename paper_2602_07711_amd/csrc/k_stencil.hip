// Compact-stencil kernels: derived k^2 fields, the modified right-hand side, and the matrix-vector product
// y = A x of the 2nd/4th/6th-order schemes with the ghost-eliminated absorbing closure.
//
// Operator (per node p, neighbour offsets o in {-1,0,1}^3, U_o the neighbour value, k_o^2 its k^2):
//   order 4 (Sec. 2.2 eq. scheme4):  sum_o c_o U_o + k_p^2 U_p / 2 + sum_faces k_o^2 U_o / 12, with the
//     grid-only coefficients c_o of Delta + sum (h_nu^2+h_mu^2)/12 T_nu T_mu (19 points).
//   order 6 (Sec. 2.3 eq. scheme6, uniform h): collecting the scheme by neighbour class,
//     y = dg U_p + (S3 + 3 S2 + 14 S1)/(30 h^2) + (SW2 - SW1)/90 + sum_nu g_nu (2 D_nu U + D_nu E + h^2 D_nu W)
//     with S1/S2/S3 the sums of U over faces/edges/corners, SW1/SW2 the sums of k^2 U over faces/edges,
//     D_nu U = U(+nu) - U(-nu), D_nu W the same for k^2 U, D_nu E the difference of the edge sums on the
//     +nu and -nu sides, g_nu = h (k^2)_nu / 120 and dg = -64/(15 h^2) + 14/15 k^2 + h^2/20 (lap k^2 - k^4).
// Ghost rule (Sec. 2.3 eq. D_bc): a neighbour outside the grid along an axis takes the boundary node's value
// times gamma of that axis (per clamped axis), and k^2 there is the boundary node's k^2, so the products
// k^2 U obey the same rule.
//
// The matvec (stencil_dev.h) streams z-planes of U and k^2 (with a one-node halo) through LDS, one thread per
// output column. Per node it streams x (16 B), k^2 (8 B), the order-6 field block (32 B), F in the residual form
// (16 B) and writes y (16 B).
#include "stencil_dev.h"

namespace helm {

namespace {

// --------------------------------------------------------------------------- derived fields
// k2 (interior copy) and, for order 6, fld = (dg, g_x, g_y, g_z). k2_halo has `halo` cells per side.
__global__ void k_derived(const double *__restrict__ k2h, int halo, double *__restrict__ k2, double4 *__restrict__ fld,
                          int nx, int ny, int nz, int order, double h, int *__restrict__ bad) {
    long long n = (long long)nx * ny * nz;
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int i = (int)(p % nx);
    int j = (int)((p / nx) % ny);
    int l = (int)(p / ((long long)nx * ny));
    const int px = nx + 2 * halo, py = ny + 2 * halo;
    auto at = [&](int di, int dj, int dl) -> double {
        return k2h[((long long)(l + halo + dl) * py + (j + halo + dj)) * px + (i + halo + di)];
    };
    double c = at(0, 0, 0);
    if (!isfinite(c)) atomicOr(bad, 1);
    k2[p] = c;
    if (order != 6) return;
    double g[3], lap = 0.0;
    for (int a = 0; a < 3; ++a) {
        int dx = (a == 0), dy = (a == 1), dz = (a == 2);
        double p1 = at(dx, dy, dz), m1 = at(-dx, -dy, -dz), p2 = at(2 * dx, 2 * dy, 2 * dz), m2 = at(-2 * dx, -2 * dy, -2 * dz);
        if (!isfinite(p1) || !isfinite(m1) || !isfinite(p2) || !isfinite(m2)) atomicOr(bad, 1);
        g[a] = (-p2 + 8.0 * p1 - 8.0 * m1 + m2) / (12.0 * h);
        lap += (-p2 + 16.0 * p1 - 30.0 * c + 16.0 * m1 - m2) / (12.0 * h * h);
    }
    double h2 = h * h;
    double dg = -64.0 / (15.0 * h2) + 14.0 / 15.0 * c + h2 / 20.0 * (lap - c * c);
    fld[p] = make_double4(dg, h * g[0] / 120.0, h * g[1] / 120.0, h * g[2] / 120.0);
}

// complex k^2: the same differences on complex samples, real and imaginary parts stored separately
__global__ void k_derived_c(const double2 *__restrict__ k2h, int halo, double *__restrict__ k2,
                            double *__restrict__ k2i, double4 *__restrict__ fld, double4 *__restrict__ fldi, int nx,
                            int ny, int nz, int order, double h, int *__restrict__ bad) {
    long long n = (long long)nx * ny * nz;
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int i = (int)(p % nx);
    int j = (int)((p / nx) % ny);
    int l = (int)(p / ((long long)nx * ny));
    const int px = nx + 2 * halo, py = ny + 2 * halo;
    auto at = [&](int di, int dj, int dl) -> double2 {
        return k2h[((long long)(l + halo + dl) * py + (j + halo + dj)) * px + (i + halo + di)];
    };
    const double2 c = at(0, 0, 0);
    if (!isfinite(c.x) || !isfinite(c.y)) atomicOr(bad, 1);
    k2[p] = c.x;
    k2i[p] = c.y;
    if (order != 6) return;
    double2 g[3], lap = make_double2(0.0, 0.0);
    for (int a = 0; a < 3; ++a) {
        int dx = (a == 0), dy = (a == 1), dz = (a == 2);
        double2 p1 = at(dx, dy, dz), m1 = at(-dx, -dy, -dz), p2 = at(2 * dx, 2 * dy, 2 * dz), m2 = at(-2 * dx, -2 * dy, -2 * dz);
        if (!isfinite(p1.x + p1.y + m1.x + m1.y + p2.x + p2.y + m2.x + m2.y)) atomicOr(bad, 1);
        g[a] = cscale(cadd(csub(m2, p2), cscale(csub(p1, m1), 8.0)), 1.0 / (12.0 * h));
        lap = cadd(lap, cscale(cadd(cadd(cscale(cadd(p1, m1), 16.0), cscale(c, -30.0)), cscale(cadd(p2, m2), -1.0)),
                               1.0 / (12.0 * h * h)));
    }
    const double h2 = h * h;
    const double2 dg = cadd(make_double2(-64.0 / (15.0 * h2) + 14.0 / 15.0 * c.x, 14.0 / 15.0 * c.y),
                            cscale(csub(lap, cmul(c, c)), h2 / 20.0));
    fld[p] = make_double4(dg.x, h * g[0].x / 120.0, h * g[1].x / 120.0, h * g[2].x / 120.0);
    fldi[p] = make_double4(dg.y, h * g[0].y / 120.0, h * g[1].y / 120.0, h * g[2].y / 120.0);
}

// --------------------------------------------------------------------------- right-hand side
// k2i, fldi: imaginary parts for complex k^2 (NULL for real k^2)
__global__ void k_rhs(const double2 *__restrict__ f, const double *__restrict__ k2, const double4 *__restrict__ fld,
                      const double *__restrict__ k2i, const double4 *__restrict__ fldi, double2 *__restrict__ F,
                      int nx, int ny, int nz, int order, double hx, double hy, double hz) {
    long long n = (long long)nx * ny * nz;
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int i = (int)(p % nx);
    int j = (int)((p / nx) % ny);
    int l = (int)(p / ((long long)nx * ny));
    const int px = nx + 4, py = ny + 4;
    auto at = [&](int di, int dj, int dl) -> double2 {
        return f[((long long)(l + 2 + dl) * py + (j + 2 + dj)) * px + (i + 2 + di)];
    };
    double2 c = at(0, 0, 0);
    if (order == 2) { F[p] = c; return; }
    double hs[3] = {hx, hy, hz};
    double2 d2[3];
    for (int a = 0; a < 3; ++a) {
        int dx = (a == 0), dy = (a == 1), dz = (a == 2);
        double2 s = cadd(at(dx, dy, dz), at(-dx, -dy, -dz));
        d2[a] = cscale(csub(s, cscale(c, 2.0)), 1.0 / (hs[a] * hs[a]));
    }
    if (order == 4) {
        double2 out = c;
        for (int a = 0; a < 3; ++a) out = cfma(hs[a] * hs[a] / 12.0, d2[a], out);
        F[p] = out;
        return;
    }
    // order 6, uniform h: f + h^2/12 Lap_h f - h^4/240 sum delta^4 f + h^4/90 P_h f - h^2/20 k^2 f
    //                    + h^4/60 sum (k^2)_nu delta_nu f      (the last uses (k^2)_nu = 120 g_nu / h)
    double h = hx, h2 = h * h;
    double2 out = c;
    out = cfma(h2 / 12.0, cadd(cadd(d2[0], d2[1]), d2[2]), out);
    const double4 fl = fld[p];
    const double4 fli = fldi ? fldi[p] : make_double4(0, 0, 0, 0);
    const double2 gg[3] = {make_double2(fl.y, fli.y), make_double2(fl.z, fli.z), make_double2(fl.w, fli.w)};
    for (int a = 0; a < 3; ++a) {
        int dx = (a == 0), dy = (a == 1), dz = (a == 2);
        double2 p1 = at(dx, dy, dz), m1 = at(-dx, -dy, -dz);
        double2 p2 = at(2 * dx, 2 * dy, 2 * dz), m2 = at(-2 * dx, -2 * dy, -2 * dz);
        double2 d4 = cadd(cadd(cadd(p2, m2), cscale(cadd(p1, m1), -4.0)), cscale(c, 6.0));
        out = cfma(-1.0 / 240.0, d4, out);                       // h^4/240 * delta^4 f (delta^4 carries 1/h^4)
        double2 d1 = csub(p1, m1);                               // 2 h delta f
        out = cadd(out, cscale(cmul(gg[a], d1), h2));            // h^4/60 * (120 g/h) * d1/(2h) = h^2 g d1
    }
    const int pairs[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int q = 0; q < 3; ++q) {
        double2 acc = make_double2(0.0, 0.0);
        for (int sa = -1; sa <= 1; ++sa)
            for (int sb = -1; sb <= 1; ++sb) {
                int d[3] = {0, 0, 0};
                d[pairs[q][0]] += sa;
                d[pairs[q][1]] += sb;
                double w = (sa == 0 ? -2.0 : 1.0) * (sb == 0 ? -2.0 : 1.0);
                acc = cfma(w, at(d[0], d[1], d[2]), acc);
            }
        out = cfma(1.0 / 90.0, acc, out);                        // h^4/90 * P_h f (P_h carries 1/h^4)
    }
    const double2 kk = make_double2(k2[p], k2i ? k2i[p] : 0.0);
    out = csub(out, cscale(cmul(kk, c), h2 / 20.0));
    F[p] = out;
}

template <int ORDER, bool RESID, typename XT, bool KC>
__global__ __launch_bounds__(NT) void k_matvec(const XT *__restrict__ x, const double *__restrict__ k2,
                                                 const double4 *__restrict__ fld, const double2 *__restrict__ F,
                                                 double2 *__restrict__ y, StencilParams p) {
    matvec_tile<ORDER, RESID, XT, KC>(x, k2, fld, F, y, p, blockIdx.x);
}

template <typename XT, bool KC>
hipError_t launch_matvec_k(const StencilParams &p, const XT *x, const double *k2, const double4 *fld,
                           const double2 *F, double2 *y, hipStream_t s) {
    int T = p.tiles_x * p.tiles_y * p.zchunks;
    int grid = 8 * ((T + 7) / 8);
    dim3 blk(64, TY);
    if (p.order == 6) {
        if (F) hipLaunchKernelGGL((k_matvec<6, true, XT, KC>), dim3(grid), blk, 0, s, x, k2, fld, F, y, p);
        else hipLaunchKernelGGL((k_matvec<6, false, XT, KC>), dim3(grid), blk, 0, s, x, k2, fld, F, y, p);
    } else if (p.order == 4) {
        if (F) hipLaunchKernelGGL((k_matvec<4, true, XT, KC>), dim3(grid), blk, 0, s, x, k2, fld, F, y, p);
        else hipLaunchKernelGGL((k_matvec<4, false, XT, KC>), dim3(grid), blk, 0, s, x, k2, fld, F, y, p);
    } else {
        if (F) hipLaunchKernelGGL((k_matvec<2, true, XT, KC>), dim3(grid), blk, 0, s, x, k2, fld, F, y, p);
        else hipLaunchKernelGGL((k_matvec<2, false, XT, KC>), dim3(grid), blk, 0, s, x, k2, fld, F, y, p);
    }
    return hipGetLastError();
}

template <typename XT>
hipError_t launch_matvec_t(const StencilParams &p, const XT *x, const double *k2, const double4 *fld,
                           const double2 *F, double2 *y, hipStream_t s) {
    if (p.k2i) return launch_matvec_k<XT, true>(p, x, k2, fld, F, y, s);
    return launch_matvec_k<XT, false>(p, x, k2, fld, F, y, s);
}

}  // namespace

hipError_t launch_derived_fields(const double *k2_halo, int halo, double *k2, double4 *fld, const StencilParams &p,
                                 double h, hipStream_t s) {
    long long n = (long long)p.nx * p.ny * p.nz;
    int *bad = nullptr;
    hipError_t e = hipMalloc(&bad, sizeof(int));
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(bad, 0, sizeof(int), s);
    if (e != hipSuccess) { hipFree(bad); return e; }
    int blocks = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_derived, dim3(blocks), dim3(256), 0, s, k2_halo, halo, k2, fld, p.nx, p.ny, p.nz, p.order, h,
                       bad);
    e = hipGetLastError();
    int hbad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(bad);
    if (e != hipSuccess) return e;
    return hbad ? hipErrorInvalidValue : hipSuccess;
}

hipError_t launch_derived_fields_c(const double2 *k2_halo, int halo, double *k2, double *k2i, double4 *fld,
                                   double4 *fldi, const StencilParams &p, double h, hipStream_t s) {
    long long n = (long long)p.nx * p.ny * p.nz;
    int *bad = nullptr;
    hipError_t e = hipMalloc(&bad, sizeof(int));
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(bad, 0, sizeof(int), s);
    if (e != hipSuccess) { hipFree(bad); return e; }
    int blocks = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_derived_c, dim3(blocks), dim3(256), 0, s, k2_halo, halo, k2, k2i, fld, fldi, p.nx, p.ny, p.nz,
                       p.order, h, bad);
    e = hipGetLastError();
    int hbad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(bad);
    if (e != hipSuccess) return e;
    return hbad ? hipErrorInvalidValue : hipSuccess;
}

hipError_t launch_matvec(const StencilParams &p, const double2 *x, const double *k2, const double4 *fld,
                         const double2 *F, double2 *y, hipStream_t s) {
    return launch_matvec_t<double2>(p, x, k2, fld, F, y, s);
}

hipError_t launch_matvec(const StencilParams &p, const float2 *x, const double *k2, const double4 *fld,
                         const double2 *F, double2 *y, hipStream_t s) {
    return launch_matvec_t<float2>(p, x, k2, fld, F, y, s);
}

hipError_t launch_rhs(const StencilParams &p, const double2 *f_halo, const double *k2, const double4 *fld,
                      double h3[3], double2 *F, hipStream_t s) {
    long long n = (long long)p.nx * p.ny * p.nz;
    int blocks = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_rhs, dim3(blocks), dim3(256), 0, s, f_halo, k2, fld, p.k2i, p.fldi, F, p.nx, p.ny, p.nz,
                       p.order, h3[0], h3[1], h3[2]);
    return hipGetLastError();
}

}  // namespace helm
