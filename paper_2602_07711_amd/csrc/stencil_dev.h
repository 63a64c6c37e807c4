// Device code of the compact-stencil matvec, shared by the single-problem and the grouped (batched) kernels.
#pragma once
#include "helm_internal.h"

namespace helm {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cfma(double s, double2 a, double2 acc) {
    return make_double2(fma(s, a.x, acc.x), fma(s, a.y, acc.y));
}

// --------------------------------------------------------------------------- matvec
constexpr int TX = 64;       // tile width along x (one wavefront row)
constexpr int TY = 8;        // tile height along y (each of the 4 thread rows computes 2 rows)
constexpr int LX = TX + 2;
constexpr int LY = TY + 2;

// One tile (64 x 8 nodes, one z-chunk) of y = A x (RESID: y = F - A x). `bid` is the block's tile slot; the
// tile order puts consecutive tiles on one XCD when blocks are dispatched round-robin over the 8 XCDs.
template <int ORDER, bool RESID>
__device__ __forceinline__ void matvec_tile(const double2 *__restrict__ x, const double *__restrict__ k2,
                                            const double4 *__restrict__ fld, const double2 *__restrict__ F,
                                            double2 *__restrict__ y, const StencilParams &p, int bid) {
    __shared__ double2 su[3][LY][LX];
    __shared__ double sk[3][LY][LX];

    const int T = p.tiles_x * p.tiles_y * p.zchunks;
    const int per = (T + 7) / 8;
    const int tile = (bid % 8) * per + bid / 8;   // consecutive tiles share an XCD (and its L2)
    if (tile >= T) return;
    const int tx_t = tile % p.tiles_x;
    const int ty_t = (tile / p.tiles_x) % p.tiles_y;
    const int tz_t = tile / (p.tiles_x * p.tiles_y);
    const int x0 = tx_t * TX, y0 = ty_t * TY;
    const int z0 = tz_t * p.zchunk;
    const int z1 = min(z0 + p.zchunk, p.nz);
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const long long plane = (long long)nx * ny;
    const int tid = threadIdx.y * 64 + threadIdx.x;

    auto load_plane = [&](int slot, int z) {
        double2 fz = make_double2(1.0, 0.0);
        int cz = z;
        if (z < 0) { cz = 0; fz = p.gz; }
        else if (z >= nz) { cz = nz - 1; fz = p.gz; }
        for (int e = tid; e < LX * LY; e += 256) {
            int lx = e % LX, ly = e / LX;
            int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
            double2 fac = fz;
            int cx = gx, cy = gy;
            if (gx < 0) { cx = 0; fac = cmul(fac, p.gx); }
            else if (gx >= nx) { cx = nx - 1; fac = cmul(fac, p.gx); }
            if (gy < 0) { cy = 0; fac = cmul(fac, p.gy); }
            else if (gy >= ny) { cy = ny - 1; fac = cmul(fac, p.gy); }
            long long idx = (long long)cz * plane + (long long)cy * nx + cx;
            su[slot][ly][lx] = cmul(fac, x[idx]);
            sk[slot][ly][lx] = k2[idx];
        }
    };

    load_plane(0, z0 - 1);
    load_plane(1, z0);
    const int lx = threadIdx.x + 1;
    for (int z = z0; z < z1; ++z) {
        const int t = z - z0;
        load_plane((t + 2) % 3, z + 1);
        __syncthreads();
        const int sl[3] = {t % 3, (t + 1) % 3, (t + 2) % 3};   // planes z-1, z, z+1
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int ly = threadIdx.y + 4 * r + 1;
            const int gxo = x0 + threadIdx.x, gyo = y0 + ly - 1;
            double2 u0 = su[sl[1]][ly][lx];
            double k0 = sk[sl[1]][ly][lx];
            double2 acc;
            if (ORDER == 6) {
                double2 S1 = make_double2(0, 0), S2 = S1, S3 = S1, SW1 = S1, SW2 = S1;
                double2 DU[3] = {S1, S1, S1}, DE[3] = {S1, S1, S1}, DW[3] = {S1, S1, S1};
#pragma unroll
                for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
                    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int nn = (dx != 0) + (dy != 0) + (dz != 0);
                            if (nn == 0) continue;
                            double2 u = su[sl[dz + 1]][ly + dy][lx + dx];
                            if (nn == 3) { S3 = cadd(S3, u); continue; }
                            double kk = sk[sl[dz + 1]][ly + dy][lx + dx];
                            double2 w = cscale(u, kk);
                            if (nn == 1) {
                                S1 = cadd(S1, u);
                                SW1 = cadd(SW1, w);
                                const int a = dx ? 0 : (dy ? 1 : 2);
                                const int s = dx + dy + dz;
                                DU[a] = cfma((double)s, u, DU[a]);
                                DW[a] = cfma((double)s, w, DW[a]);
                            } else {
                                S2 = cadd(S2, u);
                                SW2 = cadd(SW2, w);
                                if (dx) DE[0] = cfma((double)dx, u, DE[0]);
                                if (dy) DE[1] = cfma((double)dy, u, DE[1]);
                                if (dz) DE[2] = cfma((double)dz, u, DE[2]);
                            }
                        }
                if (gxo < nx && gyo < ny) {
                    long long pidx = (long long)z * plane + (long long)gyo * nx + gxo;
                    double4 fl = fld[pidx];
                    acc = cscale(u0, fl.x);
                    double2 lapc = cadd(cadd(S3, cscale(S2, 3.0)), cscale(S1, 14.0));
                    acc = cfma(p.c1, lapc, acc);
                    acc = cfma(1.0 / 90.0, csub(SW2, SW1), acc);
                    const double gg[3] = {fl.y, fl.z, fl.w};
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        double2 tnu = cadd(cadd(cscale(DU[a], 2.0), DE[a]), cscale(DW[a], p.h2));
                        acc = cfma(gg[a], tnu, acc);
                    }
                    if (RESID) acc = csub(F[pidx], acc);
                    y[pidx] = acc;
                }
            } else {
                acc = cscale(u0, p.c_center + p.w_center * k0);
                double2 fx = cadd(su[sl[1]][ly][lx - 1], su[sl[1]][ly][lx + 1]);
                double2 fy = cadd(su[sl[1]][ly - 1][lx], su[sl[1]][ly + 1][lx]);
                double2 fz = cadd(su[sl[0]][ly][lx], su[sl[2]][ly][lx]);
                acc = cfma(p.c_face[0], fx, acc);
                acc = cfma(p.c_face[1], fy, acc);
                acc = cfma(p.c_face[2], fz, acc);
                if (ORDER == 4) {
                    double2 wf = cadd(cadd(cscale(su[sl[1]][ly][lx - 1], sk[sl[1]][ly][lx - 1]),
                                           cscale(su[sl[1]][ly][lx + 1], sk[sl[1]][ly][lx + 1])),
                                      cadd(cscale(su[sl[1]][ly - 1][lx], sk[sl[1]][ly - 1][lx]),
                                           cscale(su[sl[1]][ly + 1][lx], sk[sl[1]][ly + 1][lx])));
                    wf = cadd(wf, cadd(cscale(su[sl[0]][ly][lx], sk[sl[0]][ly][lx]),
                                       cscale(su[sl[2]][ly][lx], sk[sl[2]][ly][lx])));
                    acc = cfma(p.w_face, wf, acc);
                    double2 exy = cadd(cadd(su[sl[1]][ly - 1][lx - 1], su[sl[1]][ly - 1][lx + 1]),
                                       cadd(su[sl[1]][ly + 1][lx - 1], su[sl[1]][ly + 1][lx + 1]));
                    double2 exz = cadd(cadd(su[sl[0]][ly][lx - 1], su[sl[0]][ly][lx + 1]),
                                       cadd(su[sl[2]][ly][lx - 1], su[sl[2]][ly][lx + 1]));
                    double2 eyz = cadd(cadd(su[sl[0]][ly - 1][lx], su[sl[0]][ly + 1][lx]),
                                       cadd(su[sl[2]][ly - 1][lx], su[sl[2]][ly + 1][lx]));
                    acc = cfma(p.c_edge[0], exy, acc);
                    acc = cfma(p.c_edge[1], exz, acc);
                    acc = cfma(p.c_edge[2], eyz, acc);
                }
                if (gxo < nx && gyo < ny) {
                    long long pidx = (long long)z * plane + (long long)gyo * nx + gxo;
                    if (RESID) acc = csub(F[pidx], acc);
                    y[pidx] = acc;
                }
            }
        }
        __syncthreads();
    }
}


}  // namespace
}  // namespace helm
