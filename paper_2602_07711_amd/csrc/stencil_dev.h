// Device code of the compact-stencil matvec, shared by the single-problem and the grouped (batched) kernels.
#pragma once
#include <type_traits>

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
// y = A x (RESID: y = F - A x) for the operators documented in k_stencil.hip, organised so that every node's
// value is read from LDS once per plane: a block of 64 x TY threads owns a 64 x TY column of outputs (one z-chunk)
// and streams planes p = z0-1 .. z1 through a
// double-buffered LDS tile (with the ghost rule applied on load) and scatters each plane's 3 x 3 in-plane
// neighbourhood into three register accumulators, for the outputs at p+1, p and p-1 (the plane is their lower,
// centre and upper plane). Output p-1 is complete after plane p. The plane's nine values are first reduced to
// sums that do not depend on the output (for the off-plane role: the z-face, the xz/yz edges, the corners and
// their k^2-weighted and signed forms; for the centre role: the x/y faces and xy edges), and each output adds
// them with its own coefficients (order 6: dg, g_x, g_y, g_z of that node).
// Plane loads are issued two planes ahead of their use (two register sets), the output coefficients and F one
// plane ahead, so one barrier per plane suffices. `bid` is the block's tile slot; the tile order puts
// consecutive tiles on one XCD when blocks are dispatched round-robin over the 8 XCDs.
constexpr int TX = 64;         // tile width along x (one wavefront row)
constexpr int TY = STENCIL_TY; // tile height along y, one thread row each (block 64 x TY)
constexpr int NT = TX * TY;     // threads per block
constexpr int LX = TX + 2;
constexpr int LY = TY + 2;
static_assert(2 * NT >= LX * LY, "two prefetch elements per thread cover the haloed tile");

// k^2-valued quantities: double for real k^2, double2 for complex k^2
__device__ __forceinline__ double2 kmul(double k, double2 u) { return cscale(u, k); }
__device__ __forceinline__ double2 kmul(double2 k, double2 u) { return cmul(k, u); }
__device__ __forceinline__ double2 kfma(double k, double2 u, double2 acc) { return cfma(k, u, acc); }
__device__ __forceinline__ double2 kfma(double2 k, double2 u, double2 acc) { return cadd(acc, cmul(k, u)); }
__device__ __forceinline__ double2 kfms(double k, double2 u, double2 acc) { return cfma(-k, u, acc); }        // acc - k u
__device__ __forceinline__ double2 kfms(double2 k, double2 u, double2 acc) { return csub(acc, cmul(k, u)); }
__device__ __forceinline__ double kaff(double a, double b, double k) { return a + b * k; }      // a + b k
__device__ __forceinline__ double2 kaff(double a, double b, double2 k) { return make_double2(a + b * k.x, b * k.y); }
struct F4C { double2 x, y, z, w; };          // complex order-6 field block (dg, g_x, g_y, g_z)

__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2((double)v.x, (double)v.y); }

// XT: the input's element type, complex128 or complex64 (the FP32 preconditioner's output, widened exactly).
// KC: complex k^2 (imaginary parts in p.k2i and p.fldi); the arithmetic is the same with complex k^2 factors.
// NR right-hand sides that share the operator (the first nr of them are computed; nr is uniform over the block):
// each plane of k^2 and each order-6 field block is read once for all of them, the inputs xs[r], Fs[r] and outputs
// ys[r] are per right-hand side.
template <int ORDER, bool RESID, typename XT, bool KC, int NR>
__device__ __forceinline__ void matvec_tile_n(const XT *const *xs, const double *__restrict__ k2,
                                               const double4 *__restrict__ fld, const double2 *const *Fs,
                                               double2 *const *ys, const StencilParams &p, int bid, int nr) {
    typedef typename std::conditional<KC, double2, double>::type KT;
    typedef typename std::conditional<KC, F4C, double4>::type FT;
    __shared__ double2 su[NR][2][LY][LX];
    __shared__ KT sk[2][LY][LX];
    const int T = p.tiles_x * p.tiles_y * p.zchunks;
    const int per = (T + 7) / 8;
    const int tile = (bid % 8) * per + bid / 8;   // consecutive tiles share an XCD (and its L2)
    if (tile >= T) return;
    const int x0 = (tile % p.tiles_x) * TX, y0 = ((tile / p.tiles_x) % p.tiles_y) * TY;
    const int z0 = (tile / (p.tiles_x * p.tiles_y)) * p.zchunk;
    const int z1 = min(z0 + p.zchunk, p.nz);
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const long long plane = (long long)nx * ny;
    const int tid = threadIdx.y * 64 + threadIdx.x;
    const int lx = threadIdx.x + 1, ly = threadIdx.y + 1;
    const int gxo = x0 + threadIdx.x, gyo = y0 + threadIdx.y;
    const bool valid = gxo < nx && gyo < ny;
    const long long col = valid ? (long long)gyo * nx + gxo : 0;

    // plane prefetch registers, two sets (planes alternate between them): elements tid and tid + NT of the
    // (LY x LX) tile; the in-plane part of the ghost factor is fixed per element, the z part per plane
    int offs[2];
    double2 fxy[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int e = tid + NT * q;
        const int ex = e % LX, ey = e / LX;
        const int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
        double2 fac = make_double2(1.0, 0.0);
        int cx = gx, cy = gy;
        if (gx < 0) { cx = 0; fac = cmul(fac, p.gx); }
        else if (gx >= nx) { cx = nx - 1; fac = cmul(fac, p.gx); }
        if (gy < 0) { cy = 0; fac = cmul(fac, p.gy); }
        else if (gy >= ny) { cy = ny - 1; fac = cmul(fac, p.gy); }
        offs[q] = cy * nx + cx;
        fxy[q] = fac;
    }
    // raw prefetched values: a complex64 input is widened when the plane is written to LDS, not when its load is
    // issued (that would make every plane wait for its own loads)
    XT ru[NR][2][2];
    KT rk[2][2];
    auto gload = [&](auto setc, int z) {
        constexpr int S = decltype(setc)::value;
        const int cz = z < 0 ? 0 : (z >= nz ? nz - 1 : z);
#pragma unroll
        for (int q = 0; q < 2; ++q)
            if (tid + NT * q < LX * LY) {
                const long long idx = (long long)cz * plane + offs[q];
#pragma unroll
                for (int r = 0; r < NR; ++r)
                    if (r < nr) ru[r][S][q] = xs[r][idx];
                if constexpr (KC) rk[S][q] = make_double2(k2[idx], p.k2i[idx]);
                else rk[S][q] = k2[idx];
            }
    };
    auto sstore = [&](auto setc, int z) {
        constexpr int S = decltype(setc)::value;
        const bool gh = z < 0 || z >= nz;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int e = tid + NT * q;
            if (e < LX * LY) {
                const double2 f = gh ? cmul(p.gz, fxy[q]) : fxy[q];
#pragma unroll
                for (int r = 0; r < NR; ++r)
                    if (r < nr) su[r][S][e / LX][e % LX] = cmul(f, to_d2(ru[r][S][q]));
                sk[S][e / LX][e % LX] = rk[S][q];
            }
        }
    };
    auto fload = [&](int z) -> FT {
        const bool in = ORDER == 6 && valid && z >= 0 && z < nz;
        if constexpr (KC) {
            const double4 a = in ? fld[(long long)z * plane + col] : make_double4(0, 0, 0, 0);
            const double4 b = in ? p.fldi[(long long)z * plane + col] : make_double4(0, 0, 0, 0);
            return F4C{make_double2(a.x, b.x), make_double2(a.y, b.y), make_double2(a.z, b.z), make_double2(a.w, b.w)};
        } else {
            return in ? fld[(long long)z * plane + col] : make_double4(0, 0, 0, 0);
        }
    };
    auto Fload = [&](int r, int z) -> double2 {
        return (RESID && r < nr && valid && z >= 0 && z < nz) ? Fs[r][(long long)z * plane + col]
                                                              : make_double2(0, 0);
    };

    // output coefficients for outputs p-1, p, p+1 (fm, f0, fp) and the prefetched p+2 (fn)
    FT fm = fload(-1), f0 = fload(z0 - 1), fp = fload(z0), fn;     // fload(-1) is the zero block
    double2 Fm[NR], F0[NR], Fn[NR], am[NR], a0[NR], ap[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        Fm[r] = make_double2(0, 0);
        F0[r] = Fload(r, z0 - 1);
        am[r] = a0[r] = ap[r] = make_double2(0, 0);
    }
    gload(std::integral_constant<int, 0>(), z0 - 1);
    gload(std::integral_constant<int, 1>(), z0);
    auto step = [&](auto setc, int pz) {
        constexpr int S = decltype(setc)::value;
        const int b = S;
        sstore(setc, pz);
        __syncthreads();
        if (pz + 2 <= z1) gload(setc, pz + 2);
        fn = fload(pz + 2);
#pragma unroll
        for (int r = 0; r < NR; ++r) Fn[r] = Fload(r, pz + 1);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (r >= nr) continue;
            // the plane's 3 x 3 neighbourhood of this column (names: x then y offset, m = -1, p = +1)
            const double2 uc = su[r][b][ly][lx], uxm = su[r][b][ly][lx - 1], uxp = su[r][b][ly][lx + 1];
            const double2 uym = su[r][b][ly - 1][lx], uyp = su[r][b][ly + 1][lx];
            const KT kc = sk[b][ly][lx];
            const double2 Ef = cadd(cadd(uxm, uxp), cadd(uym, uyp));          // in-plane face neighbours
            if (ORDER == 6) {
                const double2 umm = su[r][b][ly - 1][lx - 1], upm = su[r][b][ly - 1][lx + 1];
                const double2 ump = su[r][b][ly + 1][lx - 1], upp = su[r][b][ly + 1][lx + 1];
                const KT kxm = sk[b][ly][lx - 1], kxp = sk[b][ly][lx + 1];
                const KT kym = sk[b][ly - 1][lx], kyp = sk[b][ly + 1][lx];
                const KT kmm = sk[b][ly - 1][lx - 1], kpm = sk[b][ly - 1][lx + 1];
                const KT kmp = sk[b][ly + 1][lx - 1], kpp = sk[b][ly + 1][lx + 1];
                const double2 C = cadd(cadd(umm, upm), cadd(ump, upp));       // in-plane diagonal neighbours
                const double2 wxm = kmul(kxm, uxm), wxp = kmul(kxp, uxp);
                const double2 wym = kmul(kym, uym), wyp = kmul(kyp, uyp);
                const double2 Ew = cadd(cadd(wxm, wxp), cadd(wym, wyp));
                const double2 wc = kmul(kc, uc);
                const double2 Cw = cadd(cadd(kmul(kmm, umm), kmul(kpm, upm)), cadd(kmul(kmp, ump), kmul(kpp, upp)));
                const double2 Dx = csub(uxp, uxm), Dy = csub(uyp, uym);
                // role of an upper/lower plane (offsets (dx, dy, +-1)): centre = z-face, faces = xz/yz edges,
                // diagonals = corners
                double2 Piso = cfma(14.0 * p.c1, uc, cfma(3.0 * p.c1, Ef, cscale(C, p.c1)));
                Piso = cfma(1.0 / 90.0, csub(Ew, wc), Piso);
                const double2 Pz = cadd(cadd(cscale(uc, 2.0), cscale(wc, p.h2)), Ef);
                am[r] = cadd(am[r], kfma(fm.w, Pz, kfma(fm.y, Dx, kfma(fm.z, Dy, Piso))));
                ap[r] = cadd(ap[r], kfms(fp.w, Pz, kfma(fp.y, Dx, kfma(fp.z, Dy, Piso))));
                // role of the centre plane: centre, x/y faces, xy edges
                double2 Qiso = cfma(14.0 * p.c1, Ef, cscale(C, 3.0 * p.c1));
                Qiso = cfma(1.0 / 90.0, csub(Cw, Ew), Qiso);
                const double2 Qx = cadd(cfma(2.0, Dx, cscale(csub(wxp, wxm), p.h2)),
                                        csub(cadd(upm, upp), cadd(umm, ump)));
                const double2 Qy = cadd(cfma(2.0, Dy, cscale(csub(wyp, wym), p.h2)),
                                        csub(cadd(ump, upp), cadd(umm, upm)));
                a0[r] = cadd(a0[r], kfma(f0.x, uc, kfma(f0.y, Qx, kfma(f0.z, Qy, Qiso))));
            } else {
                const double2 Fx = cadd(uxm, uxp), Fy = cadd(uym, uyp);
                double2 P = cscale(uc, p.c_face[2]);
                double2 Q = cfma(p.c_face[0], Fx, cfma(p.c_face[1], Fy, kmul(kaff(p.c_center, p.w_center, kc), uc)));
                if (ORDER == 4) {
                    const KT kxm = sk[b][ly][lx - 1], kxp = sk[b][ly][lx + 1];
                    const KT kym = sk[b][ly - 1][lx], kyp = sk[b][ly + 1][lx];
                    const double2 C = cadd(cadd(su[r][b][ly - 1][lx - 1], su[r][b][ly - 1][lx + 1]),
                                           cadd(su[r][b][ly + 1][lx - 1], su[r][b][ly + 1][lx + 1]));
                    const double2 Ew = cadd(cadd(kmul(kxm, uxm), kmul(kxp, uxp)),
                                            cadd(kmul(kym, uym), kmul(kyp, uyp)));
                    P = kfma(kaff(0.0, p.w_face, kc), uc, cfma(p.c_edge[1], Fx, cfma(p.c_edge[2], Fy, P)));
                    Q = cfma(p.w_face, Ew, cfma(p.c_edge[0], C, Q));
                }
                am[r] = cadd(am[r], P);
                ap[r] = cadd(ap[r], P);
                a0[r] = cadd(a0[r], Q);
            }
        }
        const int zo = pz - 1;                        // complete after this plane
        if (zo >= z0 && valid) {
            const long long pidx = (long long)zo * plane + col;
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (r < nr) ys[r][pidx] = RESID ? csub(Fm[r], am[r]) : am[r];
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            am[r] = a0[r]; a0[r] = ap[r]; ap[r] = make_double2(0, 0);
            Fm[r] = F0[r]; F0[r] = Fn[r];
        }
        fm = f0; f0 = fp; fp = fn;
    };
    for (int pz = z0 - 1; pz <= z1; pz += 2) {
        step(std::integral_constant<int, 0>(), pz);
        if (pz + 1 <= z1) step(std::integral_constant<int, 1>(), pz + 1);
    }
}

// One right-hand side.
template <int ORDER, bool RESID, typename XT = double2, bool KC = false>
__device__ __forceinline__ void matvec_tile(const XT *__restrict__ x, const double *__restrict__ k2,
                                             const double4 *__restrict__ fld, const double2 *__restrict__ F,
                                             double2 *__restrict__ y, const StencilParams &p, int bid) {
    const XT *xs[1] = {x};
    const double2 *Fs[1] = {F};
    double2 *ys[1] = {y};
    matvec_tile_n<ORDER, RESID, XT, KC, 1>(xs, k2, fld, Fs, ys, p, bid, 1);
}

}  // namespace
}  // namespace helm
