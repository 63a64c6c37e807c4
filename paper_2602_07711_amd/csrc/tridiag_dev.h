// Device code of the z-tridiagonal solves, shared by the single-problem and the grouped (batched) kernels.
#pragma once
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
// 1/a with one reciprocal of |a|^2: correctly rounded division in FP64, the hardware reciprocal (about 1 ulp) in
// FP32, whose result the z-solve only needs to FP32 accuracy
__device__ __forceinline__ double2 crecip(double2 a) {
    const double is = 1.0 / (a.x * a.x + a.y * a.y);
    return make_double2(a.x * is, -a.y * is);
}
__device__ __forceinline__ float2 crecip(float2 a) {
    const float is = __builtin_amdgcn_rcpf(a.x * a.x + a.y * a.y);
    return make_float2(a.x * is, -a.y * is);
}

constexpr int TL = 8;    // rows per chunk of the partitioned z-solve

// Prefix composition of the chunks' affine maps x -> A x + B along a line (Kogge-Stone over the chunk index k,
// log2(P) rounds of the whole block): on return (a, b) of chunk k compose the maps of chunks k-span+1..k in the
// direction `dir` (+1: from chunk 0 upwards; -1: from chunk P-1 downwards). sA, sB: [P][LX] in LDS.
template <typename T, typename CT>
__device__ __forceinline__ void tri_scan(CT &a, CT &b, CT *sA, CT *sB, int k, int li, int P, int LX, int dir) {
    sA[k * LX + li] = a;
    sB[k * LX + li] = b;
    __syncthreads();
    for (int d = 1; d < P; d <<= 1) {
        const int src = k - dir * d;
        const bool act = k < P && src >= 0 && src < P;
        CT pa = mk<T, CT>(1, 0), pb = mk<T, CT>(0, 0);
        if (act) { pa = sA[src * LX + li]; pb = sB[src * LX + li]; }
        __syncthreads();
        if (act) {
            const CT nb = cm(a, pb);                 // x -> a (pa x + pb) + b
            b = mk<T, CT>(nb.x + b.x, nb.y + b.y);
            a = cm(a, pa);
            sA[k * LX + li] = a;
            sB[k * LX + li] = b;
        }
        __syncthreads();
    }
}

// One block of the partitioned z-solve: LX consecutive lines starting at line blk * LX, P chunks of TL rows per
// line (threads with chunk index >= P, present when the block is shaped for a larger problem, hold no rows but
// take part in every barrier). smraw: 2 * Pb * LX complex values, Pb = blockDim.x / LX. PT: element type of the
// pivot table (complex128 for the FP64 solve, complex64 for the FP32 one, which rounds the pivot to FP32 anyway).
template <typename T, typename PT>
__device__ __forceinline__ void tri_chunk_block(const typename c2<T>::t *in, typename c2<T>::t *out,
                                                const PT *__restrict__ piv, const double2 *__restrict__ dx,
                                                const double2 *__restrict__ dy, int nx, int ny, int nz, int P, int LX,
                                                double ax, double ay, double c0, double2 gz, double scale,
                                                long long blk, unsigned char *smraw, double zi = 1.0) {
    typedef typename c2<T>::t CT;
    CT *sA = reinterpret_cast<CT *>(smraw);                // [Pb][LX]
    CT *sB = sA + (blockDim.x / LX) * LX;
    const int t = threadIdx.x, li = t % LX, k = t / LX;
    const long long lines = (long long)nx * ny;
    const long long line = blk * LX + li;
    const bool lin = line < lines && k < P;
    const int s = k * TL;
    const int nrow = lin ? (nz - s < TL ? nz - s : TL) : 0;
    CT b = mk<T, CT>(0, 0);
    if (lin) {
        const double2 ex = dx[(int)(line % nx)], ey = dy[(int)(line / nx)];
        b = mk<T, CT>((T)(ax * ex.x + ay * ey.x + c0), (T)(ax * ex.y + ay * ey.y));
    }
    const CT g = mk<T, CT>((T)gz.x, (T)gz.y);
    const T sc = (T)scale;
    CT v[TL], inv[TL];
#pragma unroll
    for (int r = 0; r < TL; ++r)
        if (r < nrow) v[r] = in[line + (long long)(s + r) * lines];
    // a corner off-diagonal zeta (collocated closure): the first and last equations are divided by zeta
    // (zi = 1/zeta), which restores unit off-diagonals; end diagonal (gamma + b)/zeta, end right-hand side y/zeta
    const T zt = (T)zi;
#pragma unroll
    for (int r = 0; r < TL; ++r)
        if (r < nrow && (s + r == 0 || s + r == nz - 1)) { v[r].x *= zt; v[r].y *= zt; }
    // pivots of this chunk, restarted from the pivot entering it
    CT ip = mk<T, CT>(0, 0);
    if (lin && k > 0) {
        const PT q = piv[(long long)k * lines + line];
        ip = mk<T, CT>((T)q.x, (T)q.y);
    }
#pragma unroll
    for (int r = 0; r < TL; ++r)
        if (r < nrow) {
            const int l = s + r;
            CT d = b;
            if (l == 0 || l == nz - 1) { d.x = (d.x + g.x) * zt; d.y = (d.y + g.y) * zt; }
            if (l > 0) { d.x -= ip.x; d.y -= ip.y; }
            ip = crecip(d);
            inv[r] = ip;
        }
    // forward sweep with d'_{s-1} = 0: d'_e = A d'_{s-1} + B with A = prod(-inv)
    CT dp = mk<T, CT>(0, 0), A = mk<T, CT>(1, 0);
#pragma unroll
    for (int r = 0; r < TL; ++r)
        if (r < nrow) {
            dp = cm(mk<T, CT>(sc * v[r].x - dp.x, sc * v[r].y - dp.y), inv[r]);
            v[r] = dp;
            const CT na = cm(inv[r], A);
            A = mk<T, CT>(-na.x, -na.y);
        }
    // incoming d'_{s-1}: the composition of the maps of chunks 0..k-1 applied to 0
    CT fa = A, fb = dp;
    tri_scan<T, CT>(fa, fb, sA, sB, k, li, P, LX, 1);
    CT fix = (k > 0 && k < P) ? sB[(k - 1) * LX + li] : mk<T, CT>(0, 0);
#pragma unroll
    for (int r = 0; r < TL; ++r)
        if (r < nrow) {
            const CT m = cm(inv[r], fix);
            fix = mk<T, CT>(-m.x, -m.y);
            v[r].x += fix.x;
            v[r].y += fix.y;
        }
    // backward sweep with u_{e+1} = 0: u_s = A u_{e+1} + D
    CT un = mk<T, CT>(0, 0);
#pragma unroll
    for (int r = TL - 1; r >= 0; --r)
        if (r < nrow) {
            const CT m = cm(inv[r], un);
            un = mk<T, CT>(v[r].x - m.x, v[r].y - m.y);
            v[r] = un;
        }
    // incoming u_{e+1}: the composition of the maps of chunks P-1..k+1 applied to 0
    __syncthreads();                 // everyone has read its incoming d' before sA, sB are reused
    CT ba = A, bb = un;
    tri_scan<T, CT>(ba, bb, sA, sB, k, li, P, LX, -1);
    fix = (k + 1 < P) ? sB[(k + 1) * LX + li] : mk<T, CT>(0, 0);
#pragma unroll
    for (int r = TL - 1; r >= 0; --r)
        if (r < nrow) {
            const CT m = cm(inv[r], fix);
            fix = mk<T, CT>(-m.x, -m.y);
            v[r].x += fix.x;
            v[r].y += fix.y;
        }
#pragma unroll
    for (int r = 0; r < TL; ++r)
        if (r < nrow) out[line + (long long)(s + r) * lines] = v[r];
}


}  // namespace
}  // namespace helm
