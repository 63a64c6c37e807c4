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
template <typename CT> __device__ __forceinline__ CT crecip(CT a) {
    auto s = a.x * a.x + a.y * a.y;
    CT r;
    r.x = a.x / s;
    r.y = -a.y / s;
    return r;
}

constexpr int UNR = 8;

// Thomas elimination of one z-line (i, j) = (line % nx, line / nx).
template <typename T>
__device__ __forceinline__ void tridiag_line(const typename c2<T>::t *in, typename c2<T>::t *r,
                                             typename c2<T>::t *__restrict__ cp, const double2 *__restrict__ dx,
                                             const double2 *__restrict__ dy, int nx, int ny, int nz, double ax,
                                             double ay, double c0, double2 gz, double scale, long long line) {
    typedef typename c2<T>::t CT;
    const long long lines = (long long)nx * ny;
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
}  // namespace helm
