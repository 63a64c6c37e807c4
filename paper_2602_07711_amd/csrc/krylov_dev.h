// Device code of the Krylov block inner products, shared by the single-problem and the grouped kernels.
#pragma once
#include "helm_internal.h"

namespace helm {
namespace {

// Streaming loads of Krylov vectors: each vector is read once per pass, so the loads are marked non-temporal
// (measured at 256^3: the block inner products and the linear combination run 9-10 % faster than with
// ordinary loads).
typedef double v2d_nt __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_stream(const double2 *p) {
    const v2d_nt v = __builtin_nontemporal_load(reinterpret_cast<const v2d_nt *>(p));
    return make_double2(v.x, v.y);
}
// a complex64 basis vector (the Z basis of FGMRES with the FP32 preconditioner), widened exactly
typedef float v2f_nt __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_stream_wide(const float2 *p) {
    const v2f_nt v = __builtin_nontemporal_load(reinterpret_cast<const v2f_nt *>(p));
    return make_double2((double)v.x, (double)v.y);
}

constexpr int DOT_EPT = 16;                // elements per thread (8: 0.35 ms slower per 256^3 solve; 32: spills)
constexpr int DOT_CHUNK = 256 * DOT_EPT;   // elements per block
constexpr int MAXV = 260;                  // up to m + 2 outputs

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Partial sums of V_i^H w (i < nv) and ||w||^2 over chunk `lb` (DOT_CHUNK elements), written to
// part[lb * bstride + t * tstride] (t = 0..nv). Every thread of the block must call it.
__device__ __forceinline__ void dots_chunk(const double2 *__restrict__ V, long long ldv, int nv,
                                           const double2 *__restrict__ w, long long n, double2 *__restrict__ part,
                                           long long lb, long long bstride = -1, long long tstride = 1) {
    if (bstride < 0) bstride = nv + 1;
    __shared__ double2 red[4][MAXV];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long base = lb * DOT_CHUNK + tid;
    double2 wr[DOT_EPT];
    double ww = 0.0;
#pragma unroll
    for (int e = 0; e < DOT_EPT; ++e) {
        long long idx = base + (long long)e * 256;
        wr[e] = idx < n ? ld_stream(w + idx) : make_double2(0.0, 0.0);
        ww += wr[e].x * wr[e].x + wr[e].y * wr[e].y;
    }
    // four vectors per round: their loads and the eight reduction chains overlap
    int i = 0;
    for (; i + 4 <= nv; i += 4) {
        double re[4] = {0.0, 0.0, 0.0, 0.0}, im[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double2 *vi = V + (long long)(i + q) * ldv;
#pragma unroll
            for (int e = 0; e < DOT_EPT; ++e) {
                long long idx = base + (long long)e * 256;
                double2 v = idx < n ? ld_stream(vi + idx) : make_double2(0.0, 0.0);
                re[q] += v.x * wr[e].x + v.y * wr[e].y;   // conj(v) * w
                im[q] += v.x * wr[e].y - v.y * wr[e].x;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                re[q] += __shfl_xor(re[q], off, 64);
                im[q] += __shfl_xor(im[q], off, 64);
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) red[wave][i + q] = make_double2(re[q], im[q]);
        }
    }
    for (; i < nv; ++i) {
        const double2 *vi = V + (long long)i * ldv;
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int e = 0; e < DOT_EPT; ++e) {
            long long idx = base + (long long)e * 256;
            double2 v = idx < n ? ld_stream(vi + idx) : make_double2(0.0, 0.0);
            re += v.x * wr[e].x + v.y * wr[e].y;
            im += v.x * wr[e].y - v.y * wr[e].x;
        }
        re = wave_sum(re);
        im = wave_sum(im);
        if (lane == 0) red[wave][i] = make_double2(re, im);
    }
    ww = wave_sum(ww);
    if (lane == 0) red[wave][nv] = make_double2(ww, 0.0);
    __syncthreads();
    for (int t = tid; t <= nv; t += 256) {
        double2 s = red[0][t];
        for (int q = 1; q < 4; ++q) { s.x += red[q][t].x; s.y += red[q][t].y; }
        part[lb * bstride + t * tstride] = s;
    }
}

}  // namespace
}  // namespace helm
