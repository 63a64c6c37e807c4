// Krylov kernels of the (F)GMRES outer iteration: the block inner products V^H w together with ||w||^2 in
// one pass over the data (classical Gram-Schmidt with the norm taken from ||w||^2 - sum |h_i|^2), a fixed-
// order two-stage reduction (bitwise reproducible, no atomics), and the linear combination
// out = alpha * base + sum_i c_i V_i used for the orthogonalisation update, the end-of-cycle update
// x += Z y and the restart vector.
#include "krylov_dev.h"

namespace helm {

namespace {

// partials of output t are contiguous: part[t * gridDim.x + block], so the reduction reads them coalesced
__global__ __launch_bounds__(256) void k_dots(const double2 *__restrict__ V, long long ldv, int nv,
                                              const double2 *__restrict__ w, long long n, double2 *__restrict__ part) {
    dots_chunk(V, ldv, nv, w, n, part, blockIdx.x, 1, gridDim.x);
}

__global__ __launch_bounds__(256) void k_reduce(const double2 *__restrict__ part, int nblocks, int nout,
                                                double2 *__restrict__ out) {
    __shared__ double sr[256], si[256];
    const int t = blockIdx.x, tid = threadIdx.x;
    double re = 0.0, im = 0.0;
    for (int b = tid; b < nblocks; b += 256) {
        double2 v = part[(long long)t * nblocks + b];
        re += v.x;
        im += v.y;
    }
    sr[tid] = re;
    si[tid] = im;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) { sr[tid] += sr[tid + s]; si[tid] += si[tid + s]; }
        __syncthreads();
    }
    if (tid == 0) out[t] = make_double2(sr[0], si[0]);
}

constexpr int LC_MAX = 48;
struct LcCoef { double2 c[LC_MAX]; };
constexpr int LC_EPT = 4;   // elements per thread (independent loads in flight per vector)

__device__ __forceinline__ double2 wide(const double2 *p) { return ld_stream(p); }
__device__ __forceinline__ double2 wide(const float2 *p) { return ld_stream_wide(p); }

template <typename VT>
__global__ __launch_bounds__(256) void k_lincomb(double2 *out, const double2 *base, double2 alpha,
                                                 const VT *__restrict__ V, long long ldv, int nv, LcCoef co,
                                                 long long n) {
    const long long start = (long long)blockIdx.x * (256 * LC_EPT) + threadIdx.x;
    double2 acc[LC_EPT];
    bool ok[LC_EPT];
#pragma unroll
    for (int e = 0; e < LC_EPT; ++e) {
        const long long idx = start + (long long)e * 256;
        ok[e] = idx < n;
        acc[e] = make_double2(0.0, 0.0);
        if (base && ok[e]) {
            double2 b = ld_stream(base + idx);
            acc[e].x = alpha.x * b.x - alpha.y * b.y;
            acc[e].y = alpha.x * b.y + alpha.y * b.x;
        }
    }
    int i = 0;
    for (; i + 4 <= nv; i += 4) {            // four vectors per round: 16 loads in flight per thread
        double2 v[4][LC_EPT];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int e = 0; e < LC_EPT; ++e) {
                const long long idx = start + (long long)e * 256;
                v[q][e] = ok[e] ? wide(V + (long long)(i + q) * ldv + idx) : make_double2(0.0, 0.0);
            }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double2 c = co.c[i + q];
#pragma unroll
            for (int e = 0; e < LC_EPT; ++e) {
                acc[e].x += c.x * v[q][e].x - c.y * v[q][e].y;
                acc[e].y += c.x * v[q][e].y + c.y * v[q][e].x;
            }
        }
    }
    for (; i < nv; ++i) {
        const VT *vi = V + (long long)i * ldv;
        const double2 c = co.c[i];
        double2 v[LC_EPT];
#pragma unroll
        for (int e = 0; e < LC_EPT; ++e) {
            const long long idx = start + (long long)e * 256;
            v[e] = ok[e] ? wide(vi + idx) : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int e = 0; e < LC_EPT; ++e) {
            acc[e].x += c.x * v[e].x - c.y * v[e].y;
            acc[e].y += c.x * v[e].y + c.y * v[e].x;
        }
    }
#pragma unroll
    for (int e = 0; e < LC_EPT; ++e) {
        const long long idx = start + (long long)e * 256;
        if (ok[e]) out[idx] = acc[e];
    }
}

// The orthogonalisation update of an Arnoldi step with its coefficients taken on the device from the reduced inner
// products red[0..nv-1] = V_i^H w and red[nv] = ||w||^2: eta^2 = ||w||^2 - sum |h_i|^2 and, when no severe
// cancellation happened (eta^2 > reorth ||w||^2), w <- -(w - V h) / eta; otherwise w <- -(w - V h) unscaled, for
// the host's second Gram-Schmidt pass. Every block recomputes the (uniform) coefficients, so no host round trip sits between the
// inner products and the update.
__global__ __launch_bounds__(256) void k_lincomb_cgs(double2 *w, const double2 *__restrict__ V, long long ldv, int nv,
                                                     const double2 *__restrict__ red, long long n, double reorth) {
    double hh = 0.0;
    for (int i = 0; i < nv; ++i) {
        const double2 r = red[i];
        hh = fma(r.x, r.x, hh);
        hh = fma(r.y, r.y, hh);
    }
    const double ww = red[nv].x, eta2 = ww - hh;
    const double inv = eta2 > reorth * ww ? 1.0 / sqrt(eta2) : 1.0;
    const long long start = (long long)blockIdx.x * (256 * LC_EPT) + threadIdx.x;
    double2 acc[LC_EPT];
    bool ok[LC_EPT];
#pragma unroll
    for (int e = 0; e < LC_EPT; ++e) {
        const long long idx = start + (long long)e * 256;
        ok[e] = idx < n;
        acc[e] = make_double2(0.0, 0.0);
        if (ok[e]) {
            const double2 b = ld_stream(w + idx);
            acc[e] = make_double2(-inv * b.x, -inv * b.y);
        }
    }
    int i = 0;
    for (; i + 4 <= nv; i += 4) {
        double2 v[4][LC_EPT];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int e = 0; e < LC_EPT; ++e) {
                const long long idx = start + (long long)e * 256;
                v[q][e] = ok[e] ? ld_stream(V + (long long)(i + q) * ldv + idx) : make_double2(0.0, 0.0);
            }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double2 c = make_double2(red[i + q].x * inv, red[i + q].y * inv);
#pragma unroll
            for (int e = 0; e < LC_EPT; ++e) {
                acc[e].x += c.x * v[q][e].x - c.y * v[q][e].y;
                acc[e].y += c.x * v[q][e].y + c.y * v[q][e].x;
            }
        }
    }
    for (; i < nv; ++i) {
        const double2 c = make_double2(red[i].x * inv, red[i].y * inv);
        double2 v[LC_EPT];
#pragma unroll
        for (int e = 0; e < LC_EPT; ++e) {
            const long long idx = start + (long long)e * 256;
            v[e] = ok[e] ? ld_stream(V + (long long)i * ldv + idx) : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int e = 0; e < LC_EPT; ++e) {
            acc[e].x += c.x * v[e].x - c.y * v[e].y;
            acc[e].y += c.x * v[e].y + c.y * v[e].x;
        }
    }
#pragma unroll
    for (int e = 0; e < LC_EPT; ++e) {
        const long long idx = start + (long long)e * 256;
        if (ok[e]) w[idx] = acc[e];
    }
}

__global__ void k_to_c64(const double2 *__restrict__ x, float2 *__restrict__ y, long long n) {
    long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx < n) y[idx] = make_float2((float)x[idx].x, (float)x[idx].y);
}

__global__ void k_zero(double2 *x, long long n) {
    long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx < n) x[idx] = make_double2(0.0, 0.0);
}

}  // namespace

int dots_blocks(long long n) { return (int)((n + DOT_CHUNK - 1) / DOT_CHUNK); }

hipError_t launch_dots(const double2 *V, long long ldv, int nv, const double2 *w, long long n, double2 *partials,
                       int nblocks, double2 *red, hipStream_t s) {
    if (nv + 1 > MAXV) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dots, dim3(nblocks), dim3(256), 0, s, V, ldv, nv, w, n, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce, dim3(nv + 1), dim3(256), 0, s, partials, nblocks, nv + 1, red);
    return hipGetLastError();
}

template <typename VT>
hipError_t lincomb_t(double2 *out, const double2 *base, double2 alpha, const VT *V, long long ldv, int nv,
                     const double2 *coef, long long n, hipStream_t s) {
    long long grid_ll = (n + 256 * LC_EPT - 1) / (256 * LC_EPT);
    int grid = (int)(grid_ll < 1 ? 1 : grid_ll);
    int done = 0;
    do {
        int cnt = nv - done < LC_MAX ? nv - done : LC_MAX;
        LcCoef co;
        for (int i = 0; i < cnt; ++i) co.c[i] = coef[done + i];
        const double2 *b = done == 0 ? base : out;
        double2 a = done == 0 ? alpha : make_double2(1.0, 0.0);
        hipLaunchKernelGGL(k_lincomb<VT>, dim3(grid), dim3(256), 0, s, out, b, a, V + (long long)done * ldv, ldv, cnt,
                           co, n);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        done += cnt;
    } while (done < nv);
    return hipSuccess;
}

hipError_t launch_lincomb(double2 *out, const double2 *base, double2 alpha, const double2 *V, long long ldv, int nv,
                          const double2 *coef, long long n, hipStream_t s) {
    return lincomb_t<double2>(out, base, alpha, V, ldv, nv, coef, n, s);
}

hipError_t launch_lincomb(double2 *out, const double2 *base, double2 alpha, const float2 *V, long long ldv, int nv,
                          const double2 *coef, long long n, hipStream_t s) {
    return lincomb_t<float2>(out, base, alpha, V, ldv, nv, coef, n, s);
}

hipError_t launch_lincomb_cgs(double2 *w, const double2 *V, long long ldv, int nv, const double2 *red, long long n,
                              double reorth, hipStream_t s) {
    long long grid_ll = (n + 256 * LC_EPT - 1) / (256 * LC_EPT);
    int grid = (int)(grid_ll < 1 ? 1 : grid_ll);
    hipLaunchKernelGGL(k_lincomb_cgs, dim3(grid), dim3(256), 0, s, w, V, ldv, nv, red, n, reorth);
    return hipGetLastError();
}

hipError_t launch_to_c64(const double2 *x, float2 *y, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_c64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double2 *x, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n);
    return hipGetLastError();
}

}  // namespace helm
