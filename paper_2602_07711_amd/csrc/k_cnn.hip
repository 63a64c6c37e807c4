// Kernels of the learned warm start: a 3D encoder-decoder CNN trained and run on the GPU.
//
// MFMA operands are BF16 (v_mfma_f32_16x16x16bf16_1k) or FP32 (v_mfma_f32_16x16x4f32), accumulation FP32,
// activations stored FP32. Lane layout (checked on gfx950): A(row = lane%16, k = KL*(lane/16) + e),
// B(k = KL*(lane/16) + e, col = lane%16), accumulator register r = D(row = 4*(lane/16) + r, col = lane%16),
// KL = 4 (bf16) or 1 (f32).
//   * 27-tap layers: direct convolution from LDS tiles (k_conv_direct; the data gradient is the same kernel
//     with mirrored, transposed weights) and a direct weight-gradient kernel (k_wgrad_direct);
//   * the 1x1x1 head: an implicit GEMM out[co][v] = sum_ci W[co][ci] in[ci][v] (k_conv_fwd) and a reduction for
//     its weight gradient (k_wgrad_1x1).
// Also: bias add + ReLU in the epilogues, bias gradient, ReLU backward, 2x average pooling and nearest
// upsampling (both directions), MSE loss, Adam, the network input from the solver's arrays, and the trilinear
// or cubic prolongation of a coarse prediction to the solver's grid.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "helm_internal.h"

namespace helm {

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

struct bf16 { unsigned short u; };

__device__ __forceinline__ unsigned short f2bf(float f) {   // round to nearest even
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

template <typename T> struct MT;
template <> struct MT<float> {
    static constexpr int KL = 1;
    typedef float op;
    __device__ static float cvt(float f) { return f; }
    __device__ static v4f mma(op a, op b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <> struct MT<bf16> {
    static constexpr int KL = 4;
    typedef v4s op;
    __device__ static bf16 cvt(float f) { bf16 r; r.u = f2bf(f); return r; }
    __device__ static v4f mma(op a, op b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }
};

template <typename T> __device__ __forceinline__ typename MT<T>::op load_op(const T *p);
template <> __device__ __forceinline__ float load_op<float>(const float *p) { return *p; }
template <> __device__ __forceinline__ v4s load_op<bf16>(const bf16 *p) {
    v4s r;
    r[0] = (short)p[0].u; r[1] = (short)p[1].u; r[2] = (short)p[2].u; r[3] = (short)p[3].u;
    return r;
}

constexpr int CT = 64;   // voxels (or k columns) per workgroup
constexpr int KC = 32;   // k (or voxel) chunk staged in LDS per step

__device__ __forceinline__ void tap_off(int taps, int t, int &dz, int &dy, int &dx) {
    if (taps == 1) { dz = dy = dx = 0; return; }
    dz = t / 9 - 1;
    dy = (t / 3) % 3 - 1;
    dx = t % 3 - 1;
}

// forward / dgrad convolution (cubic volume S^3, zero padding, stride 1); out channels at out + co*V
template <typename T, int COP>
__global__ __launch_bounds__(256) void k_conv_fwd(const float *__restrict__ in, long long in_bs, int Ci, int S,
                                                  int taps, const T *__restrict__ wt, int Kp,
                                                  const float *__restrict__ bias, int Co, float *__restrict__ out,
                                                  long long out_bs, int relu) {
    constexpr int KL = MT<T>::KL;
    constexpr int FR = COP / 16;
    __shared__ __attribute__((aligned(16))) T sA[COP][KC + 4];
    __shared__ __attribute__((aligned(16))) T sB[CT][KC + 4];
    const int V = S * S * S;
    const int tiles = (V + CT - 1) / CT;
    const int b = (int)(blockIdx.x / tiles);
    const int v0 = (int)(blockIdx.x % tiles) * CT;
    const float *inb = in + (long long)b * in_bs;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // this thread stages voxel column `col` for k = kq, kq + 4, kq + 8, ... (all chunks in sequence)
    const int col = tid & 63, kq = tid >> 6;
    const int v = v0 + col;
    const bool vin = v < V;
    const int xw = v % S, yh = (v / S) % S, zd = v / (S * S);
    int ci = kq / taps, t = kq - (kq / taps) * taps;
    v4f acc[FR];
#pragma unroll
    for (int f = 0; f < FR; ++f) acc[f] = v4f{0, 0, 0, 0};
    for (int k0 = 0; k0 < Kp; k0 += KC) {
        __syncthreads();
        for (int e = tid; e < COP * KC; e += 256) {
            int r = e / KC, kk = e % KC;
            sA[r][kk] = wt[(long long)r * Kp + k0 + kk];
        }
#pragma unroll
        for (int j = 0; j < KC / 4; ++j) {
            float val = 0.f;
            if (vin && ci < Ci) {
                int dz = 0, dy = 0, dx = 0;
                if (taps == 27) { dz = t / 9 - 1; dy = (t / 3) % 3 - 1; dx = t % 3 - 1; }
                const int zz = zd + dz, yy = yh + dy, xx = xw + dx;
                if ((unsigned)zz < (unsigned)S && (unsigned)yy < (unsigned)S && (unsigned)xx < (unsigned)S)
                    val = inb[(long long)ci * V + (zz * S + yy) * S + xx];
            }
            sB[col][kq + 4 * j] = MT<T>::cvt(val);
            t += 4;
            while (t >= taps) { t -= taps; ++ci; }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KC; ks += 4 * KL) {
            const int kofs = ks + KL * (lane >> 4);
            typename MT<T>::op bf = load_op<T>(&sB[wave * 16 + (lane & 15)][kofs]);
#pragma unroll
            for (int f = 0; f < FR; ++f) {
                typename MT<T>::op af = load_op<T>(&sA[f * 16 + (lane & 15)][kofs]);
                acc[f] = MT<T>::mma(af, bf, acc[f]);
            }
        }
    }
    float *outb = out + (long long)b * out_bs;
    const int vo = v0 + wave * 16 + (lane & 15);
#pragma unroll
    for (int f = 0; f < FR; ++f)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int co = f * 16 + 4 * (lane >> 4) + r;
            if (co < Co && vo < V) {
                float y = acc[f][r] + (bias ? bias[co] : 0.f);
                if (relu) y = fmaxf(y, 0.f);
                outb[(long long)co * V + vo] = y;
            }
        }
}

// db[co] = sum_{b,v} g[b][co][v]: block (co, s) sums slice s of the B V voxels into part[co][s]; a second
// kernel adds the slices in order
constexpr int BG_SLICES = 64;
__global__ __launch_bounds__(256) void k_bias_part(const float *__restrict__ g, long long g_bs, int B, int V,
                                                   float *__restrict__ part) {
    __shared__ float sm[256];
    const int co = blockIdx.x / BG_SLICES, sl = blockIdx.x % BG_SLICES;
    const int NV = B * V;
    const int per = (NV + BG_SLICES - 1) / BG_SLICES;
    const int u0 = sl * per, u1 = u0 + per < NV ? u0 + per : NV;
    float s = 0.f;
    for (int u = u0 + threadIdx.x; u < u1; u += 256) {
        const int b = u / V;
        s += g[(long long)b * g_bs + (long long)co * V + (u - b * V)];
    }
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}
__global__ void k_bias_reduce(const float *__restrict__ part, int Co, float *__restrict__ db) {
    const int co = blockIdx.x * blockDim.x + threadIdx.x;
    if (co >= Co) return;
    float s = 0.f;
    for (int i = 0; i < BG_SLICES; ++i) s += part[co * BG_SLICES + i];
    db[co] = s;
}

// pack FP32 weights W[co][k] (k = ci*taps + tap) into the padded operand layout wt[COP][Kp];
// transpose = 1 builds the dgrad weights W'[ci][co*taps + (taps-1-tap)] from W (Co, Ci swapped)
template <typename T>
__global__ void k_pack_weights(const float *__restrict__ W, int Co, int Ci, int taps, int transpose, int COP, int Kp,
                               T *__restrict__ wt) {
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)COP * Kp) return;
    int r = (int)(i / Kp), k = (int)(i % Kp);
    float v = 0.f;
    if (!transpose) {
        if (r < Co && k < Ci * taps) v = W[(long long)r * Ci * taps + k];
    } else {   // r = ci (row of W'), k = co*taps + tap'
        if (r < Ci && k < Co * taps) {
            int co = k / taps, tp = k % taps;
            v = W[(long long)co * Ci * taps + (long long)r * taps + (taps - 1 - tp)];
        }
    }
    wt[i] = MT<T>::cvt(v);
}

__global__ void k_relu_bwd(float *__restrict__ g, long long g_bs, const float *__restrict__ y, long long y_bs,
                           long long per, int B) {
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= per * B) return;
    long long b = i / per, o = i % per;
    if (!(y[b * y_bs + o] > 0.f)) g[b * g_bs + o] = 0.f;
}

// 2x average pooling S -> S/2 over C channels; backward spreads g/8 to the 8 children (accumulate = add)
__global__ void k_pool_fwd(const float *__restrict__ in, long long in_bs, float *__restrict__ out, long long out_bs,
                           int C, int S, int B) {
    const int s2 = S / 2;
    const long long per = (long long)C * s2 * s2 * s2;
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= per * B) return;
    long long b = i / per, o = i % per;
    int c = (int)(o / ((long long)s2 * s2 * s2));
    long long r = o % ((long long)s2 * s2 * s2);
    int x = (int)(r % s2), y = (int)((r / s2) % s2), z = (int)(r / ((long long)s2 * s2));
    const float *p = in + b * in_bs + (long long)c * S * S * S;
    float s = 0.f;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) s += p[((long long)(2 * z + dz) * S + 2 * y + dy) * S + 2 * x + dx];
    out[b * out_bs + o] = 0.125f * s;
}
__global__ void k_pool_bwd(const float *__restrict__ gout, long long gout_bs, float *__restrict__ gin,
                           long long gin_bs, int C, int S, int B, int accumulate) {
    const int s2 = S / 2;
    const long long per = (long long)C * S * S * S;
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= per * B) return;
    long long b = i / per, o = i % per;
    int c = (int)(o / ((long long)S * S * S));
    long long r = o % ((long long)S * S * S);
    int x = (int)(r % S), y = (int)((r / S) % S), z = (int)(r / ((long long)S * S));
    float v = 0.125f * gout[b * gout_bs + (long long)c * s2 * s2 * s2 + ((long long)(z / 2) * s2 + y / 2) * s2 + x / 2];
    float *q = gin + b * gin_bs + o;
    *q = accumulate ? *q + v : v;
}

// nearest 2x upsampling S -> 2S; backward sums the 8 children
__global__ void k_up_fwd(const float *__restrict__ in, long long in_bs, float *__restrict__ out, long long out_bs,
                         int C, int S, int B) {
    const int S2 = 2 * S;
    const long long per = (long long)C * S2 * S2 * S2;
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= per * B) return;
    long long b = i / per, o = i % per;
    int c = (int)(o / ((long long)S2 * S2 * S2));
    long long r = o % ((long long)S2 * S2 * S2);
    int x = (int)(r % S2), y = (int)((r / S2) % S2), z = (int)(r / ((long long)S2 * S2));
    out[b * out_bs + o] = in[b * in_bs + (long long)c * S * S * S + ((long long)(z / 2) * S + y / 2) * S + x / 2];
}
__global__ void k_up_bwd(const float *__restrict__ gout, long long gout_bs, float *__restrict__ gin, long long gin_bs,
                         int C, int S, int B) {
    const int S2 = 2 * S;
    const long long per = (long long)C * S * S * S;
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= per * B) return;
    long long b = i / per, o = i % per;
    int c = (int)(o / ((long long)S * S * S));
    long long r = o % ((long long)S * S * S);
    int x = (int)(r % S), y = (int)((r / S) % S), z = (int)(r / ((long long)S * S));
    const float *p = gout + b * gout_bs + (long long)c * S2 * S2 * S2;
    float s = 0.f;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) s += p[((long long)(2 * z + dz) * S2 + 2 * y + dy) * S2 + 2 * x + dx];
    gin[b * gin_bs + o] = s;
}

// MSE: partial sums of (y - t)^2 per block and the gradient 2 (y - t) / N
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ y, const float *__restrict__ t, long long n,
                                             float *__restrict__ g, double *__restrict__ part) {
    __shared__ double sm[256];
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    double s = 0.0;
    if (i < n) {
        float d = y[i] - t[i];
        g[i] = 2.f * d / (float)n;
        s = (double)d * d;
    }
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}
__global__ __launch_bounds__(256) void k_sum_d(const double *__restrict__ part, int np, double *__restrict__ out,
                                               double scale) {
    __shared__ double sm[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) s += part[i];
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sm[0] * scale;
}

// Adam on the FP32 master parameters
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       long long n, float lr, float b1, float b2, float eps, float c1, float c2) {
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// trilinear interpolation of a coarse prediction (channels Re, Im on nodes (i+1)/(nc+1)) to the fine nodes
// (I+1)/(nf+1), times `scale`, written as complex128. Beyond the outermost coarse nodes the values follow the
// ghost rule of the scheme on the coarse grid, U(-1) = gamma U(0) and U(nc) = gamma U(nc-1) per axis (gamma = 0
// gives zero extension).
__global__ void k_prolong(const float *__restrict__ coarse, int nc, double scale, double gre, double gim,
                          double2 *__restrict__ fine, int nf) {
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    long long nfn = (long long)nf * nf * nf;
    if (i >= nfn) return;
    const int F[3] = {(int)(i % nf), (int)((i / nf) % nf), (int)(i / ((long long)nf * nf))};
    int i0[3];
    double w1[3];
    for (int a = 0; a < 3; ++a) {                          // coarse index coordinate (F+1)(nc+1)/(nf+1) - 1
        long long num = (long long)(F[a] + 1) * (nc + 1);
        long long q = num / (nf + 1);
        i0[a] = (int)q - 1;
        w1[a] = (double)(num - q * (nf + 1)) / (nf + 1);
    }
    const long long V = (long long)nc * nc * nc;
    double re = 0.0, im = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int d[3] = {dx, dy, dz};
                double w = 1.0, fr = 1.0, fi = 0.0;          // weight and ghost factor gamma^(#clamped axes)
                int idx[3];
                for (int a = 0; a < 3; ++a) {
                    w *= d[a] ? w1[a] : 1.0 - w1[a];
                    int c = i0[a] + d[a];
                    if (c < 0 || c >= nc) {
                        c = c < 0 ? 0 : nc - 1;
                        const double nr = fr * gre - fi * gim, ni = fr * gim + fi * gre;
                        fr = nr;
                        fi = ni;
                    }
                    idx[a] = c;
                }
                if (w == 0.0) continue;
                const long long o = ((long long)idx[2] * nc + idx[1]) * nc + idx[0];
                const double ur = coarse[o], ui = coarse[V + o];
                re += w * (fr * ur - fi * ui);
                im += w * (fr * ui + fi * ur);
            }
    fine[i] = make_double2(scale * re, scale * im);
}

// the same prolongation with Keys' cubic convolution (a = -1/2) per axis: coarse indices i0-1 .. i0+2 around
// the fine node; ghost indices -m and nc-1+m (m = 1, 2) fold onto the boundary node with factor gamma^m
__global__ void k_prolong3(const float *__restrict__ coarse, int nc, double scale, double gre, double gim,
                           double2 *__restrict__ fine, int nf) {
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    long long nfn = (long long)nf * nf * nf;
    if (i >= nfn) return;
    const int F[3] = {(int)(i % nf), (int)((i / nf) % nf), (int)(i / ((long long)nf * nf))};
    double w[3][4];
    int idx[3][4], pw[3][4];
    for (int a = 0; a < 3; ++a) {
        long long num = (long long)(F[a] + 1) * (nc + 1);
        long long q = num / (nf + 1);
        const int i0 = (int)q - 1;
        const double t = (double)(num - q * (nf + 1)) / (nf + 1), t2 = t * t, t3 = t2 * t;
        w[a][0] = -0.5 * t3 + t2 - 0.5 * t;
        w[a][1] = 1.5 * t3 - 2.5 * t2 + 1.0;
        w[a][2] = -1.5 * t3 + 2.0 * t2 + 0.5 * t;
        w[a][3] = 0.5 * t3 - 0.5 * t2;
        for (int k = 0; k < 4; ++k) {
            int c = i0 - 1 + k, m = 0;
            if (c < 0) { m = -c; c = 0; }
            else if (c >= nc) { m = c - nc + 1; c = nc - 1; }
            idx[a][k] = c;
            pw[a][k] = m;
        }
    }
    double gr[7], gi[7];                                   // gamma^0 .. gamma^6
    gr[0] = 1.0; gi[0] = 0.0;
    for (int m = 1; m < 7; ++m) { gr[m] = gr[m - 1] * gre - gi[m - 1] * gim; gi[m] = gr[m - 1] * gim + gi[m - 1] * gre; }
    const long long V = (long long)nc * nc * nc;
    double re = 0.0, im = 0.0;
    for (int kz = 0; kz < 4; ++kz)
        for (int ky = 0; ky < 4; ++ky)
            for (int kx = 0; kx < 4; ++kx) {
                const double wt = w[0][kx] * w[1][ky] * w[2][kz];
                if (wt == 0.0) continue;
                const int m = pw[0][kx] + pw[1][ky] + pw[2][kz];
                const long long o = ((long long)idx[2][kz] * nc + idx[1][ky]) * nc + idx[0][kx];
                const double ur = coarse[o], ui = coarse[V + o];
                re += wt * (gr[m] * ur - gi[m] * ui);
                im += wt * (gr[m] * ui + gi[m] * ur);
            }
    fine[i] = make_double2(scale * re, scale * im);
}


// Separable form of the cubic prolongation (the 3-D operator is the product of three 1-D ones, ghost factors
// included): pass a interpolates along one axis, from an array [ch][n2][n1][nin] (innermost axis interpolated) to
// [ch][n2][n1][nout] with the output axis rotated to the front: out[ch][nout][n2][n1]. Three passes (x, y, z)
// give [ch][z][y][x] again. Complex data as (re, im) doubles; the first pass reads the FP32 prediction.
template <typename TIN>
__global__ void k_prolong3_pass(const TIN *__restrict__ src, int ncplx_in, int nin, int n1, int n2, int nout,
                                double gre, double gim, double scale, double2 *__restrict__ dst) {
    const long long total = (long long)nout * n1 * n2;
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= total) return;
    // output index: [o][a2][a1] (o slowest) so writes are contiguous along a1
    const int a1 = (int)(e % n1), a2 = (int)((e / n1) % n2), o = (int)(e / ((long long)n1 * n2));
    const long long num = (long long)(o + 1) * (nin + 1);
    const long long q = num / (nout + 1);
    const int i0 = (int)q - 1;
    const double t = (double)(num - q * (nout + 1)) / (nout + 1), t2 = t * t, t3 = t2 * t;
    const double w[4] = {-0.5 * t3 + t2 - 0.5 * t, 1.5 * t3 - 2.5 * t2 + 1.0, -1.5 * t3 + 2.0 * t2 + 0.5 * t,
                         0.5 * t3 - 0.5 * t2};
    double re = 0.0, im = 0.0;
    for (int k = 0; k < 4; ++k) {
        if (w[k] == 0.0) continue;
        int c = i0 - 1 + k, m = 0;
        if (c < 0) { m = -c; c = 0; }
        else if (c >= nin) { m = c - nin + 1; c = nin - 1; }
        double fr = 1.0, fi = 0.0;                     // gamma^m
        for (int r = 0; r < m; ++r) { const double nr = fr * gre - fi * gim; fi = fr * gim + fi * gre; fr = nr; }
        const long long si = ((long long)a2 * n1 + a1) * nin + c;
        double ur, ui;
        if (ncplx_in) { const double2 z = ((const double2 *)src)[si]; ur = z.x; ui = z.y; }
        else { ur = (double)((const float *)src)[si]; ui = (double)((const float *)src)[(long long)n1 * n2 * nin + si]; }
        re += w[k] * (fr * ur - fi * ui);
        im += w[k] * (fr * ui + fi * ur);
    }
    dst[e] = make_double2(scale * re, scale * im);
}

// network input from the solver's arrays: node (i, j, l) of the S^3 grid sits at ((i, j, l) + 1)/(S+1) in the unit
// cube, which is fine-grid index coordinate (i+1)(nf+1)/(S+1) - 1 per axis; k^2 and Re f are interpolated
// trilinearly there (weights from integer arithmetic, so nested grids inject exactly). Channel 0 =
// cs (k^2/k0^2 - 1), channel 1 = fs Re f. Arrays carry `halo` >= 1 cells; the upper neighbour index can be nf
// (a halo cell) only with weight zero.
__global__ void k_features(const double *__restrict__ k2h, const double2 *__restrict__ fh, int halo, int nf, int S,
                           double inv_k0sq, double cs, double fs, float *__restrict__ x) {
    long long v = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long V = (long long)S * S * S;
    if (v >= V) return;
    const int c[3] = {(int)(v % S), (int)((v / S) % S), (int)(v / ((long long)S * S))};
    int i0[3];
    double w1[3];
    for (int a = 0; a < 3; ++a) {
        long long num = (long long)(c[a] + 1) * (nf + 1);
        i0[a] = (int)(num / (S + 1)) - 1;
        w1[a] = (double)(num % (S + 1)) / (S + 1);
    }
    const long long P = nf + 2 * halo;
    double k2 = 0.0, fr = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? w1[0] : 1.0 - w1[0]) * (dy ? w1[1] : 1.0 - w1[1]) * (dz ? w1[2] : 1.0 - w1[2]);
                if (w == 0.0) continue;
                long long o = ((long long)(i0[2] + dz + halo) * P + (i0[1] + dy + halo)) * P + (i0[0] + dx + halo);
                k2 += w * k2h[o];
                fr += w * fh[o].x;
            }
    x[v] = (float)(cs * (k2 * inv_k0sq - 1.0));
    x[V + v] = (float)(fs * fr);
}


// ---------------------------------------------------------------------------------------------- direct 3x3x3
// Direct convolution for the 27-tap layers: a workgroup owns an 8 x 8 x 4 output tile (one 8 x 8 plane per wave,
// four 16-voxel MFMA column blocks each) and all output channels (COP rows). Per chunk of 16 input channels the
// input tile with its one-voxel halo (10 x 10 x 6) is staged once in LDS, channel-last in the operand type, so the
// B fragment of tap (dz, dy, dx) is one LDS read at the shifted voxel. Weights are packed as
// wt[chunk][tap][COP][16] and read as A fragments straight from global memory (each 64-lane read is one
// contiguous 512 B block shared by every wave and workgroup).
constexpr int DT_X = 8, DT_Y = 8, DT_Z = 4;
constexpr int DH_X = DT_X + 2, DH_Y = DT_Y + 2, DH_Z = DT_Z + 2;
constexpr int DH_V = DH_X * DH_Y * DH_Z;
constexpr int DCC = 16;                    // input channels per chunk
constexpr int DPAD = 4;                    // LDS row padding (elements)

// Work split: a workgroup covers one tile, FR row blocks (16 output channels each) starting at row block rg*FR,
// and the input-channel chunks [ks*cpb, (ks+1)*cpb). With one K split (nsplit = 1) it applies bias and ReLU and
// writes the output; otherwise it writes FP32 partial sums part[ks][b][co][v] that k_conv_split_sum adds in order.
template <typename T, int FR>
__global__ __launch_bounds__(256) void k_conv_direct(const float *__restrict__ in, long long in_bs, int Ci, int S,
                                                     const T *__restrict__ wt, int COP, const float *__restrict__ bias,
                                                     int Co, float *__restrict__ out, long long out_bs, int relu,
                                                     int rowgroups, int nsplit, int cpb, float *__restrict__ part,
                                                     int B) {
    constexpr int KL = MT<T>::KL;
    __shared__ __attribute__((aligned(16))) T sIn[DH_V][DCC + DPAD];
    const int ntx = (S + DT_X - 1) / DT_X, nty = (S + DT_Y - 1) / DT_Y, ntz = (S + DT_Z - 1) / DT_Z;
    const int tiles = ntx * nty * ntz;
    int idx = blockIdx.x;
    const int ks = idx % nsplit;
    idx /= nsplit;
    const int rg = idx % rowgroups;
    idx /= rowgroups;
    const int t = idx % tiles, b = idx / tiles;
    const int x0 = (t % ntx) * DT_X, y0 = ((t / ntx) % nty) * DT_Y, z0 = (t / (ntx * nty)) * DT_Z;
    const int row0 = rg * FR * 16;
    const float *inb = in + (long long)b * in_bs;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int V = S * S * S;
    v4f acc[FR][4];
#pragma unroll
    for (int f = 0; f < FR; ++f)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[f][nb] = v4f{0, 0, 0, 0};
    const int nchunk = (Ci + DCC - 1) / DCC;
    const int c_lo = ks * cpb, c_hi = min(nchunk, c_lo + cpb);
    for (int ch = c_lo; ch < c_hi; ++ch) {
        __syncthreads();
        // the tile's loads are issued in groups of eight before their LDS stores, so they overlap
        constexpr int NIT = (DCC * DH_V + 255) / 256;
#pragma unroll 8
        for (int it = 0; it < NIT; ++it) {
            const int e = tid + it * 256;
            if (e < DCC * DH_V) {
                const int c = e / DH_V, v = e - c * DH_V;
                const int hx = v % DH_X, hy = (v / DH_X) % DH_Y, hz = v / (DH_X * DH_Y);
                const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
                const int ci = ch * DCC + c;
                float val = 0.f;
                if (ci < Ci && (unsigned)gx < (unsigned)S && (unsigned)gy < (unsigned)S && (unsigned)gz < (unsigned)S)
                    val = inb[(long long)ci * V + (gz * S + gy) * S + gx];
                sIn[v][c] = MT<T>::cvt(val);
            }
        }
        __syncthreads();
        const T *wc = wt + (long long)ch * 27 * COP * DCC;
        for (int tap = 0; tap < 27; ++tap) {
            const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
#pragma unroll
            for (int kk = 0; kk < DCC; kk += 4 * KL) {
                const int kofs = kk + KL * (lane >> 4);
                typename MT<T>::op af[FR];
#pragma unroll
                for (int f = 0; f < FR; ++f)
                    af[f] = load_op<T>(wc + ((long long)tap * COP + row0 + f * 16 + (lane & 15)) * DCC + kofs);
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) {
                    const int n = nb * 16 + (lane & 15);
                    const int hv = ((wave + dz) * DH_Y + (n / DT_X + dy)) * DH_X + (n % DT_X + dx);
                    const typename MT<T>::op bf = load_op<T>(&sIn[hv][kofs]);
#pragma unroll
                    for (int f = 0; f < FR; ++f) acc[f][nb] = MT<T>::mma(af[f], bf, acc[f][nb]);
                }
            }
        }
    }
    const int gz = z0 + wave;
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        const int n = nb * 16 + (lane & 15);
        const int gx = x0 + n % DT_X, gy = y0 + n / DT_X;
        const bool ok = gx < S && gy < S && gz < S;
        const long long vo = ((long long)gz * S + gy) * S + gx;
#pragma unroll
        for (int f = 0; f < FR; ++f)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = row0 + f * 16 + 4 * (lane >> 4) + r;
                if (!ok || co >= Co) continue;
                if (nsplit == 1) {
                    float y = acc[f][nb][r] + (bias ? bias[co] : 0.f);
                    if (relu) y = fmaxf(y, 0.f);
                    out[(long long)b * out_bs + (long long)co * V + vo] = y;
                } else {
                    part[(((long long)ks * B + b) * Co + co) * V + vo] = acc[f][nb][r];
                }
            }
    }
}

// out[b][co][v] = act(bias[co] + sum_ks part[ks][b][co][v]) in split order
__global__ void k_conv_split_sum(const float *__restrict__ part, int nsplit, int B, int Co, int V,
                                 const float *__restrict__ bias, int relu, float *__restrict__ out, long long out_bs) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long per = (long long)Co * V;
    if (i >= per * B) return;
    const int b = (int)(i / per);
    const long long o = i - (long long)b * per;
    const int co = (int)(o / V);
    float s = bias ? bias[co] : 0.f;
    for (int k = 0; k < nsplit; ++k) s += part[((long long)k * B + b) * per + o];
    if (relu) s = fmaxf(s, 0.f);
    out[(long long)b * out_bs + o] = s;
}

// direct-format weights wt[chunk][tap][COP][16] of a conv with Co outputs and Ci inputs; transpose = 1 takes
// them from a layer W[Ci][Co][27] with the tap mirrored (the data-gradient convolution of that layer)
template <typename T>
__global__ void k_pack_direct(const float *__restrict__ W, int Co, int Ci, int transpose, int COP, long long total,
                              T *__restrict__ wt) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= total) return;
    const int cc = (int)(e % DCC);
    long long r = e / DCC;
    const int o = (int)(r % COP);
    r /= COP;
    const int tap = (int)(r % 27);
    const int ch = (int)(r / 27);
    const int i = ch * DCC + cc;
    float v = 0.f;
    if (o < Co && i < Ci)
        v = transpose ? W[((long long)i * Co + o) * 27 + (26 - tap)] : W[((long long)o * Ci + i) * 27 + tap];
    wt[e] = MT<T>::cvt(v);
}


// Weight gradient of a 27-tap layer, dW[o][i][tap] = sum_{b,v} g[b][o][v] in[b][i][v + off(tap)]. A workgroup
// (input-channel chunk ch, tile group tg) loops over the tiles tg, tg + G, ... of all samples; per tile it stages
// g (COP rows x the tile's 256 voxels) and the chunk's input tile with halo in LDS. Wave w accumulates taps
// w, w+4, ... as GEMMs with M = output channels, N = the chunk's 16 channels and K = voxels (16 per step: two
// 8-voxel x-rows); the A fragment of a step is shared by the wave's taps. BF16 keeps the input tile in three
// copies shifted by dx = 0, 1, 2 so each lane's four consecutive voxels are one aligned 8-byte read.
// Partial sums per tile group: part[tg][o][i][tap] (o < Co, i < Ci), added in order by k_wgrad_direct_sum.
constexpr int WG_GPAD = 8;
template <typename T> struct WgLayout {
    static constexpr int NSH = MT<T>::KL == 4 ? 3 : 1;      // shifted copies of the input tile
    static constexpr int RW = MT<T>::KL == 4 ? DT_X : DH_X; // stored row width
};

template <typename T, int FR>
__global__ __launch_bounds__(256) void k_wgrad_direct(const float *__restrict__ g, long long g_bs, int Co,
                                                      const float *__restrict__ in, long long in_bs, int Ci, int S,
                                                      int B, int G, float *__restrict__ part) {
    constexpr int KL = MT<T>::KL;
    constexpr int COP = FR * 16;
    constexpr int NSH = WgLayout<T>::NSH, RW = WgLayout<T>::RW;
    constexpr int NT = 7;                                     // taps per wave (27 = 7 + 7 + 7 + 6)
    __shared__ __attribute__((aligned(16))) T sG[COP][DT_X * DT_Y * DT_Z + WG_GPAD];
    __shared__ __attribute__((aligned(16))) T sX[NSH][DCC][DH_Z][DH_Y][RW];
    const int ch = blockIdx.x / G, tg = blockIdx.x % G;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ntx = (S + DT_X - 1) / DT_X, nty = (S + DT_Y - 1) / DT_Y, ntz = (S + DT_Z - 1) / DT_Z;
    const int tiles = ntx * nty * ntz;
    const int V = S * S * S;
    v4f acc[NT][FR];
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
        for (int f = 0; f < FR; ++f) acc[q][f] = v4f{0, 0, 0, 0};
    for (int tt = tg; tt < B * tiles; tt += G) {
        const int b = tt / tiles, t = tt % tiles;
        const int x0 = (t % ntx) * DT_X, y0 = ((t / ntx) % nty) * DT_Y, z0 = (t / (ntx * nty)) * DT_Z;
        const float *gb = g + (long long)b * g_bs;
        const float *ib = in + (long long)b * in_bs;
        __syncthreads();
        for (int e = tid; e < COP * DT_X * DT_Y * DT_Z; e += 256) {
            const int o = e / (DT_X * DT_Y * DT_Z), v = e % (DT_X * DT_Y * DT_Z);
            const int gx = x0 + v % DT_X, gy = y0 + (v / DT_X) % DT_Y, gz = z0 + v / (DT_X * DT_Y);
            float val = 0.f;
            if (o < Co && gx < S && gy < S && gz < S) val = gb[(long long)o * V + (gz * S + gy) * S + gx];
            sG[o][v] = MT<T>::cvt(val);
        }
        // input rows (c, hz, hy): the 10 values of x0-1 .. x0+8, stored once (FP32) or as three shifted 8-wide
        // copies (BF16)
        for (int rrow = tid; rrow < DCC * DH_Z * DH_Y; rrow += 256) {
            const int c = rrow / (DH_Z * DH_Y), hz = (rrow / DH_Y) % DH_Z, hy = rrow % DH_Y;
            const int ci = ch * DCC + c, gz = z0 + hz - 1, gy = y0 + hy - 1;
            const bool rin = ci < Ci && (unsigned)gz < (unsigned)S && (unsigned)gy < (unsigned)S;
            const float *rowp = ib + (long long)ci * V + ((long long)gz * S + gy) * S;
            float r[DH_X];
#pragma unroll
            for (int hx = 0; hx < DH_X; ++hx) {
                const int gx = x0 + hx - 1;
                r[hx] = (rin && (unsigned)gx < (unsigned)S) ? rowp[gx] : 0.f;
            }
#pragma unroll
            for (int sh = 0; sh < NSH; ++sh)
#pragma unroll
                for (int j = 0; j < RW; ++j) sX[sh][c][hz][hy][j] = MT<T>::cvt(r[j + sh]);
        }
        __syncthreads();
#pragma unroll 1
        for (int ks = 0; ks < 16; ++ks) {                     // K-step: output plane ks/4, rows 2(ks%4), +1
            const int oz = ks >> 2, oy = (ks & 3) * 2;
#pragma unroll
            for (int sub = 0; sub < 4 / KL; ++sub) {
                const int k = sub * 4 + KL * (lane >> 4);      // first voxel of this lane in the step
                const int ky = oy + (k >> 3), kx = k & 7;
                typename MT<T>::op af[FR];
#pragma unroll
                for (int f = 0; f < FR; ++f)
                    af[f] = load_op<T>(&sG[f * 16 + (lane & 15)][(oz * DT_Y + ky) * DT_X + kx]);
                const int i = lane & 15;
#pragma unroll
                for (int q = 0; q < NT; ++q) {
                    const int tap = wave + 4 * q;
                    if (tap < 27) {
                        const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
                        const T *bp = (NSH == 3) ? &sX[dx][i][oz + dz][ky + dy][kx]
                                                 : &sX[0][i][oz + dz][ky + dy][kx + dx];
                        const typename MT<T>::op bf = load_op<T>(bp);
#pragma unroll
                        for (int f = 0; f < FR; ++f) acc[q][f] = MT<T>::mma(af[f], bf, acc[q][f]);
                    }
                }
            }
        }
    }
    // acc[q][f][r] = dW[o = 16 f + 4 (lane/16) + r][i = lane % 16][tap = wave + 4 q]
    const int i = ch * DCC + (lane & 15);
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        const int tap = wave + 4 * q;
        if (tap >= 27 || i >= Ci) continue;
#pragma unroll
        for (int f = 0; f < FR; ++f)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = f * 16 + 4 * (lane >> 4) + r;
                if (o < Co) part[(((long long)tg * Co + o) * Ci + i) * 27 + tap] = acc[q][f][r];
            }
    }
}

// dW[e] = sum_q part[q][e], q = 0..G-1: a block takes 64 consecutive e; thread (e, j) adds q = j, j + 4, ...
// (coalesced rows of 64 values), and the four partial sums are added in the order j = 0..3
__global__ __launch_bounds__(256) void k_wgrad_direct_sum(const float *__restrict__ part, int G, long long n,
                                                          float *__restrict__ dW) {
    __shared__ float sm[4][64];
    const int el = threadIdx.x & 63, j = threadIdx.x >> 6;
    const long long e = (long long)blockIdx.x * 64 + el;
    float s = 0.f;
    if (e < n)
        for (int q = j; q < G; q += 4) s += part[(long long)q * n + e];
    sm[j][el] = s;
    __syncthreads();
    if (j == 0 && e < n) dW[e] = ((sm[0][el] + sm[1][el]) + sm[2][el]) + sm[3][el];
}

// weight gradient of a 1x1x1 layer, dW[o][i] = sum_{b,v} g[b][o][v] in[b][i][v] (Co <= 4, Ci <= 16): each
// thread accumulates all Co x Ci products over its voxels, blocks reduce in a fixed order into part[blk][o][i]
constexpr int W1_CO = 4, W1_CI = 16, W1_VPT = 16;
__global__ __launch_bounds__(256) void k_wgrad_1x1(const float *__restrict__ g, long long g_bs, int Co,
                                                   const float *__restrict__ in, long long in_bs, int Ci, int V, int B,
                                                   float *__restrict__ part) {
    __shared__ float sm[256];
    float acc[W1_CO][W1_CI];
#pragma unroll
    for (int o = 0; o < W1_CO; ++o)
#pragma unroll
        for (int i = 0; i < W1_CI; ++i) acc[o][i] = 0.f;
    const long long NV = (long long)V * B;
    const long long u0 = ((long long)blockIdx.x * W1_VPT) * 256 + threadIdx.x;
    for (int k = 0; k < W1_VPT; ++k) {
        const long long u = u0 + (long long)k * 256;
        if (u >= NV) break;
        const int b = (int)(u / V);
        const long long v = u - (long long)b * V;
        float gv[W1_CO];
#pragma unroll
        for (int o = 0; o < W1_CO; ++o) gv[o] = o < Co ? g[(long long)b * g_bs + (long long)o * V + v] : 0.f;
#pragma unroll
        for (int i = 0; i < W1_CI; ++i) {
            const float x = i < Ci ? in[(long long)b * in_bs + (long long)i * V + v] : 0.f;
#pragma unroll
            for (int o = 0; o < W1_CO; ++o) acc[o][i] += gv[o] * x;
        }
    }
    for (int o = 0; o < Co; ++o)
        for (int i = 0; i < Ci; ++i) {
            sm[threadIdx.x] = acc[o < W1_CO ? o : 0][i < W1_CI ? i : 0];
            __syncthreads();
            for (int w = 128; w > 0; w >>= 1) {
                if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
                __syncthreads();
            }
            if (threadIdx.x == 0) part[((long long)blockIdx.x * Co + o) * Ci + i] = sm[0];
            __syncthreads();
        }
}

}  // namespace

// ---------------------------------------------------------------------------------------------- launchers
template <typename T>
hipError_t cnn_conv_fwd_t(const float *in, long long in_bs, int Ci, int S, int taps, const void *wt, int Kp, int COP,
                          const float *bias, int Co, float *out, long long out_bs, int relu, int B, hipStream_t s) {
    long long V = (long long)S * S * S;
    unsigned grid = (unsigned)(B * ((V + CT - 1) / CT));
    const T *w = (const T *)wt;
    if (COP == 16) hipLaunchKernelGGL((k_conv_fwd<T, 16>), dim3(grid), dim3(256), 0, s, in, in_bs, Ci, S, taps, w, Kp, bias, Co, out, out_bs, relu);
    else if (COP == 32) hipLaunchKernelGGL((k_conv_fwd<T, 32>), dim3(grid), dim3(256), 0, s, in, in_bs, Ci, S, taps, w, Kp, bias, Co, out, out_bs, relu);
    else if (COP == 64) hipLaunchKernelGGL((k_conv_fwd<T, 64>), dim3(grid), dim3(256), 0, s, in, in_bs, Ci, S, taps, w, Kp, bias, Co, out, out_bs, relu);
    else if (COP == 48) hipLaunchKernelGGL((k_conv_fwd<T, 48>), dim3(grid), dim3(256), 0, s, in, in_bs, Ci, S, taps, w, Kp, bias, Co, out, out_bs, relu);
    else if (COP == 96) hipLaunchKernelGGL((k_conv_fwd<T, 96>), dim3(grid), dim3(256), 0, s, in, in_bs, Ci, S, taps, w, Kp, bias, Co, out, out_bs, relu);
    else if (COP == 128) hipLaunchKernelGGL((k_conv_fwd<T, 128>), dim3(grid), dim3(256), 0, s, in, in_bs, Ci, S, taps, w, Kp, bias, Co, out, out_bs, relu);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// split the launch until it has about 1024 workgroups: first by output-row groups, then over input-channel chunks
void cnn_direct_split(int Ci, int S, int COP, int B, int &fr, int &rowgroups, int &nsplit, int &cpb) {
    const long long tiles = (long long)((S + DT_X - 1) / DT_X) * ((S + DT_Y - 1) / DT_Y) * ((S + DT_Z - 1) / DT_Z);
    const int nchunk = (Ci + DCC - 1) / DCC;
    const long long target = 1024;
    fr = COP / 16;
    rowgroups = 1;
    nsplit = 1;
    cpb = nchunk;
    if (tiles * B >= target) return;
    fr = 1;
    rowgroups = COP / 16;
    long long wg = tiles * B * rowgroups;
    if (wg >= target || nchunk == 1) return;
    int want = (int)std::min<long long>(nchunk, (target + wg - 1) / wg);
    cpb = (nchunk + want - 1) / want;
    nsplit = (nchunk + cpb - 1) / cpb;
}

template <typename T>
hipError_t cnn_conv_direct_t(const float *in, long long in_bs, int Ci, int S, const void *wt, int COP, const float *bias,
                             int Co, float *out, long long out_bs, int relu, int B, float *part, long long part_elems,
                             hipStream_t s) {
    int fr, rowgroups, nsplit, cpb;
    cnn_direct_split(Ci, S, COP, B, fr, rowgroups, nsplit, cpb);
    const long long V = (long long)S * S * S;
    if (nsplit > 1 && (!part || (long long)nsplit * B * Co * V > part_elems)) {
        nsplit = 1;                                         // no room for partial sums: one K split
        cpb = (Ci + DCC - 1) / DCC;
    }
    const int tiles = ((S + DT_X - 1) / DT_X) * ((S + DT_Y - 1) / DT_Y) * ((S + DT_Z - 1) / DT_Z);
    const unsigned grid = (unsigned)((long long)B * tiles * rowgroups * nsplit);
    const T *w = (const T *)wt;
#define DLAUNCH(F)                                                                                                   \
    hipLaunchKernelGGL((k_conv_direct<T, F>), dim3(grid), dim3(256), 0, s, in, in_bs, Ci, S, w, COP, bias, Co, out,   \
                       out_bs, relu, rowgroups, nsplit, cpb, part, B)
    switch (fr) {
    case 1: DLAUNCH(1); break;
    case 2: DLAUNCH(2); break;
    case 3: DLAUNCH(3); break;
    case 4: DLAUNCH(4); break;
    case 6: DLAUNCH(6); break;
    case 8: DLAUNCH(8); break;
    default: return hipErrorInvalidValue;
    }
#undef DLAUNCH
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nsplit == 1) return e;
    const long long n = (long long)B * Co * V;
    hipLaunchKernelGGL(k_conv_split_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, nsplit, B, Co, (int)V,
                       bias, relu, out, out_bs);
    return hipGetLastError();
}

hipError_t cnn_conv_direct(int use_bf16, const float *in, long long in_bs, int Ci, int S, const void *wt, int COP,
                           const float *bias, int Co, float *out, long long out_bs, int relu, int B, float *part,
                           long long part_elems, hipStream_t s) {
    return use_bf16 ? cnn_conv_direct_t<bf16>(in, in_bs, Ci, S, wt, COP, bias, Co, out, out_bs, relu, B, part, part_elems, s)
                    : cnn_conv_direct_t<float>(in, in_bs, Ci, S, wt, COP, bias, Co, out, out_bs, relu, B, part, part_elems, s);
}

template <typename T>
hipError_t cnn_wgrad_direct_t(const float *g, long long g_bs, int Co, const float *in, long long in_bs, int Ci, int S,
                              int B, float *part, long long part_elems, float *dW, hipStream_t s) {
    const int tiles = ((S + DT_X - 1) / DT_X) * ((S + DT_Y - 1) / DT_Y) * ((S + DT_Z - 1) / DT_Z);
    const int nchunk = (Ci + DCC - 1) / DCC;
    const long long per = (long long)Co * Ci * 27;
    long long G = std::max<long long>(1, std::min<long long>((long long)B * tiles, (1024 + nchunk - 1) / nchunk));
    G = std::min<long long>(G, part_elems / per);
    if (G < 1) return hipErrorInvalidValue;
    const int COP = (Co + 15) / 16 * 16;
    const unsigned grid = (unsigned)(nchunk * G);
    switch (COP / 16) {
    case 1: hipLaunchKernelGGL((k_wgrad_direct<T, 1>), dim3(grid), dim3(256), 0, s, g, g_bs, Co, in, in_bs, Ci, S, B, (int)G, part); break;
    case 2: hipLaunchKernelGGL((k_wgrad_direct<T, 2>), dim3(grid), dim3(256), 0, s, g, g_bs, Co, in, in_bs, Ci, S, B, (int)G, part); break;
    case 4: hipLaunchKernelGGL((k_wgrad_direct<T, 4>), dim3(grid), dim3(256), 0, s, g, g_bs, Co, in, in_bs, Ci, S, B, (int)G, part); break;
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wgrad_direct_sum, dim3((unsigned)((per + 63) / 64)), dim3(256), 0, s, part, (int)G, per, dW);
    return hipGetLastError();
}

hipError_t cnn_wgrad_1x1(const float *g, long long g_bs, int Co, const float *in, long long in_bs, int Ci, int V, int B,
                         float *part, long long part_elems, float *dW, hipStream_t s) {
    if (Co > W1_CO || Ci > W1_CI) return hipErrorInvalidValue;
    const long long NV = (long long)V * B;
    const long long nblk = (NV + 256LL * W1_VPT - 1) / (256LL * W1_VPT);
    const long long per = (long long)Co * Ci;
    if (nblk * per > part_elems) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_wgrad_1x1, dim3((unsigned)nblk), dim3(256), 0, s, g, g_bs, Co, in, in_bs, Ci, V, B, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wgrad_direct_sum, dim3((unsigned)((per + 63) / 64)), dim3(256), 0, s, part, (int)nblk, per, dW);
    return hipGetLastError();
}

hipError_t cnn_wgrad_direct(int use_bf16, const float *g, long long g_bs, int Co, const float *in, long long in_bs,
                            int Ci, int S, int B, float *part, long long part_elems, float *dW, hipStream_t s) {
    return use_bf16 ? cnn_wgrad_direct_t<bf16>(g, g_bs, Co, in, in_bs, Ci, S, B, part, part_elems, dW, s)
                    : cnn_wgrad_direct_t<float>(g, g_bs, Co, in, in_bs, Ci, S, B, part, part_elems, dW, s);
}

long long cnn_direct_size(int Co, int Ci) { return (long long)((Ci + DCC - 1) / DCC) * 27 * ((Co + 15) / 16 * 16) * DCC; }

hipError_t cnn_pack_direct(int use_bf16, const float *W, int Co, int Ci, int transpose, void *wt, hipStream_t s) {
    const int COP = (Co + 15) / 16 * 16;
    const long long total = cnn_direct_size(Co, Ci);
    const unsigned grid = (unsigned)((total + 255) / 256);
    if (use_bf16) hipLaunchKernelGGL(k_pack_direct<bf16>, dim3(grid), dim3(256), 0, s, W, Co, Ci, transpose, COP, total, (bf16 *)wt);
    else hipLaunchKernelGGL(k_pack_direct<float>, dim3(grid), dim3(256), 0, s, W, Co, Ci, transpose, COP, total, (float *)wt);
    return hipGetLastError();
}

hipError_t cnn_conv_fwd(int use_bf16, const float *in, long long in_bs, int Ci, int S, int taps, const void *wt, int Kp,
                        int COP, const float *bias, int Co, float *out, long long out_bs, int relu, int B,
                        hipStream_t s) {
    return use_bf16 ? cnn_conv_fwd_t<bf16>(in, in_bs, Ci, S, taps, wt, Kp, COP, bias, Co, out, out_bs, relu, B, s)
                : cnn_conv_fwd_t<float>(in, in_bs, Ci, S, taps, wt, Kp, COP, bias, Co, out, out_bs, relu, B, s);
}

hipError_t cnn_bias_grad(const float *g, long long g_bs, int B, long long V, int Co, float *part, float *db,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_bias_part, dim3(Co * BG_SLICES), dim3(256), 0, s, g, g_bs, B, (int)V, part);
    hipLaunchKernelGGL(k_bias_reduce, dim3((Co + 63) / 64), dim3(64), 0, s, part, Co, db);
    return hipGetLastError();
}

hipError_t cnn_pack_weights(int use_bf16, const float *W, int Co, int Ci, int taps, int transpose, int COP, int Kp,
                            void *wt, hipStream_t s) {
    long long n = (long long)COP * Kp;
    unsigned grid = (unsigned)((n + 255) / 256);
    if (use_bf16) hipLaunchKernelGGL(k_pack_weights<bf16>, dim3(grid), dim3(256), 0, s, W, Co, Ci, taps, transpose, COP, Kp, (bf16 *)wt);
    else hipLaunchKernelGGL(k_pack_weights<float>, dim3(grid), dim3(256), 0, s, W, Co, Ci, taps, transpose, COP, Kp, (float *)wt);
    return hipGetLastError();
}

hipError_t cnn_relu_bwd(float *g, long long g_bs, const float *y, long long y_bs, long long per, int B, hipStream_t s) {
    hipLaunchKernelGGL(k_relu_bwd, dim3((unsigned)((per * B + 255) / 256)), dim3(256), 0, s, g, g_bs, y, y_bs, per, B);
    return hipGetLastError();
}
hipError_t cnn_pool_fwd(const float *in, long long in_bs, float *out, long long out_bs, int C, int S, int B, hipStream_t s) {
    long long n = (long long)C * (S / 2) * (S / 2) * (S / 2) * B;
    hipLaunchKernelGGL(k_pool_fwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, in_bs, out, out_bs, C, S, B);
    return hipGetLastError();
}
hipError_t cnn_pool_bwd(const float *gout, long long gout_bs, float *gin, long long gin_bs, int C, int S, int B,
                        int accumulate, hipStream_t s) {
    long long n = (long long)C * S * S * S * B;
    hipLaunchKernelGGL(k_pool_bwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, gout, gout_bs, gin, gin_bs, C, S, B, accumulate);
    return hipGetLastError();
}
hipError_t cnn_up_fwd(const float *in, long long in_bs, float *out, long long out_bs, int C, int S, int B, hipStream_t s) {
    long long n = (long long)C * 8 * S * S * S * B;
    hipLaunchKernelGGL(k_up_fwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, in_bs, out, out_bs, C, S, B);
    return hipGetLastError();
}
hipError_t cnn_up_bwd(const float *gout, long long gout_bs, float *gin, long long gin_bs, int C, int S, int B, hipStream_t s) {
    long long n = (long long)C * S * S * S * B;
    hipLaunchKernelGGL(k_up_bwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, gout, gout_bs, gin, gin_bs, C, S, B);
    return hipGetLastError();
}
hipError_t cnn_mse(const float *y, const float *t, long long n, float *g, double *part, double *loss, hipStream_t s) {
    unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, y, t, n, g, part);
    hipLaunchKernelGGL(k_sum_d, dim3(1), dim3(256), 0, s, part, (int)nb, loss, 1.0 / (double)n);
    return hipGetLastError();
}
hipError_t cnn_adam(float *w, const float *g, float *m, float *v, long long n, float lr, float b1, float b2, float eps,
                    float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}
hipError_t cnn_features(const double *k2h, const double2 *fh, int halo, int nf, int S, double k0sq, double cs,
                        double fs, float *x, hipStream_t s) {
    long long V = (long long)S * S * S;
    hipLaunchKernelGGL(k_features, dim3((unsigned)((V + 255) / 256)), dim3(256), 0, s, k2h, fh, halo, nf, S,
                       1.0 / k0sq, cs, fs, x);
    return hipGetLastError();
}
hipError_t cnn_prolong(const float *coarse, int nc, double scale, double gre, double gim, int cubic, double2 *fine,
                       int nf, double2 *work, hipStream_t s) {
    long long n = (long long)nf * nf * nf;
    if (cubic && work) {
        // x: [z][y][x] -> [x'][z][y]; y: [x'][z][y] -> [y'][x'][z]; z: [y'][x'][z] -> [z'][y'][x']
        double2 *t1 = work, *t2 = work + (long long)nf * nc * nc;
        const long long m1 = (long long)nf * nc * nc, m2 = (long long)nf * nf * nc;
        hipLaunchKernelGGL(k_prolong3_pass<float>, dim3((unsigned)((m1 + 255) / 256)), dim3(256), 0, s, coarse, 0, nc,
                           nc, nc, nf, gre, gim, 1.0, t1);
        hipLaunchKernelGGL(k_prolong3_pass<double2>, dim3((unsigned)((m2 + 255) / 256)), dim3(256), 0, s, t1, 1, nc,
                           nc, nf, nf, gre, gim, 1.0, t2);
        hipLaunchKernelGGL(k_prolong3_pass<double2>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, t2, 1, nc,
                           nf, nf, nf, gre, gim, scale, fine);
    } else if (cubic)
        hipLaunchKernelGGL(k_prolong3, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, coarse, nc, scale, gre, gim,
                           fine, nf);
    else
        hipLaunchKernelGGL(k_prolong, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, coarse, nc, scale, gre, gim,
                           fine, nf);
    return hipGetLastError();
}

}  // namespace helm
