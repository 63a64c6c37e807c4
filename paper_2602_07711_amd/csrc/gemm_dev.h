// Device code of the complex MFMA GEMM, shared by the single-problem and the grouped (batched) kernels.
#pragma once
#include "helm_internal.h"

namespace helm {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct cplx;
template <> struct cplx<double> { typedef double2 t; typedef v4d acc; };
template <> struct cplx<float> { typedef float2 t; typedef v4f acc; };

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T, typename S> __device__ __forceinline__ typename cplx<T>::t cvt(S v) {
    typename cplx<T>::t r;
    r.x = (T)v.x;
    r.y = (T)v.y;
    return r;
}

template <typename TC, typename T> __device__ __forceinline__ TC pack(T re, T im) {
    TC r;
    r.x = re;
    r.y = im;
    return r;
}

// The MFMA products of one k-step of four: fragments fa (A, FM blocks of 16 rows) and fb (B, FN blocks of 16
// columns) into the accumulator sets t. RW = 1: A is real, RW = 2: B is real (the sine matrix of the PFFT
// transforms); then each complex MAC needs two real products. Otherwise 3M for FP32 (NS = 3) and 4M for FP64.
template <typename T, int RW, int NS, int FM, int FN>
__device__ __forceinline__ void mma_kstep(typename cplx<T>::acc (&t)[NS][FM][FN], const typename cplx<T>::t (&fa)[FM],
                                          const typename cplx<T>::t (&fb)[FN]) {
    if constexpr (RW == 1) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                t[0][i][j] = mfma(fa[i].x, fb[j].x, t[0][i][j]);
                t[1][i][j] = mfma(fa[i].x, fb[j].y, t[1][i][j]);
            }
    } else if constexpr (RW == 2) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                t[0][i][j] = mfma(fa[i].x, fb[j].x, t[0][i][j]);
                t[1][i][j] = mfma(fa[i].y, fb[j].x, t[1][i][j]);
            }
    } else if constexpr (NS == 3) {
        T sa[FM], sb[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) sa[i] = fa[i].x + fa[i].y;
#pragma unroll
        for (int j = 0; j < FN; ++j) sb[j] = fb[j].x + fb[j].y;
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) t[0][i][j] = mfma(fa[i].x, fb[j].x, t[0][i][j]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) t[1][i][j] = mfma(fa[i].y, fb[j].y, t[1][i][j]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) t[2][i][j] = mfma(sa[i], sb[j], t[2][i][j]);
    } else {
        // t[0] = real part, t[1] = imaginary part
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                t[0][i][j] = mfma(fa[i].x, fb[j].x, t[0][i][j]);
                t[1][i][j] = mfma(fa[i].x, fb[j].y, t[1][i][j]);
            }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                t[0][i][j] = mfma(-fa[i].y, fb[j].y, t[0][i][j]);
                t[1][i][j] = mfma(fa[i].y, fb[j].x, t[1][i][j]);
            }
    }
}

// Complex value held in accumulator register r of block (i, j): 3M (T1, T2, T3) -> (T1 - T2, T3 - T1 - T2).
template <typename T, int NS, int FM, int FN>
__device__ __forceinline__ void acc_value(const typename cplx<T>::acc (&t)[NS][FM][FN], int i, int j, int r, T &re,
                                          T &im) {
    if constexpr (NS == 3) {
        re = t[0][i][j][r] - t[1][i][j][r];
        im = t[2][i][j][r] - t[0][i][j][r] - t[1][i][j][r];
    } else {
        re = t[0][i][j][r];
        im = t[1][i][j][r];
    }
}

// Row of accumulator register r within a 16x16 block: f64 holds rows 4r + lane/16, f32 rows 4(lane/16) + r.
template <typename T> __device__ __forceinline__ int acc_row(int lane, int r) {
    return sizeof(T) == 8 ? 4 * r + (lane >> 4) : 4 * (lane >> 4) + r;
}

// One BM x BN output tile of C[b] = A[b] B[b]; `tile` enumerates (batch, m-tile, n-tile) with n fastest.
template <typename TA, typename TB, typename TC, typename T, int BM, int BN, int BK, int RW>
__device__ __forceinline__ void gemm_tile(const TA *__restrict__ A, const TB *__restrict__ B, TC *__restrict__ C,
                                          const GemmDesc &d, long long tile) {
    typedef typename cplx<T>::t CT;
    typedef typename cplx<T>::acc ACC;
    constexpr int FM = BM / 32;           // 16x16 blocks per wave along M (2 waves along M)
    constexpr int FN = BN / 32;           // along N (2 waves along N)
    constexpr int EA = BM * BK / 256;     // A elements per thread per chunk
    constexpr int EB = BK * BN / 256;
    __shared__ CT sA[BK][BM + 1];
    __shared__ CT sB[BK][BN];

    const int tm = (d.M + BM - 1) / BM, tn = (d.N + BN - 1) / BN;
    const int b = (int)(tile / ((long long)tm * tn));
    const int rem = (int)(tile % ((long long)tm * tn));
    const int mt = rem / tn, nt = rem % tn;
    const int m0 = mt * BM, n0 = nt * BN;
    A += (long long)b * d.sA;
    B += (long long)b * d.sB;
    C += (long long)b * d.sC;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    // RW = 1: A is real, RW = 2: B is real (the sine matrix of the PFFT transforms); then each complex MAC
    // needs two real products. Otherwise 3M for FP32 and 4M for FP64.
    constexpr bool G3 = sizeof(T) == 4 && RW == 0;
    constexpr int NS = G3 ? 3 : 2;
    ACC t[NS][FM][FN];
#pragma unroll
    for (int q = 0; q < NS; ++q)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) t[q][i][j] = ACC{0, 0, 0, 0};

    CT ra[EA], rb[EB];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int e = 0; e < EA; ++e) {
            int idx = tid + e * 256;
            int mm = idx / BK, kk = idx % BK;          // consecutive threads walk k (contiguous in A rows)
            int gm = m0 + mm, gk = k0 + kk;
            ra[e] = (gm < d.M && gk < d.K) ? cvt<T>(A[(long long)gm * d.lda + gk]) : CT{0, 0};
        }
#pragma unroll
        for (int e = 0; e < EB; ++e) {
            int idx = tid + e * 256;
            int kk = idx / BN, nn = idx % BN;          // consecutive threads walk n (contiguous in B rows)
            int gk = k0 + kk, gn = n0 + nn;
            rb[e] = (gk < d.K && gn < d.N) ? cvt<T>(B[(long long)gk * d.ldb + gn]) : CT{0, 0};
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int e = 0; e < EA; ++e) {
            int idx = tid + e * 256;
            sA[idx % BK][idx / BK] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < EB; ++e) {
            int idx = tid + e * 256;
            sB[idx / BN][idx % BN] = rb[e];
        }
    };

    const int rowA = wm * (BM / 2) + (lane & 15);
    const int colB = wn * (BN / 2) + (lane & 15);
    const int kl = lane >> 4;

    fetch(0);
    for (int k0 = 0; k0 < d.K; k0 += BK) {
        __syncthreads();
        stash();
        __syncthreads();
        if (k0 + BK < d.K) fetch(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            CT fa[FM], fb[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) fa[i] = sA[kk + kl][rowA + i * 16];
#pragma unroll
            for (int j = 0; j < FN; ++j) fb[j] = sB[kk + kl][colB + j * 16];
            mma_kstep<T, RW, NS>(t, fa, fb);
        }
    }

#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int gn = n0 + wn * (BN / 2) + j * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm * (BM / 2) + i * 16 + acc_row<T>(lane, r);
                if (gm < d.M && gn < d.N) {
                    T re, im;
                    acc_value<T>(t, i, j, r, re, im);
                    C[(long long)gm * d.ldc + gn] = pack<TC, T>(re, im);
                }
            }
        }
}

}  // namespace
}  // namespace helm
