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

// ---------------------------------------------------------------------------------------------------------
// Folded EigT transforms. Lambda-bar has the same closure at both ends, so it is centrosymmetric and its
// eigenvectors are symmetric or skew about the middle of the axis: V = Q diag(Vs, Va), V^{-1} = diag(Vs^{-1},
// Va^{-1}) Q^T with Q the butterfly (e_i +- e_{n-1-i})/sqrt(2) (plus e_m alone for odd n). A length-n transform
// is then two products with the half blocks, n^2/2 complex MACs instead of n^2; the butterfly is fused into
// the operand load (forward: the data enters as D[i] +- D[n-1-i]) or the epilogue (inverse: the two half
// products P, M are written as P + M at i and P - M at n-1-i). The 1/sqrt(2) factors (1/2 and 1 for the
// middle of an odd axis) live in the block matrices. Modes are ordered [symmetric (ms) | skew (ma)].
//   FOLD_XF  x forward:  C[c][o_p + k] = sum_{i < K_p} (D[c][i] +- D[c][n-1-i]) M_p[i][k]
//   FOLD_YF  y forward:  C[o_p + k][x] = sum_{i < K_p} M_p[k][i] (D[i][x] +- D[n-1-i][x])
//   FOLD_XI  x inverse:  P = sum_{k < ms} D[c][k] M_s[k][i],  M = sum_{k < ma} D[c][ms + k] M_a[k][i]
//   FOLD_YI  y inverse:  P = sum_{k < ms} M_s[j][k] D[k][x],  M = sum_{k < ma} M_a[j][k] D[ms + k][x]
// with p = s (sign +, K_s = ms, o_s = 0) or a (sign -, K_a = ma, o_a = ms); in the inverse, i (j) < ms and the
// middle of an odd axis (i = ma, no skew partner: M = 0 there) is written once.

template <int MODE, int BM, int BN> __host__ __device__ inline long long fold_tiles(const FoldDesc &f) {
    return fold_tile_count(MODE, f, BM, BN);
}

// Occupancy the register allocator is asked for: without it, the FP64 kernels keep their accumulators in
// AGPRs on top of the VGPRs the operand staging needs and drop to two waves per SIMD. The x-forward transforms
// with FP64 data hold two raw FP64 values per operand element across a chunk (the butterfly is formed when the
// chunk is written to LDS) and get one wave less. The FP32 inverse transforms on 64 x 64 x 16 tiles park P in LDS
// (fold_tile), 48 KiB per block in all, which fits three blocks per CU.
template <typename T, typename TD, int MODE, int BM, int BN, int BK> constexpr int fold_waves() {
    if (sizeof(T) == 4 && (MODE == FOLD_XI || MODE == FOLD_YI) && BM * BN * BK <= 64 * 64 * 16) return 3;
    return (sizeof(T) == 8 ? (BM * BN * BK <= 64 * 64 * 16 ? 3 : 1) : (BM * BN * BK <= 64 * 64 * 16 ? 4 : 2)) -
           ((MODE == FOLD_XF && sizeof(TD) == 16 && BM * BN * BK <= 64 * 64 * 16) ? 1 : 0);
}

// a +- b in the precision the data is stored in, then converted to the arithmetic type
template <typename T, typename S> __device__ __forceinline__ typename cplx<T>::t fold2(S a, S b, bool minus) {
    S r;
    r.x = minus ? a.x - b.x : a.x + b.x;
    r.y = minus ? a.y - b.y : a.y + b.y;
    return cvt<T>(r);
}

template <typename S> struct Pair { S a, b; };

// The K loop of one tile: raw operands come from loadA(local row, k) and loadB(k, local column) (zero outside) and
// are staged through LDS double buffered in registers, as in gemm_tile. finA / finB turn a raw operand into the
// arithmetic type (conversion, the butterfly's sum or difference) only when it is written to LDS, one chunk later:
// doing it at load time would make every chunk wait for its own loads before the MFMAs that should hide them.
template <typename T, int BM, int BN, int BK, int NS, int RW, typename LA, typename LB, typename FA, typename FB>
__device__ __forceinline__ void fold_kloop(typename cplx<T>::acc (&t)[NS][BM / 32][BN / 32], int K, LA loadA,
                                           LB loadB, FA finA, FB finB, typename cplx<T>::t (*sA)[BM + 1],
                                           typename cplx<T>::t (*sB)[BN]) {
    typedef typename cplx<T>::t CT;
    constexpr int FM = BM / 32, FN = BN / 32, EA = BM * BK / 256, EB = BK * BN / 256;
    // an opaque copy of the thread index: the index arithmetic of two K loops in one kernel (the inverse
    // transforms) is then not shared between them and held in registers across the first
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    decltype(loadA(0, 0)) ra[EA];
    decltype(loadB(0, 0)) rb[EB];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int e = 0; e < EA; ++e) {
            const int idx = tid + e * 256;
            ra[e] = loadA(idx / BK, k0 + idx % BK);       // consecutive threads walk k
        }
#pragma unroll
        for (int e = 0; e < EB; ++e) {
            const int idx = tid + e * 256;
            rb[e] = loadB(k0 + idx / BN, idx % BN);       // consecutive threads walk n
        }
    };
    const int rowA = wm * (BM / 2) + (lane & 15);
    const int colB = wn * (BN / 2) + (lane & 15);
    const int kl = lane >> 4;
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += BK) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EA; ++e) {
            const int idx = tid + e * 256;
            sA[idx % BK][idx / BK] = finA(ra[e]);
        }
#pragma unroll
        for (int e = 0; e < EB; ++e) {
            const int idx = tid + e * 256;
            sB[idx / BN][idx % BN] = finB(rb[e]);
        }
        __syncthreads();
        if (k0 + BK < K) fetch(k0 + BK);
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
}

// One tile (`tile` < fold_tiles) of a folded transform.
template <int MODE, typename TD, typename TM, typename TC, typename T, int BM, int BN, int BK, int RW = 0>
__device__ __forceinline__ void fold_tile(const TD *__restrict__ D, const TM *__restrict__ Ms, const TM *__restrict__ Ma,
                                          TC *__restrict__ C, const FoldDesc &f, long long tile) {
    typedef typename cplx<T>::t CT;
    typedef typename cplx<T>::acc ACC;
    constexpr int FM = BM / 32, FN = BN / 32;
    constexpr int NS = (sizeof(T) == 4 && RW == 0) ? 3 : 2;
    __shared__ CT sA[BK][BM + 1];
    __shared__ CT sB[BK][BN];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int n = f.n, ms = f.ms, ma = f.ma, rows = f.rows;
    const long long ld = f.ld;

    ACC t[NS][FM][FN];
    auto zero = [&]() {
#pragma unroll
        for (int q = 0; q < NS; ++q)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) t[q][i][j] = ACC{0, 0, 0, 0};
    };
    zero();

    if constexpr (MODE == FOLD_XF || MODE == FOLD_YF) {
        int mt, nt;
        bool skew;
        if constexpr (MODE == FOLD_XF) {
            const int hs = (ms + BN - 1) / BN, ha = (ma + BN - 1) / BN;
            mt = (int)(tile / (hs + ha));
            const int r = (int)(tile % (hs + ha));
            skew = r >= hs;
            nt = skew ? r - hs : r;
        } else {
            const int hs = (ms + BM - 1) / BM, ha = (ma + BM - 1) / BM, tn = (rows + BN - 1) / BN;
            const long long per_slice = (long long)(hs + ha) * tn;
            const long long b = tile / per_slice;
            const int rem = (int)(tile % per_slice);
            const int r = rem / tn;
            nt = rem % tn;
            skew = r >= hs;
            mt = skew ? r - hs : r;
            D += b * f.sD;
            C += b * f.sD;
        }
        const int K = skew ? ma : ms, off = skew ? f.moff : 0, mst = f.mstep;
        const TM *Mp = skew ? Ma : Ms;
        const int m0 = mt * BM, n0 = nt * BN;
        if constexpr (MODE == FOLD_XF) {
            auto la = [&](int mm, int gk) -> Pair<TD> {
                const int gm = m0 + mm;
                if (gm >= rows || gk >= K) return Pair<TD>{TD{0, 0}, TD{0, 0}};
                const TD *row = D + (long long)gm * ld;
                return Pair<TD>{row[gk], row[n - 1 - gk]};
            };
            auto lb = [&](int gk, int nn) -> TM {
                const int gn = n0 + nn;
                return (gk < K && gn < K) ? Mp[(long long)gk * K + gn] : TM{0, 0};
            };
            auto fa = [&](const Pair<TD> &p) { return fold2<T>(p.a, p.b, skew); };
            auto fb = [](const TM &v) { return cvt<T>(v); };
            fold_kloop<T, BM, BN, BK, NS, RW>(t, K, la, lb, fa, fb, sA, sB);
        } else {
            auto la = [&](int mm, int gk) -> TM {
                const int gm = m0 + mm;
                return (gm < K && gk < K) ? Mp[(long long)gm * K + gk] : TM{0, 0};
            };
            auto lb = [&](int gk, int nn) -> Pair<TD> {
                const int gn = n0 + nn;
                if (gk >= K || gn >= rows) return Pair<TD>{TD{0, 0}, TD{0, 0}};
                return Pair<TD>{D[(long long)gk * ld + gn], D[(long long)(n - 1 - gk) * ld + gn]};
            };
            auto fa = [](const TM &v) { return cvt<T>(v); };
            auto fb = [&](const Pair<TD> &p) { return fold2<T>(p.a, p.b, skew); };
            fold_kloop<T, BM, BN, BK, NS, RW>(t, K, la, lb, fa, fb, sA, sB);
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int gn = n0 + wn * (BN / 2) + j * 16 + (lane & 15);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gm = m0 + wm * (BM / 2) + i * 16 + acc_row<T>(lane, r);
                    T re, im;
                    acc_value<T>(t, i, j, r, re, im);
                    if constexpr (MODE == FOLD_XF) {
                        if (gm < rows && gn < K) C[(long long)gm * ld + off + mst * gn] = pack<TC, T>(re, im);
                    } else {
                        if (gm < K && gn < rows) C[(long long)(off + mst * gm) * ld + gn] = pack<TC, T>(re, im);
                    }
                }
            }
    } else {
        // FP32 64 x 64 tiles park P in LDS (32 KiB per block, read back only by the thread that wrote it)
        constexpr bool PLDS = sizeof(T) == 4 && FM * FN * 4 * 256 * sizeof(CT) <= 32768;
        __shared__ CT sP[PLDS ? FM * FN * 4 * 256 : 1];
        int mt, nt;
        if constexpr (MODE == FOLD_XI) {
            const int tn = (ms + BN - 1) / BN;
            mt = (int)(tile / tn);
            nt = (int)(tile % tn);
        } else {
            const int tm = (ms + BM - 1) / BM, tn = (rows + BN - 1) / BN;
            const long long b = tile / ((long long)tm * tn);
            const int rem = (int)(tile % ((long long)tm * tn));
            mt = rem / tn;
            nt = rem % tn;
            D += b * f.sD;
            C += b * f.sD;
        }
        const int m0 = mt * BM, n0 = nt * BN;
        // output slot (position i or j < ms, the other index) of accumulator register r of block (i, j)
        auto slot = [&](int ln, int i, int j, int r, int &gm, int &gn) -> bool {
            gm = m0 + wm * (BM / 2) + i * 16 + acc_row<T>(ln, r);
            gn = n0 + wn * (BN / 2) + j * 16 + (ln & 15);
            return MODE == FOLD_XI ? (gm < rows && gn < ms) : (gm < ms && gn < rows);
        };
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int K = q ? ma : ms, off = q ? f.moff : 0, mst = f.mstep;
            const TM *Mq = q ? Ma : Ms;
            if constexpr (MODE == FOLD_XI) {
                auto la = [&](int mm, int gk) -> TD {
                    const int gm = m0 + mm;
                    return (gm < rows && gk < K) ? D[(long long)gm * ld + off + mst * gk] : TD{0, 0};
                };
                auto lb = [&](int gk, int nn) -> TM {
                    const int gn = n0 + nn;
                    return (gk < K && gn < K) ? Mq[(long long)gk * K + gn] : TM{0, 0};
                };
                auto fa = [](const TD &v) { return cvt<T>(v); };
                auto fb = [](const TM &v) { return cvt<T>(v); };
                fold_kloop<T, BM, BN, BK, NS, RW>(t, K, la, lb, fa, fb, sA, sB);
            } else {
                auto la = [&](int mm, int gk) -> TM {
                    const int gm = m0 + mm;
                    return (gm < K && gk < K) ? Mq[(long long)gm * K + gk] : TM{0, 0};
                };
                auto lb = [&](int gk, int nn) -> TD {
                    const int gn = n0 + nn;
                    return (gk < K && gn < rows) ? D[(long long)(off + mst * gk) * ld + gn] : TD{0, 0};
                };
                auto fa = [](const TM &v) { return cvt<T>(v); };
                auto fb = [](const TD &v) { return cvt<T>(v); };
                fold_kloop<T, BM, BN, BK, NS, RW>(t, K, la, lb, fa, fb, sA, sB);
            }
            if (q == 0) {
                // park P in this thread's own output slots (first half of the axis; the skew results go to the
                // disjoint second half), or for the FP32 64 x 64 tile in a per-thread LDS area, instead of holding a
                // second accumulator set in registers
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            int gm, gn;
                            if (!slot(lane, i, j, r, gm, gn)) continue;
                            T re, im;
                            acc_value<T>(t, i, j, r, re, im);
                            if constexpr (PLDS) sP[((i * FN + j) * 4 + r) * 256 + threadIdx.x] = pack<CT, T>(re, im);
                            else C[(long long)gm * ld + gn] = pack<TC, T>(re, im);
                        }
                zero();
                // a compiler memory barrier: the epilogue reloads P instead of the stored values being
                // forwarded to it in registers through the second K loop
                asm volatile("" ::: "memory");
            }
        }
        // the epilogue recomputes the slot addresses (an opaque copy of the lane index) rather than keeping the
        // park step's addresses alive through the second K loop
        int lane_e = lane;
        asm volatile("" : "+v"(lane_e));
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    int gm, gn;
                    if (!slot(lane_e, i, j, r, gm, gn)) continue;
                    T re, im;
                    acc_value<T>(t, i, j, r, re, im);
                    TC *c = C + (long long)gm * ld + gn;
                    T p0, p1;
                    if constexpr (PLDS) {
                        const CT pv = sP[((i * FN + j) * 4 + r) * 256 + threadIdx.x];
                        p0 = pv.x;
                        p1 = pv.y;
                    } else {
                        const TC pv = *c;
                        p0 = (T)pv.x;
                        p1 = (T)pv.y;
                    }
                    const int h = MODE == FOLD_XI ? gn : gm;     // position along the transformed axis
                    if (h < ma) {
                        *c = pack<TC, T>(p0 + re, p1 + im);
                        TC *mirror = MODE == FOLD_XI ? C + (long long)gm * ld + (n - 1 - gn)
                                                     : C + (long long)(n - 1 - gm) * ld + gn;
                        *mirror = pack<TC, T>(p0 - re, p1 - im);
                    } else if constexpr (PLDS) {
                        *c = pack<TC, T>(p0, p1);                 // the middle of an odd axis: P alone
                    }
                }
    }
}

}  // namespace
}  // namespace helm
