// Batched complex GEMM C[b] = A[b] B[b] on MFMA (row-major, interleaved complex), FP64 or FP32 arithmetic.
//
// It carries the EigT transforms (Sec. 4.1, eq. EIG_SOLVER Steps 2 and 4), which are dense complex
// contractions of every x-line and every y-line with the N x N eigenvector matrices:
//   x-transform: C[c][p] = sum_q Y[c][q] W^T[q][p]       lines c = (j, l) are rows (lda = Nx), W^T precomputed;
//   y-transform: C_l[j][i] = sum_m W[j][m] Y_l[m][i]      one GEMM per slice l, data is the B operand (ldb = Nx).
// In both the fastest memory index of the data lands on the MFMA column index, so tile loads and the
// accumulator stores walk contiguous memory.
//
// Arithmetic, FP32: three real MFMA products per complex k-step (Gauss / 3M form: T1 += Ar Br, T2 += Ai Bi,
// T3 += (Ar + Ai)(Br + Bi); then Cr = T1 - T2, Ci = T3 - T1 - T2), 25% fewer MFMA issues than the four-product
// form at a rounding error bounded by eps (|Ar| + |Ai|)(|Br| + |Bi|) per term. FP64: the four-product form
// (Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br), since three f64 accumulator sets would halve occupancy. MFMA
// v_mfma_f64_16x16x4f64 (FP64) or v_mfma_f32_16x16x4f32 (FP32). Lane layout of the 16x16x4 products
// (checked on gfx950): A(row = lane%16, k = lane/16), B(k = lane/16, col = lane%16); accumulator register r
// of a lane holds D(row = 4*r + lane/16, col = lane%16) for f64 and D(row = 4*(lane/16) + r, col = lane%16)
// for f32.
// A workgroup of 4 waves computes a BM x BN tile; each wave a (BM/2) x (BN/2) sub-tile of 16x16 blocks.
// Global->LDS staging is double buffered through registers (the next K-chunk is fetched while the current
// one feeds the MFMAs). Tiles are mapped so that consecutive tiles run on the same XCD.
#include "gemm_dev.h"

namespace helm {

namespace {

template <typename TA, typename TB, typename TC, typename T, int BM, int BN, int BK, int RW>
__global__ __launch_bounds__(256) void k_zgemm(const TA *__restrict__ A, const TB *__restrict__ B, TC *__restrict__ C,
                                               GemmDesc d) {
    const int tm = (d.M + BM - 1) / BM, tn = (d.N + BN - 1) / BN;
    const long long total = (long long)tm * tn * d.batch;
    const long long per = (total + 7) / 8;
    const long long tile = (long long)(blockIdx.x % 8) * per + blockIdx.x / 8;   // consecutive tiles on one XCD
    if (tile >= total) return;
    gemm_tile<TA, TB, TC, T, BM, BN, BK, RW>(A, B, C, d, tile);
}

template <typename TA, typename TB, typename TC, typename T, int BM, int BN, int BK>
hipError_t launch_tile(const GemmDesc &d, const TA *A, const TB *B, TC *C, hipStream_t s, int rw) {
    long long tiles = (long long)((d.M + BM - 1) / BM) * ((d.N + BN - 1) / BN) * d.batch;
    long long grid = 8 * ((tiles + 7) / 8);
    if (tiles == 0) return hipSuccess;
    if (rw == 1)
        hipLaunchKernelGGL((k_zgemm<TA, TB, TC, T, BM, BN, BK, 1>), dim3((unsigned)grid), dim3(256), 0, s, A, B, C, d);
    else if (rw == 2)
        hipLaunchKernelGGL((k_zgemm<TA, TB, TC, T, BM, BN, BK, 2>), dim3((unsigned)grid), dim3(256), 0, s, A, B, C, d);
    else
        hipLaunchKernelGGL((k_zgemm<TA, TB, TC, T, BM, BN, BK, 0>), dim3((unsigned)grid), dim3(256), 0, s, A, B, C, d);
    return hipGetLastError();
}

// Tile configurations (BM, BN, BK) the autotuner chooses from; the real-operand (sine) products use config 0.
template <typename TA, typename TB, typename TC, typename T>
hipError_t launch(const GemmDesc &d, const TA *A, const TB *B, TC *C, hipStream_t s, int rw, int cfg) {
    if (rw != 0) cfg = 0;
    switch (cfg) {
    case 1: return launch_tile<TA, TB, TC, T, 64, 64, 32>(d, A, B, C, s, 0);
    case 2: return launch_tile<TA, TB, TC, T, 128, 64, 16>(d, A, B, C, s, 0);
    case 3: return launch_tile<TA, TB, TC, T, 64, 128, 16>(d, A, B, C, s, 0);
    default: return launch_tile<TA, TB, TC, T, 64, 64, 16>(d, A, B, C, s, rw);
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
    const long long tm = (f.rows + BM - 1) / BM, tn = (f.rows + BN - 1) / BN;
    const long long hs_m = (f.ms + BM - 1) / BM, ha_m = (f.ma + BM - 1) / BM;
    const long long hs_n = (f.ms + BN - 1) / BN, ha_n = (f.ma + BN - 1) / BN;
    if (MODE == FOLD_XF) return tm * (hs_n + ha_n);
    if (MODE == FOLD_YF) return (long long)f.batch * (hs_m + ha_m) * tn;
    if (MODE == FOLD_XI) return tm * hs_n;
    return (long long)f.batch * hs_m * tn;
}

// a +- b in the precision the data is stored in, then converted to the arithmetic type
template <typename T, typename S> __device__ __forceinline__ typename cplx<T>::t fold2(S a, S b, bool minus) {
    S r;
    r.x = minus ? a.x - b.x : a.x + b.x;
    r.y = minus ? a.y - b.y : a.y + b.y;
    return cvt<T>(r);
}

// The K loop of one tile: operands come from loadA(local row, k) and loadB(k, local column) (zero outside),
// staged through LDS double buffered in registers, as in gemm_tile.
template <typename T, int BM, int BN, int BK, int NS, typename LA, typename LB>
__device__ __forceinline__ void fold_kloop(typename cplx<T>::acc (&t)[NS][BM / 32][BN / 32], int K, LA loadA,
                                           LB loadB, typename cplx<T>::t (*sA)[BM + 1],
                                           typename cplx<T>::t (*sB)[BN]) {
    typedef typename cplx<T>::t CT;
    constexpr int FM = BM / 32, FN = BN / 32, EA = BM * BK / 256, EB = BK * BN / 256;
    // an opaque copy of the thread index: the index arithmetic of two K loops in one kernel (the inverse
    // transforms) is then not shared between them and held in registers across the first
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    CT ra[EA], rb[EB];
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
            sA[idx % BK][idx / BK] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < EB; ++e) {
            const int idx = tid + e * 256;
            sB[idx / BN][idx % BN] = rb[e];
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
            mma_kstep<T, 0, NS>(t, fa, fb);
        }
    }
}

// Occupancy the register allocator is asked for: without it, the FP64 kernels keep their accumulators in
// AGPRs on top of the VGPRs the operand staging needs and drop to two waves per SIMD.
template <typename T, int BM, int BN, int BK> constexpr int fold_waves() {
    return sizeof(T) == 8 ? (BM * BN * BK <= 64 * 64 * 16 ? 3 : 1) : (BM * BN * BK <= 64 * 64 * 16 ? 4 : 2);
}

template <int MODE, typename TD, typename TM, typename TC, typename T, int BM, int BN, int BK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(fold_waves<T, BM, BN, BK>()))) void k_fold(const TD *__restrict__ D, const TM *__restrict__ Ms,
                                              const TM *__restrict__ Ma, TC *__restrict__ C, FoldDesc f) {
    typedef typename cplx<T>::t CT;
    typedef typename cplx<T>::acc ACC;
    constexpr int FM = BM / 32, FN = BN / 32;
    constexpr int NS = sizeof(T) == 4 ? 3 : 2;
    __shared__ CT sA[BK][BM + 1];
    __shared__ CT sB[BK][BN];

    const long long total = fold_tiles<MODE, BM, BN>(f);
    const long long per = (total + 7) / 8;
    const long long tile = (long long)(blockIdx.x % 8) * per + blockIdx.x / 8;   // consecutive tiles on one XCD
    if (tile >= total) return;

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
        const int K = skew ? ma : ms, off = skew ? ms : 0;
        const TM *Mp = skew ? Ma : Ms;
        const int m0 = mt * BM, n0 = nt * BN;
        if constexpr (MODE == FOLD_XF) {
            auto la = [&](int mm, int gk) -> CT {
                const int gm = m0 + mm;
                if (gm >= rows || gk >= K) return CT{0, 0};
                const TD *row = D + (long long)gm * ld;
                return fold2<T>(row[gk], row[n - 1 - gk], skew);
            };
            auto lb = [&](int gk, int nn) -> CT {
                const int gn = n0 + nn;
                return (gk < K && gn < K) ? cvt<T>(Mp[(long long)gk * K + gn]) : CT{0, 0};
            };
            fold_kloop<T, BM, BN, BK, NS>(t, K, la, lb, sA, sB);
        } else {
            auto la = [&](int mm, int gk) -> CT {
                const int gm = m0 + mm;
                return (gm < K && gk < K) ? cvt<T>(Mp[(long long)gm * K + gk]) : CT{0, 0};
            };
            auto lb = [&](int gk, int nn) -> CT {
                const int gn = n0 + nn;
                if (gk >= K || gn >= rows) return CT{0, 0};
                return fold2<T>(D[(long long)gk * ld + gn], D[(long long)(n - 1 - gk) * ld + gn], skew);
            };
            fold_kloop<T, BM, BN, BK, NS>(t, K, la, lb, sA, sB);
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
                        if (gm < rows && gn < K) C[(long long)gm * ld + off + gn] = pack<TC, T>(re, im);
                    } else {
                        if (gm < K && gn < rows) C[(long long)(off + gm) * ld + gn] = pack<TC, T>(re, im);
                    }
                }
            }
    } else {
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
            const int K = q ? ma : ms, off = q ? ms : 0;
            const TM *Mq = q ? Ma : Ms;
            if constexpr (MODE == FOLD_XI) {
                auto la = [&](int mm, int gk) -> CT {
                    const int gm = m0 + mm;
                    return (gm < rows && gk < K) ? cvt<T>(D[(long long)gm * ld + off + gk]) : CT{0, 0};
                };
                auto lb = [&](int gk, int nn) -> CT {
                    const int gn = n0 + nn;
                    return (gk < K && gn < K) ? cvt<T>(Mq[(long long)gk * K + gn]) : CT{0, 0};
                };
                fold_kloop<T, BM, BN, BK, NS>(t, K, la, lb, sA, sB);
            } else {
                auto la = [&](int mm, int gk) -> CT {
                    const int gm = m0 + mm;
                    return (gm < K && gk < K) ? cvt<T>(Mq[(long long)gm * K + gk]) : CT{0, 0};
                };
                auto lb = [&](int gk, int nn) -> CT {
                    const int gn = n0 + nn;
                    return (gk < K && gn < rows) ? cvt<T>(D[(long long)(off + gk) * ld + gn]) : CT{0, 0};
                };
                fold_kloop<T, BM, BN, BK, NS>(t, K, la, lb, sA, sB);
            }
            if (q == 0) {
                // park P in this thread's own output slots (first half of the axis; the skew results go to the
                // disjoint second half) instead of holding a second accumulator set in registers
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
                            C[(long long)gm * ld + gn] = pack<TC, T>(re, im);
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
                    const TC pv = *c;
                    const T p0 = (T)pv.x, p1 = (T)pv.y;
                    const int h = MODE == FOLD_XI ? gn : gm;     // position along the transformed axis
                    if (h < ma) {
                        *c = pack<TC, T>(p0 + re, p1 + im);
                        TC *mirror = MODE == FOLD_XI ? C + (long long)gm * ld + (n - 1 - gn)
                                                     : C + (long long)(n - 1 - gm) * ld + gn;
                        *mirror = pack<TC, T>(p0 - re, p1 - im);
                    }
                }
    }
}

template <int MODE, typename TD, typename TM, typename TC, typename T, int BM, int BN, int BK>
hipError_t fold_launch_tile(const FoldDesc &f, const TD *D, const TM *Ms, const TM *Ma, TC *C, hipStream_t s) {
    const long long tiles = fold_tiles<MODE, BM, BN>(f);
    if (tiles == 0) return hipSuccess;
    const long long grid = 8 * ((tiles + 7) / 8);
    hipLaunchKernelGGL((k_fold<MODE, TD, TM, TC, T, BM, BN, BK>), dim3((unsigned)grid), dim3(256), 0, s, D, Ms, Ma, C, f);
    return hipGetLastError();
}

template <int MODE, typename TD, typename TM, typename TC, typename T>
hipError_t fold_launch_cfg(const FoldDesc &f, const TD *D, const TM *Ms, const TM *Ma, TC *C, hipStream_t s, int cfg) {
    switch (cfg) {
    case 1: return fold_launch_tile<MODE, TD, TM, TC, T, 64, 64, 32>(f, D, Ms, Ma, C, s);
    case 2: return fold_launch_tile<MODE, TD, TM, TC, T, 128, 64, 16>(f, D, Ms, Ma, C, s);
    case 3: return fold_launch_tile<MODE, TD, TM, TC, T, 64, 128, 16>(f, D, Ms, Ma, C, s);
    default: return fold_launch_tile<MODE, TD, TM, TC, T, 64, 64, 16>(f, D, Ms, Ma, C, s);
    }
}

}  // namespace

hipError_t launch_gemm_z64(const GemmDesc &d, const double2 *A, const double2 *B, double2 *C, hipStream_t s, int rw,
                           int cfg) {
    return launch<double2, double2, double2, double>(d, A, B, C, s, rw, cfg);
}
hipError_t launch_gemm_z32(const GemmDesc &d, const float2 *A, const float2 *B, float2 *C, hipStream_t s, int rw,
                           int cfg) {
    return launch<float2, float2, float2, float>(d, A, B, C, s, rw, cfg);
}
hipError_t launch_gemm_z32_in64(const GemmDesc &d, const double2 *A, const float2 *B, float2 *C, hipStream_t s,
                                int rw, int cfg) {
    return launch<double2, float2, float2, float>(d, A, B, C, s, rw, cfg);
}
hipError_t launch_gemm_z32_out64(const GemmDesc &d, const float2 *A, const float2 *B, double2 *C, hipStream_t s,
                                 int rw, int cfg) {
    return launch<float2, float2, double2, float>(d, A, B, C, s, rw, cfg);
}

}  // namespace helm

namespace helm {

hipError_t launch_fold_z64(int mode, const FoldDesc &f, const double2 *D, const double2 *Ms, const double2 *Ma,
                           double2 *C, hipStream_t s, int cfg) {
    switch (mode) {
    case FOLD_XF: return fold_launch_cfg<FOLD_XF, double2, double2, double2, double>(f, D, Ms, Ma, C, s, cfg);
    case FOLD_YF: return fold_launch_cfg<FOLD_YF, double2, double2, double2, double>(f, D, Ms, Ma, C, s, cfg);
    case FOLD_XI: return fold_launch_cfg<FOLD_XI, double2, double2, double2, double>(f, D, Ms, Ma, C, s, cfg);
    case FOLD_YI: return fold_launch_cfg<FOLD_YI, double2, double2, double2, double>(f, D, Ms, Ma, C, s, cfg);
    default: return hipErrorInvalidValue;
    }
}
hipError_t launch_fold_z32(int mode, const FoldDesc &f, const float2 *D, const float2 *Ms, const float2 *Ma, float2 *C,
                           hipStream_t s, int cfg) {
    switch (mode) {
    case FOLD_YF: return fold_launch_cfg<FOLD_YF, float2, float2, float2, float>(f, D, Ms, Ma, C, s, cfg);
    case FOLD_XI: return fold_launch_cfg<FOLD_XI, float2, float2, float2, float>(f, D, Ms, Ma, C, s, cfg);
    case FOLD_YI: return fold_launch_cfg<FOLD_YI, float2, float2, float2, float>(f, D, Ms, Ma, C, s, cfg);
    default: return hipErrorInvalidValue;
    }
}
hipError_t launch_fold_z32_in64(int mode, const FoldDesc &f, const double2 *D, const float2 *Ms, const float2 *Ma,
                                float2 *C, hipStream_t s, int cfg) {
    if (mode != FOLD_XF) return hipErrorInvalidValue;
    return fold_launch_cfg<FOLD_XF, double2, float2, float2, float>(f, D, Ms, Ma, C, s, cfg);
}
hipError_t launch_fold_z32_out64(int mode, const FoldDesc &f, const float2 *D, const float2 *Ms, const float2 *Ma,
                                 double2 *C, hipStream_t s, int cfg) {
    if (mode != FOLD_XI) return hipErrorInvalidValue;
    return fold_launch_cfg<FOLD_XI, float2, float2, double2, float>(f, D, Ms, Ma, C, s, cfg);
}

}  // namespace helm
