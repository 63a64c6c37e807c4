// Complex transforms on MFMA (row-major, interleaved complex), FP64 or FP32 arithmetic.
//
// The EigT transforms (Sec. 4.1, eq. EIG_SOLVER Steps 2 and 4) contract every x-line and every y-line with the
// 1D eigenvector matrices:
//   x-transform: C[c][p] = sum_q Y[c][q] W^T[q][p]       lines c = (j, l) are rows (lda = Nx);
//   y-transform: C_l[j][i] = sum_m W[j][m] Y_l[m][i]      per slice l, the data is the B operand (ldb = Nx).
// In both the fastest memory index of the data lands on the MFMA column index, so tile loads and the
// accumulator stores walk contiguous memory. They run as the folded kernels below (k_fold: two half-size
// products per axis), and so do the sine transforms of PFFT and of the FFT2/4/6 comparison preconditioners (real
// blocks, modes at stride 2). A paired product kernel (k_zgemm_pair: two independent products C = A B in one
// launch) carries PFFT's thin face-ring products.
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

// Two independent products in one launch (PFFT's row and column face products, 2 N_z x N by N x N each): the
// tiles of the first product, then those of the second, mapped to XCDs together. 32 x 32 tiles: with 64 x 64 ones
// the products made a few dozen tiles, each a whole CU's matrix work for 10 us (FP32) or 27 us (FP64), and left
// most of the chip idle.
template <typename CT, typename T, int BM, int BN, int BK>
__global__ __launch_bounds__(256) void k_zgemm_pair(const CT *__restrict__ A0, const CT *__restrict__ B0,
                                                    CT *__restrict__ C0, GemmDesc d0, const CT *__restrict__ A1,
                                                    const CT *__restrict__ B1, CT *__restrict__ C1, GemmDesc d1) {
    const long long t0 = (long long)((d0.M + BM - 1) / BM) * ((d0.N + BN - 1) / BN) * d0.batch;
    const long long t1 = (long long)((d1.M + BM - 1) / BM) * ((d1.N + BN - 1) / BN) * d1.batch;
    const long long total = t0 + t1;
    const long long per = (total + 7) / 8;
    const long long tile = (long long)(blockIdx.x % 8) * per + blockIdx.x / 8;   // consecutive tiles on one XCD
    if (tile >= total) return;
    const bool second = tile >= t0;
    gemm_tile<CT, CT, CT, T, BM, BN, BK, 0>(second ? A1 : A0, second ? B1 : B0, second ? C1 : C0, second ? d1 : d0,
                                           second ? tile - t0 : tile);
}

template <typename CT, typename T>
hipError_t launch_pair(const GemmDesc &d0, const CT *A0, const CT *B0, CT *C0, const GemmDesc &d1, const CT *A1,
                       const CT *B1, CT *C1, hipStream_t s) {
    constexpr int BM = 32, BN = 32, BK = 32;
    const long long tiles = (long long)((d0.M + BM - 1) / BM) * ((d0.N + BN - 1) / BN) * d0.batch +
                            (long long)((d1.M + BM - 1) / BM) * ((d1.N + BN - 1) / BN) * d1.batch;
    if (tiles == 0) return hipSuccess;
    const long long grid = 8 * ((tiles + 7) / 8);
    hipLaunchKernelGGL((k_zgemm_pair<CT, T, BM, BN, BK>), dim3((unsigned)grid), dim3(256), 0, s, A0, B0, C0, d0, A1, B1,
                       C1, d1);
    return hipGetLastError();
}

// RW = 0: complex blocks; RW = 1 / 2: real blocks (the sine basis) as the A (y) / B (x) operand
template <int MODE, typename TD, typename TM, typename TC, typename T, int BM, int BN, int BK, int RW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(fold_waves<T, TD, MODE, BM, BN, BK>()))) void k_fold(
    const TD *__restrict__ D, const TM *__restrict__ Ms, const TM *__restrict__ Ma, TC *__restrict__ C, FoldDesc f) {
    const long long total = fold_tiles<MODE, BM, BN>(f);
    const long long per = (total + 7) / 8;
    const long long tile = (long long)(blockIdx.x % 8) * per + blockIdx.x / 8;   // consecutive tiles on one XCD
    if (tile >= total) return;
    fold_tile<MODE, TD, TM, TC, T, BM, BN, BK, RW>(D, Ms, Ma, C, f, tile);
}

template <int MODE, typename TD, typename TM, typename TC, typename T, int BM, int BN, int BK, int RW = 0>
hipError_t fold_launch_tile(const FoldDesc &f, const TD *D, const TM *Ms, const TM *Ma, TC *C, hipStream_t s) {
    const long long tiles = fold_tiles<MODE, BM, BN>(f);
    if (tiles == 0) return hipSuccess;
    const long long grid = 8 * ((tiles + 7) / 8);
    hipLaunchKernelGGL((k_fold<MODE, TD, TM, TC, T, BM, BN, BK, RW>), dim3((unsigned)grid), dim3(256), 0, s, D, Ms, Ma,
                       C, f);
    return hipGetLastError();
}

// real blocks (the sine basis): the block as the B operand of the x-transforms and the A operand of the
// y-transforms; 64 x 64 x 16 tiles, except the FP32 forward ones (64 x 128 along x, 128 x 64 along y, measured 1%
// faster on the 256^3 PFFT solve; in FP64 these larger tiles drop to one wave per SIMD and are slower)
template <int MODE, typename TD, typename TM, typename TC, typename T>
hipError_t fold_launch_cfg(const FoldDesc &f, const TD *D, const TM *Ms, const TM *Ma, TC *C, hipStream_t s, int cfg,
                           bool real) {
    if (real) {
        constexpr int RW = (MODE == FOLD_XF || MODE == FOLD_XI) ? 2 : 1;
        constexpr bool f32 = sizeof(T) == 4;
        if constexpr (f32 && MODE == FOLD_XF) return fold_launch_tile<MODE, TD, TM, TC, T, 64, 128, 16, RW>(f, D, Ms, Ma, C, s);
        else if constexpr (f32 && MODE == FOLD_YF) return fold_launch_tile<MODE, TD, TM, TC, T, 128, 64, 16, RW>(f, D, Ms, Ma, C, s);
        else return fold_launch_tile<MODE, TD, TM, TC, T, 64, 64, 16, RW>(f, D, Ms, Ma, C, s);
    }
    switch (cfg) {
    case 1: return fold_launch_tile<MODE, TD, TM, TC, T, 64, 64, 32>(f, D, Ms, Ma, C, s);
    case 2: return fold_launch_tile<MODE, TD, TM, TC, T, 128, 64, 16>(f, D, Ms, Ma, C, s);
    case 3: return fold_launch_tile<MODE, TD, TM, TC, T, 64, 128, 16>(f, D, Ms, Ma, C, s);
    default: return fold_launch_tile<MODE, TD, TM, TC, T, 64, 64, 16>(f, D, Ms, Ma, C, s);
    }
}

}  // namespace

hipError_t launch_gemm_pair_z64(const GemmDesc &d0, const double2 *A0, const double2 *B0, double2 *C0,
                                const GemmDesc &d1, const double2 *A1, const double2 *B1, double2 *C1, hipStream_t s) {
    return launch_pair<double2, double>(d0, A0, B0, C0, d1, A1, B1, C1, s);
}
hipError_t launch_gemm_pair_z32(const GemmDesc &d0, const float2 *A0, const float2 *B0, float2 *C0,
                                const GemmDesc &d1, const float2 *A1, const float2 *B1, float2 *C1, hipStream_t s) {
    return launch_pair<float2, float>(d0, A0, B0, C0, d1, A1, B1, C1, s);
}

}  // namespace helm

namespace helm {

hipError_t launch_fold_z64(int mode, const FoldDesc &f, const double2 *D, const double2 *Ms, const double2 *Ma,
                           double2 *C, hipStream_t s, int cfg, bool real) {
    switch (mode) {
    case FOLD_XF: return fold_launch_cfg<FOLD_XF, double2, double2, double2, double>(f, D, Ms, Ma, C, s, cfg, real);
    case FOLD_YF: return fold_launch_cfg<FOLD_YF, double2, double2, double2, double>(f, D, Ms, Ma, C, s, cfg, real);
    case FOLD_XI: return fold_launch_cfg<FOLD_XI, double2, double2, double2, double>(f, D, Ms, Ma, C, s, cfg, real);
    case FOLD_YI: return fold_launch_cfg<FOLD_YI, double2, double2, double2, double>(f, D, Ms, Ma, C, s, cfg, real);
    default: return hipErrorInvalidValue;
    }
}
hipError_t launch_fold_z32(int mode, const FoldDesc &f, const float2 *D, const float2 *Ms, const float2 *Ma, float2 *C,
                           hipStream_t s, int cfg, bool real) {
    switch (mode) {
    case FOLD_YF: return fold_launch_cfg<FOLD_YF, float2, float2, float2, float>(f, D, Ms, Ma, C, s, cfg, real);
    case FOLD_XI: return fold_launch_cfg<FOLD_XI, float2, float2, float2, float>(f, D, Ms, Ma, C, s, cfg, real);
    case FOLD_YI: return fold_launch_cfg<FOLD_YI, float2, float2, float2, float>(f, D, Ms, Ma, C, s, cfg, real);
    default: return hipErrorInvalidValue;
    }
}
hipError_t launch_fold_z32_in64(int mode, const FoldDesc &f, const double2 *D, const float2 *Ms, const float2 *Ma,
                                float2 *C, hipStream_t s, int cfg, bool real) {
    if (mode != FOLD_XF) return hipErrorInvalidValue;
    return fold_launch_cfg<FOLD_XF, double2, float2, float2, float>(f, D, Ms, Ma, C, s, cfg, real);
}
hipError_t launch_fold_z32_out64(int mode, const FoldDesc &f, const float2 *D, const float2 *Ms, const float2 *Ma,
                                 double2 *C, hipStream_t s, int cfg, bool real) {
    if (mode != FOLD_XI) return hipErrorInvalidValue;
    return fold_launch_cfg<FOLD_XI, float2, float2, double2, float>(f, D, Ms, Ma, C, s, cfg, real);
}

}  // namespace helm
