// Internal declarations of libhelm: the context, kernel launchers and parameter blocks.
#pragma once

#include <complex>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/helm.h"

namespace helm {

using cd = std::complex<double>;

bool eig_lambda_bar(int n, cd gamma, std::vector<cd> &d, std::vector<cd> &V, std::vector<cd> &Vinv,
                    std::string &err, double zeta = 1.0);

// Lambda-bar = Q diag(Vs, Va) diag(ds, da) diag(Vsi, Vai) Q^T with Q the symmetric/skew butterfly (Lambda-bar is
// centrosymmetric); blocks row-major, ms = ceil(n/2), ma = floor(n/2). The modes of eig_lambda_bar are [ds, da].
struct EigFold {
    int n = 0, ms = 0, ma = 0;
    std::vector<cd> ds, Vs, Vsi, da, Va, Vai;
};
bool eig_lambda_bar_folded(int n, cd gamma, double zeta, EigFold &f, std::string &err);
// the dense V, V^{-1} and eigenvalues of a folded decomposition (what eig_lambda_bar returns)
void eig_fold_dense(const EigFold &f, std::vector<cd> &d, std::vector<cd> &V, std::vector<cd> &Vinv);

// Stencil coefficients that depend only on the grid (the k^2-dependent parts are per node).
// Matvec thread block: 64 x STENCIL_TY threads, one output column each; the z-chunk length is chosen so that a
// launch holds about STENCIL_WAVES waves in total, but no shorter than STENCIL_MINZ planes.
constexpr int STENCIL_TY = 8;
constexpr int STENCIL_WAVES = 8192;
constexpr int STENCIL_MINZ = 8;   // shortest z-chunk: each chunk reads two halo planes

struct StencilParams {
    int nx, ny, nz;
    int order;
    double2 gx, gy, gz;          // ghost factors per axis
    // order 2/4: constant coefficients
    double c_center;             // centre coefficient without the k^2 part
    double c_face[3];            // face coefficient per axis without the k^2 part
    double c_edge[3];            // edge coefficients for axis pairs (x,y), (x,z), (y,z)
    double w_center, w_face;     // k^2 U weights: centre and face (order 4: 1/2, 1/12; order 2: 1, 0)
    // order 6 (uniform h)
    double c1;                   // 1/(30 h^2)
    double h2;                   // h^2
    int zchunk;                  // z-planes per block
    int tiles_x, tiles_y, zchunks;
    // complex k^2 (NULL for real k^2): imaginary parts of k^2 and of the order-6 field block
    const double *k2i;
    const double4 *fldi;
};

// Complex GEMM description: C[b] = A[b] * B[b], row-major, complex, strides in complex elements.
struct GemmDesc {
    int M, N, K;
    long long lda, ldb, ldc;
    long long sA, sB, sC;        // batch strides (0 = shared operand)
    int batch;
};

// Folded EigT transform (Lambda-bar centrosymmetric: V = Q diag(Vs, Va), modes [symmetric | skew]) over the
// length-n axis of the data: x (rows = lines, each a contiguous row of n) or y (rows = columns x of a slice, the
// axis strided by ld; batch slices sD apart). Data and result share the layout.
struct FoldDesc {
    int n, ms, ma;               // axis length, ceil(n/2), floor(n/2)
    int rows;                    // x: number of lines; y: columns per slice
    long long ld;                // stride between consecutive rows (x) or axis positions (y)
    long long sD;                // slice stride (y)
    int batch;                   // slices (y; 1 for x)
    int moff, mstep;             // where the modes live: symmetric mode k at k * mstep, skew mode k at moff +
                                 // k * mstep ([symmetric | skew]: moff = ms, mstep = 1; the sine basis keeps its
                                 // natural order, even modes symmetric and odd ones skew: moff = 1, mstep = 2)
};
// the blocks of one axis, row-major: forward (x: [position][mode], y: [mode][position]) and inverse
// (x: [mode][position], y: [position][mode]), each for the symmetric (ms x ms) and skew (ma x ma) half
template <typename CT> struct FoldMats {
    CT *fs = nullptr, *fa = nullptr, *is = nullptr, *ia = nullptr;
};
enum { FOLD_XF = 0, FOLD_YF = 1, FOLD_XI = 2, FOLD_YI = 3 };
// tiles of a folded transform with bm x bn output tiles: the forward ones cover both halves' outputs, the inverse
// ones the first half of the positions (each writes its mirror too)
__host__ __device__ inline long long fold_tile_count(int mode, const FoldDesc &f, int bm, int bn) {
    const long long tm = (f.rows + bm - 1) / bm, tn = (f.rows + bn - 1) / bn;
    const long long hs_m = (f.ms + bm - 1) / bm, ha_m = (f.ma + bm - 1) / bm;
    const long long hs_n = (f.ms + bn - 1) / bn, ha_n = (f.ma + bn - 1) / bn;
    if (mode == FOLD_XF) return tm * (hs_n + ha_n);
    if (mode == FOLD_YF) return (long long)f.batch * (hs_m + ha_m) * tn;
    if (mode == FOLD_XI) return tm * hs_n;
    return (long long)f.batch * hs_m * tn;
}
hipError_t launch_fold_z64(int mode, const FoldDesc &f, const double2 *D, const double2 *Ms, const double2 *Ma,
                           double2 *C, hipStream_t s, int cfg, bool real = false);
hipError_t launch_fold_z32(int mode, const FoldDesc &f, const float2 *D, const float2 *Ms, const float2 *Ma, float2 *C,
                           hipStream_t s, int cfg, bool real = false);
hipError_t launch_fold_z32_in64(int mode, const FoldDesc &f, const double2 *D, const float2 *Ms, const float2 *Ma,
                                float2 *C, hipStream_t s, int cfg, bool real = false);
hipError_t launch_fold_z32_out64(int mode, const FoldDesc &f, const float2 *D, const float2 *Ms, const float2 *Ma,
                                 double2 *C, hipStream_t s, int cfg, bool real = false);
// real = true: the blocks are real (their imaginary parts are ignored), two real MFMA products per complex MAC

// symbol of the compact operators with constant k0 (FFT4 / FFT6): order, h_a^2 per axis, k0^2
struct SymParams {
    int order;
    double h2[3];
    double k2;
};
hipError_t launch_sym_divide_z64(double2 *u, const double *tx, const double *ty, const double *tz, int nx, int ny,
                                 int nz, const SymParams &q, hipStream_t s);
hipError_t launch_sym_divide_z32(float2 *u, const double *tx, const double *ty, const double *tz, int nx, int ny,
                                 int nz, const SymParams &q, hipStream_t s);

// PFFT second path (Sec. 4.2): sine matrices, Dirichlet eigenvalues, the plain/transposed eigenvector
// matrices the thin ring transforms need, and work buffers. FP64 and FP32 copies.
template <typename CT> struct PfftMats {
    CT *Sx = nullptr, *Sy = nullptr;             // orthonormal sine matrices (symmetric; imaginary part 0)
    FoldMats<CT> fsx, fsy, fsz;                  // the sine transforms (z for FFT4 / FFT6 only) as folded real
                                                 // blocks (even modes symmetric, odd ones skew; natural order)
    CT *Vxi = nullptr, *Vx = nullptr;            // V_x^{-1}, V_x row-major (the transposes are BxF, BxI)
    CT *VyiT = nullptr, *VyT = nullptr;          // transposes of V_y^{-1}, V_y (the plain ones are AyF, AyI)
    CT *yhat = nullptr;                          // sine transform of the input (reused in step 3)
    CT *ringT = nullptr, *ringW = nullptr;       // face values of Theta and W, (2 Nx + 2 Ny) per slice
    CT *rpart = nullptr, *sv = nullptr, *rsum = nullptr;   // ring inverse work: row-group partials, row sums, their total
    CT *rbuf = nullptr, *fvec = nullptr;                   // ring forward work: face data R, factors S and T
};
struct PfftPlan {
    double2 *dFx = nullptr, *dFy = nullptr;      // Dirichlet eigenvalues 2 cos(pi i/(N+1))
    double *tx = nullptr, *ty = nullptr, *tz = nullptr;   // (2 cos(pi i/(N+1)) - 2) / h^2 per axis (FFT4 / FFT6)
    PfftMats<double2> m64;
    PfftMats<float2> m32;
};

// basis vectors are KRYLOV_PAD elements longer than n so that equal indices of different vectors do not share
// DRAM address bits above the vector size
constexpr long long KRYLOV_PAD = 2048;

// pivot table of the partitioned z-solve: complex128 for the FP64 kernel, its complex64 rounding for the FP32 one
struct TriPiv {
    double2 *d = nullptr;
    float2 *f = nullptr;
};

struct KrylovWork {
    int m = 0;
    long long ld = 0;            // leading dimension of V and Z (n + KRYLOV_PAD)
    int flexible = 0;
    double2 *V = nullptr;        // (m+1) * n
    double2 *Z = nullptr;        // m * n (flexible only)
    float2 *Zf = nullptr;        // m * n complex64 instead of Z when the preconditioner runs in FP32: its outputs
                                 // are FP32 values, so this storage is exact
    double2 *tmp = nullptr;      // n
    double2 *partials = nullptr; // nblocks * (m + 2)
    double2 *red = nullptr;      // m + 2 reduced values
    double2 *red_host = nullptr; // pinned host copy
    int nblocks = 0;
    hipStream_t aux = nullptr;   // copies the reduced values to the host while the solve stream runs on
    hipEvent_t red_ev = nullptr, copy_ev = nullptr;
};

struct ProfPending { int cls; double work; hipEvent_t a, b; bool own_a; };   // own_a: a is not the previous b

struct Ctx {
    int nx, ny, nz;
    long long n;
    double hx, hy, hz;
    int order;
    int bc_kind;
    double k0;
    cd gamma[3];
    double zeta = 1.0;           // corner off-diagonal of Lambda-bar (2 for the collocated closure)
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;

    StencilParams sp{};
    double *k2 = nullptr;        // interior k^2 (n)
    double4 *fld = nullptr;      // order 6: (diag, g_x, g_y, g_z) per node
    double *k2i = nullptr;       // complex k^2 only: imaginary parts of k^2 and of the field block
    double4 *fldi = nullptr;

    // dense eigenvector matrices (complex, row-major N x N; x: transposed, y: as is), which PFFT's face corrections use
    double2 *BxF = nullptr, *BxI = nullptr, *AyF = nullptr, *AyI = nullptr;
    float2 *BxF32 = nullptr, *BxI32 = nullptr, *AyF32 = nullptr, *AyI32 = nullptr;
    // the same transforms as symmetric / skew half blocks (what the single-problem preconditioner applies)
    FoldMats<double2> fx64, fy64;
    FoldMats<float2> fx32, fy32;
    double2 *dxe = nullptr, *dye = nullptr;    // eigenvalues d_x,i and d_y,j
    double ax, ay, c0;                          // alpha_x, alpha_y, h_z^2 k0^2 - 2(alpha_x + alpha_y + 1)
    int gemm_cfg[4] = {0, 0, 0, 0};             // tile configuration of the x64, y64, x32, y32 forward transforms
    int gemm_cfg_inv[4] = {0, 0, 0, 0};         // and of the inverse ones

    // preconditioner work buffers
    double2 *t1 = nullptr, *t2 = nullptr;
    float2 *t1f = nullptr, *t2f = nullptr;
    TriPiv tpiv_eig, tpiv_dir;   // pivots entering each z-chunk (absorbing / Dirichlet x-y eigenvalues)
    TriPiv tpiv_fft2;            // the same for Dirichlet x-y eigenvalues and a Dirichlet z closure
    double2 *sg_y = nullptr, *sg_part = nullptr, *sg_red = nullptr, *sg_host = nullptr;   // helm_scale_guess work

    PfftPlan *pfft = nullptr;
    std::vector<cd> hVx, hVxi, hVy, hVyi;        // host copies of the eigenvector matrices (PFFT plan build)
    KrylovWork kw;
    std::vector<void *> allocs;  // everything to free

    // per-kernel timing
    bool prof = false;
    double prof_ms[HELM_K_COUNT] = {};
    long long prof_n[HELM_K_COUNT] = {};
    double prof_work[HELM_K_COUNT] = {};
    std::vector<ProfPending> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    hipEvent_t prof_last = nullptr;   // end event of the last timed launch (the next one's start while it is pending)
};

// Events that only time work: no system-scope fence when recorded. With the default fence every record writes back
// and invalidates the caches, which costs a few microseconds per record and slows the kernel after it; nothing is
// read through these events (results reach the host through stream synchronisation).
inline hipError_t timing_event(hipEvent_t *e) { return hipEventCreateWithFlags(e, hipEventDisableSystemFence); }

// Launch through `fn` (returning hipError_t), bracketed by profiling events when enabled. Launches that follow each
// other on the stream share events: the end of one is the start of the next (one record per launch). A fresh start
// is recorded when the previous end has already completed, i.e. when the stream may have been idle in between (a
// host synchronisation), so that idle time is not counted as kernel time. Wherever other stream work can run
// between two timed launches (an untimed kernel or copy, the caller's own work between library calls) the chain
// is broken first with prof_gap.
inline void prof_gap(Ctx &c) { c.prof_last = nullptr; }
inline hipError_t prof_event(Ctx &c, hipEvent_t *e) {
    if (!c.prof_pool.empty()) {
        *e = c.prof_pool.back();
        c.prof_pool.pop_back();
        return hipSuccess;
    }
    return timing_event(e);
}
template <typename F> hipError_t timed(Ctx &c, int cls, double work, F fn) {
    if (!c.prof) return fn();
    hipEvent_t a = c.prof_last, b = nullptr;
    const bool own_a = !a || hipEventQuery(a) != hipErrorNotReady;
    hipError_t e;
    // on an error the events taken here go back to the pool and the chain is broken
    auto fail = [&](hipError_t err) {
        if (own_a && a) c.prof_pool.push_back(a);
        if (b) c.prof_pool.push_back(b);
        c.prof_last = nullptr;
        return err;
    };
    if (own_a) {
        a = nullptr;
        if ((e = prof_event(c, &a)) != hipSuccess) return fail(e);
        if ((e = hipEventRecord(a, c.stream)) != hipSuccess) return fail(e);
    }
    if ((e = fn()) != hipSuccess) return fail(e);
    if ((e = prof_event(c, &b)) != hipSuccess) return fail(e);
    if ((e = hipEventRecord(b, c.stream)) != hipSuccess) return fail(e);
    c.prof_pending.push_back({cls, work, a, b, own_a});
    c.prof_last = b;
    return hipSuccess;
}

// Accumulate every completed pending pair (call after a stream synchronisation). Each event returns to the pool
// once: the b of every pair, and the a of pairs that recorded their own start.
inline void prof_resolve(Ctx &c) {
    for (auto &p : c.prof_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c.prof_ms[p.cls] += ms;
            c.prof_n[p.cls] += 1;
            c.prof_work[p.cls] += p.work;
        }
        if (p.own_a) c.prof_pool.push_back(p.a);
        c.prof_pool.push_back(p.b);
    }
    c.prof_pending.clear();
    c.prof_last = nullptr;
}

// Classical Gram-Schmidt takes the norm of the orthogonalised vector from ||y||^2 - sum |h_i|^2, whose rounding error
// is about eps ||y||^2. A step takes a second Gram-Schmidt pass only when that norm squared falls below
// CGS_REORTH ||y||^2: above it the norm is accurate to ~eps / CGS_REORTH and the new basis vector's loss of
// orthogonality is ~eps / sqrt(CGS_REORTH). (On the 128^3 four-inclusion medium one in two steps falls below half of
// ||y||^2; a second pass for them left every iteration count and every solution unchanged to 1e-13 and cost 30%.)
constexpr double CGS_REORTH = 1e-2;
// the threshold in force: HELM_CGS_REORTH from the environment when it holds a number in (0, 1), else CGS_REORTH
double cgs_reorth();

// ----- batched solves: per-problem descriptors and device-side GMRES state -----
struct BProb {                    // constant during a batched solve
    StencilParams sp;
    const double *k2;
    const double4 *fld;
    const void *xfs, *xfa, *xis, *xia;     // folded transform blocks (double2* or float2* by precision): x forward /
    const void *yfs, *yfa, *yis, *yia;     // inverse and y forward / inverse, symmetric and skew halves
    const double2 *dxe, *dye;
    double ax, ay, c0, hz2;
    double2 gz;
    FoldDesc fx, fy;
    double2 *V, *x;
    void *Z;                               // FGMRES directions: complex64 with the FP32 preconditioner (its outputs
                                           // are FP32 values, so this storage is exact), complex128 otherwise
    const double2 *F;
    void *t1, *t2;                         // preconditioner work (element type by precision)
    const double2 *tpiv;                   // pivots entering each z-chunk (the context's table)
    const float2 *tpiv32;                  // the same rounded to complex64 (FP32 z-solve)
    double2 *part;                         // inner-product partials, nblk_dots * (m + 2)
    long long n;
    int nx, ny, nz, nblk_dots;
};
struct BState {                   // evolves on the device
    double bnorm, beta, relres_est, relres_true;
    double2 alpha;                // scale of the base vector in the next linear combination
    int active;                   // 1 while the problem takes Arnoldi steps in the current cycle
    int done;                     // converged or out of iterations
    int converged, k, its, cycles, cancel;
    int reo;                      // 1 while the current Arnoldi step takes its second Gram-Schmidt pass
};
struct BParams { double rtol; int maxit; int m; double reorth; };
struct BArrays {                  // per-problem small arrays, problem p at p * stride
    double2 *H;                   // (m+1) x m Hessenberg (rotated), row-major
    double *cs;                   // m
    double2 *sn, *g, *coef;       // m, m+1, m+1
};
struct BOffsets {                 // prefix sums of blocks/tiles per problem for each grouped launch
    int *mv, *tri, *dot, *lc;     // np + 1 each
    int *mvp;                     // nunits + 1: blocks of the step matvec per unit (one problem or two sharing an
                                  // operator)
    long long *g[4];              // tiles of the x forward, y forward, y inverse and x inverse transforms
};

// ----- kernel launchers (defined in the .hip files); all enqueue on `s` and return hipError_t -----
// complex k^2 (complex128 samples with the same halo): real and imaginary parts into separate arrays
hipError_t launch_derived_fields_c(const double2 *k2_halo, int halo, double *k2, double *k2i, double4 *fld,
                                   double4 *fldi, const StencilParams &p, double h, hipStream_t s);
hipError_t launch_derived_fields(const double *k2_halo, int halo, double *k2, double4 *fld, const StencilParams &p,
                                 double h, hipStream_t s);
hipError_t launch_matvec(const StencilParams &p, const double2 *x, const double *k2, const double4 *fld,
                         const double2 *F, double2 *y, hipStream_t s);
// the same with a complex64 input (widened exactly to complex128 on load)
hipError_t launch_matvec(const StencilParams &p, const float2 *x, const double *k2, const double4 *fld,
                         const double2 *F, double2 *y, hipStream_t s);   // F != nullptr: y = F - A x
hipError_t launch_rhs(const StencilParams &p, const double2 *f_halo, const double *k2, const double4 *fld,
                      double h3[3], double2 *F, hipStream_t s);

// Transform tile configurations 0..GEMM_NCFG-1 = (BM, BN, BK) of (64,64,16), (64,64,32), (128,64,16), (64,128,16).
constexpr int GEMM_NCFG = 4;
// C0 = A0 B0 and C1 = A1 B1 (complex operands, 32 x 32 x 32 tiles) in one launch
hipError_t launch_gemm_pair_z64(const GemmDesc &d0, const double2 *A0, const double2 *B0, double2 *C0,
                                const GemmDesc &d1, const double2 *A1, const double2 *B1, double2 *C1, hipStream_t s);
hipError_t launch_gemm_pair_z32(const GemmDesc &d0, const float2 *A0, const float2 *B0, float2 *C0,
                                const GemmDesc &d1, const float2 *A1, const float2 *B1, float2 *C1, hipStream_t s);

// `in` (may equal r) supplies the right-hand side; the solution is written to r.
int tri_chunks(int nz);
hipError_t launch_tri_pivots(const double2 *dx, const double2 *dy, int nx, int ny, int nz, double ax, double ay,
                             double c0, double2 gz, double2 *piv, float2 *piv32, hipStream_t s, double zi = 1.0);
hipError_t launch_tridiag_chunk_z64(const double2 *in, double2 *out, const double2 *piv, const double2 *dx,
                                    const double2 *dy, int nx, int ny, int nz, double ax, double ay, double c0,
                                    double2 gz, double scale, hipStream_t s, double zi = 1.0);
hipError_t launch_tridiag_chunk_z32(const float2 *in, float2 *out, const float2 *piv, const double2 *dx,
                                    const double2 *dy, int nx, int ny, int nz, double ax, double ay, double c0,
                                    double2 gz, double scale, hipStream_t s, double zi = 1.0);
int ring_rowgroups();
int ring_max_n();            // widest N_x the PFFT ring pass supports
// layer 0: the face rows 1, N_y and columns 1, N_x; layer 1: rows 2, N_y - 1 and columns 2, N_x - 1 (zeta != 1)
hipError_t launch_ring_inverse_z64(const double2 *Xh, double2 *ring, const double2 *Vy, const double2 *VyT,
                                   const double2 *Vx, const double2 *VxT, int nx, int ny, int nz, int layer,
                                   double2 *rpart, double2 *sv, double2 *rsum, hipStream_t s);
hipError_t launch_ring_inverse_z32(const float2 *Xh, float2 *ring, const float2 *Vy, const float2 *VyT,
                                   const float2 *Vx, const float2 *VxT, int nx, int ny, int nz, int layer,
                                   float2 *rpart, float2 *sv, float2 *rsum, hipStream_t s);
// ra1, rb1: the second-layer rings (zeta != 1) or null; ex1, ey1 = -a (zeta - 1) per axis
hipError_t launch_ring_forward_z64(const double2 *ra, const double2 *rb, const double2 *ra1, const double2 *rb1,
                                   const double2 *base, double base_scale, double2 *out, const double2 *WyT,
                                   const double2 *WxT, double2 ex, double2 ey, double2 ex1, double2 ey1, int nx,
                                   int ny, int nz, double2 *rbuf, double2 *fvec, hipStream_t s);
hipError_t launch_ring_forward_z32(const float2 *ra, const float2 *rb, const float2 *ra1, const float2 *rb1,
                                   const float2 *base, double base_scale, float2 *out, const float2 *WyT,
                                   const float2 *WxT, double2 ex, double2 ey, double2 ex1, double2 ey1, int nx, int ny,
                                   int nz, float2 *rbuf, float2 *fvec, hipStream_t s);

// Krylov helpers
int dots_blocks(long long n);
hipError_t launch_dots(const double2 *V, long long ldv, int nv, const double2 *w, long long n, double2 *partials,
                       int nblocks, double2 *red, hipStream_t s);   // red[0..nv-1] = V_i^H w, red[nv] = (|w|^2, 0)
hipError_t launch_lincomb(double2 *out, const double2 *base, double2 alpha, const double2 *V, long long ldv, int nv,
                          const double2 *coef, long long n, hipStream_t s);
// the same over complex64 vectors V (the complex64 Z basis of FGMRES with the FP32 preconditioner)
hipError_t launch_lincomb(double2 *out, const double2 *base, double2 alpha, const float2 *V, long long ldv, int nv,
                          const double2 *coef, long long n, hipStream_t s);
// w <- -(w - V h)/eta with h = red[0..nv-1], eta^2 = red[nv].x - sum |h_i|^2 computed on the device (unscaled when
// eta^2 <= red[nv].x / 2, which the caller detects and corrects with a second pass)
hipError_t launch_lincomb_cgs(double2 *w, const double2 *V, long long ldv, int nv, const double2 *red, long long n,
                              double reorth, hipStream_t s);   // out = alpha base + sum coef_i V_i
hipError_t launch_to_c64(const double2 *x, float2 *y, long long n, hipStream_t s);   // complex128 -> complex64
hipError_t launch_fill_zero(double2 *x, long long n, hipStream_t s);

// grouped (batched) launches; see k_batch.hip
struct BLaunch {
    const BProb *P;               // device array of np descriptors
    BState *st;                   // device array of np states
    const BParams *prm;           // device
    BArrays a;
    BOffsets off;                 // device arrays
    int np, m, order, fp32;
    const int2 *units;                          // device: the step matvec's units (p, p2), p2 = -1 when alone
    int nunits;
    int tot_mv, tot_tri, tot_dot, tot_lc;       // total blocks per grouped launch
    int tot_mvp;                                // total blocks of the step matvec over the units
    long long tot_g[4];                         // total transform tiles per role
    int gemm_grid;                              // persistent GEMM grid size
    int cfg[4];                                 // tile configurations of the four transform roles
    int tri_lx, tri_pb;                         // z-solve block: tri_lx lines x tri_pb chunks
};
inline void gemm_cfg_tile(int cfg, int &bm, int &bn) {
    bm = cfg == 2 ? 128 : 64;
    bn = cfg == 3 ? 128 : 64;
}
helm_status ctx_tri_pivots(Ctx &c);   // pivot table of the partitioned z-solve (built once per context)
// the FP32 EigT preconditioner with caller-given staging vectors (n complex64 each); allocates nothing
helm_status eigt32_apply_ws(Ctx &c, const double2 *y, double2 *z, float2 *t1f, float2 *t2f);
hipError_t bl_init(const BLaunch &L, hipStream_t s);                 // ||F||, state reset (outside graphs)
hipError_t bl_zero_x(const BLaunch &L, hipStream_t s);
hipError_t bl_cycle(const BLaunch &L, hipStream_t s);                // one restart cycle: restart + m steps + update
hipError_t bl_restart(const BLaunch &L, hipStream_t s);              // the restart test alone

}  // namespace helm

struct helm_ctx { helm::Ctx c; };
