// Grouped kernels of the batched FGMRES solve: every launch covers all problems of a batch (uneven sizes
// included) through per-problem block or tile offsets, and every kernel skips problems that are not active.
// The Arnoldi inner-product reduction, Givens rotations and the least-squares solve run on the device, so one
// restart cycle (restart vector, m Arnoldi steps, x += Z y) is a fixed launch sequence that can be captured
// once in a hipGraph and replayed.
//
// Per Arnoldi step j (the same for every problem): EigT preconditioner z_j = M^{-1} v_j (four grouped GEMMs,
// the x- and y-transforms as one persistent launch each over all problems' tiles, and the grouped z-solves),
// the shifted matvec y = v_j - A z_j, the block inner products V^H y and ||y||^2, the device Arnoldi step
// (H column, Givens, residual estimate, stop test), and v_{j+1} = -(y - V h)/eta.
#include <type_traits>

#include "gemm_dev.h"
#include "krylov_dev.h"
#include "stencil_dev.h"
#include "tridiag_dev.h"

namespace helm {

namespace {

__device__ __forceinline__ int find_prob(const int *off, int np, int b) {
    int lo = 0, hi = np - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}
__device__ __forceinline__ int find_prob64(const long long *off, int np, long long b) {
    int lo = 0, hi = np - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------------------------- GEMMs
// ROLE 0: x-forward  t1 = V_j  W_xF       ROLE 1: y-forward  t2 = W_yF t1
// ROLE 2: y-inverse  t1 = W_yI t2         ROLE 3: x-inverse  Z_j = t1 W_xI
// (the folded transforms of the single-problem preconditioner: symmetric and skew half blocks of each axis)
template <int ROLE, typename T, int BM, int BN, int BK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    fold_waves<T, typename std::conditional<ROLE == 0, double2, typename cplx<T>::t>::type,
               ROLE == 0 ? FOLD_XF : ROLE == 1 ? FOLD_YF : ROLE == 2 ? FOLD_YI : FOLD_XI, BM, BN, BK>()))) void k_b_gemm(
    const BProb *__restrict__ P, const BState *__restrict__ st, const long long *__restrict__ toff, int np, int j) {
    typedef typename cplx<T>::t CT;
    const long long total = toff[np];
    for (long long t = blockIdx.x; t < total; t += gridDim.x) {
        const int p = find_prob64(toff, np, t);
        if (!st[p].active) continue;
        const BProb &q = P[p];
        const long long lt = t - toff[p];
        if (ROLE == 0)
            fold_tile<FOLD_XF, double2, CT, CT, T, BM, BN, BK>(q.V + (long long)j * q.n, (const CT *)q.xfs,
                                                               (const CT *)q.xfa, (CT *)q.t1, q.fx, lt);
        else if (ROLE == 1)
            fold_tile<FOLD_YF, CT, CT, CT, T, BM, BN, BK>((const CT *)q.t1, (const CT *)q.yfs, (const CT *)q.yfa,
                                                          (CT *)q.t2, q.fy, lt);
        else if (ROLE == 2)
            fold_tile<FOLD_YI, CT, CT, CT, T, BM, BN, BK>((const CT *)q.t2, (const CT *)q.yis, (const CT *)q.yia,
                                                          (CT *)q.t1, q.fy, lt);
        else
            fold_tile<FOLD_XI, CT, CT, CT, T, BM, BN, BK>((const CT *)q.t1, (const CT *)q.xis, (const CT *)q.xia,
                                                          (CT *)q.Z + (long long)j * q.n, q.fx, lt);
    }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_b_tridiag(const BProb *__restrict__ P, const BState *__restrict__ st,
                                                    const int *__restrict__ off, int np, int LX) {
    typedef typename c2<T>::t CT;
    extern __shared__ unsigned char smraw[];
    const int p = find_prob(off, np, blockIdx.x);
    if (!st[p].active) return;                 // uniform over the block
    const BProb &q = P[p];
    if constexpr (std::is_same<T, float>::value)
        tri_chunk_block<T, float2>((const CT *)q.t2, (CT *)q.t2, q.tpiv32, q.dxe, q.dye, q.nx, q.ny, q.nz,
                                   (q.nz + TL - 1) / TL, LX, q.ax, q.ay, q.c0, q.gz, q.hz2, blockIdx.x - off[p], smraw);
    else
        tri_chunk_block<T, double2>((const CT *)q.t2, (CT *)q.t2, q.tpiv, q.dxe, q.dye, q.nx, q.ny, q.nz,
                                    (q.nz + TL - 1) / TL, LX, q.ax, q.ay, q.c0, q.gz, q.hz2, blockIdx.x - off[p], smraw);
}

// ---------------------------------------------------------------------------------------------- matvec
// mode 0: restart, V_0 = F - A x (problems not done); mode 1: step j, V_{j+1} = V_j - A Z_j (active problems);
// ZT: element type of the Z basis (complex64 with the FP32 preconditioner)
template <int ORDER, typename ZT>
__global__ __launch_bounds__(NT) void k_b_matvec(const BProb *__restrict__ P, const BState *__restrict__ st,
                                                  const int *__restrict__ off, int np, int mode, int j) {
    const int p = find_prob(off, np, blockIdx.x);
    if (mode == 0 ? st[p].done : !st[p].active) return;
    const BProb &q = P[p];
    const int lb = blockIdx.x - off[p];
    if (mode == 0)
        matvec_tile<ORDER, true>(q.x, q.k2, q.fld, q.F, q.V, q.sp, lb);
    else
        matvec_tile<ORDER, true, ZT>((const ZT *)q.Z + (long long)j * q.n, q.k2, q.fld, q.V + (long long)j * q.n,
                                     q.V + (long long)(j + 1) * q.n, q.sp, lb);
}

// step j with right-hand sides paired on a shared operator: a unit is one problem or two problems of the same
// context (same k^2 and field block, e.g. two incident directions on one medium); the block reads the operator's
// planes once for both. Problems that are not active are left out of their unit.
template <int ORDER, typename ZT>
__global__ __launch_bounds__(NT) void k_b_matvec_pair(const BProb *__restrict__ P, const BState *__restrict__ st,
                                                       const int2 *__restrict__ units, const int *__restrict__ off,
                                                       int nunits, int j) {
    const int u = find_prob(off, nunits, blockIdx.x);
    const int2 pu = units[u];
    const bool a1 = st[pu.x].active != 0;
    const bool a2 = pu.y >= 0 && st[pu.y].active != 0;
    if (!a1 && !a2) return;
    const ZT *xs[2];
    const double2 *Fs[2];
    double2 *ys[2];
    int nr = 0;
    const int ps[2] = {pu.x, pu.y};
    const bool as[2] = {a1, a2};
#pragma unroll
    for (int r = 0; r < 2; ++r)
        if (as[r]) {
            const BProb &q = P[ps[r]];
            xs[nr] = (const ZT *)q.Z + (long long)j * q.n;
            Fs[nr] = q.V + (long long)j * q.n;
            ys[nr] = q.V + (long long)(j + 1) * q.n;
            ++nr;
        }
    const BProb &q = P[a1 ? pu.x : pu.y];
    matvec_tile_n<ORDER, true, ZT, false, 2>(xs, q.k2, q.fld, Fs, ys, q.sp, blockIdx.x - off[u], nr);
}

// ---------------------------------------------------------------------------------------------- inner products
// mode 0: ||F||^2 (all problems); mode 1: ||V_0||^2 (not done); mode 2: V_{0..j}^H V_{j+1}, ||V_{j+1}||^2 (active);
// mode 3: the same for the second Gram-Schmidt pass (active problems whose step cancelled)
__global__ __launch_bounds__(256) void k_b_dots(const BProb *__restrict__ P, const BState *__restrict__ st,
                                                const int *__restrict__ off, int np, int mode, int j) {
    const int p = find_prob(off, np, blockIdx.x);
    if (mode == 1 && st[p].done) return;
    if (mode == 2 && !st[p].active) return;
    if (mode == 3 && !(st[p].active && st[p].reo)) return;
    const BProb &q = P[p];
    const long long lb = blockIdx.x - off[p];
    if (mode == 0) dots_chunk(nullptr, q.n, 0, q.F, q.n, q.part, lb);
    else if (mode == 1) dots_chunk(nullptr, q.n, 0, q.V, q.n, q.part, lb);
    else dots_chunk(q.V, q.n, j + 1, q.V + (long long)(j + 1) * q.n, q.n, q.part, lb);
}

// fixed-order block reduction of the partials of output t (nout outputs); result valid in thread 0
__device__ double2 reduce_part(const double2 *part, int nblk, int nout, int t) {
    __shared__ double sr[256], si[256];
    const int tid = threadIdx.x;
    double re = 0.0, im = 0.0;
    for (int b = tid; b < nblk; b += 256) {
        double2 v = part[(long long)b * nout + t];
        re += v.x;
        im += v.y;
    }
    __syncthreads();
    sr[tid] = re;
    si[tid] = im;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) { sr[tid] += sr[tid + s]; si[tid] += si[tid + s]; }
        __syncthreads();
    }
    return make_double2(sr[0], si[0]);
}

__device__ __forceinline__ double2 cmulb(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double cabs2(double2 a) { return hypot(a.x, a.y); }

// one block per problem: ||F|| and a fresh state
__global__ __launch_bounds__(256) void k_b_init(const BProb *__restrict__ P, BState *__restrict__ st, int np,
                                                int m) {
    const int p = blockIdx.x;
    const BProb &q = P[p];
    double2 r = reduce_part(q.part, q.nblk_dots, 1, 0);
    if (threadIdx.x == 0) {
        BState s{};
        s.bnorm = sqrt(fmax(r.x, 0.0));
        s.converged = s.bnorm == 0.0;
        s.done = s.converged;
        s.relres_true = 0.0;
        s.alpha = make_double2(1.0, 0.0);
        st[p] = s;
    }
}

// one block per problem, after ||V_0||^2 of the restart vector: convergence test and the new cycle's g
__global__ __launch_bounds__(256) void k_b_restart(const BProb *__restrict__ P, BState *__restrict__ st,
                                                   BArrays a, const BParams *__restrict__ prm) {
    const int p = blockIdx.x;
    if (st[p].done) return;
    const BProb &q = P[p];
    const int m = prm->m;
    double2 r = reduce_part(q.part, q.nblk_dots, 1, 0);
    if (threadIdx.x != 0) return;
    BState s = st[p];
    s.beta = sqrt(fmax(r.x, 0.0));
    s.relres_true = s.beta / s.bnorm;
    s.k = 0;
    s.active = 0;
    if (!isfinite(s.beta)) {
        s.done = 1;
    } else if (s.beta <= prm->rtol * s.bnorm) {
        s.converged = 1;
        s.done = 1;
    } else if (s.its >= prm->maxit) {
        s.done = 1;
    } else {
        s.active = 1;
        s.alpha = make_double2(1.0 / s.beta, 0.0);
        double2 *g = a.g + (long long)p * (m + 1);
        g[0] = make_double2(s.beta, 0.0);
        for (int i = 1; i <= m; ++i) g[i] = make_double2(0.0, 0.0);
    }
    st[p] = s;
}

// Column j of H from the orthogonalisation coefficients hv[0..j] and eta (shifted Arnoldi: -h + e_j, eta), the
// previous rotations, the new rotation, g, the convergence test, and the coefficients of the update
// v_{j+1} = -(y - V h)/eta. One thread.
__device__ void arnoldi_column(BState &s, BArrays a, int p, int m, const BParams *__restrict__ prm, int j,
                               const double2 *hv, double eta) {
    double2 *H = a.H + (long long)p * (m + 1) * m;
    double *cs = a.cs + (long long)p * m;
    double2 *sn = a.sn + (long long)p * m;
    double2 *g = a.g + (long long)p * (m + 1);
    double2 *coef = a.coef + (long long)p * (m + 1);
    for (int i = 0; i <= j; ++i) H[(long long)i * m + j] = make_double2(-hv[i].x, -hv[i].y);
    H[(long long)j * m + j].x += 1.0;
    for (int i = 0; i < j; ++i) {
        double2 x0 = H[(long long)i * m + j], x1 = H[(long long)(i + 1) * m + j];
        double2 t0 = cmulb(sn[i], x1);
        H[(long long)i * m + j] = make_double2(cs[i] * x0.x + t0.x, cs[i] * x0.y + t0.y);
        double2 t1 = cmulb(cconj(sn[i]), x0);
        H[(long long)(i + 1) * m + j] = make_double2(-t1.x + cs[i] * x1.x, -t1.y + cs[i] * x1.y);
    }
    {
        double2 av = H[(long long)j * m + j];
        double aa = cabs2(av);
        if (eta == 0.0) { cs[j] = 1.0; sn[j] = make_double2(0.0, 0.0); }
        else if (aa == 0.0) { cs[j] = 0.0; sn[j] = make_double2(1.0, 0.0); H[(long long)j * m + j] = make_double2(eta, 0.0); }
        else {
            double tt = hypot(aa, eta);
            double2 ph = make_double2(av.x / aa, av.y / aa);
            cs[j] = aa / tt;
            sn[j] = make_double2(ph.x * eta / tt, ph.y * eta / tt);
            H[(long long)j * m + j] = make_double2(ph.x * tt, ph.y * tt);
        }
        double2 gj = g[j];
        double2 t1 = cmulb(cconj(sn[j]), gj);
        g[j + 1] = make_double2(-t1.x, -t1.y);
        g[j] = make_double2(cs[j] * gj.x, cs[j] * gj.y);
    }
    s.its += 1;
    s.k = j + 1;
    const double res = cabs2(g[j + 1]);
    s.relres_est = res / s.bnorm;
    if (eta == 0.0 || res <= prm->rtol * s.bnorm || s.its >= prm->maxit || j + 1 == m || !isfinite(res)) {
        s.active = 0;
    } else {
        for (int i = 0; i <= j; ++i) coef[i] = make_double2(hv[i].x / eta, hv[i].y / eta);
        s.alpha = make_double2(-1.0 / eta, 0.0);
    }
}

// one block per problem: reduce V^H y and ||y||^2 and finish the step (arnoldi_column). With severe cancellation
// (||y - V h||^2 = ||y||^2 - sum |h_i|^2 <= reorth ||y||^2, reorth = cgs_reorth()) that norm is not accurate enough: the step takes a
// second Gram-Schmidt pass instead. The update then leaves u = -(y - V h) unscaled (coefficients h, alpha = -1), and
// k_b_arnoldi2 finishes the step from the inner products of u.
__global__ __launch_bounds__(256) void k_b_arnoldi(const BProb *__restrict__ P, BState *__restrict__ st, BArrays a,
                                                   const BParams *__restrict__ prm, int j) {
    __shared__ double2 hv[130];
    const int p = blockIdx.x;
    if (!st[p].active) return;
    const BProb &q = P[p];
    const int m = prm->m;
    const int nv = j + 1;
    for (int t = 0; t <= nv; ++t) {
        double2 r = reduce_part(q.part, q.nblk_dots, nv + 1, t);
        if (threadIdx.x == 0) hv[t] = r;
    }
    if (threadIdx.x != 0) return;
    BState s = st[p];
    double hh = 0.0;
    for (int i = 0; i <= j; ++i) hh += hv[i].x * hv[i].x + hv[i].y * hv[i].y;
    const double ww = hv[nv].x;
    const double eta2 = ww - hh;
    s.reo = 0;
    if (!(eta2 > prm->reorth * ww) && isfinite(eta2)) {
        s.cancel += 1;
        s.reo = 1;
        double2 *coef = a.coef + (long long)p * (m + 1);
        for (int i = 0; i <= j; ++i) coef[i] = hv[i];
        s.alpha = make_double2(-1.0, 0.0);
    } else {
        arnoldi_column(s, a, p, m, prm, j, hv, eta2 > 0.0 ? sqrt(eta2) : 0.0);
    }
    st[p] = s;
}

// the second pass of a cancelled step: h2 = V^H u and ||u||^2 (u = -(y - V h) in V_{j+1}); then
// v_{j+1} = (u - V h2)/eta' = -(y - V (h - h2))/eta' with eta'^2 = ||u||^2 - sum |h2_i|^2
__global__ __launch_bounds__(256) void k_b_arnoldi2(const BProb *__restrict__ P, BState *__restrict__ st, BArrays a,
                                                    const BParams *__restrict__ prm, int j) {
    __shared__ double2 h2[130];
    __shared__ double2 hv[130];
    const int p = blockIdx.x;
    if (!st[p].active || !st[p].reo) return;
    const BProb &q = P[p];
    const int m = prm->m;
    const int nv = j + 1;
    for (int t = 0; t <= nv; ++t) {
        double2 r = reduce_part(q.part, q.nblk_dots, nv + 1, t);
        if (threadIdx.x == 0) h2[t] = r;
    }
    if (threadIdx.x != 0) return;
    BState s = st[p];
    double2 *coef = a.coef + (long long)p * (m + 1);
    double hh = 0.0;
    for (int i = 0; i <= j; ++i) {
        hv[i] = make_double2(coef[i].x - h2[i].x, coef[i].y - h2[i].y);
        hh += h2[i].x * h2[i].x + h2[i].y * h2[i].y;
    }
    const double e2 = h2[nv].x - hh;
    const double eta = e2 > 0.0 ? sqrt(e2) : 0.0;
    arnoldi_column(s, a, p, m, prm, j, hv, eta);
    if (s.active) {                  // the correction of u (k_b_lincomb kind 3)
        for (int i = 0; i <= j; ++i) coef[i] = make_double2(-h2[i].x / eta, -h2[i].y / eta);
        s.alpha = make_double2(1.0 / eta, 0.0);
    }
    st[p] = s;
}

// one thread per problem: y = R^{-1} g (k x k, upper triangular) into coef, for problems that iterated
__global__ void k_b_trisolve(BState *__restrict__ st, BArrays a, const BParams *__restrict__ prm, int np) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    BState s = st[p];
    if (s.done || s.k == 0) return;
    const int m = prm->m, k = s.k;
    const double2 *H = a.H + (long long)p * (m + 1) * m;
    const double2 *g = a.g + (long long)p * (m + 1);
    double2 *y = a.coef + (long long)p * (m + 1);
    for (int i = k - 1; i >= 0; --i) {
        double2 acc = g[i];
        for (int c = i + 1; c < k; ++c) {
            double2 t = cmulb(H[(long long)i * m + c], y[c]);
            acc.x -= t.x;
            acc.y -= t.y;
        }
        double2 d = H[(long long)i * m + i];
        double dd = d.x * d.x + d.y * d.y;
        y[i] = make_double2((acc.x * d.x + acc.y * d.y) / dd, (acc.y * d.x - acc.x * d.y) / dd);
    }
    s.alpha = make_double2(1.0, 0.0);
    s.cycles += 1;
    st[p] = s;
}

// ---------------------------------------------------------------------------------------------- linear combinations
constexpr int BLC_EPT = 4;
__device__ __forceinline__ double2 wide_b(const double2 *p) { return ld_stream(p); }
__device__ __forceinline__ double2 wide_b(const float2 *p) { return ld_stream_wide(p); }
// acc += sum_{i<nv} c_i V_i over BLC_EPT elements per thread, four vectors per round (16 loads in flight)
template <typename VT>
__device__ __forceinline__ void b_accum(double2 *acc, const bool *ok, long long start, const VT *V, long long ldv,
                                        int nv, const double2 *coef) {
    int i = 0;
    for (; i + 4 <= nv; i += 4) {
        double2 v[4][BLC_EPT];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int e = 0; e < BLC_EPT; ++e) {
                const long long idx = start + (long long)e * 256;
                v[q][e] = ok[e] ? wide_b(V + (long long)(i + q) * ldv + idx) : make_double2(0.0, 0.0);
            }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double2 c = coef[i + q];
#pragma unroll
            for (int e = 0; e < BLC_EPT; ++e) {
                acc[e].x += c.x * v[q][e].x - c.y * v[q][e].y;
                acc[e].y += c.x * v[q][e].y + c.y * v[q][e].x;
            }
        }
    }
    for (; i < nv; ++i) {
        const double2 c = coef[i];
        double2 v[BLC_EPT];
#pragma unroll
        for (int e = 0; e < BLC_EPT; ++e) {
            const long long idx = start + (long long)e * 256;
            v[e] = ok[e] ? wide_b(V + (long long)i * ldv + idx) : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int e = 0; e < BLC_EPT; ++e) {
            acc[e].x += c.x * v[e].x - c.y * v[e].y;
            acc[e].y += c.x * v[e].y + c.y * v[e].x;
        }
    }
}

// kind 0: V_0 *= alpha (active); kind 1: V_{j+1} = alpha V_{j+1} + sum_{i<=j} c_i V_i (active);
// kind 2: x += sum_{i<k} c_i Z_i (problems that iterated in this cycle and are not done); kind 3: kind 1 for the
// second Gram-Schmidt pass (active problems whose step cancelled); ZT: element type of Z
template <typename ZT>
__global__ __launch_bounds__(256) void k_b_lincomb(const BProb *__restrict__ P, const BState *__restrict__ st,
                                                   BArrays a, const BParams *__restrict__ prm,
                                                   const int *__restrict__ off, int np, int kind, int j) {
    const int p = find_prob(off, np, blockIdx.x);
    const BState &s = st[p];
    if (kind == 2 ? (s.done || s.k == 0) : (!s.active || (kind == 3 && !s.reo))) return;
    const BProb &q = P[p];
    const int m = prm->m;
    const double2 *coef = a.coef + (long long)p * (m + 1);
    double2 *out = kind == 2 ? q.x : (kind == 0 ? q.V : q.V + (long long)(j + 1) * q.n);
    const double2 alpha = kind == 2 ? make_double2(1.0, 0.0) : s.alpha;
    const long long start = (long long)(blockIdx.x - off[p]) * (256 * BLC_EPT) + threadIdx.x;
    double2 acc[BLC_EPT];
    bool ok[BLC_EPT];
#pragma unroll
    for (int e = 0; e < BLC_EPT; ++e) {
        const long long idx = start + (long long)e * 256;
        ok[e] = idx < q.n;
        acc[e] = make_double2(0.0, 0.0);
        if (ok[e]) acc[e] = cmulb(alpha, out[idx]);
    }
    if (kind == 1 || kind == 3) b_accum(acc, ok, start, q.V, q.n, j + 1, coef);
    else if (kind == 2) b_accum(acc, ok, start, (const ZT *)q.Z, q.n, s.k, coef);
#pragma unroll
    for (int e = 0; e < BLC_EPT; ++e) {
        const long long idx = start + (long long)e * 256;
        if (ok[e]) out[idx] = acc[e];
    }
}

__global__ void k_b_zero_x(const BProb *__restrict__ P, const int *__restrict__ off, int np) {
    const int p = find_prob(off, np, blockIdx.x);
    const BProb &q = P[p];
    const long long start = (long long)(blockIdx.x - off[p]) * (256 * BLC_EPT) + threadIdx.x;
    for (int e = 0; e < BLC_EPT; ++e) {
        const long long idx = start + (long long)e * 256;
        if (idx < q.n) q.x[idx] = make_double2(0.0, 0.0);
    }
}

template <int ROLE, typename T>
void gemm_role(const BLaunch &L, hipStream_t s, int j, int cfg, const long long *off) {
    switch (cfg) {
    case 1: hipLaunchKernelGGL((k_b_gemm<ROLE, T, 64, 64, 32>), dim3(L.gemm_grid), dim3(256), 0, s, L.P, L.st, off, L.np, j); break;
    case 2: hipLaunchKernelGGL((k_b_gemm<ROLE, T, 128, 64, 16>), dim3(L.gemm_grid), dim3(256), 0, s, L.P, L.st, off, L.np, j); break;
    case 3: hipLaunchKernelGGL((k_b_gemm<ROLE, T, 64, 128, 16>), dim3(L.gemm_grid), dim3(256), 0, s, L.P, L.st, off, L.np, j); break;
    default: hipLaunchKernelGGL((k_b_gemm<ROLE, T, 64, 64, 16>), dim3(L.gemm_grid), dim3(256), 0, s, L.P, L.st, off, L.np, j); break;
    }
}

template <typename T> hipError_t precond_steps(const BLaunch &L, hipStream_t s, int j) {
    gemm_role<0, T>(L, s, j, L.cfg[0], L.off.g[0]);
    gemm_role<1, T>(L, s, j, L.cfg[1], L.off.g[1]);
    hipLaunchKernelGGL(k_b_tridiag<T>, dim3(L.tot_tri), dim3(L.tri_lx * L.tri_pb),
                       2 * sizeof(typename c2<T>::t) * (size_t)L.tri_lx * L.tri_pb, s, L.P, L.st, L.off.tri, L.np, L.tri_lx);
    gemm_role<2, T>(L, s, j, L.cfg[2], L.off.g[2]);
    gemm_role<3, T>(L, s, j, L.cfg[3], L.off.g[3]);
    return hipGetLastError();
}

template <typename ZT> hipError_t matvec_step_t(const BLaunch &L, hipStream_t s, int mode, int j) {
    if (mode == 1) {
        if (L.order == 6)
            hipLaunchKernelGGL((k_b_matvec_pair<6, ZT>), dim3(L.tot_mvp), dim3(64, TY), 0, s, L.P, L.st, L.units,
                               L.off.mvp, L.nunits, j);
        else if (L.order == 4)
            hipLaunchKernelGGL((k_b_matvec_pair<4, ZT>), dim3(L.tot_mvp), dim3(64, TY), 0, s, L.P, L.st, L.units,
                               L.off.mvp, L.nunits, j);
        else
            hipLaunchKernelGGL((k_b_matvec_pair<2, ZT>), dim3(L.tot_mvp), dim3(64, TY), 0, s, L.P, L.st, L.units,
                               L.off.mvp, L.nunits, j);
        return hipGetLastError();
    }
    if (L.order == 6)
        hipLaunchKernelGGL((k_b_matvec<6, ZT>), dim3(L.tot_mv), dim3(64, TY), 0, s, L.P, L.st, L.off.mv, L.np, mode, j);
    else if (L.order == 4)
        hipLaunchKernelGGL((k_b_matvec<4, ZT>), dim3(L.tot_mv), dim3(64, TY), 0, s, L.P, L.st, L.off.mv, L.np, mode, j);
    else
        hipLaunchKernelGGL((k_b_matvec<2, ZT>), dim3(L.tot_mv), dim3(64, TY), 0, s, L.P, L.st, L.off.mv, L.np, mode, j);
    return hipGetLastError();
}
hipError_t matvec_step(const BLaunch &L, hipStream_t s, int mode, int j) {
    return L.fp32 ? matvec_step_t<float2>(L, s, mode, j) : matvec_step_t<double2>(L, s, mode, j);
}
hipError_t lincomb_step(const BLaunch &L, hipStream_t s, int kind, int j) {
    if (L.fp32)
        hipLaunchKernelGGL(k_b_lincomb<float2>, dim3(L.tot_lc), dim3(256), 0, s, L.P, L.st, L.a, L.prm, L.off.lc, L.np,
                           kind, j);
    else
        hipLaunchKernelGGL(k_b_lincomb<double2>, dim3(L.tot_lc), dim3(256), 0, s, L.P, L.st, L.a, L.prm, L.off.lc,
                           L.np, kind, j);
    return hipGetLastError();
}

}  // namespace

hipError_t bl_zero_x(const BLaunch &L, hipStream_t s) {
    hipLaunchKernelGGL(k_b_zero_x, dim3(L.tot_lc), dim3(256), 0, s, L.P, L.off.lc, L.np);
    return hipGetLastError();
}

hipError_t bl_init(const BLaunch &L, hipStream_t s) {
    hipLaunchKernelGGL(k_b_dots, dim3(L.tot_dot), dim3(256), 0, s, L.P, L.st, L.off.dot, L.np, 0, 0);
    hipLaunchKernelGGL(k_b_init, dim3(L.np), dim3(256), 0, s, L.P, L.st, L.np, L.m);
    return hipGetLastError();
}

hipError_t bl_restart(const BLaunch &L, hipStream_t s) {
    // restart vector V_0 = F - A x, its norm, the convergence test, V_0 /= beta
    hipError_t e;
    if ((e = matvec_step(L, s, 0, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_b_dots, dim3(L.tot_dot), dim3(256), 0, s, L.P, L.st, L.off.dot, L.np, 1, 0);
    hipLaunchKernelGGL(k_b_restart, dim3(L.np), dim3(256), 0, s, L.P, L.st, L.a, L.prm);
    return lincomb_step(L, s, 0, 0);
}

hipError_t bl_cycle(const BLaunch &L, hipStream_t s) {
    hipError_t e;
    if ((e = bl_restart(L, s)) != hipSuccess) return e;
    for (int j = 0; j < L.m; ++j) {
        e = L.fp32 ? precond_steps<float>(L, s, j) : precond_steps<double>(L, s, j);
        if (e != hipSuccess) return e;
        if ((e = matvec_step(L, s, 1, j)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_b_dots, dim3(L.tot_dot), dim3(256), 0, s, L.P, L.st, L.off.dot, L.np, 2, j);
        hipLaunchKernelGGL(k_b_arnoldi, dim3(L.np), dim3(256), 0, s, L.P, L.st, L.a, L.prm, j);
        if ((e = lincomb_step(L, s, 1, j)) != hipSuccess) return e;
        // second Gram-Schmidt pass of the steps that cancelled (every block of the other problems returns at once)
        hipLaunchKernelGGL(k_b_dots, dim3(L.tot_dot), dim3(256), 0, s, L.P, L.st, L.off.dot, L.np, 3, j);
        hipLaunchKernelGGL(k_b_arnoldi2, dim3(L.np), dim3(256), 0, s, L.P, L.st, L.a, L.prm, j);
        if ((e = lincomb_step(L, s, 3, j)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_b_trisolve, dim3((L.np + 63) / 64), dim3(64), 0, s, L.st, L.a, L.prm, L.np);
    return lincomb_step(L, s, 2, 0);
}

}  // namespace helm
