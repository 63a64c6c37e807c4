// Thin per-slice transforms of the PFFT preconditioner (Sec. 4.2): only the boundary faces of every slice
// take part, so each costs O(N_x N_y) per slice instead of a dense transform.
//
// Ring layout (all slices): rows [Nz][2][Nx] (row j = 0, then row j = Ny-1 of each slice), followed by columns
// [Nz][2][Ny] (column i = 0, then i = Nx-1, for all j); the corners appear in both a row and a column and
// consumers take them from the rows. The products with the transposed eigenvector or sine matrices are single
// complex GEMMs over all slices (M = 2 Nz).
//
// Inverse (k_ring_inv_rows, k_ring_inv_sum, two GEMMs in one launch): the inverse transform X = V_y Xh V_x^T
//   evaluated on the faces only (eq. PFFT_INV): the two boundary rows via r_j = V_y[j,:] Xh then
//   X[j,i] = sum_k V_x[i,k] r_j[k], the two boundary columns via s_i = Xh V_x[i,:]^T then
//   X[j,i] = sum_m V_y[j,m] s_i[m]. The pass over the data runs with several row groups per slice; the products
//   with V_x^T and V_y^T are GEMMs over all slices.
// Forward (k_ring_fwd_R, two GEMMs in one launch, k_ring_fwd_write): the forward transform of ring-supported
//   data R (Steps 1, 2*): R = E (a + b) with E = A_p^F - A_p restricted to the faces: on face row 1 of an axis
//   -a (gamma v_1 + (zeta - 1) v_2), and the mirror on row N (eq. lambda_mat_definition); with zeta = 1 only the
//   face layer enters. out = s * base + W_y R W_x^T computed as two rank-2 updates from the boundary rows
//   (S_m = R[m,:] W_x^T) and the interior parts of the boundary columns (T_k = W_y[:, inner] R[inner, k]); the
//   factors as GEMMs over all slices, then every element in parallel.
// Second layer (zeta != 1): the inverse is run a second time for rows 2, N_y - 1 and columns 2, N_x - 1 into a
// second ring of the same layout; R takes the inner neighbours from it (the x-neighbours of the corners from the
// full boundary rows of the first).
#include <algorithm>

#include "helm_internal.h"

namespace helm {

namespace {

template <typename T> struct c2;
template <> struct c2<double> { typedef double2 t; };
template <> struct c2<float> { typedef float2 t; };

template <typename CT> __device__ __forceinline__ CT cz() { CT r; r.x = 0; r.y = 0; return r; }
template <typename CT> __device__ __forceinline__ CT cmul(CT a, CT b) {
    CT r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename CT> __device__ __forceinline__ CT cfma(CT a, CT b, CT c) {
    c.x += a.x * b.x - a.y * b.y;
    c.y += a.x * b.y + a.y * b.x;
    return c;
}
template <typename CT> __device__ __forceinline__ CT cadd(CT a, CT b) { a.x += b.x; a.y += b.y; return a; }

template <typename T> __device__ __forceinline__ T wsum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

constexpr int RING_RG = 8; // most row groups per slice in the inverse's pass over the data
constexpr int RING_NMAX = 64 * 13;   // widest slice the ring pass supports (MAXC = 13 chunks of 64 columns)

// Inverse, pass over the data for face layer `layer` (0: rows/columns 1 and N, 1: 2 and N-1): block (slice l,
// row group rg) takes rows m of its group and accumulates, per column k, r0[k] += V_y[ja][m] X[m][k] and
// rN[k] += V_y[jb][m] X[m][k] (partials per group; ja = layer, jb = ny-1-layer), and per row the complete
// s0[m] = sum_k V_x[ia][k] X[m][k], sN[m] = sum_k V_x[ib][k] X[m][k] (ia = layer, ib = nx-1-layer). Each lane
// holds MAXC chunks of 64 columns (N_x <= 64 MAXC; the launcher picks 4, 8 or 13).
template <typename T, int MAXC>
__global__ __launch_bounds__(256) void k_ring_inv_rows(const typename c2<T>::t *__restrict__ Xh,
                                                       const typename c2<T>::t *__restrict__ Vy,
                                                       const typename c2<T>::t *__restrict__ Vx, int nx, int ny,
                                                       int layer, int rgs, typename c2<T>::t *__restrict__ rpart,
                                                       typename c2<T>::t *__restrict__ sv) {
    typedef typename c2<T>::t CT;
    __shared__ CT red[4][2][64 * MAXC];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l = blockIdx.x / rgs, rg = blockIdx.x % rgs;
    const int per = (ny + rgs - 1) / rgs;
    const int m0 = rg * per, m1 = min(ny, m0 + per);
    const CT *X = Xh + (long long)l * nx * ny;
    CT vx0[MAXC], vxN[MAXC], a0[MAXC], aN[MAXC];
#pragma unroll
    for (int c = 0; c < MAXC; ++c) {
        const int k = lane + 64 * c;
        vx0[c] = k < nx ? Vx[(long long)layer * nx + k] : cz<CT>();
        vxN[c] = k < nx ? Vx[(long long)(nx - 1 - layer) * nx + k] : cz<CT>();
        a0[c] = cz<CT>();
        aN[c] = cz<CT>();
    }
    // the wave's rows m = m0 + wave, + 4, ...; the next row is loaded while the current one is reduced (its
    // cross-lane sums would otherwise leave every row's loads exposed), where the registers allow it: slices up to
    // 512 wide in FP32, 256 in FP64
    constexpr bool PF = MAXC <= (sizeof(T) == 4 ? 8 : 4);
    CT xr[MAXC], xn[PF ? MAXC : 1];
    auto load_row = [&](CT *dst, int m) {
        const CT *row = X + (long long)m * nx;
#pragma unroll
        for (int c = 0; c < MAXC; ++c) {
            const int k = lane + 64 * c;
            dst[c] = (m < m1 && k < nx) ? row[k] : cz<CT>();
        }
    };
    if (PF) load_row(xr, m0 + wave);
    for (int m = m0 + wave; m < m1; m += 4) {
        if (PF) {
            load_row(xn, m + 4);
        } else {
            load_row(xr, m);
        }
        const CT w0 = Vy[(long long)layer * ny + m], wN = Vy[(long long)(ny - 1 - layer) * ny + m];
        CT s0 = cz<CT>(), sN = cz<CT>();
#pragma unroll
        for (int c = 0; c < MAXC; ++c) {
            const CT x = xr[c];                       // zero beyond the slice width
            a0[c] = cfma(w0, x, a0[c]);
            aN[c] = cfma(wN, x, aN[c]);
            s0 = cfma(vx0[c], x, s0);
            sN = cfma(vxN[c], x, sN);
        }
        if (PF) {
#pragma unroll
            for (int c = 0; c < MAXC; ++c) xr[c] = xn[c];
        }
        s0.x = wsum(s0.x); s0.y = wsum(s0.y);
        sN.x = wsum(sN.x); sN.y = wsum(sN.y);
        if (lane == 0) {
            sv[(long long)l * 2 * ny + m] = s0;
            sv[(long long)l * 2 * ny + ny + m] = sN;
        }
    }
#pragma unroll
    for (int c = 0; c < MAXC; ++c) {
        red[wave][0][lane + 64 * c] = a0[c];
        red[wave][1][lane + 64 * c] = aN[c];
    }
    __syncthreads();
    CT *rp = rpart + ((long long)l * rgs + rg) * 2 * nx;
    for (int k = tid; k < nx; k += 256) {
        CT r0 = red[0][0][k], rN = red[0][1][k];
        for (int w = 1; w < 4; ++w) { r0 = cadd(r0, red[w][0][k]); rN = cadd(rN, red[w][1][k]); }
        rp[k] = r0;
        rp[nx + k] = rN;
    }
}

// Inverse: r0, rN of every slice summed over the row groups in order, rsum[l][w][k]
template <typename T>
__global__ void k_ring_inv_sum(const typename c2<T>::t *__restrict__ rpart, int nx, int rgs, long long total,
                               typename c2<T>::t *__restrict__ rsum) {
    typedef typename c2<T>::t CT;
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= total) return;
    const long long l = e / (2 * nx), q = e % (2 * nx);
    const CT *rp = rpart + l * rgs * 2 * nx + q;
    CT acc = rp[0];
    for (int g = 1; g < rgs; ++g) acc = cadd(acc, rp[(long long)g * 2 * nx]);
    rsum[e] = acc;
}

// Forward: R = E (a + b) on the faces: the boundary rows Rr[l][w][k] in full and the interior parts of the
// boundary columns Rc[l][w][m] (ends zero). E on face row 1 of an axis is -a (gamma v_1 + (zeta - 1) v_2): ex, ey
// are -a gamma and ex1, ey1 -a (zeta - 1) per axis; ra1, rb1 (the second-layer rings) only when zeta != 1.
template <typename T>
__global__ void k_ring_fwd_R(const typename c2<T>::t *__restrict__ ra, const typename c2<T>::t *__restrict__ rb,
                             const typename c2<T>::t *__restrict__ ra1, const typename c2<T>::t *__restrict__ rb1,
                             double2 ex, double2 ey, double2 ex1, double2 ey1, int nx, int ny, int nz,
                             typename c2<T>::t *__restrict__ Rr, typename c2<T>::t *__restrict__ Rc) {
    typedef typename c2<T>::t CT;
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long nrow = 2LL * nz * nx, ncol = 2LL * nz * ny;
    if (e >= nrow + ncol) return;
    CT ecx, ecy, ecx1, ecy1;
    ecx.x = (T)ex.x; ecx.y = (T)ex.y;
    ecy.x = (T)ey.x; ecy.y = (T)ey.y;
    ecx1.x = (T)ex1.x; ecx1.y = (T)ex1.y;
    ecy1.x = (T)ey1.x; ecy1.y = (T)ey1.y;
    auto val = [&](const CT *a, const CT *b, long long i) {
        CT v = a[i];
        if (b) v = cadd(v, b[i]);
        return v;
    };
    const CT v = val(ra, rb, e);
    if (e < nrow) {
        const int k = (int)(e % nx);
        CT r = cmul(ecy, v);
        if (ra1) r = cfma(ecy1, val(ra1, rb1, e), r);                 // inner neighbour across the y-face
        if (k == 0 || k == nx - 1) {
            r = cfma(ecx, v, r);
            if (ra1) r = cfma(ecx1, val(ra, rb, k == 0 ? e + 1 : e - 1), r);   // inner neighbour along the row
        }
        Rr[e] = r;
    } else {
        const int m = (int)((e - nrow) % ny);
        CT r = cz<CT>();
        if (m > 0 && m < ny - 1) {
            r = cmul(ecx, v);
            if (ra1) r = cfma(ecx1, val(ra1, rb1, e), r);             // inner neighbour across the x-face
        }
        Rc[e - nrow] = r;
    }
}

// Forward, every element of every slice: out = s base + W_y[j][0] S_0[i] + W_y[j][ny-1] S_N[i]
// + T_0[j] W_x[i][0] + T_N[j] W_x[i][nx-1] (the boundary columns of W read as rows of the transposes);
// fvec = [S: Nz x 2 x Nx | T: Nz x 2 x Ny] with S = Rr W_x^T and T = Rc W_y^T. A block takes FWD_RJ rows of one
// slice; each thread keeps the four column factors of its columns i in registers and streams the rows, whose
// four factors are the same for the whole block.
constexpr int FWD_RJ = 16;
template <typename T>
__global__ __launch_bounds__(256) void k_ring_fwd_write(const typename c2<T>::t *__restrict__ fvec,
                                                        const typename c2<T>::t *base, T base_scale,
                                                        typename c2<T>::t *out,
                                                        const typename c2<T>::t *__restrict__ WyT,
                                                        const typename c2<T>::t *__restrict__ WxT, int nx, int ny,
                                                        int nz) {
    typedef typename c2<T>::t CT;
    const int rblocks = (ny + FWD_RJ - 1) / FWD_RJ;
    const int l = blockIdx.x / rblocks;
    const int j0 = (blockIdx.x % rblocks) * FWD_RJ, j1 = min(ny, j0 + FWD_RJ);
    const long long plane = (long long)nx * ny;
    const CT *S = fvec + (long long)l * 2 * nx;                                 // S_0, S_N of slice l
    const CT *Tc = fvec + 2LL * nz * nx + (long long)l * 2 * ny;                // T_0, T_N of slice l
    const CT *WyN = WyT + (long long)(ny - 1) * ny, *WxN = WxT + (long long)(nx - 1) * nx;
    for (int i = threadIdx.x; i < nx; i += 256) {
        const CT s0 = S[i], sN = S[nx + i], x0 = WxT[i], xN = WxN[i];
        for (int j = j0; j < j1; ++j) {
            const long long e = (long long)l * plane + (long long)j * nx + i;
            CT acc = cz<CT>();
            if (base) { acc = base[e]; acc.x *= base_scale; acc.y *= base_scale; }
            acc = cfma(WyT[j], s0, acc);
            acc = cfma(WyN[j], sN, acc);
            acc = cfma(Tc[j], x0, acc);
            acc = cfma(Tc[ny + j], xN, acc);
            out[e] = acc;
        }
    }
}

// the row and the column product of a face transform, in one launch
inline hipError_t gemm_pair(const GemmDesc &d0, const double2 *A0, const double2 *B0, double2 *C0, const GemmDesc &d1,
                            const double2 *A1, const double2 *B1, double2 *C1, hipStream_t s) {
    return launch_gemm_pair_z64(d0, A0, B0, C0, d1, A1, B1, C1, s);
}
inline hipError_t gemm_pair(const GemmDesc &d0, const float2 *A0, const float2 *B0, float2 *C0, const GemmDesc &d1,
                            const float2 *A1, const float2 *B1, float2 *C1, hipStream_t s) {
    return launch_gemm_pair_z32(d0, A0, B0, C0, d1, A1, B1, C1, s);
}
// C (M x N) = A (M x K) B (K x N), all row-major and contiguous
inline GemmDesc plain_desc(int M, int N, int K) { return GemmDesc{M, N, K, K, N, N, 0, 0, 0, 1}; }

// Row groups per slice for the inverse's pass (1 .. RING_RG): the count whose grid fills its rounds of resident
// blocks best (blocks / (rounds x resident blocks), from the kernel's occupancy on this device), the smaller one
// on a tie. At 256^3 that is one or two full rounds; with many slices (800^3) it stays at RING_RG, where a last
// round of a few long blocks would otherwise idle the chip.
template <typename T, int MAXC> int ring_groups(int nz) {
    static const int cap = [] {
        int dev = 0, cus = 0, nb = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ring_inv_rows<T, MAXC>, 256, 0) != hipSuccess)
            return 0;
        return nb * cus;
    }();
    if (cap <= 0) return RING_RG;
    int best = RING_RG;
    double best_eff = -1.0;
    for (int r = 1; r <= RING_RG; ++r) {
        const long long blocks = (long long)std::max(1, nz) * r;
        const long long rounds = (blocks + cap - 1) / cap;
        const double eff = (double)blocks / (double)(rounds * cap);
        if (eff > best_eff + 1e-12) { best_eff = eff; best = r; }
    }
    return best;
}

template <typename T, int MAXC>
hipError_t inv_rows_launch(const typename c2<T>::t *Xh, const typename c2<T>::t *Vy, const typename c2<T>::t *Vx,
                           int nx, int ny, int nz, int layer, int rgs, typename c2<T>::t *rpart,
                           typename c2<T>::t *sv, hipStream_t s) {
    hipLaunchKernelGGL((k_ring_inv_rows<T, MAXC>), dim3(nz * rgs), dim3(256), 0, s, Xh, Vy, Vx, nx, ny, layer, rgs,
                       rpart, sv);
    return hipGetLastError();
}

// work: rpart (Nz * RING_RG * 2 Nx), sv (Nz * 2 Ny), rsum (Nz * 2 Nx)
template <typename T>
hipError_t inv_launch(const typename c2<T>::t *Xh, typename c2<T>::t *ring, const typename c2<T>::t *Vy,
                      const typename c2<T>::t *VyT, const typename c2<T>::t *Vx, const typename c2<T>::t *VxT, int nx,
                      int ny, int nz, int layer, typename c2<T>::t *rpart, typename c2<T>::t *sv,
                      typename c2<T>::t *rsum, hipStream_t s) {
    if (nx > RING_NMAX || ny > RING_NMAX || layer < 0 || layer > 1 || nx < 2 || ny < 2) return hipErrorInvalidValue;
    int rgs;
    hipError_t e;
    if (nx <= 256) {
        rgs = ring_groups<T, 4>(nz);
        e = inv_rows_launch<T, 4>(Xh, Vy, Vx, nx, ny, nz, layer, rgs, rpart, sv, s);
    } else if (nx <= 512) {
        rgs = ring_groups<T, 8>(nz);
        e = inv_rows_launch<T, 8>(Xh, Vy, Vx, nx, ny, nz, layer, rgs, rpart, sv, s);
    } else {
        rgs = ring_groups<T, 13>(nz);
        e = inv_rows_launch<T, 13>(Xh, Vy, Vx, nx, ny, nz, layer, rgs, rpart, sv, s);
    }
    if (e != hipSuccess) return e;
    const long long nr = 2LL * nz * nx;
    hipLaunchKernelGGL(k_ring_inv_sum<T>, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s, rpart, nx, rgs, nr, rsum);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // boundary rows X[j][i] = sum_k V_x[i][k] r_j[k]: rows (2 Nz x Nx) = rsum V_x^T; boundary columns
    // X[j][i] = sum_m V_y[j][m] s_i[m]: columns (2 Nz x Ny) = sv V_y^T
    return gemm_pair(plain_desc(2 * nz, nx, nx), rsum, VxT, ring, plain_desc(2 * nz, ny, ny), sv, VyT, ring + nr, s);
}

// work: Rr (Nz * 2 Nx) and Rc (Nz * 2 Ny) contiguous in rbuf, fvec (Nz * (2 Nx + 2 Ny))
template <typename T>
hipError_t fwd_launch(const typename c2<T>::t *ra, const typename c2<T>::t *rb, const typename c2<T>::t *ra1,
                      const typename c2<T>::t *rb1, const typename c2<T>::t *base, double base_scale,
                      typename c2<T>::t *out, const typename c2<T>::t *WyT, const typename c2<T>::t *WxT, double2 ex,
                      double2 ey, double2 ex1, double2 ey1, int nx, int ny, int nz, typename c2<T>::t *rbuf,
                      typename c2<T>::t *fvec, hipStream_t s) {
    const long long nr = 2LL * nz * nx, nc = 2LL * nz * ny;
    if (nx < 2 || ny < 2 || (rb1 && !ra1)) return hipErrorInvalidValue;
    typename c2<T>::t *Rr = rbuf, *Rc = rbuf + nr;
    hipLaunchKernelGGL(k_ring_fwd_R<T>, dim3((unsigned)((nr + nc + 255) / 256)), dim3(256), 0, s, ra, rb, ra1, rb1, ex,
                       ey, ex1, ey1, nx, ny, nz, Rr, Rc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // S = Rr W_x^T and T = Rc W_y^T
    if ((e = gemm_pair(plain_desc(2 * nz, nx, nx), Rr, WxT, fvec, plain_desc(2 * nz, ny, ny), Rc, WyT, fvec + nr, s)) !=
        hipSuccess)
        return e;
    const long long blocks = (long long)nz * ((ny + FWD_RJ - 1) / FWD_RJ);
    hipLaunchKernelGGL(k_ring_fwd_write<T>, dim3((unsigned)blocks), dim3(256), 0, s, fvec, base, (T)base_scale, out,
                       WyT, WxT, nx, ny, nz);
    return hipGetLastError();
}

// FFT4 / FFT6 (the compact operators with constant k0 and Dirichlet closures): after the 3D sine transform every
// mode (p, q, r) is an eigenvector; divide by the scheme's symbol in t_a = (2 cos(pi p_a h_a) - 2) / h_a^2:
//   order 4: sum t + sum_{a<b} (h_a^2 + h_b^2)/12 t_a t_b + k0^2 (1 + sum h_a^2/12 t_a)   (eq. scheme4)
//   order 6: (1 + h^2 k0^2/30) sum t + h^4/30 t_x t_y t_z + k0^2 + h^2/6 (1 + h^2 k0^2/15) sum_{a<b} t_a t_b
//            - h^2 k0^4/20                                                                (eq. scheme6, uniform h)
template <typename T>
__global__ __launch_bounds__(256) void k_sym_divide(typename c2<T>::t *__restrict__ u, const double *__restrict__ tx,
                                                    const double *__restrict__ ty, const double *__restrict__ tz,
                                                    int nx, int ny, int nz, SymParams q) {
    const long long n = (long long)nx * ny * nz;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int i = (int)(p % nx), j = (int)((p / nx) % ny), l = (int)(p / ((long long)nx * ny));
    const double a = tx[i], b = ty[j], c = tz[l];
    const double s1 = a + b + c, s2 = a * b + a * c + b * c;
    double lam;
    if (q.order == 4) {
        lam = s1 + (q.h2[0] + q.h2[1]) / 12.0 * a * b + (q.h2[0] + q.h2[2]) / 12.0 * a * c +
              (q.h2[1] + q.h2[2]) / 12.0 * b * c + q.k2 * (1.0 + (q.h2[0] * a + q.h2[1] * b + q.h2[2] * c) / 12.0);
    } else {
        const double h2 = q.h2[0];
        lam = (1.0 + h2 * q.k2 / 30.0) * s1 + h2 * h2 / 30.0 * a * b * c + q.k2 + h2 / 6.0 * (1.0 + h2 * q.k2 / 15.0) * s2 -
              h2 * q.k2 * q.k2 / 20.0;
    }
    const T r = (T)(1.0 / lam);
    typename c2<T>::t v = u[p];
    v.x *= r;
    v.y *= r;
    u[p] = v;
}

}  // namespace

hipError_t launch_sym_divide_z64(double2 *u, const double *tx, const double *ty, const double *tz, int nx, int ny,
                                 int nz, const SymParams &q, hipStream_t s) {
    const long long n = (long long)nx * ny * nz;
    hipLaunchKernelGGL(k_sym_divide<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, u, tx, ty, tz, nx, ny,
                       nz, q);
    return hipGetLastError();
}

hipError_t launch_sym_divide_z32(float2 *u, const double *tx, const double *ty, const double *tz, int nx, int ny,
                                 int nz, const SymParams &q, hipStream_t s) {
    const long long n = (long long)nx * ny * nz;
    hipLaunchKernelGGL(k_sym_divide<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, u, tx, ty, tz, nx, ny,
                       nz, q);
    return hipGetLastError();
}

int ring_rowgroups() { return RING_RG; }
int ring_max_n() { return RING_NMAX; }

hipError_t launch_ring_inverse_z64(const double2 *Xh, double2 *ring, const double2 *Vy, const double2 *VyT,
                                   const double2 *Vx, const double2 *VxT, int nx, int ny, int nz, int layer,
                                   double2 *rpart, double2 *sv, double2 *rsum, hipStream_t s) {
    return inv_launch<double>(Xh, ring, Vy, VyT, Vx, VxT, nx, ny, nz, layer, rpart, sv, rsum, s);
}
hipError_t launch_ring_inverse_z32(const float2 *Xh, float2 *ring, const float2 *Vy, const float2 *VyT,
                                   const float2 *Vx, const float2 *VxT, int nx, int ny, int nz, int layer,
                                   float2 *rpart, float2 *sv, float2 *rsum, hipStream_t s) {
    return inv_launch<float>(Xh, ring, Vy, VyT, Vx, VxT, nx, ny, nz, layer, rpart, sv, rsum, s);
}
hipError_t launch_ring_forward_z64(const double2 *ra, const double2 *rb, const double2 *ra1, const double2 *rb1,
                                   const double2 *base, double base_scale, double2 *out, const double2 *WyT,
                                   const double2 *WxT, double2 ex, double2 ey, double2 ex1, double2 ey1, int nx,
                                   int ny, int nz, double2 *rbuf, double2 *fvec, hipStream_t s) {
    return fwd_launch<double>(ra, rb, ra1, rb1, base, base_scale, out, WyT, WxT, ex, ey, ex1, ey1, nx, ny, nz, rbuf,
                              fvec, s);
}
hipError_t launch_ring_forward_z32(const float2 *ra, const float2 *rb, const float2 *ra1, const float2 *rb1,
                                   const float2 *base, double base_scale, float2 *out, const float2 *WyT,
                                   const float2 *WxT, double2 ex, double2 ey, double2 ex1, double2 ey1, int nx, int ny,
                                   int nz, float2 *rbuf, float2 *fvec, hipStream_t s) {
    return fwd_launch<float>(ra, rb, ra1, rb1, base, base_scale, out, WyT, WxT, ex, ey, ex1, ey1, nx, ny, nz, rbuf,
                             fvec, s);
}

}  // namespace helm
