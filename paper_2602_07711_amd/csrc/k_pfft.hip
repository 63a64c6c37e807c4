// Thin per-slice transforms of the PFFT preconditioner (Sec. 4.2): only the boundary faces of every slice
// take part, so each costs O(N_x N_y) per slice instead of a dense transform.
//
// Ring layout of one slice (stride RS = 2 Nx + 2 Ny): [0, Nx) row j = 0; [Nx, 2Nx) row j = Ny-1;
// [2Nx, 2Nx+Ny) column i = 0 for all j; [2Nx+Ny, 2Nx+2Ny) column i = Nx-1 for all j (the corners appear in
// both a row and a column; consumers take them from the rows).
//
// Inverse (k_ring_inv_rows + k_ring_inv_finish): the inverse transform X = V_y Xh V_x^T evaluated on the faces
//   only (eq. PFFT_INV): the two boundary rows via r_j = V_y[j,:] Xh then X[j,i] = sum_k V_x[i,k] r_j[k], the two
//   boundary columns via s_i = Xh V_x[i,:]^T then X[j,i] = sum_m V_y[j,m] s_i[m]. The pass over the data runs
//   with several row groups per slice; the small products follow per slice.
// Forward (k_ring_fwd_prep + k_ring_fwd_write): the forward transform of ring-supported data R (Steps 1, 2*):
//   R = E (a + b) with E the diagonal (A_p^F - A_p) restricted to the faces, E = -a_x gamma_x on the x-faces plus
//   -a_y gamma_y on the y-faces; out = s * base + W_y R W_x^T computed as two rank-2 updates from the boundary rows
//   (S_m = R[m,:] W_x^T) and the interior parts of the boundary columns (T_k = W_y[:, inner] R[inner, k]); the
//   factors per slice first, then every element in parallel.
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

constexpr int MAXC = 4;   // N <= 256 (the PFFT limit): up to 4 chunks of 64 columns per lane
constexpr int RING_RG = 8; // row groups per slice in the inverse's pass over the data

// Inverse, pass over the data: block (slice l, row group rg) takes rows m of its group and accumulates, per
// column k, r0[k] += V_y[0][m] X[m][k] and rN[k] += V_y[ny-1][m] X[m][k] (partials per group), and per row the
// complete s0[m] = sum_k V_x[0][k] X[m][k], sN[m] = sum_k V_x[nx-1][k] X[m][k].
template <typename T>
__global__ __launch_bounds__(256) void k_ring_inv_rows(const typename c2<T>::t *__restrict__ Xh,
                                                       const typename c2<T>::t *__restrict__ Vy,
                                                       const typename c2<T>::t *__restrict__ Vx, int nx, int ny,
                                                       typename c2<T>::t *__restrict__ rpart,
                                                       typename c2<T>::t *__restrict__ sv) {
    typedef typename c2<T>::t CT;
    __shared__ CT red[4][2][64 * MAXC];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l = blockIdx.x / RING_RG, rg = blockIdx.x % RING_RG;
    const int per = (ny + RING_RG - 1) / RING_RG;
    const int m0 = rg * per, m1 = min(ny, m0 + per);
    const CT *X = Xh + (long long)l * nx * ny;
    CT vx0[MAXC], vxN[MAXC], a0[MAXC], aN[MAXC];
#pragma unroll
    for (int c = 0; c < MAXC; ++c) {
        const int k = lane + 64 * c;
        vx0[c] = k < nx ? Vx[k] : cz<CT>();
        vxN[c] = k < nx ? Vx[(long long)(nx - 1) * nx + k] : cz<CT>();
        a0[c] = cz<CT>();
        aN[c] = cz<CT>();
    }
    for (int m = m0 + wave; m < m1; m += 4) {
        const CT *row = X + (long long)m * nx;
        const CT w0 = Vy[m], wN = Vy[(long long)(ny - 1) * ny + m];
        CT s0 = cz<CT>(), sN = cz<CT>();
#pragma unroll
        for (int c = 0; c < MAXC; ++c) {
            const int k = lane + 64 * c;
            if (k < nx) {
                const CT x = row[k];
                a0[c] = cfma(w0, x, a0[c]);
                aN[c] = cfma(wN, x, aN[c]);
                s0 = cfma(vx0[c], x, s0);
                sN = cfma(vxN[c], x, sN);
            }
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
    CT *rp = rpart + ((long long)l * RING_RG + rg) * 2 * nx;
    for (int k = tid; k < nx; k += 256) {
        CT r0 = red[0][0][k], rN = red[0][1][k];
        for (int w = 1; w < 4; ++w) { r0 = cadd(r0, red[w][0][k]); rN = cadd(rN, red[w][1][k]); }
        rp[k] = r0;
        rp[nx + k] = rN;
    }
}

// Inverse, per slice: r0, rN summed over the row groups in order, then the boundary rows
// X[j][i] = sum_k V_x[i][k] r_j[k] and the boundary columns X[j][i] = sum_m V_y[j][m] s_i[m] into the ring.
template <typename T>
__global__ __launch_bounds__(256) void k_ring_inv_finish(const typename c2<T>::t *__restrict__ rpart,
                                                         const typename c2<T>::t *__restrict__ sv,
                                                         const typename c2<T>::t *__restrict__ VyT,
                                                         const typename c2<T>::t *__restrict__ VxT, int nx, int ny,
                                                         typename c2<T>::t *__restrict__ ring) {
    typedef typename c2<T>::t CT;
    extern __shared__ unsigned char smem[];
    CT *r = (CT *)smem;          // [2][nx]
    CT *sl = r + 2 * nx;         // [2][ny]
    const int tid = threadIdx.x, l = blockIdx.x;
    const CT *rp = rpart + (long long)l * RING_RG * 2 * nx;
    for (int k = tid; k < 2 * nx; k += 256) {
        CT acc = rp[k];
        for (int g = 1; g < RING_RG; ++g) acc = cadd(acc, rp[(long long)g * 2 * nx + k]);
        r[k] = acc;
    }
    for (int m = tid; m < 2 * ny; m += 256) sl[m] = sv[(long long)l * 2 * ny + m];
    __syncthreads();
    CT *out = ring + (long long)l * (2 * nx + 2 * ny);
    for (int i = tid; i < nx; i += 256) {
        CT o0 = cz<CT>(), oN = cz<CT>();
        for (int k = 0; k < nx; ++k) {
            const CT v = VxT[(long long)k * nx + i];
            o0 = cfma(v, r[k], o0);
            oN = cfma(v, r[nx + k], oN);
        }
        out[i] = o0;
        out[nx + i] = oN;
    }
    for (int j = tid; j < ny; j += 256) {
        CT o0 = cz<CT>(), oN = cz<CT>();
        for (int m = 0; m < ny; ++m) {
            const CT v = VyT[(long long)m * ny + j];
            o0 = cfma(v, sl[m], o0);
            oN = cfma(v, sl[ny + m], oN);
        }
        out[2 * nx + j] = o0;
        out[2 * nx + ny + j] = oN;
    }
}

// Forward, per slice: R = E (a + b) on the faces, then S_m[i] = sum_k W_x[i][k] R[m][k] for the boundary rows
// m and T_k[j] = sum_{m inner} W_y[j][m] R[m][k] for the interior parts of the boundary columns, written to
// fvec[l] = [S_0 | S_N | T_0 | T_N].
template <typename T>
__global__ __launch_bounds__(256) void k_ring_fwd_prep(const typename c2<T>::t *__restrict__ ra,
                                                       const typename c2<T>::t *__restrict__ rb,
                                                       const typename c2<T>::t *__restrict__ WyT,
                                                       const typename c2<T>::t *__restrict__ WxT, double2 ex,
                                                       double2 ey, int nx, int ny,
                                                       typename c2<T>::t *__restrict__ fvec) {
    typedef typename c2<T>::t CT;
    extern __shared__ unsigned char smem[];
    CT *R0 = (CT *)smem;        // R row 0        [nx]
    CT *RN = R0 + nx;           // R row ny-1     [nx]
    CT *C0 = RN + nx;           // R column 0     [ny] (interior rows only)
    CT *CN = C0 + ny;           // R column nx-1  [ny]
    const int tid = threadIdx.x, l = blockIdx.x;
    const int RS = 2 * nx + 2 * ny;
    const CT *A = ra + (long long)l * RS;
    const CT *B = rb ? rb + (long long)l * RS : nullptr;
    CT ecx, ecy;
    ecx.x = (T)ex.x; ecx.y = (T)ex.y;
    ecy.x = (T)ey.x; ecy.y = (T)ey.y;
    const CT ecc = cadd(ecx, ecy);
    for (int k = tid; k < nx; k += 256) {
        CT v0 = A[k], vN = A[nx + k];
        if (B) { v0 = cadd(v0, B[k]); vN = cadd(vN, B[nx + k]); }
        const CT e = (k == 0 || k == nx - 1) ? ecc : ecy;
        R0[k] = cmul(e, v0);
        RN[k] = cmul(e, vN);
    }
    for (int m = tid; m < ny; m += 256) {
        CT v0 = A[2 * nx + m], vN = A[2 * nx + ny + m];
        if (B) { v0 = cadd(v0, B[2 * nx + m]); vN = cadd(vN, B[2 * nx + ny + m]); }
        const bool inner = m > 0 && m < ny - 1;
        C0[m] = inner ? cmul(ecx, v0) : cz<CT>();
        CN[m] = inner ? cmul(ecx, vN) : cz<CT>();
    }
    __syncthreads();
    CT *fv = fvec + (long long)l * RS;
    for (int i = tid; i < nx; i += 256) {
        CT s0 = cz<CT>(), sN = cz<CT>();
        for (int k = 0; k < nx; ++k) {
            const CT v = WxT[(long long)k * nx + i];
            s0 = cfma(v, R0[k], s0);
            sN = cfma(v, RN[k], sN);
        }
        fv[i] = s0;
        fv[nx + i] = sN;
    }
    for (int j = tid; j < ny; j += 256) {
        CT t0 = cz<CT>(), tN = cz<CT>();
        for (int m = 1; m < ny - 1; ++m) {
            const CT v = WyT[(long long)m * ny + j];
            t0 = cfma(v, C0[m], t0);
            tN = cfma(v, CN[m], tN);
        }
        fv[2 * nx + j] = t0;
        fv[2 * nx + ny + j] = tN;
    }
}

// Forward, every element of every slice: out = s base + W_y[j][0] S_0[i] + W_y[j][ny-1] S_N[i]
// + T_0[j] W_x[i][0] + T_N[j] W_x[i][nx-1] (the boundary columns of W read as rows of the transposes)
template <typename T>
__global__ __launch_bounds__(256) void k_ring_fwd_write(const typename c2<T>::t *__restrict__ fvec,
                                                        const typename c2<T>::t *base, T base_scale,
                                                        typename c2<T>::t *out,
                                                        const typename c2<T>::t *__restrict__ WyT,
                                                        const typename c2<T>::t *__restrict__ WxT, int nx, int ny,
                                                        long long n) {
    typedef typename c2<T>::t CT;
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const long long plane = (long long)nx * ny;
    const int l = (int)(e / plane);
    const long long p = e - (long long)l * plane;
    const int j = (int)(p / nx), i = (int)(p % nx);
    const CT *fv = fvec + (long long)l * (2 * nx + 2 * ny);
    CT acc = cz<CT>();
    if (base) { acc = base[e]; acc.x *= base_scale; acc.y *= base_scale; }
    acc = cfma(WyT[j], fv[i], acc);
    acc = cfma(WyT[(long long)(ny - 1) * ny + j], fv[nx + i], acc);
    acc = cfma(fv[2 * nx + j], WxT[i], acc);
    acc = cfma(fv[2 * nx + ny + j], WxT[(long long)(nx - 1) * nx + i], acc);
    out[e] = acc;
}

template <typename T>
hipError_t inv_launch(const typename c2<T>::t *Xh, typename c2<T>::t *ring, const typename c2<T>::t *Vy,
                      const typename c2<T>::t *VyT, const typename c2<T>::t *Vx, const typename c2<T>::t *VxT, int nx,
                      int ny, int nz, typename c2<T>::t *rpart, typename c2<T>::t *sv, hipStream_t s) {
    if (nx > 64 * MAXC || ny > 64 * MAXC) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ring_inv_rows<T>, dim3(nz * RING_RG), dim3(256), 0, s, Xh, Vy, Vx, nx, ny, rpart, sv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t shm = sizeof(typename c2<T>::t) * (size_t)(2 * nx + 2 * ny);
    hipLaunchKernelGGL(k_ring_inv_finish<T>, dim3(nz), dim3(256), shm, s, rpart, sv, VyT, VxT, nx, ny, ring);
    return hipGetLastError();
}

template <typename T>
hipError_t fwd_launch(const typename c2<T>::t *ra, const typename c2<T>::t *rb, const typename c2<T>::t *base,
                      double base_scale, typename c2<T>::t *out, const typename c2<T>::t *WyT,
                      const typename c2<T>::t *WxT, double2 ex, double2 ey, int nx, int ny, int nz,
                      typename c2<T>::t *fvec, hipStream_t s) {
    const size_t shm = sizeof(typename c2<T>::t) * (size_t)(2 * nx + 2 * ny);
    hipLaunchKernelGGL(k_ring_fwd_prep<T>, dim3(nz), dim3(256), shm, s, ra, rb, WyT, WxT, ex, ey, nx, ny, fvec);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long n = (long long)nx * ny * nz;
    hipLaunchKernelGGL(k_ring_fwd_write<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, fvec, base,
                       (T)base_scale, out, WyT, WxT, nx, ny, n);
    return hipGetLastError();
}

}  // namespace

int ring_rowgroups() { return RING_RG; }

hipError_t launch_ring_inverse_z64(const double2 *Xh, double2 *ring, const double2 *Vy, const double2 *VyT,
                                   const double2 *Vx, const double2 *VxT, int nx, int ny, int nz, double2 *rpart,
                                   double2 *sv, hipStream_t s) {
    return inv_launch<double>(Xh, ring, Vy, VyT, Vx, VxT, nx, ny, nz, rpart, sv, s);
}
hipError_t launch_ring_inverse_z32(const float2 *Xh, float2 *ring, const float2 *Vy, const float2 *VyT,
                                   const float2 *Vx, const float2 *VxT, int nx, int ny, int nz, float2 *rpart,
                                   float2 *sv, hipStream_t s) {
    return inv_launch<float>(Xh, ring, Vy, VyT, Vx, VxT, nx, ny, nz, rpart, sv, s);
}
hipError_t launch_ring_forward_z64(const double2 *ra, const double2 *rb, const double2 *base, double base_scale,
                                   double2 *out, const double2 *WyT, const double2 *WxT, double2 ex, double2 ey,
                                   int nx, int ny, int nz, double2 *fvec, hipStream_t s) {
    return fwd_launch<double>(ra, rb, base, base_scale, out, WyT, WxT, ex, ey, nx, ny, nz, fvec, s);
}
hipError_t launch_ring_forward_z32(const float2 *ra, const float2 *rb, const float2 *base, double base_scale,
                                   float2 *out, const float2 *WyT, const float2 *WxT, double2 ex, double2 ey, int nx,
                                   int ny, int nz, float2 *fvec, hipStream_t s) {
    return fwd_launch<float>(ra, rb, base, base_scale, out, WyT, WxT, ex, ey, nx, ny, nz, fvec, s);
}

}  // namespace helm
