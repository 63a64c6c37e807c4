// Thin per-slice transforms of the PFFT preconditioner (Sec. 4.2): only the boundary faces of every slice
// take part, so each costs O(N_x N_y) per slice instead of a dense transform.
//
// Ring layout of one slice (stride RS = 2 Nx + 2 Ny): [0, Nx) row j = 0; [Nx, 2Nx) row j = Ny-1;
// [2Nx, 2Nx+Ny) column i = 0 for all j; [2Nx+Ny, 2Nx+2Ny) column i = Nx-1 for all j (the corners appear in
// both a row and a column; consumers take them from the rows).
//
// k_ring_inverse: the inverse transform X = V_y Xh V_x^T evaluated on the faces only (eq. PFFT_INV): the two
//   boundary rows via r_j = V_y[j,:] Xh then X[j,i] = sum_k V_x[i,k] r_j[k], the two boundary columns via
//   s_i = Xh V_x[i,:]^T then X[j,i] = sum_m V_y[j,m] s_i[m]. One pass over the slice.
// k_ring_forward: the forward transform of ring-supported data R (Steps 1, 2*): R = E (a + b) with E the
//   diagonal (A_p^F - A_p) restricted to the faces, E = -a_x gamma_x on the x-faces plus -a_y gamma_y on the
//   y-faces; out = s * base + W_y R W_x^T computed as two rank-2 updates from the boundary rows
//   (S_m = R[m,:] W_x^T) and the interior parts of the boundary columns (T_k = W_y[:, inner] R[inner, k]).
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

constexpr int MAXC = 8;   // N <= 512: up to 8 chunks of 64 columns per lane

template <typename T>
__global__ __launch_bounds__(256) void k_ring_inverse(const typename c2<T>::t *__restrict__ Xh,
                                                      typename c2<T>::t *__restrict__ ring,
                                                      const typename c2<T>::t *__restrict__ Vy,
                                                      const typename c2<T>::t *__restrict__ VyT,
                                                      const typename c2<T>::t *__restrict__ Vx,
                                                      const typename c2<T>::t *__restrict__ VxT, int nx, int ny) {
    typedef typename c2<T>::t CT;
    extern __shared__ unsigned char smem[];
    CT *rpart = (CT *)smem;                 // [4][2][nx]
    CT *sv = rpart + 8 * nx;                // [2][ny]
    CT *vy0 = sv + 2 * ny;                  // Vy[0][m]
    CT *vyN = vy0 + ny;                     // Vy[ny-1][m]
    CT *vx0 = vyN + ny;                     // Vx[0][k]
    CT *vxN = vx0 + nx;                     // Vx[nx-1][k]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l = blockIdx.x;
    const CT *X = Xh + (long long)l * nx * ny;
    for (int m = tid; m < ny; m += 256) { vy0[m] = Vy[m]; vyN[m] = Vy[(long long)(ny - 1) * ny + m]; }
    for (int k = tid; k < nx; k += 256) { vx0[k] = Vx[k]; vxN[k] = Vx[(long long)(nx - 1) * nx + k]; }
    __syncthreads();
    CT a0[MAXC], aN[MAXC];
#pragma unroll
    for (int c = 0; c < MAXC; ++c) { a0[c] = cz<CT>(); aN[c] = cz<CT>(); }
    for (int m = wave; m < ny; m += 4) {
        const CT *row = X + (long long)m * nx;
        const CT w0 = vy0[m], wN = vyN[m];
        CT s0 = cz<CT>(), sN = cz<CT>();
#pragma unroll
        for (int c = 0; c < MAXC; ++c) {
            const int k = lane + 64 * c;
            if (k < nx) {
                CT x = row[k];
                a0[c] = cfma(w0, x, a0[c]);
                aN[c] = cfma(wN, x, aN[c]);
                s0 = cfma(vx0[k], x, s0);
                sN = cfma(vxN[k], x, sN);
            }
        }
        s0.x = wsum(s0.x); s0.y = wsum(s0.y);
        sN.x = wsum(sN.x); sN.y = wsum(sN.y);
        if (lane == 0) { sv[m] = s0; sv[ny + m] = sN; }
    }
#pragma unroll
    for (int c = 0; c < MAXC; ++c) {
        const int k = lane + 64 * c;
        if (k < nx) { rpart[(wave * 2 + 0) * nx + k] = a0[c]; rpart[(wave * 2 + 1) * nx + k] = aN[c]; }
    }
    __syncthreads();
    for (int k = tid; k < nx; k += 256) {
        CT r0 = rpart[k], rN = rpart[nx + k];
        for (int w = 1; w < 4; ++w) { r0 = cadd(r0, rpart[(w * 2) * nx + k]); rN = cadd(rN, rpart[(w * 2 + 1) * nx + k]); }
        rpart[k] = r0;
        rpart[nx + k] = rN;
    }
    __syncthreads();
    CT *out = ring + (long long)l * (2 * nx + 2 * ny);
    for (int i = tid; i < nx; i += 256) {           // boundary rows: X[j][i] = sum_k Vx[i][k] r_j[k]
        CT o0 = cz<CT>(), oN = cz<CT>();
        for (int k = 0; k < nx; ++k) {
            CT v = VxT[(long long)k * nx + i];
            o0 = cfma(v, rpart[k], o0);
            oN = cfma(v, rpart[nx + k], oN);
        }
        out[i] = o0;
        out[nx + i] = oN;
    }
    for (int j = tid; j < ny; j += 256) {           // boundary columns: X[j][i] = sum_m Vy[j][m] s_i[m]
        CT o0 = cz<CT>(), oN = cz<CT>();
        for (int m = 0; m < ny; ++m) {
            CT v = VyT[(long long)m * ny + j];
            o0 = cfma(v, sv[m], o0);
            oN = cfma(v, sv[ny + m], oN);
        }
        out[2 * nx + j] = o0;
        out[2 * nx + ny + j] = oN;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_ring_forward(const typename c2<T>::t *__restrict__ ra,
                                                      const typename c2<T>::t *__restrict__ rb,
                                                      const typename c2<T>::t *base, T base_scale,
                                                      typename c2<T>::t *out,
                                                      const typename c2<T>::t *__restrict__ Wy,
                                                      const typename c2<T>::t *__restrict__ WyT,
                                                      const typename c2<T>::t *__restrict__ Wx,
                                                      const typename c2<T>::t *__restrict__ WxT, double2 ex, double2 ey,
                                                      int nx, int ny) {
    typedef typename c2<T>::t CT;
    extern __shared__ unsigned char smem[];
    CT *R0 = (CT *)smem;        // R row 0        [nx]
    CT *RN = R0 + nx;           // R row ny-1     [nx]
    CT *C0 = RN + nx;           // R column 0     [ny] (interior rows only)
    CT *CN = C0 + ny;           // R column nx-1  [ny]
    CT *S0 = CN + ny;           // S_0[i]         [nx]
    CT *SN = S0 + nx;           // S_N[i]         [nx]
    CT *T0 = SN + nx;           // T_0[j]         [ny]
    CT *TN = T0 + ny;           // T_N[j]         [ny]
    CT *wy0 = TN + ny;          // Wy[j][0]       [ny]
    CT *wyN = wy0 + ny;         // Wy[j][ny-1]    [ny]
    CT *wx0 = wyN + ny;         // Wx[i][0]       [nx]
    CT *wxN = wx0 + nx;         // Wx[i][nx-1]    [nx]
    const int tid = threadIdx.x;
    const int l = blockIdx.x;
    const int RS = 2 * nx + 2 * ny;
    const CT *A = ra + (long long)l * RS;
    const CT *B = rb ? rb + (long long)l * RS : nullptr;
    CT ecx, ecy, ecc;
    ecx.x = (T)ex.x; ecx.y = (T)ex.y;
    ecy.x = (T)ey.x; ecy.y = (T)ey.y;
    ecc = cadd(ecx, ecy);
    for (int k = tid; k < nx; k += 256) {
        CT v0 = A[k], vN = A[nx + k];
        if (B) { v0 = cadd(v0, B[k]); vN = cadd(vN, B[nx + k]); }
        const CT e = (k == 0 || k == nx - 1) ? ecc : ecy;
        R0[k] = cmul(e, v0);
        RN[k] = cmul(e, vN);
        wx0[k] = Wx[(long long)k * nx];
        wxN[k] = Wx[(long long)k * nx + nx - 1];
    }
    for (int m = tid; m < ny; m += 256) {
        CT v0 = A[2 * nx + m], vN = A[2 * nx + ny + m];
        if (B) { v0 = cadd(v0, B[2 * nx + m]); vN = cadd(vN, B[2 * nx + ny + m]); }
        const bool inner = m > 0 && m < ny - 1;
        C0[m] = inner ? cmul(ecx, v0) : cz<CT>();
        CN[m] = inner ? cmul(ecx, vN) : cz<CT>();
        wy0[m] = Wy[(long long)m * ny];
        wyN[m] = Wy[(long long)m * ny + ny - 1];
    }
    __syncthreads();
    for (int i = tid; i < nx; i += 256) {           // S_m[i] = sum_k Wx[i][k] R[m][k]
        CT s0 = cz<CT>(), sN = cz<CT>();
        for (int k = 0; k < nx; ++k) {
            CT v = WxT[(long long)k * nx + i];
            s0 = cfma(v, R0[k], s0);
            sN = cfma(v, RN[k], sN);
        }
        S0[i] = s0;
        SN[i] = sN;
    }
    for (int j = tid; j < ny; j += 256) {           // T_k[j] = sum_{m inner} Wy[j][m] R[m][k]
        CT t0 = cz<CT>(), tN = cz<CT>();
        for (int m = 1; m < ny - 1; ++m) {
            CT v = WyT[(long long)m * ny + j];
            t0 = cfma(v, C0[m], t0);
            tN = cfma(v, CN[m], tN);
        }
        T0[j] = t0;
        TN[j] = tN;
    }
    __syncthreads();
    CT *O = out + (long long)l * nx * ny;
    const CT *Bs = base ? base + (long long)l * nx * ny : nullptr;
    const long long total = (long long)nx * ny;
    for (long long p = tid; p < total; p += 256) {
        const int j = (int)(p / nx), i = (int)(p % nx);
        CT acc = cz<CT>();
        if (Bs) { acc = Bs[p]; acc.x *= base_scale; acc.y *= base_scale; }
        acc = cfma(wy0[j], S0[i], acc);
        acc = cfma(wyN[j], SN[i], acc);
        acc = cfma(T0[j], wx0[i], acc);
        acc = cfma(TN[j], wxN[i], acc);
        O[p] = acc;
    }
}

template <typename T>
hipError_t inv_launch(const typename c2<T>::t *Xh, typename c2<T>::t *ring, const typename c2<T>::t *Vy,
                      const typename c2<T>::t *VyT, const typename c2<T>::t *Vx, const typename c2<T>::t *VxT, int nx,
                      int ny, int nz, hipStream_t s) {
    if (nx > 64 * MAXC || ny > 64 * MAXC) return hipErrorInvalidValue;
    size_t shm = sizeof(typename c2<T>::t) * (size_t)(8 * nx + 2 * ny + 2 * ny + 2 * nx);
    hipLaunchKernelGGL(k_ring_inverse<T>, dim3(nz), dim3(256), shm, s, Xh, ring, Vy, VyT, Vx, VxT, nx, ny);
    return hipGetLastError();
}

template <typename T>
hipError_t fwd_launch(const typename c2<T>::t *ra, const typename c2<T>::t *rb, const typename c2<T>::t *base,
                      double base_scale, typename c2<T>::t *out, const typename c2<T>::t *Wy,
                      const typename c2<T>::t *WyT, const typename c2<T>::t *Wx, const typename c2<T>::t *WxT,
                      double2 ex, double2 ey, int nx, int ny, int nz, hipStream_t s) {
    size_t shm = sizeof(typename c2<T>::t) * (size_t)(6 * nx + 6 * ny);
    hipLaunchKernelGGL(k_ring_forward<T>, dim3(nz), dim3(256), shm, s, ra, rb, base, (T)base_scale, out, Wy, WyT, Wx,
                       WxT, ex, ey, nx, ny);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ring_inverse_z64(const double2 *Xh, double2 *ring, const double2 *Vy, const double2 *VyT,
                                   const double2 *Vx, const double2 *VxT, int nx, int ny, int nz, hipStream_t s) {
    return inv_launch<double>(Xh, ring, Vy, VyT, Vx, VxT, nx, ny, nz, s);
}
hipError_t launch_ring_inverse_z32(const float2 *Xh, float2 *ring, const float2 *Vy, const float2 *VyT,
                                   const float2 *Vx, const float2 *VxT, int nx, int ny, int nz, hipStream_t s) {
    return inv_launch<float>(Xh, ring, Vy, VyT, Vx, VxT, nx, ny, nz, s);
}
hipError_t launch_ring_forward_z64(const double2 *ra, const double2 *rb, const double2 *base, double base_scale,
                                   double2 *out, const double2 *Wy, const double2 *WyT, const double2 *Wx,
                                   const double2 *WxT, double2 ex, double2 ey, int nx, int ny, int nz, hipStream_t s) {
    return fwd_launch<double>(ra, rb, base, base_scale, out, Wy, WyT, Wx, WxT, ex, ey, nx, ny, nz, s);
}
hipError_t launch_ring_forward_z32(const float2 *ra, const float2 *rb, const float2 *base, double base_scale,
                                   float2 *out, const float2 *Wy, const float2 *WyT, const float2 *Wx,
                                   const float2 *WxT, double2 ex, double2 ey, int nx, int ny, int nz, hipStream_t s) {
    return fwd_launch<float>(ra, rb, base, base_scale, out, Wy, WyT, Wx, WxT, ex, ey, nx, ny, nz, s);
}

}  // namespace helm
