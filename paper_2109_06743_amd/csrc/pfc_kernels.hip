// PFC advection sweeps for gfx950: x (periodic), y (reflecting walls, pencil
// pairs +v_y / -v_y), v in 1V (zero-flux) and the five-sweep 3V velocity
// operator (zero-flux), plus the array maximum that bounds the limiter.
//
// Scheme: positive and flux-conservative semi-Lagrangian sweep (Sec. 2.1 of
// arXiv 2109.06743, which uses the PFC scheme of Filbet, Sonnendruecker and
// Bertrand).  For a uniform displacement s = K + a (K = floor, s >= 0) the
// flux-form update telescopes to
//     f'_i = f_{i-K} + phi(i-K-1) - phi(i-K),
// phi(j) the limited partial flux of cell j (pfc_phi).  Negative shifts run
// the same formula on the mirrored pencil.  Integer shifts give a = 0 and
// therefore an exact (bitwise) shift.
#include "vl_internal.h"

namespace vl {

// ---------------------------------------------------------------------------
// x sweep: layout [rows][nx][Nv]; each thread owns one velocity index v of one
// row and CX consecutive output cells; lanes run over contiguous v, so every
// load and store of a wave is one contiguous 256-byte (FP32) segment.  The
// thread keeps a window of CX+3 inputs in registers, ordered upwind to
// downwind, so both signs of the shift run the same straight-line code.
template <class T, int CX>
__global__ void __launch_bounds__(256)
pfc_x_kernel(const T* __restrict__ fin, T* __restrict__ fout, int nx, long long Nv, int inner,
             double vx_lo, double dvx, double tau_dx, const T* __restrict__ finf_p,
             typename Bits<T>::U* __restrict__ max_out) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int c0 = blockIdx.y * CX;
    const long long row = blockIdx.z;
    const T finf = *finf_p;
    T mx = T(0);
    if (v < Nv) {
        const int ivx = (int)(v / inner);
        const double s = (vx_lo + (ivx + 0.5) * dvx) * tau_dx;
        const bool pos = s >= 0.0;
        const Shift<T> sh(fabs(s));
        const int K = (int)(sh.K % nx);
        const T* __restrict__ src = fin + row * nx * Nv + v;
        T* __restrict__ dst = fout + row * nx * Nv + v;
        int idx = pos ? (c0 - K - 2) : (c0 + K + CX + 1);
        idx %= nx;
        if (idx < 0) idx += nx;
        const int step = pos ? 1 : -1;
        T W[CX + 3];
#pragma unroll
        for (int w = 0; w < CX + 3; ++w) {
            W[w] = src[(long long)idx * Nv];
            idx += step;
            if (idx >= nx) idx -= nx;
            if (idx < 0) idx += nx;
        }
        T phi_prev = pfc_phi(W[0], W[1], W[2], sh.a, sh.c1, sh.c2, finf);
#pragma unroll
        for (int r = 0; r < CX; ++r) {
            const T phi_next = pfc_phi(W[r + 1], W[r + 2], W[r + 3], sh.a, sh.c1, sh.c2, finf);
            const T o = fmax(W[r + 2] + phi_prev - phi_next, T(0));
            phi_prev = phi_next;
            const int oi = pos ? (c0 + r) : (c0 + CX - 1 - r);
            if (oi < nx) {
                dst[(long long)oi * Nv] = o;
                mx = fmax(mx, o);
            }
        }
    }
    if (max_out) block_max_to(mx, max_out);
}

// ---------------------------------------------------------------------------
// y sweep between reflecting walls: the pencil at +v_y (rows 0..ny-1) followed
// by its mirror pencil at -v_y in reverse row order is one periodic pencil of
// length 2 ny moving uniformly by v_y tau / dy > 0.  A thread owns one pair and
// CY consecutive positions of the doubled pencil.  Odd nvy: the v_y = 0 pencil
// pairs with itself at zero shift (an exact copy).
template <class T, int CY>
__global__ void __launch_bounds__(256)
pfc_y_kernel(const T* __restrict__ fin, T* __restrict__ fout, int nx, int ny, long long Nv, int nvx,
             int nvy, int nvz, double vy_lo, double dvy, double tau_dy, const T* __restrict__ finf_p,
             typename Bits<T>::U* __restrict__ max_out) {
    const int half = (nvy + 1) / 2;                 // pairs per (ivx, ivz), incl. a v_y = 0 self-pair
    const long long npairs = (long long)nvx * half * nvz;
    const long long pid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int c0 = blockIdx.y * CY;
    const int ix = blockIdx.z;
    const T finf = *finf_p;
    T mx = T(0);
    if (pid < npairs) {
        const int ivz = (int)(pid % nvz);
        const long long rest = pid / nvz;
        const int jh = (int)(rest % half);
        const int ivx = (int)(rest / half);
        const int jup = nvy - half + jh;            // v_y >= 0 half
        const int jdn = nvy - 1 - jup;              // its mirror
        const long long vup = ((long long)ivx * nvy + jup) * nvz + ivz;
        const long long vdn = ((long long)ivx * nvy + jdn) * nvz + ivz;
        const double s = (jup == jdn) ? 0.0 : (vy_lo + (jup + 0.5) * dvy) * tau_dy;
        const Shift<T> sh(s);
        const int L2 = 2 * ny;
        const int K = (int)(sh.K % L2);
        const long long rowstride = (long long)nx * Nv;
        const T* __restrict__ src = fin + (long long)ix * Nv;
        T* __restrict__ dst = fout + (long long)ix * Nv;
        int p = (c0 - K - 2) % L2;
        if (p < 0) p += L2;
        T W[CY + 3];
#pragma unroll
        for (int w = 0; w < CY + 3; ++w) {
            const long long off = (p < ny) ? (long long)p * rowstride + vup
                                           : (long long)(L2 - 1 - p) * rowstride + vdn;
            W[w] = src[off];
            if (++p == L2) p = 0;
        }
        T phi_prev = pfc_phi(W[0], W[1], W[2], sh.a, sh.c1, sh.c2, finf);
#pragma unroll
        for (int r = 0; r < CY; ++r) {
            const T phi_next = pfc_phi(W[r + 1], W[r + 2], W[r + 3], sh.a, sh.c1, sh.c2, finf);
            const T o = fmax(W[r + 2] + phi_prev - phi_next, T(0));
            phi_prev = phi_next;
            const int q = c0 + r;
            if (q < L2) {
                const long long off = (q < ny) ? (long long)q * rowstride + vup
                                               : (long long)(L2 - 1 - q) * rowstride + vdn;
                dst[off] = o;
                mx = fmax(mx, o);
            }
        }
    }
    if (max_out) block_max_to(mx, max_out);
}

// ---------------------------------------------------------------------------
// Zero-flux sweep of one pencil held in shared memory, in upwind-to-downwind
// order g[0..n-1] with two zero ghosts on each side (index k lives at g[k+2]).
// With h_k = g_k + phi(k-1) - phi(k) (h_n = phi(n-1)), the output at position
// p is 0 for p < K, h_{p-K} for K <= p < n-1, and the wall cell n-1 keeps all
// the mass that would have crossed it: sum_{k >= n-1-K} h_k.
template <class T>
__device__ __forceinline__ T zeroflux_out(const T* g, int n, int p, long long K, const Shift<T>& sh, T finf) {
    if (p < n - 1) {
        if ((long long)p < K) return T(0);
        const int k = p - (int)K;
        const T pm = pfc_phi(g[k], g[k + 1], g[k + 2], sh.a, sh.c1, sh.c2, finf);   // phi(k-1)
        const T p0 = pfc_phi(g[k + 1], g[k + 2], g[k + 3], sh.a, sh.c1, sh.c2, finf); // phi(k)
        return fmax(g[k + 2] + pm - p0, T(0));
    }
    long long k0 = (long long)(n - 1) - K;
    if (k0 < 0) k0 = 0;
    T acc = T(0);
    T pm = pfc_phi(g[k0], g[k0 + 1], g[k0 + 2], sh.a, sh.c1, sh.c2, finf);
    for (int k = (int)k0; k <= n; ++k) {
        const T p0 = pfc_phi(g[k + 1], g[k + 2], g[k + 3], sh.a, sh.c1, sh.c2, finf);
        acc += g[k + 2] + pm - p0;
        pm = p0;
    }
    return fmax(acc, T(0));
}

// 1V velocity sweep: one block per spatial cell, the pencil staged in shared
// memory (nv + 4 values).  s = (q/m) E_i tau / dv.  In place is allowed.
template <class T>
__global__ void __launch_bounds__(256)
pfc_v1_kernel(const T* fin, T* fout, int nv, const double* __restrict__ E, double qm_tau_dv,
              const T* __restrict__ finf_p, typename Bits<T>::U* __restrict__ max_out) {
    extern __shared__ unsigned char smem_raw[];
    T* g = reinterpret_cast<T*>(smem_raw);
    const int ix = blockIdx.x;
    const double s = qm_tau_dv * E[ix];
    const bool pos = s >= 0.0;
    const Shift<T> sh(fabs(s));
    const T finf = *finf_p;
    const T* src = fin + (long long)ix * nv;
    T* dst = fout + (long long)ix * nv;
    for (int k = threadIdx.x; k < nv + 4; k += blockDim.x) {
        const int j = k - 2;
        g[k] = (j >= 0 && j < nv) ? src[pos ? j : nv - 1 - j] : T(0);
    }
    __syncthreads();
    T mx = T(0);
    for (int p = threadIdx.x; p < nv; p += blockDim.x) {
        const T o = zeroflux_out(g, nv, p, sh.K, sh, finf);
        dst[pos ? p : nv - 1 - p] = o;
        mx = fmax(mx, o);
    }
    if (max_out) block_max_to(mx, max_out);
}

// ---------------------------------------------------------------------------
// 3V velocity operator V(tau): one block per spatial cell; the velocity block
// lives in shared memory with rows along v_z padded to an odd length, so a
// wave reading pencils along any of the three axes hits distinct banks.  Each
// thread owns whole pencils of the current sweep (at most NMAX long) in
// registers; the displaced results are written back in place.  The five
// sweeps are vx(tau/2) vy(tau/2) vz(tau) vy(tau/2) vx(tau/2), each a uniform
// shift by (q/m)(E_d + (v x B)_d) at the pencil's transverse velocities.
template <class T, int NMAX>
__device__ __forceinline__ void sweep3(T* blk, int d, double sigma, const V3Params& P, const double* EB,
                                       T finf) {
    const int nv[3] = {P.nvx, P.nvy, P.nvz};
    const int pz = P.nvz | 1;
    const int n = nv[d];
    const int npen = (P.nvx * P.nvy * P.nvz) / n;
    for (int pen = threadIdx.x; pen < npen; pen += blockDim.x) {
        int base, stride;
        double acc;
        if (d == 0) {           // pencil (iy, iz)
            const int iy = pen / P.nvz, iz = pen % P.nvz;
            base = iy * pz + iz;
            stride = P.nvy * pz;
            const double vy = P.lo[1] + (iy + 0.5) * P.dv[1], vz = P.lo[2] + (iz + 0.5) * P.dv[2];
            acc = EB[0] + vy * EB[5] - vz * EB[4];
        } else if (d == 1) {    // pencil (ix, iz)
            const int ix = pen / P.nvz, iz = pen % P.nvz;
            base = ix * P.nvy * pz + iz;
            stride = pz;
            const double vx = P.lo[0] + (ix + 0.5) * P.dv[0], vz = P.lo[2] + (iz + 0.5) * P.dv[2];
            acc = EB[1] + vz * EB[3] - vx * EB[5];
        } else {                // pencil (ix, iy)
            const int ix = pen / P.nvy, iy = pen % P.nvy;
            base = (ix * P.nvy + iy) * pz;
            stride = 1;
            const double vx = P.lo[0] + (ix + 0.5) * P.dv[0], vy = P.lo[1] + (iy + 0.5) * P.dv[1];
            acc = EB[2] + vx * EB[4] - vy * EB[3];
        }
        const double s = P.qm * acc * sigma / P.dv[d];
        const bool pos = s >= 0.0;
        const Shift<T> sh(fabs(s));
        // pencil in upwind-to-downwind order; element k at shared index
        const int first = pos ? base : base + (n - 1) * stride;
        const int step = pos ? stride : -stride;
        T g[NMAX + 2];
        g[0] = T(0);
        g[NMAX + 1] = T(0);
#pragma unroll
        for (int k = 0; k < NMAX; ++k) g[k + 1] = (k < n) ? blk[first + k * step] : T(0);
        // h_k = g_k + phi(k-1) - phi(k), k = 0..n; phi of ghost cells is 0
        T h[NMAX + 1];
        T pm = T(0);
#pragma unroll
        for (int k = 0; k < NMAX; ++k) {
            const T p0 = (k < n) ? pfc_phi(g[k], g[k + 1], g[k + 2], sh.a, sh.c1, sh.c2, finf) : T(0);
            h[k] = g[k + 1] + pm - p0;
            if (k == n - 1) h[NMAX] = p0;          // outflow into the ghost beyond the wall
            pm = (k < n) ? p0 : pm;
        }
        const long long K = sh.K;
        T top = h[NMAX];
#pragma unroll
        for (int k = 0; k < NMAX; ++k) {
            if (k < n) {
                const long long t = (long long)k + K;
                if (t >= n - 1) top += h[k];
                else blk[first + (int)t * step] = fmax(h[k], T(0));
                if ((long long)k < K && k < n - 1) blk[first + k * step] = T(0);
            }
        }
        blk[first + (n - 1) * step] = fmax(top, T(0));
    }
}

template <class T, int NMAX>
__global__ void __launch_bounds__(256)
pfc_v3_kernel(const T* fin, T* fout, const double* __restrict__ E, const double* __restrict__ B,
              V3Params P, const T* __restrict__ finf_p, typename Bits<T>::U* __restrict__ max_out) {
    extern __shared__ unsigned char smem_raw[];
    T* blk = reinterpret_cast<T*>(smem_raw);
    __shared__ double EB[6];
    const long long cell = blockIdx.x;
    const int nv = P.nvx * P.nvy * P.nvz;
    const int pz = P.nvz | 1;
    const T finf = *finf_p;
    if (threadIdx.x < 3) {
        EB[threadIdx.x] = E[cell * 3 + threadIdx.x];
        EB[3 + threadIdx.x] = B ? B[cell * 3 + threadIdx.x] : 0.0;
    }
    const T* src = fin + cell * nv;
    for (int e = threadIdx.x; e < nv; e += blockDim.x) {
        const int iz = e % P.nvz, r = e / P.nvz;
        blk[r * pz + iz] = src[e];
    }
    __syncthreads();
    double ebl[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) ebl[k] = EB[k];
    const double half = 0.5 * P.tau;
    sweep3<T, NMAX>(blk, 0, half, P, ebl, finf);
    __syncthreads();
    sweep3<T, NMAX>(blk, 1, half, P, ebl, finf);
    __syncthreads();
    sweep3<T, NMAX>(blk, 2, P.tau, P, ebl, finf);
    __syncthreads();
    sweep3<T, NMAX>(blk, 1, half, P, ebl, finf);
    __syncthreads();
    sweep3<T, NMAX>(blk, 0, half, P, ebl, finf);
    __syncthreads();
    T* dst = fout + cell * nv;
    T mx = T(0);
    for (int e = threadIdx.x; e < nv; e += blockDim.x) {
        const int iz = e % P.nvz, r = e / P.nvz;
        const T o = blk[r * pz + iz];
        dst[e] = o;
        mx = fmax(mx, o);
    }
    if (max_out) block_max_to(mx, max_out);
}

// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256)
array_max_kernel(const T* __restrict__ f, long long n, typename Bits<T>::U* __restrict__ out) {
    T mx = T(0);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        mx = fmax(mx, f[i]);
    block_max_to(mx, out);
}

__global__ void fill_u64_kernel(unsigned long long* p, int n, unsigned long long v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------ launchers ----
constexpr int kChunkX = 16;
constexpr int kChunkY = 16;

template <class T>
hipError_t launch_pfc_x(const T* fin, T* fout, int rows, int nx, long long Nv, int inner, double vx_lo,
                        double dvx, double tau_dx, const void* finf, void* max_out, hipStream_t st) {
    dim3 grid((unsigned)((Nv + 255) / 256), (unsigned)((nx + kChunkX - 1) / kChunkX), (unsigned)rows);
    hipLaunchKernelGGL((pfc_x_kernel<T, kChunkX>), grid, dim3(256), 0, st, fin, fout, nx, Nv, inner, vx_lo,
                       dvx, tau_dx, (const T*)finf, (typename Bits<T>::U*)max_out);
    return hipGetLastError();
}

template <class T>
hipError_t launch_pfc_y(const T* fin, T* fout, int nx, int ny, int nvx, int nvy, int nvz, double vy_lo,
                        double dvy, double tau_dy, const void* finf, void* max_out, hipStream_t st) {
    const long long Nv = (long long)nvx * nvy * nvz;
    const long long npairs = (long long)nvx * ((nvy + 1) / 2) * nvz;
    dim3 grid((unsigned)((npairs + 255) / 256), (unsigned)((2 * ny + kChunkY - 1) / kChunkY), (unsigned)nx);
    hipLaunchKernelGGL((pfc_y_kernel<T, kChunkY>), grid, dim3(256), 0, st, fin, fout, nx, ny, Nv, nvx, nvy,
                       nvz, vy_lo, dvy, tau_dy, (const T*)finf, (typename Bits<T>::U*)max_out);
    return hipGetLastError();
}

template <class T>
hipError_t launch_pfc_v1(const T* fin, T* fout, int nx, int nv, const double* E, double qm_tau_dv,
                         const void* finf, void* max_out, hipStream_t st) {
    const int threads = nv >= 256 ? 256 : ((nv + 63) / 64) * 64;
    const size_t shm = sizeof(T) * (size_t)(nv + 4);
    hipLaunchKernelGGL((pfc_v1_kernel<T>), dim3(nx), dim3(threads), shm, st, fin, fout, nv, E, qm_tau_dv,
                       (const T*)finf, (typename Bits<T>::U*)max_out);
    return hipGetLastError();
}

size_t v3_shared_bytes(int nvx, int nvy, int nvz, size_t elem) {
    return elem * (size_t)nvx * nvy * (nvz | 1);
}

template <class T>
hipError_t launch_pfc_v3(const T* fin, T* fout, long long cells, const double* E, const double* B,
                         const V3Params& P, const void* finf, void* max_out, hipStream_t st) {
    const int nmax = P.nvx > P.nvy ? (P.nvx > P.nvz ? P.nvx : P.nvz) : (P.nvy > P.nvz ? P.nvy : P.nvz);
    const size_t shm = v3_shared_bytes(P.nvx, P.nvy, P.nvz, sizeof(T));
    int maxpen = P.nvx * P.nvy;
    if (P.nvx * P.nvz > maxpen) maxpen = P.nvx * P.nvz;
    if (P.nvy * P.nvz > maxpen) maxpen = P.nvy * P.nvz;
    int threads = ((maxpen + 63) / 64) * 64;
    if (threads > 256) threads = 256;
    if (threads < 64) threads = 64;
    if (nmax <= 8) {
        hipLaunchKernelGGL((pfc_v3_kernel<T, 8>), dim3((unsigned)cells), dim3(threads), shm, st, fin, fout, E, B,
                           P, (const T*)finf, (typename Bits<T>::U*)max_out);
    } else if (nmax <= 16) {
        hipLaunchKernelGGL((pfc_v3_kernel<T, 16>), dim3((unsigned)cells), dim3(threads), shm, st, fin, fout, E,
                           B, P, (const T*)finf, (typename Bits<T>::U*)max_out);
    } else if (nmax <= 32) {
        hipLaunchKernelGGL((pfc_v3_kernel<T, 32>), dim3((unsigned)cells), dim3(threads), shm, st, fin, fout, E,
                           B, P, (const T*)finf, (typename Bits<T>::U*)max_out);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class T>
hipError_t launch_array_max(const T* f, long long n, void* out, hipStream_t st) {
    hipLaunchKernelGGL(fill_u64_kernel, dim3(1), dim3(64), 0, st, (unsigned long long*)out, 1, 0ull);
    long long blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((array_max_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, st, f, n,
                       (typename Bits<T>::U*)out);
    return hipGetLastError();
}

hipError_t launch_fill_u64(void* p, int n, unsigned long long v, hipStream_t st) {
    hipLaunchKernelGGL(fill_u64_kernel, dim3((n + 63) / 64), dim3(64), 0, st, (unsigned long long*)p, n, v);
    return hipGetLastError();
}

#define VL_INST(T)                                                                                         \
    template hipError_t launch_pfc_x<T>(const T*, T*, int, int, long long, int, double, double, double,     \
                                        const void*, void*, hipStream_t);                                  \
    template hipError_t launch_pfc_y<T>(const T*, T*, int, int, int, int, int, double, double, double,      \
                                        const void*, void*, hipStream_t);                                  \
    template hipError_t launch_pfc_v1<T>(const T*, T*, int, int, const double*, double, const void*, void*, \
                                         hipStream_t);                                                     \
    template hipError_t launch_pfc_v3<T>(const T*, T*, long long, const double*, const double*,             \
                                         const V3Params&, const void*, void*, hipStream_t);                \
    template hipError_t launch_array_max<T>(const T*, long long, void*, hipStream_t);
VL_INST(float)
VL_INST(double)
#undef VL_INST

}  // namespace vl
