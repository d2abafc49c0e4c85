// Velocity moments and moment fitting for gfx950.
//
// Moments (Sec. 2.1 of arXiv 2109.06743, definitions after Eq. 1), midpoint
// rule on the velocity cell centres, accumulated in FP64 whatever the storage
// type of f.  3V sums are separable: each thread forms the four row sums
// sum_z f v_z^k (k = 0..3) of one (v_x, v_y) row, then the row's share of the
// 20 raw moments needs 20 FP64 operations per row instead of per cell.
//
// Moment fitting (Algorithm 1, "Moment Fitting"; Sec. 2.2): per cell
//   f' = f - M[n_V, u_V, T_V] + M[n_V, u_F, T_F],  f'' = max(f', 0),
//   f_new = f'' n_V / (sum f'' dV),
// M the ten-moment Maxwellian n g / (sum g dV), g = exp(-(m/2) w^T T^-1 w),
// w = v - u.  Exponentials and f in the storage type; quadratic-form
// coefficients, normalisation sums, the rescale factor and all moments FP64.
#include "vl_internal.h"

namespace vl {

struct VGrid {
    int nvx, nvy, nvz;
    double lo[3], dv[3];
    double m;
    float inv_nvz;
};

__device__ __forceinline__ double vc(const VGrid& G, int d, int i) { return G.lo[d] + (i + 0.5) * G.dv[d]; }

// 20 raw moments (already multiplied by dV, and by m for P and Q) of a block
// held in shared memory with rows of length nvz at stride pz.  Result in
// mom[] of every thread.  red: shared scratch of 20 * (blockDim/64) doubles.
template <class T>
__device__ void block_moments3(const T* blk, int pz, const VGrid& G, double (&mom)[20], double* red) {
    double acc[20];
#pragma unroll
    for (int k = 0; k < 20; ++k) acc[k] = 0.0;
    const int rows = G.nvx * G.nvy;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
        const int ix = r / G.nvy, iy = r % G.nvy;
        const T* row = blk + r * pz;
        double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        for (int iz = 0; iz < G.nvz; ++iz) {
            const double f = (double)row[iz];
            const double z = vc(G, 2, iz);
            const double fz = f * z;
            s0 += f;
            s1 += fz;
            s2 += fz * z;
            s3 += fz * z * z;
        }
        const double X = vc(G, 0, ix), Y = vc(G, 1, iy);
        const double X2 = X * X, Y2 = Y * Y, XY = X * Y;
        acc[0] += s0;
        acc[1] += X * s0;
        acc[2] += Y * s0;
        acc[3] += s1;
        acc[4] += X2 * s0;      // xx
        acc[5] += XY * s0;      // xy
        acc[6] += X * s1;       // xz
        acc[7] += Y2 * s0;      // yy
        acc[8] += Y * s1;       // yz
        acc[9] += s2;           // zz
        acc[10] += X2 * X * s0; // xxx
        acc[11] += X2 * Y * s0; // xxy
        acc[12] += X2 * s1;     // xxz
        acc[13] += X * Y2 * s0; // xyy
        acc[14] += XY * s1;     // xyz
        acc[15] += X * s2;      // xzz
        acc[16] += Y2 * Y * s0; // yyy
        acc[17] += Y2 * s1;     // yyz
        acc[18] += Y * s2;      // yzz
        acc[19] += s3;          // zzz
    }
    block_sum<20>(acc, red);
    const double dV = G.dv[0] * G.dv[1] * G.dv[2];
#pragma unroll
    for (int k = 0; k < 20; ++k) mom[k] = acc[k] * (k < 4 ? dV : G.m * dV);
}

template <class T>
__global__ void __launch_bounds__(256) moments3_kernel(const T* __restrict__ f, double* __restrict__ mom, VGrid G) {
    extern __shared__ unsigned char smem_raw[];
    T* blk = reinterpret_cast<T*>(smem_raw);
    __shared__ double red[20 * 4];
    const long long cell = blockIdx.x;
    const int nv = G.nvx * G.nvy * G.nvz;
    const int pz = G.nvz | 1;
    const T* src = f + cell * nv;
    for (int e = threadIdx.x; e < nv; e += blockDim.x) blk[e + row_of(e, G.inv_nvz) * (pz - G.nvz)] = src[e];
    __syncthreads();
    double m[20];
    block_moments3(blk, pz, G, m, red);
    if (threadIdx.x < 20) {
        double v = 0;
#pragma unroll
        for (int k = 0; k < 20; ++k) v = (threadIdx.x == k) ? m[k] : v;
        mom[cell * 20 + threadIdx.x] = v;
    }
}

template <class T>
__global__ void __launch_bounds__(256) moments1_kernel(const T* __restrict__ f, double* __restrict__ mom, int nv,
                                                       double vlo, double dv, double mass) {
    __shared__ double red[4 * 4];
    const long long cell = blockIdx.x;
    const T* src = f + cell * nv;
    double acc[4] = {0, 0, 0, 0};
    for (int j = threadIdx.x; j < nv; j += blockDim.x) {
        const double v = vlo + (j + 0.5) * dv;
        const double x = (double)src[j];
        const double xv = x * v;
        acc[0] += x;
        acc[1] += xv;
        acc[2] += xv * v;
        acc[3] += xv * v * v;
    }
    block_sum<4>(acc, red);
    if (threadIdx.x == 0) {
        mom[cell * 4 + 0] = acc[0] * dv;
        mom[cell * 4 + 1] = acc[1] * dv;
        mom[cell * 4 + 2] = mass * acc[2] * dv;
        mom[cell * 4 + 3] = mass * acc[3] * dv;
    }
}

// ------------------------------------------------------------------ fit ----
// Symmetric 3x3 stored as (xx, xy, xz, yy, yz, zz).  Returns false unless the
// matrix is positive definite (Cholesky pivots > 0); inv receives its inverse.
__device__ __forceinline__ bool spd_inverse(const double (&a)[6], double (&inv)[6]) {
    const double l11sq = a[0];
    if (!(l11sq > 0.0)) return false;
    const double l11 = sqrt(l11sq);
    const double l21 = a[1] / l11, l31 = a[2] / l11;
    const double l22sq = a[3] - l21 * l21;
    if (!(l22sq > 0.0)) return false;
    const double l22 = sqrt(l22sq);
    const double l32 = (a[4] - l31 * l21) / l22;
    const double l33sq = a[5] - l31 * l31 - l32 * l32;
    if (!(l33sq > 0.0)) return false;
    // inverse via cofactors (the matrix is SPD, so det > 0)
    const double c00 = a[3] * a[5] - a[4] * a[4];
    const double c01 = a[2] * a[4] - a[1] * a[5];
    const double c02 = a[1] * a[4] - a[2] * a[3];
    const double c11 = a[0] * a[5] - a[2] * a[2];
    const double c12 = a[1] * a[2] - a[0] * a[4];
    const double c22 = a[0] * a[3] - a[1] * a[1];
    const double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
    const double id = 1.0 / det;
    inv[0] = c00 * id; inv[1] = c01 * id; inv[2] = c02 * id;
    inv[3] = c11 * id; inv[4] = c12 * id; inv[5] = c22 * id;
    return true;
}

// Mean velocity and temperature tensor from (n, nu, P) with T = (P - m n u u)/n.
__device__ __forceinline__ void u_and_T(const double* nuP, double n, double m, double (&u)[3], double (&T)[6]) {
    u[0] = nuP[0] / n; u[1] = nuP[1] / n; u[2] = nuP[2] / n;
    const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 0; k < 6; ++k) T[k] = (nuP[3 + k] - m * n * u[ia[k]] * u[ib[k]]) / n;
}

template <class T>
__device__ __forceinline__ T expo(T x);
template <> __device__ __forceinline__ float expo<float>(float x) { return __expf(x); }
template <> __device__ __forceinline__ double expo<double>(double x) { return exp(x); }

// Exponent -(m/2) w^T Tinv w with coefficients A = (m/2) Tinv (off-diagonals doubled).
template <class T>
struct Quad {
    T axx, axy, axz, ayy, ayz, azz;
    T ux, uy, uz;
    __device__ __forceinline__ void set(const double (&inv)[6], const double (&u)[3], double m) {
        const double h = 0.5 * m;
        axx = (T)(h * inv[0]); axy = (T)(2.0 * h * inv[1]); axz = (T)(2.0 * h * inv[2]);
        ayy = (T)(h * inv[3]); ayz = (T)(2.0 * h * inv[4]); azz = (T)(h * inv[5]);
        ux = (T)u[0]; uy = (T)u[1]; uz = (T)u[2];
    }
    __device__ __forceinline__ T g(T vx, T vy, T vz) const {
        const T wx = vx - ux, wy = vy - uy, wz = vz - uz;
        const T q = wx * (axx * wx + axy * wy + axz * wz) + wy * (ayy * wy + ayz * wz) + azz * wz * wz;
        return expo<T>(-q);
    }
};

// Per-cell fit.  One block per spatial cell; the block's f values sit in
// registers (EPT per thread, element e = tid + k * blockDim), the clipped f''
// is staged in shared memory for the separable moment sums.
template <class T, int EPT>
__global__ void __launch_bounds__(256)
fit3_kernel(const T* fin, T* fout, const double* __restrict__ mom_pre, double* __restrict__ U,
            double* __restrict__ mom_post, unsigned long long* __restrict__ counters, VGrid G,
            typename Bits<T>::U* __restrict__ max_out) {
    extern __shared__ unsigned char smem_raw[];
    T* blk = reinterpret_cast<T*>(smem_raw);
    __shared__ double red[21 * 4];
    const long long cell = blockIdx.x;
    const int nv = G.nvx * G.nvy * G.nvz;
    const int pz = G.nvz | 1;
    const double dV = G.dv[0] * G.dv[1] * G.dv[2];
    const T* src = fin + cell * nv;
    T* dst = fout + cell * nv;

    T fv[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int e = threadIdx.x + k * blockDim.x;
        fv[k] = (e < nv) ? src[e] : T(0);
    }

    // cell parameters (every thread computes the same values)
    double mp[10], Uc[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) { mp[k] = mom_pre[cell * 20 + k]; Uc[k] = U[cell * 10 + k]; }
    const double nV = mp[0], nF = Uc[0];
    double uV[3], TV[6], uF[3], TF[6], iV[6], iF[6];
    bool ok = nV > 1e-12 && nF > 1e-12;
    if (ok) {
        u_and_T(mp + 1, nV, G.m, uV, TV);
        u_and_T(Uc + 1, nF, G.m, uF, TF);
        ok = spd_inverse(TV, iV) && spd_inverse(TF, iF);
    }

    T outv[EPT];
    unsigned long long nclip = 0;
    if (ok) {
        Quad<T> qv, qf;
        qv.set(iV, uV, G.m);
        qf.set(iF, uF, G.m);
        T gv[EPT], gf[EPT];
        double sums[2] = {0.0, 0.0};
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int e = threadIdx.x + k * blockDim.x;
            gv[k] = T(0);
            gf[k] = T(0);
            if (e < nv) {
                const int iz = e % G.nvz, r = e / G.nvz;
                const T vx = (T)vc(G, 0, r / G.nvy), vy = (T)vc(G, 1, r % G.nvy), vz = (T)vc(G, 2, iz);
                gv[k] = qv.g(vx, vy, vz);
                gf[k] = qf.g(vx, vy, vz);
                sums[0] += (double)gv[k];
                sums[1] += (double)gf[k];
            }
        }
        block_sum<2>(sums, red);
        const T A = (T)(nV / (sums[0] * dV));
        const T Bc = (T)(nV / (sums[1] * dV));
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int e = threadIdx.x + k * blockDim.x;
            const T x = fv[k] - A * gv[k] + Bc * gf[k];
            if (e < nv && x < T(0)) ++nclip;
            outv[k] = fmax(x, T(0));
            if (e < nv) blk[(e / G.nvz) * pz + e % G.nvz] = outv[k];
        }
    } else {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int e = threadIdx.x + k * blockDim.x;
            outv[k] = fv[k];
            if (e < nv) blk[(e / G.nvz) * pz + e % G.nvz] = fv[k];
        }
    }
    __syncthreads();
    double mm[20];
    block_moments3(blk, pz, G, mm, red);
    const double scale = ok ? nV / mm[0] : 1.0;
    const T sc = (T)scale;
    T mx = T(0);
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int e = threadIdx.x + k * blockDim.x;
        if (e < nv) {
            const T o = ok ? outv[k] * sc : outv[k];
            dst[e] = o;
            mx = fmax(mx, o);
        }
    }
    if (threadIdx.x < 20 && mom_post) {
        double v = 0;
#pragma unroll
        for (int k = 0; k < 20; ++k) v = (threadIdx.x == k) ? mm[k] : v;
        mom_post[cell * 20 + threadIdx.x] = v * scale;
    }
    if (ok && threadIdx.x < 10) {
        const double r = nV / nF;
        double v = 0;
#pragma unroll
        for (int k = 0; k < 10; ++k) v = (threadIdx.x == k) ? Uc[k] : v;
        U[cell * 10 + threadIdx.x] = v * r;
    }
    if (counters) {
        double c[1] = {(double)nclip};
        block_sum<1>(c, red);
        if (threadIdx.x == 0) {
            if (c[0] > 0) atomicAdd(&counters[0], (unsigned long long)c[0]);
            if (!ok) atomicAdd(&counters[1], 1ull);
        }
    }
    if (max_out) block_max_part(mx, max_out);
}

// ------------------------------------------------------- cubic blocks -------
// Velocity blocks with N cells per axis: thread t < N*N owns the v_x pencil at
// (v_y, v_z) = (t / N, t % N); element (ix, t) sits at t + N*N*ix, so the loads
// of a wave are contiguous and the only coordinate that varies along a thread's
// elements is v_x, which is uniform across the block (table in the arguments).
struct XTable {
    double v[kBigCube], v2[kBigCube], v3[kBigCube];
};

// The 20 raw moments as weighted sums of the pencil sums S_k = sum_x f v_x^k
// with the thread's transverse velocities (v_y, v_z).
__device__ __forceinline__ void pencil_moments(const double (&S)[4], double vy, double vz, double (&a)[20]) {
    const double vy2 = vy * vy, vz2 = vz * vz, vyz = vy * vz;
    a[0] = S[0];        a[1] = S[1];        a[2] = vy * S[0];   a[3] = vz * S[0];
    a[4] = S[2];        a[5] = vy * S[1];   a[6] = vz * S[1];
    a[7] = vy2 * S[0];  a[8] = vyz * S[0];  a[9] = vz2 * S[0];
    a[10] = S[3];       a[11] = vy * S[2];  a[12] = vz * S[2];  a[13] = vy2 * S[1];
    a[14] = vyz * S[1]; a[15] = vz2 * S[1]; a[16] = vy2 * vy * S[0];
    a[17] = vy2 * vz * S[0]; a[18] = vy * vz2 * S[0]; a[19] = vz2 * vz * S[0];
}

// One wave per cell (four cells per 256-thread block): lane l owns the v_x
// pencils at transverse positions t = l + 64 j (t = iy * N + iz), so the 20
// sums are reduced inside one wave, with no block barrier.
template <class T, int N>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
moments3_cube_kernel(const T* __restrict__ f, double* __restrict__ mom, long long cells, VGrid G, XTable X) {
    constexpr int NT = (N * N + 63) / 64;
    const int lane = threadIdx.x & 63;
    const long long cell = (long long)xcd_work_index(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (cell >= cells) return;
    const T* src = f + cell * (N * N * N);
    T fv[NT][N];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int t = lane + 64 * j;
#pragma unroll
        for (int k = 0; k < N; ++k) fv[j][k] = (t < N * N) ? ld_f<kRowsWholeLines<T, N>>(src + t + k * N * N) : T(0);
    }
    double acc[20];
#pragma unroll
    for (int q = 0; q < 20; ++q) acc[q] = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int t = lane + 64 * j;
        double S[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double g = (double)fv[j][k];
            S[0] += g;
            S[1] = fma(g, X.v[k], S[1]);
            S[2] = fma(g, X.v2[k], S[2]);
            S[3] = fma(g, X.v3[k], S[3]);
        }
        double a[20];
        pencil_moments(S, vc(G, 1, t / N), vc(G, 2, t % N), a);
#pragma unroll
        for (int q = 0; q < 20; ++q) acc[q] += a[q];
    }
    int idx = 0, cnt = 20;
    const double v = ReduceScatter<20, 32>::run(acc, lane, idx, cnt);
    const double dV = G.dv[0] * G.dv[1] * G.dv[2];
    if ((lane & 1) == 0 && cnt > 0) mom[cell * 20 + idx] = v * (idx < 4 ? dV : G.m * dV);
}

// The same sums for FP32 blocks whose v_x planes are not whole cache lines
// (12^3: 576 B).  A cell is 6912 B, 54 whole lines: each wave reads its cell
// with 16-byte non-temporal loads (every wave instruction one 1 KB run of
// whole lines) into shared memory, then lane l takes its pencils from there
// as in moments3_cube_kernel (same arithmetic, same order).  The 27 KB of
// shared memory per workgroup allow five workgroups per CU, so the registers
// are capped for five waves per SIMD (96).  On the magnetotail grid: 869 ->
// 717 us per launch.
template <int N>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5)))
moments3_staged_kernel(const float* __restrict__ f, double* __restrict__ mom, long long cells, VGrid G, XTable X) {
    typedef float F4 __attribute__((ext_vector_type(4)));
    constexpr int NV = N * N * N;
    constexpr int NT = (N * N + 63) / 64;
    constexpr int NQ = NV / 4;                    // 16-byte pieces of a cell
    static_assert(NV % 4 == 0 && (NV * 4) % 128 == 0, "cells of whole lines");
    __shared__ F4 buf[4][NQ];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const long long cell = (long long)xcd_work_index(blockIdx.x, gridDim.x) * 4 + w;
    if (cell >= cells) return;
    const F4* src = reinterpret_cast<const F4*>(f + cell * NV);
#pragma unroll
    for (int i = 0; i < (NQ + 63) / 64; ++i) {
        const int q = lane + 64 * i;
        if (q < NQ) buf[w][q] = __builtin_nontemporal_load(src + q);
    }
    // the wave reads back what its own lanes wrote: order its shared-memory
    // accesses (no other wave touches buf[w])
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const float* cb = reinterpret_cast<const float*>(buf[w]);
    double acc[20];
#pragma unroll
    for (int q = 0; q < 20; ++q) acc[q] = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int t = lane + 64 * j;
        double S[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double g = (double)((t < N * N) ? cb[t + k * N * N] : 0.0f);
            S[0] += g;
            S[1] = fma(g, X.v[k], S[1]);
            S[2] = fma(g, X.v2[k], S[2]);
            S[3] = fma(g, X.v3[k], S[3]);
        }
        double a[20];
        pencil_moments(S, vc(G, 1, t / N), vc(G, 2, t % N), a);
#pragma unroll
        for (int q = 0; q < 20; ++q) acc[q] += a[q];
    }
    int idx = 0, cnt = 20;
    const double v = ReduceScatter<20, 32>::run(acc, lane, idx, cnt);
    const double dV = G.dv[0] * G.dv[1] * G.dv[2];
    if ((lane & 1) == 0 && cnt > 0) mom[cell * 20 + idx] = v * (idx < 4 ? dV : G.m * dV);
}

// Large cubic blocks (a cell's pencils do not fit one wave's registers): one
// block per cell; thread t sums the v_x pencils at transverse positions
// t, t + NTH, ... one pencil at a time, then a block reduction of the 20 sums.
// A 34^3 v_x plane is not a whole number of lines (4624 B in FP32), so the
// loads are ordinary and the caches merge the lines two wave accesses share
// (938 -> 839 us per 256x128x34^3 FP32 launch against non-temporal loads).
template <class T, int N, int NTH>
__global__ void __launch_bounds__(NTH)
moments3_big_kernel(const T* __restrict__ f, double* __restrict__ mom, VGrid G, XTable X) {
    __shared__ double red[(NTH / 64) * 20];
    __shared__ double fin_s[20];
    const long long cell = xcd_work_index(blockIdx.x, gridDim.x);
    const T* src = f + cell * (N * N * N);
    double acc[20];
#pragma unroll
    for (int q = 0; q < 20; ++q) acc[q] = 0.0;
    for (int t = threadIdx.x; t < N * N; t += NTH) {
        T fv[N];
#pragma unroll
        for (int k = 0; k < N; ++k) fv[k] = ld_f<kRowsWholeLines<T, N>>(src + t + k * N * N);
        double Se[4] = {0.0, 0.0, 0.0, 0.0}, So[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double g = (double)fv[k];
            double* S = (k & 1) ? So : Se;
            S[0] += g;
            S[1] = fma(g, X.v[k], S[1]);
            S[2] = fma(g, X.v2[k], S[2]);
            S[3] = fma(g, X.v3[k], S[3]);
        }
        const double S[4] = {Se[0] + So[0], Se[1] + So[1], Se[2] + So[2], Se[3] + So[3]};
        double a[20];
        pencil_moments(S, vc(G, 1, t / N), vc(G, 2, t % N), a);
#pragma unroll
        for (int q = 0; q < 20; ++q) acc[q] += a[q];
    }
    block_sum_rs<20>(acc, red, fin_s);
    const double dV = G.dv[0] * G.dv[1] * G.dv[2];
    if (threadIdx.x < 20) mom[cell * 20 + threadIdx.x] = fin_s[threadIdx.x] * (threadIdx.x < 4 ? dV : G.m * dV);
}

// Moment fitting of one cubic cell per block (see fit3_kernel for the steps).
// Per element: two exponentials of a quadratic in v_x whose other terms are
// per-thread constants, the exchange and clip, and FP64 pencil sums.
// exp(-q) with q scaled by log2(e) in FP32 (one v_exp_f32), exp() in FP64.
template <class T> struct ExpK;
template <> struct ExpK<float> {
    static constexpr double scale = 1.4426950408889634;   // log2(e)
    static __device__ __forceinline__ float e(float q) { return __builtin_amdgcn_exp2f(-q); }
};
template <> struct ExpK<double> {
    static constexpr double scale = 1.0;
    static __device__ __forceinline__ double e(double q) { return exp(-q); }
};

template <class T>
struct QuadX {       // (m/2) w^T T^-1 w = axx wx^2 + bt wx + ct for fixed (wy, wz), times ExpK::scale
    T axx, bt, ct, ux;
    // a: (m/2) ExpK::scale T^-1 as (xx, xy, xz, yy, yz, zz); u: mean velocity
    __device__ __forceinline__ void set(const double* a, const double* u, double vy, double vz) {
        const double wy = vy - u[1], wz = vz - u[2];
        axx = (T)a[0];
        bt = (T)(2.0 * (a[1] * wy + a[2] * wz));
        ct = (T)(a[3] * wy * wy + 2.0 * a[4] * wy * wz + a[5] * wz * wz);
        ux = (T)u[0];
    }
    __device__ __forceinline__ T g(T vx) const {
        const T wx = vx - ux;
        return ExpK<T>::e(fma(fma(axx, wx, bt), wx, ct));
    }
};

// Per-cell set-up of the fitting (one thread per cell), so that the f pass
// carries no FP64 divisions, square roots or branches on the moments: the
// exponent coefficients of the two Maxwellians, the density n_V, the skip
// decision; the fluid state is rescaled by n_V/n_F in place.
struct FitCell {
    double aV[6], uV[3], aF[6], uF[3];
    double nV, ok;
};
static_assert(sizeof(FitCell) == kFitCellDoubles * sizeof(double), "FitCell layout");

__global__ void __launch_bounds__(256)
fit3_params_kernel(const double* __restrict__ mom_pre, double* __restrict__ U, long long cells, double m,
                   double kscale, FitCell* __restrict__ out, unsigned long long* __restrict__ counters) {
    __shared__ int nskip;
    if (threadIdx.x == 0) nskip = 0;
    __syncthreads();
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < cells) {
        double mp[10], Uc[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) { mp[k] = mom_pre[c * 20 + k]; Uc[k] = U[c * 10 + k]; }
        const double nV = mp[0], nF = Uc[0];
        double uV[3] = {0, 0, 0}, TV[6], uF[3] = {0, 0, 0}, TF[6], iV[6] = {0, 0, 0, 0, 0, 0}, iF[6] = {0, 0, 0, 0, 0, 0};
        bool ok = nV > 1e-12 && nF > 1e-12;
        if (ok) {
            u_and_T(mp + 1, nV, m, uV, TV);
            u_and_T(Uc + 1, nF, m, uF, TF);
            ok = spd_inverse(TV, iV) && spd_inverse(TF, iF);
        }
        FitCell r;
        const double h = 0.5 * m * kscale;
#pragma unroll
        for (int k = 0; k < 6; ++k) { r.aV[k] = h * iV[k]; r.aF[k] = h * iF[k]; }
#pragma unroll
        for (int k = 0; k < 3; ++k) { r.uV[k] = uV[k]; r.uF[k] = uF[k]; }
        r.nV = nV;
        r.ok = ok ? 1.0 : 0.0;
        out[c] = r;
        if (ok) {
            const double sc = nV / nF;
#pragma unroll
            for (int k = 0; k < 10; ++k) U[c * 10 + k] = Uc[k] * sc;
        } else {
            atomicAdd(&nskip, 1);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && counters && nskip) atomicAdd(&counters[1], (unsigned long long)nskip);
}

// One block of NW waves per cell; thread t owns the v_x pencils at transverse
// positions t + 64 NW j (j < NT).  Two passes over f held in registers: the
// normalisation sums of the two Maxwellians (exponentials and pencil sums in
// the storage type, FP64 across pencils), then the exchange, clip (counted
// per wave with a ballot), FP64 post-fit moments and the FP64 rescale.  The
// block sums use the reduce-scatter (block_sum_rs).
// Launch shapes: 16^3 two waves of two pencils per thread, 12^3 one wave of
// three pencils per lane.
constexpr int kFit16Waves = 2, kFit16Pencils = 2;
constexpr int kFit12Waves = 1, kFit12Pencils = 3;
template <class T, int N, int NW, int NT>
__global__ void __launch_bounds__(64 * NW)
fit3_cube_kernel(const T* fin, T* fout, const FitCell* __restrict__ P, double* __restrict__ mom_post,
                 unsigned* __restrict__ clip_part, VGrid G, XTable X, typename Bits<T>::U* __restrict__ max_out) {
    constexpr int NTH = 64 * NW;
    // every thread owns NT whole pencils (no idle positions to mask)
    constexpr bool kFull = NT * NTH == N * N;
    // keeping the pass-1 exponentials in registers pays while they fit
    constexpr bool kKeep = NT * N <= 48;
    __shared__ double red[NW * 21];
    __shared__ double fin_s[21];
    const int tid = threadIdx.x;
    const long long cell = xcd_work_index(blockIdx.x, gridDim.x);
    const double dV = G.dv[0] * G.dv[1] * G.dv[2];
    const T* src = fin + cell * (N * N * N);
    T* dst = fout + cell * (N * N * N);
    T fv[NT][N];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int t = tid + NTH * j;
#pragma unroll
        for (int k = 0; k < N; ++k)
            fv[j][k] = (kFull || t < N * N) ? __builtin_nontemporal_load(src + t + k * N * N) : T(0);
    }
    // v_x in the storage type: held in registers for the small blocks,
    // converted at each use for the large ones (register pressure)
    constexpr bool kVx = N <= 16;
    T vxr[kVx ? N : 1];
#pragma unroll
    for (int k = 0; k < (kVx ? N : 1); ++k) vxr[k] = (T)X.v[k];
    auto vx = [&](int k) -> T { return kVx ? vxr[k] : (T)X.v[k]; };
    const FitCell& C = P[cell];
    const bool ok = C.ok != 0.0;
    const double nV = C.nV;
    unsigned nclip = 0;     // clipped elements of this wave (the same in every lane)
    if (ok) {
        QuadX<T> qv[NT], qf[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int t = tid + NTH * j;
            const double vy = vc(G, 1, t / N), vz = vc(G, 2, t % N);
            qv[j].set(C.aV, C.uV, vy, vz);
            qf[j].set(C.aF, C.uF, vy, vz);
        }
        // pencil sums of the samples in the storage type (four interleaved
        // chains; the samples carry that type's rounding already), added
        // across pencils in FP64
        double s[2] = {0.0, 0.0};
        T gv[kKeep ? NT : 1][kKeep ? N : 1], gf[kKeep ? NT : 1][kKeep ? N : 1];
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            if (kFull || tid + NTH * j < N * N) {
                T pa[4] = {T(0), T(0), T(0), T(0)}, pb[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    const T a = qv[j].g(vx(k)), b = qf[j].g(vx(k));
                    if constexpr (kKeep) {
                        gv[j][k] = a;
                        gf[j][k] = b;
                    }
                    pa[k & 3] += a;
                    pb[k & 3] += b;
                }
                s[0] += (double)((pa[0] + pa[1]) + (pa[2] + pa[3]));
                s[1] += (double)((pb[0] + pb[1]) + (pb[2] + pb[3]));
            }
        }
        block_sum_rs<2>(s, red, fin_s);
        const T A = (T)(nV / (fin_s[0] * dV));
        const T Bc = (T)(nV / (fin_s[1] * dV));
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const bool act = kFull || tid + NTH * j < N * N;
#pragma unroll
            for (int k = 0; k < N; ++k) {
                T x;
                if constexpr (kKeep) {
                    x = fv[j][k] - A * gv[j][k] + Bc * gf[j][k];
                } else {
                    x = fv[j][k] - A * qv[j].g(vx(k)) + Bc * qf[j].g(vx(k));
                }
                const bool neg = x < T(0);
                nclip += (unsigned)__builtin_popcountll(__builtin_amdgcn_ballot_w64(act && neg));
                fv[j][k] = act ? (neg ? T(0) : x) : T(0);
            }
        }
    }
    // raw moments of the clipped f'' (FP64 pencil sums)
    double acc[21];
#pragma unroll
    for (int q = 0; q < 20; ++q) acc[q] = 0.0;
    acc[20] = (tid & (kWave - 1)) == 0 ? (double)nclip : 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int t = tid + NTH * j;
        // pencil sums over even and odd v_x separately (two independent chains)
        double Se[4] = {0.0, 0.0, 0.0, 0.0}, So[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double g = (double)fv[j][k];
            double* S = (k & 1) ? So : Se;
            S[0] += g;
            S[1] = fma(g, X.v[k], S[1]);
            S[2] = fma(g, X.v2[k], S[2]);
            S[3] = fma(g, X.v3[k], S[3]);
        }
        const double S[4] = {Se[0] + So[0], Se[1] + So[1], Se[2] + So[2], Se[3] + So[3]};
        double a[20];
        pencil_moments(S, vc(G, 1, t / N), vc(G, 2, t % N), a);
#pragma unroll
        for (int q = 0; q < 20; ++q) acc[q] += a[q];
    }
    block_sum_rs<21>(acc, red, fin_s);
    const double scale = ok ? nV / (fin_s[0] * dV) : 1.0;
    const T sc = (T)scale;     // 1 exactly when the cell is skipped
    T mx = T(0);
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int t = tid + NTH * j;
        if (kFull || t < N * N) {
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const T o = fv[j][k] * sc;
                __builtin_nontemporal_store(o, dst + t + k * N * N);
                mx = fmax(mx, o);
            }
        }
    }
    if (mom_post && tid < 20) mom_post[cell * 20 + tid] = fin_s[tid] * (tid < 4 ? dV : G.m * dV) * scale;
    if (clip_part && tid == 0) clip_part[blockIdx.x] = (unsigned)fin_s[20];
    if (max_out) block_max_part(mx, max_out);
}

// Moment fitting of one large cubic cell per block (34^3) without holding the
// cell: the normalisation sums need only the two Maxwellians, so the block
// computes them first; f is then streamed once, pencil by pencil (thread t
// owns the v_x pencils t + NTH j), exchanged, clipped, summed into the FP64
// post-fit moments and stored unscaled, through the caches.  Where the
// density rescale factor rounds to one in the storage type the stored values
// are final, equal to fit3_cube_kernel's; elsewhere (a quarter to a third of
// the cells in FP32) each thread reads back the values it stored, which are
// mostly still in L2, and rescales them.  No 157 KB (FP32) or 314 KB (FP64)
// cell is held in registers or shared memory, so several cells share a CU.
// The loads are ordinary too: a 34^3 v_x plane is not a whole number of
// lines, and the caches merge the lines two wave accesses share (FP32: 2.82
// -> 2.47 ms per 256x128x34^3 launch; FP64 unchanged).
// The arithmetic is fit3_cube_kernel's (pencil sums of the samples in four
// chains in FP32, two in FP64; samples computed again in the exchange).
template <class T, int N, int NTH>
__global__ void __launch_bounds__(NTH)
fit3_stream_kernel(const T* fin, T* fout, const FitCell* __restrict__ P, double* __restrict__ mom_post,
                   unsigned* __restrict__ clip_part, VGrid G, XTable X, typename Bits<T>::U* __restrict__ max_out) {
    constexpr int NN = N * N;
    constexpr int NS = (NN + NTH - 1) / NTH;     // pencil sets
    constexpr int NW = NTH / kWave;
    constexpr int CH = sizeof(T) == 4 ? 4 : 2;   // pass-1 sum chains
    constexpr unsigned XB = NN * sizeof(T);      // bytes between v_x planes
    static_assert(NTH % kWave == 0, "launch shape");
    __shared__ double red[NW * 21];
    __shared__ double fin_s[21];
    const int tid = threadIdx.x;
    const long long cell = xcd_work_index(blockIdx.x, gridDim.x);
    const double dV = G.dv[0] * G.dv[1] * G.dv[2];
    const auto rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(fin + cell * (N * NN)), 0, N * XB, kBufWord3);
    const auto rd = __builtin_amdgcn_make_buffer_rsrc(fout + cell * (N * NN), 0, N * XB, kBufWord3);
    auto act = [&](int j) { return tid + NTH * j < NN; };
    const FitCell& C = P[cell];
    const bool ok = C.ok != 0.0;
    const double nV = C.nV;
    T A = T(0), Bc = T(0);
    if (ok) {
        // normalisation sums of the two Maxwellians (FP64 across pencils)
        double s[2] = {0.0, 0.0};
#pragma unroll 1
        for (int j = 0; j < NS; ++j) {
            if (act(j)) {
                const int t = tid + NTH * j;
                QuadX<T> qv, qf;
                qv.set(C.aV, C.uV, vc(G, 1, t / N), vc(G, 2, t % N));
                qf.set(C.aF, C.uF, vc(G, 1, t / N), vc(G, 2, t % N));
                T pa[CH], pb[CH];
#pragma unroll
                for (int c = 0; c < CH; ++c) pa[c] = pb[c] = T(0);
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    pa[k % CH] += qv.g((T)X.v[k]);
                    pb[k % CH] += qf.g((T)X.v[k]);
                }
                if constexpr (CH == 4) {
                    s[0] += (double)((pa[0] + pa[1]) + (pa[2] + pa[3]));
                    s[1] += (double)((pb[0] + pb[1]) + (pb[2] + pb[3]));
                } else {
                    s[0] += (double)(pa[0] + pa[1]);
                    s[1] += (double)(pb[0] + pb[1]);
                }
            }
        }
        block_sum_rs<2>(s, red, fin_s);
        A = (T)(nV / (fin_s[0] * dV));
        Bc = (T)(nV / (fin_s[1] * dV));
    }
    // exchange, clip, FP64 moments and the unscaled store, one pencil at a time
    double acc[21];
#pragma unroll
    for (int q = 0; q < 21; ++q) acc[q] = 0.0;
    unsigned nclip = 0;     // clipped elements of this wave (the same in every lane)
    T mx = T(0);
#pragma unroll 1
    for (int j = 0; j < NS; ++j) {
        const bool a = act(j);
        const int t = a ? tid + NTH * j : 0;
        const unsigned po = (unsigned)t * sizeof(T);
        T g[N];
#pragma unroll
        for (int k = 0; k < N; ++k) g[k] = a ? buf_ld<kBufCached>(rs, po, k * XB, T()) : T(0);
        if (ok) {
            QuadX<T> qv, qf;
            qv.set(C.aV, C.uV, vc(G, 1, t / N), vc(G, 2, t % N));
            qf.set(C.aF, C.uF, vc(G, 1, t / N), vc(G, 2, t % N));
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const T x = g[k] - A * qv.g((T)X.v[k]) + Bc * qf.g((T)X.v[k]);
                const bool neg = x < T(0);
                nclip += (unsigned)__builtin_popcountll(__builtin_amdgcn_ballot_w64(a && neg));
                g[k] = neg ? T(0) : x;
            }
        }
        if (a) {
            double Se[4] = {0.0, 0.0, 0.0, 0.0}, So[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const double v = (double)g[k];
                double* S = (k & 1) ? So : Se;
                S[0] += v;
                S[1] = fma(v, X.v[k], S[1]);
                S[2] = fma(v, X.v2[k], S[2]);
                S[3] = fma(v, X.v3[k], S[3]);
                buf_st<kBufCached>(g[k], rd, po, k * XB);
                mx = fmax(mx, g[k]);
            }
            const double S[4] = {Se[0] + So[0], Se[1] + So[1], Se[2] + So[2], Se[3] + So[3]};
            double m[20];
            pencil_moments(S, vc(G, 1, t / N), vc(G, 2, t % N), m);
#pragma unroll
            for (int q = 0; q < 20; ++q) acc[q] += m[q];
        }
    }
    acc[20] = (tid & (kWave - 1)) == 0 ? (double)nclip : 0.0;
    block_sum_rs<21>(acc, red, fin_s);
    const double scale = ok ? nV / (fin_s[0] * dV) : 1.0;
    const T sc = (T)scale;     // 1 exactly when the cell is skipped
    if (sc != T(1)) {          // uniform over the block
        mx = T(0);
#pragma unroll 1
        for (int j = 0; j < NS; ++j) {
            if (act(j)) {
                const unsigned po = (unsigned)(tid + NTH * j) * sizeof(T);
                T g[N];
#pragma unroll
                for (int k = 0; k < N; ++k) g[k] = buf_ld<kBufCached>(rd, po, k * XB, T());
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    const T o = g[k] * sc;
                    buf_st(o, rd, po, k * XB);
                    mx = fmax(mx, o);
                }
            }
        }
    }
    if (mom_post && tid < 20) mom_post[cell * 20 + tid] = fin_s[tid] * (tid < 4 ? dV : G.m * dV) * scale;
    if (clip_part && tid == 0) clip_part[blockIdx.x] = (unsigned)fin_s[20];
    if (max_out) block_max_part(mx, max_out);
}

template <class T>
__global__ void __launch_bounds__(256)
fit1_kernel(const T* fin, T* fout, const double* __restrict__ mom_pre, double* __restrict__ U,
            double* __restrict__ mom_post, unsigned long long* __restrict__ counters, int nv, double vlo,
            double dv, double mass, typename Bits<T>::U* __restrict__ max_out) {
    extern __shared__ unsigned char smem_raw[];
    T* g = reinterpret_cast<T*>(smem_raw);
    __shared__ double red[5 * 4];
    const long long cell = blockIdx.x;
    const T* src = fin + cell * nv;
    T* dst = fout + cell * nv;
    const double nV = mom_pre[cell * 4 + 0];
    const double Un = U[cell * 3 + 0], Unu = U[cell * 3 + 1], UP = U[cell * 3 + 2];
    bool ok = nV > 1e-12 && Un > 1e-12;
    double uV = 0, TV = 0, uF = 0, TF = 0;
    if (ok) {
        uV = mom_pre[cell * 4 + 1] / nV;
        TV = (mom_pre[cell * 4 + 2] - mass * nV * uV * uV) / nV;
        uF = Unu / Un;
        TF = (UP - mass * Un * uF * uF) / Un;
        ok = TV > 0.0 && TF > 0.0;
    }
    const T aV = (T)(0.5 * mass / TV), aF = (T)(0.5 * mass / TF);
    double s[2] = {0.0, 0.0};
    if (ok) {
        for (int j = threadIdx.x; j < nv; j += blockDim.x) {
            const double v = vlo + (j + 0.5) * dv;
            const T wv = (T)(v - uV), wf = (T)(v - uF);
            s[0] += (double)expo<T>(-aV * wv * wv);
            s[1] += (double)expo<T>(-aF * wf * wf);
        }
    }
    block_sum<2>(s, red);
    const T A = ok ? (T)(nV / (s[0] * dv)) : T(0);
    const T Bc = ok ? (T)(nV / (s[1] * dv)) : T(0);
    double acc[5] = {0, 0, 0, 0, 0};
    for (int j = threadIdx.x; j < nv; j += blockDim.x) {
        T x = src[j];
        if (ok) {
            const double v = vlo + (j + 0.5) * dv;
            const T wv = (T)(v - uV), wf = (T)(v - uF);
            x = x - A * expo<T>(-aV * wv * wv) + Bc * expo<T>(-aF * wf * wf);
            if (x < T(0)) acc[4] += 1.0;
            x = fmax(x, T(0));
        }
        g[j] = x;
        const double v = vlo + (j + 0.5) * dv;
        const double xd = (double)x, xv = xd * v;
        acc[0] += xd;
        acc[1] += xv;
        acc[2] += xv * v;
        acc[3] += xv * v * v;
    }
    block_sum<5>(acc, red);
    const double scale = ok ? nV / (acc[0] * dv) : 1.0;
    const T sc = (T)scale;
    T mx = T(0);
    for (int j = threadIdx.x; j < nv; j += blockDim.x) {
        const T o = ok ? g[j] * sc : g[j];
        dst[j] = o;
        mx = fmax(mx, o);
    }
    if (threadIdx.x == 0) {
        if (mom_post) {
            mom_post[cell * 4 + 0] = acc[0] * dv * scale;
            mom_post[cell * 4 + 1] = acc[1] * dv * scale;
            mom_post[cell * 4 + 2] = mass * acc[2] * dv * scale;
            mom_post[cell * 4 + 3] = mass * acc[3] * dv * scale;
        }
        if (ok) {
            const double r = nV / Un;
            U[cell * 3 + 0] = Un * r;
            U[cell * 3 + 1] = Unu * r;
            U[cell * 3 + 2] = UP * r;
        }
        if (counters) {
            if (acc[4] > 0) atomicAdd(&counters[0], (unsigned long long)acc[4]);
            if (!ok) atomicAdd(&counters[1], 1ull);
        }
    }
    if (max_out) block_max_part(mx, max_out);
}

// ------------------------------------------------------------ launchers ----
static int threads_for(int work) {
    int t = ((work + 63) / 64) * 64;
    return t > 256 ? 256 : (t < 64 ? 64 : t);
}

static XTable xtable(const VGridArgs& a) {
    XTable X{};
    for (int k = 0; k < a.nv[0] && k < kBigCube; ++k) {
        const double v = a.lo[0] + (k + 0.5) * a.dv[0];
        X.v[k] = v;
        X.v2[k] = v * v;
        X.v3[k] = v * v * v;
    }
    return X;
}

static int cube_edge(const VGridArgs& a) {
    const bool cube = a.nv[0] == a.nv[1] && a.nv[1] == a.nv[2];
    return (cube && (a.nv[0] == 8 || a.nv[0] == 12 || a.nv[0] == 16 || a.nv[0] == kBigCube)) ? a.nv[0] : 0;
}

template <class T>
hipError_t launch_moments3(const T* f, double* mom, long long cells, const VGridArgs& a, hipStream_t st) {
    VGrid G{a.nv[0], a.nv[1], a.nv[2], {a.lo[0], a.lo[1], a.lo[2]}, {a.dv[0], a.dv[1], a.dv[2]}, a.m, 1.0f / (float)a.nv[2]};
    const int N = cube_edge(a);
    if (N) {
        const XTable X = xtable(a);
        const dim3 grid((unsigned)((cells + 3) / 4)), blk(256);
        if (N == 16) hipLaunchKernelGGL((moments3_cube_kernel<T, 16>), grid, blk, 0, st, f, mom, cells, G, X);
        if (N == 12) {
            // 16-byte pieces need a 16-byte aligned f (any allocation is)
            if constexpr (sizeof(T) == 4) {
                if (reinterpret_cast<uintptr_t>(f) % 16 == 0)
                    hipLaunchKernelGGL((moments3_staged_kernel<12>), grid, blk, 0, st, f, mom, cells, G, X);
                else
                    hipLaunchKernelGGL((moments3_cube_kernel<T, 12>), grid, blk, 0, st, f, mom, cells, G, X);
            } else {
                hipLaunchKernelGGL((moments3_cube_kernel<T, 12>), grid, blk, 0, st, f, mom, cells, G, X);
            }
        }
        if (N == 8) hipLaunchKernelGGL((moments3_cube_kernel<T, 8>), grid, blk, 0, st, f, mom, cells, G, X);
        if (N == kBigCube)
            hipLaunchKernelGGL((moments3_big_kernel<T, kBigCube, 256>), dim3((unsigned)cells), blk, 0, st, f, mom,
                               G, X);
        return hipGetLastError();
    }
    const size_t shm = sizeof(T) * (size_t)a.nv[0] * a.nv[1] * (a.nv[2] | 1);
    hipLaunchKernelGGL((moments3_kernel<T>), dim3((unsigned)cells), dim3(threads_for(a.nv[0] * a.nv[1])), shm, st, f,
                       mom, G);
    return hipGetLastError();
}

template <class T>
hipError_t launch_moments1(const T* f, double* mom, long long cells, int nv, double vlo, double dv, double m,
                           hipStream_t st) {
    hipLaunchKernelGGL((moments1_kernel<T>), dim3((unsigned)cells), dim3(threads_for(nv)), 0, st, f, mom, nv, vlo, dv,
                       m);
    return hipGetLastError();
}

// counters[0] += sum of the per-block clip counts part[0..n), in two launches
// like the maxima (launch_max_finalize): up to kFinStage blocks sum ranges
// into a stage of 64-bit sums right after the partials, one wave adds the
// stage to the counter.  Integer sums: exact in any order.
__global__ void __launch_bounds__(256)
count_stage_kernel(const unsigned* __restrict__ part, long long n, long long chunk,
                   unsigned long long* __restrict__ out, int add) {
    __shared__ unsigned long long red[256 / kWave];
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = lo + chunk < n ? lo + chunk : n;
    unsigned long long acc = 0;
    for (long long b = lo; b < hi; b += 8 * 256) {
        unsigned v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const long long i = b + u * 256 + threadIdx.x;
            v[u] = i < hi ? part[i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 256 / kWave; ++w) acc += red[w];
        if (add)
            out[0] += acc;
        else
            out[blockIdx.x] = acc;
    }
}

__global__ void __launch_bounds__(kWave)
count_final_kernel(const unsigned long long* __restrict__ stage, int g, unsigned long long* __restrict__ counters) {
    unsigned long long a = (int)threadIdx.x < g ? stage[threadIdx.x] : 0ull;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) a += __shfl_xor(a, o, kWave);
    if (threadIdx.x == 0) counters[0] += a;
}

static void launch_count_finalize(const unsigned* part, long long n, unsigned long long* counters, hipStream_t st) {
    const FinSplit fs = fin_split(n);
    if (fs.blocks == 1) {
        hipLaunchKernelGGL(count_stage_kernel, dim3(1), dim3(256), 0, st, part, n, n, counters, 1);
        return;
    }
    auto* stage = (unsigned long long*)((char*)part + fin_stage(n, sizeof(unsigned)));
    hipLaunchKernelGGL(count_stage_kernel, dim3(fs.blocks), dim3(256), 0, st, part, n, fs.chunk, stage, 0);
    hipLaunchKernelGGL(count_final_kernel, dim3(1), dim3(kWave), 0, st, (const unsigned long long*)stage, fs.blocks,
                       counters);
}

template <class T>
hipError_t launch_fit3(const T* fin, T* fout, const double* mom_pre, double* U, double* mom_post, void* counters,
                       long long cells, const VGridArgs& a, void* max_out, void* part, unsigned* clip_part,
                       double* scratch, hipStream_t st) {
    VGrid G{a.nv[0], a.nv[1], a.nv[2], {a.lo[0], a.lo[1], a.lo[2]}, {a.dv[0], a.dv[1], a.dv[2]}, a.m, 1.0f / (float)a.nv[2]};
    const int nv = a.nv[0] * a.nv[1] * a.nv[2];
    const size_t shm = sizeof(T) * (size_t)a.nv[0] * a.nv[1] * (a.nv[2] | 1);
    const int threads = 256;
    const int ept = (nv + threads - 1) / threads;
    auto* cnt = (unsigned long long*)counters;
    auto* mo = (typename Bits<T>::U*)(max_out ? part : nullptr);
    unsigned* cp = cnt ? clip_part : nullptr;
    const int N = cube_edge(a);
    if (N) {
        const XTable X = xtable(a);
        const dim3 grid((unsigned)cells);
        FitCell* P = reinterpret_cast<FitCell*>(scratch);
        hipLaunchKernelGGL(fit3_params_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st, mom_pre, U,
                           cells, a.m, ExpK<T>::scale, P, cnt);
        // waves per cell and pencils per thread: every lane busy for 16^3, 3/4 for 12^3
        if constexpr (sizeof(T) == 4) {
            if (N == 16) hipLaunchKernelGGL((fit3_cube_kernel<T, 16, kFit16Waves, kFit16Pencils>), grid, dim3(64 * kFit16Waves), 0, st, fin, fout, P, mom_post, cp, G, X, mo);
            if (N == 12) hipLaunchKernelGGL((fit3_cube_kernel<T, 12, kFit12Waves, kFit12Pencils>), grid, dim3(64 * kFit12Waves), 0, st, fin, fout, P, mom_post, cp, G, X, mo);
            if (N == 8) hipLaunchKernelGGL((fit3_cube_kernel<T, 8, 1, 1>), grid, dim3(64), 0, st, fin, fout, P, mom_post, cp, G, X, mo);
            if (N == kBigCube)   // streamed: the cell is not held
                hipLaunchKernelGGL((fit3_stream_kernel<T, kBigCube, 256>), grid, dim3(256), 0, st, fin, fout, P,
                                   mom_post, cp, G, X, mo);
        } else {
            if (N == 16) hipLaunchKernelGGL((fit3_cube_kernel<T, 16, 4, 1>), grid, dim3(256), 0, st, fin, fout, P, mom_post, cp, G, X, mo);
            if (N == 12) hipLaunchKernelGGL((fit3_cube_kernel<T, 12, 3, 1>), grid, dim3(192), 0, st, fin, fout, P, mom_post, cp, G, X, mo);
            if (N == 8) hipLaunchKernelGGL((fit3_cube_kernel<T, 8, 1, 1>), grid, dim3(64), 0, st, fin, fout, P, mom_post, cp, G, X, mo);
            if (N == kBigCube)   // streamed: the cell is not held
                hipLaunchKernelGGL((fit3_stream_kernel<T, kBigCube, 256>), grid, dim3(256), 0, st, fin, fout, P,
                                   mom_post, cp, G, X, mo);
        }
        hipError_t e = hipGetLastError();
        if (e == hipSuccess && cnt)
            launch_count_finalize(clip_part, cells, cnt, st);
        if (e == hipSuccess && max_out) e = launch_max_finalize<T>(part, cells, max_out, st);
        return e == hipSuccess ? hipGetLastError() : e;
    }
    if (ept <= 4)
        hipLaunchKernelGGL((fit3_kernel<T, 4>), dim3((unsigned)cells), dim3(threads), shm, st, fin, fout, mom_pre, U,
                           mom_post, cnt, G, mo);
    else if (ept <= 8)
        hipLaunchKernelGGL((fit3_kernel<T, 8>), dim3((unsigned)cells), dim3(threads), shm, st, fin, fout, mom_pre, U,
                           mom_post, cnt, G, mo);
    else if (ept <= 16)
        hipLaunchKernelGGL((fit3_kernel<T, 16>), dim3((unsigned)cells), dim3(threads), shm, st, fin, fout, mom_pre, U,
                           mom_post, cnt, G, mo);
    else if (ept <= 32)
        hipLaunchKernelGGL((fit3_kernel<T, 32>), dim3((unsigned)cells), dim3(threads), shm, st, fin, fout, mom_pre, U,
                           mom_post, cnt, G, mo);
    else
        return hipErrorInvalidValue;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess || !max_out) return e;
    return launch_max_finalize<T>(part, cells, max_out, st);
}

template <class T>
hipError_t launch_fit1(const T* fin, T* fout, const double* mom_pre, double* U, double* mom_post, void* counters,
                       long long cells, int nv, double vlo, double dv, double m, void* max_out, void* part,
                       hipStream_t st) {
    hipLaunchKernelGGL((fit1_kernel<T>), dim3((unsigned)cells), dim3(threads_for(nv)), sizeof(T) * (size_t)nv, st,
                       fin, fout, mom_pre, U, mom_post, (unsigned long long*)counters, nv, vlo, dv, m,
                       (typename Bits<T>::U*)(max_out ? part : nullptr));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess || !max_out) return e;
    return launch_max_finalize<T>(part, cells, max_out, st);
}

#define VL_INST(T)                                                                                              \
    template hipError_t launch_moments3<T>(const T*, double*, long long, const VGridArgs&, hipStream_t);         \
    template hipError_t launch_moments1<T>(const T*, double*, long long, int, double, double, double,            \
                                           hipStream_t);                                                        \
    template hipError_t launch_fit3<T>(const T*, T*, const double*, double*, double*, void*, long long,         \
                                       const VGridArgs&, void*, void*, unsigned*, double*, hipStream_t);        \
    template hipError_t launch_fit1<T>(const T*, T*, const double*, double*, double*, void*, long long, int,    \
                                       double, double, double, void*, void*, hipStream_t);
VL_INST(float)
VL_INST(double)
#undef VL_INST

}  // namespace vl

namespace vl {

// ------------------------------------------------------------ diagnostics --
// Deterministic two-level sums: block partials in a fixed order, then one
// block adds the partials in index order.
template <class T>
__global__ void __launch_bounds__(256)
partial_sum_kernel(const T* __restrict__ f, long long n, double* __restrict__ part) {
    __shared__ double red[4];
    double acc[1] = {0.0};
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        acc[0] += (double)f[i];
    block_sum<1>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

__global__ void __launch_bounds__(256)
energy_partial_kernel(const double* __restrict__ mom, long long cells, int kmom, int dimv, double* __restrict__ part) {
    __shared__ double red[4];
    double acc[1] = {0.0};
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (long long)gridDim.x * blockDim.x)
        acc[0] += dimv == 3 ? 0.5 * (mom[c * kmom + 4] + mom[c * kmom + 7] + mom[c * kmom + 9]) : 0.5 * mom[c * kmom + 2];
    block_sum<1>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

__global__ void __launch_bounds__(256)
finish_sum_kernel(const double* __restrict__ part, int np, double scale, double* __restrict__ out) {
    __shared__ double red[4];
    // thread t adds partials t, t+256, ... in order; then a fixed-order block sum
    double acc[1] = {0.0};
    for (int i = threadIdx.x; i < np; i += blockDim.x) acc[0] += part[i];
    block_sum<1>(acc, red);
    if (threadIdx.x == 0) *out = acc[0] * scale;
}

template <class T>
hipError_t launch_mass_energy(const T* f, const double* mom, long long cells, long long nv, int kmom, int dimv,
                              double dV, double dX, double* out, double* part, hipStream_t st) {
    // out[0] = mass, out[1] = energy; part: 1024 doubles of scratch
    const int np = 1024;
    hipLaunchKernelGGL((partial_sum_kernel<T>), dim3(np), dim3(256), 0, st, f, cells * nv, part);
    hipLaunchKernelGGL(finish_sum_kernel, dim3(1), dim3(256), 0, st, part, np, dV * dX, out);
    hipLaunchKernelGGL(energy_partial_kernel, dim3(np), dim3(256), 0, st, mom, cells, kmom, dimv, part);
    hipLaunchKernelGGL(finish_sum_kernel, dim3(1), dim3(256), 0, st, part, np, dX, out + 1);
    return hipGetLastError();
}

template hipError_t launch_mass_energy<float>(const float*, const double*, long long, long long, int, int, double,
                                              double, double*, double*, hipStream_t);
template hipError_t launch_mass_energy<double>(const double*, const double*, long long, long long, int, int, double,
                                               double, double*, double*, hipStream_t);

}  // namespace vl
