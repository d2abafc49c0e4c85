// Device helpers shared by the gfx950 kernels of the Vlasov hot path.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vl {

constexpr int kWave = 64;

// Bit patterns used for atomic maxima of non-negative floating-point values:
// for x, y >= 0 the IEEE bit patterns order like the values.
template <class T> struct Bits;
template <> struct Bits<float> {
    using U = unsigned int;
    static __device__ __forceinline__ U of(float x) { return __float_as_uint(x); }
};
template <> struct Bits<double> {
    using U = unsigned long long;
    static __device__ __forceinline__ U of(double x) { return (U)__double_as_longlong(x); }
};

template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Maximum over the block, folded into *slot with one atomic per block.
// Every thread of the block must call it (it synchronises).
template <class T>
__device__ __forceinline__ void block_max_to(T v, typename Bits<T>::U* slot) {
    __shared__ T red[16];
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthr = blockDim.x * blockDim.y * blockDim.z;
    v = wave_max(v);
    if ((tid & (kWave - 1)) == 0) red[tid / kWave] = v;
    __syncthreads();
    if (tid == 0) {
        T m = red[0];
        for (int w = 1; w < (nthr + kWave - 1) / kWave; ++w) m = fmax(m, red[w]);
        atomicMax(slot, Bits<T>::of(m));
    }
}

// Sum of N doubles per thread over the block; result in out[] of every thread.
// red must hold N * (blockDim / 64) doubles of shared memory.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double* red) {
    const int tid = threadIdx.x;
    const int nw = (blockDim.x + kWave - 1) / kWave;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
    if ((tid & (kWave - 1)) == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) red[(tid / kWave) * N + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[w * N + k];
        v[k] = s;
    }
    __syncthreads();
}

// PFC partial flux phi(j, a) of the limited parabola of cell j within a cell
// widths of its downwind face.  fm, f0, fp: upwind neighbour, cell, downwind
// neighbour.  c1 = (1-a)(2-a)/6, c2 = (1-a)(1+a)/6.  The limiter is the
// division-free form of the PFC slope limiters with bound max(finf, f0):
//   L+ = clamp(fp - f0, -2 (bound - f0), 2 f0)
//   L- = clamp(f0 - fm, -2 f0, 2 (bound - f0))
template <class T>
__device__ __forceinline__ T pfc_phi(T fm, T f0, T fp, T a, T c1, T c2, T finf) {
    const T room = fmax(finf, f0) - f0;
    const T lp = fmin(fmax(fp - f0, T(-2) * room), T(2) * f0);
    const T lm = fmin(fmax(f0 - fm, T(-2) * f0), T(2) * room);
    return a * (f0 + c1 * lp + c2 * lm);
}

// Split a non-negative displacement of s cells into floor and fraction, with
// the coefficients of the partial flux (computed in FP64, rounded to T).
template <class T>
struct Shift {
    long long K;
    T a, c1, c2;
    // Displacements beyond 1e9 cells are clamped there (far past any grid).
    __device__ __forceinline__ explicit Shift(double sa) {
        sa = fmin(sa, 1.0e9);
        const double Kd = floor(sa);
        const double ad = sa - Kd;
        K = (long long)Kd;
        a = (T)ad;
        c1 = (T)((1.0 - ad) * (2.0 - ad) / 6.0);
        c2 = (T)((1.0 - ad) * (1.0 + ad) / 6.0);
    }
};

}  // namespace vl
