// Device helpers shared by the gfx950 kernels of the Vlasov hot path.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vl {

constexpr int kWave = 64;

// Bit patterns in which per-block maxima of non-negative floating-point values
// are stored: for x, y >= 0 the IEEE bit patterns order like the values.
template <class T> struct Bits;
template <> struct Bits<float> {
    using U = unsigned int;
    static __device__ __forceinline__ U of(float x) { return __float_as_uint(x); }
};
template <> struct Bits<double> {
    using U = unsigned long long;
    static __device__ __forceinline__ U of(double x) { return (U)__double_as_longlong(x); }
};

// Workgroups are handed to the 8 XCDs round-robin in launch order.  This maps
// the launch index to a work index so that each XCD gets one contiguous range
// of work items: blocks resident on one XCD (sharing its L2) then touch
// neighbouring data instead of every eighth item.
constexpr unsigned kXcds = 8;
__device__ __forceinline__ unsigned xcd_work_index(unsigned b, unsigned nblocks) {
    const unsigned xcd = b % kXcds, local = b / kXcds;
    const unsigned per = nblocks / kXcds, rem = nblocks % kXcds;
    return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

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

// Reduce-scatter of K doubles over the 64 lanes of a wave by recursive
// halving: at distance D every lane keeps one half of its array (the upper
// half where bit D of the lane index is set), sends the other half to lane^D
// and adds what it receives.  Moving ceil(K/2) + ceil(K/4) + ... values
// instead of K per step, it needs about 24 exchanges for K = 21 where a
// butterfly on every value needs 126.  Returns this lane's total; idx is the
// value index it belongs to, valid only where cnt > 0 (odd halves are padded,
// and a padding slot's running index can equal a real index of another lane
// group); lanes l and l^1 hold the same value.  Every lane must call it with
// idx = 0 and cnt = K; the summation order is fixed.
template <int K, int D>
struct ReduceScatter {
    static __device__ __forceinline__ double run(const double* a, int lane, int& idx, int& cnt) {
        constexpr int H = (K + 1) / 2;
        const bool up = (lane & D) != 0;
        double b[H];
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const double lo = a[i];
            const double hi = (H + i < K) ? a[H + i] : 0.0;
            const double send = up ? lo : hi;
            b[i] = (up ? hi : lo) + __shfl_xor(send, D, kWave);
        }
        if (up) {
            idx += H;
            cnt -= H;
        } else {
            cnt = cnt < H ? cnt : H;
        }
        return ReduceScatter<H, D / 2>::run(b, lane, idx, cnt);
    }
};
template <int D>
struct ReduceScatter<1, D> {
    static __device__ __forceinline__ double run(const double* a, int lane, int& idx, int& cnt) {
        const double v = a[0] + __shfl_xor(a[0], D, kWave);
        return ReduceScatter<1, D / 2>::run(&v, lane, idx, cnt);
    }
};
template <>
struct ReduceScatter<1, 0> {
    static __device__ __forceinline__ double run(const double* a, int, int&, int&) { return a[0]; }
};

// Block sum of K doubles per thread (waves of 64): totals in fin[0..K-1]
// (shared memory) for every thread after return.  red: NW*K doubles of shared
// scratch, NW = waves in the block.  Fixed summation order.
template <int K>
__device__ __forceinline__ void block_sum_rs(const double (&a)[K], double* red, double* fin) {
    // up to 32 values the last exchange (distance 1) is a full add, so lanes l
    // and l^1 agree and the even lanes carry every index (some more than once,
    // with identical values)
    static_assert(K >= 1 && K <= 32, "reduce-scatter of at most 32 values");
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int nw = (blockDim.x + kWave - 1) / kWave;
    int idx = 0, cnt = K;
    const double v = ReduceScatter<K, kWave / 2>::run(a, lane, idx, cnt);
    if ((lane & 1) == 0 && cnt > 0) red[w * K + idx] = v;
    __syncthreads();
    if (threadIdx.x < K) {
        double s = 0.0;
        for (int k = 0; k < nw; ++k) s += red[k * K + threadIdx.x];
        fin[threadIdx.x] = s;
    }
    __syncthreads();
}

// Streaming access to f: non-temporal (the lines are not kept in the caches)
// when NT, else an ordinary access.  Velocity blocks whose rows are not whole
// 128-byte lines (12^3 FP32: 576 B) have lines shared by two wave accesses;
// there the caches merge the halves instead of fetching or writing each line
// twice.
template <class T, int N>
constexpr bool kRowsWholeLines = (N * N * (int)sizeof(T)) % 128 == 0;
template <bool NT, class T>
__device__ __forceinline__ T ld_f(const T* p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}
template <bool NT, class T>
__device__ __forceinline__ void st_f(T v, T* p) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Raw buffer access to a block of memory (one cell's f): its base in a buffer
// descriptor (wave-uniform, scalar registers), a per-lane byte offset and a
// scalar byte offset, so a pencil of elements a plane apart costs one vector
// register of address.  Accesses past the block read 0 and write nothing.
// Word 3 of the descriptor is the gfx9 raw-buffer format (32-bit data).
constexpr int kBufWord3 = 0x00020000;
constexpr int kBufNT = 2;          // cache policy: non-temporal
constexpr int kBufCached = 0;      // cache policy: ordinary (kept in the caches)
template <int POL = kBufNT>
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, POL));
}
template <int POL = kBufNT>
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, POL));
}
template <int POL = kBufNT>
__device__ __forceinline__ void buf_st(double v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, voff, soff, POL);
}
template <int POL = kBufNT>
__device__ __forceinline__ void buf_st(float v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, POL);
}

// Maximum over the block of non-negative values, stored (as its bit pattern)
// in part[blockIdx.x].  No atomics: many blocks folding into one address
// serialise at the memory-side atomic unit, so a second launch
// (launch_max_finalize) reduces the partials.  Every thread of the block must
// call it (it synchronises).
template <class T>
__device__ __forceinline__ void block_max_part(T v, typename Bits<T>::U* part) {
    __shared__ T red[16];
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthr = blockDim.x * blockDim.y * blockDim.z;
    v = wave_max(v);
    if ((tid & (kWave - 1)) == 0) red[tid / kWave] = v;
    __syncthreads();
    if (tid == 0) {
        T m = red[0];
        for (int w = 1; w < (nthr + kWave - 1) / kWave; ++w) m = fmax(m, red[w]);
        part[blockIdx.x] = Bits<T>::of(m);
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

template <class T>
__device__ __forceinline__ T med3(T x, T lo, T hi);
template <>
__device__ __forceinline__ float med3<float>(float x, float lo, float hi) {
    return __builtin_amdgcn_fmed3f(x, lo, hi);
}
template <>
__device__ __forceinline__ double med3<double>(double x, double lo, double hi) {
    return fmin(fmax(x, lo), hi);
}

// The same partial flux in the form the sweep kernels use: from the cell value
// w and its upwind/downwind differences dm = w - w_up, dp = w_down - w (each
// difference is shared by two neighbouring cells), with a*c1, a*c2 folded and
// F2 = 2 f_inf.  2 (bound - f0) = max(F2 - 2 w, 0), and the clamps are medians
// of three (both bounds bracket 0 for w >= 0):
//   phi = a w + a c1 med3(dp, -r2, 2w) + a c2 med3(dm, -2w, r2).
template <class T>
__device__ __forceinline__ T pfc_phi_d(T w, T dm, T dp, T a, T ac1, T ac2, T F2) {
    const T x2 = w + w;
    const T r2 = fmax(F2 - x2, T(0));
    const T lp = med3(dp, -r2, x2);
    const T lm = med3(dm, -x2, r2);
    return fma(ac1, lp, fma(ac2, lm, a * w));
}

// Larger of two values in [0, hi] (none NaN): one median-of-three in FP32,
// without the quieting of the inputs that fmax carries.
template <class T>
__device__ __forceinline__ T max_nonneg(T a, T b, T hi);
template <>
__device__ __forceinline__ float max_nonneg<float>(float a, float b, float hi) {
    return __builtin_amdgcn_fmed3f(a, b, hi);
}
template <>
__device__ __forceinline__ double max_nonneg<double>(double a, double b, double) {
    return fmax(a, b);
}

// Split a non-negative displacement of s cells into floor and fraction, with
// the coefficients of the partial flux (computed in FP64, rounded to T).
template <class T>
struct Shift {
    long long K;
    T a, c1, c2, ac1, ac2;
    // Displacements beyond 1e9 cells are clamped there (far past any grid).
    __device__ __forceinline__ explicit Shift(double sa) {
        sa = fmin(sa, 1.0e9);
        const double Kd = floor(sa);
        const double ad = sa - Kd;
        K = (long long)Kd;
        a = (T)ad;
        const double d1 = (1.0 - ad) * (2.0 - ad) * (1.0 / 6.0), d2 = (1.0 - ad) * (1.0 + ad) * (1.0 / 6.0);
        c1 = (T)d1;
        c2 = (T)d2;
        ac1 = (T)(ad * d1);
        ac2 = (T)(ad * d2);
    }
};

// Shift split computed in the storage type (FP32 storage keeps the
// displacement to FP32 accuracy, which is what its cells can resolve); the
// integer part is clamped to 2^20, beyond any pencil.
template <class T>
struct ShiftT {
    int K;
    T a, ac1, ac2;
    __device__ __forceinline__ explicit ShiftT(double sa_d) { init((T)fmin(sa_d, 1048576.0)); }
    __device__ __forceinline__ explicit ShiftT(float sa_f) { init((T)fminf(sa_f, 1048576.0f)); }
    __device__ __forceinline__ void init(T sa) {
        const T Kf = floor(sa);
        a = sa - Kf;
        K = (int)Kf;
        // a c1 = t (2 - a), a c2 = t (1 + a) with t = a (1 - a) / 6
        const T t = a * (T(1) - a) * T(1.0 / 6.0);
        ac1 = fma(-t, a, t + t);
        ac2 = fma(t, a, t);
    }
};

}  // namespace vl
