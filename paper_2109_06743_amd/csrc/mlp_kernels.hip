// Learned heat-flux closure on gfx950: stencil features from the ten moments,
// a 64-64-64-64-16 tanh network evaluated and trained with BF16 MFMA
// (v_mfma_f32_16x16x16_bf16, FP32 accumulation), Adam on FP32 master
// weights, and the pieces the fluid update uses (third moment from the
// network, error of the network's heat flux against the kinetic one).
//
// Network layout (FP32 parameter vector, row-major [out][in]):
//   W1[64][64] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[16][64] b4[16]
// The network multiplies BF16-rounded weights and activations; biases,
// accumulation and tanh are FP32.
//
// Matrix products are computed transposed, H_l^T = W_l H_{l-1}^T, so that a
// 16x16 output tile of one layer (lane l holds rows 4(l/16)+j, column l%16)
// is already the B operand of the next layer (rows = the K index): samples
// run along the 16 lanes of a row group, features along (l/16, j), and no
// data moves between layers.
#include "vl_internal.h"

namespace vl {
namespace {

constexpr int kIn = 64, kWid = 64, kOutPad = 16, kOut = 10;
constexpr int kOffW1 = 0, kOffB1 = 4096, kOffW2 = 4160, kOffB2 = 8256, kOffW3 = 8320, kOffB3 = 12416,
              kOffW4 = 12480, kOffB4 = 13504, kNParam = 13520;
constexpr int kLdw = 68;    // bf16 row stride of weight tiles in LDS (136 B rows keep 8-byte alignment)
constexpr int kLdt4 = 20;   // row stride of W4^T [64][16]
constexpr int kLds = 20;    // row stride of the per-wave transpose staging tiles [16][16]
constexpr int kPartStride = 13536;   // floats per block partial: gradient (13520) + loss, padded

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_of(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);     // round to nearest, ties to even
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ bf16x4 pack4(const f32x4& v) {
    bf16x4 r;
    r[0] = (short)bf16_of(v[0]);
    r[1] = (short)bf16_of(v[1]);
    r[2] = (short)bf16_of(v[2]);
    r[3] = (short)bf16_of(v[3]);
    return r;
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x4 lds4(const unsigned short* p) { return *reinterpret_cast<const bf16x4*>(p); }

// Weights of the network in LDS as BF16 (plus FP32 biases); the transposed
// copies are for the backward products.
struct NetLds {
    unsigned short w[3][kWid * kLdw];     // W1..W3 [out][in]
    unsigned short w4[kOutPad * kLdw];    // W4 [16][64]
    float bias[3 * kWid + kOutPad];
};
struct NetLdsT {
    unsigned short wt[2][kWid * kLdw];    // W2^T, W3^T [in][out]
    unsigned short wt4[kWid * kLdt4];     // W4^T [64][16]
};

__device__ void load_net(const float* __restrict__ P, NetLds& N, NetLdsT* T) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    if (nthr == 256 && !((uintptr_t)P & 15u)) {
        // 256 threads, 16-byte aligned parameters: all 13 float4 loads of a
        // thread are issued before the first conversion
        float4 v[13];
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            const int off = i < 4 ? kOffW1 : (i < 8 ? kOffW2 : kOffW3);
            v[i] = reinterpret_cast<const float4*>(P + off)[(i & 3) * 256 + tid];
        }
        v[12] = reinterpret_cast<const float4*>(P + kOffW4)[tid];
        const float bv = tid < 3 * kWid + kOutPad
                             ? P[tid < 64 ? kOffB1 + tid
                                          : (tid < 128 ? kOffB2 + tid - 64
                                                       : (tid < 192 ? kOffB3 + tid - 128 : kOffB4 + tid - 192))]
                             : 0.f;
#pragma unroll
        for (int i = 0; i < 13; ++i) {
            const int e = 4 * ((i & 3) * 256 + tid);          // first of 4 consecutive inputs of one row
            const int r = e / kIn, c = e % kIn;
            const unsigned short h[4] = {bf16_of(v[i].x), bf16_of(v[i].y), bf16_of(v[i].z), bf16_of(v[i].w)};
            const uint2 pk = {(unsigned)h[0] | ((unsigned)h[1] << 16), (unsigned)h[2] | ((unsigned)h[3] << 16)};
            if (i < 12) {
                const int l = i / 4;
                *reinterpret_cast<uint2*>(&N.w[l][r * kLdw + c]) = pk;
                if (T && l > 0)
#pragma unroll
                    for (int k = 0; k < 4; ++k) T->wt[l - 1][(c + k) * kLdw + r] = h[k];
            } else {
                const int r4 = 4 * tid / kWid, c4 = 4 * tid % kWid;
                *reinterpret_cast<uint2*>(&N.w4[r4 * kLdw + c4]) = pk;
                if (T)
#pragma unroll
                    for (int k = 0; k < 4; ++k) T->wt4[(c4 + k) * kLdt4 + r4] = h[k];
            }
        }
        if (tid < 3 * kWid + kOutPad) N.bias[tid] = bv;
        return;
    }
    for (int e = tid; e < 3 * kWid * kIn; e += nthr) {
        const int l = e / (kWid * kIn), r = (e / kIn) % kWid, c = e % kIn;
        const int off = l == 0 ? kOffW1 : (l == 1 ? kOffW2 : kOffW3);
        const unsigned short v = bf16_of(P[off + r * kIn + c]);
        N.w[l][r * kLdw + c] = v;
        if (T && l > 0) T->wt[l - 1][c * kLdw + r] = v;
    }
    for (int e = tid; e < kOutPad * kWid; e += nthr) {
        const int r = e / kWid, c = e % kWid;
        const unsigned short v = bf16_of(P[kOffW4 + e]);
        N.w4[r * kLdw + c] = v;
        if (T) T->wt4[c * kLdt4 + r] = v;
    }
    for (int e = tid; e < 3 * kWid + kOutPad; e += nthr) {
        const int off = e < 64 ? kOffB1 + e : (e < 128 ? kOffB2 + e - 64 : (e < 192 ? kOffB3 + e - 128 : kOffB4 + e - 192));
        N.bias[e] = P[off];
    }
}

// tanh through the exponential, tanh|x| = 1 - 2 / (exp(2|x|) + 1), with the
// sign put back: absolute error below 1e-7, far under the BF16 rounding the
// activations then take; exp(2|x|) = inf gives exactly 1.
__device__ __forceinline__ float tanh_exp(float x) {
    const float e = __expf(2.f * fabsf(x));
    return copysignf(1.f - 2.f * __builtin_amdgcn_rcpf(e + 1.f), x);
}

// Forward pass of one 16-sample tile by one wave.  hb[0] = features, hb[1..3]
// = hidden activations (BF16 operands), h[0..2] = the same in FP32 (for tanh'),
// y = outputs (rows 4g+j of the 16 outputs, sample s).
struct Tile {
    bf16x4 hb[4][4];
    f32x4 h[3][4];
    f32x4 y;
};

// Source row of batch row r: idx[r] (rows outside [0, nrows) count as
// padding, -1) or r itself; -1 past the batch.
__device__ __forceinline__ long long source_row(long long r, long long n, const long long* __restrict__ idx,
                                                long long nrows) {
    if (r >= n) return -1;
    if (!idx) return r;
    const long long q = idx[r];
    return (q >= 0 && q < nrows) ? q : -1;
}

// This lane's features (sample s, inputs 16kb+4g..16kb+4g+3) of source row
// `row`; zeros for row -1.
__device__ __forceinline__ void load_features(const unsigned short* __restrict__ x, long long row, uint2 (&v)[4]) {
    const int g = (threadIdx.x & 63) >> 4;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
        v[kb] = row >= 0 ? *reinterpret_cast<const uint2*>(x + row * kIn + 16 * kb + 4 * g) : uint2{0u, 0u};
}

__device__ __forceinline__ void forward_from(const uint2 (&xv)[4], const NetLds& N, bool keep_fp32, Tile& T) {
    const int lane = threadIdx.x & 63, s = lane & 15, g = lane >> 4;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) T.hb[0][kb] = *reinterpret_cast<const bf16x4*>(&xv[kb]);
#pragma unroll
    for (int L = 0; L < 3; ++L) {
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            const float* b = N.bias + L * kWid + 16 * ob + 4 * g;
            f32x4 acc = {b[0], b[1], b[2], b[3]};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
                acc = mfma16(lds4(N.w[L] + (16 * ob + s) * kLdw + 16 * kb + 4 * g), T.hb[L][kb], acc);
            f32x4 h;
#pragma unroll
            for (int j = 0; j < 4; ++j) h[j] = tanh_exp(acc[j]);
            if (keep_fp32) T.h[L][ob] = h;
            T.hb[L + 1][ob] = pack4(h);
        }
    }
    const float* b4 = N.bias + 3 * kWid + 4 * g;
    f32x4 acc = {b4[0], b4[1], b4[2], b4[3]};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) acc = mfma16(lds4(N.w4 + s * kLdw + 16 * kb + 4 * g), T.hb[3][kb], acc);
    T.y = acc;
}

__device__ __forceinline__ void forward_tile(const unsigned short* __restrict__ x, long long n, long long tile,
                                             const NetLds& N, bool keep_fp32, Tile& T) {
    uint2 v[4];
    load_features(x, source_row(tile * 16 + (threadIdx.x & 15), n, nullptr, 0), v);
    forward_from(v, N, keep_fp32, T);
}

// Stage a 16x16 tile held in output layout (lane: rows 4g+j, column s) and
// return it in operand layout with the roles of rows and columns swapped
// (lane: row s, columns 4g+j), through this wave's LDS staging area.
__device__ __forceinline__ bf16x4 transpose_tile(unsigned short* stage, const f32x4& v) {
    const int lane = threadIdx.x & 63, s = lane & 15, g = lane >> 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) stage[(4 * g + j) * kLds + s] = bf16_of(v[j]);
    __builtin_amdgcn_wave_barrier();
    const bf16x4 r = lds4(stage + s * kLds + 4 * g);
    __builtin_amdgcn_wave_barrier();
    return r;
}
__device__ __forceinline__ bf16x4 transpose_tile(unsigned short* stage, const bf16x4& v) {
    const int lane = threadIdx.x & 63, s = lane & 15, g = lane >> 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) stage[(4 * g + j) * kLds + s] = (unsigned short)v[j];
    __builtin_amdgcn_wave_barrier();
    const bf16x4 r = lds4(stage + s * kLds + 4 * g);
    __builtin_amdgcn_wave_barrier();
    return r;
}

__device__ __forceinline__ float sum16(float v) {
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 8, 64);
    return v;
}

}  // namespace

// --------------------------------------------------------------- features --
// Per cell: n, u, T (6) of the centre and its 8 neighbours (x periodic, y
// mirrored with u_y, T_xy, T_yz negated), the species and the direction of
// the cell-centred magnetic field -> 64 features rounded FP64 -> FP32 ->
// BF16, and the scale n m v_t^3.
__device__ __forceinline__ bool local_nuT(const double* __restrict__ M, int stride, long long c, double m,
                                          bool mir, double& n, double (&u)[3], double (&T)[6]) {
    n = M[c * stride];
    const double inv = 1.0 / n;
    u[0] = M[c * stride + 1] * inv;
    u[1] = M[c * stride + 2] * inv;
    u[2] = M[c * stride + 3] * inv;
    const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 0; k < 6; ++k) T[k] = (M[c * stride + 4 + k] - m * n * u[pa[k]] * u[pb[k]]) * inv;
    if (mir) {
        u[1] = -u[1];
        T[1] = -T[1];
        T[4] = -T[4];
    }
    return true;
}

// Species blockIdx.z of the set (species index s0 + blockIdx.z); its
// features and scales are stored after those of the set's earlier species.
// A 256-thread block covers 4 rows x 64 columns of cells: n, u, T of its
// 6 x 66 stencil cells are formed once each into LDS (rather than nine times,
// once per neighbour), each thread then forms its cell's features from
// there, and the 256 feature rows (128 B each) leave through LDS, so that
// every wave store writes 256 contiguous bytes.
constexpr int kFeatCols = 64, kFeatRows = 4;
union FeatLds {
    double nut[kFeatRows + 2][kFeatCols + 2][11];   // n, u, T (padded against bank conflicts)
    unsigned out[kFeatRows * kFeatCols][33];         // packed BF16 feature rows (padded)
};

__global__ void __launch_bounds__(256)
mlp_features_kernel(MlpSet S, int s0, int stride, const double* __restrict__ B, int nx, int ny,
                    unsigned short* __restrict__ x, double* __restrict__ scale) {
    __shared__ FeatLds L;
    const int sp = blockIdx.z;
    const double* __restrict__ M = S.M[sp];
    const double m = S.m[sp];
    const int species = s0 + sp;
    x += (size_t)sp * nx * ny * kIn;
    scale += (size_t)sp * nx * ny;
    const int i0 = blockIdx.x * kFeatCols, j0 = blockIdx.y * kFeatRows;
    const int tid = threadIdx.x;
    for (int q = tid; q < (kFeatRows + 2) * (kFeatCols + 2); q += blockDim.x) {
        const int rr = q / (kFeatCols + 2), cc = q % (kFeatCols + 2);
        double* d = L.nut[rr][cc];
        int jj = j0 - 1 + rr;
        if (jj > ny) {             // below the mirror of row ny-1: feeds no cell
#pragma unroll
            for (int k = 0; k < 10; ++k) d[k] = 0.0;
            continue;
        }
        bool mir = false;
        if (jj < 0) { jj = -1 - jj; mir = true; }
        if (jj >= ny) { jj = 2 * ny - 1 - jj; mir = true; }
        const int ii = ((i0 - 1 + cc) % nx + nx) % nx;
        double nn, uu[3], TT[6];
        local_nuT(M, stride, (long long)jj * nx + ii, m, mir, nn, uu, TT);
        d[0] = nn;
#pragma unroll
        for (int k = 0; k < 3; ++k) d[1 + k] = uu[k];
#pragma unroll
        for (int k = 0; k < 6; ++k) d[4 + k] = TT[k];
    }
    __syncthreads();
    const int r = tid / kFeatCols, cl = tid % kFeatCols;
    const int i = i0 + cl, j = j0 + r;
    const bool valid = i < nx && j < ny;
    float f[64];    // features are rounded to FP32 (then BF16) anyway
#pragma unroll
    for (int k = 0; k < 64; ++k) f[k] = 0.f;
    double sc = 0.0;
    if (valid) {
        const double* C = L.nut[r + 1][cl + 1];
        const double n0 = C[0];
        const double u0[3] = {C[1], C[2], C[3]};
        double T0[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) T0[k] = C[4 + k];
        const double Tref = (T0[0] + T0[3] + T0[5]) / 3.0;
        if (n0 > 1e-12 && Tref > 0.0) {
            const double vt = sqrt(Tref / m);
            const double ivt = 1.0 / vt, iT = 1.0 / Tref, in0 = 1.0 / n0;
            sc = n0 * m * vt * vt * vt;
            f[0] = (float)(u0[0] * ivt);
            f[1] = (float)(u0[1] * ivt);
            f[2] = (float)(u0[2] * ivt);
#pragma unroll
            for (int k = 0; k < 6; ++k) f[3 + k] = (float)(T0[k] * iT);
            // stencil fields n/n_c, u/v_t, T/T_ref at offset (dj, di)
#pragma unroll
            for (int k = 0; k < 10; ++k) {
                const double sk = k == 0 ? in0 : (k < 4 ? ivt : iT);
                auto P = [&](int dj, int di) { return L.nut[r + 1 + dj][cl + 1 + di][k] * sk; };
                const double c0 = P(0, 0);
                f[9 + 5 * k + 0] = (float)((P(0, 1) - P(0, -1)) / 2.0);
                f[9 + 5 * k + 1] = (float)((P(1, 0) - P(-1, 0)) / 2.0);
                f[9 + 5 * k + 2] = (float)(P(0, 1) - 2.0 * c0 + P(0, -1));
                f[9 + 5 * k + 3] = (float)(P(1, 0) - 2.0 * c0 + P(-1, 0));
                f[9 + 5 * k + 4] = (float)((P(1, 1) - P(-1, 1) - P(1, -1) + P(-1, -1)) / 4.0);
            }
            f[59 + species] = 1.f;
            if (B) {     // direction of the cell-centred magnetic field
                const long long c = (long long)j * nx + i;
                const double bx = B[c * 3], by = B[c * 3 + 1], bz = B[c * 3 + 2];
                const double bn = sqrt(bx * bx + by * by + bz * bz);
                if (bn > 1e-12) {
                    f[61] = (float)(bx / bn);
                    f[62] = (float)(by / bn);
                    f[63] = (float)(bz / bn);
                }
            }
        }
    }
    __syncthreads();     // every read of the stencil values is done: the union now holds the output
#pragma unroll
    for (int k = 0; k < 32; ++k) L.out[tid][k] = bf16_of(f[2 * k]) | ((unsigned)bf16_of(f[2 * k + 1]) << 16);
    __syncthreads();
    for (int q = tid; q < kFeatRows * kFeatCols * 32; q += blockDim.x) {
        const int rr = q >> 5, part = q & 31;
        const int ii = i0 + rr % kFeatCols, jj = j0 + rr / kFeatCols;
        if (ii < nx && jj < ny)
            reinterpret_cast<unsigned*>(x + ((long long)jj * nx + ii) * kIn)[part] = L.out[rr][part];
    }
    if (valid) scale[(long long)j * nx + i] = sc;
}

// Heat-flux tensor of one cell from its raw moments (TRIPLES order).
__device__ __forceinline__ void heat_flux_cell(const double* __restrict__ M, long long c, double m, double (&Q)[10],
                                               double& n, double (&u)[3], double& Tref) {
    n = M[c * 20];
    const double inv = 1.0 / n;
    u[0] = M[c * 20 + 1] * inv;
    u[1] = M[c * 20 + 2] * inv;
    u[2] = M[c * 20 + 3] * inv;
    double P[3][3];
    const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 0; k < 6; ++k) P[pa[k]][pb[k]] = P[pb[k]][pa[k]] = M[c * 20 + 4 + k];
    Tref = ((P[0][0] - m * n * u[0] * u[0]) + (P[1][1] - m * n * u[1] * u[1]) + (P[2][2] - m * n * u[2] * u[2])) *
           inv / 3.0;
    const int ta[10] = {0, 0, 0, 0, 0, 0, 1, 1, 1, 2}, tb[10] = {0, 0, 0, 1, 1, 2, 1, 1, 2, 2},
              tc[10] = {0, 1, 2, 1, 2, 2, 1, 2, 2, 2};
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        const int a = ta[k], b = tb[k], d = tc[k];
        Q[k] = M[c * 20 + 10 + k] - (u[a] * P[b][d] + u[b] * P[a][d] + u[d] * P[a][b]) +
               2.0 * m * n * u[a] * u[b] * u[d];
    }
}

__global__ void mlp_targets_kernel(const double* __restrict__ M, long long cells, double m, float* __restrict__ y) {
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    double Q[10], n, u[3], Tref;
    heat_flux_cell(M, c, m, Q, n, u, Tref);
    const bool ok = n > 1e-12 && Tref > 0.0;
    const double vt = ok ? sqrt(Tref / m) : 1.0;
    const double inv = ok ? 1.0 / (n * m * vt * vt * vt) : 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) y[c * 16 + k] = k < kOut ? (float)(Q[k < kOut ? k : 0] * inv) : 0.0f;
}

// ---------------------------------------------------------------- forward --
__global__ void __launch_bounds__(256)
mlp_forward_kernel(const float* __restrict__ P, const unsigned short* __restrict__ x, long long n,
                   float* __restrict__ y) {
    __shared__ NetLds N;
    load_net(P, N, nullptr);
    __syncthreads();
    const int lane = threadIdx.x & 63, s = lane & 15, g = lane >> 4;
    const long long tiles = (n + 15) / 16;
    const long long nw = (long long)gridDim.x * (blockDim.x / 64);
    for (long long t = (long long)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; t < tiles; t += nw) {
        Tile T;
        forward_tile(x, n, t, N, false, T);
        const long long row = t * 16 + s;
        if (row < n) *reinterpret_cast<f32x4*>(y + row * 16 + 4 * g) = T.y;
    }
}

// --------------------------------------------------------------- gradient --
// Block b handles tiles [t0, t1).  Every wave of the block runs the forward
// pass and as much of the backward pass as its layer needs; wave w
// accumulates the gradient of layer w+1 (weights in MFMA accumulators,
// biases per lane) over the block's tiles, so each block writes one partial
// gradient and no floating-point atomics are used (the sum over blocks is
// done in a fixed order).
__global__ void __launch_bounds__(256)
mlp_grad_kernel(const float* __restrict__ P, const unsigned short* __restrict__ x, const float* __restrict__ t,
                long long n, long long tiles_per_block, float inv_norm, float* __restrict__ part,
                const long long* __restrict__ idx, long long nrows) {
    __shared__ NetLds N;
    __shared__ NetLdsT NT;
    __shared__ unsigned short stage_all[4][5][16 * kLds];
    load_net(P, N, &NT);
    __syncthreads();
    const int w = threadIdx.x / 64, lane = threadIdx.x & 63, s = lane & 15, g = lane >> 4;
    unsigned short(*stage)[16 * kLds] = stage_all[w];
    const long long tiles = (n + 15) / 16;
    const long long t0 = (long long)blockIdx.x * tiles_per_block;
    const long long t1 = t0 + tiles_per_block < tiles ? t0 + tiles_per_block : tiles;
    f32x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    f32x4 db[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) db[a] = f32x4{0.f, 0.f, 0.f, 0.f};
    float lsum = 0.f;
    // software pipeline: the features and targets of the next tile and the
    // source row of the one after are loaded while this tile is computed
    long long r1 = t0 < t1 ? source_row(t0 * 16 + s, n, idx, nrows) : -1;
    uint2 xv[4];
    f32x4 tv = {0.f, 0.f, 0.f, 0.f};
    load_features(x, r1, xv);
    if (r1 >= 0) tv = *reinterpret_cast<const f32x4*>(t + r1 * 16 + 4 * g);
    long long r2 = t0 + 1 < t1 ? source_row((t0 + 1) * 16 + s, n, idx, nrows) : -1;
    for (long long tile = t0; tile < t1; ++tile) {
        const long long row = r1;
        uint2 xc[4];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) xc[kb] = xv[kb];
        const f32x4 tt = tv;
        r1 = r2;
        load_features(x, r1, xv);
        if (r1 >= 0) tv = *reinterpret_cast<const f32x4*>(t + r1 * 16 + 4 * g);
        r2 = tile + 2 < t1 ? source_row((tile + 2) * 16 + s, n, idx, nrows) : -1;
        Tile T;
        forward_from(xc, N, true, T);
        f32x4 dy = {0.f, 0.f, 0.f, 0.f};
        if (row >= 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float d = (4 * g + j < kOut) ? T.y[j] - tt[j] : 0.f;
                lsum += d * d;
                dy[j] = 2.f * d * inv_norm;
            }
        }
        if (w == 3) {
            // dW4 = dY H3^T, db4 = sum dY
            const bf16x4 a = transpose_tile(stage[0], dy);
#pragma unroll
            for (int ib = 0; ib < 4; ++ib) acc[0][ib] = mfma16(a, transpose_tile(stage[1], T.hb[3][ib]), acc[0][ib]);
#pragma unroll
            for (int j = 0; j < 4; ++j) db[0][j] += dy[j];
            continue;
        }
        // dA3 = (W4^T dY) * (1 - h3^2)
        const bf16x4 dyb = pack4(dy);
        f32x4 dA[4];
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
            const f32x4 d = mfma16(lds4(NT.wt4 + (16 * ib + s) * kLdt4 + 4 * g), dyb, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
            for (int j = 0; j < 4; ++j) dA[ib][j] = d[j] * (1.f - T.h[2][ib][j] * T.h[2][ib][j]);
        }
        // layers 3, 2, 1: wave w = layer - 1 stops at its own layer
#pragma unroll
        for (int L = 2; L >= 0; --L) {
            if (w == L) {
                bf16x4 hT[4];
#pragma unroll
                for (int ib = 0; ib < 4; ++ib) hT[ib] = transpose_tile(stage[1 + ib], T.hb[L][ib]);
#pragma unroll
                for (int ob = 0; ob < 4; ++ob) {
                    const bf16x4 a = transpose_tile(stage[0], dA[ob]);
#pragma unroll
                    for (int ib = 0; ib < 4; ++ib) acc[ob][ib] = mfma16(a, hT[ib], acc[ob][ib]);
#pragma unroll
                    for (int j = 0; j < 4; ++j) db[ob][j] += dA[ob][j];
                }
                break;
            }
            if (L == 0) break;
            // gradient of the pre-activation of layer L (1-based): (W_{L+1}^T dA) * (1 - h_L^2)
            bf16x4 dAb[4];
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) dAb[kb] = pack4(dA[kb]);
            const unsigned short* WT = NT.wt[L - 1];
#pragma unroll
            for (int ib = 0; ib < 4; ++ib) {
                f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < 4; ++kb) d = mfma16(lds4(WT + (16 * ib + s) * kLdw + 16 * kb + 4 * g), dAb[kb], d);
#pragma unroll
                for (int j = 0; j < 4; ++j) dA[ib][j] = d[j] * (1.f - T.h[L - 1][ib][j] * T.h[L - 1][ib][j]);
            }
        }
    }
    // write this block's partial gradient of layer w+1
    float* out = part + (long long)blockIdx.x * kPartStride;
    if (w == 3) {
#pragma unroll
        for (int ib = 0; ib < 4; ++ib)
#pragma unroll
            for (int j = 0; j < 4; ++j) out[kOffW4 + (4 * g + j) * kWid + 16 * ib + s] = acc[0][ib][j];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float v = sum16(db[0][j]);
            if (s == 0) out[kOffB4 + 4 * g + j] = v;
        }
    } else {
        const int offW = w == 0 ? kOffW1 : (w == 1 ? kOffW2 : kOffW3);
        const int offB = w == 0 ? kOffB1 : (w == 1 ? kOffB2 : kOffB3);
#pragma unroll
        for (int ob = 0; ob < 4; ++ob)
#pragma unroll
            for (int ib = 0; ib < 4; ++ib)
#pragma unroll
                for (int j = 0; j < 4; ++j) out[offW + (16 * ob + 4 * g + j) * kWid + 16 * ib + s] = acc[ob][ib][j];
#pragma unroll
        for (int ob = 0; ob < 4; ++ob)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float v = sum16(db[ob][j]);
                if (s == 0) out[offB + 16 * ob + 4 * g + j] = v;
            }
    }
    if (w == 0) {
        float v = lsum;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) out[kNParam] = v * inv_norm;
    }
}

// One Adam update (optional, after the gradient sum).
struct AdamArgs {
    float* P;          // null: no update
    float* m1;
    float* m2;
    float lr, beta1, beta2, eps, bc1, bc2;
};

__device__ __forceinline__ void adam_update(const AdamArgs& A, int p, float gr) {
    const float a = A.beta1 * A.m1[p] + (1.f - A.beta1) * gr;
    const float b = A.beta2 * A.m2[p] + (1.f - A.beta2) * gr * gr;
    A.m1[p] = a;
    A.m2[p] = b;
    A.P[p] -= A.lr * (a / A.bc1) / (sqrtf(b / A.bc2) + A.eps);
}

// Sum of the block partials: grad[0..13519], loss at [13520].  Block i
// covers entries 64i..64i+63; wave q adds partials q, q+4, q+8, ..., sixteen
// loads in flight at a time, into four running sums, and the four waves'
// totals are added in wave order: a fixed order, the same on every call.
// With A.P set, the Adam update of the same entries follows.
__global__ void __launch_bounds__(256)
mlp_reduce_kernel(const float* __restrict__ part, int nblocks, float* __restrict__ grad, AdamArgs A) {
    __shared__ float red[4][64];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + lane;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    if (p <= kNParam) {
        const float* __restrict__ src = part + p;
        int b = q;
        for (; b + 60 < nblocks; b += 64) {
            float v[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = src[(long long)(b + 4 * k) * kPartStride];
#pragma unroll
            for (int k = 0; k < 16; ++k) acc[k & 3] += v[k];
        }
        for (; b < nblocks; b += 4) acc[0] += src[(long long)b * kPartStride];
    }
    red[q][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    if (q != 0 || p > kNParam) return;
    const float gr = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    grad[p] = gr;
    if (A.P && p < kNParam) adam_update(A, p, gr);
}

// --------------------------------------------------- closure in the fluid --
// Third moment of every cell for one RK stage: the network's heat flux
// (scale * y) turned into Q-calligraphic = Q + sym(u P) - 2 m n uuu, written
// at [c*20 + 10 + k] (the raw-moment layout the flux kernels read); or, when
// *fallback is set, the kinetic wa*QA + wb*QB.
// Species blockIdx.y of the set; scale, y and qc hold the set's species one
// after the other.
__global__ void mlp_qcal_kernel(MlpSet S, const double* __restrict__ scale, const float* __restrict__ y, double wa,
                                double wb, long long cells, double* __restrict__ qc) {
    const int sp = blockIdx.y;
    const double* __restrict__ U = S.U[sp];
    const int* __restrict__ fallback = S.fallback[sp];
    const double* __restrict__ QA = S.QA[sp];
    const double* __restrict__ QB = S.QB[sp];
    const double m = S.m[sp];
    scale += (size_t)sp * cells;
    y += (size_t)sp * cells * kOutPad;
    qc += (size_t)sp * cells * 20;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    if (fallback && *fallback) {
#pragma unroll
        for (int k = 0; k < 10; ++k)
            qc[c * 20 + 10 + k] = wa * QA[c * 20 + 10 + k] + (wb != 0.0 ? wb * QB[c * 20 + 10 + k] : 0.0);
        return;
    }
    const double n = U[c * 10];
    const double u[3] = {U[c * 10 + 1] / n, U[c * 10 + 2] / n, U[c * 10 + 3] / n};
    double P[3][3];
    const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 0; k < 6; ++k) P[pa[k]][pb[k]] = P[pb[k]][pa[k]] = U[c * 10 + 4 + k];
    const int ta[10] = {0, 0, 0, 0, 0, 0, 1, 1, 1, 2}, tb[10] = {0, 0, 0, 1, 1, 2, 1, 1, 2, 2},
              tc[10] = {0, 1, 2, 1, 2, 2, 1, 2, 2, 2};
    const double sc = scale[c];
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        const int a = ta[k], b = tb[k], d = tc[k];
        qc[c * 20 + 10 + k] = sc * (double)y[c * 16 + k] + (u[a] * P[b][d] + u[b] * P[a][d] + u[d] * P[a][b]) -
                              2.0 * m * n * u[a] * u[b] * u[d];
    }
}

// Judge: sums over cells of |q_net - q_kin|^2 and |q_kin|^2 (q_i = Q_ijj),
// per block in a fixed order.
__global__ void __launch_bounds__(256)
mlp_judge_partial_kernel(MlpSet S, const double* __restrict__ scale, const float* __restrict__ y, long long cells,
                         double* __restrict__ part) {
    const int sp = blockIdx.y;
    const double* __restrict__ M = S.M[sp];
    const double m = S.m[sp];
    scale += (size_t)sp * cells;
    y += (size_t)sp * cells * kOutPad;
    part += (size_t)sp * 2 * gridDim.x;
    __shared__ double red[2 * 4];
    double e2 = 0.0, k2 = 0.0;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < cells;
         c += (long long)gridDim.x * blockDim.x) {
        double Q[10], n, u[3], Tref;
        heat_flux_cell(M, c, m, Q, n, u, Tref);
        const double qk[3] = {Q[0] + Q[3] + Q[5], Q[1] + Q[6] + Q[8], Q[2] + Q[7] + Q[9]};
        const double sc = scale[c];
        const float* yc = y + c * 16;
        const double qn[3] = {sc * ((double)yc[0] + (double)yc[3] + (double)yc[5]),
                              sc * ((double)yc[1] + (double)yc[6] + (double)yc[8]),
                              sc * ((double)yc[2] + (double)yc[7] + (double)yc[9])};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            e2 += (qn[d] - qk[d]) * (qn[d] - qk[d]);
            k2 += qk[d] * qk[d];
        }
    }
    double v[2] = {e2, k2};
    block_sum<2>(v, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 2] = v[0];
        part[blockIdx.x * 2 + 1] = v[1];
    }
}

// One wave per species: lane l adds partials l, l + 64, ... (the loads of
// all lanes in flight together), then a butterfly over the wave: a fixed
// order of additions on every call.
__global__ void __launch_bounds__(64)
mlp_judge_finish_kernel(MlpSet S, const double* __restrict__ part, int nblocks, double tol) {
    const int sp = blockIdx.x, lane = threadIdx.x;
    int* __restrict__ fallback = S.fallback[sp];
    double* __restrict__ err = S.err[sp];
    part += (size_t)sp * 2 * nblocks;
    double e2 = 0.0, k2 = 0.0;
    for (int b = lane; b < nblocks; b += 64) {
        e2 += part[2 * b];
        k2 += part[2 * b + 1];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        e2 += __shfl_xor(e2, o, 64);
        k2 += __shfl_xor(k2, o, 64);
    }
    if (lane != 0) return;
    const double r = sqrt(e2) / fmax(sqrt(k2), 1e-300);
    *err = r;
    *fallback = !(r <= tol);
}

// --------------------------------------------------------------- launchers --
constexpr int kJudgeBlocks = 256;

hipError_t launch_mlp_features_set(const MlpSet& S, int ns, int s0, int stride, const double* B, int nx, int ny,
                                   unsigned short* x, double* scale, hipStream_t st) {
    if (ns < 1 || ns > 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(mlp_features_kernel, dim3((nx + kFeatCols - 1) / kFeatCols, (ny + kFeatRows - 1) / kFeatRows, ns),
                       dim3(kFeatRows * kFeatCols), 0, st, S, s0, stride, B, nx, ny, x, scale);
    return hipGetLastError();
}

hipError_t launch_mlp_features(const double* M, int stride, const double* B, int nx, int ny, double m, int species,
                               unsigned short* x, double* scale, hipStream_t st) {
    MlpSet S{};
    S.M[0] = M;
    S.m[0] = m;
    return launch_mlp_features_set(S, 1, species, stride, B, nx, ny, x, scale, st);
}

hipError_t launch_mlp_targets(const double* M, long long cells, double m, float* y, hipStream_t st) {
    hipLaunchKernelGGL(mlp_targets_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st, M, cells, m, y);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* P, const unsigned short* x, long long n, float* y, hipStream_t st) {
    const long long tiles = (n + 15) / 16;
    long long blocks = (tiles + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)blocks), dim3(256), 0, st, P, x, n, y);
    return hipGetLastError();
}

// At most one gradient block per compute unit: every block stages the whole
// network in LDS first, so fewer blocks with more tiles each beat more blocks
// (16384-row batches, gradient + sum + Adam: 256 blocks 1.4x faster than 512
// and 1.25x faster than 128).
constexpr long long kGradBlocks = 256;
size_t mlp_grad_blocks(long long n) {
    const long long tiles = (n + 15) / 16;
    long long blocks = tiles < kGradBlocks ? tiles : kGradBlocks;
    return blocks < 1 ? 1 : (size_t)blocks;
}
size_t mlp_part_floats(long long n) { return mlp_grad_blocks(n) * (size_t)kPartStride; }

static AdamArgs adam_args(float* P, float* m1, float* m2, long long step, double lr) {
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    const double bc1 = 1.0 - pow(b1, (double)step), bc2 = 1.0 - pow(b2, (double)step);
    return AdamArgs{P, m1, m2, (float)lr, (float)b1, (float)b2, (float)eps, (float)bc1, (float)bc2};
}

static hipError_t grad_and_sum(const float* P, const unsigned short* x, const float* t, long long n, float* part,
                               float* grad, hipStream_t st, const long long* idx, long long nrows,
                               const AdamArgs& A) {
    const long long tiles = (n + 15) / 16;
    const long long blocks = (long long)mlp_grad_blocks(n);
    const long long tpb = (tiles + blocks - 1) / blocks;
    const float inv_norm = (float)(1.0 / ((double)n * kOut));
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((unsigned)blocks), dim3(256), 0, st, P, x, t, n, tpb, inv_norm, part,
                       idx, nrows);
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kNParam + 1 + 63) / 64), dim3(256), 0, st, part, (int)blocks, grad,
                       A);
    return hipGetLastError();
}

hipError_t launch_mlp_gradient(const float* P, const unsigned short* x, const float* t, long long n, float* part,
                               float* grad, hipStream_t st, const long long* idx, long long nrows) {
    return grad_and_sum(P, x, t, n, part, grad, st, idx, nrows, AdamArgs{});
}

hipError_t launch_mlp_train_step(float* P, float* m1, float* m2, long long step, double lr,
                                 const unsigned short* x, const float* t, long long n, float* part, float* grad,
                                 hipStream_t st, const long long* idx, long long nrows) {
    return grad_and_sum(P, x, t, n, part, grad, st, idx, nrows, adam_args(P, m1, m2, step, lr));
}

hipError_t launch_mlp_qcal_set(const MlpSet& S, int ns, const double* scale, const float* y, double wa, double wb,
                               long long cells, double* qc, hipStream_t st) {
    if (ns < 1 || ns > 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(mlp_qcal_kernel, dim3((unsigned)((cells + 255) / 256), ns), dim3(256), 0, st, S, scale, y, wa,
                       wb, cells, qc);
    return hipGetLastError();
}

hipError_t launch_mlp_qcal(const double* U, const double* scale, const float* y, const int* fallback,
                           const double* QA, const double* QB, double wa, double wb, long long cells, double m,
                           double* qc, hipStream_t st) {
    MlpSet S{};
    S.U[0] = U;
    S.fallback[0] = const_cast<int*>(fallback);
    S.QA[0] = QA;
    S.QB[0] = QB;
    S.m[0] = m;
    return launch_mlp_qcal_set(S, 1, scale, y, wa, wb, cells, qc, st);
}

size_t mlp_judge_part_doubles() { return 2 * kJudgeBlocks; }

hipError_t launch_mlp_judge_set(const MlpSet& S, int ns, const double* scale, const float* y, long long cells,
                                double tol, double* part, hipStream_t st) {
    if (ns < 1 || ns > 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(mlp_judge_partial_kernel, dim3(kJudgeBlocks, ns), dim3(256), 0, st, S, scale, y, cells, part);
    hipLaunchKernelGGL(mlp_judge_finish_kernel, dim3(ns), dim3(64), 0, st, S, part, kJudgeBlocks, tol);
    return hipGetLastError();
}

hipError_t launch_mlp_judge(const double* M, const double* scale, const float* y, long long cells, double m,
                            double tol, double* part, int* fallback, double* err, hipStream_t st) {
    MlpSet S{};
    S.M[0] = M;
    S.m[0] = m;
    S.fallback[0] = fallback;
    S.err[0] = err;
    return launch_mlp_judge_set(S, 1, scale, y, cells, tol, part, st);
}

}  // namespace vl
