// Field solvers for gfx950, all FP64 (the field update is kept in double
// precision because the energy exchange with the particles depends on it).
//
// 1X1V (Sec. 3.1): Gauss's law dE/dx = rho with eps0 = 1 and a uniform static
// ion background, solved with a direct discrete Fourier transform (the grid
// is small): E_i = (2/N) sum_{m=1}^{N/2-1} Im(rho_hat_m e^{i th}) / k_m, the mean
// and Nyquist modes dropped.
//
// 2X3V (Sec. 2.1, Maxwell's equations, FDTD): Yee grid, mu0 = 1, eps0 = 1/c^2,
// x periodic, conducting walls in y with the tangential E (Ex, Ez) and normal
// B (By) odd about each wall.  A half step of length h = dt/2 is
//   B -= (h/2) curl E;  E += h c^2 (curl B - j);  B -= (h/2) curl E.
#include "vl_internal.h"

namespace vl {

// --------------------------------------------------------------- Poisson ---
__global__ void dft_rho_kernel(const double* __restrict__ mom, int N, double q, double* __restrict__ ab) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x + 1;    // 1 .. N/2-1
    if (m >= (N + 1) / 2) return;
    double a = 0.0, b = 0.0;
    for (int i = 0; i < N; ++i) {
        const double rho = q * mom[(long long)i * 4];
        double s, c;
        sincospi(2.0 * (double)(((long long)m * i) % N) / N, &s, &c);
        a += rho * c;
        b -= rho * s;
    }
    ab[2 * m] = a;
    ab[2 * m + 1] = b;
}

__global__ void dft_field_kernel(const double* __restrict__ ab, int N, double L, double* __restrict__ E) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double acc = 0.0;
    for (int m = 1; m < (N + 1) / 2; ++m) {
        double s, c;
        sincospi(2.0 * (double)(((long long)m * i) % N) / N, &s, &c);
        const double k = 2.0 * M_PI * m / L;
        acc += (ab[2 * m] * s + ab[2 * m + 1] * c) / k;
    }
    E[i] = 2.0 * acc / N;
}

hipError_t launch_poisson(const double* mom, int N, double L, double q, double* ab, double* E, hipStream_t st) {
    const int nm = (N + 1) / 2 - 1;
    if (nm > 0) hipLaunchKernelGGL(dft_rho_kernel, dim3((nm + 63) / 64), dim3(64), 0, st, mom, N, q, ab);
    hipLaunchKernelGGL(dft_field_kernel, dim3((N + 63) / 64), dim3(64), 0, st, ab, N, L, E);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Yee ----
struct YeeView {
    double *Ex, *Ey, *Ez, *Bx, *By, *Bz;
    int nx, ny;
    int per;    // 1: periodic y (rows 0 and ny of the [ny+1] arrays are the same points)
};

__host__ __device__ inline YeeView yee_view(double* base, int nx, int ny) {
    const long long a = (long long)nx * ny, b = (long long)nx * (ny + 1);
    YeeView v;
    v.Ex = base;
    v.Ey = v.Ex + a;
    v.Ez = v.Ey + b;
    v.Bx = v.Ez + a;
    v.By = v.Bx + b;
    v.Bz = v.By + a;
    v.nx = nx;
    v.ny = ny;
    v.per = 0;
    return v;
}

// integer-row component (Ex, Ez) at row j: odd ghosts beyond conducting
// walls, wrapped rows when y is periodic
__device__ __forceinline__ double odd_row(const double* a, int j, int i, int nx, int ny, int per) {
    if (per) {
        if (j < 0) j += ny;
        if (j >= ny) j -= ny;
        return a[(long long)j * nx + i];
    }
    if (j < 0) return -a[(long long)(-1 - j) * nx + i];
    if (j >= ny) return -a[(long long)(2 * ny - 1 - j) * nx + i];
    return a[(long long)j * nx + i];
}

// B -= coef * curl E.  One thread per (jh in 0..ny, i).
__global__ void yee_curl_e_kernel(YeeView F, double coef, double dx, double dy) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int jh = blockIdx.y;
    const int nx = F.nx, ny = F.ny;
    if (i >= nx) return;
    const int ip = (i + 1 == nx) ? 0 : i + 1;
    const long long h = (long long)jh * nx;
    // Bx at (i, jh-1/2): (curl E)_x = dEz/dy
    const double dEz = (odd_row(F.Ez, jh, i, nx, ny, F.per) - odd_row(F.Ez, jh - 1, i, nx, ny, F.per)) / dy;
    F.Bx[h + i] -= coef * dEz;
    // Bz at (i+1/2, jh-1/2): (curl E)_z = dEy/dx - dEx/dy
    const double dEy = (F.Ey[h + ip] - F.Ey[h + i]) / dx;
    const double dEx = (odd_row(F.Ex, jh, i, nx, ny, F.per) - odd_row(F.Ex, jh - 1, i, nx, ny, F.per)) / dy;
    F.Bz[h + i] -= coef * (dEy - dEx);
    // By at (i+1/2, j): (curl E)_y = -dEz/dx
    if (jh < ny) F.By[h + i] += coef * (F.Ez[h + ip] - F.Ez[h + i]) / dx;
}

// E += coef c^2 (curl B - j); j = sum_s q_s M1_s at cell centres averaged to
// the E positions (j_y on a wall face is 0; periodic y: the mean across the
// seam).
struct Currents {
    const double* mom[2];   // per species: n u_x, n u_y, n u_z at offsets 1..3 of each cell's record
    double q[2];
    int ns;
    int stride;             // doubles per cell record (20: raw moments, 10: fluid state)
};

__device__ __forceinline__ double jc(const Currents& J, long long cell, int d) {
    double s = 0.0;
    for (int k = 0; k < J.ns; ++k) s += J.q[k] * J.mom[k][cell * J.stride + 1 + d];
    return s;
}

__global__ void yee_curl_b_kernel(YeeView F, Currents J, double coef, double c2, double dx, double dy) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int jh = blockIdx.y;
    const int nx = F.nx, ny = F.ny;
    if (i >= nx) return;
    const int im = (i == 0) ? nx - 1 : i - 1;
    const int ip = (i + 1 == nx) ? 0 : i + 1;
    const long long h = (long long)jh * nx;
    // Ey at (i, jh-1/2): (curl B)_y = -dBz/dx
    double jy = 0.0;
    if (jh > 0 && jh < ny) jy = 0.5 * (jc(J, h - nx + i, 1) + jc(J, h + i, 1));
    else if (F.per) jy = 0.5 * (jc(J, (long long)(ny - 1) * nx + i, 1) + jc(J, i, 1));   // across the seam
    F.Ey[h + i] += coef * c2 * (-(F.Bz[h + i] - F.Bz[h + im]) / dx - jy);
    if (jh < ny) {
        // Ex at (i+1/2, j): (curl B)_x = dBz/dy
        const double jx = 0.5 * (jc(J, h + i, 0) + jc(J, h + ip, 0));
        F.Ex[h + i] += coef * c2 * ((F.Bz[h + nx + i] - F.Bz[h + i]) / dy - jx);
        // Ez at (i, j): (curl B)_z = dBy/dx - dBx/dy
        const double jz = jc(J, h + i, 2);
        F.Ez[h + i] += coef * c2 * ((F.By[h + i] - F.By[h + im]) / dx - (F.Bx[h + nx + i] - F.Bx[h + i]) / dy - jz);
    }
}

__global__ void cell_fields_kernel(YeeView F, double* __restrict__ E, double* __restrict__ B) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    const int nx = F.nx;
    if (i >= nx) return;
    const int im = (i == 0) ? nx - 1 : i - 1;
    const long long r = (long long)j * nx, rn = r + nx;
    const long long c = r + i;
    E[c * 3 + 0] = 0.5 * (F.Ex[r + im] + F.Ex[r + i]);
    E[c * 3 + 1] = 0.5 * (F.Ey[r + i] + F.Ey[rn + i]);
    E[c * 3 + 2] = F.Ez[r + i];
    B[c * 3 + 0] = 0.5 * (F.Bx[r + i] + F.Bx[rn + i]);
    B[c * 3 + 1] = 0.5 * (F.By[r + im] + F.By[r + i]);
    const double lo = 0.5 * (F.Bz[r + im] + F.Bz[r + i]);
    const double hi = 0.5 * (F.Bz[rn + im] + F.Bz[rn + i]);
    B[c * 3 + 2] = 0.5 * (lo + hi);
}

__global__ void axpby_kernel(const double* __restrict__ x, const double* __restrict__ y, double a, double b,
                             double* __restrict__ out, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a * x[i] + b * y[i];
}

// The B-curl kernel reads the current from the species' moment records (8-byte
// lanes 80 or 160 bytes apart, several records per lane): dynamic LDS that it
// does not use caps it at eight one-wave blocks per CU (two waves per SIMD),
// so fewer waves evict the lines those loads share.  2048 x 1024 cells: the
// three half-step kernels 0.74 -> 0.50 ms per fluid-only step (one wave per
// SIMD 0.63, three 0.49, four 0.66).
constexpr unsigned kCurlBLdsCap = 20480;

hipError_t launch_maxwell_half(double* yee, int nx, int ny, const double* const* mom, const double* q, int ns,
                               double dt, double c, double dx, double dy, hipStream_t st, int mstride, int per) {
    YeeView F = yee_view(yee, nx, ny);
    F.per = per;
    Currents J;
    J.ns = ns;
    J.stride = mstride;
    for (int k = 0; k < 2; ++k) {
        J.mom[k] = k < ns ? mom[k] : nullptr;
        J.q[k] = k < ns ? q[k] : 0.0;
    }
    const double h = 0.5 * dt;
    dim3 blk(64), grid((nx + 63) / 64, ny + 1);
    hipLaunchKernelGGL(yee_curl_e_kernel, grid, blk, 0, st, F, 0.5 * h, dx, dy);
    hipLaunchKernelGGL(yee_curl_b_kernel, grid, blk, kCurlBLdsCap, st, F, J, h, c * c, dx, dy);
    hipLaunchKernelGGL(yee_curl_e_kernel, grid, blk, 0, st, F, 0.5 * h, dx, dy);
    return hipGetLastError();
}

hipError_t launch_cell_fields(const double* yee, int nx, int ny, double* E, double* B, hipStream_t st) {
    YeeView F = yee_view(const_cast<double*>(yee), nx, ny);
    hipLaunchKernelGGL(cell_fields_kernel, dim3((nx + 63) / 64, ny), dim3(64), 0, st, F, E, B);
    return hipGetLastError();
}

hipError_t launch_axpby(const double* x, const double* y, double a, double b, double* out, long long n,
                        hipStream_t st) {
    hipLaunchKernelGGL(axpby_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, y, a, b, out, n);
    return hipGetLastError();
}

// Field energy, deterministic: block partials over the rows jh = 0..ny (one
// block column per row, fixed order), then one block adds them.
// 2X3V: sum of B^2/2 + E^2/(2 c^2) over the Yee points, wall rows of the
// [ny+1] arrays (Ey, Bx, Bz) at half weight; 1X1V: sum of E^2/2.
__global__ void __launch_bounds__(256)
field_energy_rows_kernel(YeeView F, double inv_c2, double* __restrict__ part) {
    __shared__ double red[4];
    const int jh = blockIdx.x;
    const int nx = F.nx, ny = F.ny;
    double acc[1] = {0.0};
    const double w = (jh == 0 || jh == ny) ? 0.5 : 1.0;
    const long long h = (long long)jh * nx;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        double e = w * (F.Bx[h + i] * F.Bx[h + i] + F.Bz[h + i] * F.Bz[h + i] + inv_c2 * F.Ey[h + i] * F.Ey[h + i]);
        if (jh < ny) e += F.By[h + i] * F.By[h + i] + inv_c2 * (F.Ex[h + i] * F.Ex[h + i] + F.Ez[h + i] * F.Ez[h + i]);
        acc[0] += 0.5 * e;
    }
    block_sum<1>(acc, red);
    if (threadIdx.x == 0) part[jh] = acc[0];
}

__global__ void __launch_bounds__(256)
line_energy_kernel(const double* __restrict__ E, int n, double* __restrict__ part) {
    __shared__ double red[4];
    double acc[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc[0] += 0.5 * E[i] * E[i];
    block_sum<1>(acc, red);
    if (threadIdx.x == 0) part[0] = acc[0];
}

__global__ void __launch_bounds__(256)
ordered_sum_kernel(const double* __restrict__ part, int np, double scale, double* __restrict__ out) {
    __shared__ double red[4];
    // thread t adds partials t, t+256, ... in order; then a fixed-order block sum
    double acc[1] = {0.0};
    for (int i = threadIdx.x; i < np; i += blockDim.x) acc[0] += part[i];
    block_sum<1>(acc, red);
    if (threadIdx.x == 0) *out = acc[0] * scale;
}

hipError_t launch_field_energy(const double* fields, int dim_x, int nx, int ny, double c, double dX, double* part,
                               double* out, hipStream_t st) {
    if (dim_x == 2) {
        const YeeView F = yee_view(const_cast<double*>(fields), nx, ny);
        hipLaunchKernelGGL(field_energy_rows_kernel, dim3(ny + 1), dim3(256), 0, st, F, 1.0 / (c * c), part);
        hipLaunchKernelGGL(ordered_sum_kernel, dim3(1), dim3(256), 0, st, part, ny + 1, dX, out);
    } else {
        hipLaunchKernelGGL(line_energy_kernel, dim3(1), dim3(256), 0, st, fields, nx, part);
        hipLaunchKernelGGL(ordered_sum_kernel, dim3(1), dim3(256), 0, st, part, 1, dX, out);
    }
    return hipGetLastError();
}

}  // namespace vl
