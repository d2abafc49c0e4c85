// Ten-moment fluid step for gfx950 (FP64): Eqs. 2-4 of arXiv 2109.06743 with
// the flux of the second moment P given by the third moment Qcal taken from f
// (Algorithm 1).  Semi-discrete finite volumes: CWENO-3 (Kurganov-Levy)
// point values at the faces, local Lax-Friedrichs flux with speed
// |u_d| + sqrt(3 p_dd / (m n)), and SSP-RK3 (Shu-Osher) in time.
//
// Face fluxes are computed once per face (both directions in one launch, one
// thread per face and component), then a per-cell kernel forms
// L(U) = -div H + S(U, E, B) and the RK stage combination
// U_out = a U_n + b (U_s + dt L).
//
// Component orders: U = (n, nu_x, nu_y, nu_z, Pxx, Pxy, Pxz, Pyy, Pyz, Pzz);
// Qcal (from the raw moment vector, offset 10) = (xxx, xxy, xxz, xyy, xyz,
// xzz, yyy, yyz, yzz, zzz).  1V: U = (n, nu, P), Qcal = raw moment 3.
#include "vl_internal.h"

namespace vl {

constexpr double kCwenoEps = 1e-6;

// CWENO-3 point values of cell j at its left (x_j - h/2) and right (x_j + h/2)
// faces from the averages a = u_{j-1}, b = u_j, c = u_{j+1}.  The left, right
// and centred polynomials evaluated at +-h/2 are
//   P_L = b -+ (b - a)/2,  P_R = b -+ (c - b)/2,  P_C = b + d2/6 -+ (c - a)/4,
// d2 = c - 2b + a, weighted with (1/4, 1/2, 1/4) / (eps + IS)^2, normalised.
__device__ __forceinline__ void cweno(double a, double b, double c, double& left, double& right) {
    const double dl = b - a, dr = c - b, d2 = c - 2.0 * b + a, dc = c - a;
    const double isl = dl * dl, isr = dr * dr, isc = (13.0 / 3.0) * d2 * d2 + 0.25 * dc * dc;
    const double al = 0.25 / ((kCwenoEps + isl) * (kCwenoEps + isl));
    const double ac = 0.5 / ((kCwenoEps + isc) * (kCwenoEps + isc));
    const double ar = 0.25 / ((kCwenoEps + isr) * (kCwenoEps + isr));
    const double inv = 1.0 / (al + ac + ar);
    const double wl = al * inv, wc = ac * inv, wr = ar * inv;
    const double cen = b + d2 / 6.0;
    right = wl * (b + 0.5 * dl) + wc * (cen + 0.25 * dc) + wr * (b + 0.5 * dr);
    left = wl * (b - 0.5 * dl) + wc * (cen - 0.25 * dc) + wr * (b - 0.5 * dr);
}

// index helpers for the symmetric second and third moments
__device__ __forceinline__ int p_index(int a, int b) {
    if (a > b) { int t = a; a = b; b = t; }
    return a == 0 ? b : (a == 1 ? 2 + b : 5);
}
__device__ __forceinline__ int q_index(int a, int b, int c) {
    // sort a <= b <= c
    if (a > b) { int t = a; a = b; b = t; }
    if (b > c) { int t = b; b = c; c = t; }
    if (a > b) { int t = a; a = b; b = t; }
    // (0,0,0)0 (0,0,1)1 (0,0,2)2 (0,1,1)3 (0,1,2)4 (0,2,2)5 (1,1,1)6 (1,1,2)7 (1,2,2)8 (2,2,2)9
    if (a == 0) {
        if (b == 0) return c;
        if (b == 1) return 2 + c;
        return 5;
    }
    if (a == 1) return b == 1 ? 5 + c : 8;
    return 9;
}

// y-parity (+1/-1) of U and Qcal components under y -> -y
__device__ __forceinline__ double par_u(int k) {
    return (k == 2 || k == 5 || k == 8) ? -1.0 : 1.0;       // nu_y, Pxy, Pyz
}
__device__ __forceinline__ double par_q(int k) {
    return (k == 1 || k == 4 || k == 6 || k == 8) ? -1.0 : 1.0;  // xxy, xyz, yyy, yzz
}

struct FluidArgs {
    int nx, ny;
    double m, q;
    double dx, dy;
};

__device__ __forceinline__ double speed3(const double* U, int d, double m) {
    const double n = U[0];
    const double u = U[1 + d] / n;
    const double p = U[4 + p_index(d, d)] - m * n * u * u;
    return fabs(u) + sqrt(fmax(3.0 * p / (m * n), 0.0));
}

// Both face directions in one launch, one thread per (face, component): a
// block takes kFaceTile consecutive faces of one row (x faces i+1/2 of row j,
// or y faces jh-1/2 at columns i), reconstructs the 20 components (U and
// Qcal) at both sides of each face into shared memory, then forms the 10
// flux components.  Blocks [0, nbx) are x faces, the rest y faces.
constexpr int kFaceTile = 32;

__device__ __forceinline__ double load_comp(const double* U, const double* QA, const double* QB, double wa,
                                            double wb, int j, int i, int k, const FluidArgs& A) {
    bool mir = false;
    if (j < 0) { j = -1 - j; mir = true; }
    if (j >= A.ny) { j = 2 * A.ny - 1 - j; mir = true; }
    i = (i % A.nx + A.nx) % A.nx;
    const long long c = (long long)j * A.nx + i;
    double v;
    if (k < 10) {
        v = U[c * 10 + k];
        if (mir) v *= par_u(k);
    } else {
        v = wa * QA[c * 20 + k] + (wb != 0.0 ? wb * QB[c * 20 + k] : 0.0);
        if (mir) v *= par_q(k - 10);
    }
    return v;
}

__global__ void __launch_bounds__(kFaceTile * 20)
faces3_kernel(const double* __restrict__ U, const double* __restrict__ QA, const double* __restrict__ QB, double wa,
              double wb, FluidArgs A, int nbx_row, int nbx, double* __restrict__ Hx, double* __restrict__ Hy) {
    __shared__ double Lm[kFaceTile][20], Lp[kFaceTile][20];   // minus (left/below) and plus sides
    const bool yface = (int)blockIdx.x >= nbx;
    const int b = yface ? (int)blockIdx.x - nbx : (int)blockIdx.x;
    const int row = b / nbx_row;                   // j for x faces, jh for y faces
    const int i0 = (b % nbx_row) * kFaceTile;
    const int f = threadIdx.x % kFaceTile, k = threadIdx.x / kFaceTile;
    const int i = i0 + f;
    if (i < A.nx) {
        double c0, c1, c2, c3;
        if (!yface) {
            c0 = load_comp(U, QA, QB, wa, wb, row, i - 1, k, A);
            c1 = load_comp(U, QA, QB, wa, wb, row, i, k, A);
            c2 = load_comp(U, QA, QB, wa, wb, row, i + 1, k, A);
            c3 = load_comp(U, QA, QB, wa, wb, row, i + 2, k, A);
        } else {
            c0 = load_comp(U, QA, QB, wa, wb, row - 2, i, k, A);
            c1 = load_comp(U, QA, QB, wa, wb, row - 1, i, k, A);
            c2 = load_comp(U, QA, QB, wa, wb, row, i, k, A);
            c3 = load_comp(U, QA, QB, wa, wb, row + 1, i, k, A);
        }
        double l1, r1, l2, r2;
        cweno(c0, c1, c2, l1, r1);   // cell below/left of the face: its upper face value
        cweno(c1, c2, c3, l2, r2);   // cell above/right: its lower face value
        Lm[f][k] = r1;
        Lp[f][k] = l2;
    }
    __syncthreads();
    if (k >= 10 || i >= A.nx) return;
    const int d = yface ? 1 : 0;
    const double a = fmax(speed3(Lm[f], d, A.m), speed3(Lp[f], d, A.m));
    // flux component k: n -> nu_d, nu_i -> P_id / m, P_ab -> Qcal_abd
    int src;
    double sc = 1.0;
    if (k == 0) {
        src = 1 + d;
    } else if (k < 4) {
        src = 4 + p_index(k - 1, d);
        sc = 1.0 / A.m;
    } else {
        const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
        src = 10 + q_index(ia[k - 4], ib[k - 4], d);
    }
    const double Fm = Lm[f][src] * sc, Fp = Lp[f][src] * sc;
    double* H = yface ? Hy : Hx;
    H[((long long)row * A.nx + i) * 10 + k] = 0.5 * (Fp + Fm) - 0.5 * a * (Lp[f][k] - Lm[f][k]);
}

// U_out = a U_n + b (U_s + dt L(U_s)); U_out may alias U_n (each cell reads
// only its own U_n entry) but not U_s.
__global__ void update3_kernel(const double* __restrict__ Us, const double* Un, double* Uout,
                               const double* __restrict__ Hx, const double* __restrict__ Hy,
                               const double* __restrict__ E, const double* __restrict__ B, double a, double b,
                               double dt, FluidArgs A) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= A.nx) return;
    const int im = (i == 0) ? A.nx - 1 : i - 1;
    const long long c = (long long)j * A.nx + i;
    double u[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) u[k] = Us[c * 10 + k];
    const double ex = E[c * 3], ey = E[c * 3 + 1], ez = E[c * 3 + 2];
    const double bx = B[c * 3], by = B[c * 3 + 1], bz = B[c * 3 + 2];
    const double qm = A.q / A.m;
    double L[10];
    // sources: momentum (q/m)(n E + nu x B)
    L[0] = 0.0;
    L[1] = qm * (u[0] * ex + u[2] * bz - u[3] * by);
    L[2] = qm * (u[0] * ey + u[3] * bx - u[1] * bz);
    L[3] = qm * (u[0] * ez + u[1] * by - u[2] * bx);
    // second moment: q (nu_i E_j + nu_j E_i) + (q/m)(eps_jkl P_ik B_l + eps_ikl P_jk B_l)
    double P[3][3];
    P[0][0] = u[4]; P[0][1] = P[1][0] = u[5]; P[0][2] = P[2][0] = u[6];
    P[1][1] = u[7]; P[1][2] = P[2][1] = u[8]; P[2][2] = u[9];
    const double Ev[3] = {ex, ey, ez}, Bv[3] = {bx, by, bz}, nu[3] = {u[1], u[2], u[3]};
    // (P x B)_{ij} = eps_jkl P_ik B_l: row i of P crossed with B
    double PxB[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        PxB[r][0] = P[r][1] * Bv[2] - P[r][2] * Bv[1];
        PxB[r][1] = P[r][2] * Bv[0] - P[r][0] * Bv[2];
        PxB[r][2] = P[r][0] * Bv[1] - P[r][1] * Bv[0];
    }
    const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int p = ia[k], r = ib[k];
        L[4 + k] = A.q * (nu[p] * Ev[r] + nu[r] * Ev[p]) + qm * (PxB[p][r] + PxB[r][p]);
    }
    const double* hxr = Hx + c * 10;
    const double* hxl = Hx + ((long long)j * A.nx + im) * 10;
    const double* hyt = Hy + ((long long)(j + 1) * A.nx + i) * 10;
    const double* hyb = Hy + ((long long)j * A.nx + i) * 10;
#pragma unroll
    for (int k = 0; k < 10; ++k) L[k] -= (hxr[k] - hxl[k]) / A.dx + (hyt[k] - hyb[k]) / A.dy;
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        const double s = u[k] + dt * L[k];
        Uout[c * 10 + k] = (a != 0.0 ? a * Un[c * 10 + k] : 0.0) + b * s;
    }
}

// ------------------------------------------------------------------- 1V ----
__global__ void flux_x1_kernel(const double* __restrict__ U, const double* __restrict__ QA,
                               const double* __restrict__ QB, double wa, double wb, int nx, double m,
                               double* __restrict__ Hx) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nx) return;
    double c[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int ii = ((i - 1 + t) % nx + nx) % nx;
#pragma unroll
        for (int k = 0; k < 3; ++k) c[t][k] = U[(long long)ii * 3 + k];
        c[t][3] = wa * QA[(long long)ii * 4 + 3] + (wb != 0.0 ? wb * QB[(long long)ii * 4 + 3] : 0.0);
    }
    double Um[4], Up[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double l1, r1, l2, r2;
        cweno(c[0][k], c[1][k], c[2][k], l1, r1);
        cweno(c[1][k], c[2][k], c[3][k], l2, r2);
        Um[k] = r1;
        Up[k] = l2;
    }
    auto spd = [m](const double* V) {
        const double u = V[1] / V[0];
        const double p = V[2] - m * V[0] * u * u;
        return fabs(u) + sqrt(fmax(3.0 * p / (m * V[0]), 0.0));
    };
    const double a = fmax(spd(Um), spd(Up));
    const double Fm[3] = {Um[1], Um[2] / m, Um[3]}, Fp[3] = {Up[1], Up[2] / m, Up[3]};
#pragma unroll
    for (int k = 0; k < 3; ++k) Hx[(long long)i * 3 + k] = 0.5 * (Fp[k] + Fm[k]) - 0.5 * a * (Up[k] - Um[k]);
}

__global__ void update1_kernel(const double* __restrict__ Us, const double* Un, double* Uout,
                               const double* __restrict__ Hx, const double* __restrict__ E, double a, double b,
                               double dt, int nx, double q, double m, double dx) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nx) return;
    const int im = (i == 0) ? nx - 1 : i - 1;
    const double n = Us[i * 3], nu = Us[i * 3 + 1];
    const double e = E[i];
    const double L[3] = {0.0, (q / m) * n * e, 2.0 * q * nu * e};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double s = Us[i * 3 + k] + dt * (L[k] - (Hx[i * 3 + k] - Hx[im * 3 + k]) / dx);
        Uout[i * 3 + k] = (a != 0.0 ? a * Un[i * 3 + k] : 0.0) + b * s;
    }
}

// -------------------------------------------------------------- launchers --
// One SSP-RK3 step.  work: U1, U2 (10 or 3 doubles per cell each), Hx, Hy.
hipError_t launch_fluid_rk3_3v(double* U, const double* mom_t, const double* mom_t1, const double* E_t,
                               const double* B_t, const double* E_t1, const double* B_t1, const double* E_th,
                               const double* B_th, double dt, int nx, int ny, double q, double m, double dx,
                               double dy, double* work, hipStream_t st) {
    const long long cells = (long long)nx * ny;
    double* U1 = work;
    double* U2 = U1 + cells * 10;
    double* Hx = U2 + cells * 10;
    double* Hy = Hx + cells * 10;
    struct Stage { const double* Us; const double* Un; double* Uo; const double* QA; const double* QB; double wa, wb;
                   const double* E; const double* B; double a, b; };
    const Stage S[3] = {
        {U, U, U1, mom_t, mom_t, 1.0, 0.0, E_t, B_t, 0.0, 1.0},
        {U1, U, U2, mom_t1, mom_t1, 1.0, 0.0, E_t1, B_t1, 0.75, 0.25},
        {U2, U, U, mom_t, mom_t1, 0.5, 0.5, E_th, B_th, 1.0 / 3.0, 2.0 / 3.0},
    };
    for (int k = 0; k < 3; ++k) {
        const hipError_t e = launch_fluid_stage_3v(S[k].Us, S[k].Un, S[k].Uo, S[k].QA, S[k].QB, S[k].wa, S[k].wb,
                                                   S[k].E, S[k].B, S[k].a, S[k].b, dt, nx, ny, q, m, dx, dy, Hx, Hy,
                                                   st);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t launch_fluid_stage_3v(const double* Us, const double* Un, double* Uo, const double* QA, const double* QB,
                                 double wa, double wb, const double* E, const double* B, double a, double b, double dt,
                                 int nx, int ny, double q, double m, double dx, double dy, double* Hx, double* Hy,
                                 hipStream_t st) {
    FluidArgs A{nx, ny, m, q, dx, dy};
    dim3 blk(64), gc((nx + 63) / 64, ny);
    const int nbx_row = (nx + kFaceTile - 1) / kFaceTile;
    const int nbx = nbx_row * ny, nby = nbx_row * (ny + 1);
    hipLaunchKernelGGL(faces3_kernel, dim3(nbx + nby), dim3(kFaceTile * 20), 0, st, Us, QA, QB, wa, wb, A, nbx_row,
                       nbx, Hx, Hy);
    hipLaunchKernelGGL(update3_kernel, gc, blk, 0, st, Us, Un, Uo, Hx, Hy, E, B, a, b, dt, A);
    return hipGetLastError();
}

hipError_t launch_fluid_rk3_1v(double* U, const double* mom_t, const double* mom_t1, const double* E_t,
                               const double* E_t1, const double* E_th, double dt, int nx, double q, double m,
                               double dx, double* work, hipStream_t st) {
    double* U1 = work;
    double* U2 = U1 + (long long)nx * 3;
    double* Hx = U2 + (long long)nx * 3;
    dim3 blk(64), g((nx + 63) / 64);
    struct Stage { const double* Us; const double* Un; double* Uo; const double* QA; const double* QB; double wa, wb;
                   const double* E; double a, b; };
    const Stage S[3] = {
        {U, U, U1, mom_t, mom_t, 1.0, 0.0, E_t, 0.0, 1.0},
        {U1, U, U2, mom_t1, mom_t1, 1.0, 0.0, E_t1, 0.75, 0.25},
        {U2, U, U, mom_t, mom_t1, 0.5, 0.5, E_th, 1.0 / 3.0, 2.0 / 3.0},
    };
    for (int k = 0; k < 3; ++k) {
        hipLaunchKernelGGL(flux_x1_kernel, g, blk, 0, st, S[k].Us, S[k].QA, S[k].QB, S[k].wa, S[k].wb, nx, m, Hx);
        hipLaunchKernelGGL(update1_kernel, g, blk, 0, st, S[k].Us, S[k].Un, S[k].Uo, Hx, S[k].E, S[k].a, S[k].b, dt,
                           nx, q, m, dx);
    }
    return hipGetLastError();
}

}  // namespace vl
