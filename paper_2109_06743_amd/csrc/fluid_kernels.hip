// Ten-moment fluid step for gfx950 (FP64): Eqs. 2-4 of arXiv 2109.06743 with
// the flux of the second moment P given by the third moment Qcal taken from f
// (Algorithm 1).  Semi-discrete finite volumes: CWENO-3 (Kurganov-Levy)
// point values at the faces, local Lax-Friedrichs flux with speed
// |u_d| + sqrt(3 p_dd / (m n)), and SSP-RK3 (Shu-Osher) in time.
//
// Face fluxes are computed once per face by their own kernels (x faces, y
// faces), then a per-cell kernel forms L(U) = -div H + S(U, E, B) and the RK
// stage combination U_out = a U_n + b (U_s + dt L).
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

// Load U and Qcal (20 values) of cell (j, i); j may lie beyond a wall: the
// mirror cell with odd components negated.  x is periodic.
__device__ __forceinline__ void load_uq(const double* U, const double* QA, const double* QB, double wa, double wb,
                                        int j, int i, const FluidArgs& A, double (&v)[20]) {
    double sgn = 1.0;
    bool mir = false;
    if (j < 0) { j = -1 - j; mir = true; }
    if (j >= A.ny) { j = 2 * A.ny - 1 - j; mir = true; }
    i = (i % A.nx + A.nx) % A.nx;
    const long long c = (long long)j * A.nx + i;
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        sgn = mir ? par_u(k) : 1.0;
        v[k] = sgn * U[c * 10 + k];
    }
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        sgn = mir ? par_q(k) : 1.0;
        v[10 + k] = sgn * (wa * QA[c * 20 + 10 + k] + (wb != 0.0 ? wb * QB[c * 20 + 10 + k] : 0.0));
    }
}

__device__ __forceinline__ double speed3(const double* U, int d, double m) {
    const double n = U[0];
    const double u = U[1 + d] / n;
    const double p = U[4 + p_index(d, d)] - m * n * u * u;
    return fabs(u) + sqrt(fmax(3.0 * p / (m * n), 0.0));
}

__device__ __forceinline__ void flux3(const double* U, const double* Q, int d, double m, double* F) {
    F[0] = U[1 + d];
    F[1] = U[4 + p_index(0, d)] / m;
    F[2] = U[4 + p_index(1, d)] / m;
    F[3] = U[4 + p_index(2, d)] / m;
    const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 0; k < 6; ++k) F[4 + k] = Q[q_index(ia[k], ib[k], d)];
}

// Numerical flux through the face between cells "left" (index 1 of the four)
// and "right" (index 2), given the four cells along direction d.
__device__ __forceinline__ void face_flux3(const double (&c0)[20], const double (&c1)[20], const double (&c2)[20],
                                           const double (&c3)[20], int d, double m, double* H) {
    double Um[10], Up[10], Qm[10], Qp[10];
#pragma unroll
    for (int k = 0; k < 20; ++k) {
        double l1, r1, l2, r2;
        cweno(c0[k], c1[k], c2[k], l1, r1);   // cell 1: its right face
        cweno(c1[k], c2[k], c3[k], l2, r2);   // cell 2: its left face
        if (k < 10) { Um[k] = r1; Up[k] = l2; }
        else { Qm[k - 10] = r1; Qp[k - 10] = l2; }
    }
    const double a = fmax(speed3(Um, d, m), speed3(Up, d, m));
    double Fm[10], Fp[10];
    flux3(Um, Qm, d, m, Fm);
    flux3(Up, Qp, d, m, Fp);
#pragma unroll
    for (int k = 0; k < 10; ++k) H[k] = 0.5 * (Fp[k] + Fm[k]) - 0.5 * a * (Up[k] - Um[k]);
}

// x faces: face i+1/2 of row j, i = 0..nx-1 -> Hx[(j*nx + i)*10]
__global__ void flux_x3_kernel(const double* __restrict__ U, const double* __restrict__ QA,
                               const double* __restrict__ QB, double wa, double wb, FluidArgs A,
                               double* __restrict__ Hx) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= A.nx) return;
    double c0[20], c1[20], c2[20], c3[20];
    load_uq(U, QA, QB, wa, wb, j, i - 1, A, c0);
    load_uq(U, QA, QB, wa, wb, j, i, A, c1);
    load_uq(U, QA, QB, wa, wb, j, i + 1, A, c2);
    load_uq(U, QA, QB, wa, wb, j, i + 2, A, c3);
    face_flux3(c0, c1, c2, c3, 0, A.m, Hx + ((long long)j * A.nx + i) * 10);
}

// y faces: face jh-1/2 (between rows jh-1 and jh), jh = 0..ny -> Hy[(jh*nx + i)*10]
__global__ void flux_y3_kernel(const double* __restrict__ U, const double* __restrict__ QA,
                               const double* __restrict__ QB, double wa, double wb, FluidArgs A,
                               double* __restrict__ Hy) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int jh = blockIdx.y;
    if (i >= A.nx) return;
    double c0[20], c1[20], c2[20], c3[20];
    load_uq(U, QA, QB, wa, wb, jh - 2, i, A, c0);
    load_uq(U, QA, QB, wa, wb, jh - 1, i, A, c1);
    load_uq(U, QA, QB, wa, wb, jh, i, A, c2);
    load_uq(U, QA, QB, wa, wb, jh + 1, i, A, c3);
    face_flux3(c0, c1, c2, c3, 1, A.m, Hy + ((long long)jh * A.nx + i) * 10);
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
    dim3 blk(64), gc((nx + 63) / 64, ny), gy((nx + 63) / 64, ny + 1);
    hipLaunchKernelGGL(flux_x3_kernel, gc, blk, 0, st, Us, QA, QB, wa, wb, A, Hx);
    hipLaunchKernelGGL(flux_y3_kernel, gy, blk, 0, st, Us, QA, QB, wa, wb, A, Hy);
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
