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
// With D = (eps + IS)^2 the normalised weights are
//   w_L = Dc Dr / S, w_C = 2 Dl Dr / S, w_R = Dl Dc / S,
//   S = Dc Dr + 2 Dl Dr + Dl Dc
// (one division), and since they sum to one the point values are b plus the
// weighted corrections (a constant state reconstructs to itself exactly).
__device__ __forceinline__ void cweno(double a, double b, double c, double& left, double& right) {
    const double dl = b - a, dr = c - b, d2 = c - 2.0 * b + a, dc = c - a;
    const double el = kCwenoEps + dl * dl, er = kCwenoEps + dr * dr;
    const double ec = kCwenoEps + (13.0 / 3.0) * d2 * d2 + 0.25 * dc * dc;
    const double Dl = el * el, Dc = ec * ec, Dr = er * er;
    const double tl = Dc * Dr, tc = 2.0 * Dl * Dr, tr = Dl * Dc;
    const double inv = 1.0 / (tl + tc + tr);
    const double wl = tl * inv, wc = tc * inv, wr = tr * inv;
    const double side = 0.5 * (wl * dl + wr * dr) + 0.25 * wc * dc;   // odd part
    const double even = wc * (d2 * (1.0 / 6.0));                         // even part
    right = b + (even + side);
    left = b + (even - side);
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
    double idx, idy;      // 1/dx, 1/dy
    int per;              // 1: periodic y, 0: reflecting walls
};

// Both face directions in one launch.  An x tile is kXTile consecutive faces
// i+1/2 of one cell row; a y tile is kYRows consecutive face rows jh-1/2 of
// kYCols adjacent columns.  A block stages the cell values (U and Qcal,
// wrapped in x, mirrored at the y walls) that its faces need in shared
// memory, forms the CWENO-3 point values once per cell and component, the two
// wave speeds once per face, then the 10 flux components of each face.
// Blocks [0, nbx) are x tiles, the rest y tiles.
constexpr int kXTile = 32;
constexpr int kYRows = 8, kYCols = 4;
constexpr int kFaceThreads = 256;   // eight blocks per CU: a launch is about one round
constexpr int kStageCells = (kYRows + 3) * kYCols;   // >= kXTile + 3
constexpr int kRecCells = (kYRows + 1) * kYCols;     // >= kXTile + 1
static_assert(kXTile + 3 <= kStageCells && kXTile + 1 <= kRecCells, "x tile must fit the staging arrays");
static_assert(kYRows * kYCols == kXTile, "both tiles hold the same number of faces");

__device__ __forceinline__ double stage_comp(const double* U, const double* QA, const double* QB, double wa,
                                             double wb, int j, int i, int k, const FluidArgs& A) {
    bool mir = false;
    if (A.per) {
        while (j < 0) j += A.ny;
        while (j >= A.ny) j -= A.ny;
    } else {
        if (j < 0) { j = -1 - j; mir = true; }
        if (j >= A.ny) { j = 2 * A.ny - 1 - j; mir = true; }
    }
    while (i < 0) i += A.nx;
    while (i >= A.nx) i -= A.nx;
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

// Species sp = blockIdx.y of the set.
__global__ void __launch_bounds__(kFaceThreads)
faces3_kernel(FluidSet S, double wa, double wb, FluidArgs A, int nbx_row, int nbx, int nby_col) {
    const int sp = blockIdx.y;
    const double* __restrict__ U = S.Us[sp];
    const double* __restrict__ QA = S.QA[sp];
    const double* __restrict__ QB = S.QB[sp];
    double* __restrict__ Hx = S.Hx[sp];
    double* __restrict__ Hy = S.Hy[sp];
    A.m = S.m[sp];
    __shared__ double raw[kStageCells][20];
    __shared__ double lo[kRecCells][20], hi[kRecCells][20];   // point values at a cell's lower / upper face
    __shared__ double spd[2][kXTile];
    const bool yface = (int)blockIdx.x >= nbx;
    const int b = yface ? (int)blockIdx.x - nbx : (int)blockIdx.x;
    const int row0 = yface ? (b / nby_col) * kYRows : b / nbx_row;
    const int col0 = yface ? (b % nby_col) * kYCols : (b % nbx_row) * kXTile;
    const int nstage = yface ? kStageCells : kXTile + 3;
    const int nrec = yface ? kRecCells : kXTile + 1;
    // Thread t < 240 handles component k = t % 20 of cells t / 20, + 12, + 24, ...
    // in the staging and reconstruction loops (no index division per element).
    constexpr int kCellsPerPass = kFaceThreads / 20;
    const int kc = (int)threadIdx.x % 20, c0 = (int)threadIdx.x / 20;
    // staged cell l: x tile (row0, col0 - 1 + l); y tile (row0 - 2 + l / kYCols, col0 + l % kYCols)
    for (int l = c0 < kCellsPerPass ? c0 : nstage; l < nstage; l += kCellsPerPass) {
        const int k = kc;
        const int j = yface ? row0 - 2 + l / kYCols : row0;
        const int i = yface ? col0 + l % kYCols : col0 - 1 + l;
        // y tiles: rows past ny + 1 and columns past nx feed no valid face
        const bool need = !yface || (j <= A.ny + 1 && i < A.nx);
        raw[l][k] = need ? stage_comp(U, QA, QB, wa, wb, j, i, k, A) : 0.0;
    }
    __syncthreads();
    // reconstructed cell r: x tile (row0, col0 + r); y tile (row0 - 1 + r / kYCols, col0 + r % kYCols)
    const int sstep = yface ? kYCols : 1;
    for (int r = c0 < kCellsPerPass ? c0 : nrec; r < nrec; r += kCellsPerPass) {
        const int k = kc;
        double l, h;
        cweno(raw[r][k], raw[r + sstep][k], raw[r + 2 * sstep][k], l, h);
        lo[r][k] = l;
        hi[r][k] = h;
    }
    __syncthreads();
    // face f: x tile i+1/2 with i = col0 + f of row0; y tile face row jh = row0 + f / kYCols at column
    // col0 + f % kYCols.  Minus side (cell i, or row jh - 1): r = f; plus side: r = f + sstep.
    const int d = yface ? 1 : 0;
    auto face_ok = [&](int f) {
        return yface ? (row0 + f / kYCols <= A.ny && col0 + f % kYCols < A.nx) : (col0 + f < A.nx);
    };
    for (int t = threadIdx.x; t < 2 * kXTile; t += kFaceThreads) {
        const int f = t % kXTile, side = t / kXTile;
        if (face_ok(f)) {
            const double* V = side ? lo[f + sstep] : hi[f];
            const double n = V[0];
            const double u = V[1 + d] / n;
            const double p = V[4 + p_index(d, d)] - A.m * n * u * u;
            spd[side][f] = fabs(u) + sqrt(fmax(3.0 * p / (A.m * n), 0.0));
        }
    }
    __syncthreads();
    // thread t < 250: flux component k = t % 10 of faces t / 10 and t / 10 + 25
    const int k = (int)threadIdx.x % 10;
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
    constexpr int kFacesPerPass = kFaceThreads / 10;
    for (int f = (int)threadIdx.x < 10 * kFacesPerPass ? (int)threadIdx.x / 10 : kXTile; f < kXTile;
         f += kFacesPerPass) {
        if (!face_ok(f)) continue;
        const double* Lm = hi[f];
        const double* Lp = lo[f + sstep];
        const double a = fmax(spd[0][f], spd[1][f]);
        const double Fm = Lm[src] * sc, Fp = Lp[src] * sc;
        long long h;
        if (yface) h = (long long)(row0 + f / kYCols) * A.nx + col0 + f % kYCols;
        else h = (long long)row0 * A.nx + col0 + f;
        (yface ? Hy : Hx)[h * 10 + k] = 0.5 * (Fp + Fm) - 0.5 * a * (Lp[k] - Lm[k]);
    }
}

// Temperature tensor T = (P - m n u u) / n of a fluid record (PAIRS order).
__device__ __forceinline__ void temperature6(const double* V, double m, double* T) {
    const double n = V[0];
    const double u[3] = {V[1] / n, V[2] / n, V[3] / n};
    const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 0; k < 6; ++k) T[k] = (V[4 + k] - m * n * u[pa[k]] * u[pb[k]]) / n;
}

// Temperature of cell (j, i) with x periodic and the y walls mirrored (the
// mirrored record has n u_y, P_xy, P_yz negated, so T_xy and T_yz flip).
__device__ __forceinline__ void temperature_at(const double* __restrict__ U, int j, int i, const FluidArgs& A,
                                               double* T) {
    bool mir = false;
    if (A.per) {
        if (j < 0) j += A.ny;
        if (j >= A.ny) j -= A.ny;
    } else {
        if (j < 0) { j = -1 - j; mir = true; }
        if (j >= A.ny) { j = 2 * A.ny - 1 - j; mir = true; }
    }
    if (i < 0) i += A.nx;
    if (i >= A.nx) i -= A.nx;
    const long long c = (long long)j * A.nx + i;
    double V[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) V[k] = U[c * 10 + k] * (mir ? par_u(k) : 1.0);
    temperature6(V, A.m, T);
}

// Temperature-gradient closure of Eq. 5 as a source of the second moment:
// S = -div Q = gchi n v_t lap T (gchi = chi / k0), lap by central second
// differences, x periodic, y walls mirrored; S[cells][6] in PAIRS order.
// Species blockIdx.z of the set; species without the closure are skipped.
__global__ void closure_source3_kernel(FluidSet Set, FluidArgs A) {
    const int sp = blockIdx.z;
    const double gchi = Set.gchi[sp];
    const double* __restrict__ Us = Set.Us[sp];
    double* __restrict__ S = Set.Sg[sp];
    A.m = Set.m[sp];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= A.nx || gchi == 0.0) return;
    double Tc[6], T1[6], T2[6], lx[6];
    temperature_at(Us, j, i, A, Tc);
    temperature_at(Us, j, i + 1, A, T1);
    temperature_at(Us, j, i - 1, A, T2);
#pragma unroll
    for (int k = 0; k < 6; ++k) lx[k] = (T1[k] - 2.0 * Tc[k]) + T2[k];
    temperature_at(Us, j + 1, i, A, T1);
    temperature_at(Us, j - 1, i, A, T2);
    const long long c = (long long)j * A.nx + i;
    const double vt = sqrt((Tc[0] + Tc[3] + Tc[5]) / (3.0 * A.m));
    const double w = gchi * (Us[c * 10] * vt);
    const double ix2 = A.idx * A.idx, iy2 = A.idy * A.idy;
#pragma unroll
    for (int k = 0; k < 6; ++k) S[c * 6 + k] = w * (lx[k] * ix2 + ((T1[k] - 2.0 * Tc[k]) + T2[k]) * iy2);
}

// U_out = a U_n + b (U_s + dt L(U_s)); U_out may alias U_n (each cell reads
// only its own U_n entry) but not U_s.  Where the species has the Eq. 5
// closure, Sg is an extra source of the second moment, [cells][6].  Species
// blockIdx.z of the set.
__global__ void update3_kernel(FluidSet S, const double* __restrict__ E, const double* __restrict__ B, double a,
                               double b, double dt, FluidArgs A) {
    const int sp = blockIdx.z;
    const double* __restrict__ Us = S.Us[sp];
    const double* Un = S.Un[sp];
    double* Uout = S.Uo[sp];
    const double* __restrict__ Hx = S.Hx[sp];
    const double* __restrict__ Hy = S.Hy[sp];
    const double* __restrict__ Sg = S.gchi[sp] != 0.0 ? S.Sg[sp] : nullptr;
    A.m = S.m[sp];
    A.q = S.q[sp];
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
    for (int k = 0; k < 10; ++k) L[k] -= (hxr[k] - hxl[k]) * A.idx + (hyt[k] - hyb[k]) * A.idy;
    if (Sg) {
#pragma unroll
        for (int k = 0; k < 6; ++k) L[4 + k] += Sg[c * 6 + k];
    }
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        const double s = u[k] + dt * L[k];
        Uout[c * 10 + k] = (a != 0.0 ? a * Un[c * 10 + k] : 0.0) + b * s;
    }
}

// Third moment of a fluid record with zero heat flux:
// Qcal_abc = u_a P_bc + u_b P_ac + u_c P_ab - 2 m n u_a u_b u_c, written at
// offsets 10..19 of 20-double records (the layout the face kernel reads).
__global__ void qcal_q0_kernel(const double* __restrict__ U, long long cells, double m, double* __restrict__ qc) {
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    const double n = U[c * 10];
    const double u[3] = {U[c * 10 + 1] / n, U[c * 10 + 2] / n, U[c * 10 + 3] / n};
    double P[3][3];
    const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 0; k < 6; ++k) P[pa[k]][pb[k]] = P[pb[k]][pa[k]] = U[c * 10 + 4 + k];
    const int ta[10] = {0, 0, 0, 0, 0, 0, 1, 1, 1, 2}, tb[10] = {0, 0, 0, 1, 1, 2, 1, 1, 2, 2},
              tc[10] = {0, 1, 2, 1, 2, 2, 1, 2, 2, 2};
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        const int x = ta[k], y = tb[k], z = tc[k];
        qc[c * 20 + 10 + k] = (u[x] * P[y][z] + u[y] * P[x][z] + u[z] * P[x][y]) - 2.0 * m * n * u[x] * u[y] * u[z];
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
// One SSP-RK3 step of ns species (one launch per kernel for all of them).
// work: per species U1, U2 (10 doubles per cell each), Hx (10 per cell), Hy
// (10 per face of ny + 1 rows), fluid_rk3_3v_doubles(nx, ny) in all.
hipError_t launch_fluid_rk3_3v_set(int ns, double* const* U, const double* const* mom_t, const double* const* mom_t1,
                                   const double* E_t, const double* B_t, const double* E_t1, const double* B_t1,
                                   const double* E_th, const double* B_th, double dt, int nx, int ny, const double* q,
                                   const double* m, double dx, double dy, double* work, hipStream_t st, int per) {
    if (ns < 1 || ns > 2) return hipErrorInvalidValue;
    const long long cells = (long long)nx * ny;
    FluidSet S[3] = {};
    for (int s = 0; s < ns; ++s) {
        double* w = work + (size_t)s * fluid_rk3_3v_doubles(nx, ny);
        double* U1 = w;
        double* U2 = U1 + cells * 10;
        double* Hx = U2 + cells * 10;
        double* Hy = Hx + cells * 10;
        const double* Us[3] = {U[s], U1, U2};
        double* Uo[3] = {U1, U2, U[s]};
        const double* QA[3] = {mom_t[s], mom_t1[s], mom_t[s]};
        const double* QB[3] = {mom_t[s], mom_t1[s], mom_t1[s]};
        for (int k = 0; k < 3; ++k) {
            S[k].Us[s] = Us[k];
            S[k].Un[s] = U[s];
            S[k].Uo[s] = Uo[k];
            S[k].QA[s] = QA[k];
            S[k].QB[s] = QB[k];
            S[k].Hx[s] = Hx;
            S[k].Hy[s] = Hy;
            S[k].Sg[s] = nullptr;
            S[k].m[s] = m[s];
            S[k].q[s] = q[s];
            S[k].gchi[s] = 0.0;
        }
    }
    const double wa[3] = {1.0, 1.0, 0.5}, wb[3] = {0.0, 0.0, 0.5};
    const double* E[3] = {E_t, E_t1, E_th};
    const double* B[3] = {B_t, B_t1, B_th};
    const double a[3] = {0.0, 0.75, 1.0 / 3.0}, b[3] = {1.0, 0.25, 2.0 / 3.0};
    for (int k = 0; k < 3; ++k) {
        const hipError_t e = launch_fluid_stage_3v_set(S[k], ns, wa[k], wb[k], E[k], B[k], a[k], b[k], dt, nx, ny,
                                                       dx, dy, st, per);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t launch_fluid_rk3_3v(double* U, const double* mom_t, const double* mom_t1, const double* E_t,
                               const double* B_t, const double* E_t1, const double* B_t1, const double* E_th,
                               const double* B_th, double dt, int nx, int ny, double q, double m, double dx,
                               double dy, double* work, hipStream_t st, int per) {
    double* Ul[1] = {U};
    const double* mt[1] = {mom_t};
    const double* mt1[1] = {mom_t1};
    return launch_fluid_rk3_3v_set(1, Ul, mt, mt1, E_t, B_t, E_t1, B_t1, E_th, B_th, dt, nx, ny, &q, &m, dx, dy, work,
                                   st, per);
}

// The update kernel reads each cell's 10-double records with 8-byte lane
// accesses 80 bytes apart, so a wave's ten loads share the same lines; with
// many waves per CU those lines are evicted between the loads and fetched
// again.  Dynamic LDS that the kernel does not use caps it at four one-wave
// blocks per CU (one wave per SIMD): 2048 x 1024 cells x 2 species, 7.35 ->
// 6.89 ms per fluid-only step (two waves per SIMD: 7.08, five: 7.86).  The
// faces kernel goes the other way (capped at four blocks per CU: 9.03 ms).
constexpr unsigned kUpdateLdsCap = 40960;

hipError_t launch_fluid_stage_3v_set(const FluidSet& S, int ns, double wa, double wb, const double* E,
                                     const double* B, double a, double b, double dt, int nx, int ny, double dx,
                                     double dy, hipStream_t st, int per) {
    if (ns < 1 || ns > 2) return hipErrorInvalidValue;
    FluidArgs A{nx, ny, 0.0, 0.0, 1.0 / dx, 1.0 / dy, per};
    dim3 blk(64), gc((nx + 63) / 64, ny, ns);
    const int nbx_row = (nx + kXTile - 1) / kXTile;
    const int nby_col = (nx + kYCols - 1) / kYCols;
    const int nbx = nbx_row * ny, nby = nby_col * ((ny + 1 + kYRows - 1) / kYRows);
    hipLaunchKernelGGL(faces3_kernel, dim3(nbx + nby, ns), dim3(kFaceThreads), 0, st, S, wa, wb, A, nbx_row, nbx,
                       nby_col);
    bool grad = false;
    for (int s = 0; s < ns; ++s) {
        if (S.gchi[s] != 0.0 && !S.Sg[s]) return hipErrorInvalidValue;
        grad = grad || S.gchi[s] != 0.0;
    }
    if (grad) hipLaunchKernelGGL(closure_source3_kernel, gc, blk, 0, st, S, A);
    hipLaunchKernelGGL(update3_kernel, gc, blk, kUpdateLdsCap, st, S, E, B, a, b, dt, A);
    return hipGetLastError();
}

hipError_t launch_fluid_stage_3v(const double* Us, const double* Un, double* Uo, const double* QA, const double* QB,
                                 double wa, double wb, const double* E, const double* B, double a, double b, double dt,
                                 int nx, int ny, double q, double m, double dx, double dy, double* Hx, double* Hy,
                                 hipStream_t st, double gchi, double* Sg, int per) {
    FluidSet S{};
    S.Us[0] = Us;
    S.Un[0] = Un;
    S.Uo[0] = Uo;
    S.QA[0] = QA;
    S.QB[0] = QB;
    S.Hx[0] = Hx;
    S.Hy[0] = Hy;
    S.Sg[0] = Sg;
    S.m[0] = m;
    S.q[0] = q;
    S.gchi[0] = gchi;
    return launch_fluid_stage_3v_set(S, 1, wa, wb, E, B, a, b, dt, nx, ny, dx, dy, st, per);
}

hipError_t launch_qcal_q0(const double* U, long long cells, double m, double* qc, hipStream_t st) {
    hipLaunchKernelGGL(qcal_q0_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st, U, cells, m, qc);
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
