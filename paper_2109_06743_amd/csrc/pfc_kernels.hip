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
#include <climits>

#include "vl_internal.h"

namespace vl {

// ---------------------------------------------------------------------------
// x sweep: layout [rows][nx][Nv]; each thread owns one velocity index v of one
// row and CX consecutive output cells; lanes run over contiguous v, so every
// load and store of a wave is one contiguous 256-byte (FP32) segment.  The
// thread keeps a window of CX+3 inputs in registers, ordered upwind to
// downwind, so both signs of the shift run the same straight-line code.
// Offsets within a row are 32-bit (nx * Nv < 2^31 is checked on the host) and
// advance by one row per element; only windows that cross the periodic seam
// take the wrapping path.
template <class T, int CX>
__global__ void __launch_bounds__(256)
pfc_x_kernel(const T* __restrict__ fin, T* __restrict__ fout, int nx, int Nv, float inv_inner, double vx_lo,
             double dvx, double tau_dx, const T* __restrict__ finf_p, typename Bits<T>::U* __restrict__ max_out) {
    // work index = (v block fastest, then x chunk, then row), XCD-contiguous
    const unsigned nvb = (Nv + 255) / 256, nch = (nx + CX - 1) / CX;
    const unsigned w = xcd_work_index(blockIdx.x, gridDim.x);
    const int v = (int)(w % nvb) * 256 + threadIdx.x;
    const int c0 = (int)((w / nvb) % nch) * CX;
    const size_t rowoff = (size_t)(w / (nvb * nch)) * nx * Nv;
    const T* __restrict__ src = fin + rowoff;
    T* __restrict__ dst = fout + rowoff;
    const T F2 = T(2) * *finf_p;
    T mx = T(0);
    if (v < Nv) {
        const int ivx = row_of(v, inv_inner);
        const double s = (vx_lo + (ivx + 0.5) * dvx) * tau_dx;
        const bool pos = s >= 0.0;
        const Shift<T> sh(fabs(s));
        const int K = sh.K < nx ? (int)sh.K : (int)(sh.K % nx);
        int idx = pos ? (c0 - K - 2) : (c0 + K + CX + 1);
        while (idx < 0) idx += nx;
        while (idx >= nx) idx -= nx;
        const int step = pos ? 1 : -1;
        const unsigned dstep = pos ? (unsigned)Nv : (unsigned)(-Nv);
        unsigned off = (unsigned)idx * (unsigned)Nv + (unsigned)v;
        T W[CX + 3];
        const bool wraps = pos ? (idx + CX + 2 >= nx) : (idx - CX - 2 < 0);
        if (!wraps) {
#pragma unroll
            for (int w = 0; w < CX + 3; ++w) {
                W[w] = src[off];
                off += dstep;
            }
        } else {
            const unsigned span = (unsigned)nx * (unsigned)Nv;
#pragma unroll
            for (int w = 0; w < CX + 3; ++w) {
                W[w] = src[off];
                idx += step;
                off += dstep;
                if (idx == nx) {
                    idx = 0;
                    off -= span;
                } else if (idx < 0) {
                    idx = nx - 1;
                    off += span;
                }
            }
        }
        T o[CX];
        T D = W[2] - W[1];
        T phi_prev = pfc_phi_d(W[1], W[1] - W[0], D, sh.a, sh.ac1, sh.ac2, F2);
#pragma unroll
        for (int r = 0; r < CX; ++r) {
            const T Dn = W[r + 3] - W[r + 2];
            const T phi_next = pfc_phi_d(W[r + 2], D, Dn, sh.a, sh.ac1, sh.ac2, F2);
            o[r] = fmax(W[r + 2] + phi_prev - phi_next, T(0));
            phi_prev = phi_next;
            D = Dn;
        }
        unsigned ooff = (unsigned)(pos ? c0 : c0 + CX - 1) * (unsigned)Nv + (unsigned)v;
        if (c0 + CX <= nx) {
#pragma unroll
            for (int r = 0; r < CX; ++r) {
                dst[ooff] = o[r];
                mx = fmax(mx, o[r]);
                ooff += dstep;
            }
        } else {
#pragma unroll
            for (int r = 0; r < CX; ++r) {
                if ((pos ? c0 + r : c0 + CX - 1 - r) < nx) {
                    dst[ooff] = o[r];
                    mx = fmax(mx, o[r]);
                }
                ooff += dstep;
            }
        }
    }
    if (max_out) block_max_part(mx, max_out);
}

// Partial flux a w + cA A + cB B of a cell with value w and neighbour
// differences Dm (below) and Dp (above), F2 = 2 f_inf: the limited slopes are
// A = med3(Dp, -r2, 2w) and B = med3(Dm, -2w, r2) with r2 = F2 - 2w taken
// without its clamp at zero (see the cubic velocity sweeps below).
template <class T>
__device__ __forceinline__ T sub_cell_flux(T w, T Dm, T Dp, T a, T cA, T cB, T F2) {
    const T x2 = w + w;
    const T r2 = F2 - x2;
    const T A = med3(Dp, -r2, x2);
    const T B = med3(Dm, -x2, r2);
    return fma(cA, A, fma(cB, B, a * w));
}

// ---------------------------------------------------------------------------
// Fused X(tau) for 2X3V: the x sweep and then the y sweep with one f_inf, in
// one pass over f.
//
// Work item: one wave = 64 consecutive velocity indices of the block (a
// "chunk"; the block of a cell is contiguous, so a wave's access to one cell
// is a 256-byte run -- whole 128-byte lines wherever the block size is a
// multiple of 32 elements), C adjacent x cells (a strip) and a segment of S
// rows.  Every lane owns one velocity v and writes only v.  All lanes walk
// the rows upward together, so each step reads the same row in every lane
// and the wave reads whole lines of it: a lane whose v_y is negative walks
// against its flow and emits each output K_y + 1 rows after the upward
// lanes (its output at row r depends on the x-swept rows r+K_y-1 .. r+K_y+2,
// which it holds by then).
//
// y boundary, with virtual rows q outside [0, ny): periodic: row q mod ny of
// v itself.  Reflecting walls: the pencil of v continues beyond a wall with
// the pencil of its mirror velocity v' (v_y -> -v_y) read backwards, i.e.
// q mod 2ny = q' < ny is row q' of v and q' >= ny is row 2ny-1-q' of v'.
// Both velocities of a mirror pair take the shift of the positive one, so
// the flux through a wall that the lane of v sends out and the flux the lane
// of v' takes in are computed from the same values in the same order: the
// wall exchange conserves mass exactly.
//
// For each row the x sweep of the C cells runs on the fly (a window of C+3
// inputs in registers, three rows of loads in flight while one is
// computed) and feeds the y update, so the x-swept array never reaches
// memory.  A load is a wave-uniform row base plus a per-lane 32-bit byte
// offset; the stores of one step (rows i-2-Kmax .. i-1+Kmax across the wave)
// are a wave-uniform base plus per-lane 32-bit offsets where those rows span
// less than 4 GiB (WIDE = false), else a per-lane 64-bit address.
// Work order: chunk fastest, then strip, then segment, so the waves in
// flight cover whole rows and neighbouring strips (x halos) together.
struct XYArgs {
    int nx, ny, Nv, nvy, nvz, S, nchunks, nst, nseg, per;
    float inv_nvz, inv_nvyz;
    double vx_lo, dvx, tau_dx, vy_lo, dvy, tau_dy;
};

template <class T, int C, bool WIDE>
__global__ void __launch_bounds__(256)
pfc_xy_kernel(const T* __restrict__ fin, T* __restrict__ fout, XYArgs A, const T* __restrict__ finf_p,
              typename Bits<T>::U* __restrict__ max_out) {
    const unsigned gw = xcd_work_index(blockIdx.x, gridDim.x) * 4u + (threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const unsigned chunk = gw % (unsigned)A.nchunks;
    const unsigned rest = gw / (unsigned)A.nchunks;
    const int c0 = (int)(rest % (unsigned)A.nst) * C;
    const unsigned seg = rest / (unsigned)A.nst;
    const T F2 = T(2) * *finf_p;
    T mx = T(0);
    if (seg < (unsigned)A.nseg) {                    // wave-uniform
        const int nx = A.nx, ny = A.ny, Nv = A.Nv;
        const int vl = (int)chunk * kWave + lane;
        const bool active = vl < Nv;
        const int v = active ? vl : Nv - 1;          // idle lanes walk a real pencil and store nothing
        const int ivx = row_of(v, A.inv_nvyz);
        const int jy = row_of(v, A.inv_nvz) - ivx * A.nvy;
        const int jm = A.nvy - 1 - jy;
        const bool up = jy >= jm;                    // v_y >= 0 (an odd grid's middle cell does not move)
        // y: both members of a mirror pair move by the shift of the positive one
        const double syd = (jy == jm) ? 0.0 : (A.vy_lo + ((up ? jy : jm) + 0.5) * A.dvy) * A.tau_dy;
        const ShiftT<T> shy(syd);
        const int L = A.per ? ny : 2 * ny;
        const int Ky = shy.K < L ? shy.K : shy.K % L;
        int Kmax = Ky;
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) Kmax = max(Kmax, __shfl_xor(Kmax, o, kWave));
        Kmax = __builtin_amdgcn_readfirstlane(Kmax);
        // x: uniform shift along the row
        const double sxd = (A.vx_lo + (ivx + 0.5) * A.dvx) * A.tau_dx;
        const bool posx = sxd >= 0.0;
        const Shift<T> shx(fabs(sxd));
        const int Kx = shx.K < nx ? (int)shx.K : (int)(shx.K % nx);
        int col = posx ? c0 - Kx - 2 : c0 + Kx + C + 1;  // first (upwind) column of the x window
        while (col < 0) col += nx;
        while (col >= nx) col -= nx;
        unsigned boff[C + 3];
#pragma unroll
        for (int w = 0; w < C + 3; ++w) {
            boff[w] = ((unsigned)col * (unsigned)Nv + (unsigned)v) * (unsigned)sizeof(T);
            col += posx ? 1 : -1;
            if (col == nx) col = 0;
            if (col < 0) col = nx - 1;
        }
        const unsigned dmir = (unsigned)((jm - jy) * A.nvz) * (unsigned)sizeof(T);   // v' - v (mod 2^32)
        const size_t rowbytes = (size_t)nx * Nv * sizeof(T);
        // output rows of the segment and the steps that produce them
        const int r0 = (int)seg * A.S;
        const int r1 = min(r0 + A.S, ny);
        const int ib = r0 + 1 - Kmax, ie = r1 + 1 + Kmax;
        const int dr = up ? Ky - 1 : -2 - Ky;        // output row = step + dr
        const int ilo = active ? r0 - dr : INT_MAX, ihi = r1 - dr;
        const int drmin = -2 - Kmax;
        unsigned soff[C];
        bool colok[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int oc = posx ? c0 + c : c0 + C - 1 - c;   // the x outputs run upwind to downwind
            colok[c] = oc < nx;
            const unsigned within = ((unsigned)oc * (unsigned)Nv + (unsigned)v) * (unsigned)sizeof(T);
            soff[c] = WIDE ? within : (unsigned)(dr - drmin) * (unsigned)rowbytes + within;
        }
        const bool full = c0 + C <= nx;
        // virtual row q -> (row, mirror?): wave-uniform
        auto load = [&](int q, T (&W)[C + 3]) {
            int row = q;
            bool mir = false;
            if ((unsigned)q >= (unsigned)ny) {
                row = q % L;
                if (row < 0) row += L;
                if (!A.per && row >= ny) {
                    mir = true;
                    row = L - 1 - row;
                }
            }
            const char* base = reinterpret_cast<const char*>(fin) + (size_t)row * rowbytes;
            if (!mir) {
#pragma unroll
                for (int w = 0; w < C + 3; ++w) W[w] = *reinterpret_cast<const T*>(base + boff[w]);
            } else {
#pragma unroll
                for (int w = 0; w < C + 3; ++w) W[w] = *reinterpret_cast<const T*>(base + (boff[w] + dmir));
            }
        };
        // partial flux without the clamp of r2 at zero: every sweep's input
        // lies in [0, f_inf] up to rounding (as in the velocity sweeps)
        auto xsweep = [&](const T (&W)[C + 3], T (&P)[C]) {
            T D = W[2] - W[1];
            T phi_prev = sub_cell_flux(W[1], W[1] - W[0], D, shx.a, shx.ac1, shx.ac2, F2);
#pragma unroll
            for (int r = 0; r < C; ++r) {
                const T Dn = W[r + 3] - W[r + 2];
                const T phi_next = sub_cell_flux(W[r + 2], D, Dn, shx.a, shx.ac1, shx.ac2, F2);
                P[r] = fmax(W[r + 2] + phi_prev - phi_next, T(0));
                phi_prev = phi_next;
                D = Dn;
            }
        };
        // y state per column: P1 = P(i-1), P2 = P(i-2) and ph = the flux of
        // cell i-2 in the lane's direction of motion (up: through its upper
        // face, from P(i-3), P(i-2), P(i-1); down: through its lower face)
        T P1[C], P2[C], ph[C];
        {
            T Wa[C + 3], Pa[C];
            load(ib - 3, Wa);
            xsweep(Wa, Pa);
            load(ib - 2, Wa);
            xsweep(Wa, P2);
            load(ib - 1, Wa);
            xsweep(Wa, P1);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const T d1 = P2[c] - Pa[c], d0 = P1[c] - P2[c];
                ph[c] = sub_cell_flux(P2[c], up ? d1 : -d0, up ? d0 : -d1, shy.a, shy.ac1, shy.ac2, F2);
            }
        }
        // step i: x-sweep row i (window Wc), the flux of cell i-1, the
        // output of cell i-1 (up, stored at row i-1+Ky) or i-2 (down, at row
        // i-2-Ky); the window of row i+3 is loaded into Wn meanwhile
        auto step = [&](int i, const T (&Wc)[C + 3], T (&Wn)[C + 3]) {
            if (i + 3 <= ie) load(i + 3, Wn);
            T P0[C];
            xsweep(Wc, P0);
            T o[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const T d1 = P1[c] - P2[c], d0 = P0[c] - P1[c];
                const T phn = sub_cell_flux(P1[c], up ? d1 : -d0, up ? d0 : -d1, shy.a, shy.ac1, shy.ac2, F2);
                const T base = up ? P1[c] : P2[c];
                const T fin_ = up ? ph[c] : phn;
                const T fout_ = up ? phn : ph[c];
                o[c] = fmax(base + fin_ - fout_, T(0));
                ph[c] = phn;
                P2[c] = P1[c];
                P1[c] = P0[c];
            }
            if (i >= ilo && i < ihi) {
                char* ob = WIDE ? reinterpret_cast<char*>(fout) + (size_t)(i + dr) * rowbytes
                                : reinterpret_cast<char*>(fout) + (long long)(i + drmin) * (long long)rowbytes;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    if (full || colok[c]) {
                        *reinterpret_cast<T*>(ob + soff[c]) = o[c];
                        mx = max_nonneg(mx, o[c], F2);
                    }
                }
            }
        };
        T W0[C + 3], W1[C + 3], W2[C + 3], W3[C + 3];
        load(ib, W0);
        if (ib + 1 <= ie) load(ib + 1, W1);
        if (ib + 2 <= ie) load(ib + 2, W2);
        int i = ib;
        for (; i + 3 <= ie; i += 4) {                 // four rows: the windows rotate
            step(i, W0, W3);
            step(i + 1, W1, W0);
            step(i + 2, W2, W1);
            step(i + 3, W3, W2);
        }
        if (i <= ie) step(i, W0, W3);
        if (i + 1 <= ie) step(i + 1, W1, W0);
        if (i + 2 <= ie) step(i + 2, W2, W1);
    }
    if (max_out) block_max_part(mx, max_out);
}

// ---------------------------------------------------------------------------
// 3V velocity operator by the backsubstitution split.  The step's velocity
// map under the cell's uniform E, B is the implicit-midpoint (Boris) map
// v -> R v + c, R = I + [s](I + [t]) with t = (q tau/2m) B, s = 2t/(1+t.t)
// and [a]v = v x a, c = (I + R)(q tau/2m) E.  Row by row it factors into an
// x-, a y- and a z-map that each change one component from the components
// already updated (x' = a x + b y + e z + cx; y' = d x' + g y + h z + cy;
// z' = k x' + l y' + n z + cz).  Each map is affine along its pencils: the
// stretch is the cell's (a, g or n), the shift linear in the pencil's
// transverse cell-centre velocities.  Coefficients in FP64.
__device__ __forceinline__ void backsub_coeffs(const double* EB, double qm, double tau, double* C) {
    const double h = 0.5 * qm * tau;
    const double t[3] = {h * EB[3], h * EB[4], h * EB[5]};
    const double k = 2.0 / (1.0 + t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    const double s[3] = {k * t[0], k * t[1], k * t[2]};
    // [a] as a matrix: [a]v = v x a
    auto X = [](const double* a, double (&M)[3][3]) {
        M[0][0] = 0.0;   M[0][1] = a[2];  M[0][2] = -a[1];
        M[1][0] = -a[2]; M[1][1] = 0.0;   M[1][2] = a[0];
        M[2][0] = a[1];  M[2][1] = -a[0]; M[2][2] = 0.0;
    };
    double S[3][3], T[3][3], R[3][3];
    X(s, S);
    X(t, T);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = S[i][j] + (i == j ? 1.0 : 0.0);
            for (int l = 0; l < 3; ++l) acc += S[i][l] * T[l][j];
            R[i][j] = acc;
        }
    double c[3];
    for (int i = 0; i < 3; ++i) c[i] = h * (EB[i] + R[i][0] * EB[0] + R[i][1] * EB[1] + R[i][2] * EB[2]);
    const double a = R[0][0], b = R[0][1], e = R[0][2];
    const double d = R[1][0] / a;
    const double g = R[1][1] - d * b, hh = R[1][2] - d * e;
    const double det = R[0][0] * R[1][1] - R[0][1] * R[1][0];
    const double kk = (R[2][0] * R[1][1] - R[2][1] * R[1][0]) / det;
    const double l = (R[0][0] * R[2][1] - R[0][1] * R[2][0]) / det;
    const double n = R[2][2] - kk * R[0][2] - l * R[1][2];
    C[0] = a;  C[1] = b;  C[2] = e;  C[3] = c[0];
    C[4] = d;  C[5] = g;  C[6] = hh; C[7] = c[1] - d * c[0];
    C[8] = kk; C[9] = l;  C[10] = n; C[11] = c[2] - kk * c[0] - l * c[1];
}

// One affine sweep of the block in shared memory along axis dd: the content
// at cell coordinate xi (cell j = [j, j+1]) moves to alpha xi + sigma.  Each
// thread owns whole pencils.  Face i of the output has its foot
// F_i = (i - sigma)/alpha, clamped to the box [0, n] (the wall faces keep
// F_0 = 0, F_n = n: zero flux); F = j + t (0 <= t < 1) splits it, and
// R_i = phi(j, 1 - t), the mass of cell j above the foot (phi the limited
// partial flux; R = f_j exactly at t = 0, 0 beyond the box).  Output cell i
// holds the mass between its two feet:
//   j_{i+1} == j_i:  R_i - R_{i+1}
//   else:            R_i + f_{j_i+1} + ... + f_{j_{i+1}-1} + (f_{j_{i+1}} - R_{i+1}),
// so whole-cell moves are exact and the pencil's mass telescopes.
template <class T, int NMAX>
__device__ __forceinline__ void sweep_affine(T* blk, int dd, const double* C, const V3Params& P, T finf) {
    const int nv[3] = {P.nvx, P.nvy, P.nvz};
    const int pz = P.nvz | 1;
    const int n = nv[dd];
    const int npen = (P.nvx * P.nvy * P.nvz) / n;
    const double alpha = C[dd == 0 ? 0 : (dd == 1 ? 5 : 10)];
    for (int pen = threadIdx.x; pen < npen; pen += blockDim.x) {
        int base, stride;
        double vs;          // shift in velocity units
        if (dd == 0) {      // x' = a x + b y + e z + cx
            const int iy = pen / P.nvz, iz = pen % P.nvz;
            base = iy * pz + iz;
            stride = P.nvy * pz;
            vs = C[1] * (P.lo[1] + (iy + 0.5) * P.dv[1]) + C[2] * (P.lo[2] + (iz + 0.5) * P.dv[2]) + C[3];
        } else if (dd == 1) {   // y' = d x' + g y + h z + cy
            const int ix = pen / P.nvz, iz = pen % P.nvz;
            base = ix * P.nvy * pz + iz;
            stride = pz;
            vs = C[4] * (P.lo[0] + (ix + 0.5) * P.dv[0]) + C[6] * (P.lo[2] + (iz + 0.5) * P.dv[2]) + C[7];
        } else {            // z' = k x' + l y' + n z + cz
            const int ix = pen / P.nvy, iy = pen % P.nvy;
            base = (ix * P.nvy + iy) * pz;
            stride = 1;
            vs = C[8] * (P.lo[0] + (ix + 0.5) * P.dv[0]) + C[9] * (P.lo[1] + (iy + 0.5) * P.dv[1]) + C[11];
        }
        // v -> alpha v + vs in cell units: xi -> alpha xi + sigma
        const double sigma = ((alpha - 1.0) * P.lo[dd] + vs) * P.inv_dv[dd];
        const T ia = (T)(1.0 / alpha), ib = (T)(-sigma / alpha);
        const T* pc = blk + base;
        auto val = [&](int j) -> T { return (j >= 0 && j < n) ? pc[j * stride] : T(0); };
        // right part of cell j above a foot at j + t
        auto rpart = [&](int j, T t) -> T {
            if (j >= n) return T(0);
            const T a = T(1) - t;
            const T c1 = t * (T(1) + t) * T(1.0 / 6.0), c2 = t * (T(2) - t) * T(1.0 / 6.0);
            return pfc_phi(val(j - 1), val(j), val(j + 1), a, c1, c2, finf);
        };
        T out[NMAX];
        int jp = 0;
        T Rp = val(0);                                  // face 0: F = 0
        const T nT = (T)n;
#pragma unroll
        for (int i = 0; i < NMAX; ++i) {
            if (i < n) {
                T F = (i + 1 == n) ? nT : fmin(fmax(fma((T)(i + 1), ia, ib), T(0)), nT);
                const T fj = floor(F);
                const int j = (int)fj;
                const T t = F - fj;
                const T R = rpart(j, t);
                T o;
                if (j == jp) {
                    o = Rp - R;
                } else {
                    T acc = Rp;
                    for (int m = jp + 1; m < j; ++m) acc += val(m);
                    o = acc + (val(j) - R);
                }
                out[i] = fmax(o, T(0));
                jp = j;
                Rp = R;
            }
        }
        T* pw = blk + base;
#pragma unroll
        for (int i = 0; i < NMAX; ++i)
            if (i < n) pw[i * stride] = out[i];
    }
}

template <class T, int NMAX, int NTH = 256>
__global__ void __launch_bounds__(NTH)
pfc_v3b_kernel(const T* fin, T* fout, const double* __restrict__ E, const double* __restrict__ B,
               V3Params P, const T* __restrict__ finf_p, typename Bits<T>::U* __restrict__ max_out) {
    extern __shared__ unsigned char smem_raw[];
    T* blk = reinterpret_cast<T*>(smem_raw);
    __shared__ double EB[6];
    __shared__ double Cs[12];
    const long long cell = blockIdx.x;
    const int nv = P.nvx * P.nvy * P.nvz;
    const int pz = P.nvz | 1;
    const T finf = *finf_p;
    if (threadIdx.x < 3) {
        EB[threadIdx.x] = E[cell * 3 + threadIdx.x];
        EB[3 + threadIdx.x] = B ? B[cell * 3 + threadIdx.x] : 0.0;
    }
    const T* src = fin + cell * nv;
    for (int e = threadIdx.x; e < nv; e += blockDim.x) blk[e + row_of(e, P.inv_nvz) * (pz - P.nvz)] = src[e];
    __syncthreads();
    if (threadIdx.x == 0) backsub_coeffs(EB, P.qm, P.tau, Cs);
    __syncthreads();
    double C[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) C[k] = Cs[k];
    sweep_affine<T, NMAX>(blk, 0, C, P, finf);
    __syncthreads();
    sweep_affine<T, NMAX>(blk, 1, C, P, finf);
    __syncthreads();
    sweep_affine<T, NMAX>(blk, 2, C, P, finf);
    __syncthreads();
    T* dst = fout + cell * nv;
    T mx = T(0);
    for (int e = threadIdx.x; e < nv; e += blockDim.x) {
        const T o = blk[e + row_of(e, P.inv_nvz) * (pz - P.nvz)];
        dst[e] = o;
        mx = fmax(mx, o);
    }
    if (max_out) block_max_part(mx, max_out);
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
    if (max_out) block_max_part(mx, max_out);
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
        const double s = P.qm * acc * sigma * P.inv_dv[d];
        const bool pos = s >= 0.0;
        const Shift<T> sh(fabs(s));
        // beyond n + 2 cells every output but the wall cell is 0 either way
        const int K = sh.K > (long long)(n + 2) ? n + 2 : (int)sh.K;
        // pencil in upwind-to-downwind order: element k lives at first + k * step
        const int first = pos ? base : base + (n - 1) * stride;
        const int step = pos ? stride : -stride;
        // shifted window W[j + 2] = g_{j - K} for j = -2 .. n-1 (zero outside the box),
        // so output p reads W at static positions p-2 .. p+1
        T W[NMAX + 2];
#pragma unroll
        for (int j = -2; j < NMAX; ++j) {
            const int src = j - K;
            const bool in = j < n && src >= 0;
            const T v = blk[first + (in ? src : 0) * step];
            W[j + 2] = in ? v : T(0);
        }
        // wall cell: every cell that reaches it stays, plus the partial flux of
        // the cell K below: sum_{m >= n-1-K} g_m + phi(g_{n-3-K}, g_{n-2-K}, g_{n-1-K})
        T top = T(0);
        for (int m = (n - 1 - K > 0 ? n - 1 - K : 0); m < n; ++m) top += blk[first + m * step];
#pragma unroll
        for (int p = 0; p < NMAX; ++p)
            if (p == n - 1) top += pfc_phi(W[p], W[p + 1], W[p + 2], sh.a, sh.c1, sh.c2, finf);
        T phi_prev = pfc_phi(W[0], W[1], W[2], sh.a, sh.c1, sh.c2, finf);   // phi at window position -1
#pragma unroll
        for (int p = 0; p < NMAX; ++p) {
            // W[p + 3] exists for p < NMAX - 1; the last position is the wall cell or unused
            const T wn = (p + 3 < NMAX + 2) ? W[(p + 3 < NMAX + 2) ? p + 3 : NMAX + 1] : T(0);
            const T phi_next = pfc_phi(W[p + 1], W[p + 2], wn, sh.a, sh.c1, sh.c2, finf);
            const T o = (p == n - 1) ? top : W[p + 2] + phi_prev - phi_next;
            phi_prev = phi_next;
            if (p < n) blk[first + p * step] = fmax(o, T(0));
        }
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
    for (int e = threadIdx.x; e < nv; e += blockDim.x) blk[e + row_of(e, P.inv_nvz) * (pz - P.nvz)] = src[e];
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
        const T o = blk[e + row_of(e, P.inv_nvz) * (pz - P.nvz)];
        dst[e] = o;
        mx = fmax(mx, o);
    }
    if (max_out) block_max_part(mx, max_out);
}

// ---------------------------------------------------------------------------
// The same operator for cubic velocity blocks with compile-time edge N: every
// pencil has length N and a stride known at compile time, so a pencil is
// straight-line code with constant shared-memory offsets.
//
// The block is stored [v_x][v_y][v_z] with v_z padded to N | 1; a wave takes
// 64 / N values of the first transverse index and all of the second.
//
// Sub-cell shifts (K = 0, the common case): with D_m = g_m - g_{m-1} (zero
// ghosts), r2 = 2 f_inf - 2 g_m and
//   A_m = med3(D_{m+1}, -r2, 2 g_m),  B_m = med3(D_m, -2 g_m, r2),
// the partial flux leaving cell m downwind is a g_m + a c1 A_m + a c2 B_m for
// s > 0 and, by reflecting the pencil, a g_m - a c1 B_m - a c2 A_m for s < 0.
// The flux through face m+1/2 (positive towards m+1) is the first for cell m
// or minus the second for cell m+1; the wall faces carry none.
//
// Every sweep keeps 0 <= g <= f_inf, so 2 f_inf - 2 g_m >= 0 up to rounding
// and r2 is taken without its clamp at zero: where rounding puts g_m an ulp
// above f_inf the bound moves by that ulp.  A wave whose pencils all shift the
// same way walks them in the downwind order (a negative shift reads the
// pencil backwards, which with constant offsets costs nothing): one
// difference, seven operations for the partial flux and three for the update
// per element.  A wave with both signs keeps the storage order and selects
// per lane, one operation more.

// Sub-cell sweep of a pencil held in registers (updated in place) whose
// wave's lanes all shift one way: REV walks it from its far end (s < 0), so
// the downwind direction is always +m.
template <class T, int N, bool REV>
__device__ __forceinline__ void regs_one_way(T (&g)[N], T a, T c1, T c2, T F2) {
    auto u = [&](int m) -> T& { return g[REV ? N - 1 - m : m]; };
    T Dm = u(0);                 // D_m = g_m - g_{m-1}, zero ghost below
    T Dp = u(1) - u(0);
    T Fprev = T(0);              // flux through the lower wall
#pragma unroll
    for (int m = 0; m < N; ++m) {
        T F = T(0);              // flux through face m+1/2 (none through the upper wall)
        const T w = u(m);
        if (m + 1 < N) {
            F = sub_cell_flux(w, Dm, Dp, a, c1, c2, F2);
            Dm = Dp;
            Dp = (m + 2 < N ? u(m + 2) : T(0)) - u(m + 1);
        }
        u(m) = fmax(w + Fprev - F, T(0));
        Fprev = F;
    }
}

// The same for a wave holding both signs: storage order, the sign folded
// into the coefficients and a per-lane select of the face flux.
template <class T, int N>
__device__ __forceinline__ void regs_mixed(T (&g)[N], bool pos, T a, T ac1, T ac2, T F2) {
    const T cA = pos ? ac1 : -ac2;
    const T cB = pos ? ac2 : -ac1;
    // phi_m: partial flux of cell m in the lane's direction
    T Dm = g[0];
    T Dp = g[1] - g[0];
    T phi_m = sub_cell_flux(g[0], Dm, Dp, a, cA, cB, F2);
    T Fprev = T(0);
#pragma unroll
    for (int m = 0; m < N; ++m) {
        T Fnext = T(0), phi_n = T(0);
        if (m + 1 < N) {
            Dm = Dp;
            Dp = (m + 2 < N ? g[m + 2] : T(0)) - g[m + 1];
            phi_n = sub_cell_flux(g[m + 1], Dm, Dp, a, cA, cB, F2);
            Fnext = pos ? phi_m : -phi_n;
        }
        g[m] = fmax(g[m] + Fprev - Fnext, T(0));
        Fprev = Fnext;
        phi_m = phi_n;
    }
}

// Shifts of a cell or more (any lane of the wave): windows gathered in the
// sweep direction, the cells within K of the far wall summed into it.
template <class T, int N>
__device__ __attribute__((noinline)) void pencil_shifted(T* blk, int first, int step, int K, T a, T ac1, T ac2,
                                                          T F2) {
    T W[N + 2];
    int q = first - (K + 2) * step;
#pragma unroll
    for (int j = -2; j < N; ++j) {
        const bool in = j - K >= 0;
        const T v = blk[in ? q : first];
        W[j + 2] = in ? v : T(0);
        q += step;
    }
    T top = T(0);
    for (int m = (N - 1 - K > 0 ? N - 1 - K : 0); m < N; ++m) top += blk[first + m * step];
    T D = W[1] - W[0];
    T Dn = W[2] - W[1];
    T phi_prev = pfc_phi_d(W[1], D, Dn, a, ac1, ac2, F2);
    D = Dn;
    q = first;
#pragma unroll
    for (int p = 0; p < N - 1; ++p) {
        Dn = W[p + 3] - W[p + 2];
        const T phi_next = pfc_phi_d(W[p + 2], D, Dn, a, ac1, ac2, F2);
        blk[q] = fmax(W[p + 2] + phi_prev - phi_next, T(0));
        phi_prev = phi_next;
        D = Dn;
        q += step;
    }
    blk[q] = fmax(top + phi_prev, T(0));
}

// One PFC sweep of a pencil held in registers, its displacement split into
// its sign pos and the shift sh (cells).
// Shifts of a cell or more (any lane of the wave) go through the pencil's own
// cells blk[base + m stride] of the shared block, which no other thread
// touches meanwhile.
template <class T, int N>
__device__ __forceinline__ void sweep_pencil_regs(T (&g)[N], bool pos, const ShiftT<T>& sh, T F2, T* blk, int base,
                                                  int stride) {
    if (__all(sh.K == 0) && __all(pos)) {
        regs_one_way<T, N, false>(g, sh.a, sh.ac1, sh.ac2, F2);
    } else if (__all(sh.K == 0) && __all(!pos)) {
        regs_one_way<T, N, true>(g, sh.a, sh.ac1, sh.ac2, F2);
    } else if (__all(sh.K == 0)) {
        regs_mixed<T, N>(g, pos, sh.a, sh.ac1, sh.ac2, F2);
    } else {
#pragma unroll
        for (int m = 0; m < N; ++m) blk[base + m * stride] = g[m];
        const int K = sh.K > N + 2 ? N + 2 : sh.K;
        const int first = pos ? base : base + (N - 1) * stride;
        pencil_shifted<T, N>(blk, first, pos ? stride : -stride, K, sh.a, sh.ac1, sh.ac2, F2);
#pragma unroll
        for (int m = 0; m < N; ++m) g[m] = blk[base + m * stride];
    }
}

// Displacement coefficients of sweep d: s = s0 + s1 i1 + s2 i2 over the
// pencil's two transverse indices (in FP64, then the storage type).
template <class T>
__device__ __forceinline__ void sweep_coeffs(int d, double sigma, const V3Params& P, const double* EB, T& s0, T& s1,
                                             T& s2) {
    const double C = P.qm * sigma * P.inv_dv[d];
    const double c0 = P.lo[0] + 0.5 * P.dv[0], c1 = P.lo[1] + 0.5 * P.dv[1], c2 = P.lo[2] + 0.5 * P.dv[2];
    double d0, d1, d2;
    if (d == 0) {           // pencil (iy, iz): a_x = (q/m)(Ex + vy Bz - vz By)
        d0 = C * (EB[0] + EB[5] * c1 - EB[4] * c2); d1 = C * EB[5] * P.dv[1]; d2 = -C * EB[4] * P.dv[2];
    } else if (d == 1) {    // pencil (ix, iz): a_y = (q/m)(Ey + vz Bx - vx Bz)
        d0 = C * (EB[1] + EB[3] * c2 - EB[5] * c0); d1 = -C * EB[5] * P.dv[0]; d2 = C * EB[3] * P.dv[2];
    } else {                // pencil (ix, iy): a_z = (q/m)(Ez + vx By - vy Bx)
        d0 = C * (EB[2] + EB[4] * c0 - EB[3] * c1); d1 = C * EB[4] * P.dv[0]; d2 = -C * EB[3] * P.dv[1];
    }
    s0 = (T)d0;
    s1 = (T)d1;
    s2 = (T)d2;
}

// One pencil of the cubic block along d (d = 0: (iy, iz); 1: (ix, iz); 2:
// (ix, iy)) with its shift split as pos / sh.
template <class T, int N>
__device__ __forceinline__ void sweep_cube_pencil(T* blk, int d, int pen, bool pos, const ShiftT<T>& sh, T F2) {
    constexpr int PZ = N | 1;
    const int stride = d == 0 ? N * PZ : (d == 1 ? PZ : 1);
    const int i1 = pen / N, i2 = pen % N;
    const int base = d == 0 ? i1 * PZ + i2 : (d == 1 ? i1 * N * PZ + i2 : (i1 * N + i2) * PZ);
    if (__all(sh.K == 0)) {
        T* pb = blk + base;
        T g[N];
#pragma unroll
        for (int m = 0; m < N; ++m) g[m] = pb[m * stride];
        if (__all(pos))
            regs_one_way<T, N, false>(g, sh.a, sh.ac1, sh.ac2, F2);
        else if (__all(!pos))
            regs_one_way<T, N, true>(g, sh.a, sh.ac1, sh.ac2, F2);
        else
            regs_mixed<T, N>(g, pos, sh.a, sh.ac1, sh.ac2, F2);
#pragma unroll
        for (int m = 0; m < N; ++m) pb[m * stride] = g[m];
    } else {
        const int K = sh.K > N + 2 ? N + 2 : sh.K;
        const int first = pos ? base : base + (N - 1) * stride;
        pencil_shifted<T, N>(blk, first, pos ? stride : -stride, K, sh.a, sh.ac1, sh.ac2, F2);
    }
}

// Shift of pencil pen of sweep d from the sweep's coefficients.
template <class T, int N>
__device__ __forceinline__ T cube_pencil_shift(int pen, T s0, T s1, T s2) {
    return fma(s1, (T)(pen / N), fma(s2, (T)(pen % N), s0));
}

template <class T, int N>
__device__ __forceinline__ void sweep_cube(T* blk, int d, double sigma, const V3Params& P, const double* EB, T F2) {
    T s0, s1, s2;
    sweep_coeffs<T>(d, sigma, P, EB, s0, s1, s2);
    for (int pen = threadIdx.x; pen < N * N; pen += blockDim.x) {
        const T s = cube_pencil_shift<T, N>(pen, s0, s1, s2);
        sweep_cube_pencil<T, N>(blk, d, pen, s >= T(0), ShiftT<T>(fabs(s)), F2);
    }
}

template <class T, int N, int NTH>
__global__ void __launch_bounds__(NTH)
pfc_v3_cube_kernel(const T* fin, T* fout, const double* __restrict__ E, const double* __restrict__ B, V3Params P,
                   const T* __restrict__ finf_p, typename Bits<T>::U* __restrict__ max_out) {
    constexpr int PZ = N | 1;
    constexpr int NV = N * N * N;
    constexpr int PER = NV / NTH;            // values per thread (NTH divides N^3)
    static_assert(PER * NTH == NV, "thread count must divide the block");
    // one v_x pencil per thread, or two: the two v_x sweeps run in registers
    constexpr bool kRegX = N * N <= NTH;
    constexpr bool kRegX2 = !kRegX && N * N <= 2 * NTH;
    __shared__ T blk[N * N * PZ];
    __shared__ double EB[6];
    const long long cell = xcd_work_index(blockIdx.x, gridDim.x);
    const T F2 = T(2) * *finf_p;
    if (threadIdx.x < 3) {
        EB[threadIdx.x] = E[cell * 3 + threadIdx.x];
        EB[3 + threadIdx.x] = B ? B[cell * 3 + threadIdx.x] : 0.0;
    }
    const double half = 0.5 * P.tau;
    const T* src = fin + cell * NV;
    T* dst = fout + cell * NV;
    T mx = T(0);
    if constexpr (kRegX) {
        // Thread t owns the v_x pencil at (iy, iz) = (t / N, t % N): it loads it
        // (unit stride across the wave), sweeps it, and stores it into the block
        // for the v_y, v_z, v_y sweeps; then reads it back for the last v_x
        // sweep and writes it out.  The fields come straight from global
        // memory for the first sweep, which runs before any barrier.
        const int t = threadIdx.x;
        const bool own = t < N * N;
        const int xb = (t / N) * PZ + t % N;
        constexpr int XS = N * PZ;
        double eb[6];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            eb[k] = E[cell * 3 + k];
            eb[3 + k] = B ? B[cell * 3 + k] : 0.0;
        }
        T xs0, xs1, xs2;
        sweep_coeffs<T>(0, half, P, eb, xs0, xs1, xs2);
        const T sx = fma(xs1, (T)(t / N), fma(xs2, (T)(t % N), xs0));
        const bool posx = sx >= T(0);
        const ShiftT<T> shx(fabs(sx));         // both v_x sweeps
        T g[N];
        if (own) {
#pragma unroll
            for (int k = 0; k < N; ++k) g[k] = __builtin_nontemporal_load(src + t + k * N * N);
            sweep_pencil_regs<T, N>(g, posx, shx, F2, blk, xb, XS);
#pragma unroll
            for (int k = 0; k < N; ++k) blk[xb + k * XS] = g[k];
        }
        __syncthreads();
        // one v_y and one v_z pencil per thread: their shifts are set up once,
        // the v_y one serving both v_y sweeps
        {
            T c0, c1, c2;
            sweep_coeffs<T>(1, half, P, EB, c0, c1, c2);
            const T sy = cube_pencil_shift<T, N>(t, c0, c1, c2);
            sweep_coeffs<T>(2, P.tau, P, EB, c0, c1, c2);
            const T sz = cube_pencil_shift<T, N>(t, c0, c1, c2);
            const ShiftT<T> shy(fabs(sy)), shz(fabs(sz));
            if (own) sweep_cube_pencil<T, N>(blk, 1, t, sy >= T(0), shy, F2);
            __syncthreads();
            if (own) sweep_cube_pencil<T, N>(blk, 2, t, sz >= T(0), shz, F2);
            __syncthreads();
            if (own) sweep_cube_pencil<T, N>(blk, 1, t, sy >= T(0), shy, F2);
            __syncthreads();
        }
        if (own) {
#pragma unroll
            for (int k = 0; k < N; ++k) g[k] = blk[xb + k * XS];
            sweep_pencil_regs<T, N>(g, posx, shx, F2, blk, xb, XS);
#pragma unroll
            for (int k = 0; k < N; ++k) {
                __builtin_nontemporal_store(g[k], dst + t + k * N * N);
                mx = fmax(mx, g[k]);
            }
        }
    } else if constexpr (kRegX2) {
        // Thread t owns the v_x pencils t and t + NTH (those below N^2): each is
        // loaded from global memory, swept in registers and stored into the
        // block; after the v_y, v_z, v_y sweeps in the block each is read back,
        // swept again and written out.  One pencil is in registers at a time.
        // A 34^3 v_x plane is not a whole number of lines (4624 B in FP32):
        // ordinary loads and stores let the caches merge the lines two wave
        // accesses share (4.01 -> 3.83 ms per 256x128x34^3 launch).
        const int t = threadIdx.x;
        constexpr int XS = N * PZ;
        double eb[6];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            eb[k] = E[cell * 3 + k];
            eb[3 + k] = B ? B[cell * 3 + k] : 0.0;
        }
        T xs0, xs1, xs2;
        sweep_coeffs<T>(0, half, P, eb, xs0, xs1, xs2);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int p = t + j * NTH;
            if (p < N * N) {
                const int xb = (p / N) * PZ + p % N;
                const T sx = cube_pencil_shift<T, N>(p, xs0, xs1, xs2);
                T g[N];
#pragma unroll
                for (int k = 0; k < N; ++k) g[k] = ld_f<kRowsWholeLines<T, N>>(src + p + k * N * N);
                sweep_pencil_regs<T, N>(g, sx >= T(0), ShiftT<T>(fabs(sx)), F2, blk, xb, XS);
#pragma unroll
                for (int k = 0; k < N; ++k) blk[xb + k * XS] = g[k];
            }
        }
        __syncthreads();
        sweep_cube<T, N>(blk, 1, half, P, EB, F2);
        __syncthreads();
        sweep_cube<T, N>(blk, 2, P.tau, P, EB, F2);
        __syncthreads();
        sweep_cube<T, N>(blk, 1, half, P, EB, F2);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int p = t + j * NTH;
            if (p < N * N) {
                const int xb = (p / N) * PZ + p % N;
                const T sx = cube_pencil_shift<T, N>(p, xs0, xs1, xs2);
                T g[N];
#pragma unroll
                for (int k = 0; k < N; ++k) g[k] = blk[xb + k * XS];
                sweep_pencil_regs<T, N>(g, sx >= T(0), ShiftT<T>(fabs(sx)), F2, blk, xb, XS);
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    st_f<kRowsWholeLines<T, N>>(g[k], dst + p + k * N * N);
                    mx = fmax(mx, g[k]);
                }
            }
        }
    } else {
        // large blocks stream through registers in chunks of four values per
        // thread
        constexpr int CH = PER > 16 ? 4 : PER;
        static_assert(PER % CH == 0, "chunks must tile the block");
#pragma unroll 1
        for (int c0 = 0; c0 < PER; c0 += CH) {
            T v[CH];
#pragma unroll
            for (int j = 0; j < CH; ++j) v[j] = __builtin_nontemporal_load(src + threadIdx.x + (c0 + j) * NTH);
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int e = threadIdx.x + (c0 + j) * NTH;
                blk[e + (e / N) * (PZ - N)] = v[j];
            }
        }
        __syncthreads();
        // each sweep reads the fields from shared memory after its barrier, which
        // keeps the five sweeps' shift set-ups from being hoisted (and held live)
        sweep_cube<T, N>(blk, 0, half, P, EB, F2);
        __syncthreads();
        sweep_cube<T, N>(blk, 1, half, P, EB, F2);
        __syncthreads();
        sweep_cube<T, N>(blk, 2, P.tau, P, EB, F2);
        __syncthreads();
        sweep_cube<T, N>(blk, 1, half, P, EB, F2);
        __syncthreads();
        sweep_cube<T, N>(blk, 0, half, P, EB, F2);
        __syncthreads();
#pragma unroll 1
        for (int c0 = 0; c0 < PER; c0 += CH) {
            T v[CH];
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int e = threadIdx.x + (c0 + j) * NTH;
                v[j] = blk[e + (e / N) * (PZ - N)];
            }
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                __builtin_nontemporal_store(v[j], dst + threadIdx.x + (c0 + j) * NTH);
                mx = fmax(mx, v[j]);
            }
        }
    }
    if (max_out) block_max_part(mx, max_out);
}

// ---------------------------------------------------------------------------
// The same operator when the block is larger than a CU's shared memory (the
// FP64 34^3 block, 314 KB, against 160 KB).  The v_y, v_z, v_y sweeps stay
// inside the planes of fixed v_x, so they run on PL planes at a time in shared
// memory (N / PL = 2 rounds); the rest of the block waits in registers.
// Thread t owns the v_x pencils p = t + NTH j (p < N^2):
//  1. each pencil is loaded, swept along v_x in registers, and split: its
//     values in the first PL planes go to shared memory, the others wait in
//     registers (a[j]; those of the partial last pencil set, which only some
//     threads own, in the pencil's own positions of the output block);
//  2. round 0 sweeps the first PL planes; each thread then swaps its own
//     plane values with a[j] (no other thread touches them), and round 1
//     sweeps the last PL planes;
//  3. each pencil is reassembled from a[j] and shared memory, swept along v_x
//     again and stored.
// Eight waves per block leave 256 registers per lane.  A v_x pencil that
// shifts by a cell or more is swept in the cell's output block, in its own
// positions, which nothing else reads or writes meanwhile (in place as well:
// the pencil's input has been read by then).
template <class T, int N, int NTH, int PL>
__global__ void __launch_bounds__(NTH)
pfc_v3_planes_kernel(const T* fin, T* fout, const double* __restrict__ E, const double* __restrict__ B,
                     V3Params P, const T* __restrict__ finf_p, typename Bits<T>::U* __restrict__ max_out) {
    constexpr int PZ = N | 1;
    constexpr int NN = N * N;
    constexpr int NP = (NN + NTH - 1) / NTH;     // v_x pencils per thread (the last one partial)
    constexpr unsigned XB = NN * sizeof(T);      // bytes between v_x planes
    static_assert(2 * PL == N, "two rounds of PL planes");
    static_assert(NN <= NP * NTH, "pencils cover the block");
    __shared__ T blk[PL * N * PZ];
    const int t = threadIdx.x;
    const long long cell = xcd_work_index(blockIdx.x, gridDim.x);
    const T F2 = T(2) * *finf_p;
    T* dst = fout + cell * (N * NN);
    const auto rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(fin + cell * (N * NN)), 0, N * XB, kBufWord3);
    const auto rd = __builtin_amdgcn_make_buffer_rsrc(dst, 0, N * XB, kBufWord3);
    double eb[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        eb[k] = E[cell * 3 + k];
        eb[3 + k] = B ? B[cell * 3 + k] : 0.0;
    }
    const double half = 0.5 * P.tau;
    T xs0, xs1, xs2, y0, y1, y2, z0, z1, z2;
    sweep_coeffs<T>(0, half, P, eb, xs0, xs1, xs2);
    sweep_coeffs<T>(1, half, P, eb, y0, y1, y2);
    sweep_coeffs<T>(2, P.tau, P, eb, z0, z1, z2);
    // v_x sweep of pencil p held in g; shifts of a cell or more go through the
    // pencil's own positions of the output block
    auto sweep_x = [&](T (&g)[N], int p) {
        const T sx = cube_pencil_shift<T, N>(p, xs0, xs1, xs2);
        const bool pos = sx >= T(0);
        const ShiftT<T> sh(fabs(sx));
        if (__all(sh.K == 0) && __all(pos)) {
            regs_one_way<T, N, false>(g, sh.a, sh.ac1, sh.ac2, F2);
        } else if (__all(sh.K == 0) && __all(!pos)) {
            regs_one_way<T, N, true>(g, sh.a, sh.ac1, sh.ac2, F2);
        } else if (__all(sh.K == 0)) {
            regs_mixed<T, N>(g, pos, sh.a, sh.ac1, sh.ac2, F2);
        } else {
            const unsigned po = (unsigned)p * sizeof(T);
#pragma unroll
            for (int m = 0; m < N; ++m) buf_st(g[m], rd, po, m * XB);
            const int K = sh.K > N + 2 ? N + 2 : sh.K;
            const int first = pos ? p : p + (N - 1) * NN;
            pencil_shifted<T, N>(dst, first, pos ? NN : -NN, K, sh.a, sh.ac1, sh.ac2, F2);
#pragma unroll
            for (int m = 0; m < N; ++m) g[m] = buf_ld(rd, po, m * XB, T());
        }
    };
    // the last plane halves of the full pencils wait in registers, those of
    // the partial last pencil (NN - (NP - 1) NTH of them) in its own
    // positions of the output block
    T a[NP - 1][PL];
    // 1. v_x half sweep; the first PL planes to shared memory
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int p = t + NTH * j;
        if (p < NN) {
            const int o = (p / N) * PZ + p % N;
            const unsigned po = (unsigned)p * sizeof(T);
            T g[N];
#pragma unroll
            for (int k = 0; k < N; ++k) g[k] = buf_ld(rs, po, k * XB, T());
            sweep_x(g, p);
#pragma unroll
            for (int k = 0; k < PL; ++k) {
                blk[k * N * PZ + o] = g[k];
                if (j < NP - 1)
                    a[j < NP - 1 ? j : 0][k] = g[PL + k];
                else
                    buf_st(g[PL + k], rd, po, (PL + k) * XB);
            }
        }
    }
    // 2. in-plane sweeps, round r on planes r PL .. r PL + PL - 1
    auto in_plane = [&](int r) {
        for (int pen = t; pen < PL * N; pen += NTH) {
            const int pg = pen + r * PL * N;        // (v_x plane, second index) over the whole block
            const T sy = cube_pencil_shift<T, N>(pg, y0, y1, y2);
            sweep_cube_pencil<T, N>(blk, 1, pen, sy >= T(0), ShiftT<T>(fabs(sy)), F2);
        }
        __syncthreads();
        for (int pen = t; pen < PL * N; pen += NTH) {
            const int pg = pen + r * PL * N;
            const T sz = cube_pencil_shift<T, N>(pg, z0, z1, z2);
            sweep_cube_pencil<T, N>(blk, 2, pen, sz >= T(0), ShiftT<T>(fabs(sz)), F2);
        }
        __syncthreads();
        for (int pen = t; pen < PL * N; pen += NTH) {
            const int pg = pen + r * PL * N;
            const T sy = cube_pencil_shift<T, N>(pg, y0, y1, y2);
            sweep_cube_pencil<T, N>(blk, 1, pen, sy >= T(0), ShiftT<T>(fabs(sy)), F2);
        }
        __syncthreads();
    };
    __syncthreads();
    in_plane(0);
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int p = t + NTH * j;
        if (p < NN) {
            const int o = (p / N) * PZ + p % N;
            const unsigned po = (unsigned)p * sizeof(T);
#pragma unroll
            for (int k = 0; k < PL; ++k) {
                const T v = blk[k * N * PZ + o];
                if (j < NP - 1) {
                    blk[k * N * PZ + o] = a[j < NP - 1 ? j : 0][k];
                    a[j < NP - 1 ? j : 0][k] = v;
                } else {
                    blk[k * N * PZ + o] = buf_ld(rd, po, (PL + k) * XB, T());
                    buf_st(v, rd, po, k * XB);
                }
            }
        }
    }
    __syncthreads();
    in_plane(1);
    // 3. second v_x half sweep and the store
    T mx = T(0);
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int p = t + NTH * j;
        if (p < NN) {
            const int o = (p / N) * PZ + p % N;
            const unsigned po = (unsigned)p * sizeof(T);
            T g[N];
#pragma unroll
            for (int k = 0; k < PL; ++k) {
                g[k] = j < NP - 1 ? a[j < NP - 1 ? j : 0][k] : buf_ld(rd, po, k * XB, T());
                g[PL + k] = blk[k * N * PZ + o];
            }
            sweep_x(g, p);
#pragma unroll
            for (int k = 0; k < N; ++k) {
                buf_st(g[k], rd, po, k * XB);
                mx = fmax(mx, g[k]);
            }
        }
    }
    if (max_out) block_max_part(mx, max_out);
}

// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256)
array_max_kernel(const T* __restrict__ f, long long n, typename Bits<T>::U* __restrict__ out) {
    T mx = T(0);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        mx = fmax(mx, f[i]);
    block_max_part(mx, out);
}

// Maximum of the per-block partial maxima part[0..n) into *slot (bits of
// non-negative values order like the values), in two launches: up to
// kFinStage blocks each fold a contiguous range of the partials (eight loads
// in flight per thread) into stage[b], placed right after the partials
// (fin_stage); one wave folds the stage into the slot.  With a single range
// the first launch writes the slot itself.  Fixed order.
template <class U>
__global__ void __launch_bounds__(256)
max_stage_kernel(const U* __restrict__ part, long long n, long long chunk, U* __restrict__ out) {
    __shared__ U red[256 / kWave];
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = lo + chunk < n ? lo + chunk : n;
    U m = 0;
    for (long long b = lo; b < hi; b += 8 * 256) {
        U v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const long long i = b + u * 256 + threadIdx.x;
            v[u] = i < hi ? part[i] : U(0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) m = v[u] > m ? v[u] : m;
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const U y = __shfl_xor(m, o, kWave);
        m = y > m ? y : m;
    }
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 256 / kWave; ++w) m = red[w] > m ? red[w] : m;
        out[blockIdx.x] = m;
    }
}

template <class U>
__global__ void __launch_bounds__(kWave) max_final_kernel(const U* __restrict__ stage, int g, U* __restrict__ slot) {
    U m = (int)threadIdx.x < g ? stage[threadIdx.x] : U(0);
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const U y = __shfl_xor(m, o, kWave);
        m = y > m ? y : m;
    }
    if (threadIdx.x == 0) *slot = m;
}

template <class T>
hipError_t launch_max_finalize(const void* part, long long n, void* slot, hipStream_t st) {
    using U = typename Bits<T>::U;
    const FinSplit fs = fin_split(n);
    if (fs.blocks == 1) {
        hipLaunchKernelGGL((max_stage_kernel<U>), dim3(1), dim3(256), 0, st, (const U*)part, n, n, (U*)slot);
        return hipGetLastError();
    }
    U* stage = (U*)((char*)part + fin_stage(n, sizeof(U)));
    hipLaunchKernelGGL((max_stage_kernel<U>), dim3(fs.blocks), dim3(256), 0, st, (const U*)part, n, fs.chunk, stage);
    hipLaunchKernelGGL((max_final_kernel<U>), dim3(1), dim3(kWave), 0, st, (const U*)stage, fs.blocks, (U*)slot);
    return hipGetLastError();
}

// ------------------------------------------------------------ launchers ----
// A launcher given max_out (the slot that receives the maximum of its output)
// has its kernel store per-block maxima in part (>= grid-size entries of 8
// bytes) and then reduces them into the slot.
constexpr int kChunkX = 16;

long long pfc_x_blocks(int rows, int nx, long long Nv) { return ((Nv + 255) / 256) * ((nx + kChunkX - 1) / kChunkX) * rows; }
constexpr long long kArrayMaxBlocks = 4096;

template <class T>
static hipError_t finish_max(void* max_out, void* part, long long blocks, hipStream_t st) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess || !max_out) return e;
    return launch_max_finalize<T>(part, blocks, max_out, st);
}

template <class T>
hipError_t launch_pfc_x(const T* fin, T* fout, int rows, int nx, long long Nv, int inner, double vx_lo,
                        double dvx, double tau_dx, const void* finf, void* max_out, void* part, hipStream_t st) {
    const long long blocks = pfc_x_blocks(rows, nx, Nv);
    hipLaunchKernelGGL((pfc_x_kernel<T, kChunkX>), dim3((unsigned)blocks), dim3(256), 0, st, fin, fout, nx, (int)Nv,
                       1.0f / (float)inner, vx_lo, dvx, tau_dx, (const T*)finf,
                       (typename Bits<T>::U*)(max_out ? part : nullptr));
    return finish_max<T>(max_out, part, blocks, st);
}

// x cells per thread: 8 in both storage types (FP64: 256 registers, one wave
// per SIMD, no spill; against 4 columns 3292 -> 3061 us per 1024x512x12^3
// launch and 456 -> 395 us per 256x128x16^3 launch; 12 columns: 3134 us),
// and 16 for FP32 velocity blocks of 64 KB or more (below)
template <class T> constexpr int xy_cols() { return 8; }
template <class T> constexpr int xy_cols_big() { return sizeof(T) == 4 ? 16 : 8; }

// Rows per segment of the fused X operator.  Waves in flight per CU the
// model assumes: 12 in FP32 (register-limited to 3 per SIMD), 8 in FP64 (the
// value the FP64 strip widths were measured with).  A wave walks
// S + 2 Kmax + 4 rows for S outputs.  Beyond the one-round case in
// xy_segment, the model cost rounds(S) * (S + 4 + 2 Kmax), with rounds the
// number of times the waves of the launch refill the GPU, picks the segment
// count (at most 64, segments of at least 8 rows).
static int xy_cus() {
    static int cus = 0;
    if (cus <= 0) {
        int d = 0;
        if (hipGetDevice(&d) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}
constexpr int kXyMaxSeg = 64;
static int xy_segment(int ny, long long waves_per_seg, int kb, int waves_per_cu) {
    const long long resident = (long long)waves_per_cu * xy_cus();
    // segments of 128 rows that fill at least half the GPU in one round: one
    // round of long walks (GEM 256x128x16^3: 200 us per launch against 212
    // for the two rounds of 43-row segments the cost model picks)
    const int s128 = ny < 128 ? ny : 128;
    const long long w128 = waves_per_seg * ((ny + s128 - 1) / s128);
    if (w128 <= resident && 2 * w128 >= resident) return s128;
    int bestS = ny;
    double best = 0.0;
    for (int n = 1; n <= kXyMaxSeg && n <= ny; ++n) {
        const int S = (ny + n - 1) / n;
        if (n > 1 && S < 8) break;
        if ((ny + S - 1) / S != n) continue;      // the same split as a smaller n
        const long long w = waves_per_seg * n;
        const double cost = (double)((w + resident - 1) / resident) * (double)(S + 4 + 2 * kb);
        if (n == 1 || cost < best * 0.999) {
            best = cost;
            bestS = S;
        }
    }
    return bestS;
}

static long long xy_waves_per_seg(int nx, long long Nv, int cols) {
    return ((Nv + kWave - 1) / kWave) * ((nx + cols - 1) / cols);
}

// Upper bound of the launch's blocks over every segment length it can pick
// (sizes the per-block partial maxima).
long long pfc_xy_blocks(int nx, int ny, int nvx, int nvy, int nvz) {
    const long long Nv = (long long)nvx * nvy * nvz;
    const long long nseg = ny < kXyMaxSeg ? ny : kXyMaxSeg;
    const long long w = xy_waves_per_seg(nx, Nv, 4) * nseg;    // 4 columns: a bound for every strip width
    return (w + 3) / 4;
}

template <class T, int C>
static hipError_t launch_pfc_xy_cols(const T* fin, T* fout, int nx, int ny, int nvx, int nvy, int nvz, double vx_lo,
                                     double dvx, double tau_dx, double vy_lo, double dvy, double tau_dy, int per,
                                     const void* finf, void* max_out, void* part, hipStream_t st) {
    XYArgs A;
    A.nx = nx;
    A.ny = ny;
    A.Nv = nvx * nvy * nvz;
    A.nvy = nvy;
    A.nvz = nvz;
    A.per = per;
    A.inv_nvz = 1.0f / (float)nvz;
    A.inv_nvyz = 1.0f / (float)(nvy * nvz);
    A.vx_lo = vx_lo;
    A.dvx = dvx;
    A.tau_dx = tau_dx;
    A.vy_lo = vy_lo;
    A.dvy = dvy;
    A.tau_dy = tau_dy;
    A.nchunks = (A.Nv + kWave - 1) / kWave;
    A.nst = (nx + C - 1) / C;
    // bound of the whole-cell y shift (one more than the FP64 estimate: the
    // kernel splits the shift in the storage type)
    const double vymax = fmax(fabs(vy_lo), fabs(vy_lo + nvy * dvy));
    const double kd = floor(vymax * tau_dy) + 1.0;
    const int L = per ? ny : 2 * ny;
    const int kb = kd >= (double)L ? L - 1 : (int)kd;
    A.S = xy_segment(ny, xy_waves_per_seg(nx, A.Nv, C), kb, sizeof(T) == 4 ? 12 : 8);
    A.nseg = (ny + A.S - 1) / A.S;
    const long long waves = xy_waves_per_seg(nx, A.Nv, C) * A.nseg;
    const long long blocks = (waves + 3) / 4;
    // the stores of one step span rows i-2-Kmax .. i-1+Kmax of one pass
    const size_t rowbytes = (size_t)nx * A.Nv * sizeof(T);
    const bool wide = (double)(2 * kb + 3) * (double)rowbytes >= 4294967296.0;
    auto* mo = (typename Bits<T>::U*)(max_out ? part : nullptr);
    // Workgroups resident per CU, set through a reservation of shared memory
    // the kernel does not use: with fewer waves in flight the walks of large
    // velocity blocks thrash the caches and the address translation less.
    // Measured per launch (FP32): 34^3 blocks (157 KB per cell) one workgroup
    // per CU, 12.9 -> 11.0 ms on 512x256; blocks of at most 8 KB (12^3) two,
    // 1.70 -> 1.57 ms on 1024x512; 16^3 unchanged with the register limit's
    // three (two: +1 %, one: +33 %).
    const size_t cellb = (size_t)A.Nv * sizeof(T);
    const size_t shm = cellb >= 65536 ? 102400 : (cellb <= 8192 ? 61440 : 0);
    if (wide)
        hipLaunchKernelGGL((pfc_xy_kernel<T, C, true>), dim3((unsigned)blocks), dim3(256), shm, st, fin, fout, A,
                           (const T*)finf, mo);
    else
        hipLaunchKernelGGL((pfc_xy_kernel<T, C, false>), dim3((unsigned)blocks), dim3(256), shm, st, fin, fout, A,
                           (const T*)finf, mo);
    return finish_max<T>(max_out, part, blocks, st);
}

// Columns per lane: xy_cols for most blocks; for FP32 velocity blocks of 64 KB
// or more (34^3) twice that, where the wider strip's fewer halo loads per
// output pay for the registers (one wave per SIMD; the launcher keeps one
// workgroup per CU there anyway): 11.0 -> 10.2 ms per 512x256x34^3 FP32
// launch (FP64 34^3: 8 against 4 columns, 5.28 -> 4.68 ms per 256x128x34^3
// launch).  At 12^3 and 16^3 the wider FP32 strip is 3-18 % slower, and 4,
// 6, 10 or 12 columns are slower than 8 at 12^3.
template <class T>
hipError_t launch_pfc_xy(const T* fin, T* fout, int nx, int ny, int nvx, int nvy, int nvz, double vx_lo, double dvx,
                         double tau_dx, double vy_lo, double dvy, double tau_dy, int per, const void* finf,
                         void* max_out, void* part, hipStream_t st) {
    const size_t cellb = (size_t)nvx * nvy * nvz * sizeof(T);
    if (cellb >= 65536)
        return launch_pfc_xy_cols<T, xy_cols_big<T>()>(fin, fout, nx, ny, nvx, nvy, nvz, vx_lo, dvx, tau_dx, vy_lo, dvy, tau_dy,
                                             per, finf, max_out, part, st);
    return launch_pfc_xy_cols<T, xy_cols<T>()>(fin, fout, nx, ny, nvx, nvy, nvz, vx_lo, dvx, tau_dx, vy_lo, dvy,
                                               tau_dy, per, finf, max_out, part, st);
}

template <class T>
hipError_t launch_pfc_v1(const T* fin, T* fout, int nx, int nv, const double* E, double qm_tau_dv,
                         const void* finf, void* max_out, void* part, hipStream_t st) {
    const int threads = nv >= 256 ? 256 : ((nv + 63) / 64) * 64;
    const size_t shm = sizeof(T) * (size_t)(nv + 4);
    hipLaunchKernelGGL((pfc_v1_kernel<T>), dim3(nx), dim3(threads), shm, st, fin, fout, nv, E, qm_tau_dv,
                       (const T*)finf, (typename Bits<T>::U*)(max_out ? part : nullptr));
    return finish_max<T>(max_out, part, nx, st);
}

size_t v3_shared_bytes(int nvx, int nvy, int nvz, size_t elem) {
    return elem * (size_t)nvx * nvy * (nvz | 1);
}

template <class T>
hipError_t launch_pfc_v3(const T* fin, T* fout, long long cells, const double* E, const double* B,
                         const V3Params& P, const void* finf, void* max_out, void* part, hipStream_t st) {
    const int nmax = P.nvx > P.nvy ? (P.nvx > P.nvz ? P.nvx : P.nvz) : (P.nvy > P.nvz ? P.nvy : P.nvz);
    const size_t shm = v3_shared_bytes(P.nvx, P.nvy, P.nvz, sizeof(T));
    int maxpen = P.nvx * P.nvy;
    if (P.nvx * P.nvz > maxpen) maxpen = P.nvx * P.nvz;
    if (P.nvy * P.nvz > maxpen) maxpen = P.nvy * P.nvz;
    int threads = ((maxpen + 63) / 64) * 64;
    if (threads > 256) threads = 256;
    if (threads < 64) threads = 64;
    const bool cube = P.nvx == P.nvy && P.nvy == P.nvz;
    auto* mo = (typename Bits<T>::U*)(max_out ? part : nullptr);
    const dim3 grid((unsigned)cells);
    if (cube && P.nvx == kBigCube) {
        // one cell per CU (its LDS); 578 threads = two v_x pencils each
        if constexpr (sizeof(T) == 4)
            hipLaunchKernelGGL((pfc_v3_cube_kernel<T, kBigCube, 578>), grid, dim3(578), 0, st, fin, fout, E, B, P,
                               (const T*)finf, mo);
        else        // the FP64 block is twice the LDS: half its v_x planes at a time
            hipLaunchKernelGGL((pfc_v3_planes_kernel<T, kBigCube, 512, 17>), grid, dim3(512), 0, st, fin, fout, E, B,
                               P, (const T*)finf, mo);
        return finish_max<T>(max_out, part, cells, st);
    }
    if (cube && P.nvx == 16) {
        hipLaunchKernelGGL((pfc_v3_cube_kernel<T, 16, 256>), grid, dim3(256), 0, st, fin, fout, E, B, P, (const T*)finf, mo);
    } else if (cube && P.nvx == 12) {
        hipLaunchKernelGGL((pfc_v3_cube_kernel<T, 12, 192>), grid, dim3(192), 0, st, fin, fout, E, B, P, (const T*)finf, mo);
    } else if (cube && P.nvx == 8) {
        hipLaunchKernelGGL((pfc_v3_cube_kernel<T, 8, 64>), grid, dim3(64), 0, st, fin, fout, E, B, P, (const T*)finf, mo);
    } else if (nmax <= 8) {
        hipLaunchKernelGGL((pfc_v3_kernel<T, 8>), grid, dim3(threads), shm, st, fin, fout, E, B, P, (const T*)finf, mo);
    } else if (nmax <= 16) {
        hipLaunchKernelGGL((pfc_v3_kernel<T, 16>), grid, dim3(threads), shm, st, fin, fout, E, B, P, (const T*)finf, mo);
    } else if (nmax <= 32) {
        hipLaunchKernelGGL((pfc_v3_kernel<T, 32>), grid, dim3(threads), shm, st, fin, fout, E, B, P, (const T*)finf, mo);
    } else {
        return hipErrorInvalidValue;
    }
    return finish_max<T>(max_out, part, cells, st);
}

// V(tau) by the backsubstitution split (any grid with every axis <= 32, and
// the 34^3 cube in FP32, whose padded block, 158 KB, fills one CU's LDS).
template <class T>
hipError_t launch_pfc_v3b(const T* fin, T* fout, long long cells, const double* E, const double* B,
                          const V3Params& P, const void* finf, void* max_out, void* part, hipStream_t st) {
    const int nmax = P.nvx > P.nvy ? (P.nvx > P.nvz ? P.nvx : P.nvz) : (P.nvy > P.nvz ? P.nvy : P.nvz);
    const size_t shm = v3_shared_bytes(P.nvx, P.nvy, P.nvz, sizeof(T));
    auto* mo = (typename Bits<T>::U*)(max_out ? part : nullptr);
    const dim3 grid((unsigned)cells);
    const bool cube12 = P.nvx == 12 && P.nvy == 12 && P.nvz == 12;
    if (nmax <= 8)
        hipLaunchKernelGGL((pfc_v3b_kernel<T, 8>), grid, dim3(64), shm, st, fin, fout, E, B, P, (const T*)finf, mo);
    else if (cube12)    // 144 pencils per sweep: three waves instead of four (8.2 -> 6.0 ms per
                        // 1024x512x12^3 launch)
        hipLaunchKernelGGL((pfc_v3b_kernel<T, 12, 192>), grid, dim3(192), shm, st, fin, fout, E, B, P,
                           (const T*)finf, mo);
    else if (nmax <= 16)
        hipLaunchKernelGGL((pfc_v3b_kernel<T, 16>), grid, dim3(256), shm, st, fin, fout, E, B, P, (const T*)finf, mo);
    else if (nmax <= 32)
        hipLaunchKernelGGL((pfc_v3b_kernel<T, 32>), grid, dim3(256), shm, st, fin, fout, E, B, P, (const T*)finf, mo);
    else if constexpr (sizeof(T) == 4) {
        if (nmax > kBigCube || shm > 160 * 1024) return hipErrorInvalidValue;
        // one workgroup per CU (the block fills the LDS): 1024 threads, about
        // one pencil each per sweep (1156 per sweep); 256 threads: 7.6 -> 3.0
        // ms per 128x64x34^3 launch
        hipLaunchKernelGGL((pfc_v3b_kernel<T, kBigCube, 1024>), grid, dim3(1024), shm, st, fin, fout, E, B, P,
                           (const T*)finf, mo);
    } else {
        return hipErrorInvalidValue;
    }
    return finish_max<T>(max_out, part, cells, st);
}

template <class T>
hipError_t launch_array_max(const T* f, long long n, void* out, void* part, hipStream_t st) {
    long long blocks = (n + 255) / 256;
    if (blocks > kArrayMaxBlocks) blocks = kArrayMaxBlocks;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((array_max_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, st, f, n,
                       (typename Bits<T>::U*)part);
    return finish_max<T>(out, part, blocks, st);
}

#define VL_INST(T)                                                                                         \
    template hipError_t launch_pfc_x<T>(const T*, T*, int, int, long long, int, double, double, double,     \
                                        const void*, void*, void*, hipStream_t);                           \
    template hipError_t launch_pfc_v1<T>(const T*, T*, int, int, const double*, double, const void*, void*, \
                                         void*, hipStream_t);                                              \
    template hipError_t launch_pfc_v3<T>(const T*, T*, long long, const double*, const double*,             \
                                         const V3Params&, const void*, void*, void*, hipStream_t);         \
    template hipError_t launch_pfc_v3b<T>(const T*, T*, long long, const double*, const double*,            \
                                          const V3Params&, const void*, void*, void*, hipStream_t);        \
    template hipError_t launch_array_max<T>(const T*, long long, void*, void*, hipStream_t);                \
    template hipError_t launch_pfc_xy<T>(const T*, T*, int, int, int, int, int, double, double, double, double, \
                                         double, double, int, const void*, void*, void*, hipStream_t);     \
    template hipError_t launch_max_finalize<T>(const void*, long long, void*, hipStream_t);
VL_INST(float)
VL_INST(double)
#undef VL_INST

}  // namespace vl
