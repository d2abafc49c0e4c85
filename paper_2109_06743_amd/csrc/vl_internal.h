// Internal interface between the C ABI (vl_api.hip) and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/vl.h"
#include "vl_common.h"

namespace vl {

struct VGridArgs {
    int nv[3];
    double lo[3], dv[3];
    double m;
};

struct V3Params;  // pfc_kernels.hip

template <class T>
hipError_t launch_pfc_x(const T* fin, T* fout, int rows, int nx, long long Nv, int inner, double vx_lo, double dvx,
                        double tau_dx, const void* finf, void* max_out, void* part, hipStream_t st);
template <class T>
hipError_t launch_pfc_v1(const T* fin, T* fout, int nx, int nv, const double* E, double qm_tau_dv, const void* finf,
                         void* max_out, void* part, hipStream_t st);
struct V3Params {
    int nvx, nvy, nvz;
    double lo[3], dv[3], inv_dv[3];
    double qm, tau;
    float inv_nvz;   // 1/nvz, for the exact row index (e + 0.5) / nvz of small e
};

// Row index e / n for 0 <= e < 2^16 without integer division: (e + 0.5)/n is
// at least 1/(2n) away from an integer, while the float product is off by at
// most 2^16/n * 2^-23 < 1/(2n).
__device__ __forceinline__ int row_of(int e, float inv_n) { return (int)(((float)e + 0.5f) * inv_n); }
template <class T>
hipError_t launch_pfc_v3(const T* fin, T* fout, long long cells, const double* E, const double* B, const V3Params& P,
                         const void* finf, void* max_out, void* part, hipStream_t st);
size_t v3_shared_bytes(int nvx, int nvy, int nvz, size_t elem);
// V(tau) by the backsubstitution split: three affine sweeps with per-face
// feet (every velocity axis <= 32).
template <class T>
hipError_t launch_pfc_v3b(const T* fin, T* fout, long long cells, const double* E, const double* B, const V3Params& P,
                          const void* finf, void* max_out, void* part, hipStream_t st);
template <class T>
hipError_t launch_array_max(const T* f, long long n, void* out, void* part, hipStream_t st);
// Launchers that produce a maximum store per-block partials in `part` (8 bytes
// per block of their grid) and reduce them into the slot in a second launch;
// these give the grid sizes, to size `part`.
long long pfc_x_blocks(int rows, int nx, long long Nv);
long long pfc_xy_blocks(int nx, int ny, int nvx, int nvy, int nvz);
// Fused X(tau) of 2X3V (x then y sweep, one f_inf); fout must not alias fin.
// per = 0: reflecting y walls, 1: periodic y.
template <class T>
hipError_t launch_pfc_xy(const T* fin, T* fout, int nx, int ny, int nvx, int nvy, int nvz, double vx_lo, double dvx,
                         double tau_dx, double vy_lo, double dvy, double tau_dy, int per, const void* finf,
                         void* max_out, void* part, hipStream_t st);
constexpr long long kMaxArrayBlocks = 4096;
// Reductions of per-block partials (maxima, clip counts) run in two launches:
// fin_split(n).blocks <= kFinStage blocks fold ranges of fin_split(n).chunk
// partials into a stage of kFinStage entries that sits fin_stage(n, size)
// bytes after the partials' start, then one wave folds the stage.  A partials
// buffer of n entries of `size` bytes therefore needs kFinSlack bytes beyond
// its n * size.
constexpr int kFinStage = 64;
constexpr long long kFinRange = 8192;          // partials per first-level block, at least
constexpr size_t kFinSlack = 128 + kFinStage * 8;
struct FinSplit {
    int blocks;
    long long chunk;
};
inline FinSplit fin_split(long long n) {
    long long g = (n + kFinRange - 1) / kFinRange;
    g = g < 1 ? 1 : (g > kFinStage ? kFinStage : g);
    return {(int)g, (n + g - 1) / g};
}
inline size_t fin_stage(long long n, size_t size) { return ((size_t)n * size + 127) / 128 * 128; }
template <class T>
hipError_t launch_max_finalize(const void* part, long long n, void* slot, hipStream_t st);

template <class T>
hipError_t launch_moments3(const T* f, double* mom, long long cells, const VGridArgs& a, hipStream_t st);
template <class T>
hipError_t launch_moments1(const T* f, double* mom, long long cells, int nv, double vlo, double dv, double m,
                           hipStream_t st);
// Per-cell fitting parameters (cubic velocity blocks): kFitCellDoubles doubles
// per spatial cell of device scratch.
// Edge of the large cubic velocity grid with fixed-size kernels (FP32 only:
// 34 x 34 x 35 floats = 161840 bytes of LDS per cell in the V operator).
constexpr int kBigCube = 34;
constexpr int kFitCellDoubles = 20;
template <class T>
hipError_t launch_fit3(const T* fin, T* fout, const double* mom_pre, double* U, double* mom_post, void* counters,
                       long long cells, const VGridArgs& a, void* max_out, void* part, unsigned* clip_part,
                       double* scratch, hipStream_t st);
template <class T>
hipError_t launch_fit1(const T* fin, T* fout, const double* mom_pre, double* U, double* mom_post, void* counters,
                       long long cells, int nv, double vlo, double dv, double m, void* max_out, void* part,
                       hipStream_t st);

hipError_t launch_poisson(const double* mom, int N, double L, double q, double* ab, double* E, hipStream_t st);
// mom[s]: per-cell records of mstride doubles holding n u at offsets 1..3
// (raw moments: 20; fluid state: 10).
hipError_t launch_maxwell_half(double* yee, int nx, int ny, const double* const* mom, const double* q, int ns,
                               double dt, double c, double dx, double dy, hipStream_t st, int mstride = 20,
                               int per = 0);
hipError_t launch_cell_fields(const double* yee, int nx, int ny, double* E, double* B, hipStream_t st);
hipError_t launch_field_energy(const double* fields, int dim_x, int nx, int ny, double c, double dX, double* part,
                               double* out, hipStream_t st);
hipError_t launch_axpby(const double* x, const double* y, double a, double b, double* out, long long n,
                        hipStream_t st);

// Per-species operands of one fluid stage: up to two species per launch.
struct FluidSet {
    const double* Us[2];
    const double* Un[2];
    double* Uo[2];
    const double* QA[2];
    const double* QB[2];
    double* Hx[2];
    double* Hy[2];
    double* Sg[2];        // Eq. 5 source scratch, [cells][6] (needed where gchi != 0)
    double m[2], q[2], gchi[2];
};

// Scratch of one species' SSP-RK3 step of the 3V fluid (doubles).
inline size_t fluid_rk3_3v_doubles(int nx, int ny) { return 30 * (size_t)nx * ny + 10 * (size_t)nx * (ny + 1); }

// One SSP-RK3 step of ns (1 or 2) species, each kernel launched once for all
// of them; work: ns * fluid_rk3_3v_doubles(nx, ny) doubles.
hipError_t launch_fluid_rk3_3v_set(int ns, double* const* U, const double* const* mom_t, const double* const* mom_t1,
                                   const double* E_t, const double* B_t, const double* E_t1, const double* B_t1,
                                   const double* E_th, const double* B_th, double dt, int nx, int ny, const double* q,
                                   const double* m, double dx, double dy, double* work, hipStream_t st, int per);
hipError_t launch_fluid_stage_3v_set(const FluidSet& S, int ns, double wa, double wb, const double* E,
                                     const double* B, double a, double b, double dt, int nx, int ny, double dx,
                                     double dy, hipStream_t st, int per);
hipError_t launch_fluid_rk3_3v(double* U, const double* mom_t, const double* mom_t1, const double* E_t,
                               const double* B_t, const double* E_t1, const double* B_t1, const double* E_th,
                               const double* B_th, double dt, int nx, int ny, double q, double m, double dx,
                               double dy, double* work, hipStream_t st, int per = 0);
hipError_t launch_fluid_rk3_1v(double* U, const double* mom_t, const double* mom_t1, const double* E_t,
                               const double* E_t1, const double* E_th, double dt, int nx, double q, double m,
                               double dx, double* work, hipStream_t st);

// One SSP-RK3 stage of the 3V fluid: Uo = a Un + b (Us + dt L(Us)), third
// moment wa QA + wb QB (raw-moment layout, entries 10..19 of 20 per cell).
// One RK stage of the ten-moment fluid.  gchi != 0 adds the Eq. 5
// temperature-gradient closure gchi n v_t lap T as a source of P, computed
// into Sg ([cells][6] scratch, required then).
hipError_t launch_fluid_stage_3v(const double* Us, const double* Un, double* Uo, const double* QA, const double* QB,
                                 double wa, double wb, const double* E, const double* B, double a, double b, double dt,
                                 int nx, int ny, double q, double m, double dx, double dy, double* Hx, double* Hy,
                                 hipStream_t st, double gchi = 0.0, double* Sg = nullptr, int per = 0);
// Qcal of fluid records U[cells][10] with zero heat flux, into qc[cells][20] (offsets 10..19).
hipError_t launch_qcal_q0(const double* U, long long cells, double m, double* qc, hipStream_t st);

// learned heat-flux closure (mlp_kernels.hip)
constexpr int kMlpParams = 13520;
// Per-species operands of the network kernels for up to two species per
// launch; the features, scales, outputs and third moments of the set's
// species are stored one after the other (cells of species 0, then 1).
struct MlpSet {
    const double* M[2];     // features and judge: moment (stride 20) or fluid (stride 10) records
    const double* U[2];     // qcal: the stage's fluid state
    const double* QA[2];    // qcal: kinetic third moments for the fallback
    const double* QB[2];
    int* fallback[2];       // judge output / qcal input (or null)
    double* err[2];         // judge output
    double m[2];
};
hipError_t launch_mlp_features_set(const MlpSet& S, int ns, int s0, int stride, const double* B, int nx, int ny,
                                   unsigned short* x, double* scale, hipStream_t st);
hipError_t launch_mlp_qcal_set(const MlpSet& S, int ns, const double* scale, const float* y, double wa, double wb,
                               long long cells, double* qc, hipStream_t st);
hipError_t launch_mlp_judge_set(const MlpSet& S, int ns, const double* scale, const float* y, long long cells,
                                double tol, double* part, hipStream_t st);
hipError_t launch_mlp_features(const double* M, int stride, const double* B, int nx, int ny, double m, int species,
                               unsigned short* x, double* scale, hipStream_t st);
hipError_t launch_mlp_targets(const double* M, long long cells, double m, float* y, hipStream_t st);
hipError_t launch_mlp_forward(const float* P, const unsigned short* x, long long n, float* y, hipStream_t st);
size_t mlp_grad_blocks(long long n);
size_t mlp_part_floats(long long n);
hipError_t launch_mlp_gradient(const float* P, const unsigned short* x, const float* t, long long n, float* part,
                               float* grad, hipStream_t st,
                               const long long* idx = nullptr, long long nrows = 0);
// gradient (as launch_mlp_gradient) and the Adam update of step `step`, fused
// into the gradient sum
hipError_t launch_mlp_train_step(float* P, float* m1, float* m2, long long step, double lr,
                                 const unsigned short* x, const float* t, long long n, float* part, float* grad,
                                 hipStream_t st, const long long* idx = nullptr, long long nrows = 0);
hipError_t launch_mlp_qcal(const double* U, const double* scale, const float* y, const int* fallback,
                           const double* QA, const double* QB, double wa, double wb, long long cells, double m,
                           double* qc, hipStream_t st);
size_t mlp_judge_part_doubles();
hipError_t launch_mlp_judge(const double* M, const double* scale, const float* y, long long cells, double m,
                            double tol, double* part, int* fallback, double* err, hipStream_t st);

template <class T>
hipError_t launch_mass_energy(const T* f, const double* mom, long long cells, long long nv, int kmom, int dimv,
                              double dV, double dX, double* out, double* part, hipStream_t st);

}  // namespace vl
