/*
 * vl.h - C ABI of the MI355X (gfx950) moment-fitting Vlasov hot path.
 *
 * Method: arXiv 2109.06743 (Allmann-Rahn, Lautenbach, Grauer), "An Energy
 * Conserving Vlasov Solver That Tolerates Coarse Velocity Space
 * Resolutions".  The library advances the distribution function f of each
 * species by dimensionally split PFC advection (Eq. 1; Sec. 2.1), computes
 * its velocity moments (Sec. 2.1, definitions after Eq. 1), fits the
 * ten-moment Maxwellian part of f to the fluid solver's moments (Sec. 2.2,
 * Algorithm 1) and runs the full time step of Algorithm 1 with the Yee
 * FDTD (2X3V) or spectral Poisson (1X1V) field solver and the ten-moment
 * CWENO/SSP-RK3 fluid solver.
 *
 * Conventions shared by every entry point
 * - Every large buffer is caller-owned DEVICE memory (HIP global memory on
 *   the current device).  The library never frees it.
 * - f layouts (C order, fastest index last):
 *     1X1V  f[nx][nv]
 *     2X3V  f[ny][nx][nvx][nvy][nvz]
 *   f is FP32 or FP64 as fixed by vl_config.f_dtype.  f >= 0 is required.
 * - Velocity cell centres: v_j = v_lo + (j + 1/2) (v_hi - v_lo) / n.
 *   Spatial cell centres likewise; x is periodic, y (2X3V) is bounded by
 *   conducting walls for the fields and reflecting walls for particles,
 *   which needs each species' v_y grid symmetric about 0.
 * - Moment vectors per spatial cell, FP64 (raw moments, midpoint rule):
 *     3V: [n, M1x, M1y, M1z, P(xx,xy,xz,yy,yz,zz), Q(xxx,xxy,xxz,xyy,xyz,
 *          xzz,yyy,yyz,yzz,zzz)]  (20 doubles), with P = m sum v v f dV,
 *          Q = m sum v v v f dV;
 *     1V: [n, M1, P, Q]  (4 doubles).
 * - Fluid state per spatial cell, FP64: 3V [n, nu(3), P(6)] (10 doubles),
 *   1V [n, nu, P] (3 doubles).
 * - Every call validates its arguments on the host before any launch and
 *   returns a status; nothing is thrown across the ABI.  Launches are
 *   asynchronous on the given stream (NULL = the default stream).  A device
 *   fault surfaces as VL_EHIP on a later call or on vl_sync.
 * - A context is not thread-safe; separate contexts are independent.
 */
#ifndef VL_H
#define VL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* vl_stream; /* a hipStream_t */

typedef enum {
    VL_OK = 0,
    VL_EINVAL = 1,   /* bad argument: NULL, size, non-finite or non-positive step, ... */
    VL_EALIAS = 2,   /* an output aliases an input where that is not allowed */
    VL_ENOTSUP = 3,  /* valid request the library does not implement */
    VL_EDEVICE = 4,  /* no usable HIP device */
    VL_EHIP = 5,     /* a HIP runtime call failed (message in vl_last_error) */
    VL_ENUMERIC = 6  /* non-finite values found by a guard */
} vl_status;

enum { VL_F32 = 0, VL_F64 = 1 };
enum { VL_BC_REFLECT = 0, VL_BC_PERIODIC = 1 };
enum { VL_CLOSURE_KINETIC = 0, VL_CLOSURE_MLP = 1 };
enum { VL_VSPLIT_STRANG = 0, VL_VSPLIT_BACKSUB = 1 };
enum { VL_MAX_SPECIES = 2 };

typedef struct {
    double q, m;          /* charge and mass (normalised units of Sec. 2.1 / Sec. 3.1) */
    double v_lo[3];       /* velocity box, per axis (1V uses index 0) */
    double v_hi[3];
    int32_t nv[3];        /* velocity cells per axis (1V: nv[1] = nv[2] = 1) */
} vl_species;

typedef struct {
    int32_t dim_x;        /* 1 or 2 */
    int32_t dim_v;        /* 1 (with dim_x = 1) or 3 (with dim_x = 2) */
    int32_t nx, ny;       /* spatial cells; ny = 1 when dim_x = 1 */
    double x_lo, x_hi;    /* periodic x extent */
    double y_lo, y_hi;    /* y extent between walls (2X3V) */
    int32_t bc_y;         /* 2X3V y boundary: VL_BC_REFLECT (conducting walls, reflecting f;
                             Sec. 3.3) or VL_BC_PERIODIC (Sec. 3.2); the learned closure
                             needs VL_BC_REFLECT */
    int32_t nspecies;     /* 1 .. VL_MAX_SPECIES */
    vl_species sp[VL_MAX_SPECIES];
    int32_t f_dtype;      /* VL_F32 or VL_F64 */
    double c;             /* speed of light (2X3V); eps0 = 1/c^2, mu0 = 1 */
    int32_t fit;          /* 0: standard PFC step, 1: moment fitting (Algorithm 1) */
    int32_t closure;      /* VL_CLOSURE_KINETIC: third moment from f (Algorithm 1);
                             VL_CLOSURE_MLP (2X3V with fit = 1): heat flux from the learned
                             network, the kinetic one as judge and fallback (see vl_step) */
    double closure_tol;   /* VL_CLOSURE_MLP: largest accepted relative L2 error of the network's
                             heat-flux vector against the kinetic one (e.g. 0.05) */
    int32_t vsplit;       /* 3V velocity splitting (Sec. 2.1 names "backsubstitution"):
                             VL_VSPLIT_STRANG: five uniform shear sweeps vx(tau/2) vy(tau/2)
                             vz(tau) vy(tau/2) vx(tau/2);
                             VL_VSPLIT_BACKSUB: the cell's implicit-midpoint (Boris) map of
                             the step, v -> R v + c, factored row by row into an x-, y- and
                             z-map that each change one component from the ones already
                             updated, swept with a foot per cell face (every velocity axis
                             <= 32 cells, or the 34^3 cube with FP32 f -- FP64 f on 34^3
                             gives VL_ENOTSUP; valid while |q B/m| tau < 2, a turn below
                             90 degrees per step) */
} vl_config;

typedef struct vl_ctx vl_ctx;

/* Create a context for one problem geometry.  Host-only: validates and copies
 * *cfg; device scratch (a few kilobytes, plus 160 bytes per spatial cell for
 * the 3V moment fitting on its first call) is allocated on first use on the
 * device current at that time and freed by vl_destroy.  Errors: VL_EINVAL (bad geometry, velocity
 * grid not symmetric in v_y for 2X3V), VL_ENOTSUP (unsupported combination, or a row of f --
 * nx velocity blocks -- of 4 GiB or more). */
vl_status vl_create(const vl_config* cfg, vl_ctx** out);
vl_status vl_destroy(vl_ctx* ctx);

/* Free streaming X(tau) of species s (Eq. 1, v . grad f; split PFC sweeps,
 * Sec. 2.1): x-sweep by v_x tau/dx cells (periodic), then in 2X3V a y-sweep
 * by v_y tau/dy cells between reflecting walls, both with the PFC limiter
 * bound max(f_in).  In 2X3V the two sweeps run fused in one pass (the
 * x-swept array is never stored).  f_in is not modified.  f_out must not
 * alias f_in (VL_EALIAS). */
vl_status vl_pfc_advect_x(vl_ctx* ctx, int32_t s, const void* f_in, void* f_out, double tau,
                          vl_stream stream);

/* Acceleration V(tau) of species s (Eq. 1, (q/m)(E + v x B) . grad_v f) with
 * zero-flux velocity boundaries (Sec. 2.1).  E, B are cell-centred FP64
 * fields [cells][3] (cells = ny*nx); B may be NULL (treated as 0).  1V uses
 * E[cells] (one double per cell) and ignores B.  3V with VL_VSPLIT_STRANG
 * applies the sweeps vx(tau/2) vy(tau/2) vz(tau) vy(tau/2) vx(tau/2), each a
 * uniform shift by the acceleration at the pencil's transverse velocities;
 * with VL_VSPLIT_BACKSUB the three affine sweeps of the factored Boris map
 * (see vl_config.vsplit).  Limiter bound: max of f_in.  f_out must not alias
 * f_in. */
vl_status vl_pfc_advect_v(vl_ctx* ctx, int32_t s, const void* f_in, void* f_out,
                          const double* E, const double* B, double tau, vl_stream stream);

/* Raw velocity moments of species s (Sec. 2.1) per spatial cell into mom
 * (FP64, [cells][20] in 3V, [cells][4] in 1V; layout in the header comment). */
vl_status vl_moments(vl_ctx* ctx, int32_t s, const void* f, double* mom, vl_stream stream);

/* Moment fitting of species s (Algorithm 1, "Moment Fitting"; Sec. 2.2):
 * per cell, with n_V, u_V, T_V from mom_pre (raw moments of f_in) and u_F,
 * T_F from the fluid state U, f_out = f_in - M[n_V,u_V,T_V] + M[n_V,u_F,T_F],
 * negatives set to 0, then rescaled to density n_V.  M is the ten-moment
 * Maxwellian normalised by its discrete sum.  U is rescaled by n_V/n_F in
 * place.  Cells with n_V <= 1e-12, n_F <= 1e-12 or a temperature tensor that
 * is not positive definite are copied unchanged and counted as skipped.
 * mom_post (may be NULL) receives the raw moments of f_out; counters (may
 * be NULL; int64[2] device) accumulates {clipped values, skipped cells}.
 * f_out may equal f_in (in place). */
vl_status vl_moment_fit(vl_ctx* ctx, int32_t s, const void* f_in, void* f_out, const double* mom_pre,
                        double* U, double* mom_post, int64_t* counters, vl_stream stream);

/* vl_moment_fit without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same computation and results as vl_moment_fit,
 * with its scratch (the fitting parameters of every spatial cell, 160 bytes,
 * a clip partial, 4 bytes, and 640 bytes for the sum of the clip partials)
 * in a static device array of 7.7 MiB that each
 * GPU the library runs on holds until the process ends, instead of context
 * scratch.  At most 49152 spatial cells (nx*ny): larger contexts get
 * VL_EINVAL before any device call.  The call allocates nothing (the context
 * is not used for device memory); its first call on a device looks up the
 * array's address there.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (several streams, threads or processes)
 * race and must be serialised by the caller. */
vl_status vl_moment_fit_noalloc(vl_ctx* ctx, int32_t s, const void* f_in, void* f_out, const double* mom_pre,
                                double* U, double* mom_post, int64_t* counters, vl_stream stream);

/* Fields.  1X1V: E[nx] at cell centres from Gauss's law with the uniform
 * neutralising background (Sec. 3.1), spectral, E_0 = 0.  The density is
 * taken from mom (species 0 moments, [nx][4]). */
vl_status vl_poisson(vl_ctx* ctx, const double* mom, double* E, vl_stream stream);

/* 2X3V Yee fields, FP64, concatenated: Ex[ny][nx] (i+1/2, j), Ey[ny+1][nx]
 * (i, j-1/2), Ez[ny][nx] (i, j), Bx[ny+1][nx] (i, j-1/2), By[ny][nx]
 * (i+1/2, j), Bz[ny+1][nx] (i+1/2, j-1/2); rows 0 and ny of the [ny+1]
 * arrays lie on the walls.  One Maxwell half step (Algorithm 1, first and
 * last line; the reading is B -= dt/4 curl E, E += dt/2 c^2 (curl B - j),
 * B -= dt/4 curl E) with the current j = sum_s q_s M1_s taken from the
 * species' moment arrays mom[s] ([cells][20]). */
size_t vl_yee_size(const vl_ctx* ctx);   /* doubles in the Yee array */
vl_status vl_maxwell_half_step(vl_ctx* ctx, double* yee, const double* const* mom, double dt,
                               vl_stream stream);
/* Cell-centred E, B ([cells][3] each) averaged from the Yee array. */
vl_status vl_cell_fields(vl_ctx* ctx, const double* yee, double* E, double* B, vl_stream stream);

/* One SSP-RK3 step of the ten-moment fluid (Eqs. 2-4) for species s with the
 * third moment supplied from f (Algorithm 1): Qcal at t and t+1 are taken
 * from mom_t and mom_t1 (raw moment arrays), t+1/2 is their mean.  Fields at
 * the stage times t, t+1, t+1/2: 3V E_*, B_* [cells][3]; 1V E_* [cells]
 * (B_* ignored).  U is updated in place.  work: vl_fluid_work_size doubles. */
size_t vl_fluid_work_size(const vl_ctx* ctx);
vl_status vl_fluid_step(vl_ctx* ctx, int32_t s, double* U, const double* mom_t, const double* mom_t1,
                        const double* E_t, const double* B_t, const double* E_t1, const double* B_t1,
                        const double* E_th, const double* B_th, double dt, double* work,
                        vl_stream stream);

/* Full time step (Algorithm 1).  All pointers are device buffers.
 *   f[s]        in: f^t, out: f^{t+1}
 *   f_tmp[s]    scratch of the same size as f[s] (holds f between X(dt/2) and
 *               the second X(dt/2))
 *   mom_post[s] in: raw moments of f^t; out: of f^{t+1} (after fitting)
 *   mom_pre[s]  out: raw moments of f^{t+1} before fitting
 *   U[s]        fluid state (used when fit = 1), in/out
 *   fields      2X3V: the Yee array (in/out); 1X1V: E at t+1/2 (out, [nx])
 *   work        vl_step_work_size doubles of scratch
 *   counters    int64[2] {clipped, skipped} accumulated, or NULL
 * Sequence (2X3V): Maxwell half step with j^t; X(dt/2); V(dt) with the
 * cell-centred fields at t+1/2; X(dt/2); raw moments; fluid RK3 with Qcal at
 * t, t+1, t+1/2; moment fitting; Maxwell half step with j^{t+1}.  1X1V: X(dt/2);
 * Poisson; V(dt); X(dt/2); moments; fluid; fitting.  fit = 0 skips fluid and
 * fitting (standard PFC step, mom_post = mom_pre).
 * f_max_valid: host flag; 0 tells the step to compute max f[s] itself, the
 * step sets it to 1 (the maximum of f^{t+1} is kept in the context for the
 * next step).  Set it to 0 whenever f changes outside vl_step.
 * Graph capture (the kinetic closure): every launch goes to `stream`, with no
 * memset and no host synchronisation; the context allocates its scratch on
 * first use, so after one eager vl_step on a state with f_max_valid = 1 a
 * vl_step captured on `stream` replays as further steps of that state (the
 * buffers are the ones named at capture). */
typedef struct {
    void* f[VL_MAX_SPECIES];
    void* f_tmp[VL_MAX_SPECIES];
    double* mom_post[VL_MAX_SPECIES];
    double* mom_pre[VL_MAX_SPECIES];
    double* U[VL_MAX_SPECIES];
    double* fields;
    double* work;
    int64_t* counters;
    int32_t f_max_valid;
    /* VL_CLOSURE_MLP only (NULL otherwise) */
    const float* mlp_params;    /* VL_MLP_NPARAM network parameters (device) */
    int32_t* closure_fallback;  /* out, int32[nspecies] (device): 1 where the step used the kinetic
                                   third moment because the network's error exceeded closure_tol */
    double* closure_err;        /* out, double[nspecies] (device): that relative L2 error */
} vl_state;

size_t vl_step_work_size(const vl_ctx* ctx);
vl_status vl_step(vl_ctx* ctx, vl_state* st, double dt, vl_stream stream);
/* With closure = VL_CLOSURE_MLP the fluid RK3 of every species takes its
 * third moment at each stage from the network applied to that stage's fluid
 * state and that stage's magnetic field (Q-calligraphic = Q_net + sym(u P) -
 * 2 m n uuu), instead of from f.
 * Before the fluid update the network is judged on the moments of f^{t+1}:
 * the relative L2 error (over the species' cells) of its heat-flux vector
 * q_i = Q_ijj against the kinetic one goes to closure_err[s]; above
 * closure_tol the step uses the kinetic third moment instead (as with
 * VL_CLOSURE_KINETIC) and sets closure_fallback[s].  No host synchronisation:
 * the decision is taken on the device. */

/* ---- Ten-moment multi-fluid step with a heat-flux closure (2X3V) ----------
 * The fluid solver of Sec. 2.3 run on its own, without a distribution
 * function (the paper's gradient-closure fluid model).  One step:
 * Maxwell half step with j^t = sum_s q_s (n u)_s taken from the fluid states;
 * per species one SSP-RK3 step of Eqs. 2-4 with the fields at t, t+1
 * (extrapolated, 2 X^{t+1/2} - X^t) and t+1/2 as in vl_step, whose third
 * moment at every stage is a closure of that stage's state; Maxwell half step
 * with j^{t+1}.
 *   VL_FLUID_GRADIENT  zero heat flux in the faces' third moment
 *                      (Qcal = sym(u P) - 2 m n uuu) and Eq. 5 as a source of
 *                      P: -div Q = (chi/k0) n v_t lap T, chi = 2 sqrt(2/pi),
 *                      k0 = 1/d_s, d_s = sqrt(m/q^2) (reference density 1),
 *                      v_t = sqrt(tr T / (3 m)), lap T by central second
 *                      differences (x periodic, y walls mirrored);
 *   VL_FLUID_MLP       the network's heat flux at every stage (as the learned
 *                      closure of vl_step, without the judge: there is no
 *                      kinetic reference), from that stage's state and B.
 * U[s] ([cells][10], FP64) and fields (the Yee array) are advanced in place;
 * work: vl_fluid_closure_work_size doubles; mlp_params (device, VL_MLP_NPARAM
 * floats) only for VL_FLUID_MLP.  Errors: VL_ENOTSUP unless the context is
 * 2X3V; VL_EINVAL for a null buffer, an unknown closure or dt not finite and
 * > 0; VL_EALIAS if U[0] == U[1]. */
enum { VL_FLUID_GRADIENT = 0, VL_FLUID_MLP = 1 };
typedef struct {
    double* U[VL_MAX_SPECIES];
    double* fields;
    double* work;
    const float* mlp_params;
} vl_fluid_state;
size_t vl_fluid_closure_work_size(const vl_ctx* ctx);   /* 0 unless 2X3V */
vl_status vl_fluid_closure_step(vl_ctx* ctx, vl_fluid_state* st, int32_t closure, double dt, vl_stream stream);

/* ---- Learned heat-flux closure (a network of this library, not of the paper;
 * the paper's fluid-only closure is the temperature-gradient one, Eq. 5).
 * Network: features (64) -> tanh 64 -> tanh 64 -> tanh 64 -> 16 outputs, of
 * which the first 10 are the heat-flux tensor Q_ijk / (n m v_t^3) in the
 * order xxx,xxy,xxz,xyy,xyz,xzz,yyy,yyz,yzz,zzz (v_t^2 = tr(T)/(3m)).
 * Parameters: one FP32 vector of VL_MLP_NPARAM values, row-major [out][in]:
 * W1[64][64] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[16][64] b4[16];
 * rows 10..15 of W4 and b4 are padding (kept 0 by training).  Products use
 * BF16-rounded weights and activations with FP32 accumulation (MFMA). */
enum { VL_MLP_IN = 64, VL_MLP_WIDTH = 64, VL_MLP_OUT = 10, VL_MLP_OUT_PAD = 16, VL_MLP_NPARAM = 13520 };

/* Features of every spatial cell of species s (2X3V) from a moment array whose
 * first ten entries per cell are (n, nu, P): raw moments (stride 20) or a
 * fluid state (stride 10), and the cell-centred magnetic field B [cells][3]
 * (may be NULL: zero direction).  x: uint16 BF16 [cells][64]; scale: double
 * [cells] = n m v_t^3 (0 for a cell with n <= 1e-12 or tr T <= 0, whose
 * features are 0).  Features: u/v_t, T/T_ref, then for n/n_c, u/v_t, T/T_ref
 * on the 3x3 stencil the differences d_x, d_y, d_xx, d_yy, d_xy (grid units;
 * x periodic, y mirrored at the walls), a species one-hot, B/|B|.  The heat
 * flux follows the field direction (Sec. 4.1 discussion), which a
 * temperature-gradient closure cannot represent. */
vl_status vl_mlp_features(vl_ctx* ctx, int32_t s, const double* mom, int32_t stride, const double* B,
                          uint16_t* x, double* scale, vl_stream stream);
/* Training targets: normalised kinetic heat flux [cells][16] (FP32, entries
 * 10..15 zero) from raw moments [cells][20] of species s. */
vl_status vl_mlp_targets(vl_ctx* ctx, int32_t s, const double* mom, float* y, vl_stream stream);
/* y[n][16] = network(x[n][64]).  n >= 1.  x must be 8-byte and y 16-byte
 * aligned (VL_EINVAL otherwise), as for the training calls below. */
vl_status vl_mlp_forward(vl_ctx* ctx, const float* params, const uint16_t* x, int64_t n, float* y,
                         vl_stream stream);
/* Scratch (floats) for vl_mlp_gradient / vl_mlp_train_step with n samples. */
size_t vl_mlp_work_size(int64_t n);
/* Mean squared error over the n samples and 10 outputs and its gradient:
 * grad_loss[0..VL_MLP_NPARAM-1] = gradient, grad_loss[VL_MLP_NPARAM] = loss
 * (FP32, device).  Deterministic (fixed-order sums). */
vl_status vl_mlp_gradient(vl_ctx* ctx, const float* params, const uint16_t* x, const float* y, int64_t n,
                          float* work, float* grad_loss, vl_stream stream);
/* vl_mlp_gradient followed by one Adam step (beta1 0.9, beta2 0.999, eps 1e-8,
 * bias correction with the 1-based step) on params, with moment vectors
 * adam_m, adam_v (VL_MLP_NPARAM floats each, zero before step 1). */
vl_status vl_mlp_train_step(vl_ctx* ctx, float* params, float* adam_m, float* adam_v, int64_t step, double lr,
                            const uint16_t* x, const float* y, int64_t n, float* work, float* grad_loss,
                            vl_stream stream);
/* nsteps Adam steps as vl_mlp_train_step, step k (0-based) on the batch of
 * rows idx[k*batch .. (k+1)*batch) of x ([nrows][64] BF16) and y ([nrows][16]
 * FP32): the rows are gathered inside the gradient kernel, and the steps run
 * with the 1-based Adam steps step0 .. step0 + nsteps - 1.  idx: device int64
 * array of nsteps*batch entries; an entry outside [0, nrows) counts as a
 * padding row (no features, no loss) but still in the batch's mean.  work:
 * vl_mlp_work_size(batch) floats.  grad_loss ends with the last step's
 * gradient and loss.  Same results as nsteps calls of vl_mlp_train_step on the
 * gathered batches. */
vl_status vl_mlp_train_epoch(vl_ctx* ctx, float* params, float* adam_m, float* adam_v, int64_t step0, double lr,
                             const uint16_t* x, const float* y, int64_t nrows, const int64_t* idx, int64_t batch,
                             int64_t nsteps, float* work, float* grad_loss, vl_stream stream);

/* Diagnostics: total mass of species s (sum f dV dX, FP64) and the
 * kinetic+thermal energy sum tr(P)/2 dX (3V) or P/2 dX (1V) from a raw
 * moment array, written to out[0..1] (device doubles). */
vl_status vl_mass_energy(vl_ctx* ctx, int32_t s, const void* f, const double* mom, double* out,
                         vl_stream stream);
/* Field energy (Sec. 3.2 energy budget) written to *out (device double).
 * 2X3V: sum over the Yee points of B^2/2 + E^2/(2 c^2) times the cell area,
 * points on the walls (rows 0 and ny of Ey, Bx, Bz) at half weight; fields is
 * the Yee array.  1X1V: sum of E^2/2 dx over fields = E[nx].  Fixed-order
 * sums (deterministic).  2X3V needs ny < 1024. */
vl_status vl_field_energy(vl_ctx* ctx, const double* fields, double* out, vl_stream stream);

/* Kernel timing (tracing aid).  mask selects categories: bit k (1u << VL_T_k)
 * brackets every launch group of category k issued by the entry points of
 * ctx with two HIP events recorded on the stream it runs on; 0 turns timing
 * off, VL_T_ALL times everything.  Each bracket adds two event records to the
 * stream, so timing few categories perturbs the step least.  vl_timing_read
 * waits for the recorded events, returns the summed milliseconds and
 * launch-group counts per category (arrays of VL_T_COUNT entries) since the
 * previous read, and clears them. */
enum { VL_T_MAX = 0, VL_T_PFC_X, VL_T_PFC_Y, VL_T_PFC_V, VL_T_MOMENTS, VL_T_FLUID, VL_T_FIT, VL_T_FIELDS,
       VL_T_COPY, VL_T_COUNT };
#define VL_T_ALL ((uint32_t)((1u << VL_T_COUNT) - 1u))
vl_status vl_timing_enable(vl_ctx* ctx, uint32_t mask);
vl_status vl_timing_read(vl_ctx* ctx, double* ms, int64_t* count);

vl_status vl_sync(vl_ctx* ctx, vl_stream stream);       /* wait for the stream, report device errors */
const char* vl_status_str(vl_status st);
const char* vl_last_error(const vl_ctx* ctx);          /* message of the last failure on ctx */
const char* vl_version(void);

#ifdef __cplusplus
}
#endif
#endif /* VL_H */
