// C ABI of the moment-fitting Vlasov hot path (include/vl.h): host-side
// validation, dispatch on the storage type of f, and the orchestration of the
// full time step (Algorithm 1 of arXiv 2109.06743) as a sequence of kernel
// launches on one stream.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "vl_internal.h"

struct vl_timer {
    hipEvent_t start, stop;
    int cat;
};

struct vl_ctx {
    vl_config cfg;
    int device = -1;
    // kernel timing (vl_timing_enable / vl_timing_read)
    uint32_t timing = 0;   // bit k: time launch groups of category k
    std::vector<vl_timer> pending;
    std::vector<hipEvent_t> pool;
    double t_ms[VL_T_COUNT] = {0};
    int64_t t_cnt[VL_T_COUNT] = {0};
    // device scratch: kSlots maxima per species, then the DFT coefficients,
    // then the diagnostics partials
    unsigned long long* slots = nullptr;
    double* dft = nullptr;
    double* part = nullptr;
    long long cells = 0;
    long long nv[VL_MAX_SPECIES] = {0, 0};
    // per-cell fitting parameters (3V), allocated on the first fit
    double* fit_scratch = nullptr;
    // per-block partial maxima (8 bytes each) and clip counts (4 bytes each)
    // of the largest grid any launch of this geometry uses
    void* bpart = nullptr;
    unsigned* bclip = nullptr;
    long long max_blocks = 0;
    char err[512] = {0};
};

namespace {

constexpr int kSlots = 4;   // A: input of the step, B: after first X, C: after V, S: standalone
constexpr int kPartials = 1024;

vl_status fail(vl_ctx* c, vl_status st, const char* fmt, ...) {
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(c->err, sizeof(c->err), fmt, ap);
        va_end(ap);
    }
    return st;
}

#define VL_HIP(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess) return fail(ctx, VL_EHIP, "%s: %s", #call, hipGetErrorString(e_));       \
    } while (0)

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

hipEvent_t take_event(vl_ctx* c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    // timing only: no system-scope fence at the record (the host never reads
    // memory through these events), which also keeps the records from
    // stretching the gaps between the timed kernel and its neighbours
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

// Brackets the launches issued during its lifetime with events on `st` when
// timing is enabled on the context.
struct Timed {
    vl_ctx* c;
    hipStream_t st;
    vl_timer t{};
    bool on;
    Timed(vl_ctx* c_, int cat, hipStream_t st_) : c(c_), st(st_), on(((c_->timing >> cat) & 1u) != 0) {
        if (!on) return;
        t.cat = cat;
        t.start = take_event(c);
        t.stop = take_event(c);
        on = t.start && t.stop;
        if (on) (void)hipEventRecord(t.start, st);
    }
    ~Timed() {
        if (!on) return;
        (void)hipEventRecord(t.stop, st);
        c->pending.push_back(t);
    }
};

double dx_of(const vl_config& c) { return (c.x_hi - c.x_lo) / c.nx; }
double dy_of(const vl_config& c) { return c.dim_x == 2 ? (c.y_hi - c.y_lo) / c.ny : 1.0; }
double dv_of(const vl_species& s, int d) { return (s.v_hi[d] - s.v_lo[d]) / s.nv[d]; }

unsigned long long* slot(vl_ctx* c, int which, int s) { return c->slots + which * VL_MAX_SPECIES + s; }

vl_status ensure_device(vl_ctx* ctx) {
    int dev = -1;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return fail(ctx, VL_EDEVICE, "no HIP device");
    if (hipGetDevice(&dev) != hipSuccess) return fail(ctx, VL_EDEVICE, "hipGetDevice failed");
    if (ctx->slots && ctx->device == dev) return VL_OK;
    if (ctx->slots && ctx->device != dev)
        return fail(ctx, VL_EDEVICE, "context was first used on device %d, current device is %d", ctx->device, dev);
    const size_t bytes = sizeof(unsigned long long) * kSlots * VL_MAX_SPECIES +
                         sizeof(double) * (2 * (size_t)ctx->cfg.nx + 2 + kPartials);
    void* p = nullptr;
    VL_HIP(hipMalloc(&p, bytes));
    VL_HIP(hipMemset(p, 0, bytes));
    void* q = nullptr;
    // per-block maxima (8 bytes a block), then the clip counts (4 bytes), each
    // followed by the stage of its two-level reduction
    const size_t part_bytes = 8 * (size_t)ctx->max_blocks + vl::kFinSlack;
    VL_HIP(hipMalloc(&q, part_bytes + 4 * (size_t)ctx->max_blocks + vl::kFinSlack));
    ctx->bpart = q;
    ctx->bclip = (unsigned*)((char*)q + part_bytes);
    ctx->slots = (unsigned long long*)p;
    ctx->dft = (double*)(ctx->slots + kSlots * VL_MAX_SPECIES);
    ctx->part = ctx->dft + 2 * (size_t)ctx->cfg.nx + 2;
    ctx->device = dev;
    return VL_OK;
}

vl_status check_species(vl_ctx* ctx, int32_t s) {
    if (!ctx) return VL_EINVAL;
    if (s < 0 || s >= ctx->cfg.nspecies) return fail(ctx, VL_EINVAL, "species index %d out of range", s);
    return VL_OK;
}

int per_y(const vl_config& c) { return c.dim_x == 2 && c.bc_y == VL_BC_PERIODIC ? 1 : 0; }

size_t yee_doubles(const vl_config& c) {
    return c.dim_x == 2 ? (size_t)c.nx * (3 * (size_t)c.ny + 3 * ((size_t)c.ny + 1)) : 0;
}

size_t fluid_doubles(const vl_config& c) {
    if (c.dim_v == 3) return vl::fluid_rk3_3v_doubles(c.nx, c.ny);
    return 9 * (size_t)c.nx;
}

// Learned-closure scratch of the step: features (BF16 [cells][64] = 16
// doubles per cell), scale (1), network outputs (FP32 [cells][16] = 8), third
// moment (20 per cell, raw-moment layout), judge partials.
size_t mlp_step_doubles(const vl_config& c) {
    if (c.closure != VL_CLOSURE_MLP) return 0;
    const size_t cells = (size_t)c.nx * c.ny;
    return (size_t)c.nspecies * (45 * cells + vl::mlp_judge_part_doubles()) + 2;   // every species at once
}

// Fluid-only closure step: the step's field arrays, the fluid scratch, the
// third moment (20 per cell), the Eq. 5 source (6 per cell) and the
// network's scratch (25 per cell + 2).
size_t fluid_closure_doubles(const vl_config& c) {
    const size_t cells = (size_t)c.nx * c.ny;
    return 18 * cells + fluid_doubles(c) + 20 * cells + 6 * cells + 25 * cells + 2;
}

size_t step_doubles(const vl_config& c) {
    const size_t cells = (size_t)c.nx * c.ny;
    // the fluid steps of all species run together (a fluid scratch each)
    if (c.dim_v == 3) return 18 * cells + (size_t)c.nspecies * fluid_doubles(c) + mlp_step_doubles(c);
    return 4 * (size_t)c.nx + 3 * (size_t)c.nx + fluid_doubles(c);
}

// ------------------------------------------------------------ typed paths --
template <class T>
vl_status advect_x_typed(vl_ctx* ctx, int s, const T* fin, T* fout, double tau, const void* finf,
                         void* max_x, void* max_y, hipStream_t st) {
    const vl_config& c = ctx->cfg;
    const vl_species& sp = c.sp[s];
    if (c.dim_x == 1) {
        Timed tm(ctx, VL_T_PFC_X, st);
        VL_HIP((vl::launch_pfc_x<T>(fin, fout, 1, c.nx, sp.nv[0], 1, sp.v_lo[0], dv_of(sp, 0), tau / dx_of(c), finf,
                                    max_x, ctx->bpart, st)));
        return VL_OK;
    }
    // 2X3V: x and y sweeps fused into one pass (the x-swept array stays in registers)
    Timed tm(ctx, VL_T_PFC_X, st);
    VL_HIP((vl::launch_pfc_xy<T>(fin, fout, c.nx, c.ny, sp.nv[0], sp.nv[1], sp.nv[2], sp.v_lo[0], dv_of(sp, 0),
                                 tau / dx_of(c), sp.v_lo[1], dv_of(sp, 1), tau / dy_of(c),
                                 c.bc_y == VL_BC_PERIODIC ? 1 : 0, finf, max_y, ctx->bpart, st)));
    return VL_OK;
}

template <class T>
vl_status advect_v_typed(vl_ctx* ctx, int s, const T* fin, T* fout, const double* E, const double* B, double tau,
                         const void* finf, void* max_out, hipStream_t st) {
    const vl_config& c = ctx->cfg;
    const vl_species& sp = c.sp[s];
    Timed tm(ctx, VL_T_PFC_V, st);
    if (c.dim_v == 1) {
        VL_HIP((vl::launch_pfc_v1<T>(fin, fout, c.nx, sp.nv[0], E, sp.q / sp.m * tau / dv_of(sp, 0), finf, max_out,
                                     ctx->bpart, st)));
        return VL_OK;
    }
    vl::V3Params P;
    P.nvx = sp.nv[0];
    P.nvy = sp.nv[1];
    P.nvz = sp.nv[2];
    for (int d = 0; d < 3; ++d) {
        P.lo[d] = sp.v_lo[d];
        P.dv[d] = dv_of(sp, d);
        P.inv_dv[d] = 1.0 / P.dv[d];
    }
    P.qm = sp.q / sp.m;
    P.tau = tau;
    P.inv_nvz = 1.0f / (float)sp.nv[2];
    if (c.vsplit == VL_VSPLIT_BACKSUB)
        VL_HIP((vl::launch_pfc_v3b<T>(fin, fout, ctx->cells, E, B, P, finf, max_out, ctx->bpart, st)));
    else
        VL_HIP((vl::launch_pfc_v3<T>(fin, fout, ctx->cells, E, B, P, finf, max_out, ctx->bpart, st)));
    return VL_OK;
}

vl::VGridArgs grid_args(const vl_species& sp) {
    vl::VGridArgs a;
    for (int d = 0; d < 3; ++d) {
        a.nv[d] = sp.nv[d];
        a.lo[d] = sp.v_lo[d];
        a.dv[d] = dv_of(sp, d);
    }
    a.m = sp.m;
    return a;
}

template <class T>
vl_status moments_typed(vl_ctx* ctx, int s, const T* f, double* mom, hipStream_t st) {
    const vl_config& c = ctx->cfg;
    const vl_species& sp = c.sp[s];
    Timed tm(ctx, VL_T_MOMENTS, st);
    if (c.dim_v == 1)
        VL_HIP((vl::launch_moments1<T>(f, mom, ctx->cells, sp.nv[0], sp.v_lo[0], dv_of(sp, 0), sp.m, st)));
    else
        VL_HIP((vl::launch_moments3<T>(f, mom, ctx->cells, grid_args(sp), st)));
    return VL_OK;
}

template <class T>
vl_status fit_typed(vl_ctx* ctx, int s, const T* fin, T* fout, const double* mom_pre, double* U, double* mom_post,
                    int64_t* counters, void* max_out, hipStream_t st) {
    const vl_config& c = ctx->cfg;
    const vl_species& sp = c.sp[s];
    Timed tm(ctx, VL_T_FIT, st);
    if (c.dim_v == 1)
        VL_HIP((vl::launch_fit1<T>(fin, fout, mom_pre, U, mom_post, counters, ctx->cells, sp.nv[0], sp.v_lo[0],
                                   dv_of(sp, 0), sp.m, max_out, ctx->bpart, st)));
    else {
        if (!ctx->fit_scratch) {
            void* p = nullptr;
            VL_HIP(hipMalloc(&p, sizeof(double) * vl::kFitCellDoubles * (size_t)ctx->cells));
            ctx->fit_scratch = (double*)p;
        }
        VL_HIP((vl::launch_fit3<T>(fin, fout, mom_pre, U, mom_post, counters, ctx->cells, grid_args(sp), max_out,
                                   ctx->bpart, ctx->bclip, ctx->fit_scratch, st)));
    }
    return VL_OK;
}

template <class T>
vl_status array_max_typed(vl_ctx* ctx, int s, const T* f, void* out, hipStream_t st) {
    Timed tm(ctx, VL_T_MAX, st);
    VL_HIP((vl::launch_array_max<T>(f, ctx->cells * ctx->nv[s], out, ctx->bpart, st)));
    return VL_OK;
}

vl_status fluid_step_impl(vl_ctx* ctx, int s, double* U, const double* mom_t, const double* mom_t1, const double* E_t,
                          const double* B_t, const double* E_t1, const double* B_t1, const double* E_th,
                          const double* B_th, double dt, double* work, hipStream_t st) {
    const vl_config& c = ctx->cfg;
    const vl_species& sp = c.sp[s];
    Timed tm(ctx, VL_T_FLUID, st);
    if (c.dim_v == 3)
        VL_HIP(vl::launch_fluid_rk3_3v(U, mom_t, mom_t1, E_t, B_t, E_t1, B_t1, E_th, B_th, dt, c.nx, c.ny, sp.q, sp.m,
                                       dx_of(c), dy_of(c), work, st, per_y(c)));
    else
        VL_HIP(vl::launch_fluid_rk3_1v(U, mom_t, mom_t1, E_t, E_t1, E_th, dt, c.nx, sp.q, sp.m, dx_of(c), work, st));
    return VL_OK;
}

// Fluid RK3 of all species with the learned third moment (2X3V): judge the
// network on the moments of f^{t+1}, then run the three stages, each with
// the network's Q-calligraphic of that stage's state, or the kinetic one for
// a species whose judge set the fallback flag.  Each kernel is launched once
// for all species; their features, outputs and third moments are stored one
// species after the other in mwork.
vl_status fluid_step_mlp_all(vl_ctx* ctx, const vl_state* S, const double* E_t, const double* B_t,
                             const double* E_t1, const double* B_t1, const double* E_th, const double* B_th,
                             double dt, double* fwork, double* mwork, hipStream_t st) {
    const vl_config& c = ctx->cfg;
    const int ns = c.nspecies;
    const long long cells = ctx->cells;
    float* y = (float*)mwork;                           // 16-byte aligned (the caller aligns mwork)
    unsigned short* x = (unsigned short*)(mwork + 8 * ns * cells);
    double* scale = mwork + 24 * ns * cells;
    double* qc = mwork + 25 * ns * cells;
    double* part = mwork + 45 * ns * cells;
    Timed tm(ctx, VL_T_FLUID, st);
    vl::MlpSet J{};
    for (int s = 0; s < ns; ++s) {
        J.M[s] = S->mom_pre[s];
        J.m[s] = c.sp[s].m;
        J.fallback[s] = S->closure_fallback + s;
        J.err[s] = S->closure_err + s;
    }
    VL_HIP(vl::launch_mlp_features_set(J, ns, 0, 20, B_t1, c.nx, c.ny, x, scale, st));
    VL_HIP(vl::launch_mlp_forward(S->mlp_params, x, ns * cells, y, st));
    VL_HIP(vl::launch_mlp_judge_set(J, ns, scale, y, cells, c.closure_tol, part, st));
    const double wa[3] = {1.0, 1.0, 0.5}, wb[3] = {0.0, 0.0, 0.5};
    const double a[3] = {0.0, 0.75, 1.0 / 3.0}, b[3] = {1.0, 0.25, 2.0 / 3.0};
    const double* E[3] = {E_t, E_t1, E_th};
    const double* B[3] = {B_t, B_t1, B_th};
    for (int k = 0; k < 3; ++k) {
        vl::MlpSet F{};
        vl::FluidSet G{};
        for (int s = 0; s < ns; ++s) {
            double* U = S->U[s];
            double* U1 = fwork + (size_t)s * fluid_doubles(c);
            double* U2 = U1 + cells * 10;
            const double* Us[3] = {U, U1, U2};
            double* Uo[3] = {U1, U2, U};
            const double* QA[3] = {S->mom_post[s], S->mom_pre[s], S->mom_post[s]};
            const double* QB[3] = {S->mom_post[s], S->mom_pre[s], S->mom_pre[s]};
            F.M[s] = Us[k];
            F.U[s] = Us[k];
            F.QA[s] = QA[k];
            F.QB[s] = QB[k];
            F.fallback[s] = S->closure_fallback + s;
            F.m[s] = c.sp[s].m;
            G.Us[s] = Us[k];
            G.Un[s] = U;
            G.Uo[s] = Uo[k];
            G.QA[s] = qc + (size_t)s * 20 * cells;
            G.QB[s] = G.QA[s];
            G.Hx[s] = U2 + cells * 10;
            G.Hy[s] = G.Hx[s] + cells * 10;
            G.Sg[s] = nullptr;
            G.m[s] = c.sp[s].m;
            G.q[s] = c.sp[s].q;
            G.gchi[s] = 0.0;
        }
        VL_HIP(vl::launch_mlp_features_set(F, ns, 0, 10, B[k], c.nx, c.ny, x, scale, st));
        VL_HIP(vl::launch_mlp_forward(S->mlp_params, x, ns * cells, y, st));
        VL_HIP(vl::launch_mlp_qcal_set(F, ns, scale, y, wa[k], wb[k], cells, qc, st));
        VL_HIP(vl::launch_fluid_stage_3v_set(G, ns, 1.0, 0.0, E[k], B[k], a[k], b[k], dt, c.nx, c.ny, dx_of(c),
                                             dy_of(c), st, per_y(c)));
    }
    return VL_OK;
}

// Ten-moment multi-fluid step without a distribution function (the fluid
// solver of Sec. 2.3 run on its own): the field half steps of the Vlasov step
// with the currents q n u of the fluid states, and per species the SSP-RK3
// step whose third moment at every stage comes from a closure of that
// stage's state: zero heat flux with the temperature-gradient closure of
// Eq. 5 as a source of P, or the heat flux of the network.
vl_status fluid_closure_step_impl(vl_ctx* ctx, const vl_fluid_state* S, int closure, double dt, hipStream_t st) {
    const vl_config& c = ctx->cfg;
    const int ns = c.nspecies;
    const long long cells = ctx->cells;
    const double q[2] = {c.sp[0].q, ns > 1 ? c.sp[1].q : 0.0};
    double* E_t = S->work;
    double* B_t = E_t + 3 * cells;
    double* E_h = B_t + 3 * cells;
    double* B_h = E_h + 3 * cells;
    double* E_1 = B_h + 3 * cells;
    double* B_1 = E_1 + 3 * cells;
    double* fwork = B_1 + 3 * cells;
    double* qc = fwork + fluid_doubles(c);
    double* sg = qc + 20 * cells;                         // Eq. 5 source of P, [cells][6]
    double* mw = sg + 6 * cells;
    mw += ((uintptr_t)mw & 15u) ? 1 : 0;                 // network outputs are stored as 16-byte vectors
    float* y = (float*)mw;
    unsigned short* x = (unsigned short*)(mw + 8 * cells);
    double* scale = mw + 24 * cells;
    const double* Uc[2] = {S->U[0], ns > 1 ? S->U[1] : nullptr};
    {
        Timed tm(ctx, VL_T_FIELDS, st);
        VL_HIP(vl::launch_cell_fields(S->fields, c.nx, c.ny, E_t, B_t, st));   // the fields at t
        VL_HIP(vl::launch_maxwell_half(S->fields, c.nx, c.ny, Uc, q, ns, dt, c.c, dx_of(c), dy_of(c), st, 10,
                                       per_y(c)));
        VL_HIP(vl::launch_cell_fields(S->fields, c.nx, c.ny, E_h, B_h, st));
        // E^1 = 2 E^{t+1/2} - E^t and the same for B (E and B arrays adjacent)
        VL_HIP(vl::launch_axpby(E_h, E_t, 2.0, -1.0, E_1, 6 * cells, st));
    }
    for (int s = 0; s < ns; ++s) {
        const vl_species& sp = c.sp[s];
        Timed tm(ctx, VL_T_FLUID, st);
        double* U = S->U[s];
        double* U1 = fwork;
        double* U2 = U1 + cells * 10;
        double* Hx = U2 + cells * 10;
        double* Hy = Hx + cells * 10;
        struct Stage { const double* Us; double* Uo; const double* E; const double* B; double a, b; };
        const Stage G[3] = {
            {U, U1, E_t, B_t, 0.0, 1.0},
            {U1, U2, E_1, B_1, 0.75, 0.25},
            {U2, U, E_h, B_h, 1.0 / 3.0, 2.0 / 3.0},
        };
        // chi / k0 with chi = 2 sqrt(2/pi), k0 = 1/d_s, d_s = sqrt(m / q^2)
        const double gchi = 2.0 * sqrt(2.0 / 3.14159265358979323846) * sqrt(sp.m / (sp.q * sp.q));
        for (int k = 0; k < 3; ++k) {
            if (closure == VL_FLUID_GRADIENT) {
                VL_HIP(vl::launch_qcal_q0(G[k].Us, cells, sp.m, qc, st));
            } else {
                VL_HIP(vl::launch_mlp_features(G[k].Us, 10, G[k].B, c.nx, c.ny, sp.m, s, x, scale, st));
                VL_HIP(vl::launch_mlp_forward(S->mlp_params, x, cells, y, st));
                VL_HIP(vl::launch_mlp_qcal(G[k].Us, scale, y, nullptr, qc, qc, 1.0, 0.0, cells, sp.m, qc, st));
            }
            VL_HIP(vl::launch_fluid_stage_3v(G[k].Us, U, G[k].Uo, qc, qc, 1.0, 0.0, G[k].E, G[k].B, G[k].a, G[k].b,
                                             dt, c.nx, c.ny, sp.q, sp.m, dx_of(c), dy_of(c), Hx, Hy, st,
                                             closure == VL_FLUID_GRADIENT ? gchi : 0.0, sg, per_y(c)));
        }
    }
    Timed tm(ctx, VL_T_FIELDS, st);
    VL_HIP(vl::launch_maxwell_half(S->fields, c.nx, c.ny, Uc, q, ns, dt, c.c, dx_of(c), dy_of(c), st, 10,
                                   per_y(c)));
    return VL_OK;
}

#define DISPATCH(ctx, call_f32, call_f64) ((ctx)->cfg.f_dtype == VL_F32 ? (call_f32) : (call_f64))

template <class T>
vl_status step_typed(vl_ctx* ctx, vl_state* S, double dt, hipStream_t st) {
    const vl_config& c = ctx->cfg;
    const int ns = c.nspecies;
    const double q[2] = {c.sp[0].q, ns > 1 ? c.sp[1].q : 0.0};
    vl_status r;
    for (int s = 0; s < ns; ++s)
        if (!S->f_max_valid)
            if ((r = array_max_typed<T>(ctx, s, (const T*)S->f[s], slot(ctx, 0, s), st)) != VL_OK) return r;

    if (c.dim_x == 2) {
        const long long cells = ctx->cells;
        double* E_t = S->work;
        double* B_t = E_t + 3 * cells;
        double* E_h = B_t + 3 * cells;
        double* B_h = E_h + 3 * cells;
        double* E_1 = B_h + 3 * cells;
        double* B_1 = E_1 + 3 * cells;
        double* fwork = B_1 + 3 * cells;
        double* mwork = fwork + (size_t)ns * fluid_doubles(c);
        mwork += ((uintptr_t)mwork & 15u) ? 1 : 0;         // network outputs are stored as 16-byte vectors
        {
            Timed tm(ctx, VL_T_FIELDS, st);
            if (c.fit) {
                VL_HIP(vl::launch_cell_fields(S->fields, c.nx, c.ny, E_t, B_t, st));   // the fields at t
            }
            const double* mom_t[2] = {S->mom_post[0], ns > 1 ? S->mom_post[1] : nullptr};
            VL_HIP(vl::launch_maxwell_half(S->fields, c.nx, c.ny, mom_t, q, ns, dt, c.c, dx_of(c), dy_of(c), st, 20,
                                            per_y(c)));
            VL_HIP(vl::launch_cell_fields(S->fields, c.nx, c.ny, E_h, B_h, st));
            if (c.fit) {
                // E^1 = 2 E^{t+1/2} - E^t and the same for B (E and B arrays adjacent)
                VL_HIP(vl::launch_axpby(E_h, E_t, 2.0, -1.0, E_1, 6 * cells, st));
            }
        }
        for (int s = 0; s < ns; ++s) {
            T* f = (T*)S->f[s];
            T* tmp = (T*)S->f_tmp[s];
            // X(dt/2): f -> tmp; V(dt): tmp in place; X(dt/2): tmp -> f
            if ((r = advect_x_typed<T>(ctx, s, f, tmp, 0.5 * dt, slot(ctx, 0, s), nullptr, slot(ctx, 1, s),
                                       st)) != VL_OK)
                return r;
            if ((r = advect_v_typed<T>(ctx, s, tmp, tmp, E_h, B_h, dt, slot(ctx, 1, s), slot(ctx, 2, s), st)) !=
                VL_OK)
                return r;
            if ((r = advect_x_typed<T>(ctx, s, tmp, f, 0.5 * dt, slot(ctx, 2, s), nullptr,
                                       c.fit ? nullptr : slot(ctx, 0, s), st)) != VL_OK)
                return r;
            if ((r = moments_typed<T>(ctx, s, f, S->mom_pre[s], st)) != VL_OK) return r;
            if (!c.fit) {
                Timed tm(ctx, VL_T_COPY, st);
                VL_HIP(hipMemcpyAsync(S->mom_post[s], S->mom_pre[s], cells * 20 * sizeof(double),
                                      hipMemcpyDeviceToDevice, st));
            }
        }
        if (c.fit) {
            // the fluid steps of all species (one launch per kernel with the
            // kinetic closure), then the fits
            if (c.closure == VL_CLOSURE_MLP) {
                if ((r = fluid_step_mlp_all(ctx, S, E_t, B_t, E_1, B_1, E_h, B_h, dt, fwork, mwork, st)) != VL_OK)
                    return r;
            } else {
                Timed tm(ctx, VL_T_FLUID, st);
                const double ms[2] = {c.sp[0].m, ns > 1 ? c.sp[1].m : 1.0};
                const double* mt[2] = {S->mom_post[0], ns > 1 ? S->mom_post[1] : nullptr};
                const double* mt1[2] = {S->mom_pre[0], ns > 1 ? S->mom_pre[1] : nullptr};
                VL_HIP(vl::launch_fluid_rk3_3v_set(ns, S->U, mt, mt1, E_t, B_t, E_1, B_1, E_h, B_h, dt, c.nx, c.ny, q,
                                                   ms, dx_of(c), dy_of(c), fwork, st, per_y(c)));
            }
            for (int s = 0; s < ns; ++s)
                if ((r = fit_typed<T>(ctx, s, (T*)S->f[s], (T*)S->f[s], S->mom_pre[s], S->U[s], S->mom_post[s],
                                      S->counters, slot(ctx, 0, s), st)) != VL_OK)
                    return r;
        }
        const double* mom_t1[2] = {S->mom_post[0], ns > 1 ? S->mom_post[1] : nullptr};
        Timed tm(ctx, VL_T_FIELDS, st);
        VL_HIP(vl::launch_maxwell_half(S->fields, c.nx, c.ny, mom_t1, q, ns, dt, c.c, dx_of(c), dy_of(c), st, 20,
                                        per_y(c)));
    } else {
        const int nx = c.nx;
        double* mom_half = S->work;
        double* E_t = mom_half + 4 * nx;
        double* E_t1 = E_t + nx;
        double* E_th = E_t1 + nx;
        double* fwork = E_th + nx;
        const int s = 0;
        T* f = (T*)S->f[s];
        T* tmp = (T*)S->f_tmp[s];
        const double L = c.x_hi - c.x_lo;
        if ((r = advect_x_typed<T>(ctx, s, f, tmp, 0.5 * dt, slot(ctx, 0, s), slot(ctx, 1, s), nullptr, st)) !=
            VL_OK)
            return r;
        if ((r = moments_typed<T>(ctx, s, tmp, mom_half, st)) != VL_OK) return r;
        {
            Timed tm(ctx, VL_T_FIELDS, st);
            VL_HIP(vl::launch_poisson(mom_half, nx, L, c.sp[0].q, ctx->dft, S->fields, st));
        }
        if ((r = advect_v_typed<T>(ctx, s, tmp, tmp, S->fields, nullptr, dt, slot(ctx, 1, s), slot(ctx, 2, s), st)) !=
            VL_OK)
            return r;
        if ((r = advect_x_typed<T>(ctx, s, tmp, f, 0.5 * dt, slot(ctx, 2, s),
                                   c.fit ? nullptr : slot(ctx, 0, s), nullptr, st)) != VL_OK)
            return r;
        if ((r = moments_typed<T>(ctx, s, f, S->mom_pre[s], st)) != VL_OK) return r;
        if (c.fit) {
            {
                Timed tm(ctx, VL_T_FIELDS, st);
                VL_HIP(vl::launch_poisson(S->mom_post[s], nx, L, c.sp[0].q, ctx->dft, E_t, st));
                VL_HIP(vl::launch_poisson(S->mom_pre[s], nx, L, c.sp[0].q, ctx->dft, E_t1, st));
                VL_HIP(vl::launch_axpby(E_t, E_t1, 0.5, 0.5, E_th, nx, st));
            }
            if ((r = fluid_step_impl(ctx, s, S->U[s], S->mom_post[s], S->mom_pre[s], E_t, nullptr, E_t1, nullptr, E_th,
                                     nullptr, dt, fwork, st)) != VL_OK)
                return r;
            if ((r = fit_typed<T>(ctx, s, f, f, S->mom_pre[s], S->U[s], S->mom_post[s], S->counters, slot(ctx, 0, s),
                                  st)) != VL_OK)
                return r;
        } else {
            Timed tm(ctx, VL_T_COPY, st);
            VL_HIP(hipMemcpyAsync(S->mom_post[s], S->mom_pre[s], (size_t)nx * 4 * sizeof(double),
                                  hipMemcpyDeviceToDevice, st));
        }
    }
    S->f_max_valid = 1;
    return VL_OK;
}

}  // namespace

// ------------------------------------------------ allocation-free fitting --
// vl_moment_fit_noalloc keeps the fitting parameters of every spatial cell
// (kFitCellDoubles doubles) and the per-cell clip partials (with the stage of
// their sum) in one static device array instead of context scratch, so the
// call allocates nothing.
// Host code never uses the array's name as an address: the device address
// is looked up once per device (hipGetSymbolAddress) and kept.
constexpr long long kNoAllocCells = 49152;                       // 48 Ki spatial cells
constexpr size_t kNoAllocParamBytes = (size_t)kNoAllocCells * vl::kFitCellDoubles * sizeof(double);
constexpr size_t kNoAllocBytes = kNoAllocParamBytes + (size_t)kNoAllocCells * sizeof(unsigned) + vl::kFinSlack;
static_assert(kNoAllocParamBytes % 256 == 0, "clip partials start 256-byte aligned");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device).
vl_status noalloc_scratch(vl_ctx* ctx, void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return fail(ctx, VL_EDEVICE, "no current HIP device");
    if (dev >= kMaxDevices) return fail(ctx, VL_EDEVICE, "device %d beyond the %d the library tracks", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(ctx, VL_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return VL_OK;
}

template <class T>
vl_status fit_noalloc_typed(vl_ctx* ctx, int s, const T* fin, T* fout, const double* mom_pre, double* U,
                            double* mom_post, int64_t* counters, void* sp, hipStream_t st) {
    const vl_config& c = ctx->cfg;
    const vl_species& sc = c.sp[s];
    if (c.dim_v == 1) {
        VL_HIP((vl::launch_fit1<T>(fin, fout, mom_pre, U, mom_post, counters, ctx->cells, sc.nv[0], sc.v_lo[0],
                                   dv_of(sc, 0), sc.m, nullptr, nullptr, st)));
        return VL_OK;
    }
    double* params = (double*)sp;
    unsigned* clip = (unsigned*)((char*)sp + kNoAllocParamBytes);
    VL_HIP((vl::launch_fit3<T>(fin, fout, mom_pre, U, mom_post, counters, ctx->cells, grid_args(sc), nullptr, nullptr,
                               clip, params, st)));
    return VL_OK;
}

}  // namespace

// ====================================================================== ABI ==
extern "C" {

const char* vl_version(void) { return "vl 0.1 gfx950"; }

const char* vl_status_str(vl_status st) {
    switch (st) {
        case VL_OK: return "ok";
        case VL_EINVAL: return "invalid argument";
        case VL_EALIAS: return "output aliases an input";
        case VL_ENOTSUP: return "not supported";
        case VL_EDEVICE: return "no usable device";
        case VL_EHIP: return "HIP runtime error";
        case VL_ENUMERIC: return "non-finite values";
    }
    return "unknown status";
}

const char* vl_last_error(const vl_ctx* ctx) { return ctx ? ctx->err : "null context"; }

vl_status vl_create(const vl_config* cfg, vl_ctx** out) {
    if (!cfg || !out) return VL_EINVAL;
    *out = nullptr;
    const vl_config& c = *cfg;
    if (!((c.dim_x == 1 && c.dim_v == 1) || (c.dim_x == 2 && c.dim_v == 3))) return VL_ENOTSUP;
    if (c.nx < 1 || c.nx > (1 << 24) || c.ny < 1 || c.ny > (1 << 24)) return VL_EINVAL;
    if (c.dim_x == 1 && c.ny != 1) return VL_EINVAL;
    if (c.dim_x == 2 && c.ny < 2) return VL_EINVAL;   // the wall ghosts mirror two interior rows
    if (!(std::isfinite(c.x_lo) && std::isfinite(c.x_hi) && c.x_hi > c.x_lo)) return VL_EINVAL;
    if (c.dim_x == 2 && !(std::isfinite(c.y_lo) && std::isfinite(c.y_hi) && c.y_hi > c.y_lo)) return VL_EINVAL;
    if (c.dim_x == 2 && c.bc_y != VL_BC_REFLECT && c.bc_y != VL_BC_PERIODIC) return VL_EINVAL;
    // the network closure's features mirror at the walls
    if (c.dim_x == 2 && c.bc_y == VL_BC_PERIODIC && c.closure == VL_CLOSURE_MLP) return VL_ENOTSUP;
    if (c.nspecies < 1 || c.nspecies > VL_MAX_SPECIES) return VL_EINVAL;
    if (c.dim_x == 1 && c.nspecies != 1) return VL_ENOTSUP;
    if (c.f_dtype != VL_F32 && c.f_dtype != VL_F64) return VL_EINVAL;
    if (c.dim_x == 2 && !finite_pos(c.c)) return VL_EINVAL;
    if (c.fit != 0 && c.fit != 1) return VL_EINVAL;
    if (c.closure == VL_CLOSURE_MLP) {
        if (c.dim_v != 3 || c.fit != 1) return VL_ENOTSUP;   // the learned closure serves the 2X3V fitting step
        if (!(std::isfinite(c.closure_tol) && c.closure_tol >= 0.0)) return VL_EINVAL;
    } else if (c.closure != VL_CLOSURE_KINETIC) {
        return VL_ENOTSUP;
    }
    if (c.vsplit != VL_VSPLIT_STRANG && c.vsplit != VL_VSPLIT_BACKSUB) return VL_EINVAL;
    if (c.vsplit == VL_VSPLIT_BACKSUB && c.dim_v != 3) return VL_ENOTSUP;   // a 3V splitting
    const size_t elem = c.f_dtype == VL_F32 ? 4 : 8;
    for (int s = 0; s < c.nspecies; ++s) {
        const vl_species& sp = c.sp[s];
        if (!finite_pos(sp.m) || !std::isfinite(sp.q)) return VL_EINVAL;
        const int nd = c.dim_v;
        for (int d = 0; d < 3; ++d) {
            if (d < nd) {
                if (sp.nv[d] < 2 || !(std::isfinite(sp.v_lo[d]) && std::isfinite(sp.v_hi[d]) && sp.v_hi[d] > sp.v_lo[d]))
                    return VL_EINVAL;
            } else if (sp.nv[d] != 1) {
                return VL_EINVAL;
            }
        }
        if (nd == 1 && sp.nv[0] > 4096) return VL_ENOTSUP;
        // the X operators address a row of f (nx velocity blocks) with 32-bit
        // element and byte offsets
        if ((long long)c.nx * sp.nv[0] * sp.nv[1] * sp.nv[2] * elem >= (1LL << 32)) return VL_ENOTSUP;
        if (nd == 3) {
            // the 34^3 cube has its own kernels (FP32: the block fills one CU's
            // LDS; FP64: half the block at a time)
            const bool big = sp.nv[0] == vl::kBigCube && sp.nv[1] == vl::kBigCube && sp.nv[2] == vl::kBigCube;
            // the affine sweeps hold the whole block in LDS: axes <= 32, or the
            // 34^3 cube in FP32 (158 KB padded)
            if (big && c.vsplit == VL_VSPLIT_BACKSUB && elem != 4) return VL_ENOTSUP;
            for (int d = 0; d < 3 && !big; ++d)
                if (sp.nv[d] > 32) return VL_ENOTSUP;
            if (!big && (long long)sp.nv[0] * sp.nv[1] * sp.nv[2] > 8192) return VL_ENOTSUP;
            if (!big && vl::v3_shared_bytes(sp.nv[0], sp.nv[1], sp.nv[2], elem) > 64 * 1024) return VL_ENOTSUP;
            // reflecting walls pair v_y with -v_y: the v_y grid must be symmetric about 0
            if (std::fabs(sp.v_lo[1] + sp.v_hi[1]) > 1e-12 * std::fabs(sp.v_hi[1])) return VL_EINVAL;
        }
    }
    vl_ctx* ctx = new (std::nothrow) vl_ctx;
    if (!ctx) return VL_EINVAL;
    ctx->cfg = c;
    ctx->cells = (long long)c.nx * c.ny;
    for (int s = 0; s < c.nspecies; ++s) ctx->nv[s] = (long long)c.sp[s].nv[0] * c.sp[s].nv[1] * c.sp[s].nv[2];
    // largest grid of a launch that produces a maximum (sizes the per-block partials)
    long long mb = vl::kMaxArrayBlocks;
    if (ctx->cells > mb) mb = ctx->cells;
    for (int s = 0; s < c.nspecies; ++s) {
        const vl_species& sp = c.sp[s];
        const long long bx = c.dim_x == 1 ? vl::pfc_x_blocks(1, c.nx, sp.nv[0])
                                          : vl::pfc_x_blocks(c.ny, c.nx, ctx->nv[s]);
        if (bx > mb) mb = bx;
        if (c.dim_x == 2) {
            const long long by = vl::pfc_xy_blocks(c.nx, c.ny, sp.nv[0], sp.nv[1], sp.nv[2]);
            if (by > mb) mb = by;
        }
    }
    ctx->max_blocks = (mb + 3) / 4 * 4;   // keeps the clip partials 16-byte aligned after the maxima
    *out = ctx;
    return VL_OK;
}

vl_status vl_destroy(vl_ctx* ctx) {
    if (!ctx) return VL_EINVAL;
    for (const vl_timer& t : ctx->pending) {
        (void)hipEventSynchronize(t.stop);
        ctx->pool.push_back(t.start);
        ctx->pool.push_back(t.stop);
    }
    for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
    if (ctx->slots) (void)hipFree(ctx->slots);
    if (ctx->fit_scratch) (void)hipFree(ctx->fit_scratch);
    if (ctx->bpart) (void)hipFree(ctx->bpart);
    delete ctx;
    return VL_OK;
}

vl_status vl_pfc_advect_x(vl_ctx* ctx, int32_t s, const void* f_in, void* f_out, double tau, vl_stream stream) {
    vl_status r = check_species(ctx, s);
    if (r != VL_OK) return r;
    if (!f_in || !f_out) return fail(ctx, VL_EINVAL, "null f");
    if (!finite_pos(tau)) return fail(ctx, VL_EINVAL, "tau must be finite and > 0");
    if (f_out == f_in) return fail(ctx, VL_EALIAS, "f_out aliases f_in");
    if ((r = ensure_device(ctx)) != VL_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    void* S = slot(ctx, 3, s);
    if (ctx->cfg.f_dtype == VL_F32) {
        if ((r = array_max_typed<float>(ctx, s, (const float*)f_in, S, st)) != VL_OK) return r;
        return advect_x_typed<float>(ctx, s, (const float*)f_in, (float*)f_out, tau, S, nullptr,
                                     nullptr, st);
    }
    if ((r = array_max_typed<double>(ctx, s, (const double*)f_in, S, st)) != VL_OK) return r;
    return advect_x_typed<double>(ctx, s, (const double*)f_in, (double*)f_out, tau, S, nullptr,
                                  nullptr, st);
}

vl_status vl_pfc_advect_v(vl_ctx* ctx, int32_t s, const void* f_in, void* f_out, const double* E, const double* B,
                          double tau, vl_stream stream) {
    vl_status r = check_species(ctx, s);
    if (r != VL_OK) return r;
    if (!f_in || !f_out || !E) return fail(ctx, VL_EINVAL, "null argument");
    if (!finite_pos(tau)) return fail(ctx, VL_EINVAL, "tau must be finite and > 0");
    if (f_out == f_in) return fail(ctx, VL_EALIAS, "f_out aliases f_in");
    if ((r = ensure_device(ctx)) != VL_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    void* S = slot(ctx, 3, s);
    if (ctx->cfg.f_dtype == VL_F32) {
        if ((r = array_max_typed<float>(ctx, s, (const float*)f_in, S, st)) != VL_OK) return r;
        return advect_v_typed<float>(ctx, s, (const float*)f_in, (float*)f_out, E, B, tau, S, nullptr, st);
    }
    if ((r = array_max_typed<double>(ctx, s, (const double*)f_in, S, st)) != VL_OK) return r;
    return advect_v_typed<double>(ctx, s, (const double*)f_in, (double*)f_out, E, B, tau, S, nullptr, st);
}

vl_status vl_moments(vl_ctx* ctx, int32_t s, const void* f, double* mom, vl_stream stream) {
    vl_status r = check_species(ctx, s);
    if (r != VL_OK) return r;
    if (!f || !mom) return fail(ctx, VL_EINVAL, "null argument");
    if ((r = ensure_device(ctx)) != VL_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    return DISPATCH(ctx, moments_typed<float>(ctx, s, (const float*)f, mom, st),
                    moments_typed<double>(ctx, s, (const double*)f, mom, st));
}

vl_status vl_moment_fit(vl_ctx* ctx, int32_t s, const void* f_in, void* f_out, const double* mom_pre, double* U,
                        double* mom_post, int64_t* counters, vl_stream stream) {
    vl_status r = check_species(ctx, s);
    if (r != VL_OK) return r;
    if (!f_in || !f_out || !mom_pre || !U) return fail(ctx, VL_EINVAL, "null argument");
    if ((r = ensure_device(ctx)) != VL_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    return DISPATCH(ctx,
                    fit_typed<float>(ctx, s, (const float*)f_in, (float*)f_out, mom_pre, U, mom_post, counters,
                                     nullptr, st),
                    fit_typed<double>(ctx, s, (const double*)f_in, (double*)f_out, mom_pre, U, mom_post, counters,
                                      nullptr, st));
}

vl_status vl_moment_fit_noalloc(vl_ctx* ctx, int32_t s, const void* f_in, void* f_out, const double* mom_pre,
                                double* U, double* mom_post, int64_t* counters, vl_stream stream) {
    vl_status r = check_species(ctx, s);
    if (r != VL_OK) return r;
    if (!f_in || !f_out || !mom_pre || !U) return fail(ctx, VL_EINVAL, "null argument");
    if (ctx->cells > kNoAllocCells)
        return fail(ctx, VL_EINVAL, "vl_moment_fit_noalloc: %lld spatial cells exceed the %lld its static scratch holds",
                    ctx->cells, kNoAllocCells);
    void* sp = nullptr;
    if ((r = noalloc_scratch(ctx, &sp)) != VL_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    return DISPATCH(ctx,
                    fit_noalloc_typed<float>(ctx, s, (const float*)f_in, (float*)f_out, mom_pre, U, mom_post,
                                             counters, sp, st),
                    fit_noalloc_typed<double>(ctx, s, (const double*)f_in, (double*)f_out, mom_pre, U, mom_post,
                                              counters, sp, st));
}

vl_status vl_poisson(vl_ctx* ctx, const double* mom, double* E, vl_stream stream) {
    if (!ctx) return VL_EINVAL;
    if (ctx->cfg.dim_x != 1) return fail(ctx, VL_ENOTSUP, "Poisson solver is the 1X1V field solver");
    if (!mom || !E) return fail(ctx, VL_EINVAL, "null argument");
    vl_status r;
    if ((r = ensure_device(ctx)) != VL_OK) return r;
    VL_HIP(vl::launch_poisson(mom, ctx->cfg.nx, ctx->cfg.x_hi - ctx->cfg.x_lo, ctx->cfg.sp[0].q, ctx->dft, E,
                              (hipStream_t)stream));
    return VL_OK;
}

size_t vl_yee_size(const vl_ctx* ctx) { return ctx ? yee_doubles(ctx->cfg) : 0; }
size_t vl_fluid_work_size(const vl_ctx* ctx) { return ctx ? fluid_doubles(ctx->cfg) : 0; }
size_t vl_step_work_size(const vl_ctx* ctx) { return ctx ? step_doubles(ctx->cfg) : 0; }

vl_status vl_maxwell_half_step(vl_ctx* ctx, double* yee, const double* const* mom, double dt, vl_stream stream) {
    if (!ctx) return VL_EINVAL;
    const vl_config& c = ctx->cfg;
    if (c.dim_x != 2) return fail(ctx, VL_ENOTSUP, "Maxwell solver is the 2X3V field solver");
    if (!yee || !mom) return fail(ctx, VL_EINVAL, "null argument");
    for (int s = 0; s < c.nspecies; ++s)
        if (!mom[s]) return fail(ctx, VL_EINVAL, "null moment array");
    if (!finite_pos(dt)) return fail(ctx, VL_EINVAL, "dt must be finite and > 0");
    vl_status r;
    if ((r = ensure_device(ctx)) != VL_OK) return r;
    const double q[2] = {c.sp[0].q, c.nspecies > 1 ? c.sp[1].q : 0.0};
    VL_HIP(vl::launch_maxwell_half(yee, c.nx, c.ny, mom, q, c.nspecies, dt, c.c, dx_of(c), dy_of(c),
                                   (hipStream_t)stream, 20, per_y(c)));
    return VL_OK;
}

vl_status vl_cell_fields(vl_ctx* ctx, const double* yee, double* E, double* B, vl_stream stream) {
    if (!ctx) return VL_EINVAL;
    if (ctx->cfg.dim_x != 2) return fail(ctx, VL_ENOTSUP, "Yee fields exist in 2X3V only");
    if (!yee || !E || !B) return fail(ctx, VL_EINVAL, "null argument");
    vl_status r;
    if ((r = ensure_device(ctx)) != VL_OK) return r;
    VL_HIP(vl::launch_cell_fields(yee, ctx->cfg.nx, ctx->cfg.ny, E, B, (hipStream_t)stream));
    return VL_OK;
}

vl_status vl_fluid_step(vl_ctx* ctx, int32_t s, double* U, const double* mom_t, const double* mom_t1,
                        const double* E_t, const double* B_t, const double* E_t1, const double* B_t1,
                        const double* E_th, const double* B_th, double dt, double* work, vl_stream stream) {
    vl_status r = check_species(ctx, s);
    if (r != VL_OK) return r;
    if (!U || !mom_t || !mom_t1 || !E_t || !E_t1 || !E_th || !work) return fail(ctx, VL_EINVAL, "null argument");
    if (ctx->cfg.dim_v == 3 && (!B_t || !B_t1 || !B_th)) return fail(ctx, VL_EINVAL, "3V fluid needs B");
    if (!finite_pos(dt)) return fail(ctx, VL_EINVAL, "dt must be finite and > 0");
    if ((r = ensure_device(ctx)) != VL_OK) return r;
    return fluid_step_impl(ctx, s, U, mom_t, mom_t1, E_t, B_t, E_t1, B_t1, E_th, B_th, dt, work, (hipStream_t)stream);
}

vl_status vl_step(vl_ctx* ctx, vl_state* S, double dt, vl_stream stream) {
    if (!ctx || !S) return VL_EINVAL;
    const vl_config& c = ctx->cfg;
    if (!finite_pos(dt)) return fail(ctx, VL_EINVAL, "dt must be finite and > 0");
    if (!S->fields || !S->work) return fail(ctx, VL_EINVAL, "null fields/work");
    for (int s = 0; s < c.nspecies; ++s) {
        if (!S->f[s] || !S->f_tmp[s] || !S->mom_post[s] || !S->mom_pre[s])
            return fail(ctx, VL_EINVAL, "null buffer for species %d", s);
        if (c.fit && !S->U[s]) return fail(ctx, VL_EINVAL, "fit needs U[%d]", s);
        if (S->f[s] == S->f_tmp[s]) return fail(ctx, VL_EALIAS, "f and f_tmp alias");
        if (S->mom_pre[s] == S->mom_post[s]) return fail(ctx, VL_EALIAS, "mom_pre and mom_post alias");
    }
    if (c.closure == VL_CLOSURE_MLP && (!S->mlp_params || !S->closure_fallback || !S->closure_err))
        return fail(ctx, VL_EINVAL, "the learned closure needs mlp_params, closure_fallback and closure_err");
    vl_status r;
    if ((r = ensure_device(ctx)) != VL_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    return DISPATCH(ctx, step_typed<float>(ctx, S, dt, st), step_typed<double>(ctx, S, dt, st));
}

size_t vl_fluid_closure_work_size(const vl_ctx* ctx) {
    return (ctx && ctx->cfg.dim_x == 2 && ctx->cfg.dim_v == 3) ? fluid_closure_doubles(ctx->cfg) : 0;
}

vl_status vl_fluid_closure_step(vl_ctx* ctx, vl_fluid_state* S, int32_t closure, double dt, vl_stream stream) {
    if (!ctx || !S) return VL_EINVAL;
    const vl_config& c = ctx->cfg;
    if (c.dim_x != 2 || c.dim_v != 3) return fail(ctx, VL_ENOTSUP, "the ten-moment fluid step is 2X3V");
    if (closure != VL_FLUID_GRADIENT && closure != VL_FLUID_MLP) return fail(ctx, VL_EINVAL, "unknown closure");
    if (!finite_pos(dt)) return fail(ctx, VL_EINVAL, "dt must be finite and > 0");
    if (!S->fields || !S->work) return fail(ctx, VL_EINVAL, "null fields/work");
    for (int s = 0; s < c.nspecies; ++s)
        if (!S->U[s]) return fail(ctx, VL_EINVAL, "null U[%d]", s);
    if (c.nspecies > 1 && S->U[0] == S->U[1]) return fail(ctx, VL_EALIAS, "U[0] and U[1] alias");
    if (closure == VL_FLUID_MLP && !S->mlp_params) return fail(ctx, VL_EINVAL, "the network closure needs mlp_params");
    if (closure == VL_FLUID_MLP && c.bc_y != VL_BC_REFLECT)
        return fail(ctx, VL_ENOTSUP, "the network closure's features need reflecting y walls");
    vl_status r;
    if ((r = ensure_device(ctx)) != VL_OK) return r;
    return fluid_closure_step_impl(ctx, S, closure, dt, (hipStream_t)stream);
}

vl_status vl_mlp_features(vl_ctx* ctx, int32_t s, const double* mom, int32_t stride, const double* B, uint16_t* x,
                          double* scale, vl_stream stream) {
    vl_status r = check_species(ctx, s);
    if (r != VL_OK) return r;
    if (ctx->cfg.dim_v != 3) return fail(ctx, VL_ENOTSUP, "the learned closure is defined for 2X3V");
    if (!mom || !x || !scale) return fail(ctx, VL_EINVAL, "null argument");
    if (stride != 10 && stride != 20) return fail(ctx, VL_EINVAL, "stride must be 10 or 20");
    if ((r = ensure_device(ctx)) != VL_OK) return r;
    const vl_config& c = ctx->cfg;
    VL_HIP(vl::launch_mlp_features(mom, stride, B, c.nx, c.ny, c.sp[s].m, s, x, scale, (hipStream_t)stream));
    return VL_OK;
}

vl_status vl_mlp_targets(vl_ctx* ctx, int32_t s, const double* mom, float* y, vl_stream stream) {
    vl_status r = check_species(ctx, s);
    if (r != VL_OK) return r;
    if (ctx->cfg.dim_v != 3) return fail(ctx, VL_ENOTSUP, "the learned closure is defined for 2X3V");
    if (!mom || !y) return fail(ctx, VL_EINVAL, "null argument");
    if ((r = ensure_device(ctx)) != VL_OK) return r;
    VL_HIP(vl::launch_mlp_targets(mom, ctx->cells, ctx->cfg.sp[s].m, y, (hipStream_t)stream));
    return VL_OK;
}

vl_status vl_mlp_forward(vl_ctx* ctx, const float* params, const uint16_t* x, int64_t n, float* y,
                         vl_stream stream) {
    if (!ctx) return VL_EINVAL;
    if (!params || !x || !y) return fail(ctx, VL_EINVAL, "null argument");
    if (n < 1) return fail(ctx, VL_EINVAL, "n must be >= 1");
    if (((uintptr_t)x & 7u) || ((uintptr_t)y & 15u)) return fail(ctx, VL_EINVAL, "x must be 8-, y 16-byte aligned");
    vl_status r;
    if ((r = ensure_device(ctx)) != VL_OK) return r;
    VL_HIP(vl::launch_mlp_forward(params, x, n, y, (hipStream_t)stream));
    return VL_OK;
}

size_t vl_mlp_work_size(int64_t n) { return n < 1 ? 0 : vl::mlp_part_floats(n); }

vl_status vl_mlp_gradient(vl_ctx* ctx, const float* params, const uint16_t* x, const float* y, int64_t n,
                          float* work, float* grad_loss, vl_stream stream) {
    if (!ctx) return VL_EINVAL;
    if (!params || !x || !y || !work || !grad_loss) return fail(ctx, VL_EINVAL, "null argument");
    if (n < 1) return fail(ctx, VL_EINVAL, "n must be >= 1");
    if (((uintptr_t)x & 7u) || ((uintptr_t)y & 15u)) return fail(ctx, VL_EINVAL, "x must be 8-, y 16-byte aligned");
    vl_status r;
    if ((r = ensure_device(ctx)) != VL_OK) return r;
    VL_HIP(vl::launch_mlp_gradient(params, x, y, n, work, grad_loss, (hipStream_t)stream));
    return VL_OK;
}

vl_status vl_mlp_train_step(vl_ctx* ctx, float* params, float* adam_m, float* adam_v, int64_t step, double lr,
                            const uint16_t* x, const float* y, int64_t n, float* work, float* grad_loss,
                            vl_stream stream) {
    if (!ctx) return VL_EINVAL;
    if (!params || !adam_m || !adam_v || !x || !y || !work || !grad_loss) return fail(ctx, VL_EINVAL, "null argument");
    if (n < 1 || step < 1) return fail(ctx, VL_EINVAL, "n and step must be >= 1");
    if (((uintptr_t)x & 7u) || ((uintptr_t)y & 15u)) return fail(ctx, VL_EINVAL, "x must be 8-, y 16-byte aligned");
    if (!finite_pos(lr)) return fail(ctx, VL_EINVAL, "lr must be finite and > 0");
    vl_status r;
    if ((r = ensure_device(ctx)) != VL_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    VL_HIP(vl::launch_mlp_train_step(params, adam_m, adam_v, step, lr, x, y, n, work, grad_loss, st));
    return VL_OK;
}

vl_status vl_mlp_train_epoch(vl_ctx* ctx, float* params, float* adam_m, float* adam_v, int64_t step0, double lr,
                             const uint16_t* x, const float* y, int64_t nrows, const int64_t* idx, int64_t batch,
                             int64_t nsteps, float* work, float* grad_loss, vl_stream stream) {
    if (!ctx) return VL_EINVAL;
    if (!params || !adam_m || !adam_v || !x || !y || !idx || !work || !grad_loss)
        return fail(ctx, VL_EINVAL, "null argument");
    if (nrows < 1 || batch < 1 || nsteps < 1 || step0 < 1) return fail(ctx, VL_EINVAL, "nrows, batch, nsteps, step0 must be >= 1");
    if (((uintptr_t)x & 7u) || ((uintptr_t)y & 15u)) return fail(ctx, VL_EINVAL, "x must be 8-, y 16-byte aligned");
    if (!finite_pos(lr)) return fail(ctx, VL_EINVAL, "lr must be finite and > 0");
    vl_status r;
    if ((r = ensure_device(ctx)) != VL_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    const long long* ix = (const long long*)idx;
    for (int64_t k = 0; k < nsteps; ++k)
        VL_HIP(vl::launch_mlp_train_step(params, adam_m, adam_v, step0 + k, lr, x, y, batch, work, grad_loss, st,
                                         ix + k * batch, nrows));
    return VL_OK;
}

vl_status vl_mass_energy(vl_ctx* ctx, int32_t s, const void* f, const double* mom, double* out, vl_stream stream) {
    vl_status r = check_species(ctx, s);
    if (r != VL_OK) return r;
    if (!f || !mom || !out) return fail(ctx, VL_EINVAL, "null argument");
    if ((r = ensure_device(ctx)) != VL_OK) return r;
    const vl_config& c = ctx->cfg;
    const vl_species& sp = c.sp[s];
    double dV = 1.0;
    for (int d = 0; d < c.dim_v; ++d) dV *= dv_of(sp, d);
    const double dX = dx_of(c) * dy_of(c);
    const int kmom = c.dim_v == 3 ? 20 : 4;
    hipStream_t st = (hipStream_t)stream;
    if (c.f_dtype == VL_F32)
        VL_HIP(vl::launch_mass_energy<float>((const float*)f, mom, ctx->cells, ctx->nv[s], kmom, c.dim_v, dV, dX, out,
                                             ctx->part, st));
    else
        VL_HIP(vl::launch_mass_energy<double>((const double*)f, mom, ctx->cells, ctx->nv[s], kmom, c.dim_v, dV, dX,
                                              out, ctx->part, st));
    return VL_OK;
}

vl_status vl_field_energy(vl_ctx* ctx, const double* fields, double* out, vl_stream stream) {
    if (!ctx) return VL_EINVAL;
    if (!fields || !out) return fail(ctx, VL_EINVAL, "null argument");
    vl_status r;
    if ((r = ensure_device(ctx)) != VL_OK) return r;
    const vl_config& c = ctx->cfg;
    if (c.dim_x == 2 && (size_t)c.ny + 1 > (size_t)kPartials)
        return fail(ctx, VL_ENOTSUP, "field energy partials hold at most %d rows", kPartials - 1);
    VL_HIP(vl::launch_field_energy(fields, c.dim_x, c.nx, c.ny, c.c, dx_of(c) * dy_of(c), ctx->part, out,
                                   (hipStream_t)stream));
    return VL_OK;
}

vl_status vl_timing_enable(vl_ctx* ctx, uint32_t mask) {
    if (!ctx) return VL_EINVAL;
    ctx->timing = mask & ((1u << VL_T_COUNT) - 1u);
    return VL_OK;
}

vl_status vl_timing_read(vl_ctx* ctx, double* ms, int64_t* count) {
    if (!ctx || !ms || !count) return VL_EINVAL;
    for (const vl_timer& t : ctx->pending) {
        VL_HIP(hipEventSynchronize(t.stop));
        float e = 0.f;
        VL_HIP(hipEventElapsedTime(&e, t.start, t.stop));
        ctx->t_ms[t.cat] += e;
        ctx->t_cnt[t.cat] += 1;
        ctx->pool.push_back(t.start);
        ctx->pool.push_back(t.stop);
    }
    ctx->pending.clear();
    for (int k = 0; k < VL_T_COUNT; ++k) {
        ms[k] = ctx->t_ms[k];
        count[k] = ctx->t_cnt[k];
        ctx->t_ms[k] = 0.0;
        ctx->t_cnt[k] = 0;
    }
    return VL_OK;
}

vl_status vl_sync(vl_ctx* ctx, vl_stream stream) {
    if (!ctx) return VL_EINVAL;
    VL_HIP(hipStreamSynchronize((hipStream_t)stream));
    VL_HIP(hipGetLastError());
    return VL_OK;
}

}  // extern "C"
