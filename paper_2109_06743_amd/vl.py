"""Python binding of libvl.so (include/vl.h): argument marshalling only.

Every computation runs in the library's HIP kernels; PyTorch provides device
memory (tensors) and the stream.  The binding refuses to work without the
built library: there is no fallback path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvl.so")

VL_F32, VL_F64 = 0, 1
VL_BC_REFLECT, VL_BC_PERIODIC = 0, 1
MAX_SPECIES = 2
STATUS = {0: "VL_OK", 1: "VL_EINVAL", 2: "VL_EALIAS", 3: "VL_ENOTSUP", 4: "VL_EDEVICE", 5: "VL_EHIP",
          6: "VL_ENUMERIC"}
EXPORTS = ["vl_create", "vl_destroy", "vl_pfc_advect_x", "vl_pfc_advect_v", "vl_moments", "vl_moment_fit",
           "vl_poisson", "vl_yee_size", "vl_maxwell_half_step", "vl_cell_fields", "vl_fluid_work_size",
           "vl_fluid_step", "vl_step_work_size", "vl_step", "vl_mass_energy", "vl_sync", "vl_status_str",
           "vl_last_error", "vl_version", "vl_timing_enable", "vl_timing_read", "vl_mlp_features",
           "vl_mlp_targets", "vl_mlp_forward", "vl_mlp_work_size", "vl_mlp_gradient", "vl_mlp_train_step",
           "vl_mlp_train_epoch", "vl_field_energy", "vl_fluid_closure_work_size", "vl_fluid_closure_step",
           "vl_moment_fit_noalloc"]
VL_CLOSURE_KINETIC, VL_CLOSURE_MLP = 0, 1
VL_VSPLIT_STRANG, VL_VSPLIT_BACKSUB = 0, 1
VL_FLUID_GRADIENT, VL_FLUID_MLP = 0, 1
MLP_IN, MLP_OUT, MLP_OUT_PAD, MLP_NPARAM = 64, 10, 16, 13520
TIMING_CATEGORIES = ["max", "pfc_x", "pfc_y", "pfc_v", "moments", "fluid", "fit", "fields", "copy"]


class VLError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Species(ctypes.Structure):
    _fields_ = [("q", ctypes.c_double), ("m", ctypes.c_double), ("v_lo", ctypes.c_double * 3),
                ("v_hi", ctypes.c_double * 3), ("nv", ctypes.c_int32 * 3)]


class Config(ctypes.Structure):
    _fields_ = [("dim_x", ctypes.c_int32), ("dim_v", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("x_lo", ctypes.c_double), ("x_hi", ctypes.c_double),
                ("y_lo", ctypes.c_double), ("y_hi", ctypes.c_double), ("bc_y", ctypes.c_int32),
                ("nspecies", ctypes.c_int32), ("sp", Species * MAX_SPECIES), ("f_dtype", ctypes.c_int32),
                ("c", ctypes.c_double), ("fit", ctypes.c_int32), ("closure", ctypes.c_int32),
                ("closure_tol", ctypes.c_double), ("vsplit", ctypes.c_int32)]


class State(ctypes.Structure):
    _fields_ = [("f", ctypes.c_void_p * MAX_SPECIES), ("f_tmp", ctypes.c_void_p * MAX_SPECIES),
                ("mom_post", ctypes.c_void_p * MAX_SPECIES), ("mom_pre", ctypes.c_void_p * MAX_SPECIES),
                ("U", ctypes.c_void_p * MAX_SPECIES), ("fields", ctypes.c_void_p), ("work", ctypes.c_void_p),
                ("counters", ctypes.c_void_p), ("f_max_valid", ctypes.c_int32), ("mlp_params", ctypes.c_void_p),
                ("closure_fallback", ctypes.c_void_p), ("closure_err", ctypes.c_void_p)]


class FluidClosureState(ctypes.Structure):
    _fields_ = [("U", ctypes.c_void_p * MAX_SPECIES), ("fields", ctypes.c_void_p), ("work", ctypes.c_void_p),
                ("mlp_params", ctypes.c_void_p)]


_lib = None


def load():
    """Load libvl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2109_06743_amd.build`")
    # torch's HIP runtime carries the same soname as ROCm's (libamdhip64.so.7):
    # importing torch first makes libvl.so bind to that one runtime, so device
    # pointers and streams from torch are valid inside the library
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, d, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    sig = {
        "vl_create": ([ctypes.POINTER(Config), ctypes.POINTER(vp)], i32),
        "vl_destroy": ([vp], i32),
        "vl_pfc_advect_x": ([vp, i32, vp, vp, d, vp], i32),
        "vl_pfc_advect_v": ([vp, i32, vp, vp, vp, vp, d, vp], i32),
        "vl_moments": ([vp, i32, vp, vp, vp], i32),
        "vl_moment_fit": ([vp, i32, vp, vp, vp, vp, vp, vp, vp], i32),
        "vl_moment_fit_noalloc": ([vp, i32, vp, vp, vp, vp, vp, vp, vp], i32),
        "vl_poisson": ([vp, vp, vp, vp], i32),
        "vl_yee_size": ([vp], sz),
        "vl_maxwell_half_step": ([vp, vp, vp, d, vp], i32),
        "vl_cell_fields": ([vp, vp, vp, vp, vp], i32),
        "vl_fluid_work_size": ([vp], sz),
        "vl_fluid_step": ([vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, d, vp, vp], i32),
        "vl_step_work_size": ([vp], sz),
        "vl_step": ([vp, ctypes.POINTER(State), d, vp], i32),
        "vl_fluid_closure_work_size": ([vp], sz),
        "vl_fluid_closure_step": ([vp, ctypes.POINTER(FluidClosureState), i32, d, vp], i32),
        "vl_mass_energy": ([vp, i32, vp, vp, vp, vp], i32),
        "vl_field_energy": ([vp, vp, vp, vp], i32),
        "vl_sync": ([vp, vp], i32),
        "vl_timing_enable": ([vp, ctypes.c_uint32], i32),
        "vl_timing_read": ([vp, vp, vp], i32),
        "vl_mlp_features": ([vp, i32, vp, i32, vp, vp, vp, vp], i32),
        "vl_mlp_targets": ([vp, i32, vp, vp, vp], i32),
        "vl_mlp_forward": ([vp, vp, vp, ctypes.c_int64, vp, vp], i32),
        "vl_mlp_work_size": ([ctypes.c_int64], sz),
        "vl_mlp_gradient": ([vp, vp, vp, vp, ctypes.c_int64, vp, vp, vp], i32),
        "vl_mlp_train_step": ([vp, vp, vp, vp, ctypes.c_int64, d, vp, vp, ctypes.c_int64, vp, vp, vp], i32),
        "vl_mlp_train_epoch": ([vp, vp, vp, vp, ctypes.c_int64, d, vp, vp, ctypes.c_int64, vp, ctypes.c_int64,
                                ctypes.c_int64, vp, vp, vp], i32),
        "vl_status_str": ([i32], ctypes.c_char_p),
        "vl_last_error": ([vp], ctypes.c_char_p),
        "vl_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def make_config(cfg, f_dtype="f32"):
    """ctypes vl_config from a set-up dict (paper_2109_06743_amd.workloads)."""
    c = Config()
    c.f_dtype = VL_F32 if f_dtype in ("f32", "float32", np.float32) else VL_F64
    c.fit = int(bool(cfg.get("fit", False)))
    c.closure = VL_CLOSURE_MLP if cfg.get("closure") == "mlp" else VL_CLOSURE_KINETIC
    c.closure_tol = float(cfg.get("closure_tol", 0.0))
    c.vsplit = VL_VSPLIT_BACKSUB if cfg.get("vsplit") == "backsub" else VL_VSPLIT_STRANG
    c.bc_y = VL_BC_PERIODIC if cfg.get("bc_y") == "periodic" else VL_BC_REFLECT
    if cfg["kind"] == "1x1v":
        c.dim_x, c.dim_v = 1, 1
        c.nx, c.ny = cfg["nx"], 1
        c.x_lo, c.x_hi = cfg["x_lo"], cfg["x_hi"]
        c.y_lo, c.y_hi = 0.0, 1.0
        c.nspecies = 1
        sp = c.sp[0]
        sp.q, sp.m = cfg["q"], cfg["m"]
        sp.v_lo[:] = [cfg["v_lo"], 0.0, 0.0]
        sp.v_hi[:] = [cfg["v_hi"], 1.0, 1.0]
        sp.nv[:] = [cfg["nv"], 1, 1]
        c.c = 1.0
    else:
        c.dim_x, c.dim_v = 2, 3
        c.nx, c.ny = cfg["nx"], cfg["ny"]
        c.x_lo, c.x_hi, c.y_lo, c.y_hi = cfg["x_lo"], cfg["x_hi"], cfg["y_lo"], cfg["y_hi"]
        c.nspecies = len(cfg["species"])
        for k, s in enumerate(cfg["species"]):
            c.sp[k].q, c.sp[k].m = s["q"], s["m"]
            c.sp[k].v_lo[:] = list(s["v_lo"])
            c.sp[k].v_hi[:] = list(s["v_hi"])
            c.sp[k].nv[:] = list(s["nv"])
        c.c = cfg["c"]
    return c


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """One problem geometry (vl_create).  Arrays are torch CUDA tensors."""

    def __init__(self, cfg, f_dtype="f32"):
        self.lib = load()
        self.cfg_dict = cfg
        self.cfg = make_config(cfg, f_dtype)
        self.f_dtype = f_dtype
        h = ctypes.c_void_p()
        st = self.lib.vl_create(ctypes.byref(self.cfg), ctypes.byref(h))
        if st != 0:
            raise VLError(st, "vl_create rejected the configuration")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.vl_destroy(h)
            self.h = None

    def _check(self, st):
        if st != 0:
            raise VLError(st, (self.lib.vl_last_error(self.h) or b"").decode())

    # ---- entry points -----------------------------------------------------
    def pfc_advect_x(self, s, f_in, f_out, tau, stream=None):
        self._check(self.lib.vl_pfc_advect_x(self.h, s, _ptr(f_in), _ptr(f_out), float(tau), _stream(stream)))

    def pfc_advect_v(self, s, f_in, f_out, E, B, tau, stream=None):
        self._check(self.lib.vl_pfc_advect_v(self.h, s, _ptr(f_in), _ptr(f_out), _ptr(E), _ptr(B), float(tau),
                                             _stream(stream)))

    def moments(self, s, f, mom, stream=None):
        self._check(self.lib.vl_moments(self.h, s, _ptr(f), _ptr(mom), _stream(stream)))

    def moment_fit(self, s, f_in, f_out, mom_pre, U, mom_post=None, counters=None, stream=None):
        self._check(self.lib.vl_moment_fit(self.h, s, _ptr(f_in), _ptr(f_out), _ptr(mom_pre), _ptr(U),
                                           _ptr(mom_post), _ptr(counters), _stream(stream)))

    def moment_fit_noalloc(self, s, f_in, f_out, mom_pre, U, mom_post=None, counters=None, stream=None):
        self._check(self.lib.vl_moment_fit_noalloc(self.h, s, _ptr(f_in), _ptr(f_out), _ptr(mom_pre), _ptr(U),
                                                   _ptr(mom_post), _ptr(counters), _stream(stream)))

    def poisson(self, mom, E, stream=None):
        self._check(self.lib.vl_poisson(self.h, _ptr(mom), _ptr(E), _stream(stream)))

    def yee_size(self):
        return int(self.lib.vl_yee_size(self.h))

    def maxwell_half_step(self, yee, moms, dt, stream=None):
        arr = (ctypes.c_void_p * MAX_SPECIES)(*[m.data_ptr() for m in moms])
        self._check(self.lib.vl_maxwell_half_step(self.h, _ptr(yee), ctypes.cast(arr, ctypes.c_void_p), float(dt),
                                                  _stream(stream)))

    def cell_fields(self, yee, E, B, stream=None):
        self._check(self.lib.vl_cell_fields(self.h, _ptr(yee), _ptr(E), _ptr(B), _stream(stream)))

    def fluid_work_size(self):
        return int(self.lib.vl_fluid_work_size(self.h))

    def fluid_step(self, s, U, mom_t, mom_t1, E_t, B_t, E_t1, B_t1, E_th, B_th, dt, work, stream=None):
        self._check(self.lib.vl_fluid_step(self.h, s, _ptr(U), _ptr(mom_t), _ptr(mom_t1), _ptr(E_t), _ptr(B_t),
                                           _ptr(E_t1), _ptr(B_t1), _ptr(E_th), _ptr(B_th), float(dt), _ptr(work),
                                           _stream(stream)))

    def step_work_size(self):
        return int(self.lib.vl_step_work_size(self.h))

    def step(self, state, dt, stream=None):
        self._check(self.lib.vl_step(self.h, ctypes.byref(state.c), float(dt), _stream(stream)))

    def fluid_closure_work_size(self):
        return int(self.lib.vl_fluid_closure_work_size(self.h))

    def fluid_closure_step(self, state, dt, closure="gradient", stream=None):
        """One ten-moment multi-fluid step (vl_fluid_closure_step) of a
        FluidState with the Eq. 5 gradient closure or the network."""
        kind = {"gradient": VL_FLUID_GRADIENT, "mlp": VL_FLUID_MLP}[closure]
        self._check(self.lib.vl_fluid_closure_step(self.h, ctypes.byref(state.c), kind, float(dt),
                                                   _stream(stream)))

    def mass_energy(self, s, f, mom, out, stream=None):
        self._check(self.lib.vl_mass_energy(self.h, s, _ptr(f), _ptr(mom), _ptr(out), _stream(stream)))

    def field_energy(self, fields, out, stream=None):
        self._check(self.lib.vl_field_energy(self.h, _ptr(fields), _ptr(out), _stream(stream)))

    def sync(self, stream=None):
        self._check(self.lib.vl_sync(self.h, _stream(stream)))

    # ---- learned heat-flux closure -----------------------------------------
    def mlp_features(self, s, mom, stride, x, scale, B=None, stream=None):
        """x: int16 tensor [cells, 64] (BF16 bits), scale: float64 [cells];
        B: cell-centred magnetic field [cells, 3] or None."""
        self._check(self.lib.vl_mlp_features(self.h, s, _ptr(mom), int(stride), _ptr(B), _ptr(x), _ptr(scale),
                                             _stream(stream)))

    def mlp_targets(self, s, mom, y, stream=None):
        self._check(self.lib.vl_mlp_targets(self.h, s, _ptr(mom), _ptr(y), _stream(stream)))

    def mlp_forward(self, params, x, y, n=None, stream=None):
        n = x.shape[0] if n is None else n
        self._check(self.lib.vl_mlp_forward(self.h, _ptr(params), _ptr(x), int(n), _ptr(y), _stream(stream)))

    def mlp_work_size(self, n):
        return int(self.lib.vl_mlp_work_size(int(n)))

    def mlp_gradient(self, params, x, y, work, grad_loss, n=None, stream=None):
        n = x.shape[0] if n is None else n
        self._check(self.lib.vl_mlp_gradient(self.h, _ptr(params), _ptr(x), _ptr(y), int(n), _ptr(work),
                                             _ptr(grad_loss), _stream(stream)))

    def mlp_train_step(self, params, m1, m2, step, lr, x, y, work, grad_loss, n=None, stream=None):
        n = x.shape[0] if n is None else n
        self._check(self.lib.vl_mlp_train_step(self.h, _ptr(params), _ptr(m1), _ptr(m2), int(step), float(lr),
                                               _ptr(x), _ptr(y), int(n), _ptr(work), _ptr(grad_loss),
                                               _stream(stream)))

    def mlp_train_epoch(self, params, m1, m2, step0, lr, x, y, idx, batch, work, grad_loss, stream=None):
        """len(idx) // batch Adam steps on the rows idx of x and y (idx: int64 device tensor)."""
        nsteps = idx.shape[0] // batch
        self._check(self.lib.vl_mlp_train_epoch(self.h, _ptr(params), _ptr(m1), _ptr(m2), int(step0), float(lr),
                                                _ptr(x), _ptr(y), int(x.shape[0]), _ptr(idx), int(batch),
                                                int(nsteps), _ptr(work), _ptr(grad_loss), _stream(stream)))
        return nsteps

    def timing_enable(self, on=True):
        """on: True/False for every category, or an iterable of category names."""
        if on is True:
            mask = (1 << len(TIMING_CATEGORIES)) - 1
        elif not on:
            mask = 0
        else:
            mask = 0
            for name in on:
                mask |= 1 << TIMING_CATEGORIES.index(name)
        self._check(self.lib.vl_timing_enable(self.h, mask))

    def timing_read(self):
        """{category: (total_ms, launch_groups)} since the previous read."""
        n = len(TIMING_CATEGORIES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        self._check(self.lib.vl_timing_read(self.h, ctypes.cast(ms, ctypes.c_void_p),
                                            ctypes.cast(cnt, ctypes.c_void_p)))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(TIMING_CATEGORIES)}


class StepState:
    """Device buffers of vl_step for one context (allocated with torch)."""

    def __init__(self, ctx, f_list, fields, U_list=None, mom_post_list=None, mlp_params=None, device="cuda"):
        import torch
        cfg = ctx.cfg
        dt = torch.float32 if ctx.f_dtype == "f32" else torch.float64
        self.ctx = ctx
        ns = cfg.nspecies
        cells = cfg.nx * cfg.ny
        kmom = 20 if cfg.dim_v == 3 else 4
        kU = 10 if cfg.dim_v == 3 else 3
        self.f = [torch.as_tensor(f, device=device).to(dt).contiguous() for f in f_list]
        self.f_tmp = [torch.empty_like(f) for f in self.f]
        self.mom_pre = [torch.zeros(cells * kmom, dtype=torch.float64, device=device) for _ in range(ns)]
        if mom_post_list is None:
            self.mom_post = [torch.zeros(cells * kmom, dtype=torch.float64, device=device) for _ in range(ns)]
            for s in range(ns):
                ctx.moments(s, self.f[s], self.mom_post[s])
        else:
            self.mom_post = [torch.as_tensor(m, device=device).to(torch.float64).reshape(-1).contiguous()
                             for m in mom_post_list]
        if U_list is None:
            self.U = [self.mom_post[s].view(cells, kmom)[:, :kU].contiguous().reshape(-1) for s in range(ns)]
        else:
            self.U = [torch.as_tensor(u, device=device).to(torch.float64).reshape(-1).contiguous() for u in U_list]
        self.fields = torch.as_tensor(fields, device=device).to(torch.float64).reshape(-1).contiguous()
        self.work = torch.zeros(max(ctx.step_work_size(), 1), dtype=torch.float64, device=device)
        self.counters = torch.zeros(2, dtype=torch.int64, device=device)
        c = State()
        for s in range(ns):
            c.f[s] = self.f[s].data_ptr()
            c.f_tmp[s] = self.f_tmp[s].data_ptr()
            c.mom_post[s] = self.mom_post[s].data_ptr()
            c.mom_pre[s] = self.mom_pre[s].data_ptr()
            c.U[s] = self.U[s].data_ptr()
        c.fields = self.fields.data_ptr()
        c.work = self.work.data_ptr()
        c.counters = self.counters.data_ptr()
        c.f_max_valid = 0
        if cfg.closure == VL_CLOSURE_MLP:
            self.mlp_params = torch.as_tensor(mlp_params, device=device).to(torch.float32).contiguous()
            self.closure_fallback = torch.zeros(ns, dtype=torch.int32, device=device)
            self.closure_err = torch.zeros(ns, dtype=torch.float64, device=device)
            c.mlp_params = self.mlp_params.data_ptr()
            c.closure_fallback = self.closure_fallback.data_ptr()
            c.closure_err = self.closure_err.data_ptr()
        self.c = c


def yee_pack(F):
    """Concatenate Yee components (Ex, Ey, Ez, Bx, By, Bz) in the library's order."""
    return np.concatenate([np.asarray(getattr(F, k), dtype=np.float64).reshape(-1)
                           for k in ("Ex", "Ey", "Ez", "Bx", "By", "Bz")])


class FluidState:
    """Device buffers of vl_fluid_closure_step: the fluid states U[s]
    ([cells][10], FP64), the Yee array, scratch, and the network parameters
    for the network closure."""

    def __init__(self, ctx, U_list, fields, mlp_params=None, device="cuda"):
        import torch
        ns = ctx.cfg.nspecies
        self.U = [torch.as_tensor(np.asarray(u, dtype=np.float64).reshape(-1)).to(device) for u in U_list[:ns]]
        self.fields = torch.as_tensor(np.asarray(fields, dtype=np.float64).reshape(-1)).to(device)
        self.work = torch.zeros(max(ctx.fluid_closure_work_size(), 1), dtype=torch.float64, device=device)
        c = FluidClosureState()
        for k in range(ns):
            c.U[k] = self.U[k].data_ptr()
        c.fields = self.fields.data_ptr()
        c.work = self.work.data_ptr()
        if mlp_params is not None:
            self.mlp_params = torch.as_tensor(mlp_params, device=device).to(torch.float32).contiguous()
            c.mlp_params = self.mlp_params.data_ptr()
        self.c = c


def yee_unpack(arr, nx, ny):
    arr = np.asarray(arr)
    a, b = nx * ny, nx * (ny + 1)
    sizes = [a, b, a, b, a, b]
    shapes = [(ny, nx), (ny + 1, nx), (ny, nx), (ny + 1, nx), (ny, nx), (ny + 1, nx)]
    out, off = {}, 0
    for k, n, sh in zip(("Ex", "Ey", "Ez", "Bx", "By", "Bz"), sizes, shapes):
        out[k] = arr[off:off + n].reshape(sh)
        off += n
    return out
