"""Python binding of the C ABI in include/lwfr.h (argument marshalling only).

Every function mirrors the C entry point of the same name.  Device buffers are
torch tensors on a ROCm device; torch provides memory and the HIP stream, all
arithmetic of the step runs in the HIP kernels of liblwfr.so.  The module
raises at import of the library if it is not built: there is no fallback.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# LWFR_LIBRARY selects another build of the same library (e.g. a tuning variant)
LIBPATH = os.environ.get("LWFR_LIBRARY", os.path.join(_HERE, "liblwfr.so"))
ABI_VERSION = 3

LWFR_OK, LWFR_E_INVALID_ARG, LWFR_E_UNSUPPORTED, LWFR_E_HIP = 0, 1, 2, 3
LWFR_E_INADMISSIBLE, LWFR_E_NONFINITE, LWFR_E_WORKSPACE, LWFR_E_STATE = 4, 5, 6, 7
LWFR_EQ_SW1D, LWFR_EQ_SW2D, LWFR_EQ_GLMMHD2D, LWFR_EQ_LINADV1D, LWFR_EQ_VARADV1D = 1, 2, 3, 4, 5
LWFR_EQ_JINXIN1D = 6
LWFR_CFG_ADJOINT = 1
LWFR_CFG_GLL = 2
LWFR_CFG_IMEX_HT112, LWFR_CFG_IMEX_SSP3 = 4, 8
LWFR_CFG_ALW = 16
LWFR_BC_PERIODIC, LWFR_BC_OUTFLOW, LWFR_BC_WALL, LWFR_BC_DIRICHLET = 0, 1, 2, 3
LWFR_FLAG_ALG2, LWFR_FLAG_LOW_INADM, LWFR_FLAG_ALG1, LWFR_FLAG_NONFINITE, LWFR_FLAG_ALG1_GUARD = 1, 2, 4, 8, 16

NVARS = {1: 3, 2: 4, 3: 9, 4: 1, 5: 2, 6: 2}
DIMS = {1: 1, 2: 2, 3: 2, 4: 1, 5: 1, 6: 1}


class LwfrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lwfr status {status}: {msg}")
        self.status = status


class lwfr_config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32),
        ("equation", ctypes.c_int32),
        ("degree", ctypes.c_int32),
        ("nelem", ctypes.c_int32 * 2),
        ("lo", ctypes.c_double * 2),
        ("hi", ctypes.c_double * 2),
        ("gamma", ctypes.c_double),
        ("gravity", ctypes.c_double),
        ("cfl_safety", ctypes.c_double),
        ("cfl_number", ctypes.c_double),
        ("blending", ctypes.c_int32),
        ("alpha_max", ctypes.c_double),
        ("alpha_min", ctypes.c_double),
        ("alpha_force", ctypes.c_double),
        ("flags", ctypes.c_uint32),
        ("bc", ctypes.c_int32 * 4),
        ("source", ctypes.c_double * 4),
    ]


class lwfr_stats(ctypes.Structure):
    """Mirror of lwfr_stats (include/lwfr.h): statistics of one step."""
    _fields_ = [
        ("dt", ctypes.c_double),
        ("ch", ctypes.c_double),
        ("mass", ctypes.c_double * 9),
        ("min_constraint", ctypes.c_double * 2),
        ("alpha_hist", ctypes.c_uint32 * 11),
        ("n_alg1", ctypes.c_uint32),
        ("n_alg2", ctypes.c_uint32),
        ("n_low_inadm", ctypes.c_uint32),
        ("n_nonfinite", ctypes.c_uint32),
        ("n_alg1_guard", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


STATS_BYTES = ctypes.sizeof(lwfr_stats)


def stats_buffer(device="cuda:0"):
    """A device buffer for one lwfr_stats (uint8 tensor, 8-byte aligned by the allocator)."""
    import torch

    return torch.zeros(STATS_BYTES, dtype=torch.uint8, device=device)


def read_stats(buf):
    """Host dict of an lwfr_stats held in the device tensor buf (synchronising copy)."""
    raw = bytes(buf.cpu().numpy().tobytes())
    st = lwfr_stats.from_buffer_copy(raw)
    return {
        "dt": st.dt, "ch": st.ch, "mass": list(st.mass), "min_constraint": list(st.min_constraint),
        "alpha_hist": list(st.alpha_hist), "n_alg1": st.n_alg1, "n_alg2": st.n_alg2,
        "n_low_inadm": st.n_low_inadm, "n_nonfinite": st.n_nonfinite, "n_alg1_guard": st.n_alg1_guard,
    }


_lib = None
_SIGS = {
    "lwfr_init": [ctypes.POINTER(lwfr_config), ctypes.POINTER(ctypes.c_void_p)],
    "lwfr_workspace_bytes": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "lwfr_state_size": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "lwfr_reference_nodes": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
    "lwfr_cfl_number": [ctypes.c_int32, ctypes.POINTER(ctypes.c_double)],
    "lwfr_cfl_number_for": [ctypes.c_int32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_double)],
    "lwfr_bind": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "lwfr_boundary_data_size": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "lwfr_set_boundary_data": [ctypes.c_void_p, ctypes.c_void_p],
    "lwfr_step": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "lwfr_step_noalloc": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                          ctypes.c_void_p, ctypes.c_void_p],
    "lwfr_step_fixed": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                        ctypes.c_void_p, ctypes.c_void_p],
    "lwfr_residual": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_void_p],
    "lwfr_query": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32)],
    "lwfr_adjoint_step": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_void_p],
    "lwfr_tape_bytes": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "lwfr_step_taped": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                        ctypes.c_void_p],
    "lwfr_timing_begin": [ctypes.c_void_p, ctypes.c_int32],
    "lwfr_timing_end": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint32)],
    "lwfr_graph_capture": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p],
    "lwfr_graph_launch": [ctypes.c_void_p],
    "lwfr_destroy": [ctypes.c_void_p],
    "lwfr_batch_init": [ctypes.POINTER(lwfr_config), ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)],
    "lwfr_batch_workspace_bytes": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "lwfr_batch_state_offsets": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)],
    "lwfr_batch_problem": [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)],
    "lwfr_batch_bind": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "lwfr_batch_step": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "lwfr_batch_set_launch": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
    "lwfr_batch_get_launch": [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
    "lwfr_batch_autotune": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32],
    "lwfr_batch_graph_capture": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                 ctypes.c_void_p],
    "lwfr_batch_graph_launch": [ctypes.c_void_p],
    "lwfr_batch_query": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32)],
    "lwfr_batch_timing_begin": [ctypes.c_void_p, ctypes.c_int32],
    "lwfr_batch_timing_end": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint32)],
    "lwfr_batch_destroy": [ctypes.c_void_p],
}
TIMING_KERNELS = ("k_pre", "k_dt", "k_ch", "k_ch_fin", "k_stages", "k_faces", "k_update", "k_residual",
                  "k_adj_update", "k_adj_faces", "k_adj_stages", "kb_pre", "kb_dt", "kb_stages", "kb_faces",
                  "kb_update", "k_bfaces")
LWFR_PHASE_PRE, LWFR_PHASE_STAGES, LWFR_PHASE_FACES, LWFR_PHASE_UPDATE = 0, 1, 2, 3


def lib():
    """The loaded liblwfr.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIBPATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.lwfr_last_error.argtypes = []
        L.lwfr_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def lwfr_last_error():
    return lib().lwfr_last_error().decode()


def _check(status):
    if status != LWFR_OK:
        raise LwfrError(status, lwfr_last_error())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def make_config(equation, degree, nelem, lo=(0.0, 0.0), hi=(1.0, 1.0), gamma=5.0 / 3.0, gravity=9.81,
                cfl_safety=0.9, cfl_number=0.0, blending=2, alpha_max=0.5, alpha_min=1e-3, alpha_force=-1.0,
                flags=0, bc=(0, 0, 0, 0), source=(3.0, 1e-2, 0.0, 1.0)):
    """bc: LWFR_BC_* of the sides (x lo, x hi, y lo, y hi); periodic by default.
    source: Jin-Xin (a, eps, l, q), f(u) = l u + q u^2/2 (LWFR_EQ_JINXIN1D only)."""
    c = lwfr_config()
    c.abi_version = ABI_VERSION
    c.equation, c.degree = equation, degree
    nel = (nelem, 1) if isinstance(nelem, int) else tuple(nelem)
    c.nelem[0], c.nelem[1] = nel[0], (nel[1] if len(nel) > 1 else 1)
    c.lo[0], c.lo[1] = lo
    c.hi[0], c.hi[1] = hi
    c.gamma, c.gravity, c.cfl_safety, c.cfl_number = gamma, gravity, cfl_safety, cfl_number
    c.blending, c.alpha_max, c.alpha_min, c.alpha_force = blending, alpha_max, alpha_min, alpha_force
    c.flags = flags
    for i in range(4):
        c.bc[i] = bc[i]
        c.source[i] = source[i]
    return c


def lwfr_init(cfg):
    ctx = ctypes.c_void_p()
    _check(lib().lwfr_init(ctypes.byref(cfg), ctypes.byref(ctx)))
    return ctx


def lwfr_workspace_bytes(ctx):
    n = ctypes.c_size_t()
    _check(lib().lwfr_workspace_bytes(ctx, ctypes.byref(n)))
    return n.value


def lwfr_state_size(ctx):
    n = ctypes.c_size_t()
    _check(lib().lwfr_state_size(ctx, ctypes.byref(n)))
    return n.value


def lwfr_reference_nodes(ctx, n1):
    xi = (ctypes.c_double * n1)()
    w = (ctypes.c_double * n1)()
    _check(lib().lwfr_reference_nodes(ctx, xi, w))
    return list(xi), list(w)


def lwfr_cfl_number(degree, flags=0):
    """Fourier CFL(N) of the scheme that the config flags select (LWFR_CFG_GLL)."""
    c = ctypes.c_double()
    _check(lib().lwfr_cfl_number_for(degree, int(flags), ctypes.byref(c)))
    return c.value


def lwfr_bind(ctx, workspace, stream=None):
    """workspace: a device tensor of at least lwfr_workspace_bytes(ctx) bytes, 256-byte aligned."""
    import torch

    if stream is None:
        stream = torch.cuda.current_stream(workspace.device)
    nbytes = workspace.numel() * workspace.element_size()
    _check(lib().lwfr_bind(ctx, ctypes.c_void_p(workspace.data_ptr()), nbytes, ctypes.c_void_p(stream.cuda_stream)))


def lwfr_boundary_data_size(ctx):
    n = ctypes.c_size_t()
    _check(lib().lwfr_boundary_data_size(ctx, ctypes.byref(n)))
    return n.value


def lwfr_set_boundary_data(ctx, ghost):
    """ghost: float64 device tensor of lwfr_boundary_data_size(ctx) doubles, kept alive by the caller."""
    _check(lib().lwfr_set_boundary_data(ctx, _ptr(ghost)))


def lwfr_step(ctx, u_in, u_out, dt=0.0, dt_ch=None, alpha=None, flags=None, stats=None):
    """stats: nullable device buffer of STATS_BYTES (stats_buffer()); read it with read_stats."""
    _check(lib().lwfr_step(ctx, _ptr(u_in), _ptr(u_out), float(dt), _ptr(dt_ch), _ptr(alpha), _ptr(flags),
                           _ptr(stats)))


def lwfr_step_noalloc(ctx, u_in, u_out, dt=0.0, dt_ch=None, flags=None, stream=None):
    """One step with the library's static scratch as workspace (no bind needed);
    stream: a torch stream (None: the current one)."""
    import torch

    if stream is None:
        stream = torch.cuda.current_stream(u_in.device)
    _check(lib().lwfr_step_noalloc(ctx, _ptr(u_in), _ptr(u_out), float(dt), _ptr(dt_ch), _ptr(flags),
                                   ctypes.c_void_p(stream.cuda_stream)))


def lwfr_step_fixed(ctx, u_in, u_out, dt, ch, alpha=None, flags=None):
    _check(lib().lwfr_step_fixed(ctx, _ptr(u_in), _ptr(u_out), float(dt), float(ch), _ptr(alpha), _ptr(flags)))


def lwfr_residual(ctx, u, dt, mode, R):
    _check(lib().lwfr_residual(ctx, _ptr(u), float(dt), int(mode), _ptr(R)))


def lwfr_adjoint_step(ctx, u_n, dt, lam_np1, lam_n, tape=None):
    _check(lib().lwfr_adjoint_step(ctx, _ptr(u_n), float(dt), _ptr(lam_np1), _ptr(lam_n), _ptr(tape)))


def lwfr_tape_bytes(ctx):
    n = ctypes.c_size_t()
    _check(lib().lwfr_tape_bytes(ctx, ctypes.byref(n)))
    return n.value


def lwfr_step_taped(ctx, u_in, u_out, dt, dt_ch, tape):
    _check(lib().lwfr_step_taped(ctx, _ptr(u_in), _ptr(u_out), float(dt), _ptr(dt_ch), _ptr(tape)))


def lwfr_query(ctx):
    """(status, flags_or) without raising."""
    f = ctypes.c_uint32()
    st = lib().lwfr_query(ctx, ctypes.byref(f))
    return st, f.value


def lwfr_timing_begin(ctx, max_launches):
    _check(lib().lwfr_timing_begin(ctx, int(max_launches)))


def lwfr_timing_end(ctx):
    """{kernel name: (total ms, launches)} of the launches since lwfr_timing_begin."""
    return _timing_dict(lib().lwfr_timing_end, ctx)


def lwfr_graph_capture(ctx, u_a, u_b, nsteps, dt_ch_hist=None):
    _check(lib().lwfr_graph_capture(ctx, _ptr(u_a), _ptr(u_b), int(nsteps), _ptr(dt_ch_hist)))


def lwfr_graph_launch(ctx):
    _check(lib().lwfr_graph_launch(ctx))


def lwfr_destroy(ctx):
    _check(lib().lwfr_destroy(ctx))


def _timing_dict(fn, handle):
    n = len(TIMING_KERNELS)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_uint32 * n)()
    _check(fn(handle, ms, cnt))
    return {TIMING_KERNELS[k]: (ms[k], cnt[k]) for k in range(n)}


def _aligned(nbytes, device):
    import torch

    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off: off + nbytes]


class Stepper:
    """Owns a context, a workspace tensor and the stream binding for one configuration."""

    def __init__(self, cfg, device="cuda:0", stream=None):
        import torch

        self.cfg = cfg
        self.ctx = lwfr_init(cfg)
        self.device = torch.device(device)
        self.nbytes = lwfr_workspace_bytes(self.ctx)
        # 256-byte aligned workspace from the caching allocator
        self.workspace = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self.ws = self.workspace[off: off + self.nbytes]
        self.stream = stream
        lwfr_bind(self.ctx, self.ws, stream)
        n1 = cfg.degree + 1
        self.dim = DIMS[cfg.equation]
        self.nvars = NVARS[cfg.equation]
        self.nelem = cfg.nelem[0] * (cfg.nelem[1] if self.dim == 2 else 1)
        self.npts = n1 ** self.dim
        self.shape = (self.nvars, self.nelem, self.npts)
        self.xi, self.w = lwfr_reference_nodes(self.ctx, n1)

    def boundary_data_size(self):
        return lwfr_boundary_data_size(self.ctx)

    def set_boundary_data(self, ghost):
        self.ghost = ghost  # the library reads it at every step
        lwfr_set_boundary_data(self.ctx, ghost)

    def step(self, u_in, u_out, dt=0.0, dt_ch=None, alpha=None, flags=None, stats=None):
        lwfr_step(self.ctx, u_in, u_out, dt, dt_ch, alpha, flags, stats)

    def step_fixed(self, u_in, u_out, dt, ch, alpha=None, flags=None):
        lwfr_step_fixed(self.ctx, u_in, u_out, dt, ch, alpha, flags)

    def residual(self, u, dt, mode, R):
        lwfr_residual(self.ctx, u, dt, mode, R)

    def query(self):
        return lwfr_query(self.ctx)

    def adjoint_step(self, u_n, dt, lam_np1, lam_n, tape=None):
        lwfr_adjoint_step(self.ctx, u_n, dt, lam_np1, lam_n, tape)

    def new_tape(self):
        """A 256-byte aligned device buffer for one step's tape."""
        import torch

        n = lwfr_tape_bytes(self.ctx)
        buf = torch.empty(n + 256, dtype=torch.uint8, device=self.device)
        off = (-buf.data_ptr()) % 256
        return buf[off: off + n]

    def step_taped(self, u_in, u_out, dt, tape, dt_ch=None):
        lwfr_step_taped(self.ctx, u_in, u_out, dt, dt_ch, tape)

    def graph_capture(self, u_a, u_b, nsteps, dt_ch_hist=None):
        lwfr_graph_capture(self.ctx, u_a, u_b, nsteps, dt_ch_hist)

    def graph_launch(self):
        lwfr_graph_launch(self.ctx)

    def close(self):
        if self.ctx is not None:
            lwfr_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent problems advanced together (lwfr_batch_*).

    cfgs: a list of lwfr_config of one equation system.  The batch state is one
    flat float64 device tensor; view(u, i) is problem i's (nvars, nelem, npts)
    view of it."""

    def __init__(self, cfgs, device="cuda:0", stream=None):
        import torch

        self.cfgs = list(cfgs)
        arr = (lwfr_config * len(self.cfgs))(*self.cfgs)
        self.handle = ctypes.c_void_p()
        _check(lib().lwfr_batch_init(arr, len(self.cfgs), ctypes.byref(self.handle)))
        self.device = torch.device(device)
        n = ctypes.c_size_t()
        _check(lib().lwfr_batch_workspace_bytes(self.handle, ctypes.byref(n)))
        self.nbytes = n.value
        self.ws = _aligned(self.nbytes, self.device)
        offs = (ctypes.c_int64 * (len(self.cfgs) + 1))()
        _check(lib().lwfr_batch_state_offsets(self.handle, offs))
        self.offsets = list(offs)
        self.size = self.offsets[-1]
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(lib().lwfr_batch_bind(self.handle, ctypes.c_void_p(self.ws.data_ptr()), self.nbytes,
                                     ctypes.c_void_p(self.stream.cuda_stream)))
        self.shapes = []
        for c in self.cfgs:
            dim = DIMS[c.equation]
            ne = c.nelem[0] * (c.nelem[1] if dim == 2 else 1)
            self.shapes.append((NVARS[c.equation], ne, (c.degree + 1) ** dim))

    def __len__(self):
        return len(self.cfgs)

    def empty(self):
        import torch

        return torch.empty(self.size, dtype=torch.float64, device=self.device)

    def view(self, u, i):
        return u[self.offsets[i]: self.offsets[i + 1]].view(self.shapes[i])

    def problem(self, i):
        ctx = ctypes.c_void_p()
        _check(lib().lwfr_batch_problem(self.handle, int(i), ctypes.byref(ctx)))
        return ctx

    def step(self, u_in, u_out, dt=None):
        _check(lib().lwfr_batch_step(self.handle, _ptr(u_in), _ptr(u_out), _ptr(dt)))

    def set_launch(self, phase, tile_threads, grid, xcd):
        _check(lib().lwfr_batch_set_launch(self.handle, int(phase), int(tile_threads), int(grid), int(xcd)))

    def get_launch(self, phase):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().lwfr_batch_get_launch(self.handle, int(phase), ctypes.byref(a), ctypes.byref(b),
                                           ctypes.byref(c)))
        return a.value, b.value, c.value

    def autotune(self, u_in, u_out, reps=3):
        _check(lib().lwfr_batch_autotune(self.handle, _ptr(u_in), _ptr(u_out), int(reps)))

    def graph_capture(self, u_a, u_b, nsteps, dt_hist=None):
        _check(lib().lwfr_batch_graph_capture(self.handle, _ptr(u_a), _ptr(u_b), int(nsteps), _ptr(dt_hist)))

    def graph_launch(self):
        _check(lib().lwfr_batch_graph_launch(self.handle))

    def query(self):
        f = ctypes.c_uint32()
        st = lib().lwfr_batch_query(self.handle, ctypes.byref(f))
        return st, f.value

    def timing_begin(self, max_launches):
        _check(lib().lwfr_batch_timing_begin(self.handle, int(max_launches)))

    def timing_end(self):
        return _timing_dict(lib().lwfr_batch_timing_end, self.handle)

    def close(self):
        if self.handle is not None:
            lwfr_destroy_batch(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lwfr_destroy_batch(handle):
    _check(lib().lwfr_batch_destroy(handle))
