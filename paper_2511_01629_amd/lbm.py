"""Thin ctypes binding of liblbmpen.so (the C ABI in include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  PyTorch provides the device workspace (one uint8 tensor the
library carves its buffers from) and the stream the library queues on.

The library must have been built (python -m paper_2511_01629_amd.build, or
__graft_entry__.build()); loading raises LbmUnavailable otherwise -- there is
no CPU fallback.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbmpen.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ESTATE, LBM_EUNSTABLE, LBM_EDOMAIN = 0, -1, -2, -3, -4, -5, -6
LATTICES = {"D2Q9": 0, "D3Q19": 1}
STORAGES = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
SHAPES = {"disk": 0, "ellipse": 1, "sphere": 2}
CODES = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESTATE", -5: "EUNSTABLE", -6: "EDOMAIN"}

EXPORTS = ["lbm_workspace_size", "lbm_create", "lbm_destroy", "lbm_set_particles", "lbm_step", "lbm_step_record",
           "lbm_sync", "lbm_get_fields", "lbm_get_populations", "lbm_set_populations", "lbm_get_particles",
           "lbm_get_step", "lbm_last_error", "lbm_profile", "lbm_profile_read", "lbm_copy", "lbm_copy_arrays",
           "lbm_forward_checkpointed", "lbm_backward", "lbm_get_fields_device", "lbm_set_params",
           "lbm_state_size", "lbm_save_state", "lbm_load_state", "lbm_step_record_noalloc",
           "lbm_step_slabs", "lbm_grad_workspace_size", "lbm_forward_checkpointed_ws", "lbm_backward_ws",
           "lbm_grad_positions"]


class LbmUnavailable(RuntimeError):
    pass


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{CODES.get(code, code)}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [
        ("lattice", C.c_int32), ("storage", C.c_int32), ("n", C.c_int32 * 3), ("periodic", C.c_int32 * 3),
        ("tau", C.c_double), ("alpha", C.c_double), ("rho_f", C.c_double), ("g", C.c_double * 3),
        ("u0", C.c_double * 3), ("p0", C.c_double), ("eps_p", C.c_double), ("eps_w", C.c_double),
        ("delta", C.c_double), ("K", C.c_int32), ("collision_form", C.c_int32), ("gravity_form", C.c_int32),
        ("fluid_accel", C.c_double * 3), ("penalize_all", C.c_int32), ("device", C.c_int32),
        ("stream", C.c_void_p), ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
        ("max_particles", C.c_int32), ("wall_velocity", C.c_double * 18), ("check_every", C.c_int32),
        ("rigid_beta", C.c_double), ("no_stress_penalty", C.c_int32), ("max_radius", C.c_double),
        ("fractional_indicator", C.c_int32),
    ]


class Particle(C.Structure):
    _fields_ = [
        ("shape", C.c_int32), ("rho_s", C.c_double), ("a", C.c_double), ("b", C.c_double), ("x", C.c_double * 3),
        ("theta", C.c_double), ("U", C.c_double * 3), ("omega", C.c_double * 3), ("U_prev", C.c_double * 3),
        ("omega_prev", C.c_double * 3), ("A", C.c_double * 3), ("n_nodes", C.c_int32),
    ]


_LIB = None


def load():
    """Load liblbmpen.so; raise LbmUnavailable if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise LbmUnavailable(f"{LIB_PATH} is not built; run `python -m paper_2511_01629_amd.build`")
    # torch ships its own HIP runtime under the same soname as the system one;
    # load torch first so the library binds to the runtime that owns torch's
    # device memory and streams
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
    dp = C.POINTER(C.c_double)
    lib.lbm_workspace_size.argtypes = [C.POINTER(Config), C.POINTER(C.c_size_t)]
    lib.lbm_create.argtypes = [C.POINTER(Config), C.POINTER(P)]
    lib.lbm_destroy.argtypes = [P]
    lib.lbm_set_particles.argtypes = [P, C.POINTER(Particle), I32]
    lib.lbm_step.argtypes = [P, I64]
    lib.lbm_step_record.argtypes = [P, I64, dp]
    lib.lbm_sync.argtypes = [P]
    lib.lbm_get_fields.argtypes = [P, dp, dp, C.POINTER(C.c_int32)]
    lib.lbm_get_populations.argtypes = [P, dp]
    lib.lbm_set_populations.argtypes = [P, dp]
    lib.lbm_get_particles.argtypes = [P, C.POINTER(Particle), I32]
    lib.lbm_get_step.argtypes = [P, C.POINTER(C.c_int64)]
    lib.lbm_last_error.argtypes = [P]
    lib.lbm_last_error.restype = C.c_char_p
    lib.lbm_profile.argtypes = [P, I32]
    lib.lbm_profile_read.argtypes = [P, dp, C.POINTER(C.c_int64), I32]
    lib.lbm_copy.argtypes = [P, P, C.c_size_t, P]
    lib.lbm_copy_arrays.argtypes = [P, P, I32, C.c_size_t, P]
    lib.lbm_forward_checkpointed.argtypes = [P, I64, I32]
    lib.lbm_backward.argtypes = [P, dp, dp, dp, dp]
    lib.lbm_get_fields_device.argtypes = [P, P, P, P]
    lib.lbm_set_params.argtypes = [P, dp, C.c_double, dp]
    lib.lbm_state_size.argtypes = [P, C.POINTER(C.c_size_t)]
    lib.lbm_save_state.argtypes = [P, P]
    lib.lbm_load_state.argtypes = [P, P]
    lib.lbm_step_record_noalloc.argtypes = [P, I64, dp]
    lib.lbm_step_slabs.argtypes = [P, I64, I32]
    lib.lbm_grad_workspace_size.argtypes = [P, I64, I32, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
    lib.lbm_forward_checkpointed_ws.argtypes = [P, I64, I32, P, C.c_size_t]
    lib.lbm_backward_ws.argtypes = [P, dp, dp, dp, dp, P, C.c_size_t]
    lib.lbm_grad_positions.argtypes = [P, dp]
    _LIB = lib
    return lib


def _vec3(v):
    v = [float(t) for t in v] + [0.0] * 3
    return (C.c_double * 3)(*v[:3])


def make_config(cfg, storage=None, device=0, max_particles=0):
    c = Config()
    c.lattice = LATTICES[cfg.get("lattice", "D2Q9")]
    c.storage = STORAGES[storage or cfg.get("storage", "f64")]
    n = list(cfg["n"]) + [1, 1]
    c.n = (C.c_int32 * 3)(*[int(v) for v in n[:3]])
    per = list(cfg.get("periodic", (0, 0, 0))) + [0, 0, 0]
    c.periodic = (C.c_int32 * 3)(*[int(bool(v)) for v in per[:3]])
    c.tau = float(cfg["tau"])
    c.alpha = float(cfg.get("alpha", 0.0))
    c.rho_f = float(cfg.get("rho_f", 1.0))
    c.g = _vec3(cfg.get("g", (0, 0, 0)))
    c.u0 = _vec3(cfg.get("u0", (0, 0, 0)))
    c.p0 = float(cfg.get("p0", 0.0))
    c.eps_p = float(cfg.get("eps_p", 2.0))
    c.eps_w = float(cfg.get("eps_w", 1.0))
    c.delta = float(cfg.get("delta", 1.0))
    c.K = int(cfg.get("K", 1))
    c.collision_form = int(cfg.get("collision_form", 0))
    c.gravity_form = int(cfg.get("gravity_form", 0))
    c.fluid_accel = _vec3(cfg.get("fluid_accel", (0, 0, 0)))
    c.penalize_all = int(bool(cfg.get("penalize_all", 0)))
    c.device = int(device)
    c.max_particles = int(max_particles)
    # wall_velocity: [axis][low, high wall][component], tangential velocities of moving walls
    wv = np.zeros((3, 2, 3))
    if cfg.get("wall_velocity") is not None:
        w = np.asarray(cfg["wall_velocity"], dtype=np.float64)
        wv[: w.shape[0], : w.shape[1], : w.shape[2]] = w
    c.wall_velocity = (C.c_double * 18)(*wv.ravel())
    c.check_every = int(cfg.get("check_every", 0))
    c.rigid_beta = float(cfg.get("rigid_beta", 0.0))
    c.no_stress_penalty = int(bool(cfg.get("no_stress_penalty", 0)))
    c.max_radius = float(cfg.get("max_radius", 0.0))
    c.fractional_indicator = int(bool(cfg.get("fractional", 0)))
    return c


def make_particles(parts):
    arr = (Particle * max(1, len(parts)))()
    for i, p in enumerate(parts):
        arr[i].shape = SHAPES[p["shape"]] if isinstance(p["shape"], str) else int(p["shape"])
        arr[i].rho_s = float(p["rho_s"])
        arr[i].a = float(p["a"])
        arr[i].b = float(p.get("b", p["a"]))
        arr[i].x = _vec3(p["x"])
        arr[i].theta = float(p.get("theta", 0.0))
    return arr


def copy(dst_ptr, src_ptr, nbytes, stream_handle):
    """Device copy with the library's streaming copy kernel (measurement aid)."""
    rc = load().lbm_copy(C.c_void_p(dst_ptr), C.c_void_p(src_ptr), int(nbytes), C.c_void_p(stream_handle))
    if rc != LBM_OK:
        raise LbmError(rc, "lbm_copy failed")


def copy_arrays(dst_ptr, src_ptr, narrays, bytes_per_array, stream_handle):
    """Copy of narrays consecutive arrays in one kernel (measurement aid: the
    lattice update's pattern of Q concurrent streams)."""
    rc = load().lbm_copy_arrays(C.c_void_p(dst_ptr), C.c_void_p(src_ptr), int(narrays), int(bytes_per_array),
                                C.c_void_p(stream_handle))
    if rc != LBM_OK:
        raise LbmError(rc, "lbm_copy_arrays failed")


class Simulation:
    """One context of the HIP library on cuda:`device`.

    cfg/particles are the plain dicts of paper_2511_01629_amd.workloads;
    `storage` overrides cfg["storage"] ("f64", "f32", "f16", "bf16")."""

    def __init__(self, cfg, particles=(), storage=None, device=0, max_particles=None, stream=None):
        import torch

        self.lib = load()
        self.torch = torch
        self.device = device
        self.cfg = dict(cfg)
        self.d = 2 if cfg.get("lattice", "D2Q9") == "D2Q9" else 3
        self.Q = 9 if self.d == 2 else 19
        n = list(cfg["n"]) + [1, 1]
        self.shape = (n[2] if self.d == 3 else 1, n[1], n[0])
        self.N = int(np.prod(self.shape))
        cap = max_particles if max_particles is not None else max(len(particles), 1)
        if "max_radius" not in cfg and len(particles):
            # the workspace (a torch tensor) then also holds the momentum-sum slot tables
            cfg = dict(cfg, max_radius=max(float(p["a"]) for p in particles))
        self._cfg = make_config(cfg, storage, device, cap)
        size = C.c_size_t()
        self._check(self.lib.lbm_workspace_size(C.byref(self._cfg), C.byref(size)), None)
        dev = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.workspace = torch.empty(int(size.value), dtype=torch.uint8, device=dev)
        self._cfg.workspace = C.c_void_p(self.workspace.data_ptr())
        self._cfg.workspace_bytes = int(size.value)
        self._cfg.stream = C.c_void_p(self.stream.cuda_stream)
        self.ctx = C.c_void_p()
        self._check(self.lib.lbm_create(C.byref(self._cfg), C.byref(self.ctx)), None)
        self.np = 0
        if len(particles):
            self.set_particles(particles)

    # ------------------------------------------------------------ plumbing
    def _check(self, rc, ctx=...):
        if rc != LBM_OK:
            c = self.ctx if ctx is ... else ctx
            msg = self.lib.lbm_last_error(c if c else None).decode()
            raise LbmError(rc, msg)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ the ABI
    def set_particles(self, parts):
        arr = make_particles(parts)
        self._check(self.lib.lbm_set_particles(self.ctx, arr, len(parts)))
        self.np = len(parts)

    def step(self, n=1):
        self._check(self.lib.lbm_step(self.ctx, int(n)))

    def step_slabs(self, n, nslabs=2):
        """n steps with the lattice cut into nslabs slabs (explicit halo
        copies and cross-slab momentum sums); same result as step(n)."""
        self._check(self.lib.lbm_step_slabs(self.ctx, int(n), int(nslabs)))

    def step_record(self, n):
        rec = np.zeros((int(n), max(self.np, 1), 14))
        self._check(self.lib.lbm_step_record(self.ctx, int(n), rec.ctypes.data_as(C.POINTER(C.c_double))))
        return rec[:, : self.np]

    def step_record_noalloc(self, n):
        """step_record through the library's static record array (no device
        allocation by the library)."""
        rec = np.zeros((int(n), max(self.np, 1), 14))
        self._check(self.lib.lbm_step_record_noalloc(self.ctx, int(n), rec.ctypes.data_as(C.POINTER(C.c_double))))
        return rec[:, : self.np]

    def sync(self):
        self._check(self.lib.lbm_sync(self.ctx))

    @property
    def step_index(self):
        s = C.c_int64()
        self._check(self.lib.lbm_get_step(self.ctx, C.byref(s)))
        return s.value

    def grad_workspace_size(self, nsteps, every):
        f, b = C.c_size_t(), C.c_size_t()
        self._check(self.lib.lbm_grad_workspace_size(self.ctx, int(nsteps), int(every), C.byref(f), C.byref(b)))
        return int(f.value), int(b.value)

    def forward_checkpointed(self, nsteps, every, torch_memory=False):
        """The differentiated forward run.  torch_memory: its checkpoints live
        in a torch tensor held by this object (torch's allocator owns them),
        and backward() takes its scratch from torch too."""
        self._grad_torch = bool(torch_memory)
        if not torch_memory:
            self._fwd_ws = None
            self._check(self.lib.lbm_forward_checkpointed(self.ctx, int(nsteps), int(every)))
            return
        fb, self._bwd_bytes = self.grad_workspace_size(nsteps, every)
        self._fwd_ws = self.torch.empty(fb, dtype=self.torch.uint8, device=self.workspace.device)
        self._check(self.lib.lbm_forward_checkpointed_ws(self.ctx, int(nsteps), int(every),
                                                         C.c_void_p(self._fwd_ws.data_ptr()), fb))

    def backward(self, dL_dX):
        """Gradients (d rho_s [n], d tau, d |g|) of a loss whose gradient with
        respect to the final centres is dL_dX (n x 3)."""
        seed = np.ascontiguousarray(np.asarray(dL_dX, dtype=np.float64).reshape(self.np, 3))
        g_rho = np.zeros(max(self.np, 1))
        g_tau = C.c_double()
        g_g = C.c_double()
        dp = C.POINTER(C.c_double)
        if getattr(self, "_grad_torch", False):
            ws = self.torch.empty(self._bwd_bytes, dtype=self.torch.uint8, device=self.workspace.device)
            self._check(self.lib.lbm_backward_ws(self.ctx, seed.ctypes.data_as(dp), g_rho.ctypes.data_as(dp),
                                                 C.byref(g_tau), C.byref(g_g), C.c_void_p(ws.data_ptr()),
                                                 self._bwd_bytes))
            del ws
        else:
            self._check(self.lib.lbm_backward(self.ctx, seed.ctypes.data_as(dp), g_rho.ctypes.data_as(dp),
                                              C.byref(g_tau), C.byref(g_g)))
        return g_rho[: self.np], g_tau.value, g_g.value

    def grad_positions(self):
        """dL/dX^0 (n x 3) of the last backward sweep."""
        out = np.zeros((max(self.np, 1), 3))
        self._check(self.lib.lbm_grad_positions(self.ctx, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out[: self.np]

    KERNELS = ("stream_collide", "reduce_clear", "rigid_raster", "raster_after_substeps", "rigid_forcing")

    def profile(self, enable=True):
        self._check(self.lib.lbm_profile(self.ctx, int(bool(enable))))

    def profile_read(self, reset=True):
        ms = np.zeros(len(self.KERNELS))
        cnt = np.zeros(len(self.KERNELS), dtype=np.int64)
        self._check(self.lib.lbm_profile_read(self.ctx, ms.ctypes.data_as(C.POINTER(C.c_double)),
                                              cnt.ctypes.data_as(C.POINTER(C.c_int64)), int(bool(reset))))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(self.KERNELS)}

    def fields(self):
        u = np.zeros(self.N * self.d)
        p = np.zeros(self.N)
        own = np.zeros(self.N, dtype=np.int32)
        self._check(self.lib.lbm_get_fields(self.ctx, u.ctypes.data_as(C.POINTER(C.c_double)),
                                            p.ctypes.data_as(C.POINTER(C.c_double)),
                                            own.ctypes.data_as(C.POINTER(C.c_int32))))
        return u.reshape(*self.shape, self.d), p.reshape(self.shape), own.reshape(self.shape)

    def populations(self):
        """f^n as (nz, ny, nx, Q) FP64."""
        f = np.zeros(self.Q * self.N)
        self._check(self.lib.lbm_get_populations(self.ctx, f.ctypes.data_as(C.POINTER(C.c_double))))
        return np.moveaxis(f.reshape(self.Q, *self.shape), 0, -1)

    def set_populations(self, f):
        f = np.ascontiguousarray(np.moveaxis(np.asarray(f, dtype=np.float64).reshape(*self.shape, self.Q), -1, 0))
        self._check(self.lib.lbm_set_populations(self.ctx, f.ctypes.data_as(C.POINTER(C.c_double))))

    def fields_device(self):
        """u (nz, ny, nx, d), p (nz, ny, nx) float64 and owner (nz, ny, nx) int32
        as torch tensors on the context's device, filled on its stream (no
        host round trip)."""
        t = self.torch
        dev = self.workspace.device
        u = t.empty((*self.shape, self.d), dtype=t.float64, device=dev)
        p = t.empty(self.shape, dtype=t.float64, device=dev)
        own = t.empty(self.shape, dtype=t.int32, device=dev)
        self._check(self.lib.lbm_get_fields_device(self.ctx, C.c_void_p(u.data_ptr()), C.c_void_p(p.data_ptr()),
                                                   C.c_void_p(own.data_ptr())))
        return u, p, own

    def set_params(self, rho_s=None, tau=None, g=None):
        """Replace the solid densities (n), tau and/or the gravity vector;
        None keeps a value."""
        rho = None
        if rho_s is not None:
            rho = np.ascontiguousarray(np.asarray(rho_s, dtype=np.float64).reshape(self.np))
        gv = None
        if g is not None:
            gv = np.ascontiguousarray((list(np.asarray(g, dtype=np.float64).ravel()) + [0.0, 0.0, 0.0])[:3])
        dp = C.POINTER(C.c_double)
        self._check(self.lib.lbm_set_params(self.ctx, rho.ctypes.data_as(dp) if rho is not None else None,
                                            float(tau) if tau is not None else 0.0,
                                            gv.ctypes.data_as(dp) if gv is not None else None))

    def state_size(self):
        n = C.c_size_t()
        self._check(self.lib.lbm_state_size(self.ctx, C.byref(n)))
        return int(n.value)

    def save_state(self, on_device=False):
        """The whole between-step state as bytes: a numpy uint8 array (host) or,
        with on_device, a torch uint8 tensor on the context's device."""
        n = self.state_size()
        if on_device:
            buf = self.torch.empty(n, dtype=self.torch.uint8, device=self.workspace.device)
            ptr = buf.data_ptr()
        else:
            buf = np.zeros(n, dtype=np.uint8)
            ptr = buf.ctypes.data
        self._check(self.lib.lbm_save_state(self.ctx, C.c_void_p(ptr)))
        return buf

    def load_state(self, buf):
        """Install a state saved by save_state (host array or device tensor)."""
        if hasattr(buf, "data_ptr"):
            ptr = buf.data_ptr()
        else:
            buf = np.ascontiguousarray(buf, dtype=np.uint8)
            ptr = buf.ctypes.data
        self._check(self.lib.lbm_load_state(self.ctx, C.c_void_p(ptr)))
        hdr = np.frombuffer(bytes(buf[:64].cpu().numpy()) if hasattr(buf, "cpu") else bytes(buf[:64]), dtype=np.int32)
        self.np = int(hdr[11])

    def particles(self):
        arr = (Particle * max(self.np, 1))()
        self._check(self.lib.lbm_get_particles(self.ctx, arr, self.np))
        g = lambda name: np.array([list(getattr(arr[i], name)) for i in range(self.np)]).reshape(self.np, 3)
        return {
            "X": g("x"), "theta": np.array([arr[i].theta for i in range(self.np)]), "U": g("U"), "omega": g("omega"),
            "U_prev": g("U_prev"), "omega_prev": g("omega_prev"), "A": g("A"),
            "N": np.array([arr[i].n_nodes for i in range(self.np)], dtype=np.int64),
        }
