"""ctypes front end of the FP64 CPU oracle (lbm_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it; the product path never does.  It imports nothing
from the GPU package.

Configurations and particles are plain dicts:
  cfg = dict(lattice="D2Q9"|"D3Q19", n=(nx, ny, nz), periodic=(px, py, pz),
             tau=..., alpha=0 (-> 1/tau), rho_f=1, g=(gx, gy, gz), u0=(...),
             p0=0, eps_p=2, eps_w=1, delta=1, K=1, collision_form=0,
             gravity_form=0, fluid_accel=(0, 0, 0), penalize_all=0,
             wall_velocity=None or [axis][low, high wall][component],
             rigid_beta=0 (rigid-velocity forcing, an extension), no_stress_penalty=0,
             fractional=0 (1: the fractional indicator, an extension; disks and spheres))
  particle = dict(shape="disk"|"ellipse"|"sphere", rho_s=..., a=..., b=...,
                  x=(X, Y, Z), theta=...)
Fields come back with shape (nz, ny, nx, ...) (x fastest).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

SHAPES = {"disk": 0, "ellipse": 1, "sphere": 2}
LATTICES = {"D2Q9": 0, "D3Q19": 1}
REC_W = 14  # X[3] theta U[3] W[3] A[3] N
PART_W = 22  # X[3] theta U[3] W[3] Uprev[3] Wprev[3] A[3] N Nw pad


class _Cfg(C.Structure):
    _fields_ = [
        ("lattice", C.c_int), ("n", C.c_int * 3), ("periodic", C.c_int * 3),
        ("tau", C.c_double), ("alpha", C.c_double), ("rho_f", C.c_double),
        ("g", C.c_double * 3), ("u0", C.c_double * 3), ("p0", C.c_double),
        ("eps_p", C.c_double), ("eps_w", C.c_double), ("delta", C.c_double),
        ("K", C.c_int), ("collision_form", C.c_int), ("gravity_form", C.c_int),
        ("fluid_accel", C.c_double * 3), ("penalize_all", C.c_int),
        ("wall_u", C.c_double * 18), ("rigid_beta", C.c_double), ("no_stress_penalty", C.c_int),
        ("fractional", C.c_int),
    ]


class _Pin(C.Structure):
    _fields_ = [
        ("shape", C.c_int), ("rho_s", C.c_double), ("a", C.c_double), ("b", C.c_double),
        ("x", C.c_double * 3), ("theta", C.c_double),
    ]


_LIBS = {}


def _lib(complex_step=False):
    if complex_step not in _LIBS:
        path = _build.lib_path(complex_step)
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build(force=True)
        lib = C.CDLL(path)
        P, D, I, L = C.c_void_p, C.c_double, C.c_int, C.c_long
        dp = C.POINTER(C.c_double)
        lib.ora_create.argtypes = [C.POINTER(_Cfg), C.POINTER(P)]
        lib.ora_destroy.argtypes = [P]
        lib.ora_destroy.restype = None
        lib.ora_perturb.argtypes = [P, dp, I, D, D, D, dp]
        lib.ora_set_particles.argtypes = [P, I, C.POINTER(_Pin)]
        lib.ora_set_replay.argtypes = [P, L, L, dp, dp]
        lib.ora_step.argtypes = [P, L, dp, dp]
        lib.ora_get_step.argtypes = [P]
        lib.ora_get_step.restype = L
        lib.ora_get_f.argtypes = [P, dp, dp]
        lib.ora_set_f.argtypes = [P, dp]
        lib.ora_get_fields.argtypes = [P, dp, dp, C.POINTER(C.c_int32)]
        lib.ora_get_particles.argtypes = [P, dp, dp]
        lib.ora_load_particles.argtypes = [P, dp, L]
        if not complex_step:
            ip = C.POINTER(C.c_int)
            lib.ora_lattice.argtypes = [I, ip, ip, ip, dp, ip]
            lib.ora_feq.argtypes = [I, D, dp, dp]
            lib.ora_macro.argtypes = [I, dp, dp, dp, dp]
            lib.ora_guo.argtypes = [I, D, dp, dp, dp]
            lib.ora_penal.argtypes = [I, D, dp, dp, dp]
            lib.ora_collide.argtypes = [I, D, D, I, dp, dp, dp]
            lib.ora_coll_forces.argtypes = [P, dp]
        _LIBS[complex_step] = lib
    return _LIBS[complex_step]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _vec3(v):
    v = list(v) + [0.0] * (3 - len(v))
    return (C.c_double * 3)(*[float(t) for t in v[:3]])


def _make_cfg(cfg):
    c = _Cfg()
    c.lattice = LATTICES[cfg.get("lattice", "D2Q9")]
    n = list(cfg["n"]) + [1] * (3 - len(cfg["n"]))
    c.n = (C.c_int * 3)(*n)
    per = list(cfg.get("periodic", (0, 0, 0))) + [0] * 3
    c.periodic = (C.c_int * 3)(*[int(bool(p)) for p in per[:3]])
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
    # wall_velocity: [axis][low, high][component] tangential wall velocities
    wv = np.zeros((3, 2, 3))
    if cfg.get("wall_velocity") is not None:
        w = np.asarray(cfg["wall_velocity"], dtype=np.float64)
        wv[: w.shape[0], : w.shape[1], : w.shape[2]] = w
    c.wall_u = (C.c_double * 18)(*wv.ravel())
    c.rigid_beta = float(cfg.get("rigid_beta", 0.0))
    c.no_stress_penalty = int(bool(cfg.get("no_stress_penalty", 0)))
    c.fractional = int(bool(cfg.get("fractional", 0)))
    return c


def _make_pins(parts):
    arr = (_Pin * max(1, len(parts)))()
    for i, p in enumerate(parts):
        arr[i].shape = SHAPES[p["shape"]] if isinstance(p["shape"], str) else int(p["shape"])
        arr[i].rho_s = float(p["rho_s"])
        arr[i].a = float(p["a"])
        arr[i].b = float(p.get("b", p["a"]))
        arr[i].x = _vec3(p["x"])
        arr[i].theta = float(p.get("theta", 0.0))
    return arr


class Oracle:
    """One oracle run.  complex_step=dict(d_rho_s=[...], d_tau=.., d_gmag=.., d_X=[[..]]*np, h=..)
    selects the complex-step build and seeds the perturbation of the
    parameters and of the initial centres."""

    def __init__(self, cfg, particles=(), complex_step=None):
        self.cs = complex_step is not None
        self.lib = _lib(self.cs)
        self.cfg = dict(cfg)
        self._c = _make_cfg(cfg)
        self.Q = 9 if self._c.lattice == 0 else 19
        self.d = 2 if self._c.lattice == 0 else 3
        n = list(cfg["n"]) + [1] * 3
        self.shape = (n[2] if self.d == 3 else 1, n[1], n[0])
        self.N = int(np.prod(self.shape))
        self.ctx = C.c_void_p()
        rc = self.lib.ora_create(C.byref(self._c), C.byref(self.ctx))
        if rc != 0:
            raise ValueError(f"oracle rejected the configuration (rc={rc})")
        self.np = len(particles)
        if self.cs:
            cs = complex_step
            drho = np.ascontiguousarray(np.asarray(cs.get("d_rho_s", np.zeros(self.np)), dtype=np.float64))
            dX = np.zeros((max(self.np, 1), 3))
            if cs.get("d_X") is not None:
                dX[: self.np] = np.asarray(cs["d_X"], dtype=np.float64).reshape(self.np, 3)
            dX = np.ascontiguousarray(dX)
            rc = self.lib.ora_perturb(self.ctx, _dp(drho), len(drho), float(cs.get("d_tau", 0.0)),
                                      float(cs.get("d_gmag", 0.0)), float(cs["h"]), _dp(dX))
            if rc != 0:
                raise RuntimeError("complex-step seed rejected")
        pins = _make_pins(particles)
        if self.lib.ora_set_particles(self.ctx, self.np, pins) != 0:
            raise ValueError("oracle rejected the particles (the fractional indicator takes disks and spheres)")

    def reset_particles(self, particles):
        """Copy particles in again: re-rasterise and re-measure U^0 (= U^{-1})
        from the current populations."""
        self.np = len(particles)
        if self.lib.ora_set_particles(self.ctx, self.np, _make_pins(particles)) != 0:
            raise ValueError("oracle rejected the particles (the fractional indicator takes disks and spheres)")

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            self.lib.ora_destroy(ctx)
            self.ctx = None

    @property
    def step_index(self):
        return self.lib.ora_get_step(self.ctx)

    def step(self, n=1, record=False):
        if not record:
            self.lib.ora_step(self.ctx, int(n), None, None)
            return None
        re = np.zeros((n, self.np, REC_W))
        im = np.zeros((n, self.np, REC_W)) if self.cs else None
        self.lib.ora_step(self.ctx, int(n), _dp(re), _dp(im) if im is not None else None)
        return (re, im) if self.cs else re

    def set_replay(self, n0, X, theta):
        X = np.ascontiguousarray(X, dtype=np.float64)
        th = np.ascontiguousarray(theta, dtype=np.float64)
        assert X.shape[1:] == (self.np, 3) and th.shape == X.shape[:2]
        self._rep = (X, th)
        self.lib.ora_set_replay(self.ctx, int(n0), X.shape[0], _dp(X), _dp(th))

    def f(self, imag=False):
        out = np.zeros(self.N * self.Q)
        if imag:
            self.lib.ora_get_f(self.ctx, None, _dp(out))
        else:
            self.lib.ora_get_f(self.ctx, _dp(out), None)
        return out.reshape(*self.shape, self.Q)

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        assert f.size == self.N * self.Q
        self.lib.ora_set_f(self.ctx, _dp(f))

    def fields(self):
        u = np.zeros(self.N * 3)
        p = np.zeros(self.N)
        own = np.zeros(self.N, dtype=np.int32)
        self.lib.ora_get_fields(self.ctx, _dp(u), _dp(p), own.ctypes.data_as(C.POINTER(C.c_int32)))
        return u.reshape(*self.shape, 3)[..., : self.d], p.reshape(self.shape), own.reshape(self.shape)

    def particles(self, imag=False):
        raw = np.zeros((max(self.np, 1), PART_W))
        if imag:
            self.lib.ora_get_particles(self.ctx, None, _dp(raw))
        else:
            self.lib.ora_get_particles(self.ctx, _dp(raw), None)
        raw = raw[: self.np]
        return {
            "X": raw[:, 0:3], "theta": raw[:, 3], "U": raw[:, 4:7], "omega": raw[:, 7:10],
            "U_prev": raw[:, 10:13], "omega_prev": raw[:, 13:16], "A": raw[:, 16:19],
            "N": raw[:, 19].astype(np.int64), "Nw": raw[:, 20], "raw": raw,
        }

    def load_particles(self, raw, step):
        raw = np.ascontiguousarray(raw, dtype=np.float64)
        self.lib.ora_load_particles(self.ctx, _dp(raw), int(step))

    def collision_forces(self):
        F = np.zeros((max(self.np, 1), 3))
        self.lib.ora_coll_forces(self.ctx, _dp(F))
        return F[: self.np]


# ---------------------------------------------------------------- per node

def lattice(kind="D2Q9"):
    lib = _lib(False)
    Q, d = C.c_int(), C.c_int()
    c = (C.c_int * 57)()
    w = np.zeros(19)
    opp = (C.c_int * 19)()
    lib.ora_lattice(LATTICES[kind], C.byref(Q), C.byref(d), c, _dp(w), opp)
    q = Q.value
    return np.array(c[: 3 * q]).reshape(q, 3), w[:q].copy(), np.array(opp[:q])


def _q(kind):
    return 9 if kind == "D2Q9" else 19


def feq(kind, p, u):
    out = np.zeros(_q(kind))
    u = np.ascontiguousarray(list(u) + [0.0] * (3 - len(u)), dtype=np.float64)
    _lib(False).ora_feq(LATTICES[kind], float(p), _dp(u), _dp(out))
    return out


def macro(kind, f, acc=(0, 0, 0)):
    f = np.ascontiguousarray(f, dtype=np.float64)
    a = np.ascontiguousarray(list(acc) + [0.0] * (3 - len(acc)), dtype=np.float64)
    u = np.zeros(3)
    p = np.zeros(1)
    _lib(False).ora_macro(LATTICES[kind], _dp(f), _dp(a), _dp(u), _dp(p))
    return u, float(p[0])


def guo(kind, tau, u, acc):
    out = np.zeros(_q(kind))
    u = np.ascontiguousarray(list(u) + [0.0] * (3 - len(u)), dtype=np.float64)
    a = np.ascontiguousarray(list(acc) + [0.0] * (3 - len(acc)), dtype=np.float64)
    _lib(False).ora_guo(LATTICES[kind], float(tau), _dp(u), _dp(a), _dp(out))
    return out


def penal(kind, alpha, f, fe):
    out = np.zeros(_q(kind))
    f = np.ascontiguousarray(f, dtype=np.float64)
    fe = np.ascontiguousarray(fe, dtype=np.float64)
    _lib(False).ora_penal(LATTICES[kind], float(alpha), _dp(f), _dp(fe), _dp(out))
    return out


def collide(kind, tau, alpha, solid, f, acc=(0, 0, 0)):
    out = np.zeros(_q(kind))
    f = np.ascontiguousarray(f, dtype=np.float64)
    a = np.ascontiguousarray(list(acc) + [0.0] * (3 - len(acc)), dtype=np.float64)
    _lib(False).ora_collide(LATTICES[kind], float(tau), float(alpha), int(bool(solid)), _dp(f), _dp(a), _dp(out))
    return out
