"""ctypes binding of the FP64 CPU oracle (``oracle/lco.c``).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  Shares no code with the HIP library.

Arrays are numpy float64 in structure-of-arrays layout
``[component, z, y, x]``; Q has the five components (xx, xy, xz, yy, yz).
"""
import ctypes
import math
import os

import numpy as np

from . import build as _build

ANCHOR_NONE, ANCHOR_NORMAL, ANCHOR_PLANAR = 0, 1, 2
FIXED, PRESCRIBED, FREE = 0, 1, 2
MAX_COLLOIDS = 16
COLLOID_GAP = 3.0

_lib = None


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("hydro", ctypes.c_int),
                ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
                ("A0", ctypes.c_double), ("gamma", ctypes.c_double), ("K", ctypes.c_double),
                ("q0", ctypes.c_double), ("xi", ctypes.c_double), ("Gamma", ctypes.c_double),
                ("body_force", ctypes.c_double * 3),
                ("advection", ctypes.c_int), ("stencil", ctypes.c_int)]


class Colloid(ctypes.Structure):
    _fields_ = [("present", ctypes.c_int), ("motion", ctypes.c_int),
                ("anchoring", ctypes.c_int), ("pad_", ctypes.c_int),
                ("pos", ctypes.c_double * 3), ("a0", ctypes.c_double),
                ("vel", ctypes.c_double * 3), ("omega", ctypes.c_double * 3),
                ("S0", ctypes.c_double), ("W", ctypes.c_double),
                ("fext", ctypes.c_double * 3), ("rho_c", ctypes.c_double)]


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        L.lco_create.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(vp)]
        L.lco_destroy.argtypes = [vp]
        L.lco_destroy.restype = None
        L.lco_set_colloid.argtypes = [vp, ctypes.POINTER(Colloid)]
        L.lco_get_colloid.argtypes = [vp, ctypes.POINTER(Colloid)]
        L.lco_set_colloids.argtypes = [vp, ctypes.c_int, ctypes.POINTER(Colloid)]
        L.lco_get_colloids.argtypes = [vp, ctypes.c_int, ctypes.POINTER(Colloid)]
        L.lco_num_colloids.argtypes = [vp]
        L.lco_get_forces.argtypes = [vp, ctypes.c_int, dp]
        for name in ("lco_set_Q", "lco_set_f", "lco_set_u", "lco_get_Q", "lco_get_f",
                     "lco_get_u", "lco_get_force", "lco_get_diag", "lco_ghost"):
            getattr(L, name).argtypes = [vp, dp]
        L.lco_get_solid.argtypes = [vp, ctypes.POINTER(ctypes.c_ubyte)]
        L.lco_step.argtypes = [vp, ctypes.c_int]
        L.lco_get_nstep.argtypes = [vp]
        L.lco_get_nstep.restype = ctypes.c_long
        L.lco_fields.argtypes = [vp, dp, dp, dp]
        L.lco_bulk_field.argtypes = [ctypes.POINTER(Params), dp, dp]
        L.lco_bulk_field.restype = None
        L.lco_corotation.argtypes = [ctypes.c_double, dp, dp, dp]
        L.lco_corotation.restype = None
        L.lco_feq.argtypes = [ctypes.c_double, dp, dp]
        L.lco_feq.restype = None
        L.lco_lattice.argtypes = [ctypes.POINTER(ctypes.c_int), dp]
        L.lco_lattice.restype = None
        L.lco_principal_axis.argtypes = [dp, dp, dp]
        L.lco_single_site.argtypes = [ctypes.POINTER(Params), dp, ctypes.c_long, dp]
        L.lco_single_site.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(nx, ny, nz, hydro=1, tau=1.0, rho0=1.0, A0=0.01, gamma=3.0, K=0.01, q0=0.0,
                xi=0.7, Gamma=0.5, body_force=(0.0, 0.0, 0.0), advection=1, stencil=7):
    p = Params()
    p.advection, p.stencil = advection, stencil
    p.nx, p.ny, p.nz, p.hydro = nx, ny, nz, hydro
    p.tau, p.rho0, p.A0, p.gamma, p.K, p.q0, p.xi, p.Gamma = tau, rho0, A0, gamma, K, q0, xi, Gamma
    for a in range(3):
        p.body_force[a] = body_force[a]
    return p


def make_colloid(pos, a0, anchoring=ANCHOR_NORMAL, W=math.inf, S0=0.5, vel=(0, 0, 0),
                 omega=(0, 0, 0), motion=FIXED, present=1, fext=(0, 0, 0), rho_c=0.0):
    c = Colloid()
    c.present, c.motion, c.anchoring = present, motion, anchoring
    for a in range(3):
        c.pos[a], c.vel[a], c.omega[a], c.fext[a] = pos[a], vel[a], omega[a], fext[a]
    c.a0, c.S0, c.W, c.rho_c = a0, S0, W, rho_c
    return c


def lattice():
    c = (ctypes.c_int * 57)()
    w = np.zeros(19)
    lib().lco_lattice(c, _dp(w))
    return np.array(list(c), dtype=np.int64).reshape(19, 3), w


def feq(rho, u):
    out = np.zeros(19)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    lib().lco_feq(rho, _dp(uu), _dp(out))
    return out


def bulk_field(params, Q5):
    q = np.ascontiguousarray(Q5, dtype=np.float64)
    h = np.zeros(5)
    lib().lco_bulk_field(ctypes.byref(params), _dp(q), _dp(h))
    return h


def corotation(xi, W, Q5):
    w = np.ascontiguousarray(np.asarray(W, dtype=np.float64).reshape(9))
    q = np.ascontiguousarray(Q5, dtype=np.float64)
    s = np.zeros(5)
    lib().lco_corotation(xi, _dp(w), _dp(q), _dp(s))
    return s


def principal_axis(A):
    a = np.ascontiguousarray(np.asarray(A, dtype=np.float64).reshape(9))
    n = np.zeros(3)
    lam = np.zeros(1)
    lib().lco_principal_axis(_dp(a), _dp(n), _dp(lam))
    return n, float(lam[0])


def single_site(params, W, nsteps, Q5):
    w = np.ascontiguousarray(np.asarray(W, dtype=np.float64).reshape(9))
    q = np.array(Q5, dtype=np.float64)
    lib().lco_single_site(ctypes.byref(params), _dp(w), nsteps, _dp(q))
    return q


class Sim:
    """One periodic box with up to 16 colloids, stepped in FP64."""

    def __init__(self, nx, ny=None, nz=None, **kw):
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        self.params = make_params(nx, ny, nz, **kw)
        h = ctypes.c_void_p()
        rc = lib().lco_create(ctypes.byref(self.params), ctypes.byref(h))
        if rc != 0:
            raise ValueError("lco_create failed with code %d" % rc)
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().lco_destroy(h)
            self._h = None

    def _chk(self, rc, what):
        if rc != 0:
            raise ValueError("%s failed with code %d" % (what, rc))

    def set_colloid(self, pos, a0, **kw):
        self.colloid = make_colloid(pos, a0, **kw)
        self._chk(lib().lco_set_colloid(self._h, ctypes.byref(self.colloid)), "lco_set_colloid")

    def get_colloid(self):
        c = Colloid()
        self._chk(lib().lco_get_colloid(self._h, ctypes.byref(c)), "lco_get_colloid")
        return c

    def set_colloids(self, specs):
        """specs: list of dicts with pos, a0 and make_colloid's keywords."""
        arr = (Colloid * max(1, len(specs)))()
        for k, sp in enumerate(specs):
            sp = dict(sp)
            arr[k] = make_colloid(sp.pop("pos"), sp.pop("a0"), **sp)
        self._chk(lib().lco_set_colloids(self._h, len(specs), arr), "lco_set_colloids")

    def num_colloids(self):
        return int(lib().lco_num_colloids(self._h))

    def get_colloids(self):
        n = self.num_colloids()
        arr = (Colloid * max(1, n))()
        self._chk(lib().lco_get_colloids(self._h, n, arr), "lco_get_colloids")
        return [arr[k] for k in range(n)]

    def forces(self):
        n = self.num_colloids()
        out = np.zeros((max(1, n), 12))
        self._chk(lib().lco_get_forces(self._h, n, _dp(out)), "lco_get_forces")
        return out[:n]

    def solid_id(self):
        """0 at fluid nodes, k + 1 inside colloid k."""
        a = np.zeros(self.shape, dtype=np.uint8)
        self._chk(lib().lco_get_solid(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))),
                  "lco_get_solid")
        return a

    def _set(self, name, arr, ncomp):
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(ncomp, *self.shape)
        self._chk(getattr(lib(), name)(self._h, _dp(a)), name)

    def _get(self, name, ncomp):
        a = np.zeros((ncomp,) + self.shape)
        self._chk(getattr(lib(), name)(self._h, _dp(a)), name)
        return a

    def set_Q(self, Q):
        self._set("lco_set_Q", Q, 5)

    def set_f(self, f):
        self._set("lco_set_f", f, 19)

    def set_u(self, u):
        self._set("lco_set_u", u, 3)

    def get_Q(self):
        return self._get("lco_get_Q", 5)

    def get_f(self):
        return self._get("lco_get_f", 19)

    def get_u(self):
        return self._get("lco_get_u", 3)

    def ghost(self):
        return self._get("lco_ghost", 5)

    def solid(self):
        a = np.zeros(self.shape, dtype=np.uint8)
        self._chk(lib().lco_get_solid(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))),
                  "lco_get_solid")
        return a.astype(bool)

    def step(self, n=1):
        rc = lib().lco_step(self._h, int(n))
        if rc == 5:
            raise RuntimeError("lco_step refused: two colloids closer than the gap")
        self._chk(rc, "lco_step")

    @property
    def nstep(self):
        return int(lib().lco_get_nstep(self._h))

    def force(self):
        out = np.zeros(12)
        self._chk(lib().lco_get_force(self._h, _dp(out)), "lco_get_force")
        return out

    def diag(self):
        out = np.zeros(6)
        self._chk(lib().lco_get_diag(self._h, _dp(out)), "lco_get_diag")
        return {"free_energy": out[0], "mass": out[1], "momentum": out[2:5].copy(),
                "umax": out[5]}

    def fields(self):
        H = np.zeros((5,) + self.shape)
        P = np.zeros((9,) + self.shape)
        F = np.zeros((3,) + self.shape)
        self._chk(lib().lco_fields(self._h, _dp(H), _dp(P), _dp(F)), "lco_fields")
        return H, P, F
