"""ctypes binding of ``liblc.so`` (C ABI in include/lc.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides the device memory of the fields (bound with
``lc_bind_buffers``) and the HIP stream.  There is no CPU fallback: if the
library is missing or no GPU is present, construction raises.
"""
import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# LC_LIBRARY: another build of the same library (e.g. the host-sanitizer
# build made by build.py --host-sanitize)
LIB_PATH = os.environ.get("LC_LIBRARY") or os.path.join(HERE, "liblc.so")

FP32, FP64 = 0, 1
ANCHOR_NONE, ANCHOR_NORMAL, ANCHOR_PLANAR = 0, 1, 2
FIXED, PRESCRIBED, FREE = 0, 1, 2
ANCHORING = {"none": ANCHOR_NONE, "normal": ANCHOR_NORMAL, "planar": ANCHOR_PLANAR}

STATUS = {0: "LC_OK", 1: "LC_EINVAL", 2: "LC_ENOMEM", 3: "LC_EDEVICE", 4: "LC_ENUMERIC", 5: "LC_ESTATE"}

EXPORTS = [
    "lc_create", "lc_create_batch", "lc_destroy", "lc_last_error", "lc_buffer_bytes", "lc_bind_buffers",
    "lc_set_colloid", "lc_get_colloid", "lc_set_colloids", "lc_get_colloids", "lc_num_colloids",
    "lc_get_colloid_force", "lc_get_colloid_force_history", "lc_get_solid", "lc_set_Q", "lc_set_f", "lc_set_u", "lc_get_Q", "lc_get_f",
    "lc_get_u", "lc_state_bytes", "lc_get_state", "lc_set_state", "lc_step", "lc_sync", "lc_get_nstep", "lc_prepare",
    "lc_get_force", "lc_get_force_history",
    "lc_history_capacity", "lc_get_diag", "lc_get_diag_noalloc", "lc_defects", "lc_num_tiles", "lc_tile_shape", "lc_set_tile",
    "lc_get_tile", "lc_use_graph", "lc_launch_info", "lc_time_kernel",
]


class LCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("precision", ctypes.c_int), ("hydro", ctypes.c_int), ("pad_", ctypes.c_int),
                ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
                ("A0", ctypes.c_double), ("gamma", ctypes.c_double), ("K", ctypes.c_double),
                ("q0", ctypes.c_double), ("xi", ctypes.c_double), ("Gamma", ctypes.c_double),
                ("body_force", ctypes.c_double * 3),
                ("advection", ctypes.c_int), ("stencil", ctypes.c_int)]


class Colloid(ctypes.Structure):
    _fields_ = [("present", ctypes.c_int), ("motion", ctypes.c_int), ("anchoring", ctypes.c_int),
                ("pad_", ctypes.c_int), ("pos", ctypes.c_double * 3), ("a0", ctypes.c_double),
                ("vel", ctypes.c_double * 3), ("omega", ctypes.c_double * 3),
                ("S0", ctypes.c_double), ("W", ctypes.c_double),
                ("fext", ctypes.c_double * 3), ("rho_c", ctypes.c_double)]


class Diag(ctypes.Structure):
    _fields_ = [("free_energy", ctypes.c_double), ("mass", ctypes.c_double),
                ("momentum", ctypes.c_double * 3), ("umax", ctypes.c_double)]


_lib = None


def load():
    """Load liblc.so (built by __graft_entry__.build()); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblc.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    # The library runs on the HIP runtime torch has loaded (same soname).  Let
    # torch initialise it before the library's code objects (and its static
    # device array) are registered with it: loaded first, the library's own
    # calls later failed with "no ROCm-capable device" while torch's worked.
    import torch
    torch.cuda.is_available()
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    L.lc_create.argtypes = [ctypes.POINTER(Params), vp, ctypes.POINTER(vp)]
    L.lc_create_batch.argtypes = [ip, ctypes.POINTER(Params), vp, ctypes.POINTER(vp)]
    L.lc_destroy.argtypes = [vp]
    L.lc_destroy.restype = None
    L.lc_last_error.argtypes = [vp]
    L.lc_last_error.restype = ctypes.c_char_p
    L.lc_buffer_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.lc_bind_buffers.argtypes = [vp] + [vp] * 6
    L.lc_set_colloid.argtypes = [vp, ip, ctypes.POINTER(Colloid)]
    L.lc_get_colloid.argtypes = [vp, ip, ctypes.POINTER(Colloid)]
    L.lc_set_colloids.argtypes = [vp, ip, ip, ctypes.POINTER(Colloid)]
    L.lc_get_colloids.argtypes = [vp, ip, ip, ctypes.POINTER(Colloid)]
    L.lc_num_colloids.argtypes = [vp, ip]
    L.lc_get_colloid_force.argtypes = [vp, ip, ip, dp]
    L.lc_get_colloid_force_history.argtypes = [vp, ip, ip, ip, dp]
    L.lc_get_solid.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_ubyte)]
    for n in ("lc_set_Q", "lc_set_f", "lc_set_u", "lc_get_Q", "lc_get_f", "lc_get_u", "lc_get_force"):
        getattr(L, n).argtypes = [vp, ip, dp]
    L.lc_state_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.lc_get_state.argtypes = [vp, vp, ctypes.c_size_t]
    L.lc_set_state.argtypes = [vp, vp, ctypes.c_size_t]
    L.lc_step.argtypes = [vp, ip]
    L.lc_sync.argtypes = [vp]
    L.lc_prepare.argtypes = [vp]
    L.lc_get_nstep.argtypes = [vp]
    L.lc_get_nstep.restype = ctypes.c_long
    L.lc_get_force_history.argtypes = [vp, ip, ip, dp]
    L.lc_history_capacity.argtypes = [vp]
    L.lc_get_diag.argtypes = [vp, ip, ctypes.POINTER(Diag)]
    L.lc_get_diag_noalloc.argtypes = [vp, ip, ctypes.POINTER(Diag)]
    L.lc_defects.argtypes = [vp, ip, ctypes.c_double, ctypes.POINTER(ctypes.c_ubyte),
                             ctypes.POINTER(ctypes.c_long)]
    L.lc_num_tiles.argtypes = [vp]
    L.lc_tile_shape.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_int)]
    L.lc_set_tile.argtypes = [vp, ip]
    L.lc_get_tile.argtypes = [vp]
    L.lc_use_graph.argtypes = [vp, ip]
    L.lc_launch_info.argtypes = [vp, ctypes.POINTER(ctypes.c_long)]
    L.lc_time_kernel.argtypes = [vp, ip, dp]
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(nx, ny=None, nz=None, precision=FP32, hydro=1, tau=1.0, rho0=1.0, A0=0.01, gamma=3.0,
                K=0.01, q0=0.0, xi=0.7, Gamma=0.5, body_force=(0.0, 0.0, 0.0), advection=1, stencil=7):
    p = Params()
    p.advection, p.stencil = int(advection), int(stencil)
    p.nx = nx
    p.ny = nx if ny is None else ny
    p.nz = nx if nz is None else nz
    p.precision = {"fp32": FP32, "fp64": FP64}.get(precision, precision)
    p.hydro = int(hydro)
    p.tau, p.rho0, p.A0, p.gamma, p.K, p.q0, p.xi, p.Gamma = tau, rho0, A0, gamma, K, q0, xi, Gamma
    for a in range(3):
        p.body_force[a] = body_force[a]
    return p


def make_colloid(pos, a0, anchoring=ANCHOR_NORMAL, W=math.inf, S0=0.5, vel=(0, 0, 0), omega=(0, 0, 0),
                 motion=FIXED, present=1, fext=(0, 0, 0), rho_c=0.0):
    c = Colloid()
    c.present, c.motion = int(present), int(motion)
    c.anchoring = ANCHORING.get(anchoring, anchoring)
    for a in range(3):
        c.pos[a], c.vel[a], c.omega[a], c.fext[a] = pos[a], vel[a], omega[a], fext[a]
    c.a0, c.S0, c.W, c.rho_c = a0, S0, W, rho_c
    return c


class Context:
    """A batch of periodic boxes stepped together on one GPU.

    ``boxes`` is a list of parameter dicts (keys of make_params).  Device
    fields are torch tensors bound to the library; work runs on a dedicated
    torch stream (``self.stream``).
    """

    def __init__(self, boxes, bind_torch=True, device="cuda:0"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP library has no CPU path")
        L = load()
        self._L = L
        self.torch = torch
        self.device = torch.device(device)
        self.box_params = [make_params(**b) for b in boxes]
        self.shapes = [(p.nz, p.ny, p.nx) for p in self.box_params]
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.Stream(self.device)
        arr = (Params * len(boxes))(*self.box_params)
        h = ctypes.c_void_p()
        rc = L.lc_create_batch(len(boxes), arr, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise LCError(rc, L.lc_last_error(None).decode())
        self._h = h
        self._bufs = None
        if bind_torch:
            sz = (ctypes.c_size_t * 3)()
            self._chk(L.lc_buffer_bytes(h, sz))
            with torch.cuda.stream(self.stream):
                bufs = [torch.empty(int(sz[k // 2]), dtype=torch.uint8, device=self.device) for k in range(6)]
            self.stream.synchronize()
            self._chk(L.lc_bind_buffers(h, *[ctypes.c_void_p(b.data_ptr()) for b in bufs]))
            self._bufs = bufs

    def _chk(self, rc):
        if rc != 0:
            raise LCError(rc, self._L.lc_last_error(self._h).decode())

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._L.lc_destroy(h)
            self._h = None
        self._bufs = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- setup -----------------------------------------------------------
    def set_colloid(self, box, pos, a0, **kw):
        c = make_colloid(pos, a0, **kw)
        self._chk(self._L.lc_set_colloid(self._h, box, ctypes.byref(c)))

    def get_colloid(self, box=0):
        c = Colloid()
        self._chk(self._L.lc_get_colloid(self._h, box, ctypes.byref(c)))
        return c

    def set_colloids(self, box, specs):
        """specs: list of dicts with pos, a0 and make_colloid's keywords."""
        arr = (Colloid * max(1, len(specs)))()
        for k, sp in enumerate(specs):
            sp = dict(sp)
            arr[k] = make_colloid(sp.pop("pos"), sp.pop("a0"), **sp)
        self._chk(self._L.lc_set_colloids(self._h, box, len(specs), arr))

    def num_colloids(self, box=0):
        return int(self._L.lc_num_colloids(self._h, box))

    def get_colloids(self, box=0):
        n = self.num_colloids(box)
        arr = (Colloid * max(1, n))()
        self._chk(self._L.lc_get_colloids(self._h, box, n, arr))
        return [arr[k] for k in range(n)]

    def colloid_force(self, box, k):
        out = np.zeros(12)
        self._chk(self._L.lc_get_colloid_force(self._h, box, k, _dp(out)))
        return out

    def colloid_force_history(self, box, k, n):
        out = np.zeros((n, 12))
        self._chk(self._L.lc_get_colloid_force_history(self._h, box, k, int(n), _dp(out)))
        return out

    def solid_id(self, box=0):
        """The library's solid map: 1 + colloid index, 0 at fluid sites."""
        out = np.zeros(self.shapes[box], dtype=np.uint8)
        self._chk(self._L.lc_get_solid(self._h, box, out.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))))
        return out

    def _put(self, fn, box, arr, ncomp):
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape((ncomp,) + self.shapes[box])
        self._chk(getattr(self._L, fn)(self._h, box, _dp(a)))

    def _get(self, fn, box, ncomp):
        a = np.zeros((ncomp,) + self.shapes[box])
        self._chk(getattr(self._L, fn)(self._h, box, _dp(a)))
        return a

    def set_Q(self, box, Q):
        self._put("lc_set_Q", box, Q, 5)

    def set_f(self, box, f):
        self._put("lc_set_f", box, f, 19)

    def set_u(self, box, u):
        self._put("lc_set_u", box, u, 3)

    def get_Q(self, box=0):
        return self._get("lc_get_Q", box, 5)

    def get_f(self, box=0):
        return self._get("lc_get_f", box, 19)

    def get_u(self, box=0):
        return self._get("lc_get_u", box, 3)

    # ---- checkpoint ------------------------------------------------------
    def get_state(self):
        """The whole evolving state as a uint8 array (lc_get_state)."""
        n = ctypes.c_size_t()
        self._chk(self._L.lc_state_bytes(self._h, ctypes.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        self._chk(self._L.lc_get_state(self._h, ctypes.c_void_p(buf.ctypes.data), buf.nbytes))
        return buf

    def set_state(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._chk(self._L.lc_set_state(self._h, ctypes.c_void_p(buf.ctypes.data), buf.nbytes))

    def save(self, path):
        self.get_state().tofile(path)

    def load(self, path):
        self.set_state(np.fromfile(path, dtype=np.uint8))

    # ---- stepping --------------------------------------------------------
    def step(self, n=1):
        self._chk(self._L.lc_step(self._h, int(n)))

    def sync(self):
        self._chk(self._L.lc_sync(self._h))

    def prepare(self):
        """Capture the step graph ahead of the next step (lc_prepare)."""
        self._chk(self._L.lc_prepare(self._h))

    @property
    def nstep(self):
        return int(self._L.lc_get_nstep(self._h))

    def force(self, box=0):
        out = np.zeros(12)
        self._chk(self._L.lc_get_force(self._h, box, _dp(out)))
        return out

    def force_history(self, box, n):
        out = np.zeros((n, 12))
        self._chk(self._L.lc_get_force_history(self._h, box, int(n), _dp(out)))
        return out

    def diag(self, box=0):
        d = Diag()
        self._chk(self._L.lc_get_diag(self._h, box, ctypes.byref(d)))
        return {"free_energy": d.free_energy, "mass": d.mass, "momentum": np.array(list(d.momentum)),
                "umax": d.umax}

    def defects(self, box=0, threshold=0.435):
        mask = np.zeros(self.shapes[box], dtype=np.uint8)
        cnt = ctypes.c_long()
        self._chk(self._L.lc_defects(self._h, box, threshold,
                                     mask.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)), ctypes.byref(cnt)))
        return mask.astype(bool), int(cnt.value)

    # ---- execution controls ----------------------------------------------
    def num_tiles(self):
        return int(self._L.lc_num_tiles(self._h))

    def tile_shape(self, tid):
        out = (ctypes.c_int * 3)()
        self._chk(self._L.lc_tile_shape(self._h, tid, out))
        return tuple(out)

    def set_tile(self, tid):
        self._chk(self._L.lc_set_tile(self._h, int(tid)))

    def get_tile(self):
        return int(self._L.lc_get_tile(self._h))

    def use_graph(self, enable):
        self._chk(self._L.lc_use_graph(self._h, int(bool(enable))))

    def launch_info(self):
        out = (ctypes.c_long * 2)()
        self._chk(self._L.lc_launch_info(self._h, out))
        return int(out[0]), int(out[1])

    def time_kernel(self, n):
        out = np.zeros(3)
        self._chk(self._L.lc_time_kernel(self._h, int(n), _dp(out)))
        return {"kernel_ms": out[0], "step_ms": out[1], "total_ms": out[2]}
