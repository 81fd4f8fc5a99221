"""Python binding of liblbm.so (ctypes).  Argument marshalling only: every
step of the solver runs in the library's HIP kernels.  PyTorch supplies the
device memory (lbm_create_in) and the HIP stream.

The library must have been built (python -m paper_0904_4504_amd.build); a
missing library raises -- there is no fallback.
"""
import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbm.so")

ABI_VERSION = 2
OK, EINVAL, ENOMEM, EHIP, ERANGE, EUNSTABLE, EABI, ESCRATCH = 0, -1, -2, -3, -4, -5, -6, -7
# size of the library's static scratch array (lbm_create_static), per device
STATIC_SCRATCH_BYTES = 64 << 20
D2Q9, D2Q37 = 9, 37
STORE_F64, STORE_F32_DEV = 0, 1
COLL_REGULARIZED, COLL_BGK = 0, 1
WALL_BB, WALL_DS, WALL_MAXWELL = 0, 1, 2
GEOM_PLATE, GEOM_BOX, GEOM_PERIODIC = 0, 1, 2
REPR_AUTO, REPR_POPULATIONS, REPR_COEFFICIENTS, REPR_COEFFICIENTS_NOLOAD = 0, 1, 2, 3
FAR_WALL, FAR_EQ = 0, 1

# every symbol include/lbm.h declares
EXPORTS = (
    "lbm_params_init", "lbm_lattice", "lbm_required_bytes", "lbm_create", "lbm_create_in",
    "lbm_step", "lbm_synchronize", "lbm_steps_done", "lbm_force_history", "lbm_lockin",
    "lbm_impedance", "lbm_get_populations", "lbm_set_populations", "lbm_destroy",
    "lbm_strerror", "lbm_seek", "lbm_get_deviations", "lbm_set_deviations", "lbm_batch_create", "lbm_batch_add", "lbm_batch_remove",
    "lbm_batch_size", "lbm_batch_step", "lbm_batch_synchronize", "lbm_batch_set_graphs",
    "lbm_batch_timing", "lbm_batch_kernel_time", "lbm_batch_destroy", "lbm_state_size",
    "lbm_get_state", "lbm_set_state", "lbm_representation", "lbm_create_static",
)


class LbmError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


class Params(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("lattice", C.c_uint32), ("storage", C.c_uint32),
        ("collision", C.c_uint32), ("wall", C.c_uint32), ("geometry", C.c_uint32),
        ("far", C.c_uint32), ("tile", C.c_uint32), ("representation", C.c_uint32),
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("box_x0", C.c_int32), ("box_y0", C.c_int32), ("box_lx", C.c_int32),
        ("box_ly", C.c_int32), ("tau", C.c_double), ("omega", C.c_double),
        ("u0", C.c_double), ("rho0", C.c_double), ("max_steps", C.c_int64),
        ("lockin_first", C.c_int64), ("lockin_count", C.c_int64),
        ("history_capacity", C.c_int64), ("accommodation", C.c_double),
    ]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_0904_4504_amd.build`")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER(Params)
        vp = C.c_void_p
        dp = C.POINTER(C.c_double)
        L.lbm_params_init.argtypes = [P]
        L.lbm_lattice.argtypes = [C.c_int, vp, vp, vp, dp]
        L.lbm_required_bytes.argtypes = [P, C.POINTER(C.c_uint64)]
        L.lbm_create.argtypes = [P, vp, C.POINTER(vp)]
        L.lbm_create_in.argtypes = [P, vp, vp, C.c_uint64, C.POINTER(vp)]
        L.lbm_create_static.argtypes = [P, vp, C.POINTER(vp)]
        L.lbm_step.argtypes = [vp, C.c_int64]
        L.lbm_synchronize.argtypes = [vp]
        L.lbm_steps_done.argtypes = [vp, C.POINTER(C.c_int64)]
        L.lbm_force_history.argtypes = [vp, C.c_int64, C.c_int64, vp, vp]
        L.lbm_lockin.argtypes = [vp, vp, C.POINTER(C.c_int64)]
        L.lbm_impedance.argtypes = [vp, vp]
        L.lbm_get_populations.argtypes = [vp, vp, C.c_uint64]
        L.lbm_set_populations.argtypes = [vp, vp, C.c_uint64]
        L.lbm_seek.argtypes = [vp, C.c_int64, vp]
        L.lbm_state_size.argtypes = [vp, C.POINTER(C.c_uint64)]
        L.lbm_get_state.argtypes = [vp, vp, C.c_uint64]
        L.lbm_set_state.argtypes = [vp, vp, C.c_uint64]
        L.lbm_representation.argtypes = [vp, C.POINTER(C.c_int)]
        L.lbm_get_deviations.argtypes = [vp, vp, C.c_uint64]
        L.lbm_set_deviations.argtypes = [vp, vp, C.c_uint64]
        L.lbm_destroy.argtypes = [vp]
        L.lbm_batch_create.argtypes = [vp, C.POINTER(vp)]
        L.lbm_batch_add.argtypes = [vp, vp]
        L.lbm_batch_remove.argtypes = [vp, vp]
        L.lbm_batch_size.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.lbm_batch_step.argtypes = [vp, C.c_int64]
        L.lbm_batch_synchronize.argtypes = [vp]
        L.lbm_batch_set_graphs.argtypes = [vp, C.c_int]
        L.lbm_batch_timing.argtypes = [vp, C.c_int]
        L.lbm_batch_kernel_time.argtypes = [vp, dp, C.POINTER(C.c_int64)]
        L.lbm_batch_destroy.argtypes = [vp]
        L.lbm_strerror.argtypes = [C.c_int]
        L.lbm_strerror.restype = C.c_char_p
        _lib = L
    return _lib


def strerror(code):
    return lib().lbm_strerror(code).decode()


def _check(rc, what):
    if rc != OK:
        raise LbmError(rc, what)


def lattice(Q):
    """(v[Q,2] int32, w[Q] float64, theta) in the library's canonical order."""
    vx = np.zeros(Q, np.int32)
    vy = np.zeros(Q, np.int32)
    w = np.zeros(Q)
    th = C.c_double()
    _check(lib().lbm_lattice(Q, vx.ctypes.data, vy.ctypes.data, w.ctypes.data, C.byref(th)),
           "lbm_lattice")
    return np.stack([vx, vy], 1), w, th.value


def default_params():
    p = Params()
    _check(lib().lbm_params_init(C.byref(p)), "lbm_params_init")
    return p


def keeps_coefficients(s):
    """True if the automatic representation keeps this solve as H2
    coefficients: regularized collision, nx >= 64 and one coefficient plane
    (ny x nx rounded up to 64) below 2 GiB -- the library's rule."""
    es = 8 if s.storage == "f64" else 4
    return (s.collision == "regularized" and s.nx >= 64
            and s.ny * ((s.nx + 63) // 64 * 64) * es < 2 ** 31)


def params_from_solve(s, history_capacity=0, tile=0, representation=REPR_AUTO, loads=True):
    """lbm_params for an lbm_inputs.Solve.  loads=False: a solve that will not
    load populations and that the automatic representation keeps as
    coefficients is created without the population buffer
    (REPR_COEFFICIENTS_NOLOAD)."""
    p = default_params()
    p.tile = tile
    if not loads and representation == REPR_AUTO and keeps_coefficients(s):
        representation = REPR_COEFFICIENTS_NOLOAD
    p.representation = representation
    p.lattice = s.Q
    p.storage = STORE_F64 if s.storage == "f64" else STORE_F32_DEV
    p.collision = COLL_REGULARIZED if s.collision == "regularized" else COLL_BGK
    p.geometry = {"plate": GEOM_PLATE, "box": GEOM_BOX, "periodic": GEOM_PERIODIC}[s.geometry]
    p.far = FAR_WALL if s.far == "wall" else FAR_EQ
    p.wall = {"bb": WALL_BB, "ds": WALL_DS, "maxwell": WALL_MAXWELL}[getattr(s, "wall", "bb")]
    p.accommodation = getattr(s, "accommodation", 1.0)
    p.nx, p.ny = s.nx, s.ny
    p.box_x0, p.box_y0, p.box_lx, p.box_ly = s.box
    p.tau, p.omega, p.u0, p.rho0 = s.tau, s.omega, s.u0, s.rho0
    p.max_steps = s.nsteps
    p.lockin_first, p.lockin_count = s.window_first, s.window_count
    p.history_capacity = history_capacity
    return p


def required_bytes(p):
    n = C.c_uint64()
    _check(lib().lbm_required_bytes(C.byref(p), C.byref(n)), "lbm_required_bytes")
    return n.value


class Solver:
    """One solve on the current GPU.

    memory="torch": device memory is a torch uint8 tensor handed to
    lbm_create_in; memory="library": lbm_create allocates it;
    memory="static": the library's static scratch array (lbm_create_static,
    no device allocation; one such solver per device at a time).  The stream
    is torch's current stream unless one is given (a torch.cuda.Stream)."""

    def __init__(self, params, stream=None, memory="torch"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the solver runs only on the HIP device")
        self.p = params
        self.Q = params.lattice
        self._torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._h = C.c_void_p()
        self._mem = None
        sp = C.c_void_p(self.stream.cuda_stream)
        if memory == "torch":
            nbytes = required_bytes(params)
            # allocated on the solver's stream: the caching allocator orders
            # reuse of a freed block only on the stream it was allocated on,
            # and the library initialises and steps this memory on self.stream
            with torch.cuda.stream(self.stream):
                self._mem = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            ptr = self._mem.data_ptr()
            ptr += (-ptr) % 256
            _check(lib().lbm_create_in(C.byref(params), sp, C.c_void_p(ptr), nbytes,
                                       C.byref(self._h)), "lbm_create_in")
        elif memory == "static":
            _check(lib().lbm_create_static(C.byref(params), sp, C.byref(self._h)),
                   "lbm_create_static")
        else:
            _check(lib().lbm_create(C.byref(params), sp, C.byref(self._h)), "lbm_create")

    # ---------------------------------------------------------------- control
    def step(self, n):
        _check(lib().lbm_step(self._h, n), "lbm_step")

    def synchronize(self):
        _check(lib().lbm_synchronize(self._h), "lbm_synchronize")

    @property
    def steps_done(self):
        n = C.c_int64()
        _check(lib().lbm_steps_done(self._h, C.byref(n)), "lbm_steps_done")
        return n.value

    # ---------------------------------------------------------------- read-out
    def force_history(self, first=0, count=None):
        if count is None:
            count = self.steps_done - first
        fx = np.zeros(count)
        fy = np.zeros(count)
        _check(lib().lbm_force_history(self._h, first, count, fx.ctypes.data, fy.ctypes.data),
               "lbm_force_history")
        return fx, fy

    def lockin(self):
        s = np.zeros(6)
        n = C.c_int64()
        _check(lib().lbm_lockin(self._h, s.ctypes.data, C.byref(n)), "lbm_lockin")
        return s, n.value

    def impedance(self):
        out = np.zeros(5)
        _check(lib().lbm_impedance(self._h, out.ctypes.data), "lbm_impedance")
        a, b, c, R, X = (float(v) for v in out)
        return {"a": a, "b": b, "c": c, "R": R, "X": X, "Z": complex(R, X)}

    def get_populations(self):
        f = np.zeros((self.Q, self.p.ny, self.p.nx))
        _check(lib().lbm_get_populations(self._h, f.ctypes.data, f.size), "lbm_get_populations")
        return f

    def set_populations(self, f):
        f = np.ascontiguousarray(f, np.float64)
        if f.shape != (self.Q, self.p.ny, self.p.nx):
            raise ValueError(f"populations must have shape {(self.Q, self.p.ny, self.p.nx)}")
        _check(lib().lbm_set_populations(self._h, f.ctypes.data, f.size), "lbm_set_populations")

    def get_deviations(self):
        f = np.zeros((self.Q, self.p.ny, self.p.nx))
        _check(lib().lbm_get_deviations(self._h, f.ctypes.data, f.size), "lbm_get_deviations")
        return f

    def set_deviations(self, d):
        d = np.ascontiguousarray(d, np.float64)
        if d.shape != (self.Q, self.p.ny, self.p.nx):
            raise ValueError(f"deviations must have shape {(self.Q, self.p.ny, self.p.nx)}")
        _check(lib().lbm_set_deviations(self._h, d.ctypes.data, d.size), "lbm_set_deviations")

    @property
    def representation(self):
        r = C.c_int()
        _check(lib().lbm_representation(self._h, C.byref(r)), "lbm_representation")
        return r.value

    def get_state(self):
        n = C.c_uint64()
        _check(lib().lbm_state_size(self._h, C.byref(n)), "lbm_state_size")
        buf = np.zeros(n.value, np.uint8)
        _check(lib().lbm_get_state(self._h, buf.ctypes.data, n.value), "lbm_get_state")
        return buf

    def set_state(self, blob):
        blob = np.ascontiguousarray(blob, np.uint8)
        _check(lib().lbm_set_state(self._h, blob.ctypes.data, blob.size), "lbm_set_state")

    def seek(self, step, lockin_sums=None):
        sums = None if lockin_sums is None else np.ascontiguousarray(lockin_sums, np.float64)
        _check(lib().lbm_seek(self._h, step, None if sums is None else sums.ctypes.data),
               "lbm_seek")

    def close(self):
        if self._h:
            rc = lib().lbm_destroy(self._h)
            self._h = C.c_void_p()
            self._mem = None
            _check(rc, "lbm_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several solvers advanced by one fused launch per kind of member and step (lbm_batch_*).
    Members must share the batch's stream, lattice, storage and collision."""

    def __init__(self, stream=None):
        import torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._h = C.c_void_p()
        self.members = []
        _check(lib().lbm_batch_create(C.c_void_p(self.stream.cuda_stream), C.byref(self._h)),
               "lbm_batch_create")

    def add(self, solver):
        _check(lib().lbm_batch_add(self._h, solver._h), "lbm_batch_add")
        self.members.append(solver)

    def remove(self, solver):
        _check(lib().lbm_batch_remove(self._h, solver._h), "lbm_batch_remove")
        self.members.remove(solver)

    def size(self):
        m, a = C.c_int(), C.c_int()
        _check(lib().lbm_batch_size(self._h, C.byref(m), C.byref(a)), "lbm_batch_size")
        return m.value, a.value

    def step(self, n):
        _check(lib().lbm_batch_step(self._h, n), "lbm_batch_step")

    def synchronize(self):
        _check(lib().lbm_batch_synchronize(self._h), "lbm_batch_synchronize")

    def set_graphs(self, steps_per_graph):
        _check(lib().lbm_batch_set_graphs(self._h, steps_per_graph), "lbm_batch_set_graphs")

    def timing(self, enable):
        _check(lib().lbm_batch_timing(self._h, int(bool(enable))), "lbm_batch_timing")

    def kernel_time(self):
        ms = C.c_double()
        n = C.c_int64()
        _check(lib().lbm_batch_kernel_time(self._h, C.byref(ms), C.byref(n)),
               "lbm_batch_kernel_time")
        return ms.value, n.value

    def close(self):
        if self._h:
            rc = lib().lbm_batch_destroy(self._h)
            self._h = C.c_void_p()
            self.members = []
            _check(rc, "lbm_batch_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
