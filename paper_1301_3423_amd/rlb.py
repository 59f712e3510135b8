"""Thin ctypes binding of the C ABI in include/rlb.h (argument marshalling
only: every step of the update runs in the HIP library).  PyTorch provides
the device memory and the stream.

    from paper_1301_3423_amd import rlb
    s = rlb.Solver(64, 64, 64, precision="fp64", eta_s=0.2)   # order=2: Appendix A model
    s.init_fields(n, eps, vx, vy, vz)        # numpy (host) or torch (device)
    s.step(100)
    out = s.read_fields()                    # dict of numpy arrays

The library is loaded on first use; if librlb.so is missing this raises
instead of falling back to anything else.
"""
import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librlb.so")

OK, EINVAL, ENOMEM, ENONPHYS, EHIP, ESTATE, EIO = 0, -1, -2, -3, -4, -5, -6
FP64, MIXED = 0, 1
TAU_FIXED, TAU_ETA_S = 0, 1
ORDER3, ORDER2 = 3, 2
PATTERN_AB, PATTERN_AA = 0, 1
FLAG_NONFINITE, FLAG_NONPHYSICAL, FLAG_LANDAU, FLAG_STALL = 1, 2, 4, 8
MAX_Q = 128

# every symbol include/rlb.h declares
EXPORTS = ("rlb_lattice_info", "rlb_state_bytes", "rlb_create", "rlb_init_fields", "rlb_step",
           "rlb_read_fields", "rlb_conserved", "rlb_status", "rlb_save", "rlb_load", "rlb_destroy",
           "rlb_batch_bytes", "rlb_batch_create", "rlb_batch_init", "rlb_batch_step", "rlb_batch_read",
           "rlb_batch_status", "rlb_batch_destroy", "rlb_request_bytes", "rlb_server_create",
           "rlb_server_submit", "rlb_server_poll", "rlb_server_pending", "rlb_server_destroy",
           "rlb_walls_bytes", "rlb_set_walls", "rlb_strerror", "rlb_last_error", "rlb_conserved_noalloc")
REQ_TUBE, REQ_BOX = 0, 1


class RLBError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_name(code), code, msg))
        self.code = code


def _name(code):
    return {OK: "RLB_OK", EINVAL: "RLB_EINVAL", ENOMEM: "RLB_ENOMEM", ENONPHYS: "RLB_ENONPHYS",
            EHIP: "RLB_EHIP", ESTATE: "RLB_ESTATE", EIO: "RLB_EIO"}.get(code, "RLB_?")


class Lattice(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int32), ("r2", ctypes.c_int32), ("nshell", ctypes.c_int32),
                ("theta", (ctypes.c_int8 * 3) * MAX_Q), ("p0", ctypes.c_double * MAX_Q),
                ("w", ctypes.c_double * MAX_Q), ("inv", ctypes.c_int32 * MAX_Q),
                ("shell", ctypes.c_int32 * MAX_Q), ("sha256", ctypes.c_char * 65)]


class Config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("tau_mode", ctypes.c_int32),
                ("tau", ctypes.c_double), ("eta_s", ctypes.c_double), ("order", ctypes.c_int32),
                ("pattern", ctypes.c_int32)]


class Tube(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("tau_mode", ctypes.c_int32), ("tau", ctypes.c_double),
                ("eta_s", ctypes.c_double)]


_DP = ctypes.POINTER(ctypes.c_double)


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("tau_mode", ctypes.c_int32), ("order", ctypes.c_int32),
                ("tau", ctypes.c_double), ("eta_s", ctypes.c_double), ("steps", ctypes.c_int64),
                ("n", _DP), ("eps", _DP), ("vx", _DP), ("vy", _DP), ("vz", _DP),
                ("out_n", _DP), ("out_eps", _DP), ("out_U4", _DP), ("out_P", _DP)]


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("rc", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


_lib = None


def lib():
    """The loaded librlb.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librlb.so is not built: run python -m paper_1301_3423_amd.build")
        # torch ships its own HIP runtime under the same soname as the
        # system's.  Imported first, it provides the one runtime the library
        # then binds to; loading the library first would map the system's
        # runtime beside torch's, and the second runtime to start finds no
        # device.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, i32, i64 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_int64
        L.rlb_lattice_info.argtypes = [i32, ctypes.POINTER(Lattice)]
        L.rlb_state_bytes.argtypes = [i32, i32, i32, i32, i32, i32]
        L.rlb_state_bytes.restype = ctypes.c_size_t
        L.rlb_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Config), vp, ctypes.c_size_t, vp]
        L.rlb_init_fields.argtypes = [vp, vp, vp, vp, vp, vp, i32]
        L.rlb_step.argtypes = [vp, i64]
        L.rlb_read_fields.argtypes = [vp, vp, vp, vp, vp, i32]
        L.rlb_conserved.argtypes = [vp, dp]
        L.rlb_conserved_noalloc.argtypes = [vp, dp]
        L.rlb_status.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(i64)]
        L.rlb_save.argtypes = [vp, ctypes.c_char_p]
        L.rlb_load.argtypes = [vp, ctypes.c_char_p]
        L.rlb_destroy.argtypes = [vp]
        L.rlb_destroy.restype = None
        L.rlb_batch_bytes.argtypes = [ctypes.POINTER(Tube), i32, i32, i32]
        L.rlb_batch_bytes.restype = ctypes.c_size_t
        L.rlb_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Tube), i32, i32, i32, vp, ctypes.c_size_t,
                                       vp]
        L.rlb_batch_init.argtypes = [vp, i32, vp, vp, vp, vp, vp, i32]
        L.rlb_batch_step.argtypes = [vp, ctypes.POINTER(i64)]
        L.rlb_batch_read.argtypes = [vp, i32, vp, vp, vp, vp, i32]
        L.rlb_batch_status.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(i64)]
        L.rlb_batch_destroy.argtypes = [vp]
        L.rlb_batch_destroy.restype = None
        L.rlb_request_bytes.argtypes = [ctypes.POINTER(Request)]
        L.rlb_request_bytes.restype = ctypes.c_size_t
        L.rlb_server_create.argtypes = [ctypes.POINTER(vp), vp, ctypes.c_size_t, i32, i32]
        L.rlb_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(i64)]
        L.rlb_server_poll.argtypes = [vp, ctypes.POINTER(Completion), i32, ctypes.POINTER(i32), i32]
        L.rlb_server_pending.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.rlb_server_destroy.argtypes = [vp]
        L.rlb_server_destroy.restype = None
        L.rlb_walls_bytes.argtypes = [i32, i32, i32, i32, vp]
        L.rlb_walls_bytes.restype = ctypes.c_size_t
        L.rlb_set_walls.argtypes = [vp, vp, vp, ctypes.c_size_t]
        L.rlb_strerror.argtypes = [ctypes.c_int]
        L.rlb_strerror.restype = ctypes.c_char_p
        L.rlb_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def check(rc):
    if rc != OK:
        raise RLBError(rc, lib().rlb_last_error().decode())
    return rc


def lattice_info(order=ORDER3):
    lat = Lattice()
    check(lib().rlb_lattice_info(int(order), ctypes.byref(lat)))
    q = lat.q
    return dict(q=q, r2=lat.r2, nshell=lat.nshell,
                theta=np.array([[lat.theta[i][k] for k in range(3)] for i in range(q)], dtype=np.int64),
                p0=np.array(lat.p0[:q]), w=np.array(lat.w[:q]), inv=np.array(lat.inv[:q]),
                shell=np.array(lat.shell[:q]), sha256=lat.sha256.decode())


def state_bytes(nx, ny, nz, precision="fp64", order=ORDER3, pattern="ab"):
    return lib().rlb_state_bytes(nx, ny, nz, _prec(precision), int(order), _pattern(pattern))


def _pattern(p):
    if p in ("ab", PATTERN_AB):
        return PATTERN_AB
    if p in ("aa", PATTERN_AA):
        return PATTERN_AA
    raise ValueError("pattern must be 'ab' or 'aa'")


def _prec(p):
    if p in ("fp64", FP64):
        return FP64
    if p in ("mixed", MIXED):
        return MIXED
    raise ValueError("precision must be 'fp64' or 'mixed'")


def _stream_ptr(stream):
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(st.cuda_stream)


def _order_buffer(buf, stream):
    """torch's caching allocator orders a block's reuse after work on the
    stream it was allocated on.  When the library runs on another stream,
    wait for that stream's pending work (an earlier owner of the memory) and
    record the library's stream on the block, so that it is not handed out
    again while the library may still use it."""
    import torch
    cur = torch.cuda.current_stream(buf.device)
    if stream != cur:
        cur.synchronize()
        buf.record_stream(stream)


class Solver:
    """One periodic nx x ny x nz box on the current HIP device, third-order
    (order=3) or second-order (order=2) model, two population buffers
    (pattern="ab") or one updated in place (pattern="aa").

    Device memory is a torch uint8 tensor owned by this object; the solver
    runs on `stream` (default: torch's current stream at construction)."""

    def __init__(self, nx, ny, nz, precision="fp64", tau=None, eta_s=None, stream=None, device=None, order=ORDER3,
                 pattern="ab"):
        import torch
        if (tau is None) == (eta_s is None):
            raise ValueError("give exactly one of tau, eta_s")
        self.shape = (nz, ny, nx)
        self.cells = nx * ny * nz
        self.precision = precision
        self.order = int(order)
        self.pattern = _pattern(pattern)
        cfg = Config(nx, ny, nz, _prec(precision), TAU_FIXED if tau is not None else TAU_ETA_S,
                     float(tau) if tau is not None else 0.0, float(eta_s) if eta_s is not None else 0.0,
                     self.order, self.pattern)
        self.cfg = cfg
        nbytes = state_bytes(nx, ny, nz, precision, self.order, self.pattern)
        if nbytes == 0:
            raise RLBError(EINVAL, "invalid lattice size, precision, order or pattern")
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.buffer = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        _order_buffer(self.buffer, self.stream)
        h = ctypes.c_void_p()
        check(lib().rlb_create(ctypes.byref(h), ctypes.byref(cfg), ctypes.c_void_p(self.buffer.data_ptr()),
                               nbytes, _stream_ptr(self.stream)))
        self._h = h
        self._free = lib().rlb_destroy

    def __del__(self):
        # the destroy function is kept on the object: at interpreter exit the
        # module's globals may already be gone
        h, free = getattr(self, "_h", None), getattr(self, "_free", None)
        if h is not None and h.value and free is not None:
            free(h)
            self._h = None

    # -- fields -------------------------------------------------------------
    def init_fields(self, n, eps, vx, vy, vz):
        import torch
        arrs = (n, eps, vx, vy, vz)
        if all(isinstance(a, torch.Tensor) and a.is_cuda for a in arrs):
            ts = [a.contiguous().to(torch.float64) for a in arrs]
            for t in ts:
                if t.numel() != self.cells:
                    raise ValueError("field has %d values, expected %d" % (t.numel(), self.cells))
            check(lib().rlb_init_fields(self._h, *[ctypes.c_void_p(t.data_ptr()) for t in ts], 1))
            self._keep = ts          # alive until the stream has consumed them
            return
        hs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)).ravel() for a in arrs]
        for h in hs:
            if h.size != self.cells:
                raise ValueError("field has %d values, expected %d" % (h.size, self.cells))
        check(lib().rlb_init_fields(self._h, *[ctypes.c_void_p(h.ctypes.data) for h in hs], 0))

    def release_inputs(self):
        """Wait until the solver's stream has consumed device fields given to
        init_fields, then drop the references kept to them."""
        if getattr(self, "_keep", None) is not None:
            self.stream.synchronize()
            self._keep = None

    def step(self, nsteps=1):
        check(lib().rlb_step(self._h, int(nsteps)))

    def read_fields(self, on_device=False):
        """n, eps, P (cells,) and U (4, cells) of the current state."""
        C = self.cells
        if on_device:
            import torch
            out = dict(n=torch.empty(C, dtype=torch.float64, device=self.device),
                       eps=torch.empty(C, dtype=torch.float64, device=self.device),
                       U=torch.empty(4, C, dtype=torch.float64, device=self.device),
                       P=torch.empty(C, dtype=torch.float64, device=self.device))
            check(lib().rlb_read_fields(self._h, *[ctypes.c_void_p(out[k].data_ptr()) for k in ("n", "eps", "U", "P")], 1))
            return out
        out = dict(n=np.empty(C), eps=np.empty(C), U=np.empty((4, C)), P=np.empty(C))
        check(lib().rlb_read_fields(self._h, *[ctypes.c_void_p(out[k].ctypes.data) for k in ("n", "eps", "U", "P")], 0))
        return out

    def conserved(self):
        out = (ctypes.c_double * 5)()
        check(lib().rlb_conserved(self._h, out))
        return np.array(out[:])

    def conserved_noalloc(self):
        """conserved() through rlb_conserved_noalloc (partial sums in the
        library's fixed scratch array; no walls, at most 2^25 cells)."""
        out = (ctypes.c_double * 5)()
        check(lib().rlb_conserved_noalloc(self._h, out))
        return np.array(out[:])

    def status(self):
        fl = ctypes.c_uint32()
        t = ctypes.c_int64()
        check(lib().rlb_status(self._h, ctypes.byref(fl), ctypes.byref(t)))
        return fl.value, t.value

    def set_walls(self, solid):
        """Solid cells (array of nz*ny*nx, non-zero = solid; bounce-back
        walls), or None to remove them.  The device copy lives in a torch
        buffer owned by this object."""
        if solid is None:
            check(lib().rlb_set_walls(self._h, None, None, 0))
            self._walls = None
            return
        mask = np.ascontiguousarray(np.asarray(solid).ravel() != 0, dtype=np.uint8)
        if mask.size != self.cells:
            raise ValueError("mask has %d values, expected %d" % (mask.size, self.cells))
        nz, ny, nx = self.shape
        nbytes = lib().rlb_walls_bytes(self.order, nx, ny, nz, ctypes.c_void_p(mask.ctypes.data))
        if nbytes == 0:
            raise RLBError(EINVAL, "invalid mask (every cell solid?)")
        import torch
        buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        check(lib().rlb_set_walls(self._h, ctypes.c_void_p(mask.ctypes.data), ctypes.c_void_p(buf.data_ptr()),
                                  nbytes))
        self._walls = buf

    def save(self, path):
        check(lib().rlb_save(self._h, str(path).encode()))

    def load(self, path):
        check(lib().rlb_load(self._h, str(path).encode()))


def _tube_struct(t):
    """A tube given as dict(n=..., tau=...) or dict(n=..., eta_s=...)."""
    if ("tau" in t) == ("eta_s" in t):
        raise ValueError("a tube needs exactly one of tau, eta_s")
    if "tau" in t:
        return Tube(int(t["n"]), TAU_FIXED, float(t["tau"]), 0.0)
    return Tube(int(t["n"]), TAU_ETA_S, 0.0, float(t["eta_s"]))


def batch_bytes(tubes, precision="fp64", order=ORDER3):
    arr = (Tube * len(tubes))(*[_tube_struct(t) for t in tubes])
    return lib().rlb_batch_bytes(arr, len(tubes), _prec(precision), int(order))


class Batch:
    """Many independent 1 x 1 x n shock tubes of one precision and one model,
    advanced together by one persistent launch per step() call."""

    def __init__(self, tubes, precision="fp64", stream=None, device=None, order=ORDER3):
        import torch
        self.tubes = [dict(t) for t in tubes]
        self.precision = precision
        self.order = int(order)
        arr = (Tube * len(tubes))(*[_tube_struct(t) for t in tubes])
        nbytes = lib().rlb_batch_bytes(arr, len(tubes), _prec(precision), self.order)
        if nbytes == 0:
            raise RLBError(EINVAL, "invalid tube list")
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.buffer = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        _order_buffer(self.buffer, self.stream)
        h = ctypes.c_void_p()
        check(lib().rlb_batch_create(ctypes.byref(h), arr, len(tubes), _prec(precision), self.order,
                                     ctypes.c_void_p(self.buffer.data_ptr()), nbytes, _stream_ptr(self.stream)))
        self._h = h
        self._free = lib().rlb_batch_destroy

    def __len__(self):
        return len(self.tubes)

    def __del__(self):
        h, free = getattr(self, "_h", None), getattr(self, "_free", None)
        if h is not None and h.value and free is not None:
            free(h)
            self._h = None

    def init_tube(self, j, n, eps, vx, vy, vz):
        hs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)).ravel() for a in (n, eps, vx, vy, vz)]
        for h in hs:
            if h.size != self.tubes[j]["n"]:
                raise ValueError("tube %d has %d cells, got %d values" % (j, self.tubes[j]["n"], h.size))
        check(lib().rlb_batch_init(self._h, int(j), *[ctypes.c_void_p(h.ctypes.data) for h in hs], 0))

    def step(self, steps):
        """steps: one count for every tube, or a sequence with one per tube."""
        if np.isscalar(steps):
            steps = [int(steps)] * len(self.tubes)
        arr = (ctypes.c_int64 * len(self.tubes))(*[int(s) for s in steps])
        check(lib().rlb_batch_step(self._h, arr))

    def read_tube(self, j):
        C = self.tubes[j]["n"]
        out = dict(n=np.empty(C), eps=np.empty(C), U=np.empty((4, C)), P=np.empty(C))
        check(lib().rlb_batch_read(self._h, int(j), *[ctypes.c_void_p(out[k].ctypes.data)
                                                      for k in ("n", "eps", "U", "P")], 0))
        return out

    def status(self, j):
        fl = ctypes.c_uint32()
        t = ctypes.c_int64()
        check(lib().rlb_batch_status(self._h, int(j), ctypes.byref(fl), ctypes.byref(t)))
        return fl.value, t.value


def _dp(a):
    return a.ctypes.data_as(_DP) if a is not None else None


def make_request(kind, shape, precision, steps, fields, tau=None, eta_s=None, outputs=True, order=ORDER3):
    """A Request plus the numpy arrays it points to (keep them alive)."""
    nx, ny, nz = shape
    if (tau is None) == (eta_s is None):
        raise ValueError("give exactly one of tau, eta_s")
    ins = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)).ravel() for a in fields]
    C = nx * ny * nz
    outs = dict(n=np.empty(C), eps=np.empty(C), U=np.empty((4, C)), P=np.empty(C)) if outputs else None
    r = Request(REQ_TUBE if kind == "tube" else REQ_BOX, nx, ny, nz, _prec(precision),
                TAU_FIXED if tau is not None else TAU_ETA_S, int(order), float(tau or 0.0), float(eta_s or 0.0),
                int(steps),
                *[_dp(a) for a in ins],
                *([_dp(outs[k]) for k in ("n", "eps", "U", "P")] if outs else [None] * 4))
    return r, ins, outs


def request_bytes(kind, shape, precision, order=ORDER3):
    nx, ny, nz = shape
    r = Request(REQ_TUBE if kind == "tube" else REQ_BOX, nx, ny, nz, _prec(precision), TAU_FIXED, int(order), 1.0,
                0.0, 0)
    one = np.ones(1)
    r.n = r.eps = r.vx = r.vy = r.vz = _dp(one)
    return lib().rlb_request_bytes(ctypes.byref(r))


class Server:
    """Continuous-batching server over a torch-owned device pool."""

    def __init__(self, pool_bytes, chunk_steps=50, max_tubes=1024, device=None):
        import torch
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=self.device)
        # the server writes the pool only on its own streams: let work still
        # queued on torch's stream with an earlier owner of this memory finish
        torch.cuda.current_stream(self.device).synchronize()
        h = ctypes.c_void_p()
        check(lib().rlb_server_create(ctypes.byref(h), ctypes.c_void_p(self.pool.data_ptr()), int(pool_bytes),
                                      int(chunk_steps), int(max_tubes)))
        self._h = h
        self._free = lib().rlb_server_destroy
        self._live = {}      # id -> (request, inputs, outputs)

    def submit(self, kind, shape, precision, steps, fields, tau=None, eta_s=None, outputs=True, order=ORDER3):
        r, ins, outs = make_request(kind, shape, precision, steps, fields, tau, eta_s, outputs, order)
        rid = ctypes.c_int64()
        check(lib().rlb_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid)))
        self._live[rid.value] = (r, outs)    # outputs stay alive until reported
        return rid.value

    def poll(self, max_n=256, wait_ms=0):
        buf = (Completion * max_n)()
        cnt = ctypes.c_int32()
        check(lib().rlb_server_poll(self._h, buf, max_n, ctypes.byref(cnt), int(wait_ms)))
        out = []
        for c in buf[:cnt.value]:
            _, outs = self._live.pop(c.id, (None, None))
            out.append(dict(id=c.id, rc=c.rc, flags=c.flags, t_submit=c.t_submit, t_admit=c.t_admit,
                            t_done=c.t_done, fields=outs))
        return out

    def pending(self):
        p = ctypes.c_int64()
        r = ctypes.c_int64()
        check(lib().rlb_server_pending(self._h, ctypes.byref(p), ctypes.byref(r)))
        return p.value, r.value

    def drain(self, timeout_s=600.0):
        """Poll until every submitted request has been reported."""
        import time
        done = []
        t_end = time.time() + timeout_s
        while self.pending()[0] > 0:
            if time.time() > t_end:
                raise TimeoutError("server did not finish in %.0f s" % timeout_s)
            done.extend(self.poll(wait_ms=100))
        done.extend(self.poll())
        return done

    def close(self):
        h, free = getattr(self, "_h", None), getattr(self, "_free", None)
        if h is not None and h.value and free is not None:
            free(h)
            self._h = None

    def __del__(self):
        self.close()
