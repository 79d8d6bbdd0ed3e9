"""ctypes binding of libpsmdem.so (the C ABI in include/psmdem.h).

Argument marshalling only: every step of the coupled time step runs in the HIP
library.  PyTorch supplies the HIP stream and, by default, device memory (the
library's allocator callback is routed to torch's caching allocator).  There is
no fallback: if the library is missing or no GPU is present, the calls raise.

A configuration is a plain dict and a particle set a dict of numpy arrays; see
paper_2512_04997_amd.workloads for the keys.
"""
import atexit
import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsmdem.so")
_lib = None

OK, E_INVALID, E_NOMEM, E_CAPACITY, E_UNSTABLE, E_HIP, E_STATE, E_NODEVICE = 0, -1, -2, -3, -4, -5, -6, -7
PRECISION = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3}
BC = {"periodic": 0, "noslip": 1, "moving": 2}
COLLISION = {"bgk": 0, "trt": 1}
CONTACT_LAW = {"linear": 0, "hertz": 1}
STAGE = {"lists": 0, "voxelize": 1, "lbm": 2, "contacts": 3}
TIMER = {"lbm": 0, "voxel": 1, "dem": 2, "hydro": 3}


class PsmdemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"psmdem error {code}: {msg}")
        self.code = code


class Desc(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("tau", C.c_double), ("rho0", C.c_double),
        ("bc", C.c_int32 * 6), ("wall_u", (C.c_double * 3) * 6),
        ("body_force", C.c_double * 3), ("kolm_amp", C.c_double),
        ("kolm_axis", C.c_int32), ("kolm_dir", C.c_int32),
        ("gravity", C.c_double * 3),
        ("precision", C.c_int32), ("sf_method", C.c_int32), ("sf_subdiv", C.c_int32),
        ("fluid_on", C.c_int32), ("dem_on", C.c_int32), ("n_sub", C.c_int32),
        ("dem_cell", C.c_double),
        ("kn", C.c_double), ("restitution", C.c_double), ("mu", C.c_double),
        ("kt_ratio", C.c_double), ("gt_ratio", C.c_double),
        ("max_solids", C.c_int32), ("pair_capacity", C.c_int64),
        ("collision", C.c_int32), ("trt_magic", C.c_double),
        ("contact_law", C.c_int32), ("young", C.c_double), ("poisson", C.c_double),
    ]


class Particles(C.Structure):
    _fields_ = [("n", C.c_int32), ("shape", C.c_void_p), ("semi_axes", C.c_void_p),
                ("density_ratio", C.c_void_p), ("pos", C.c_void_p), ("quat", C.c_void_p),
                ("vel", C.c_void_p), ("omega", C.c_void_p), ("fixed", C.c_void_p)]


class Counters(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("n_pairs", "n_contacts", "n_registrations", "n_entries",
                                         "n_dropped", "n_solid_tiles", "step", "flags")]


class Info(C.Structure):
    _fields_ = [("n_sub", C.c_int32), ("dem_cells", C.c_int32 * 3), ("dem_h", C.c_double * 3),
                ("n_cells", C.c_int64), ("n_particles", C.c_int32), ("precision", C.c_int32),
                ("device_bytes", C.c_int64), ("tile", C.c_int32 * 3)]


class ServerDesc(C.Structure):
    _fields_ = [("max_jobs", C.c_int32), ("hbm_budget", C.c_int64), ("max_inflight", C.c_int32),
                ("precision", C.c_int32)]


class JobInfo(C.Structure):
    _fields_ = [("state", C.c_int32), ("slot", C.c_int32), ("steps", C.c_int64), ("steps_done", C.c_int64),
                ("footprint", C.c_int64), ("status", C.c_int32), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double)]


JOB_STATE = {0: "queued", 1: "active", 2: "finishing", 3: "done", 4: "failed"}

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)


def lib():
    """Loads libpsmdem.so; raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(the HIP library is the only compute path)")
    # torch first: the library's libamdhip64.so.7 then resolves to the HIP
    # runtime torch already loaded, so one runtime owns the device, the streams
    # and the memory of the process
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    st = C.c_int
    L.psmdem_create.argtypes = [C.POINTER(Desc), C.POINTER(Particles), P, ALLOC_FN, FREE_FN, P,
                                C.POINTER(P)]
    L.psmdem_create.restype = st
    L.psmdem_destroy.argtypes = [P]
    L.psmdem_destroy.restype = None
    L.psmdem_step.argtypes = [P, C.c_int64]
    L.psmdem_sync.argtypes = [P]
    L.psmdem_stage.argtypes = [P, C.c_int32]
    L.psmdem_read_populations.argtypes = [P, P]
    L.psmdem_write_populations.argtypes = [P, P]
    L.psmdem_read_fields.argtypes = [P, P, P]
    L.psmdem_read_fields_noalloc.argtypes = [P, P, P]
    L.psmdem_read_particles.argtypes = [P] + [P] * 10
    L.psmdem_write_particles.argtypes = [P] + [P] * 8
    L.psmdem_read_predicted.argtypes = [P, P, P]
    L.psmdem_write_predicted.argtypes = [P, P, P]
    L.psmdem_read_pairs.argtypes = [P, C.c_int64, P, P, C.POINTER(C.c_int64)]
    L.psmdem_write_pairs.argtypes = [P, C.c_int64, P, P]
    L.psmdem_read_contacts.argtypes = [P, C.c_int64, P, P, P, P, C.POINTER(C.c_int64)]
    L.psmdem_read_cells.argtypes = [P, C.c_int64, P, C.POINTER(C.c_int64)]
    L.psmdem_read_solid.argtypes = [P, C.c_int64, P, P, P, C.POINTER(C.c_int64)]
    L.psmdem_counters.argtypes = [P, C.POINTER(Counters)]
    L.psmdem_info.argtypes = [P, C.POINTER(Info)]
    L.psmdem_set_timing.argtypes = [P, C.c_int32]
    L.psmdem_timing.argtypes = [P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.psmdem_footprint.argtypes = [C.POINTER(Desc), C.POINTER(Particles), C.POINTER(C.c_int64)]
    L.psmdem_read_state.argtypes = [P, P, C.c_size_t, C.POINTER(C.c_size_t)]
    L.psmdem_write_state.argtypes = [P, P, C.c_size_t]
    L.psmdem_clock.argtypes = []
    L.psmdem_clock.restype = C.c_double
    L.psmdem_server_create.argtypes = [C.POINTER(ServerDesc), P, P, ALLOC_FN, FREE_FN, P, C.POINTER(P)]
    L.psmdem_server_destroy.argtypes = [P]
    L.psmdem_server_destroy.restype = None
    L.psmdem_server_submit.argtypes = [P, C.POINTER(Desc), C.POINTER(Particles), C.c_int64,
                                       C.POINTER(C.c_int64)]
    L.psmdem_server_iterate.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.psmdem_server_drain.argtypes = [P]
    L.psmdem_server_job.argtypes = [P, C.c_int64, C.POINTER(JobInfo)]
    L.psmdem_server_domain.argtypes = [P, C.c_int64, C.POINTER(P)]
    L.psmdem_server_release.argtypes = [P, C.c_int64]
    L.psmdem_last_error.restype = C.c_char_p
    L.psmdem_last_error.argtypes = []
    L.psmdem_version.restype = C.c_char_p
    L.psmdem_version.argtypes = []
    for name in ("psmdem_step", "psmdem_sync", "psmdem_stage", "psmdem_read_populations",
                 "psmdem_write_populations", "psmdem_read_fields", "psmdem_read_fields_noalloc",
                 "psmdem_read_particles",
                 "psmdem_write_particles", "psmdem_read_predicted", "psmdem_write_predicted",
                 "psmdem_read_pairs", "psmdem_write_pairs", "psmdem_read_contacts",
                 "psmdem_read_cells", "psmdem_read_solid", "psmdem_counters", "psmdem_info",
                 "psmdem_set_timing", "psmdem_timing", "psmdem_footprint", "psmdem_read_state",
                 "psmdem_write_state",
                 "psmdem_server_create",
                 "psmdem_server_submit", "psmdem_server_iterate", "psmdem_server_drain", "psmdem_server_job",
                 "psmdem_server_domain", "psmdem_server_release"):
        getattr(L, name).restype = st
    _lib = L
    return L


def _check(code):
    if code != OK:
        raise PsmdemError(code, lib().psmdem_last_error().decode())


# live domains and servers, closed at interpreter exit while torch (whose
# caching allocator takes their device memory back) is still up
_LIVE = weakref.WeakSet()


@atexit.register
def _close_live():
    for obj in list(_LIVE):
        try:
            obj.close()
        except Exception:
            pass


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_desc(cfg):
    d = Desc()
    d.nx, d.ny, d.nz = (int(v) for v in cfg["n"])
    d.tau = float(cfg["tau"])
    d.rho0 = float(cfg.get("rho0", 1.0))
    bc = cfg.get("bc", ["periodic"] * 6)
    wu = cfg.get("wall_u", [[0.0] * 3] * 6)
    for f in range(6):
        d.bc[f] = BC[bc[f]] if isinstance(bc[f], str) else int(bc[f])
        for k in range(3):
            d.wall_u[f][k] = float(wu[f][k])
    for k in range(3):
        d.body_force[k] = float(cfg.get("body_force", [0.0] * 3)[k])
        d.gravity[k] = float(cfg.get("gravity", [0.0] * 3)[k])
    d.kolm_amp = float(cfg.get("kolm_amp", 0.0))
    d.kolm_axis = int(cfg.get("kolm_axis", 1))
    d.kolm_dir = int(cfg.get("kolm_dir", 0))
    prec = cfg.get("precision", "fp64")
    d.precision = PRECISION[prec] if isinstance(prec, str) else int(prec)
    d.sf_method = {"subdivision": 0, "distance": 1}[cfg.get("sf_method", "subdivision")]
    d.sf_subdiv = int(cfg.get("sf_subdiv", 10))
    d.fluid_on = int(bool(cfg.get("fluid_on", True)))
    d.dem_on = int(bool(cfg.get("dem_on", True)))
    d.n_sub = int(cfg.get("n_sub", 0))
    d.dem_cell = float(cfg.get("dem_cell", 0.0))
    d.kn = float(cfg.get("kn", 1e3))
    d.restitution = float(cfg.get("restitution", 1.0))
    d.mu = float(cfg.get("mu", 0.0))
    d.kt_ratio = float(cfg.get("kt_ratio", 1.0))
    d.gt_ratio = float(cfg.get("gt_ratio", 1.0))
    d.max_solids = int(cfg.get("max_solids", 2))
    d.pair_capacity = int(cfg.get("pair_capacity", 0))
    d.collision = COLLISION[cfg.get("collision", "bgk")]
    d.trt_magic = float(cfg.get("trt_magic", 0.0))
    d.contact_law = CONTACT_LAW[cfg.get("contact_law", "linear")]
    d.young = float(cfg.get("young", 0.0))
    d.poisson = float(cfg.get("poisson", 0.0))
    return d


def _particle_struct(parts):
    parts = parts or {}
    n = int(len(parts.get("pos", [])))

    def arr(key, shape, dtype, default=None):
        v = parts.get(key)
        if v is None:
            if default is None:
                return None
            a = np.zeros(shape, dtype)
            a[...] = default
            return a
        return np.ascontiguousarray(np.asarray(v, dtype=dtype).reshape(shape))

    keep = dict(shape=arr("shape", (n,), np.int32, 0), semi=arr("semi", (n, 3), np.float64, 0.0),
                dens=arr("dens", (n,), np.float64, 1.0), pos=arr("pos", (n, 3), np.float64, 0.0),
                quat=arr("quat", (n, 4), np.float64), vel=arr("vel", (n, 3), np.float64),
                omega=arr("omega", (n, 3), np.float64), fixed=arr("fixed", (n,), np.uint8))
    s = Particles(n, _ptr(keep["shape"]), _ptr(keep["semi"]), _ptr(keep["dens"]), _ptr(keep["pos"]),
                  _ptr(keep["quat"]), _ptr(keep["vel"]), _ptr(keep["omega"]), _ptr(keep["fixed"]))
    return s, keep, n


class _TorchAlloc:
    """Routes the library's device allocations to torch's caching allocator."""

    def __init__(self, stream_ptr):
        import torch
        self.torch = torch
        self.stream = stream_ptr
        self.dev = torch.cuda.current_device()
        self.live = {}

        def _alloc(n, ctx):
            try:
                p = torch.cuda.caching_allocator_alloc(int(n), self.dev, self.stream)
            except Exception:  # out of memory: the library reports E_NOMEM
                return None
            self.live[p] = n
            return p

        def _free(p, n, ctx):
            if p in self.live:
                del self.live[p]
                try:
                    torch.cuda.caching_allocator_delete(p)
                except Exception:  # the interpreter is shutting down: the process frees the device
                    pass

        self.alloc = ALLOC_FN(_alloc)
        self.free = FREE_FN(_free)


class Domain:
    """One coupled LBM-PSM-DEM domain on the current GPU (psmdem_create)."""

    def __init__(self, cfg, parts=None, stream=None, allocator="torch", strict=True):
        """strict: reads raise on the device flags (E_UNSTABLE, E_CAPACITY);
        otherwise they return the outputs and leave the flag in self.flag."""
        L = lib()
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP library is the only compute path")
        self.strict = strict
        self.flag = OK
        self.cfg = dict(cfg)
        self.desc = make_desc(cfg)
        self.n = tuple(int(v) for v in cfg["n"])
        self.N = self.n[0] * self.n[1] * self.n[2]
        ps, self._keep, self.np = _particle_struct(parts)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        sptr = C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        self._alloc = _TorchAlloc(sptr.value) if allocator == "torch" else None
        h = C.c_void_p()
        code = L.psmdem_create(C.byref(self.desc), C.byref(ps), sptr,
                               self._alloc.alloc if self._alloc else ALLOC_FN(),
                               self._alloc.free if self._alloc else FREE_FN(), None, C.byref(h))
        _check(code)
        self.h = h
        _LIVE.add(self)

    @classmethod
    def _attach(cls, handle, cfg, parts):
        """A non-owning view of a domain held elsewhere (a served job)."""
        self = cls.__new__(cls)
        self.cfg = dict(cfg)
        self.desc = make_desc(cfg)
        self.n = tuple(int(v) for v in cfg["n"])
        self.N = self.n[0] * self.n[1] * self.n[2]
        _, self._keep, self.np = _particle_struct(parts)
        self.stream = None
        self._alloc = None
        self.h = handle
        self._owner = False
        self.strict = True
        self.flag = OK
        return self

    def close(self):
        if getattr(self, "h", None):
            if getattr(self, "_owner", True):
                lib().psmdem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- stepping -------------------------------------------------------------
    def step(self, n=1):
        _check(lib().psmdem_step(self.h, int(n)))

    def _rd(self, code):
        """Status of a read: the device flags raise only in strict mode."""
        if code in (E_CAPACITY, E_UNSTABLE):
            self.flag = code
            if not self.strict:
                return
        _check(code)

    def sync(self):
        """Waits for the device; returns the device flag status (0 OK)."""
        code = lib().psmdem_sync(self.h)
        self._rd(code)
        return code

    def stage(self, name):
        _check(lib().psmdem_stage(self.h, STAGE[name]))

    def info(self):
        i = Info()
        _check(lib().psmdem_info(self.h, C.byref(i)))
        return dict(n_sub=i.n_sub, dem_cells=list(i.dem_cells), dem_h=list(i.dem_h), n_cells=i.n_cells,
                    n_particles=i.n_particles, precision=i.precision, device_bytes=i.device_bytes,
                    tile=list(i.tile))

    @property
    def n_sub(self):
        return self.info()["n_sub"]

    def counters(self):
        c = Counters()
        _check(lib().psmdem_counters(self.h, C.byref(c)))
        return {n: getattr(c, n) for n, _ in Counters._fields_}

    def set_timing(self, on=True):
        _check(lib().psmdem_set_timing(self.h, int(bool(on))))

    def timing(self, which):
        ms = C.c_double()
        n = C.c_int64()
        _check(lib().psmdem_timing(self.h, TIMER[which], C.byref(ms), C.byref(n)))
        return ms.value, n.value

    # ---- state ----------------------------------------------------------------
    def populations(self):
        f = np.zeros(19 * self.N)
        self._rd(lib().psmdem_read_populations(self.h, _ptr(f)))
        return f.reshape(19, self.N)

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        if f.size != 19 * self.N:
            raise ValueError("populations must have 19 * n_cells entries")
        _check(lib().psmdem_write_populations(self.h, _ptr(f)))

    def fields(self, noalloc=False):
        """Density [N] and velocity [N, 3] (noalloc: the entry point that
        allocates no device memory)."""
        rho = np.zeros(self.N)
        u = np.zeros(3 * self.N)
        fn = lib().psmdem_read_fields_noalloc if noalloc else lib().psmdem_read_fields
        self._rd(fn(self.h, _ptr(rho), _ptr(u)))
        return rho, u.reshape(self.N, 3)

    def particles(self):
        n = self.np
        out = {k: np.zeros((n, 3)) for k in ("pos", "vel", "omega", "acc", "alpha",
                                             "f_hyd", "m_hyd", "f_dem", "m_dem")}
        out["quat"] = np.zeros((n, 4))
        self._rd(lib().psmdem_read_particles(self.h, *[_ptr(out[k]) for k in (
            "pos", "quat", "vel", "omega", "acc", "alpha", "f_hyd", "m_hyd", "f_dem", "m_dem")]))
        return out

    def set_particles(self, **kw):
        keys = ("pos", "quat", "vel", "omega", "acc", "alpha", "f_hyd", "m_hyd")
        arrs = [np.ascontiguousarray(kw[k], dtype=np.float64) if kw.get(k) is not None else None
                for k in keys]
        _check(lib().psmdem_write_particles(self.h, *[_ptr(a) for a in arrs]))

    def predicted(self):
        vp = np.zeros((self.np, 3))
        wp = np.zeros((self.np, 3))
        self._rd(lib().psmdem_read_predicted(self.h, _ptr(vp), _ptr(wp)))
        return vp, wp

    def set_predicted(self, vp, wp):
        _check(lib().psmdem_write_predicted(self.h, _ptr(np.ascontiguousarray(vp, np.float64)),
                                            _ptr(np.ascontiguousarray(wp, np.float64))))

    def pairs(self):
        n = C.c_int64()
        self._rd(lib().psmdem_read_pairs(self.h, 0, None, None, C.byref(n)))
        k = np.zeros(n.value, np.uint64)
        hst = np.zeros((n.value, 3))
        self._rd(lib().psmdem_read_pairs(self.h, n.value, _ptr(k), _ptr(hst), C.byref(n)))
        return k, hst

    def set_pairs(self, keys, hist):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        hist = np.ascontiguousarray(hist, dtype=np.float64)
        _check(lib().psmdem_write_pairs(self.h, keys.size, _ptr(keys), _ptr(hist)))

    def contacts(self):
        n = C.c_int64()
        self._rd(lib().psmdem_read_contacts(self.h, 0, None, None, None, None, C.byref(n)))
        m = n.value
        k = np.zeros(m, np.uint64)
        F = np.zeros((m, 3))
        mi = np.zeros((m, 3))
        mj = np.zeros((m, 3))
        self._rd(lib().psmdem_read_contacts(self.h, m, _ptr(k), _ptr(F), _ptr(mi), _ptr(mj), C.byref(n)))
        return k, F, mi, mj

    def cells(self):
        n = C.c_int64()
        self._rd(lib().psmdem_read_cells(self.h, 0, None, C.byref(n)))
        k = np.zeros(n.value, np.uint64)
        self._rd(lib().psmdem_read_cells(self.h, n.value, _ptr(k), C.byref(n)))
        return k

    def state(self):
        """The whole domain state as a host byte image (psmdem_read_state)."""
        n = C.c_size_t()
        _check(lib().psmdem_read_state(self.h, None, 0, C.byref(n)))
        buf = np.empty(n.value, np.uint8)
        self._rd(lib().psmdem_read_state(self.h, _ptr(buf), buf.size, C.byref(n)))
        return buf

    def set_state(self, buf):
        """Restores an image of state() from a domain of the same layout."""
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(lib().psmdem_write_state(self.h, _ptr(buf), buf.size))
        self.flag = OK

    def solid(self):
        n = C.c_int64()
        self._rd(lib().psmdem_read_solid(self.h, 0, None, None, None, C.byref(n)))
        m = n.value
        c = np.zeros(m, np.uint32)
        p = np.zeros(m, np.uint32)
        b = np.zeros(m)
        self._rd(lib().psmdem_read_solid(self.h, m, _ptr(c), _ptr(p), _ptr(b), C.byref(n)))
        return c, p, b


def footprint(cfg, parts=None):
    """Device bytes a domain of this configuration allocates (no device needed)."""
    d = make_desc(cfg)
    ps, _keep, _ = _particle_struct(parts)
    b = C.c_int64()
    _check(lib().psmdem_footprint(C.byref(d), C.byref(ps), C.byref(b)))
    return b.value


def clock():
    """The library's monotonic host clock in seconds (the clock of job times)."""
    return lib().psmdem_clock()


class Server:
    """Continuous batching of many coupled domains (psmdem_server_*).

    Jobs are created on a separate admission stream; every active job steps on
    the compute stream in batched launches."""

    def __init__(self, max_jobs=32, hbm_budget=0, max_inflight=2, precision="fp32", stream=None,
                 admit_stream=None, allocator="torch"):
        L = lib()
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP library is the only compute path")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.admit_stream = admit_stream if admit_stream is not None else torch.cuda.Stream()
        sp = C.c_void_p(self.stream.cuda_stream)
        sa = C.c_void_p(self.admit_stream.cuda_stream)
        self._alloc = _TorchAlloc(sa.value) if allocator == "torch" else None
        d = ServerDesc(int(max_jobs), int(hbm_budget), int(max_inflight),
                       PRECISION[precision] if isinstance(precision, str) else int(precision))
        h = C.c_void_p()
        _LIVE.add(self)
        _check(L.psmdem_server_create(C.byref(d), sp, sa, self._alloc.alloc if self._alloc else ALLOC_FN(),
                                      self._alloc.free if self._alloc else FREE_FN(), None, C.byref(h)))
        self.h = h
        self._jobs = {}

    def submit(self, cfg, parts, steps):
        d = make_desc(cfg)
        ps, keep, _ = _particle_struct(parts)
        j = C.c_int64()
        _check(lib().psmdem_server_submit(self.h, C.byref(d), C.byref(ps), int(steps), C.byref(j)))
        self._jobs[j.value] = (dict(cfg), parts)
        return j.value

    def iterate(self):
        a = C.c_int32()
        q = C.c_int32()
        _check(lib().psmdem_server_iterate(self.h, C.byref(a), C.byref(q)))
        return a.value, q.value

    def drain(self):
        _check(lib().psmdem_server_drain(self.h))

    def job(self, jid):
        i = JobInfo()
        _check(lib().psmdem_server_job(self.h, int(jid), C.byref(i)))
        return dict(state=JOB_STATE.get(i.state, i.state), slot=i.slot, steps=i.steps, steps_done=i.steps_done,
                    footprint=i.footprint, status=i.status, t_submit=i.t_submit, t_admit=i.t_admit,
                    t_done=i.t_done)

    def domain(self, jid):
        """Read-only view of a done job's domain (valid until release)."""
        h = C.c_void_p()
        _check(lib().psmdem_server_domain(self.h, int(jid), C.byref(h)))
        cfg, parts = self._jobs[jid]
        return Domain._attach(h, cfg, parts)

    def release(self, jid):
        _check(lib().psmdem_server_release(self.h, int(jid)))
        self._jobs.pop(jid, None)

    def close(self):
        if getattr(self, "h", None):
            lib().psmdem_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def version():
    return lib().psmdem_version().decode()
