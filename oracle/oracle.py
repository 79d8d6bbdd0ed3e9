"""ctypes wrapper of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline leg of bench.py, never by the product package.  A configuration is a
plain dict and a particle set a dict of numpy arrays (the same plain-data
format the product binding accepts; each side converts it on its own).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class OrDesc(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("tau", C.c_double), ("rho0", C.c_double),
        ("bc", C.c_int32 * 6), ("wall_u", (C.c_double * 3) * 6),
        ("body_force", C.c_double * 3), ("kolm_amp", C.c_double),
        ("kolm_axis", C.c_int32), ("kolm_dir", C.c_int32),
        ("gravity", C.c_double * 3),
        ("sf_method", C.c_int32), ("sf_subdiv", C.c_int32),
        ("fluid_on", C.c_int32), ("dem_on", C.c_int32), ("n_sub", C.c_int32),
        ("dem_cell", C.c_double),
        ("kn", C.c_double), ("restitution", C.c_double), ("mu", C.c_double),
        ("kt_ratio", C.c_double), ("gt_ratio", C.c_double),
        ("max_solids", C.c_int32),
        ("collision", C.c_int32), ("trt_magic", C.c_double),
        ("contact_law", C.c_int32), ("young", C.c_double), ("poisson", C.c_double),
    ]


def lib():
    global _lib
    if _lib is not None:
        return _lib
    path = _build.LIB
    src = os.path.join(_build.HERE, "oracle.c")
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
        _build.build()
    L = C.CDLL(path)
    P = C.c_void_p
    dp = C.POINTER(C.c_double)
    L.or_create.restype = P
    L.or_create.argtypes = [C.POINTER(OrDesc), C.c_int32, P, P, P, P, P, P, P, P]
    L.or_error.restype = C.c_char_p
    L.or_destroy.argtypes = [P]
    L.or_step.argtypes = [P, C.c_int64]
    L.or_nsub.argtypes = [P]
    L.or_nsub.restype = C.c_int32
    L.or_dem_grid.argtypes = [P, P, P]
    L.or_mass.argtypes = [P, C.c_int32]
    L.or_mass.restype = C.c_double
    for n in ("or_get_populations", "or_set_populations"):
        getattr(L, n).argtypes = [P, P]
    L.or_get_fields.argtypes = [P, P, P]
    L.or_get_particles.argtypes = [P] + [P] * 10
    L.or_set_particles.argtypes = [P] + [P] * 8
    L.or_get_predicted.argtypes = [P, P, P]
    L.or_get_scales.argtypes = [P, P, P, P, P]
    L.or_get_rounding_scales.argtypes = [P, P, P, P, P]
    L.or_set_predicted.argtypes = [P, P, P]
    L.or_get_pairs.argtypes = [P, C.c_int64, P, P]
    L.or_get_pairs.restype = C.c_int64
    L.or_set_pairs.argtypes = [P, C.c_int64, P, P]
    L.or_get_cells.argtypes = [P, C.c_int64, P]
    L.or_get_cells.restype = C.c_int64
    L.or_get_solid.argtypes = [P, C.c_int64, P, P, P]
    L.or_get_solid.restype = C.c_int64
    L.or_get_contacts.argtypes = [P, C.c_int64, P, P, P, P]
    L.or_get_contacts.restype = C.c_int64
    L.or_counters.argtypes = [P, P]
    for n in ("or_stage_lists", "or_stage_voxelize", "or_stage_lbm", "or_stage_contacts"):
        getattr(L, n).argtypes = [P]
    L.or_brute_pairs.argtypes = [P, C.c_int64, P]
    L.or_brute_pairs.restype = C.c_int64
    L.or_feq.argtypes = [C.c_double, P, P]
    L.or_collide_cell.argtypes = [P, P, C.c_int32, P, P, P, P, P]
    L.or_beta_subdiv_sphere.argtypes = [C.c_double] * 4 + [C.c_int32] * 4
    L.or_beta_subdiv_sphere.restype = C.c_double
    L.or_beta_distance.argtypes = [C.c_double] * 4 + [C.c_int32] * 3
    L.or_beta_distance.restype = C.c_double
    L.or_contact_geometry.argtypes = [P, C.c_int32, C.c_int32, P, P, P, P, P]
    L.or_contact_geometry.restype = C.c_int32
    L.or_set_threads.argtypes = [C.c_int32]
    L.or_get_threads.restype = C.c_int32
    _lib = L
    return L


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


_BC = {"periodic": 0, "noslip": 1, "moving": 2}


def make_desc(cfg):
    d = OrDesc()
    d.nx, d.ny, d.nz = (int(v) for v in cfg["n"])
    d.tau = float(cfg["tau"])
    d.rho0 = float(cfg.get("rho0", 1.0))
    bc = cfg.get("bc", ["periodic"] * 6)
    for f in range(6):
        d.bc[f] = _BC[bc[f]] if isinstance(bc[f], str) else int(bc[f])
        for k in range(3):
            d.wall_u[f][k] = float(cfg.get("wall_u", [[0.0] * 3] * 6)[f][k])
    for k in range(3):
        d.body_force[k] = float(cfg.get("body_force", [0.0] * 3)[k])
        d.gravity[k] = float(cfg.get("gravity", [0.0] * 3)[k])
    d.kolm_amp = float(cfg.get("kolm_amp", 0.0))
    d.kolm_axis = int(cfg.get("kolm_axis", 1))
    d.kolm_dir = int(cfg.get("kolm_dir", 0))
    d.sf_method = {"subdivision": 0, "distance": 1}[cfg.get("sf_method", "subdivision")]
    d.sf_subdiv = int(cfg.get("sf_subdiv", 10))
    d.fluid_on = int(cfg.get("fluid_on", True))
    d.dem_on = int(cfg.get("dem_on", True))
    d.n_sub = int(cfg.get("n_sub", 0))
    d.dem_cell = float(cfg.get("dem_cell", 0.0))
    d.kn = float(cfg.get("kn", 1e3))
    d.restitution = float(cfg.get("restitution", 1.0))
    d.mu = float(cfg.get("mu", 0.0))
    d.kt_ratio = float(cfg.get("kt_ratio", 1.0))
    d.gt_ratio = float(cfg.get("gt_ratio", 1.0))
    d.max_solids = int(cfg.get("max_solids", 2))
    d.collision = {"bgk": 0, "trt": 1}[cfg.get("collision", "bgk")]
    d.trt_magic = float(cfg.get("trt_magic", 0.0))
    d.contact_law = {"linear": 0, "hertz": 1}[cfg.get("contact_law", "linear")]
    d.young = float(cfg.get("young", 0.0))
    d.poisson = float(cfg.get("poisson", 0.0))
    return d


class OracleDomain:
    """One oracle domain; the API mirrors the product's Domain."""

    def __init__(self, cfg, parts):
        L = lib()
        self.cfg = dict(cfg)
        self.desc = make_desc(cfg)
        self.n = tuple(int(v) for v in cfg["n"])
        self.N = self.n[0] * self.n[1] * self.n[2]
        p = _particle_arrays(parts)
        self.np = p["n"]
        self._keep = p
        h = L.or_create(C.byref(self.desc), self.np, _ptr(p["shape"]), _ptr(p["semi"]),
                        _ptr(p["dens"]), _ptr(p["pos"]), _ptr(p["quat"]), _ptr(p["vel"]),
                        _ptr(p["omega"]), _ptr(p["fixed"]))
        if not h:
            raise ValueError("oracle rejected the configuration: " + L.or_error().decode())
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_destroy(self.h)
            self.h = None

    # ---- stepping -------------------------------------------------------------
    def step(self, n=1):
        lib().or_step(self.h, int(n))

    @property
    def n_sub(self):
        return lib().or_nsub(self.h)

    def dem_grid(self):
        nc = np.zeros(3, np.int32)
        h = np.zeros(3)
        lib().or_dem_grid(self.h, _ptr(nc), _ptr(h))
        return nc, h

    def mass(self):
        return np.array([lib().or_mass(self.h, k) for k in range(self.np)])

    # ---- state ----------------------------------------------------------------
    def populations(self):
        f = np.zeros(19 * self.N)
        lib().or_get_populations(self.h, _ptr(f))
        return f.reshape(19, self.N)

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        assert f.size == 19 * self.N
        lib().or_set_populations(self.h, _ptr(f))

    def fields(self):
        rho = np.zeros(self.N)
        u = np.zeros(3 * self.N)
        lib().or_get_fields(self.h, _ptr(rho), _ptr(u))
        return rho, u.reshape(self.N, 3)

    def particles(self):
        n = self.np
        out = {k: np.zeros((n, 3)) for k in ("pos", "vel", "omega", "acc", "alpha",
                                             "f_hyd", "m_hyd", "f_dem", "m_dem")}
        out["quat"] = np.zeros((n, 4))
        lib().or_get_particles(self.h, *[_ptr(out[k]) for k in (
            "pos", "quat", "vel", "omega", "acc", "alpha", "f_hyd", "m_hyd", "f_dem", "m_dem")])
        return out

    def set_particles(self, **kw):
        keys = ("pos", "quat", "vel", "omega", "acc", "alpha", "f_hyd", "m_hyd")
        arrs = [np.ascontiguousarray(kw[k], dtype=np.float64) if kw.get(k) is not None else None
                for k in keys]
        lib().or_set_particles(self.h, *[_ptr(a) for a in arrs])

    def scales(self):
        """Per-particle, per-component scales of the forces of the last step:
        f_hyd, m_hyd: the rounding scale of the momentum exchange, the
            population magnitudes each per-cell term is formed from (a
            difference of O(w_i) populations rounds relative to them);
        f_hyd_g, m_hyd_g: the same of the deviations f - w_i and f^eq - w_i,
            the quantities a shifted (f - w) storage and arithmetic round;
        f_hyd_sum, m_hyd_sum: the L1 norm of the per-cell terms themselves;
        f_dem, m_dem: the L1 norm of the pair forces and torques."""
        keys = ("f_hyd_sum", "m_hyd_sum", "f_dem", "m_dem")
        out = {k: np.zeros((self.np, 3)) for k in keys + ("f_hyd", "m_hyd", "f_hyd_g", "m_hyd_g")}
        lib().or_get_scales(self.h, *[_ptr(out[k]) for k in keys])
        lib().or_get_rounding_scales(self.h, *[_ptr(out[k]) for k in ("f_hyd", "m_hyd", "f_hyd_g", "m_hyd_g")])
        return out

    def predicted(self):
        vp = np.zeros((self.np, 3))
        wp = np.zeros((self.np, 3))
        lib().or_get_predicted(self.h, _ptr(vp), _ptr(wp))
        return vp, wp

    def set_predicted(self, vp, wp):
        vp = np.ascontiguousarray(vp, dtype=np.float64)
        wp = np.ascontiguousarray(wp, dtype=np.float64)
        lib().or_set_predicted(self.h, _ptr(vp), _ptr(wp))

    def pairs(self):
        n = lib().or_get_pairs(self.h, 0, None, None)
        k = np.zeros(n, np.uint64)
        hst = np.zeros((n, 3))
        lib().or_get_pairs(self.h, n, _ptr(k), _ptr(hst))
        return k, hst

    def set_pairs(self, keys, hist):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        hist = np.ascontiguousarray(hist, dtype=np.float64)
        lib().or_set_pairs(self.h, keys.size, _ptr(keys), _ptr(hist))

    def cells(self):
        n = lib().or_get_cells(self.h, 0, None)
        k = np.zeros(n, np.uint64)
        lib().or_get_cells(self.h, n, _ptr(k))
        return k

    def solid(self):
        n = lib().or_get_solid(self.h, 0, None, None, None)
        c = np.zeros(n, np.uint32)
        p = np.zeros(n, np.uint32)
        b = np.zeros(n)
        lib().or_get_solid(self.h, n, _ptr(c), _ptr(p), _ptr(b))
        return c, p, b

    def contacts(self):
        n = lib().or_get_contacts(self.h, 0, None, None, None, None)
        k = np.zeros(n, np.uint64)
        F = np.zeros((n, 3))
        mi = np.zeros((n, 3))
        mj = np.zeros((n, 3))
        lib().or_get_contacts(self.h, n, _ptr(k), _ptr(F), _ptr(mi), _ptr(mj))
        return k, F, mi, mj

    def counters(self):
        out = np.zeros(6, np.int64)
        lib().or_counters(self.h, _ptr(out))
        return dict(zip(("pairs", "contacts", "entries", "overflow", "registrations", "step"),
                        out.tolist()))

    # ---- stages ---------------------------------------------------------------
    def stage_lists(self):
        lib().or_stage_lists(self.h)

    def stage_voxelize(self):
        lib().or_stage_voxelize(self.h)

    def stage_lbm(self):
        lib().or_stage_lbm(self.h)

    def stage_contacts(self):
        lib().or_stage_contacts(self.h)

    def brute_pairs(self):
        n = lib().or_brute_pairs(self.h, 0, None)
        k = np.zeros(n, np.uint64)
        lib().or_brute_pairs(self.h, n, _ptr(k))
        return np.sort(k)

    def collide_cell(self, f, B, uk, F=(0.0, 0.0, 0.0)):
        f = np.ascontiguousarray(f, dtype=np.float64)
        B = np.ascontiguousarray(B, dtype=np.float64)
        uk = np.ascontiguousarray(uk, dtype=np.float64).reshape(-1)
        F = np.ascontiguousarray(F, dtype=np.float64)
        out = np.zeros(19)
        P = np.zeros(max(1, 3 * B.size))
        lib().or_collide_cell(self.h, _ptr(f), B.size, _ptr(B), _ptr(uk), _ptr(F), _ptr(out), _ptr(P))
        return out, P[:3 * B.size].reshape(-1, 3)

    def contact_geometry(self, i, j):
        d = C.c_double()
        en = np.zeros(3)
        rci = np.zeros(3)
        rcj = np.zeros(3)
        it = C.c_int32()
        ok = lib().or_contact_geometry(self.h, i, j, C.byref(d), _ptr(en), _ptr(rci), _ptr(rcj),
                                       C.byref(it))
        return dict(ok=bool(ok), delta=d.value, en=en, rci=rci, rcj=rcj, iters=it.value)


def feq(rho, u):
    out = np.zeros(19)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    lib().or_feq(float(rho), _ptr(uu), _ptr(out))
    return out


def beta_subdiv_sphere(c, R, X, Y, Z, ns=10):
    return lib().or_beta_subdiv_sphere(float(c[0]), float(c[1]), float(c[2]), float(R),
                                       int(X), int(Y), int(Z), int(ns))


def beta_distance(c, R, X, Y, Z):
    return lib().or_beta_distance(float(c[0]), float(c[1]), float(c[2]), float(R),
                                  int(X), int(Y), int(Z))


def set_threads(n):
    lib().or_set_threads(int(n))


def get_threads():
    return lib().or_get_threads()


def _particle_arrays(parts):
    if parts is None:
        parts = {}
    n = int(len(parts.get("pos", [])))

    def arr(key, shape, default, dtype=np.float64):
        v = parts.get(key)
        if v is None:
            a = np.zeros(shape, dtype)
            if default is not None:
                a[...] = default
            return a
        return np.ascontiguousarray(np.asarray(v, dtype=dtype).reshape(shape))

    q = arr("quat", (n, 4), None)
    if parts.get("quat") is None:
        q[:, 0] = 1.0
    return dict(n=n, shape=arr("shape", (n,), 0, np.int32), semi=arr("semi", (n, 3), None),
                dens=arr("dens", (n,), 1.0), pos=arr("pos", (n, 3), None), quat=q,
                vel=arr("vel", (n, 3), None), omega=arr("omega", (n, 3), None),
                fixed=arr("fixed", (n,), 0, np.uint8))
