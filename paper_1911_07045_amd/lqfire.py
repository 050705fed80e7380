"""Python binding of liblqfire (ctypes): argument marshalling only.

Every computation happens in the HIP kernels behind include/lqfire.h; this
module converts torch tensors (device memory, streams) and Python geometry
descriptions into the C structs and checks shapes and dtypes.  It raises when
the library is missing: there is no other code path.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblqfire.so")

LQ_OK, LQ_EINVAL, LQ_EUNSUPPORTED, LQ_ENOMEM, LQ_EHIP, LQ_ENONFINITE, LQ_ESTATE = 0, -1, -2, -3, -4, -5, -6
LQ_F64, LQ_F32 = 0, 1
# bytes of the fixed per-GPU workspace of lq_minimize_noalloc (LQ_NOALLOC_WORKSPACE_BYTES)
NOALLOC_WORKSPACE_BYTES = 32 << 20
LQ_OBJ_WALL, LQ_OBJ_SPHERE, LQ_OBJ_PATTERNED_WALL = 1, 2, 3
LQ_LAW_ND, LQ_LAW_RP, LQ_LAW_FG = 0, 1, 2
LAWS = {"nd": LQ_LAW_ND, "rp": LQ_LAW_RP, "fg": LQ_LAW_FG}
ANCH_STRIDE = 21
LQ_DIR_NORMAL, LQ_DIR_FIXED = 0, 1
RUNNING, CONVERGED, MAX_STEPS, NONFINITE = 0, 1, 2, 3
LQ_METHOD_FIRE, LQ_METHOD_GD, LQ_METHOD_NESTEROV = 0, 1, 2

ERR_NAMES = {LQ_EINVAL: "LQ_EINVAL", LQ_EUNSUPPORTED: "LQ_EUNSUPPORTED", LQ_ENOMEM: "LQ_ENOMEM",
             LQ_EHIP: "LQ_EHIP", LQ_ENONFINITE: "LQ_ENONFINITE", LQ_ESTATE: "LQ_ESTATE"}


class LQError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("n", C.c_int64 * 3), ("periodic", C.c_int32 * 3), ("prec", C.c_int32),
                ("A", C.c_double), ("B", C.c_double), ("C", C.c_double),
                ("L1", C.c_double), ("L2", C.c_double), ("L3", C.c_double),
                ("L4", C.c_double), ("L6", C.c_double)]


class Object(C.Structure):
    _fields_ = [("kind", C.c_int32), ("law", C.c_int32), ("dir_mode", C.c_int32), ("axis", C.c_int32),
                ("plane", C.c_int64), ("W", C.c_double), ("center", C.c_double * 3),
                ("radius", C.c_double), ("dir", C.c_double * 3), ("pitch", C.c_double * 2),
                ("offset", C.c_double * 2), ("count", C.c_int32 * 2)]


class SiteAnchor(C.Structure):
    _fields_ = [("site", C.c_int64), ("law", C.c_int32), ("pad", C.c_int32), ("W", C.c_double),
                ("n0", C.c_double * 3)]


class EnergyTerms(C.Structure):
    _fields_ = [("bulk", C.c_double), ("elastic", C.c_double), ("anchoring", C.c_double),
                ("external", C.c_double), ("total", C.c_double), ("n_sim", C.c_int64)]


class FireParams(C.Structure):
    _fields_ = [("dt0", C.c_double), ("dt_max", C.c_double), ("alpha0", C.c_double),
                ("f_inc", C.c_double), ("f_dec", C.c_double), ("f_alpha", C.c_double),
                ("n_min", C.c_int64), ("force_tol", C.c_double), ("max_steps", C.c_int64)]


class FireReport(C.Structure):
    _fields_ = [("step", C.c_int64), ("n_pos", C.c_int64), ("restarts", C.c_int64),
                ("status", C.c_int32), ("pad", C.c_int32), ("dt", C.c_double),
                ("alpha", C.c_double), ("P", C.c_double), ("normF", C.c_double),
                ("normv", C.c_double), ("maxF", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class MinResult(C.Structure):
    """lq_min_result: the final controller, the energy of the final q and
    |F| / sqrt(N_sim).  Attributes of the controller (status, step, maxF, ...)
    read through to `fire`."""
    _fields_ = [("fire", FireReport), ("energy", EnergyTerms), ("normF_per_site", C.c_double)]

    def __getattr__(self, name):
        return getattr(self.fire, name)

    def as_dict(self):
        d = self.fire.as_dict()
        d.update({k: getattr(self.energy, k) for k, _ in EnergyTerms._fields_})
        d["normF_per_site"] = self.normF_per_site
        return d


class DescentParams(C.Structure):
    _fields_ = [("method", C.c_int32), ("pad", C.c_int32), ("dt", C.c_double),
                ("momentum", C.c_double), ("force_tol", C.c_double), ("max_steps", C.c_int64)]


_lib = None


def lib():
    """Loads liblqfire.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "or python paper_1911_07045_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, dp = C.c_void_p, C.c_int64, C.c_int32, C.POINTER(C.c_double)
        sig = {
            "lq_lattice_create": (C.c_int, [C.POINTER(Params), vp, C.POINTER(vp)]),
            "lq_lattice_destroy": (C.c_int, [vp]),
            "lq_bulk_S0": (C.c_double, [vp]),
            "lq_set_field": (C.c_int, [vp, C.POINTER(C.c_double), C.POINTER(C.c_double), i32]),
            "lq_set_boundaries": (C.c_int, [vp, C.POINTER(Object), i32, C.POINTER(SiteAnchor), i64,
                                            C.POINTER(C.c_int64), i64]),
            "lq_rasterize": (C.c_int, [C.POINTER(Params), C.POINTER(Object), i32, C.POINTER(SiteAnchor),
                                       i64, C.POINTER(C.c_int64), i64, C.POINTER(C.c_uint8),
                                       C.POINTER(C.c_int64), C.POINTER(C.c_int64), dp, i64]),
            "lq_set_uniaxial": (C.c_int, [vp, vp, C.c_double, vp]),
            "lq_compute_forces": (C.c_int, [vp, vp, vp]),
            "lq_energy": (C.c_int, [vp, vp, C.POINTER(EnergyTerms)]),
            "lq_workspace_bytes": (C.c_int64, [vp]),
            "lq_fire_init": (C.c_int, [vp, C.POINTER(FireParams), vp, vp, vp, vp, i64,
                                       C.POINTER(FireReport)]),
            "lq_fire_step": (C.c_int, [vp, i64, C.POINTER(FireReport)]),
            "lq_minimize": (C.c_int, [vp, C.POINTER(FireParams), vp, vp, vp, vp, i64,
                                      C.POINTER(MinResult)]),
            "lq_minimize_noalloc": (C.c_int, [vp, C.POINTER(FireParams), vp, vp, vp, C.POINTER(MinResult)]),
            "lq_descent_init": (C.c_int, [vp, C.POINTER(DescentParams), vp, vp, vp, vp, i64,
                                          C.POINTER(FireReport)]),
            "lq_descent_minimize": (C.c_int, [vp, C.POINTER(DescentParams), vp, vp, vp, vp, i64,
                                              C.POINTER(MinResult)]),
            "lq_director_field": (C.c_int, [vp, vp, vp, vp, vp, C.c_double, C.POINTER(C.c_int64)]),
            "lq_stream_copy": (C.c_int, [C.POINTER(vp), C.POINTER(vp), i32, i64, i32, vp]),
            "lq_step_plan": (C.c_int, [C.POINTER(Params), C.POINTER(Object), i32, i64, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_uint8), C.POINTER(C.c_int32), i64, C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
            "lq_last_error": (C.c_char_p, [vp]),
            "lq_batch_create": (C.c_int, [i32, vp, C.POINTER(vp)]),
            "lq_batch_destroy": (C.c_int, [vp]),
            "lq_batch_add": (C.c_int, [vp, vp]),
            "lq_batch_remove": (C.c_int, [vp, vp]),
            "lq_batch_size": (i32, [vp]),
            "lq_batch_step": (C.c_int, [vp, i64, C.POINTER(FireReport)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc, handle=None):
    if rc != LQ_OK:
        msg = lib().lq_last_error(handle)
        raise LQError(rc, msg.decode() if msg else "")


def make_params(shape, periodic=(True, True, True), prec="f64", A=-0.172, B=-2.12, C_=1.73,
                L1=2.32, L2=0.0, L3=0.0, L4=0.0, L6=0.0) -> Params:
    p = Params()
    p.n = (C.c_int64 * 3)(*[int(s) for s in shape])
    p.periodic = (C.c_int32 * 3)(*[int(bool(x)) for x in periodic])
    p.prec = LQ_F64 if prec in ("f64", LQ_F64) else LQ_F32
    p.A, p.B, p.C, p.L1, p.L2, p.L3, p.L4, p.L6 = A, B, C_, L1, L2, L3, L4, L6
    return p


def make_objects(objects):
    arr = (Object * max(len(objects), 1))()
    for i, o in enumerate(objects):
        t = arr[i]
        t.kind = {"wall": LQ_OBJ_WALL, "sphere": LQ_OBJ_SPHERE,
                  "patterned_wall": LQ_OBJ_PATTERNED_WALL}[o["kind"]]
        t.law = LAWS[o.get("law", "nd")]
        d = o.get("dir", "normal")
        if isinstance(d, str):
            if d != "normal":
                raise ValueError(f"unknown director mode {d!r}")
            t.dir_mode = LQ_DIR_NORMAL
        else:
            t.dir_mode = LQ_DIR_FIXED
            t.dir = (C.c_double * 3)(*[float(x) for x in d])
        t.axis = int(o.get("axis", 0))
        t.plane = int(o.get("plane", 0))
        t.W = float(o["W"])
        t.center = (C.c_double * 3)(*[float(x) for x in o.get("center", (0, 0, 0))])
        t.radius = float(o.get("radius", 0.0))
        t.pitch = (C.c_double * 2)(*[float(x) for x in o.get("pitch", (0, 0))])
        t.offset = (C.c_double * 2)(*[float(x) for x in o.get("offset", (0, 0))])
        t.count = (C.c_int32 * 2)(*[int(x) for x in o.get("count", (0, 0))])
    return arr, len(objects)


def _is_fg(law, W):
    return law == "fg" or (law == "rp" and float(W) < 0)


def make_records(records):
    """Per-site records {site, law, W, n0} (Nobili-Durand) or {site, law, W, nu}
    (Fournier-Galatola: law "fg", or "rp" with W < 0)."""
    arr = (SiteAnchor * max(len(records), 1))()
    for i, r in enumerate(records):
        law = r.get("law", "nd")
        arr[i].site = int(r["site"])
        arr[i].law = LAWS[law]
        arr[i].W = float(r["W"])
        v = r["nu"] if _is_fg(law, r["W"]) else r["n0"]
        arr[i].n0 = (C.c_double * 3)(*[float(x) for x in v])
    return arr, len(records)


def make_descent_params(method, dt, momentum=0.0, force_tol=1e-9, max_steps=2000) -> DescentParams:
    """method: "gd" or "nesterov" (or LQ_METHOD_*)."""
    m = {"gd": LQ_METHOD_GD, "nesterov": LQ_METHOD_NESTEROV}.get(method, method)
    return DescentParams(int(m), 0, float(dt), float(momentum), float(force_tol), int(max_steps))


def make_fire_params(dt0=1e-3, dt_max=1e-2, alpha0=0.99, f_inc=1.1, f_dec=0.5, f_alpha=0.99, n_min=5,
                     force_tol=1e-9, max_steps=2000) -> FireParams:
    return FireParams(dt0, dt_max, alpha0, f_inc, f_dec, f_alpha, n_min, force_tol, max_steps)


def rasterize(shape, periodic, objects=(), site_records=(), object_sites=(), A=-0.172, B=-2.12, C_=1.73):
    """Host-only rasterization (lq_rasterize): (types, anch_site, anch_data[n, ANCH_STRIDE]) as
    numpy; row i holds the upper triangle of K (15), b (5) and c of the site's anchoring energy
    1/2 q^T K q + b^T q + c."""
    import numpy as np
    p = make_params(shape, periodic, A=A, B=B, C_=C_)
    objs, no = make_objects(list(objects))
    recs, nr = make_records(list(site_records))
    osites = np.ascontiguousarray(np.asarray(object_sites, dtype=np.int64).reshape(-1))
    N = int(shape[0]) * int(shape[1]) * int(shape[2])
    types = np.zeros(N, dtype=np.uint8)
    n_anch = C.c_int64(0)
    args = [C.byref(p), objs, no, recs, nr, osites.ctypes.data_as(C.POINTER(C.c_int64)), len(osites),
            types.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(n_anch)]
    _check(lib().lq_rasterize(*args, None, None, 0))
    n = n_anch.value
    sites = np.zeros(max(n, 1), dtype=np.int64)
    data = np.zeros((max(n, 1), ANCH_STRIDE))
    _check(lib().lq_rasterize(*args, sites.ctypes.data_as(C.POINTER(C.c_int64)),
                              data.ctypes.data_as(C.POINTER(C.c_double)), n))
    return types, sites[:n], data[:n]


class Lattice:
    """One lattice handle (lq_lattice) bound to the current torch device and stream."""

    def __init__(self, shape, periodic=(True, True, True), prec="f64", A=-0.172, B=-2.12, C_=1.73,
                 L1=2.32, L2=0.0, L3=0.0, L4=0.0, L6=0.0, stream=None):
        import torch
        self.torch = torch
        self.shape = tuple(int(s) for s in shape)
        self.prec = "f64" if prec in ("f64", LQ_F64) else "f32"
        self.dtype = torch.float64 if self.prec == "f64" else torch.float32
        self.N = self.shape[0] * self.shape[1] * self.shape[2]
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._p = make_params(self.shape, periodic, self.prec, A, B, C_, L1, L2, L3, L4, L6)
        h = C.c_void_p()
        _check(lib().lq_lattice_create(C.byref(self._p), C.c_void_p(self.stream.cuda_stream),
                                       C.byref(h)))
        self.h = h
        self._ws = None
        self._bound = None

    def close(self):
        if getattr(self, "h", None):
            b = self._batch() if getattr(self, "_batch", None) else None
            if b is not None and self in b.members:
                b.members.remove(self)  # the library removes it from the batch too
            self._batch = None
            lib().lq_lattice_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def field_shape(self):
        nx, ny, nz = self.shape
        return (5, nz, ny, nx)

    @property
    def S0(self):
        return lib().lq_bulk_S0(self.h)

    def empty(self):
        return self.torch.empty(self.field_shape, dtype=self.dtype, device=self.device)

    def zeros(self):
        return self.torch.zeros(self.field_shape, dtype=self.dtype, device=self.device)

    def _field(self, t, name):
        if not (t.is_cuda and t.dtype == self.dtype and t.is_contiguous() and t.numel() == 5 * self.N
                and t.device == self.device):
            raise ValueError(f"{name} must be a contiguous {self.dtype} CUDA tensor of {5 * self.N} "
                             f"elements on {self.device}")
        return C.c_void_p(t.data_ptr())

    def set_boundaries(self, objects=(), site_records=(), object_sites=()):
        import numpy as np
        objs, no = make_objects(list(objects))
        recs, nr = make_records(list(site_records))
        osites = np.ascontiguousarray(np.asarray(object_sites, dtype=np.int64).reshape(-1))
        _check(lib().lq_set_boundaries(self.h, objs, no, recs, nr,
                                       osites.ctypes.data_as(C.POINTER(C.c_int64)), len(osites)), self.h)
        self._bound = None

    def set_field(self, fields=()):
        """fields: (h, chi) pairs, each adding -(chi/3) h.Q.h per simulated site."""
        import numpy as np
        fields = list(fields)
        h = np.ascontiguousarray(np.array([np.asarray(f[0], dtype=np.float64) for f in fields]
                                          if fields else np.zeros((1, 3))).reshape(-1))
        chi = np.ascontiguousarray(np.array([float(f[1]) for f in fields] if fields else [0.0]))
        _check(lib().lq_set_field(self.h, h.ctypes.data_as(C.POINTER(C.c_double)),
                                  chi.ctypes.data_as(C.POINTER(C.c_double)), len(fields)), self.h)
        self._bound = None

    def set_uniaxial(self, directors, q, S=None):
        """directors: float64 CUDA tensor (3, N) of unit vectors."""
        S = self.S0 if S is None else float(S)
        t = directors
        if not (t.is_cuda and t.dtype == self.torch.float64 and t.is_contiguous() and t.numel() == 3 * self.N):
            raise ValueError("directors must be a contiguous float64 CUDA tensor of 3*N elements")
        _check(lib().lq_set_uniaxial(self.h, C.c_void_p(t.data_ptr()), S, self._field(q, "q")), self.h)
        return q

    def compute_forces(self, q, F=None):
        F = self.empty() if F is None else F
        _check(lib().lq_compute_forces(self.h, self._field(q, "q"), self._field(F, "F")), self.h)
        return F

    def energy(self, q):
        out = EnergyTerms()
        _check(lib().lq_energy(self.h, self._field(q, "q"), C.byref(out)), self.h)
        return {"bulk": out.bulk, "elastic": out.elastic, "anchoring": out.anchoring,
                "external": out.external, "total": out.total, "n_sim": out.n_sim}

    def director_field(self, q, threshold, dirs=None, lambda_max=None, defect=None):
        """(dirs [3, N...], lambda_max [N...], defect [N...] uint8, n_defects) of q."""
        torch = self.torch
        shp = tuple(q.shape[1:])
        dirs = torch.empty((3,) + shp, dtype=self.dtype, device=self.device) if dirs is None else dirs
        lam = torch.empty(shp, dtype=self.dtype, device=self.device) if lambda_max is None else lambda_max
        dfc = torch.empty(shp, dtype=torch.uint8, device=self.device) if defect is None else defect
        for t, n, dt in ((dirs, 3 * self.N, self.dtype), (lam, self.N, self.dtype), (dfc, self.N, torch.uint8)):
            if not (t.is_cuda and t.dtype == dt and t.is_contiguous() and t.numel() == n and t.device == self.device):
                raise ValueError("director outputs must be contiguous CUDA tensors of the lattice's size")
        n = C.c_int64(0)
        _check(lib().lq_director_field(self.h, self._field(q, "q"), C.c_void_p(dirs.data_ptr()),
                                       C.c_void_p(lam.data_ptr()), C.c_void_p(dfc.data_ptr()),
                                       float(threshold), C.byref(n)), self.h)
        return dirs, lam, dfc, n.value

    def workspace_bytes(self):
        return int(lib().lq_workspace_bytes(self.h))

    def workspace(self):
        nb = self.workspace_bytes()
        if self._ws is None or self._ws.numel() < nb:
            self._ws = self.torch.empty(nb + 256, dtype=self.torch.uint8, device=self.device)
        off = (-self._ws.data_ptr()) % 256
        return self._ws, off

    def fire_init(self, params, q, v, F, resume=None):
        ws, off = self.workspace()
        rep = None if resume is None else C.byref(resume)
        _check(lib().lq_fire_init(self.h, C.byref(params), self._field(q, "q"), self._field(v, "v"),
                                  self._field(F, "F"), C.c_void_p(ws.data_ptr() + off),
                                  ws.numel() - off, rep), self.h)
        self._bound = (q, v, F)

    def fire_step(self, n_steps):
        r = FireReport()
        rc = lib().lq_fire_step(self.h, int(n_steps), C.byref(r))
        _check(rc, self.h)
        return r

    def minimize(self, params, q, v=None, F=None):
        """lq_minimize: returns (MinResult, q, v, F)."""
        v = self.empty() if v is None else v
        F = self.empty() if F is None else F
        ws, off = self.workspace()
        r = MinResult()
        _check(lib().lq_minimize(self.h, C.byref(params), self._field(q, "q"), self._field(v, "v"),
                                 self._field(F, "F"), C.c_void_p(ws.data_ptr() + off),
                                 ws.numel() - off, C.byref(r)), self.h)
        self._bound = (q, v, F)
        return r, q, v, F

    def minimize_noalloc(self, params, q, v, F):
        """lq_minimize_noalloc: lq_minimize with the library's fixed workspace;
        q, v, F are the caller's (nothing is allocated).  Returns MinResult;
        the lattice is left unbound."""
        r = MinResult()
        _check(lib().lq_minimize_noalloc(self.h, C.byref(params), self._field(q, "q"), self._field(v, "v"),
                                         self._field(F, "F"), C.byref(r)), self.h)
        self._bound = None
        return r

    def descent_init(self, params, q, v, F, resume=None):
        """Binds a gradient-descent or Nesterov run (lq_descent_init); advance it with fire_step."""
        ws, off = self.workspace()
        rep = None if resume is None else C.byref(resume)
        _check(lib().lq_descent_init(self.h, C.byref(params), self._field(q, "q"), self._field(v, "v"),
                                     self._field(F, "F"), C.c_void_p(ws.data_ptr() + off),
                                     ws.numel() - off, rep), self.h)
        self._bound = (q, v, F)

    def descent_minimize(self, params, q, v=None, F=None):
        v = self.zeros() if v is None else v
        F = self.empty() if F is None else F
        ws, off = self.workspace()
        r = MinResult()
        _check(lib().lq_descent_minimize(self.h, C.byref(params), self._field(q, "q"), self._field(v, "v"),
                                         self._field(F, "F"), C.c_void_p(ws.data_ptr() + off),
                                         ws.numel() - off, C.byref(r)), self.h)
        self._bound = (q, v, F)
        return r, q, v, F


class Batch:
    """lq_batch: many bound lattices advanced by one launch per FIRE step."""

    def __init__(self, capacity=256, stream=None):
        import torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _check(lib().lq_batch_create(int(capacity), C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.capacity = int(capacity)
        self.members = []

    def close(self):
        if getattr(self, "h", None):
            lib().lq_batch_destroy(self.h)
            self.h = None
            for m in self.members:
                m._batch = None
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return len(self.members)

    def add(self, lat: Lattice):
        _check(lib().lq_batch_add(self.h, lat.h), lat.h)
        self.members.append(lat)
        lat._batch = weakref.ref(self)

    def remove(self, lat: Lattice):
        _check(lib().lq_batch_remove(self.h, lat.h), lat.h)
        self.members.remove(lat)
        lat._batch = None

    def step(self, n_steps):
        """Returns one FireReport per member, in member order."""
        n = len(self.members)
        reps = (FireReport * max(n, 1))()
        rc = lib().lq_batch_step(self.h, int(n_steps), reps)
        if rc not in (LQ_OK, LQ_ENONFINITE):
            _check(rc)
        return [reps[i] for i in range(n)]


def step_plan(shape, periodic=(True, True, True), prec="f64", objects=(), resident=256, A=-0.172, B=-2.12,
              C_=1.73, L1=2.32, L2=0.0, L3=0.0, L4=0.0):
    """lq_step_plan (host only): the step kernels' chunks for this lattice on a
    device with `resident` resident step blocks.  Returns (chunks, bulk,
    (tile_x, tile_y), block) with chunks an int32 array of rows (x0, y0, z0,
    zc) in launch order, bulk a uint8 array and block the int32 index of the
    block that marches each chunk."""
    import numpy as np
    p = make_params(shape, periodic, prec, A, B, C_, L1, L2, L3, L4)
    objs, no = make_objects(list(objects))
    n = C.c_int64()
    tx, ty = C.c_int32(), C.c_int32()
    _check(lib().lq_step_plan(C.byref(p), objs, no, int(resident), None, None, None, 0, C.byref(n),
                              C.byref(tx), C.byref(ty)))
    chunks = np.zeros((n.value, 4), dtype=np.int32)
    bulk = np.zeros(n.value, dtype=np.uint8)
    block = np.zeros(n.value, dtype=np.int32)
    _check(lib().lq_step_plan(C.byref(p), objs, no, int(resident),
                              chunks.ctypes.data_as(C.POINTER(C.c_int32)),
                              bulk.ctypes.data_as(C.POINTER(C.c_uint8)),
                              block.ctypes.data_as(C.POINTER(C.c_int32)), n.value, C.byref(n), C.byref(tx),
                              C.byref(ty)))
    return chunks, bulk, (tx.value, ty.value), block


def stream_copy(src, dst, width=16, stream=None):
    """lq_stream_copy: copies each device tensor of src into the matching one
    of dst (same byte size) with the step kernel's streaming pattern; only
    enqueues on stream (default: torch's current stream)."""
    import torch
    if len(src) != len(dst) or not src:
        raise ValueError("src and dst must be equally long and non-empty")
    nbytes = src[0].numel() * src[0].element_size()
    for a, b in zip(src, dst):
        if a.numel() * a.element_size() != nbytes or b.numel() * b.element_size() != nbytes:
            raise ValueError("every stream must have the same byte size")
    s = (stream if stream is not None else torch.cuda.current_stream()).cuda_stream
    sp = (C.c_void_p * len(src))(*[t.data_ptr() for t in src])
    dp = (C.c_void_p * len(dst))(*[t.data_ptr() for t in dst])
    _check(lib().lq_stream_copy(sp, dp, len(src), nbytes, int(width), C.c_void_p(s)))


def lattice_from_config(cfg, prec=None, **kw) -> Lattice:
    """Lattice + geometry for one of the workload descriptions in synth."""
    lat = Lattice(cfg["shape"], cfg.get("periodic", (True, True, True)), prec or cfg.get("prec", "f64"),
                  L1=cfg["L1"], L2=cfg.get("L2", 0.0), L3=cfg.get("L3", 0.0), **kw)
    if cfg.get("objects"):
        lat.set_boundaries(cfg["objects"])
    if cfg.get("fields"):
        lat.set_field(cfg["fields"])
    return lat


def fire_params_from_config(cfg, **over) -> FireParams:
    f = dict(cfg["fire"])
    f.update(over)
    return make_fire_params(**f)
