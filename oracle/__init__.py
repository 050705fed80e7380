"""FP64 CPU oracle for the lattice Landau-de Gennes force and FIRE step.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check in __graft_entry__.py
and the cpu_baseline leg of bench.py may import this package.  The GPU library
never imports it and shares no code with it.

The arithmetic lives in lq_oracle.c (energy, its explicit gradient, FIRE,
gradient descent, Nesterov), geometry.py (site types and anchoring pairs) and
director.py (director and defect extraction); this module loads the C part
with ctypes and wraps it.  Every function cites the passage of the paper it
follows in its source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from .director import directors  # noqa: F401
from .geometry import q_from_director, rasterize  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lq_oracle.c")
_LIB = os.path.join(_HERE, "liblqoracle.so")


def build(force: bool = True) -> str:
    """Compiles the C oracle with gcc (OpenMP over z-planes)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC,
                        "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [("n", C.c_int64 * 3), ("periodic", C.c_int32 * 3),
                ("A", C.c_double), ("B", C.c_double), ("C", C.c_double),
                ("L1", C.c_double), ("L2", C.c_double), ("L3", C.c_double), ("L4", C.c_double),
                ("type", C.c_void_p), ("n_pairs", C.c_int64), ("pair_site", C.c_void_p),
                ("pair_W", C.c_void_p), ("pair_Q0", C.c_void_p), ("pair_kind", C.c_void_p),
                ("pair_nu", C.c_void_p), ("S0", C.c_double), ("hfield", C.c_double * 9)]


class FireParams(C.Structure):
    _fields_ = [("dt0", C.c_double), ("dt_max", C.c_double), ("alpha0", C.c_double),
                ("f_inc", C.c_double), ("f_dec", C.c_double), ("f_alpha", C.c_double),
                ("n_min", C.c_int64), ("force_tol", C.c_double), ("max_steps", C.c_int64)]


class FireState(C.Structure):
    _fields_ = [("dt", C.c_double), ("alpha", C.c_double), ("n_pos", C.c_int64),
                ("step", C.c_int64), ("restarts", C.c_int64), ("status", C.c_int32),
                ("pad", C.c_int32), ("P", C.c_double), ("normF", C.c_double),
                ("normv", C.c_double), ("maxF", C.c_double)]


class DescentParams(C.Structure):
    _fields_ = [("method", C.c_int32), ("pad", C.c_int32), ("dt", C.c_double),
                ("momentum", C.c_double), ("force_tol", C.c_double), ("max_steps", C.c_int64)]


RUNNING, CONVERGED, MAX_STEPS, NONFINITE = 0, 1, 2, 3
GD, NESTEROV = 1, 2

FORCE_FN = C.CFUNCTYPE(None, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double))

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.ora_threads.restype = C.c_int
        L.ora_threads.argtypes = []
        L.ora_S0.restype = C.c_double
        L.ora_S0.argtypes = [C.c_double, C.c_double, C.c_double]
        L.ora_energy.restype = C.c_double
        L.ora_energy.argtypes = [C.POINTER(_Problem), dp, dp]
        L.ora_forces.restype = None
        L.ora_forces.argtypes = [C.POINTER(_Problem), dp, dp]
        L.ora_forces_at.restype = None
        L.ora_forces_at.argtypes = [C.POINTER(_Problem), dp, C.c_int64, C.POINTER(C.c_int64), dp]
        L.ora_fire_init.restype = None
        L.ora_fire_init.argtypes = [C.POINTER(FireParams), C.POINTER(FireState), C.c_int64, dp, dp,
                                    dp, FORCE_FN, C.c_void_p, C.c_int]
        L.ora_fire_steps.restype = C.c_int64
        L.ora_fire_steps.argtypes = [C.POINTER(FireParams), C.POINTER(FireState), C.c_int64, dp,
                                     dp, dp, FORCE_FN, C.c_void_p, C.c_int64, dp]
        L.ora_fire_init_lattice.restype = None
        L.ora_fire_init_lattice.argtypes = [C.POINTER(_Problem), C.POINTER(FireParams),
                                            C.POINTER(FireState), dp, dp, dp, C.c_int]
        L.ora_fire_steps_lattice.restype = C.c_int64
        L.ora_fire_steps_lattice.argtypes = [C.POINTER(_Problem), C.POINTER(FireParams),
                                             C.POINTER(FireState), dp, dp, dp, C.c_int64, dp]
        L.ora_descent_init.restype = None
        L.ora_descent_init.argtypes = [C.POINTER(DescentParams), C.POINTER(FireState), C.c_int64, dp,
                                       dp, dp, FORCE_FN, C.c_void_p, C.c_int]
        L.ora_descent_steps.restype = C.c_int64
        L.ora_descent_steps.argtypes = [C.POINTER(DescentParams), C.POINTER(FireState), C.c_int64,
                                        dp, dp, dp, FORCE_FN, C.c_void_p, C.c_int64, dp]
        L.ora_descent_init_lattice.restype = None
        L.ora_descent_init_lattice.argtypes = [C.POINTER(_Problem), C.POINTER(DescentParams),
                                               C.POINTER(FireState), dp, dp, dp, C.c_int]
        L.ora_descent_steps_lattice.restype = C.c_int64
        L.ora_descent_steps_lattice.argtypes = [C.POINTER(_Problem), C.POINTER(DescentParams),
                                                C.POINTER(FireState), dp, dp, dp, C.c_int64, dp]
        _lib = L
    return _lib


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def threads() -> int:
    """Threads the oracle's parallel loops use (OpenMP)."""
    return int(lib().ora_threads())


def S0(A, B, C_):
    """Eq. (S0def)."""
    return lib().ora_S0(A, B, C_)


def descent_params(method, dt, momentum=0.0, force_tol=1e-9, max_steps=2000) -> DescentParams:
    """Gradient descent (method GD) or Nesterov's accelerated gradient
    (method NESTEROV, momentum mu)."""
    m = {"gd": GD, "nesterov": NESTEROV}.get(method, method)
    return DescentParams(int(m), 0, float(dt), float(momentum), float(force_tol), int(max_steps))


def fire_params(dt0=1e-3, dt_max=1e-2, alpha0=0.99, f_inc=1.1, f_dec=0.5, f_alpha=0.99,
                n_min=5, force_tol=1e-9, max_steps=2000) -> FireParams:
    return FireParams(dt0, dt_max, alpha0, f_inc, f_dec, f_alpha, n_min, force_tol, max_steps)


class Problem:
    """One lattice: shape (nx, ny, nz), periodic flags, constants, geometry.

    Fields are SoA numpy arrays of shape (5, nz, ny, nx), float64.
    """

    def __init__(self, shape, periodic=(True, True, True), A=-0.172, B=-2.12, C_=1.73,
                 L1=2.32, L2=0.0, L3=0.0, objects=(), site_records=(), object_sites=(),
                 types=None, pairs=None, fields=(), L4=0.0):
        """fields: (h, chi) pairs giving f_ext = -(1/3) sum chi (h.Q.h), sec. II.A.3
        (chi = mu0 dchi or eps0 deps in units of |A|, h the field vector)."""
        self.shape = tuple(int(s) for s in shape)
        self.periodic = tuple(bool(p) for p in periodic)
        for k in range(3):
            if self.periodic[k] and self.shape[k] < 3:
                raise ValueError("a periodic axis needs at least 3 sites")
        self.A, self.B, self.C, self.L1, self.L2, self.L3, self.L4 = A, B, C_, L1, L2, L3, L4
        self.S0 = S0(A, B, C_)
        if types is None:
            types, ps, pw, pq, pk, pn = rasterize(self.shape, self.periodic, list(objects), self.S0,
                                                  site_records, object_sites, full=True)
        else:
            ps, pw, pq = pairs
            pk = np.zeros(len(ps), np.uint8)
            pn = np.zeros((len(ps), 3))
        self.types = np.ascontiguousarray(types, dtype=np.uint8)
        self.pair_site = np.ascontiguousarray(ps, dtype=np.int64)
        self.pair_W = np.ascontiguousarray(pw, dtype=np.float64)
        self.pair_Q0 = np.ascontiguousarray(pq, dtype=np.float64).reshape(-1, 5)
        self.pair_kind = np.ascontiguousarray(pk, dtype=np.uint8)
        self.pair_nu = np.ascontiguousarray(pn, dtype=np.float64).reshape(-1, 3)
        self.hfield = np.zeros((3, 3))
        for h, chi in fields:
            h = np.asarray(h, dtype=np.float64)
            self.hfield += chi / 3.0 * np.outer(h, h)
        nx, ny, nz = self.shape
        self.N = nx * ny * nz
        self._s = _Problem((C.c_int64 * 3)(nx, ny, nz),
                           (C.c_int32 * 3)(*[int(p) for p in self.periodic]),
                           A, B, C_, L1, L2, L3, L4, self.types.ctypes.data, len(self.pair_site),
                           self.pair_site.ctypes.data, self.pair_W.ctypes.data,
                           self.pair_Q0.ctypes.data, self.pair_kind.ctypes.data,
                           self.pair_nu.ctypes.data, self.S0,
                           (C.c_double * 9)(*self.hfield.reshape(-1).tolist()))

    @property
    def field_shape(self):
        nx, ny, nz = self.shape
        return (5, nz, ny, nx)

    @property
    def n_sim(self):
        return int((self.types != 2).sum())

    def _chk(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        assert q.size == 5 * self.N
        return q

    def uniaxial(self, directors, S=None):
        """q = 3/2 S (n n - I/3) at simulated sites, 0 inside objects."""
        S = self.S0 if S is None else S
        nx, ny, nz = self.shape
        q = q_from_director(np.asarray(directors, dtype=np.float64).reshape(3, -1), S)
        q[:, self.types == 2] = 0.0
        return np.ascontiguousarray(q.reshape(self.field_shape))

    def energy(self, q, terms=False):
        q = self._chk(q)
        t = np.zeros(4)
        e = lib().ora_energy(C.byref(self._s), _dp(q), _dp(t))
        return (e, t) if terms else e

    def forces(self, q):
        q = self._chk(q)
        F = np.empty(self.field_shape)
        lib().ora_forces(C.byref(self._s), _dp(q), _dp(F))
        return F

    def forces_at(self, q, sites):
        q = self._chk(q)
        sites = np.ascontiguousarray(sites, dtype=np.int64)
        out = np.empty((len(sites), 5))
        lib().ora_forces_at(C.byref(self._s), _dp(q), len(sites),
                            sites.ctypes.data_as(C.POINTER(C.c_int64)), _dp(out))
        return out

    # ---- FIRE (Algorithm 1) ----
    def fire_init(self, params, q, v=None, keep_v=False):
        """Returns (state, q, v, F) with fresh FIRE state."""
        q = self._chk(q).copy()
        v = np.zeros(self.field_shape) if v is None else self._chk(v).copy()
        F = np.empty(self.field_shape)
        st = FireState()
        lib().ora_fire_init_lattice(C.byref(self._s), C.byref(params), C.byref(st), _dp(q),
                                    _dp(v), _dp(F), int(keep_v))
        return st, q, v, F

    def fire_steps(self, params, st, q, v, F, n_steps, trace=False):
        tr = np.zeros((max(int(n_steps), 1), 6)) if trace else None
        taken = lib().ora_fire_steps_lattice(C.byref(self._s), C.byref(params), C.byref(st),
                                             _dp(q), _dp(v), _dp(F), int(n_steps),
                                             _dp(tr) if trace else None)
        return (taken, tr[:taken]) if trace else taken

    def minimize(self, params, q):
        st, q, v, F = self.fire_init(params, q)
        self.fire_steps(params, st, q, v, F, params.max_steps)
        return st, q, v, F

    # ---- gradient descent / Nesterov (sec. III.B) ----
    def descent_init(self, params, q, m=None):
        """Returns (state, q, m, F); F is the force at q (GD) or q + mu m (Nesterov)."""
        q = self._chk(q).copy()
        keep = m is not None
        m = np.zeros(self.field_shape) if m is None else self._chk(m).copy()
        F = np.empty(self.field_shape)
        st = FireState()
        lib().ora_descent_init_lattice(C.byref(self._s), C.byref(params), C.byref(st), _dp(q),
                                       _dp(m), _dp(F), int(keep))
        return st, q, m, F

    def descent_steps(self, params, st, q, m, F, n_steps, trace=False):
        tr = np.zeros((max(int(n_steps), 1), 6)) if trace else None
        taken = lib().ora_descent_steps_lattice(C.byref(self._s), C.byref(params), C.byref(st),
                                                _dp(q), _dp(m), _dp(F), int(n_steps),
                                                _dp(tr) if trace else None)
        return (taken, tr[:taken]) if trace else taken


def descent_generic(params, x0, force, n_steps, m0=None):
    """GD / Nesterov of the oracle over an arbitrary force(x) -> F callable.
    Returns (state, iterates x_0..x_t, trace, m, F)."""
    x = np.ascontiguousarray(x0, dtype=np.float64).copy()
    n = x.size
    m = np.zeros(n) if m0 is None else np.ascontiguousarray(m0, dtype=np.float64).copy()
    F = np.empty(n)

    def cb(ctx, xp, Fp):
        xa = np.ctypeslib.as_array(xp, shape=(n,))
        Fa = np.ctypeslib.as_array(Fp, shape=(n,))
        Fa[:] = force(xa.copy())

    fn = FORCE_FN(cb)
    st = FireState()
    lib().ora_descent_init(C.byref(params), C.byref(st), n, _dp(x), _dp(m), _dp(F), fn, None,
                           int(m0 is not None))
    tr = np.zeros((max(int(n_steps), 1), 6))
    xs = [x.copy()]
    taken = 0
    for _ in range(int(n_steps)):
        t = lib().ora_descent_steps(C.byref(params), C.byref(st), n, _dp(x), _dp(m), _dp(F), fn,
                                    None, 1, _dp(tr[taken:]))
        if t == 0:
            break
        taken += t
        xs.append(x.copy())
    return st, np.array(xs), tr[:taken], m, F


def fire_generic(params, x0, force, n_steps, v0=None, trace=True):
    """FIRE of the oracle over an arbitrary force(x) -> F callable (numpy)."""
    x = np.ascontiguousarray(x0, dtype=np.float64).copy()
    n = x.size
    v = np.zeros(n) if v0 is None else np.ascontiguousarray(v0, dtype=np.float64).copy()
    F = np.empty(n)

    def cb(ctx, xp, Fp):
        xa = np.ctypeslib.as_array(xp, shape=(n,))
        Fa = np.ctypeslib.as_array(Fp, shape=(n,))
        Fa[:] = force(xa.copy())

    fn = FORCE_FN(cb)
    st = FireState()
    lib().ora_fire_init(C.byref(params), C.byref(st), n, _dp(x), _dp(v), _dp(F), fn, None,
                        int(v0 is not None))
    tr = np.zeros((max(int(n_steps), 1), 6))
    xs = [x.copy()]
    taken = 0
    # one step at a time so the caller can see every iterate
    for _ in range(int(n_steps)):
        t = lib().ora_fire_steps(C.byref(params), C.byref(st), n, _dp(x), _dp(v), _dp(F), fn,
                                 None, 1, _dp(tr[taken:]))
        if t == 0:
            break
        taken += t
        xs.append(x.copy())
    return st, np.array(xs), tr[:taken], v, F
