"""ctypes wrapper of the plain-C FP64 oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

NCOMP = 9
COMP = {"ex": 0, "ey": 1, "ez": 2, "bx": 3, "by": 4, "bz": 5,
        "jx": 6, "jy": 7, "jz": 8}
GUARD = 3


class _Grid(C.Structure):
    _fields_ = [("dims", C.c_int), ("nx", C.c_long), ("ny", C.c_long),
                ("dx", C.c_double), ("dy", C.c_double), ("dt", C.c_double)]


class _Incident(C.Structure):
    _fields_ = [("kind", C.c_int), ("a0", C.c_double), ("fwhm_t", C.c_double),
                ("t0", C.c_double), ("ka", C.c_double), ("s", C.c_double),
                ("phi0", C.c_double), ("x_focus", C.c_double),
                ("y_focus", C.c_double), ("t_focus", C.c_double),
                ("norm", C.c_double), ("on_nodes", C.c_int),
                ("w0", C.c_double), ("z_focus", C.c_double)]


class _Grid3(C.Structure):
    _fields_ = [("nx", C.c_long), ("ny", C.c_long), ("nz", C.c_long),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("dt", C.c_double)]


_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)


def lib():
    global _lib
    if _lib is None:
        # SFPIC_ORACLE_LIB names another build of these sources (the CPU
        # tests build copies with a mistake planted, to show that a pin
        # catches it); the default is the in-tree library
        path = os.environ.get("SFPIC_ORACLE_LIB")
        if not path:
            path = os.path.join(_HERE, "liboracle.so")
            srcs = [os.path.join(_HERE, f) for f in _build.SOURCES]
            if not os.path.exists(path) or any(
                    os.path.getmtime(path) < os.path.getmtime(f)
                    for f in srcs):
                _build.build(force=True)
        L = C.CDLL(path)
        L.orc_april_ka_from_w0.restype = C.c_double
        L.orc_april_ka_from_w0.argtypes = [C.c_double]
        L.orc_incident_setup.argtypes = [C.POINTER(_Incident)]
        L.orc_incident_eval.argtypes = [C.POINTER(_Incident), C.c_int,
                                        C.c_double, C.c_double, C.c_double,
                                        _D, _D]
        L.orc_april_complex.argtypes = [C.c_int] + [C.c_double] * 7 + \
            [C.c_int, _D]
        L.orc_shape2.restype = C.c_double
        L.orc_shape2.argtypes = [C.c_double]
        L.orc_boris.argtypes = [C.c_double, C.c_double, _D, _D, _D]
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(_Grid), C.POINTER(_Incident)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_add_species.argtypes = [C.c_void_p, C.c_double, C.c_double,
                                      C.c_double, C.c_long, _D, _D, _D, _D, _D]
        L.orc_step.argtypes = [C.c_void_p, C.c_long]
        for f in ("orc_nx_alloc", "orc_ny_alloc", "orc_step_index"):
            getattr(L, f).restype = C.c_long
            getattr(L, f).argtypes = [C.c_void_p]
        L.orc_set_step_index.argtypes = [C.c_void_p, C.c_long]
        L.orc_field.restype = _D
        L.orc_field.argtypes = [C.c_void_p, C.c_int]
        L.orc_count.restype = C.c_long
        L.orc_count.argtypes = [C.c_void_p, C.c_int]
        L.orc_alive.restype = C.c_long
        L.orc_alive.argtypes = [C.c_void_p, C.c_int]
        L.orc_get_particles.argtypes = [C.c_void_p, C.c_int, _D, _D, _D, _D,
                                        _D, _I]
        L.orc_set_particles.argtypes = [C.c_void_p, C.c_int, _D, _D, _D, _D,
                                        _D, _I]
        L.orc_gather_arrays.argtypes = [C.c_void_p, C.c_double, C.c_double,
                                        _D, _D]
        L.orc_deposit_rho.argtypes = [C.c_void_p, _D]
        L.orc_diagnostics.argtypes = [C.c_void_p, _D]
        L.orc_em_energy_total.restype = C.c_double
        L.orc_em_energy_total.argtypes = [C.c_void_p]
        L.orc_energy_angle.argtypes = [C.c_void_p, C.c_int, C.c_int,
                                       C.c_double, C.c_int, C.c_double,
                                       C.c_int, _D, _D]
        L.orc3_incident_eval.argtypes = [C.POINTER(_Incident)] + \
            [C.c_double] * 4 + [_D, _D]
        L.orc3_create.restype = C.c_void_p
        L.orc3_create.argtypes = [C.POINTER(_Grid3), C.POINTER(_Incident)]
        L.orc3_destroy.argtypes = [C.c_void_p]
        L.orc3_add_species.argtypes = [C.c_void_p, C.c_double, C.c_double,
                                       C.c_double, C.c_long] + [_D] * 6
        L.orc3_n_alloc.restype = C.c_long
        L.orc3_n_alloc.argtypes = [C.c_void_p, C.c_int]
        L.orc3_step_index.restype = C.c_long
        L.orc3_step_index.argtypes = [C.c_void_p]
        L.orc3_field.restype = _D
        L.orc3_field.argtypes = [C.c_void_p, C.c_int]
        L.orc3_count.restype = C.c_long
        L.orc3_count.argtypes = [C.c_void_p, C.c_int]
        L.orc3_get_particles.argtypes = [C.c_void_p, C.c_int] + [_D] * 6 + [_I]
        L.orc3_gather.argtypes = [C.c_void_p] + [C.c_double] * 3 + [_D, _D]
        L.orc3_step.argtypes = [C.c_void_p, C.c_long]
        L.orc3_deposit_rho.argtypes = [C.c_void_p, _D]
        L.orc3_diagnostics.argtypes = [C.c_void_p, _D]
        L.orc3_em_energy_total.restype = C.c_double
        L.orc3_em_energy_total.argtypes = [C.c_void_p]
        L.orc3_energy_angle.argtypes = [C.c_void_p, C.c_int, C.c_int,
                                        C.c_double, C.c_int, C.c_double,
                                        C.c_int, _D, _D]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_D)


def ka_from_w0(w0: float) -> float:
    return lib().orc_april_ka_from_w0(w0)


def _make_incident(inc) -> _Incident:
    """inc: workloads.Incident (or any object with the same attributes)."""
    ci = _Incident()
    ci.kind = int(inc.kind)
    ci.a0 = float(inc.a0)
    ci.fwhm_t = float(getattr(inc, "fwhm_t", 0.0))
    ci.t0 = float(getattr(inc, "t0", 0.0))
    w0 = float(getattr(inc, "w0", 0.0))
    ci.ka = ka_from_w0(w0) if w0 > 0 else float(getattr(inc, "ka", 0.0))
    ci.s = float(getattr(inc, "s", 10.0))
    ci.phi0 = float(getattr(inc, "phi0", 0.0))
    ci.x_focus = float(getattr(inc, "x_focus", 0.0))
    ci.y_focus = float(getattr(inc, "y_focus", 0.0))
    ci.t_focus = float(getattr(inc, "t_focus", 0.0))
    ci.on_nodes = int(getattr(inc, "on_nodes", 0))
    ci.w0 = w0
    ci.z_focus = float(getattr(inc, "z_focus", 0.0))
    if lib().orc_incident_setup(C.byref(ci)) != 0:
        raise ValueError("incident setup failed")
    return ci


def incident_norm(inc) -> float:
    return _make_incident(inc).norm


def incident_eval(inc, dims, x, y, t):
    ci = _make_incident(inc)
    E = np.zeros(3)
    B = np.zeros(3)
    lib().orc_incident_eval(C.byref(ci), dims, x, y, t, _dp(E), _dp(B))
    return E, B


def april_complex(kind, X, Y, Z, T, ka, s, phi0=0.0, use_series=-1):
    out = np.zeros(12)
    lib().orc_april_complex(kind, X, Y, Z, T, ka, s, phi0, use_series,
                            _dp(out))
    v = out[0::2] + 1j * out[1::2]
    return v[:3], v[3:]


def shape2(d: float) -> float:
    return lib().orc_shape2(d)


def boris(qm, dt, u, E, B):
    u = np.array(u, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    lib().orc_boris(qm, dt, _dp(u), _dp(E), _dp(B))
    return u


class OracleSim:
    """One simulation held by the oracle."""

    def __init__(self, grid, incident):
        g = _Grid()
        g.dims, g.nx, g.ny = int(grid.dims), int(grid.nx), int(grid.ny)
        g.dx, g.dy, g.dt = float(grid.dx), float(grid.dy), float(grid.dt)
        self.grid = grid
        self._inc = _make_incident(incident)
        self._h = lib().orc_create(C.byref(g), C.byref(self._inc))
        if not self._h:
            raise ValueError("orc_create failed")
        self.NX = lib().orc_nx_alloc(self._h)
        self.NY = lib().orc_ny_alloc(self._h)
        self.nsp = 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    @property
    def norm(self):
        return self._inc.norm

    def add_species(self, q, m, w, x, y, ux, uy, uz):
        arrs = [np.ascontiguousarray(a, dtype=np.float64)
                for a in (x, y, ux, uy, uz)]
        n = len(arrs[0])
        r = lib().orc_add_species(self._h, q, m, w, n, *[_dp(a) for a in arrs])
        if r < 0:
            raise ValueError("too many species")
        self.nsp += 1
        return r

    def step(self, n=1):
        lib().orc_step(self._h, int(n))

    @property
    def step_index(self):
        return lib().orc_step_index(self._h)

    def set_step_index(self, n):
        lib().orc_set_step_index(self._h, int(n))

    def field(self, comp) -> np.ndarray:
        """Live (writable) view of one field array, shape (NY, NX)."""
        c = COMP[comp] if isinstance(comp, str) else int(comp)
        p = lib().orc_field(self._h, c)
        return np.ctypeslib.as_array(p, shape=(self.NY, self.NX))

    def particles(self, sp=0):
        n = lib().orc_count(self._h, sp)
        out = [np.zeros(n) for _ in range(5)]
        alive = np.zeros(n, dtype=np.int32)
        lib().orc_get_particles(self._h, sp, *[_dp(a) for a in out],
                                alive.ctypes.data_as(_I))
        return (*out, alive.astype(bool))

    def set_particles(self, sp, x, y, ux, uy, uz, alive):
        arrs = [np.ascontiguousarray(a, dtype=np.float64)
                for a in (x, y, ux, uy, uz)]
        al = np.ascontiguousarray(alive, dtype=np.int32)
        lib().orc_set_particles(self._h, sp, *[_dp(a) for a in arrs],
                                al.ctypes.data_as(_I))

    def n_alive(self, sp=0):
        return lib().orc_alive(self._h, sp)

    def gather(self, x, y):
        E = np.zeros(3)
        B = np.zeros(3)
        lib().orc_gather_arrays(self._h, x, y, _dp(E), _dp(B))
        return E, B

    def rho(self):
        r = np.zeros((self.NY, self.NX))
        lib().orc_deposit_rho(self._h, _dp(r))
        return r

    def diagnostics(self):
        o = np.zeros(4)
        lib().orc_diagnostics(self._h, _dp(o))
        return {"w_kin": o[0], "w_em": o[1], "charge": o[2],
                "n_alive": int(o[3]),
                "w_em_total": lib().orc_em_energy_total(self._h)}

    def energy_angle(self, sp=0, n_e=256, emax=1.0, n_theta=180,
                     ek_min=1.0e3 / 510998.95, plane=0):
        """plane: 0 angle from +x, 1 (2) of the momentum projected on the
        x-z (x-y) plane."""
        h = np.zeros((n_e, n_theta))
        mom = np.zeros(5)
        lib().orc_energy_angle(self._h, sp, n_e, emax, n_theta, ek_min,
                               int(plane), _dp(h), _dp(mom))
        return h, mom


def incident_eval3(inc, x, y, z, t):
    """Incident field at a 3D point (build axes)."""
    ci = _make_incident(inc)
    E = np.zeros(3)
    B = np.zeros(3)
    lib().orc3_incident_eval(C.byref(ci), x, y, z, t, _dp(E), _dp(B))
    return E, B


class OracleSim3:
    """One 3D3V simulation held by the oracle; arrays are (NZ, NY, NX)."""

    def __init__(self, grid, incident):
        g = _Grid3()
        g.nx, g.ny, g.nz = int(grid.nx), int(grid.ny), int(grid.nz)
        g.dx, g.dy, g.dz = float(grid.dx), float(grid.dy), float(grid.dz)
        g.dt = float(grid.dt)
        self.grid = grid
        self._inc = _make_incident(incident)
        self._h = lib().orc3_create(C.byref(g), C.byref(self._inc))
        if not self._h:
            raise ValueError("orc3_create failed")
        self.shape = tuple(lib().orc3_n_alloc(self._h, a) for a in (2, 1, 0))
        self.nsp = 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc3_destroy(h)
            self._h = None

    def add_species(self, q, m, w, x, y, z, ux, uy, uz):
        arrs = [np.ascontiguousarray(a, dtype=np.float64)
                for a in (x, y, z, ux, uy, uz)]
        r = lib().orc3_add_species(self._h, q, m, w, len(arrs[0]),
                                   *[_dp(a) for a in arrs])
        if r < 0:
            raise ValueError("too many species")
        self.nsp += 1
        return r

    def step(self, n=1):
        lib().orc3_step(self._h, int(n))

    @property
    def step_index(self):
        return lib().orc3_step_index(self._h)

    def field(self, comp) -> np.ndarray:
        """Live (writable) view of one field array, shape (NZ, NY, NX)."""
        c = COMP[comp] if isinstance(comp, str) else int(comp)
        return np.ctypeslib.as_array(lib().orc3_field(self._h, c),
                                     shape=self.shape)

    def particles(self, sp=0):
        n = lib().orc3_count(self._h, sp)
        out = [np.zeros(n) for _ in range(6)]
        alive = np.zeros(n, dtype=np.int32)
        lib().orc3_get_particles(self._h, sp, *[_dp(a) for a in out],
                                 alive.ctypes.data_as(_I))
        return (*out, alive.astype(bool))

    def gather(self, x, y, z):
        E = np.zeros(3)
        B = np.zeros(3)
        lib().orc3_gather(self._h, x, y, z, _dp(E), _dp(B))
        return E, B

    def rho(self):
        r = np.zeros(self.shape)
        lib().orc3_deposit_rho(self._h, _dp(r))
        return r

    def diagnostics(self):
        o = np.zeros(4)
        lib().orc3_diagnostics(self._h, _dp(o))
        return {"w_kin": o[0], "w_em": o[1], "charge": o[2],
                "n_alive": int(o[3]),
                "w_em_total": lib().orc3_em_energy_total(self._h)}

    def energy_angle(self, sp=0, n_e=256, emax=1.0, n_theta=180,
                     ek_min=1.0e3 / 510998.95, plane=0):
        """plane: 0 angle from +x, 1 (2) of the momentum projected on the
        x-z (x-y) plane."""
        h = np.zeros((n_e, n_theta))
        mom = np.zeros(5)
        lib().orc3_energy_angle(self._h, sp, n_e, emax, n_theta, ek_min,
                                int(plane), _dp(h), _dp(mom))
        return h, mom
