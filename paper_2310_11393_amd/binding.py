"""Thin ctypes binding of the C ABI in include/sfpic.h (same names).

Argument marshalling only: every step of the method runs in the gfx950
kernels of libsfpic.so.  PyTorch, when present, supplies device memory (its
caching allocator) and the HIP stream.  If the library is not built this
module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfpic.so")

SFPIC_OK = 0
ERRORS = {-1: "E_INVAL", -2: "E_SIZE", -3: "E_NOMEM", -4: "E_DEVICE",
          -5: "E_NUMERIC", -6: "E_BUSY", -7: "E_STATE"}
GUARD = 3
COMP = {"ex": 0, "ey": 1, "ez": 2, "bx": 3, "by": 4, "bz": 5,
        "jx": 6, "jy": 7, "jz": 8}
FP64, FP32 = 0, 1


class SfpicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class sfpic_grid(C.Structure):
    _fields_ = [("dims", C.c_int32), ("nx", C.c_int64), ("ny", C.c_int64),
                ("dx", C.c_double), ("dy", C.c_double), ("dt", C.c_double)]


_DP = C.POINTER(C.c_double)


class sfpic_species(C.Structure):
    _fields_ = [("q", C.c_double), ("m", C.c_double),
                ("density", C.c_double), ("region", C.c_int64 * 4),
                ("ppc", C.c_int32), ("temperature_ev", C.c_double),
                ("seed", C.c_uint64), ("species_index", C.c_int32),
                ("n_explicit", C.c_int64), ("weight", C.c_double),
                ("x", _DP), ("y", _DP), ("ux", _DP), ("uy", _DP),
                ("uz", _DP)]


class sfpic_incident(C.Structure):
    _fields_ = [("kind", C.c_int32), ("a0", C.c_double),
                ("fwhm_t", C.c_double), ("t0", C.c_double),
                ("w0", C.c_double), ("s", C.c_double), ("phi0", C.c_double),
                ("x_focus", C.c_double), ("y_focus", C.c_double),
                ("t_focus", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)


class sfpic_runtime(C.Structure):
    _fields_ = [("stream", C.c_void_p), ("alloc", ALLOC_FN),
                ("free", FREE_FN), ("alloc_ctx", C.c_void_p),
                ("tile_x", C.c_int32), ("tile_y", C.c_int32),
                ("sort_every", C.c_int32), ("device", C.c_int32)]


class sfpic_diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("time", C.c_double),
                ("n_alive", C.c_int64), ("w_kin", C.c_double),
                ("w_em", C.c_double), ("charge", C.c_double),
                ("gauss_residual", C.c_double), ("rho_max", C.c_double),
                ("nonfinite", C.c_int32)]


class sfpic_hist_spec(C.Structure):
    _fields_ = [("species", C.c_int32), ("n_energy", C.c_int32),
                ("e_max", C.c_double), ("n_theta", C.c_int32),
                ("ek_min", C.c_double)]


_lib = None

# every symbol declared in include/sfpic.h
EXPORTS = ["sfpic_create", "sfpic_step", "sfpic_sync", "sfpic_read_field",
           "sfpic_write_field", "sfpic_set_step_index",
           "sfpic_particle_count", "sfpic_read_particles",
           "sfpic_diagnostics", "sfpic_histogram", "sfpic_get_state",
           "sfpic_set_state", "sfpic_profile", "sfpic_profile_read",
           "sfpic_destroy", "sfpic_last_error", "sfpic_version"]

KCLASSES = ("faraday", "push", "ampere", "sort", "stragglers")


class sfpic_kernel_stats(C.Structure):
    _fields_ = [("launches", C.c_int64 * 5), ("total_ms", C.c_double * 5)]


def lib():
    """Load libsfpic.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # Load torch's HIP runtime first: libsfpic.so then binds to the same
    # libamdhip64.so.7, so streams and allocations are shared, not duplicated.
    try:
        import torch  # noqa: F401
    except Exception:
        pass
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run "
                           "`python -c 'import __graft_entry__ as g; g.build()'`"
                           " or `python paper_2310_11393_amd/build.py`")
    L = C.CDLL(LIB_PATH)
    vp, i64, sz = C.c_void_p, C.c_int64, C.c_size_t
    L.sfpic_create.argtypes = [C.POINTER(sfpic_grid), C.POINTER(sfpic_species),
                               C.c_int, C.POINTER(sfpic_incident), C.c_int,
                               C.POINTER(sfpic_runtime), C.POINTER(vp)]
    L.sfpic_step.argtypes = [vp, i64]
    L.sfpic_sync.argtypes = [vp]
    L.sfpic_read_field.argtypes = [vp, C.c_int, _DP, sz]
    L.sfpic_write_field.argtypes = [vp, C.c_int, _DP, sz]
    L.sfpic_set_step_index.argtypes = [vp, i64]
    L.sfpic_particle_count.argtypes = [vp, C.c_int, C.POINTER(i64)]
    L.sfpic_read_particles.argtypes = [vp, C.c_int, _DP, _DP, _DP, _DP, _DP,
                                       C.POINTER(C.c_uint32), sz,
                                       C.POINTER(sz)]
    L.sfpic_diagnostics.argtypes = [vp, C.POINTER(sfpic_diag)]
    L.sfpic_histogram.argtypes = [vp, C.POINTER(sfpic_hist_spec), _DP, sz,
                                  _DP]
    L.sfpic_get_state.argtypes = [vp, vp, C.POINTER(sz)]
    L.sfpic_set_state.argtypes = [vp, vp, sz]
    L.sfpic_profile.argtypes = [vp, C.c_int]
    L.sfpic_profile_read.argtypes = [vp, C.POINTER(sfpic_kernel_stats)]
    L.sfpic_destroy.argtypes = [vp]
    L.sfpic_destroy.restype = None
    L.sfpic_last_error.restype = C.c_char_p
    L.sfpic_version.restype = C.c_char_p
    _lib = L
    return L


def _check(code):
    if code != SFPIC_OK:
        raise SfpicError(code, lib().sfpic_last_error().decode())


def _dp(a):
    return a.ctypes.data_as(_DP) if a is not None else None


class _TorchMemory:
    """Device memory from torch's caching allocator, on torch's stream."""

    def __init__(self, device=0):
        import torch
        self.torch = torch
        self.device = device
        self.stream = torch.cuda.current_stream(device)
        self.live = {}

        def _alloc(nbytes, ctx):
            try:
                p = torch.cuda.caching_allocator_alloc(nbytes, device,
                                                       self.stream)
            except Exception:
                return None
            self.live[p] = nbytes
            return p

        def _free(ptr, nbytes, ctx):
            if ptr in self.live:
                del self.live[ptr]
                torch.cuda.caching_allocator_delete(ptr)

        self.alloc_fn = ALLOC_FN(_alloc)
        self.free_fn = FREE_FN(_free)


def make_runtime(use_torch: bool = True, device: int = 0, tile=(0, 0),
                 sort_every: int = 0):
    rt = sfpic_runtime()
    rt.device = device
    rt.tile_x, rt.tile_y = tile
    rt.sort_every = sort_every
    keep = None
    if use_torch:
        try:
            import torch
            ok = torch.cuda.is_available()
        except Exception:
            ok = False
        if ok:
            keep = _TorchMemory(device)
            rt.stream = keep.stream.cuda_stream
            rt.alloc = keep.alloc_fn
            rt.free = keep.free_fn
    return rt, keep


def _grid_struct(g) -> sfpic_grid:
    s = sfpic_grid()
    s.dims, s.nx, s.ny = int(g.dims), int(g.nx), int(g.ny)
    s.dx, s.dy, s.dt = float(g.dx), float(g.dy), float(g.dt)
    return s


def _incident_struct(inc) -> sfpic_incident:
    s = sfpic_incident()
    for f, _ in sfpic_incident._fields_:
        if hasattr(inc, f):
            setattr(s, f, getattr(inc, f))
    return s


class Simulation:
    """One simulation held by the library (owns the sfpic_sim handle)."""

    def __init__(self, grid, incident, species: Sequence = (),
                 explicit: Optional[Sequence] = None, precision: int = FP64,
                 use_torch: bool = True, device: int = 0, tile=(0, 0),
                 sort_every: int = 0):
        """species: workloads.Species list (generated on the device), or
        explicit: list of dicts {q, m, weight, x, y, ux, uy, uz}."""
        L = lib()
        self.grid = grid
        self.precision = precision
        self._rt, self._mem = make_runtime(use_torch, device, tile, sort_every)
        self._keep = []
        arr = []
        if explicit is not None:
            for e in explicit:
                sp = sfpic_species()
                sp.q, sp.m = e["q"], e["m"]
                sp.weight = e["weight"]
                cols = [np.ascontiguousarray(e[k], dtype=np.float64)
                        for k in ("x", "y", "ux", "uy", "uz")]
                self._keep += cols
                sp.n_explicit = len(cols[0])
                sp.x, sp.y, sp.ux, sp.uy, sp.uz = [_dp(c) for c in cols]
                arr.append(sp)
        else:
            for k, spec in enumerate(species):
                sp = sfpic_species()
                sp.q, sp.m, sp.density = spec.q, spec.m, spec.density
                for i in range(4):
                    sp.region[i] = int(spec.region[i])
                sp.ppc = spec.ppc
                sp.temperature_ev = spec.temperature_ev
                sp.seed = spec.seed
                sp.species_index = spec.species_index
                arr.append(sp)
        self.nspecies = len(arr)
        sp_arr = (sfpic_species * max(1, len(arr)))(*arr)
        g = _grid_struct(grid)
        inc = _incident_struct(incident)
        h = C.c_void_p()
        _check(L.sfpic_create(C.byref(g), sp_arr, len(arr), C.byref(inc),
                              precision, C.byref(self._rt), C.byref(h)))
        self._keep = []
        self.h = h
        self.NX = int(grid.nx) + 2 * GUARD
        self.NY = int(grid.ny) + 2 * GUARD if grid.dims == 2 else 1

    @classmethod
    def from_workload(cls, wl, **kw):
        return cls(wl.grid, wl.incident, species=wl.species,
                   precision=wl.precision, **kw)

    def close(self):
        if getattr(self, "h", None):
            lib().sfpic_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        _check(lib().sfpic_step(self.h, int(n)))

    def sync(self):
        _check(lib().sfpic_sync(self.h))

    def read_field(self, comp) -> np.ndarray:
        c = COMP[comp] if isinstance(comp, str) else int(comp)
        out = np.empty((self.NY, self.NX))
        _check(lib().sfpic_read_field(self.h, c, _dp(out), out.size))
        return out

    def write_field(self, comp, arr):
        c = COMP[comp] if isinstance(comp, str) else int(comp)
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(self.NY,
                                                                self.NX)
        _check(lib().sfpic_write_field(self.h, c, _dp(a), a.size))

    def set_step_index(self, n):
        _check(lib().sfpic_set_step_index(self.h, int(n)))

    def particle_count(self, sp=0) -> int:
        n = C.c_int64()
        _check(lib().sfpic_particle_count(self.h, sp, C.byref(n)))
        return n.value

    def particles(self, sp=0):
        """(x, y, ux, uy, uz, id) of the live particles, in device order."""
        n = self.particle_count(sp)
        cols = [np.empty(n) for _ in range(5)]
        ids = np.empty(n, dtype=np.uint32)
        got = C.c_size_t()
        _check(lib().sfpic_read_particles(
            self.h, sp, *[_dp(c) for c in cols],
            ids.ctypes.data_as(C.POINTER(C.c_uint32)), n, C.byref(got)))
        return (*cols, ids)

    def diagnostics(self) -> dict:
        d = sfpic_diag()
        _check(lib().sfpic_diagnostics(self.h, C.byref(d)))
        return {f: getattr(d, f) for f, _ in sfpic_diag._fields_}

    def histogram(self, sp=0, n_e=256, emax=1.0, n_theta=180,
                  ek_min=1.0e3 / 510998.95):
        spec = sfpic_hist_spec(sp, n_e, emax, n_theta, ek_min)
        out = np.empty((n_e, n_theta))
        mom = np.empty(5)
        _check(lib().sfpic_histogram(self.h, C.byref(spec), _dp(out),
                                     out.size, _dp(mom)))
        return out, mom

    def profile(self, enable=True):
        _check(lib().sfpic_profile(self.h, 1 if enable else 0))

    def profile_read(self) -> dict:
        st = sfpic_kernel_stats()
        _check(lib().sfpic_profile_read(self.h, C.byref(st)))
        return {k: (st.launches[i], st.total_ms[i])
                for i, k in enumerate(KCLASSES)}

    def get_state(self) -> bytes:
        n = C.c_size_t()
        _check(lib().sfpic_get_state(self.h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib().sfpic_get_state(self.h, buf, C.byref(n)))
        return buf.raw[:n.value]

    def set_state(self, state: bytes):
        buf = C.create_string_buffer(state, len(state))
        _check(lib().sfpic_set_state(self.h, buf, len(state)))
