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
# SFPIC_LIB names another build of the same library (e.g. a variant under
# test); the default is the in-tree build.
LIB_PATH = os.environ.get("SFPIC_LIB") or os.path.join(HERE, "libsfpic.so")

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
                ("uz", _DP),
                ("profile", C.c_int32), ("profile_center", C.c_double),
                ("profile_fwhm", C.c_double), ("profile_order", C.c_double),
                ("profile_xmin", C.c_double)]


class sfpic_incident(C.Structure):
    _fields_ = [("kind", C.c_int32), ("a0", C.c_double),
                ("fwhm_t", C.c_double), ("t0", C.c_double),
                ("w0", C.c_double), ("s", C.c_double), ("phi0", C.c_double),
                ("x_focus", C.c_double), ("y_focus", C.c_double),
                ("t_focus", C.c_double), ("on_nodes", C.c_int32),
                ("z_focus", C.c_double)]


class sfpic3_grid(C.Structure):
    _fields_ = [("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("dt", C.c_double)]


class sfpic3_species(C.Structure):
    _fields_ = [("q", C.c_double), ("m", C.c_double),
                ("density", C.c_double), ("region", C.c_int64 * 6),
                ("ppc", C.c_int32), ("temperature_ev", C.c_double),
                ("seed", C.c_uint64), ("species_index", C.c_int32),
                ("n_explicit", C.c_int64), ("weight", C.c_double),
                ("x", _DP), ("y", _DP), ("z", _DP), ("ux", _DP),
                ("uy", _DP), ("uz", _DP),
                ("profile", C.c_int32), ("profile_center", C.c_double),
                ("profile_fwhm", C.c_double), ("profile_order", C.c_double),
                ("profile_xmin", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)


class sfpic_runtime(C.Structure):
    _fields_ = [("stream", C.c_void_p), ("alloc", ALLOC_FN),
                ("free", FREE_FN), ("alloc_ctx", C.c_void_p),
                ("tile_x", C.c_int32), ("tile_y", C.c_int32),
                ("sort_every", C.c_int32), ("device", C.c_int32),
                ("flags", C.c_int32), ("item_particles", C.c_int32)]


RT_NO_GRAPH, RT_NO_AUTOTUNE = 1, 2


class sfpic_diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("time", C.c_double),
                ("n_alive", C.c_int64), ("w_kin", C.c_double),
                ("w_em", C.c_double), ("charge", C.c_double),
                ("gauss_residual", C.c_double), ("rho_max", C.c_double),
                ("nonfinite", C.c_int32), ("w_em_total", C.c_double),
                ("continuity_residual", C.c_double),
                ("rho_abs_max", C.c_double),
                ("continuity_steps", C.c_int64)]


class sfpic_hist_spec(C.Structure):
    _fields_ = [("species", C.c_int32), ("n_energy", C.c_int32),
                ("e_max", C.c_double), ("n_theta", C.c_int32),
                ("ek_min", C.c_double), ("plane", C.c_int32)]


ANGLE_POLAR, ANGLE_XZ, ANGLE_XY = 0, 1, 2


class sfpic_sim_desc(C.Structure):
    _fields_ = [("grid", sfpic_grid), ("species", C.POINTER(sfpic_species)),
                ("nspecies", C.c_int32), ("incident", sfpic_incident),
                ("precision", C.c_int), ("nsteps", C.c_int64),
                ("hist", sfpic_hist_spec)]


class sfpic_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("error", C.c_char * 128),
                ("diag", sfpic_diag), ("moments", C.c_double * 5),
                ("steps", C.c_int64), ("pushes", C.c_double),
                ("t_submit", C.c_double), ("t_start", C.c_double),
                ("t_done", C.c_double), ("device_bytes", C.c_size_t)]


MAX_GROUPS, MAX_CANDIDATES = 4, 32
_GI = C.c_int32 * MAX_GROUPS
_GC = (C.c_int32 * MAX_CANDIDATES) * MAX_GROUPS


class sfpic_batch_info(C.Structure):
    _fields_ = [("ngroups", C.c_int32), ("precision", _GI), ("dims", _GI),
                ("members", _GI), ("tile_x", _GI), ("tile_y", _GI),
                ("sort_every", _GI), ("tuned", _GI),
                ("push_workgroups", _GI), ("n_candidates", _GI),
                ("cand_tile_x", _GC), ("cand_tile_y", _GC),
                ("cand_sort_every", _GC),
                ("cand_ns_per_push", (C.c_double * MAX_CANDIDATES)
                 * MAX_GROUPS),
                ("run_ms", C.c_double), ("step_ms", C.c_double),
                ("pushes", C.c_double), ("graph_launches", C.c_int64)]


class sfpic_server_info(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64),
                ("completed", C.c_int64), ("failed", C.c_int64),
                ("queued", C.c_int64), ("running", C.c_int64),
                ("p50_s", C.c_double), ("p99_s", C.c_double),
                ("mean_s", C.c_double), ("max_s", C.c_double),
                ("pushes", C.c_double), ("busy_s", C.c_double),
                ("pushes_per_s", C.c_double), ("bytes_in_use", C.c_size_t),
                ("bytes_peak", C.c_size_t), ("budget", C.c_size_t),
                ("ticks", C.c_int64), ("max_running", C.c_int32)]


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 1, 2, 3, 4

_lib = None

# every symbol declared in include/sfpic.h
EXPORTS = ["sfpic_create", "sfpic_step", "sfpic_sync", "sfpic_read_field",
           "sfpic_write_field", "sfpic_read_total_field",
           "sfpic_set_step_index",
           "sfpic_particle_count", "sfpic_read_particles",
           "sfpic_diagnostics", "sfpic_histogram",
           "sfpic_histogram_noalloc", "sfpic_get_state",
           "sfpic_set_state", "sfpic_profile", "sfpic_profile_read",
           "sfpic_destroy", "sfpic_device_bytes", "sfpic_last_error",
           "sfpic_version", "sfpic_desc_footprint", "sfpic_batch_create",
           "sfpic_batch_run", "sfpic_batch_result", "sfpic_batch_member",
           "sfpic_batch_stats", "sfpic_batch_destroy", "sfpic_server_create",
           "sfpic_server_submit", "sfpic_server_poll", "sfpic_server_wait",
           "sfpic_server_result", "sfpic_server_histogram",
           "sfpic_server_stats", "sfpic_server_destroy",
           "sfpic_april_field", "sfpic_april_power",
           "sfpic3_create", "sfpic3_step", "sfpic3_sync", "sfpic3_dims",
           "sfpic3_read_field", "sfpic3_write_field",
           "sfpic3_read_total_field",
           "sfpic3_particle_count", "sfpic3_read_particles",
           "sfpic3_diagnostics", "sfpic3_histogram", "sfpic3_get_state",
           "sfpic3_set_state", "sfpic3_destroy"]

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
    L.sfpic_read_total_field.argtypes = [vp, C.c_int, _DP, sz]
    L.sfpic_set_step_index.argtypes = [vp, i64]
    L.sfpic_particle_count.argtypes = [vp, C.c_int, C.POINTER(i64)]
    L.sfpic_read_particles.argtypes = [vp, C.c_int, _DP, _DP, _DP, _DP, _DP,
                                       C.POINTER(C.c_uint32), sz,
                                       C.POINTER(sz)]
    L.sfpic_diagnostics.argtypes = [vp, C.POINTER(sfpic_diag)]
    L.sfpic_histogram.argtypes = [vp, C.POINTER(sfpic_hist_spec), _DP, sz,
                                  _DP]
    L.sfpic_histogram_noalloc.argtypes = [vp, C.POINTER(sfpic_hist_spec),
                                          _DP, sz, _DP]
    L.sfpic_get_state.argtypes = [vp, vp, C.POINTER(sz)]
    L.sfpic_set_state.argtypes = [vp, vp, sz]
    L.sfpic_profile.argtypes = [vp, C.c_int]
    L.sfpic_profile_read.argtypes = [vp, C.POINTER(sfpic_kernel_stats)]
    L.sfpic_destroy.argtypes = [vp]
    L.sfpic_destroy.restype = None
    L.sfpic_device_bytes.argtypes = [vp, C.POINTER(sz)]
    L.sfpic3_create.argtypes = [C.POINTER(sfpic3_grid),
                                C.POINTER(sfpic3_species), C.c_int,
                                C.POINTER(sfpic_incident), C.c_int,
                                C.POINTER(sfpic_runtime), C.POINTER(vp)]
    L.sfpic3_step.argtypes = [vp, i64]
    L.sfpic3_sync.argtypes = [vp]
    L.sfpic3_dims.argtypes = [vp, C.POINTER(i64)]
    L.sfpic3_read_field.argtypes = [vp, C.c_int, _DP, sz]
    L.sfpic3_write_field.argtypes = [vp, C.c_int, _DP, sz]
    L.sfpic3_read_total_field.argtypes = [vp, C.c_int, _DP, sz]
    L.sfpic3_particle_count.argtypes = [vp, C.c_int, C.POINTER(i64)]
    L.sfpic3_read_particles.argtypes = [vp, C.c_int] + [_DP] * 6 + \
        [C.POINTER(C.c_uint8), sz]
    L.sfpic3_diagnostics.argtypes = [vp, C.POINTER(sfpic_diag)]
    L.sfpic3_histogram.argtypes = [vp, C.POINTER(sfpic_hist_spec), _DP, sz,
                                   _DP]
    L.sfpic3_get_state.argtypes = [vp, vp, C.POINTER(sz)]
    L.sfpic3_set_state.argtypes = [vp, vp, sz]
    L.sfpic3_destroy.argtypes = [vp]
    L.sfpic3_destroy.restype = None
    L.sfpic_april_field.argtypes = [C.POINTER(sfpic_incident), C.c_double,
                                    C.c_double, C.c_double, C.c_double, _DP]
    L.sfpic_april_power.argtypes = [C.POINTER(sfpic_incident),
                                    C.POINTER(C.c_double)]
    L.sfpic_last_error.restype = C.c_char_p
    L.sfpic_last_error.argtypes = [C.c_void_p]
    L.sfpic_version.restype = C.c_char_p
    D = C.POINTER(sfpic_sim_desc)
    RT = C.POINTER(sfpic_runtime)
    L.sfpic_desc_footprint.argtypes = [D, RT, C.POINTER(sz)]
    L.sfpic_batch_create.argtypes = [C.c_int, D, RT, C.POINTER(vp)]
    L.sfpic_batch_run.argtypes = [vp]
    L.sfpic_batch_result.argtypes = [vp, C.c_int, C.POINTER(sfpic_result)]
    L.sfpic_batch_member.argtypes = [vp, C.c_int, C.POINTER(vp)]
    L.sfpic_batch_stats.argtypes = [vp, C.POINTER(sfpic_batch_info)]
    L.sfpic_batch_destroy.argtypes = [vp]
    L.sfpic_batch_destroy.restype = None
    L.sfpic_server_create.argtypes = [sz, C.c_int, RT, C.POINTER(vp)]
    L.sfpic_server_submit.argtypes = [vp, D, C.POINTER(C.c_uint64)]
    L.sfpic_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(C.c_int)]
    L.sfpic_server_wait.argtypes = [vp, C.c_uint64, C.c_double]
    L.sfpic_server_result.argtypes = [vp, C.c_uint64,
                                      C.POINTER(sfpic_result)]
    L.sfpic_server_histogram.argtypes = [vp, C.c_uint64, _DP, sz]
    L.sfpic_server_stats.argtypes = [vp, C.POINTER(sfpic_server_info)]
    L.sfpic_server_destroy.argtypes = [vp]
    L.sfpic_server_destroy.restype = None
    _lib = L
    return L


def _check(code):
    if code != SFPIC_OK:
        raise SfpicError(code, lib().sfpic_last_error(None).decode())


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
                try:
                    torch.cuda.caching_allocator_delete(ptr)
                except Exception:  # interpreter shutdown: torch is gone
                    pass

        self.alloc_fn = ALLOC_FN(_alloc)
        self.free_fn = FREE_FN(_free)


def make_runtime(use_torch: bool = True, device: int = 0, tile=(0, 0),
                 sort_every: int = 0, flags: int = 0, item_particles: int = 0):
    rt = sfpic_runtime()
    rt.device = device
    rt.tile_x, rt.tile_y = tile
    rt.sort_every = sort_every
    rt.flags = flags
    rt.item_particles = item_particles
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


def april_field(inc, x, y, z, t):
    """Complex (E, cB) of an April incident at (x, y, z) from the focus and
    t from the focal time, paper axes, normalized units (two length-3
    complex arrays)."""
    out = np.zeros(12)
    _check(lib().sfpic_april_field(C.byref(_incident_struct(inc)), x, y, z, t,
                                   _dp(out)))
    v = out[0::2] + 1j * out[1::2]
    return v[:3], v[3:]


def april_power(inc) -> float:
    """Peak power of an April incident (focal plane, focal time, cycle
    average) in units of eps0 c (m_e c omega / e)^2 / k^2."""
    p = C.c_double()
    _check(lib().sfpic_april_power(C.byref(_incident_struct(inc)), C.byref(p)))
    return p.value


def _incident_struct(inc) -> sfpic_incident:
    s = sfpic_incident()
    for f, _ in sfpic_incident._fields_:
        if hasattr(inc, f):
            setattr(s, f, getattr(inc, f))
    return s


def _species_structs(species=(), explicit=None):
    """sfpic_species array from workloads.Species (generated on the device)
    or explicit dicts {q, m, weight, x, y, ux, uy, uz}; returns the array,
    its length and the numpy columns it points into (keep them alive)."""
    keep = []
    arr = []
    if explicit is not None:
        for e in explicit:
            sp = sfpic_species()
            sp.q, sp.m = e["q"], e["m"]
            sp.weight = e["weight"]
            cols = [np.ascontiguousarray(e[k], dtype=np.float64)
                    for k in ("x", "y", "ux", "uy", "uz")]
            keep += cols
            sp.n_explicit = len(cols[0])
            sp.x, sp.y, sp.ux, sp.uy, sp.uz = [_dp(c) for c in cols]
            arr.append(sp)
    else:
        for spec in species:
            sp = sfpic_species()
            sp.q, sp.m, sp.density = spec.q, spec.m, spec.density
            for i in range(4):
                sp.region[i] = int(spec.region[i])
            sp.ppc = spec.ppc
            sp.temperature_ev = spec.temperature_ev
            sp.seed = spec.seed
            sp.species_index = spec.species_index
            _set_profile(sp, spec)
            arr.append(sp)
    return (sfpic_species * max(1, len(arr)))(*arr), len(arr), keep


def _set_profile(sp, spec):
    """Copy a workloads species' density profile (if any) into a struct."""
    sp.profile = int(getattr(spec, "profile", 0))
    for f in ("center", "fwhm", "order", "xmin"):
        setattr(sp, "profile_" + f, float(getattr(spec, "profile_" + f, 0.0)))


def hist_spec(sp=0, n_e=256, emax=1.0, n_theta=180,
              ek_min=1.0e3 / 510998.95, plane=ANGLE_POLAR) -> sfpic_hist_spec:
    """Energy-angle histogram: n_e energy bins over [0, emax) m_e c^2,
    n_theta one-degree bins of the angle `plane` selects (ANGLE_*), moments
    over E_k > ek_min (default 1 keV)."""
    return sfpic_hist_spec(sp, n_e, emax, n_theta, ek_min, plane)


class SimDesc:
    """sfpic_sim_desc of a workload (keeps the arrays it points into)."""

    def __init__(self, wl, nsteps=None, hist=None, explicit=None,
                 precision=None):
        arr, n, keep = _species_structs(wl.species if explicit is None
                                        else (), explicit)
        self._keep = (arr, keep)
        d = sfpic_sim_desc()
        d.grid = _grid_struct(wl.grid)
        d.species = C.cast(arr, C.POINTER(sfpic_species))
        d.nspecies = n
        d.incident = _incident_struct(wl.incident)
        d.precision = wl.precision if precision is None else precision
        d.nsteps = wl.steps if nsteps is None else int(nsteps)
        if hist is not None:
            d.hist = hist
        self.desc = d
        self.workload = wl

    def footprint(self, tile=(0, 0)) -> int:
        rt = make_runtime(False, 0, tile)[0]
        n = C.c_size_t()
        _check(lib().sfpic_desc_footprint(C.byref(self.desc), C.byref(rt),
                                          C.byref(n)))
        return n.value


def _result_dict(r: sfpic_result) -> dict:
    return {"status": r.status, "error": r.error.decode(errors="replace"),
            "diag": {f: getattr(r.diag, f) for f, _ in sfpic_diag._fields_},
            "moments": list(r.moments), "steps": r.steps,
            "pushes": r.pushes, "t_submit": r.t_submit,
            "t_start": r.t_start, "t_done": r.t_done,
            "device_bytes": r.device_bytes}


class Simulation:
    """One simulation held by the library (owns the sfpic_sim handle)."""

    def __init__(self, grid, incident, species: Sequence = (),
                 explicit: Optional[Sequence] = None, precision: int = FP64,
                 use_torch: bool = True, device: int = 0, tile=(0, 0),
                 sort_every: int = 0, item_particles: int = 0):
        """species: workloads.Species list (generated on the device), or
        explicit: list of dicts {q, m, weight, x, y, ux, uy, uz}."""
        L = lib()
        self.grid = grid
        self.precision = precision
        self._borrowed = False
        self._rt, self._mem = make_runtime(use_torch, device, tile, sort_every,
                                           item_particles=item_particles)
        sp_arr, n, keep = _species_structs(species, explicit)
        self.nspecies = n
        g = _grid_struct(grid)
        inc = _incident_struct(incident)
        h = C.c_void_p()
        _check(L.sfpic_create(C.byref(g), sp_arr, n, C.byref(inc),
                              precision, C.byref(self._rt), C.byref(h)))
        del keep
        self.h = h
        self.NX = int(grid.nx) + 2 * GUARD
        self.NY = int(grid.ny) + 2 * GUARD if grid.dims == 2 else 1

    @classmethod
    def _borrow(cls, handle, grid, precision, nspecies, owner):
        """View of a sim owned by a batch (never destroyed from here)."""
        self = object.__new__(cls)
        self.grid = grid
        self.precision = precision
        self.nspecies = nspecies
        self._borrowed = True
        self._owner = owner
        self.h = handle
        self.NX = int(grid.nx) + 2 * GUARD
        self.NY = int(grid.ny) + 2 * GUARD if grid.dims == 2 else 1
        return self

    @classmethod
    def from_workload(cls, wl, **kw):
        return cls(wl.grid, wl.incident, species=wl.species,
                   precision=wl.precision, **kw)

    def close(self):
        if getattr(self, "h", None) and not getattr(self, "_borrowed", False):
            lib().sfpic_destroy(self.h)
        self.h = None

    def device_bytes(self) -> int:
        n = C.c_size_t()
        _check(lib().sfpic_device_bytes(self.h, C.byref(n)))
        return n.value

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

    def read_total_field(self, comp) -> np.ndarray:
        """Scattered plus incident field of one E or B component at its Yee
        nodes (E at t^n, B at t^{n-1/2}), shape (NY, NX) with guards."""
        c = COMP[comp] if isinstance(comp, str) else int(comp)
        out = np.empty((self.NY, self.NX))
        _check(lib().sfpic_read_total_field(self.h, c, _dp(out), out.size))
        return out

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
                  ek_min=1.0e3 / 510998.95, plane=ANGLE_POLAR):
        spec = sfpic_hist_spec(sp, n_e, emax, n_theta, ek_min, plane)
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


class Batch:
    """Many simulations advanced together (sfpic_batch_*).  members: list of
    workloads.Workload; nsteps (default each workload's steps) may be one
    number or a list.  Memory comes from hipMalloc, work runs on the batch's
    own stream."""

    def __init__(self, members, nsteps=None, hist=None, device=0,
                 tile=(0, 0), sort_every=0, graph=True, autotune=True,
                 item_particles=0):
        L = lib()
        if not isinstance(nsteps, (list, tuple)):
            nsteps = [nsteps] * len(members)
        self.descs = [SimDesc(wl, n, hist) for wl, n in zip(members, nsteps)]
        arr = (sfpic_sim_desc * len(self.descs))(
            *[d.desc for d in self.descs])
        flags = (0 if graph else RT_NO_GRAPH) | (0 if autotune
                                                 else RT_NO_AUTOTUNE)
        self._rt, _ = make_runtime(False, device, tile, sort_every, flags,
                                   item_particles)
        h = C.c_void_p()
        _check(L.sfpic_batch_create(len(self.descs), arr, C.byref(self._rt),
                                    C.byref(h)))
        self.h = h
        self.n = len(self.descs)

    def run(self):
        _check(lib().sfpic_batch_run(self.h))

    def result(self, i) -> dict:
        r = sfpic_result()
        _check(lib().sfpic_batch_result(self.h, i, C.byref(r)))
        return _result_dict(r)

    def member(self, i) -> Simulation:
        h = C.c_void_p()
        _check(lib().sfpic_batch_member(self.h, i, C.byref(h)))
        wl = self.descs[i].workload
        return Simulation._borrow(h, wl.grid, self.descs[i].desc.precision,
                                  self.descs[i].desc.nspecies, self)

    def stats(self) -> dict:
        st = sfpic_batch_info()
        _check(lib().sfpic_batch_stats(self.h, C.byref(st)))
        groups = []
        for g in range(st.ngroups):
            nc = st.n_candidates[g]
            groups.append({
                "precision": st.precision[g], "dims": st.dims[g],
                "members": st.members[g],
                "tile": (st.tile_x[g], st.tile_y[g]),
                "sort_every": st.sort_every[g], "tuned": bool(st.tuned[g]),
                "push_workgroups": st.push_workgroups[g],
                "trials": [((st.cand_tile_x[g][k], st.cand_tile_y[g][k]),
                            st.cand_sort_every[g][k],
                            st.cand_ns_per_push[g][k]) for k in range(nc)]})
        return {"groups": groups, "run_ms": st.run_ms,
                "step_ms": st.step_ms, "pushes": st.pushes,
                "graph_launches": st.graph_launches}

    def close(self):
        if getattr(self, "h", None):
            lib().sfpic_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request loop on a library thread (sfpic_server_*)."""

    def __init__(self, budget_bytes=0, max_slots=64, device=0, tile=(0, 0),
                 sort_every=0, graph=True):
        L = lib()
        flags = 0 if graph else RT_NO_GRAPH
        self._rt, _ = make_runtime(False, device, tile, sort_every, flags)
        h = C.c_void_p()
        _check(L.sfpic_server_create(int(budget_bytes), int(max_slots),
                                     C.byref(self._rt), C.byref(h)))
        self.h = h
        self._descs = {}

    def submit(self, wl, nsteps=None, hist=None, explicit=None) -> int:
        d = SimDesc(wl, nsteps, hist, explicit)
        t = C.c_uint64()
        _check(lib().sfpic_server_submit(self.h, C.byref(d.desc),
                                         C.byref(t)))
        self._descs[t.value] = d.desc.hist
        return t.value

    def poll(self, ticket) -> int:
        s = C.c_int()
        _check(lib().sfpic_server_poll(self.h, ticket, C.byref(s)))
        return s.value

    def wait(self, ticket, timeout_s=600.0):
        _check(lib().sfpic_server_wait(self.h, ticket, float(timeout_s)))

    def result(self, ticket) -> dict:
        r = sfpic_result()
        _check(lib().sfpic_server_result(self.h, ticket, C.byref(r)))
        return _result_dict(r)

    def histogram(self, ticket) -> np.ndarray:
        h = self._descs[ticket]
        out = np.empty((h.n_energy, h.n_theta))
        _check(lib().sfpic_server_histogram(self.h, ticket, _dp(out),
                                            out.size))
        return out

    def stats(self) -> dict:
        st = sfpic_server_info()
        _check(lib().sfpic_server_stats(self.h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in sfpic_server_info._fields_}

    def close(self):
        if getattr(self, "h", None):
            lib().sfpic_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Simulation3:
    """One 3D3V simulation held by the library (sfpic3_*).  Field arrays are
    (NZ, NY, NX) as FP64 on the host; precision FP64, or FP32 (fields and
    momenta stored as float, arithmetic in FP64)."""

    def __init__(self, grid, incident, species: Sequence = (),
                 explicit: Optional[Sequence] = None, use_torch: bool = True,
                 device: int = 0, precision: int = FP64):
        """grid: nx, ny, nz, dx, dy, dz, dt.  species: objects with q, m,
        density, region (x0, x1, y0, y1, z0, z1), ppc, temperature_ev, seed
        (generated on the device, species index = position in the list);
        explicit: dicts {q, m, weight, x, y, z, ux, uy, uz}."""
        L = lib()
        self.grid = grid
        self._rt, self._mem = make_runtime(use_torch, device)
        keep = []
        arr = []
        for e in (explicit or ()):
            sp = sfpic3_species()
            sp.q, sp.m, sp.weight = e["q"], e["m"], e["weight"]
            cols = [np.ascontiguousarray(e[k], dtype=np.float64)
                    for k in ("x", "y", "z", "ux", "uy", "uz")]
            keep += cols
            sp.n_explicit = len(cols[0])
            sp.x, sp.y, sp.z, sp.ux, sp.uy, sp.uz = [_dp(c) for c in cols]
            arr.append(sp)
        for k, d in enumerate(species):
            sp = sfpic3_species()
            sp.q, sp.m, sp.density = d.q, d.m, d.density
            for a in range(6):
                sp.region[a] = int(d.region[a])
            sp.ppc = int(d.ppc)
            sp.temperature_ev = float(getattr(d, "temperature_ev", 0.0))
            sp.seed = int(getattr(d, "seed", 0))
            sp.species_index = k
            _set_profile(sp, d)
            arr.append(sp)
        n = len(arr)
        sp_arr = (sfpic3_species * max(n, 1))(*arr)
        g = sfpic3_grid()
        for f, _ in sfpic3_grid._fields_:
            setattr(g, f, getattr(grid, f))
        inc = _incident_struct(incident)
        h = C.c_void_p()
        _check(L.sfpic3_create(C.byref(g), sp_arr, n, C.byref(inc),
                               int(precision), C.byref(self._rt), C.byref(h)))
        self.precision = precision
        del keep
        self.h = h
        self.nspecies = n
        dims = (C.c_int64 * 3)()
        _check(L.sfpic3_dims(h, dims))
        self.shape = (int(dims[2]), int(dims[1]), int(dims[0]))

    def close(self):
        if getattr(self, "h", None):
            lib().sfpic3_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        _check(lib().sfpic3_step(self.h, int(n)))

    def sync(self):
        _check(lib().sfpic3_sync(self.h))

    def field(self, comp) -> np.ndarray:
        c = COMP[comp] if isinstance(comp, str) else int(comp)
        out = np.empty(self.shape)
        _check(lib().sfpic3_read_field(self.h, c, _dp(out), out.size))
        return out

    def write_field(self, comp, a):
        c = COMP[comp] if isinstance(comp, str) else int(comp)
        a = np.ascontiguousarray(a, dtype=np.float64)
        if a.shape != self.shape:
            raise ValueError(f"field must have shape {self.shape}")
        _check(lib().sfpic3_write_field(self.h, c, _dp(a), a.size))

    def total_field(self, comp) -> np.ndarray:
        """Scattered plus incident field of one E or B component at its Yee
        nodes (E at t^n, B at t^{n-1/2}), shape (NZ, NY, NX)."""
        c = COMP[comp] if isinstance(comp, str) else int(comp)
        out = np.empty(self.shape)
        _check(lib().sfpic3_read_total_field(self.h, c, _dp(out), out.size))
        return out

    # the single-simulation names, so helpers written for Simulation (for
    # example convergence.full_field_start) take a Simulation3 as well
    read_field = field
    read_total_field = total_field

    def particles(self, sp=0):
        """(x, y, z, ux, uy, uz, alive) of every slot in creation order."""
        n = C.c_int64()
        _check(lib().sfpic3_particle_count(self.h, sp, C.byref(n)))
        cols = [np.empty(n.value) for _ in range(6)]
        alive = np.empty(n.value, dtype=np.uint8)
        _check(lib().sfpic3_read_particles(
            self.h, sp, *[_dp(c) for c in cols],
            alive.ctypes.data_as(C.POINTER(C.c_uint8)), n.value))
        return (*cols, alive.astype(bool))

    def diagnostics(self) -> dict:
        d = sfpic_diag()
        _check(lib().sfpic3_diagnostics(self.h, C.byref(d)))
        return {f: getattr(d, f) for f, _ in sfpic_diag._fields_}

    def histogram(self, sp=0, n_e=256, emax=1.0, n_theta=180,
                  ek_min=1.0e3 / 510998.95, plane=ANGLE_POLAR):
        """(n_e, n_theta) energy-angle histogram of the angle `plane`
        selects (ANGLE_*) and its moments."""
        spec = sfpic_hist_spec(sp, n_e, emax, n_theta, ek_min, plane)
        out = np.empty((n_e, n_theta))
        mom = np.empty(5)
        _check(lib().sfpic3_histogram(self.h, C.byref(spec), _dp(out),
                                      out.size, _dp(mom)))
        return out, mom

    def get_state(self) -> bytes:
        """Checkpoint of the simulation (step, E, B, particles)."""
        n = C.c_size_t()
        _check(lib().sfpic3_get_state(self.h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib().sfpic3_get_state(self.h, buf, C.byref(n)))
        return buf.raw

    def set_state(self, state: bytes):
        buf = C.create_string_buffer(state, len(state))
        _check(lib().sfpic3_set_state(self.h, buf, len(state)))


def detector_spectra(hist, angle_deg=20.0, half_width_deg=1.0):
    """Electron energy spectra seen at `angle_deg` forward and backward
    (Secs. 4.2 and 4.3: 20 degrees, in the plane across the polarization,
    from a histogram with plane=ANGLE_XZ): the sums over the angle bins
    inside [angle - w, angle + w) and [180 - angle - w, 180 - angle + w),
    as two arrays over the energy bins.  The bin edges must fall on those
    limits (n_theta a multiple of 180 / w)."""
    n_t = hist.shape[1]
    width = 180.0 / n_t

    def cols(lo, hi):
        a, b = lo / width, hi / width
        if abs(a - round(a)) > 1e-9 or abs(b - round(b)) > 1e-9:
            raise ValueError("angle limits do not fall on bin edges")
        return slice(int(round(a)), int(round(b)))

    fwd = cols(angle_deg - half_width_deg, angle_deg + half_width_deg)
    back = cols(180.0 - angle_deg - half_width_deg,
                180.0 - angle_deg + half_width_deg)
    return hist[:, fwd].sum(axis=1), hist[:, back].sum(axis=1)
