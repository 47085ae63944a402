"""ctypes binding of libcpic.so (include/cpic.h): argument marshalling only.

Every step of the PIC cycle runs in the library's HIP kernels; this module
converts numpy arrays / torch tensors to pointers and back.  PyTorch provides
device memory (the library allocates through a torch-backed allocator) and
the stream.  Loading fails loudly when the built library is missing."""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcpic.so")

MAP_IDENTITY, MAP_SINUSOIDAL, MAP_POLAR_LOG, MAP_SPHERICAL_RZ, MAP_TABULATED = 0, 1, 2, 3, 4
PUSH_BORIS, PUSH_CYCLOTRONIC = 0, 1
BC_PERIODIC, BC_DIRICHLET, BC_NEUMANN, BC_FLOATING = 0, 1, 2, 3
PBC_PERIODIC, PBC_ABSORB, PBC_OUTFLOW = 0, 1, 2
SHAPE_B1, SHAPE_B2 = 1, 2
FP32, FP64 = 0, 1
MG_FCG, MG_VCYCLE, MG_BOXMG = 0, 1, 2
MOVER_NEWTON, MOVER_PC = 0, 1
FIELD_Q, FIELD_CHARGE, FIELD_PHI, FIELD_EV, FIELD_JC, FIELD_RHO, FIELD_BACKGROUND = range(7)
(STAGE_SORT, STAGE_DEPOSIT, STAGE_CHARGE, STAGE_SOLVE, STAGE_EFIELD, STAGE_PUSH, STAGE_HALFSTEP,
 STAGE_INJECT) = range(8)

EXPORTED = ["cpic_create", "cpic_add_species", "cpic_set_particles", "cpic_get_particles",
            "cpic_initialize", "cpic_step", "cpic_run_stage", "cpic_get_field", "cpic_set_field",
            "cpic_field_bytes", "cpic_get_diag", "cpic_sync", "cpic_set_timing", "cpic_get_timing",
            "cpic_status_str", "cpic_last_error", "cpic_destroy", "cpic_set_graphs", "cpic_server_create",
            "cpic_server_submit", "cpic_server_pump", "cpic_server_poll", "cpic_server_get_stats",
            "cpic_server_destroy", "cpic_get_diag_noalloc", "cpic_step_batch",
            "cpic_batch_signature", "cpic_set_stream", "cpic_step_ready"]
MAX_SPECIES = 8
E_ARG, E_MAP, E_NOMEM, E_BUDGET, E_HIP, E_OVERFLOW, E_NONFINITE, E_STATE, E_UNSUPPORTED = range(-1, -10, -1)
E_PENDING = 1


class MapDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("dim", ctypes.c_int), ("L", ctypes.c_double * 3),
                ("eps", ctypes.c_double), ("r_in", ctypes.c_double), ("r_out", ctypes.c_double),
                ("omega", ctypes.c_int), ("vertices", ctypes.c_void_p)]


class GridDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("bc_lo", ctypes.c_int * 3), ("bc_hi", ctypes.c_int * 3),
                ("phi_lo", ctypes.c_double * 3), ("phi_hi", ctypes.c_double * 3),
                ("shape", ctypes.c_int), ("precision", ctypes.c_int), ("dt", ctypes.c_double),
                ("B0", ctypes.c_double * 3), ("background", ctypes.c_int),
                ("background_n0", ctypes.c_double), ("mg_rtol", ctypes.c_double),
                ("mg_max_cycles", ctypes.c_int), ("sort_every", ctypes.c_int),
                ("track_ids", ctypes.c_int), ("mg_method", ctypes.c_int), ("mover", ctypes.c_int),
                ("pusher", ctypes.c_int)]


class SpeciesDesc(ctypes.Structure):
    _fields_ = [("q", ctypes.c_double), ("m", ctypes.c_double), ("w", ctypes.c_double),
                ("pbc_lo", ctypes.c_int * 3), ("pbc_hi", ctypes.c_int * 3),
                ("capacity", ctypes.c_size_t), ("inject", ctypes.c_int),
                ("inject_n0", ctypes.c_double), ("inject_vth", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("inject_drift", ctypes.c_double)]


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)),
                ("free", ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)),
                ("ctx", ctypes.c_void_p)]


class Diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_longlong), ("kinetic", ctypes.c_double),
                ("field_energy", ctypes.c_double), ("mg_relres", ctypes.c_double),
                ("mg_cycles", ctypes.c_int), ("nspecies", ctypes.c_int),
                ("count", ctypes.c_longlong * 8), ("absorbed", ctypes.c_longlong * 8),
                ("outflow", ctypes.c_longlong * 8), ("qsum_lo", ctypes.c_uint64 * 8),
                ("qsum_hi", ctypes.c_uint64 * 8), ("newton_fallback", ctypes.c_longlong),
                ("far_deposits", ctypes.c_longlong), ("newton_failed", ctypes.c_longlong),
                ("injected", ctypes.c_longlong * 8), ("step_graphs", ctypes.c_int),
                ("sorts", ctypes.c_longlong * 8), ("phi_wall", ctypes.c_double),
                ("wall_charge", ctypes.c_double), ("inject_lost", ctypes.c_longlong * 8),
                ("batched_steps", ctypes.c_longlong)]


class CaseDesc(ctypes.Structure):
    _fields_ = [("map", MapDesc), ("grid", GridDesc), ("nspecies", ctypes.c_int),
                ("species", SpeciesDesc * MAX_SPECIES), ("count", ctypes.c_size_t * MAX_SPECIES),
                ("cell", ctypes.c_void_p * MAX_SPECIES), ("off", ctypes.c_void_p * MAX_SPECIES),
                ("vel", ctypes.c_void_p * MAX_SPECIES), ("nsteps", ctypes.c_int),
                ("phi_out", ctypes.c_void_p)]


class CaseResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("steps", ctypes.c_int), ("kinetic", ctypes.c_double),
                ("field_energy", ctypes.c_double), ("mg_relres", ctypes.c_double),
                ("nspecies", ctypes.c_int), ("count", ctypes.c_longlong * MAX_SPECIES),
                ("absorbed", ctypes.c_longlong * MAX_SPECIES),
                ("outflow", ctypes.c_longlong * MAX_SPECIES),
                ("injected", ctypes.c_longlong * MAX_SPECIES),
                ("qsum_lo", ctypes.c_uint64 * MAX_SPECIES), ("qsum_hi", ctypes.c_uint64 * MAX_SPECIES),
                ("pushes", ctypes.c_longlong), ("queue_ms", ctypes.c_double),
                ("service_ms", ctypes.c_double), ("step_p50_ms", ctypes.c_double),
                ("step_p99_ms", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_longlong), ("completed", ctypes.c_longlong),
                ("failed", ctypes.c_longlong), ("queued", ctypes.c_longlong),
                ("active", ctypes.c_longlong), ("peak_active", ctypes.c_longlong),
                ("budget_bytes", ctypes.c_size_t),
                ("used_bytes", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t),
                ("pushes", ctypes.c_longlong), ("step_samples", ctypes.c_longlong),
                ("step_p50_ms", ctypes.c_double), ("step_p99_ms", ctypes.c_double),
                ("batched_steps", ctypes.c_longlong)]


_lib = None


def load():
    """Load libcpic.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libcpic.so is not built: run python -m paper_1311_2286_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, vp, i32, sz = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    L.cpic_create.argtypes = [P(MapDesc), P(GridDesc), P(Allocator), vp, P(vp)]
    L.cpic_add_species.argtypes = [vp, P(SpeciesDesc), P(i32)]
    L.cpic_set_particles.argtypes = [vp, i32, sz, vp, vp, vp, vp, i32]
    L.cpic_get_particles.argtypes = [vp, i32, sz, vp, vp, vp, vp, P(sz), i32]
    L.cpic_initialize.argtypes = [vp]
    L.cpic_step.argtypes = [vp, i32]
    L.cpic_step_batch.argtypes = [P(vp), i32, P(i32)]
    L.cpic_batch_signature.argtypes = [vp, P(ctypes.c_uint64)]
    L.cpic_set_stream.argtypes = [vp, vp]
    L.cpic_step_ready.argtypes = [vp, P(i32)]
    L.cpic_run_stage.argtypes = [vp, i32]
    L.cpic_get_field.argtypes = [vp, i32, i32, vp, sz, i32]
    L.cpic_set_field.argtypes = [vp, i32, i32, vp, sz, i32]
    L.cpic_field_bytes.argtypes = [vp, i32]
    L.cpic_field_bytes.restype = sz
    L.cpic_get_diag.argtypes = [vp, P(Diag)]
    L.cpic_get_diag_noalloc.argtypes = [vp, P(Diag)]
    L.cpic_sync.argtypes = [vp]
    L.cpic_set_timing.argtypes = [vp, i32]
    L.cpic_get_timing.argtypes = [vp, i32, vp, vp, vp, vp, P(i32)]
    L.cpic_status_str.argtypes = [i32]
    L.cpic_status_str.restype = ctypes.c_char_p
    L.cpic_last_error.argtypes = [vp]
    L.cpic_last_error.restype = ctypes.c_char_p
    L.cpic_destroy.argtypes = [vp]
    L.cpic_destroy.restype = None
    L.cpic_set_graphs.argtypes = [vp, i32]
    L.cpic_server_create.argtypes = [sz, i32, P(Allocator), vp, P(vp)]
    L.cpic_server_submit.argtypes = [vp, P(CaseDesc), P(ctypes.c_uint64)]
    L.cpic_server_pump.argtypes = [vp, i32]
    L.cpic_server_poll.argtypes = [vp, ctypes.c_uint64, P(CaseResult)]
    L.cpic_server_get_stats.argtypes = [vp, P(ServerStats)]
    L.cpic_server_destroy.argtypes = [vp]
    L.cpic_server_destroy.restype = None
    for name in ("cpic_create", "cpic_add_species", "cpic_set_particles", "cpic_get_particles",
                 "cpic_initialize", "cpic_step", "cpic_step_batch", "cpic_batch_signature", "cpic_set_stream",
                 "cpic_step_ready", "cpic_run_stage", "cpic_get_field",
                 "cpic_set_field", "cpic_get_diag", "cpic_get_diag_noalloc", "cpic_sync", "cpic_set_timing",
                 "cpic_get_timing", "cpic_set_graphs", "cpic_server_create", "cpic_server_submit",
                 "cpic_server_pump", "cpic_server_poll", "cpic_server_get_stats"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


class CpicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (load().cpic_status_str(status).decode(), status, msg))
        self.status = status


class TorchAllocator:
    """Library memory from torch's caching allocator on the current device."""

    def __init__(self):
        import torch
        self._torch = torch
        self._live = {}
        self._alloc_cb = Allocator._fields_[0][1](self._alloc)
        self._free_cb = Allocator._fields_[1][1](self._free)
        self.struct = Allocator(self._alloc_cb, self._free_cb, None)

    def _alloc(self, nbytes, ctx):
        try:
            t = self._torch.empty(int(nbytes), dtype=self._torch.uint8, device="cuda")
        except Exception:
            return None
        p = t.data_ptr()
        self._live[p] = t
        return p

    def _free(self, ptr, ctx):
        self._live.pop(ptr, None)


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(ctypes.c_void_p)
    return ctypes.c_void_p(a.data_ptr())  # torch tensor


def _pad(t, v):
    return tuple(t)[:3] + (v,) * (3 - len(tuple(t)[:3]))


def make_map_desc(map_kind, dim, L=(1.0, 1.0, 1.0), eps=0.0, r_in=1.0, r_out=2.0, omega=0, vertices=None):
    """vertices: a tabulated map's (dim, nverts) float64 array; the caller keeps
    it alive until the descriptor has been used (cpic_create, or a server submit,
    which copies it)."""
    ptr = None
    if vertices is not None:
        assert vertices.dtype == np.float64 and vertices.flags["C_CONTIGUOUS"]
        ptr = vertices.ctypes.data
    return MapDesc(map_kind, dim, (ctypes.c_double * 3)(*_pad(L, 1.0)), eps, r_in, r_out, int(omega), ptr)


def make_grid_desc(n, bc_lo=(0, 0, 0), bc_hi=(0, 0, 0), phi_lo=(0.0, 0.0, 0.0),
                   phi_hi=(0.0, 0.0, 0.0), shape=SHAPE_B2, precision=FP32, dt=0.1,
                   B0=(0.0, 0.0, 0.0), background=False, background_n0=1.0, mg_rtol=1e-10,
                   mg_max_cycles=30, sort_every=1, track_ids=False, mg_method=0, mover=0, pusher=0):
    return GridDesc((ctypes.c_int * 3)(*_pad(n, 1)), (ctypes.c_int * 3)(*_pad(bc_lo, 0)),
                    (ctypes.c_int * 3)(*_pad(bc_hi, 0)), (ctypes.c_double * 3)(*_pad(phi_lo, 0.0)),
                    (ctypes.c_double * 3)(*_pad(phi_hi, 0.0)), shape, precision, dt,
                    (ctypes.c_double * 3)(*_pad(B0, 0.0)), int(background), background_n0,
                    mg_rtol, mg_max_cycles, sort_every, int(track_ids), int(mg_method), int(mover), int(pusher))


def make_species_desc(q, m, w, capacity=0, pbc_lo=(0, 0, 0), pbc_hi=(0, 0, 0), inject=None,
                      seed=0):
    inj = inject or {}
    return SpeciesDesc(q, m, w, (ctypes.c_int * 3)(*_pad(pbc_lo, 0)),
                       (ctypes.c_int * 3)(*_pad(pbc_hi, 0)), int(capacity),
                       int(inject is not None), float(inj.get("n0", 0.0)),
                       float(inj.get("vth", 0.0)), int(seed), float(inj.get("drift", 0.0)))


class Sim:
    """One simulation: a map, a grid, species and the PIC step (include/cpic.h)."""

    def __init__(self, map_kind, dim, n, L=(1.0, 1.0, 1.0), eps=0.0, r_in=1.0, r_out=2.0,
                 bc_lo=(0, 0, 0), bc_hi=(0, 0, 0), phi_lo=(0.0, 0.0, 0.0), phi_hi=(0.0, 0.0, 0.0),
                 shape=SHAPE_B2, precision=FP32, dt=0.1, B0=(0.0, 0.0, 0.0), background=False,
                 background_n0=1.0, mg_rtol=1e-10, mg_max_cycles=30, sort_every=1, track_ids=False,
                 stream=None, torch_alloc=True, mg_method=0, mover=0, omega=0, vertices=None, pusher=0):
        self.lib = load()
        pad = lambda t, v: tuple(t)[:3] + (v,) * (3 - len(tuple(t)[:3]))
        self.dim = dim
        self.n = tuple(n)[:dim]
        self.precision = precision
        self.rdtype = np.float64 if precision == FP64 else np.float32
        vtab = None
        if vertices is not None:  # tabulated map: (dim, nverts) vertex coordinates, read by cpic_create
            vtab = np.ascontiguousarray(vertices, dtype=np.float64)
        m = MapDesc(map_kind, dim, (ctypes.c_double * 3)(*pad(L, 1.0)), eps, r_in, r_out, int(omega),
                    vtab.ctypes.data if vtab is not None else None)
        g = GridDesc((ctypes.c_int * 3)(*pad(n, 1)), (ctypes.c_int * 3)(*pad(bc_lo, 0)),
                     (ctypes.c_int * 3)(*pad(bc_hi, 0)), (ctypes.c_double * 3)(*pad(phi_lo, 0.0)),
                     (ctypes.c_double * 3)(*pad(phi_hi, 0.0)), shape, precision, dt,
                     (ctypes.c_double * 3)(*pad(B0, 0.0)), int(background), background_n0,
                     mg_rtol, mg_max_cycles, sort_every, int(track_ids), int(mg_method), int(mover),
                     int(pusher))
        self._alloc = TorchAllocator() if torch_alloc else None
        if stream is None:
            try:
                import torch
                stream = torch.cuda.current_stream().cuda_stream
            except Exception:
                stream = 0
        self.stream = stream
        h = ctypes.c_void_p()
        st = self.lib.cpic_create(ctypes.byref(m), ctypes.byref(g),
                                  ctypes.byref(self._alloc.struct) if self._alloc else None,
                                  ctypes.c_void_p(stream), ctypes.byref(h))
        if st != 0:
            raise CpicError(st, "cpic_create")
        self.h = h
        self.nspecies = 0

    # ---------------------------------------------------------------- helpers
    def _check(self, st, what):
        if st != 0:
            raise CpicError(st, "%s: %s" % (what, self.lib.cpic_last_error(self.h).decode()))

    def close(self):
        if getattr(self, "h", None):
            self.lib.cpic_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ncells(self):
        return int(np.prod(self.n))

    # ---------------------------------------------------------------- species
    def add_species(self, q, m, w, capacity, pbc_lo=(0, 0, 0), pbc_hi=(0, 0, 0), inject=None,
                    seed=0):
        """inject: None or dict(n0=..., vth=...[, drift=...]) for flux injection at the
        outer wall (drift: speed along the inward normal)."""
        d = make_species_desc(q, m, w, capacity, pbc_lo, pbc_hi, inject, seed)
        sid = ctypes.c_int()
        self._check(self.lib.cpic_add_species(self.h, ctypes.byref(d), ctypes.byref(sid)),
                    "add_species")
        self.nspecies += 1
        return sid.value

    def set_particles(self, sid, cell, off, vel, ids=None):
        """cell int32 [n]; off [dim, n]; vel [3, n] (numpy on host or torch on device)."""
        on_dev = not isinstance(cell, np.ndarray)
        if on_dev:
            n = int(cell.numel())
        else:
            cell = np.ascontiguousarray(cell, dtype=np.int32)
            off = np.ascontiguousarray(off, dtype=self.rdtype)
            vel = np.ascontiguousarray(vel, dtype=self.rdtype)
            if ids is not None:
                ids = np.ascontiguousarray(ids, dtype=np.uint32)
            n = cell.size
        self._check(self.lib.cpic_set_particles(self.h, sid, n, _ptr(cell), _ptr(off), _ptr(vel),
                                                _ptr(ids), int(on_dev)), "set_particles")

    def get_particles(self, sid, cap=None):
        """All slots in use (see cpic_get_particles): the live particles and,
        until the species' next sort, those that left (cell -1 or -2)."""
        if cap is None:
            n = ctypes.c_size_t()
            st = self.lib.cpic_get_particles(self.h, sid, 0, None, None, None, None, ctypes.byref(n), 0)
            if st not in (0, -4):  # -4: the slot count came back in n
                self._check(st, "get_particles")
            cap = int(n.value)
        cell = np.zeros(max(cap, 1), dtype=np.int32)
        off = np.zeros((self.dim, max(cap, 1)), dtype=self.rdtype)
        vel = np.zeros((3, max(cap, 1)), dtype=self.rdtype)
        ids = np.zeros(max(cap, 1), dtype=np.uint32)
        n = ctypes.c_size_t()
        # arrays are [a][n] with stride n = cap: pass flat buffers sized for n live
        flat_off = np.zeros(self.dim * max(cap, 1), dtype=self.rdtype)
        flat_vel = np.zeros(3 * max(cap, 1), dtype=self.rdtype)
        self._check(self.lib.cpic_get_particles(self.h, sid, cap, _ptr(cell), _ptr(flat_off),
                                                _ptr(flat_vel), _ptr(ids), ctypes.byref(n), 0),
                    "get_particles")
        k = n.value
        off = flat_off[: self.dim * k].reshape(self.dim, k)
        vel = flat_vel[: 3 * k].reshape(3, k)
        return dict(cell=cell[:k], off=off, vel=vel, id=ids[:k])

    # ---------------------------------------------------------------- running
    def initialize(self):
        self._check(self.lib.cpic_initialize(self.h), "initialize")

    def step(self, nsteps=1):
        self._check(self.lib.cpic_step(self.h, nsteps), "step")

    def stage(self, stage):
        self._check(self.lib.cpic_run_stage(self.h, stage), "run_stage")

    def sync(self):
        self._check(self.lib.cpic_sync(self.h), "sync")

    # ---------------------------------------------------------------- fields
    def field_bytes(self, which):
        return int(self.lib.cpic_field_bytes(self.h, which))

    def get_field(self, which, sid=0):
        nb = self.field_bytes(which)
        if which == FIELD_Q:
            dt = np.float64 if self.precision == FP64 else np.uint64
        elif which == FIELD_EV:
            dt = self.rdtype
        else:
            dt = np.float64
        out = np.zeros(nb // np.dtype(dt).itemsize, dtype=dt)
        self._check(self.lib.cpic_get_field(self.h, which, sid, _ptr(out), nb, 0), "get_field")
        if which == FIELD_EV:
            ec = 4 if self.dim == 3 else 2
            out = out.reshape(-1, ec)
        return out

    def set_field(self, which, arr, sid=0):
        arr = np.ascontiguousarray(arr)
        self._check(self.lib.cpic_set_field(self.h, which, sid, _ptr(arr), arr.nbytes, 0),
                    "set_field")

    def diag(self):
        d = Diag()
        self._check(self.lib.cpic_get_diag(self.h, ctypes.byref(d)), "get_diag")
        return d

    def diag_noalloc(self):
        """cpic_get_diag_noalloc: the diagnostics computed in the library's
        per-device scratch array (allocates nothing)."""
        d = Diag()
        self._check(self.lib.cpic_get_diag_noalloc(self.h, ctypes.byref(d)), "get_diag_noalloc")
        return d

    def batch_signature(self):
        """0 when the field phase cannot be batched, else the value that
        simulations batchable together share (cpic_batch_signature)."""
        v = ctypes.c_uint64()
        self._check(self.lib.cpic_batch_signature(self.h, ctypes.byref(v)), "batch_signature")
        return int(v.value)

    def set_stream(self, stream):
        self._check(self.lib.cpic_set_stream(self.h, ctypes.c_void_p(stream)), "set_stream")
        self.stream = stream

    def step_ready(self):
        """True when the next step would not wait for the device."""
        r = ctypes.c_int(0)
        self._check(self.lib.cpic_step_ready(self.h, ctypes.byref(r)), "step_ready")
        return bool(r.value)

    def set_graphs(self, on=True):
        """Replay recorded HIP graphs of the step (needs a non-null stream)."""
        self._check(self.lib.cpic_set_graphs(self.h, int(on)), "set_graphs")

    def set_timing(self, on=True):
        self._check(self.lib.cpic_set_timing(self.h, int(on)), "set_timing")

    def get_timing(self, max_samples=100000):
        bufs = [np.zeros(max_samples) for _ in range(4)]
        n = ctypes.c_int()
        self._check(self.lib.cpic_get_timing(self.h, max_samples, *[_ptr(b) for b in bufs],
                                             ctypes.byref(n)), "get_timing")
        k = min(n.value, max_samples)
        return dict(push=bufs[0][:k], solve=bufs[1][:k], sort=bufs[2][:k], step=bufs[3][:k])


def step_batch(sims):
    """One step of each simulation, field phases batched (cpic_step_batch).
    Returns the per-case statuses; raises when any is an error."""
    sims = list(sims)
    arr = (ctypes.c_void_p * len(sims))(*[s.h for s in sims])
    status = (ctypes.c_int * len(sims))()
    st = load().cpic_step_batch(arr, len(sims), status)
    if st != 0:
        msgs = ["case %d: %d %s" % (i, status[i], s.lib.cpic_last_error(s.h).decode())
                for i, s in enumerate(sims) if status[i] != 0]
        raise CpicError(st, "step_batch: %s" % "; ".join(msgs))
    return list(status)


def qsum(d: Diag, sid: int) -> int:
    return int(d.qsum_lo[sid]) + (int(d.qsum_hi[sid]) << 64)


class Server:
    """The serving loop of include/cpic.h: cases admitted by slot and HBM
    budget, advanced one step per pump iteration on per-slot streams."""

    def __init__(self, budget_bytes, max_slots, torch_alloc=True, stream=None):
        self.lib = load()
        self._alloc = TorchAllocator() if torch_alloc else None
        self._keep = {}  # ticket -> host arrays that must outlive submit (phi_out)
        h = ctypes.c_void_p()
        st = self.lib.cpic_server_create(int(budget_bytes), int(max_slots),
                                         ctypes.byref(self._alloc.struct) if self._alloc else None,
                                         ctypes.c_void_p(stream) if stream else None, ctypes.byref(h))
        if st != 0:
            raise CpicError(st, "cpic_server_create")
        self.h = h

    def submit(self, map_desc, grid_desc, species, particles, nsteps, want_phi=False):
        """species: list of SpeciesDesc; particles: list of dicts cell [n], off [dim, n],
        vel [3, n] (numpy, the grid's precision).  Returns the ticket."""
        d = CaseDesc()
        d.map = map_desc
        d.grid = grid_desc
        d.nspecies = len(species)
        rdt = np.float64 if grid_desc.precision == FP64 else np.float32
        held = []
        for k, (sd, p) in enumerate(zip(species, particles)):
            d.species[k] = sd
            cell = np.ascontiguousarray(p["cell"], dtype=np.int32)
            off = np.ascontiguousarray(p["off"], dtype=rdt)
            vel = np.ascontiguousarray(p["vel"], dtype=rdt)
            held += [cell, off, vel]
            d.count[k] = cell.size
            d.cell[k] = cell.ctypes.data
            d.off[k] = off.ctypes.data
            d.vel[k] = vel.ctypes.data
        d.nsteps = int(nsteps)
        phi = None
        if want_phi:
            phi = np.zeros(int(np.prod(list(grid_desc.n)[: map_desc.dim])), dtype=np.float64)
            d.phi_out = phi.ctypes.data
        t = ctypes.c_uint64()
        st = self.lib.cpic_server_submit(self.h, ctypes.byref(d), ctypes.byref(t))
        if st != 0:
            raise CpicError(st, "cpic_server_submit")
        self._keep[t.value] = phi
        return t.value

    def pump(self, max_iterations=1):
        st = self.lib.cpic_server_pump(self.h, int(max_iterations))
        if st not in (0, E_PENDING):
            raise CpicError(st, "cpic_server_pump")
        return st == 0

    def poll(self, ticket):
        """None while pending, else a dict of the case result (phi when requested)."""
        r = CaseResult()
        st = self.lib.cpic_server_poll(self.h, ctypes.c_uint64(ticket), ctypes.byref(r))
        if st == E_PENDING:
            return None
        if st != 0:
            raise CpicError(st, "cpic_server_poll")
        out = {f: getattr(r, f) for f, _ in CaseResult._fields_}
        for f in ("count", "absorbed", "outflow", "injected", "qsum_lo", "qsum_hi"):
            out[f] = list(out[f])[: r.nspecies]
        out["phi"] = self._keep.get(ticket)
        return out

    def stats(self):
        s = ServerStats()
        st = self.lib.cpic_server_get_stats(self.h, ctypes.byref(s))
        if st != 0:
            raise CpicError(st, "cpic_server_get_stats")
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.lib.cpic_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
