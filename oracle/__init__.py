"""Plain FP64 CPU oracle for the curvilinear PIC hot path (arXiv:1311.2286).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code with
the HIP library and imports nothing from it; the two meet only through the
seeded input generators, which hold none of the method's arithmetic.

The arithmetic lives in ``oracle.c`` (plain loops, FP64, no FMA contraction);
this module is ctypes marshalling plus a few one-line numpy reductions
(charge per cell, energies) and ``OracleSim``, which strings the routines
together in the order of the PIC cycle (Sec. II: mover, particle-to-grid,
field solve, grid-to-particle).

Parity pins: every routine here is pinned by a test in ``tests/test_oracle_*``
against a closed form, an invariant, a brute-force evaluation or a value the
paper prints.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

IDENTITY, SINUSOIDAL, POLAR_LOG, SPHERICAL_RZ, TABULATED = 0, 1, 2, 3, 4
# FLOATING: a conducting wall of unknown potential at the lower face of axis 0
# whose charge is what the particles absorbed there (Gauss' law); handled by
# poisson_solve_floating and OracleSim, which pass the C routines a Dirichlet copy
PERIODIC, DIRICHLET, NEUMANN, FLOATING = 0, 1, 2, 3
B1, B2 = 1, 2


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (FP64, -ffp-contract=off, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
             "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Map(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("dim", ctypes.c_int), ("L", ctypes.c_double * 3),
                ("eps", ctypes.c_double), ("r_in", ctypes.c_double), ("r_out", ctypes.c_double),
                ("omega", ctypes.c_int), ("tn", ctypes.c_int * 3), ("tper", ctypes.c_int * 3),
                ("tx", ctypes.POINTER(ctypes.c_double))]


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("bc_lo", ctypes.c_int * 3),
                ("bc_hi", ctypes.c_int * 3), ("phi_lo", ctypes.c_double * 3),
                ("phi_hi", ctypes.c_double * 3)]


def make_map(kind, dim, L=(1.0, 1.0, 1.0), eps=0.0, r_in=1.0, r_out=2.0, omega=0) -> Map:
    L = tuple(L) + (1.0,) * (3 - len(L))
    return Map(kind, dim, (ctypes.c_double * 3)(*L), eps, r_in, r_out, omega)


def make_tabulated_map(dim, n, periodic, table, L=(1.0, 1.0, 1.0)) -> Map:
    """A map known at the cell vertices only: table[a] holds x^a at every
    vertex (vertex (i, j, k) at i + nv0 (j + nv1 k), nv_a = n_a on a periodic
    axis, n_a + 1 on a bounded one); on a periodic axis a the map continues as
    x(xi + e_a) = x(xi) + L_a e_a."""
    n = tuple(n)[:dim] + (1,) * (3 - dim)
    per = tuple(int(bool(p)) for p in periodic)[:dim] + (1,) * (3 - dim)
    tn = tuple((n[a] if per[a] else n[a] + 1) if a < dim else 1 for a in range(3))
    tab = np.ascontiguousarray(np.asarray(table, dtype=np.float64).reshape(dim, -1))
    assert tab.shape[1] == tn[0] * tn[1] * tn[2]
    L = tuple(L) + (1.0,) * (3 - len(L))
    m = Map(TABULATED, dim, (ctypes.c_double * 3)(*L), 0.0, 1.0, 2.0, 0, (ctypes.c_int * 3)(*tn),
            (ctypes.c_int * 3)(*per), tab.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    m._table = tab  # keeps the table alive while the map is
    return m


def sample_map_vertices(m: Map, n, periodic):
    """The analytic map m at the vertices of an n grid, as a tabulated map's
    table (shape (dim, nverts))."""
    dim = m.dim
    nv = [(n[a] if periodic[a] else n[a] + 1) for a in range(dim)]
    axes = [np.arange(nv[a]) / n[a] for a in range(dim)]
    G = np.meshgrid(*axes, indexing="ij")
    xi = np.zeros((int(np.prod(nv)), 3))
    for a in range(dim):
        xi[:, a] = G[a].ravel(order="F")
    x, _, _, _ = map_eval(m, xi)
    return np.ascontiguousarray(x[:, :dim].T)


def make_grid(n, bc_lo=(0, 0, 0), bc_hi=(0, 0, 0), phi_lo=(0.0, 0.0, 0.0),
              phi_hi=(0.0, 0.0, 0.0)) -> Grid:
    dim = len(n)
    nn = tuple(n) + (1,) * (3 - dim)
    f = lambda t, v: tuple(t) + (v,) * (3 - len(t))
    return Grid(dim, (ctypes.c_int * 3)(*nn), (ctypes.c_int * 3)(*f(bc_lo, 0)),
                (ctypes.c_int * 3)(*f(bc_hi, 0)), (ctypes.c_double * 3)(*f(phi_lo, 0.0)),
                (ctypes.c_double * 3)(*f(phi_hi, 0.0)))


_lib_handle = None


def lib():
    global _lib_handle
    if _lib_handle is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, i32, u64, u8, u32 = (ctypes.c_double, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint8,
                                ctypes.c_uint32)
        lg = ctypes.c_long
        L.or_map_eval.argtypes = [P(Map), lg, P(d), P(d), P(d), P(d), P(d)]
        L.or_coef_eval.argtypes = [P(Map), lg, P(d), P(d)]
        L.or_map_invert.argtypes = [P(Map), lg, P(d), P(d), P(d)]
        L.or_deposit_fixed.argtypes = [P(Grid), ctypes.c_int, ctypes.c_int, lg, P(i32), P(d),
                                       P(u8), P(u64)]
        L.or_deposit_fixed.restype = lg
        L.or_deposit_f64.argtypes = [P(Grid), ctypes.c_int, lg, P(i32), P(d), P(d)]
        L.or_deposit_f64.restype = lg
        L.or_gl8.argtypes = [P(d), P(d)]
        L.or_ion_background.argtypes = [P(Map), P(Grid), ctypes.c_int, d, P(d)]
        L.or_poisson_assemble.argtypes = [P(Map), P(Grid), P(d), P(d)]
        L.or_apply.argtypes = [P(Grid), P(d), P(d), P(d)]
        L.or_cg.argtypes = [P(Grid), P(d), P(d), P(d), d, ctypes.c_int, P(d)]
        L.or_poisson_solve.argtypes = [P(Map), P(Grid), P(d), P(d), d, ctypes.c_int, P(d)]
        L.or_efield.argtypes = [P(Map), P(Grid), P(d), P(d)]
        L.or_gather.argtypes = [P(Grid), P(d), lg, P(i32), P(d), P(d)]
        L.or_boris.argtypes = [lg, P(d), P(d), P(d), d, d]
        L.or_push.argtypes = [P(Map), P(Grid), d, d, P(d), lg, P(i32), P(d), P(d), P(d), P(lg)]
        L.or_push_cyclo.argtypes = [P(Map), P(Grid), d, d, P(d), lg, P(i32), P(d), P(d), P(d), P(lg)]
        L.or_cyclotronic.argtypes = [lg, P(d), P(d), P(d), d, d, P(d)]
        L.or_push_pc.argtypes = [P(Map), P(Grid), d, d, P(d), lg, P(i32), P(d), P(d), P(d),
                                 ctypes.c_int, P(lg)]
        L.or_philox4x32_10.argtypes = [P(u32), P(u32), P(u32)]
        L.or_num_threads.restype = ctypes.c_int
        L.or_face_area.argtypes = [P(Map)]
        L.or_face_area.restype = d
        L.or_inject.argtypes = [P(Map), P(Grid), d, d, d, d, d, u32, u32, u32, u32, lg, P(i32), P(d),
                                P(d), P(lg), P(lg)]
        L.or_drift_flux.argtypes = [d, d, d]
        L.or_drift_flux.restype = d
        L.or_wall_flux.argtypes = [P(Map), P(Grid), P(d), d]
        L.or_wall_flux.restype = d
        L.or_inject.restype = lg
        _lib_handle = L
    return _lib_handle


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _pts(a):
    """(n, d) or (n, 3) -> contiguous (n, 3) float64."""
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a[None, :]
    out = np.zeros((a.shape[0], 3))
    out[:, :a.shape[1]] = a
    return out


def ncells(g: Grid) -> int:
    return int(np.prod([g.n[a] for a in range(g.dim)]))


def nverts(g: Grid) -> int:
    return int(np.prod([g.n[a] if g.bc_lo[a] == PERIODIC else g.n[a] + 1 for a in range(g.dim)]))


# ---------------------------------------------------------------- maps
def map_eval(m: Map, xi):
    xi = _pts(xi)
    n = xi.shape[0]
    x = np.zeros((n, 3)); jac = np.zeros((n, 9)); k = np.zeros((n, 9)); J = np.zeros(n)
    lib().or_map_eval(ctypes.byref(m), n, _p(xi, ctypes.c_double), _p(x, ctypes.c_double),
                      _p(jac, ctypes.c_double), _p(k, ctypes.c_double), _p(J, ctypes.c_double))
    return x, jac.reshape(n, 3, 3), k.reshape(n, 3, 3), J


def coef_eval(m: Map, xi):
    xi = _pts(xi)
    n = xi.shape[0]
    a = np.zeros((n, 9))
    lib().or_coef_eval(ctypes.byref(m), n, _p(xi, ctypes.c_double), _p(a, ctypes.c_double))
    return a.reshape(n, 3, 3)


def map_invert(m: Map, x, xi_old=None):
    x = _pts(x)
    n = x.shape[0]
    xi = np.zeros((n, 3))
    xo = _pts(xi_old) if xi_old is not None else None
    lib().or_map_invert(ctypes.byref(m), n, _p(x, ctypes.c_double),
                        _p(xo, ctypes.c_double) if xo is not None else None,
                        _p(xi, ctypes.c_double))
    return xi


# ---------------------------------------------------------------- deposit
def deposit_fixed(g: Grid, shape: int, S1: int, cell, off, cell_mask=None):
    """Integer weights at scale 2^S1 per axis, summed exactly (uint64)."""
    cell = np.ascontiguousarray(cell, dtype=np.int32)
    off = _pts(off)
    Q = np.zeros(ncells(g), dtype=np.uint64)
    mask = None
    if cell_mask is not None:
        mask = np.ascontiguousarray(cell_mask, dtype=np.uint8)
    r = lib().or_deposit_fixed(ctypes.byref(g), shape, S1, cell.size, _p(cell, ctypes.c_int32),
                               _p(off, ctypes.c_double),
                               _p(mask, ctypes.c_uint8) if mask is not None else None,
                               _p(Q, ctypes.c_uint64))
    if r < 0:
        raise MemoryError("oracle deposit")
    return Q


def deposit_f64(g: Grid, shape: int, cell, off):
    cell = np.ascontiguousarray(cell, dtype=np.int32)
    off = _pts(off)
    Q = np.zeros(ncells(g))
    lib().or_deposit_f64(ctypes.byref(g), shape, cell.size, _p(cell, ctypes.c_int32),
                         _p(off, ctypes.c_double), _p(Q, ctypes.c_double))
    return Q


def gl8():
    x = np.zeros(8); w = np.zeros(8)
    lib().or_gl8(_p(x, ctypes.c_double), _p(w, ctypes.c_double))
    return x, w


def ion_background(m: Map, g: Grid, shape: int, n0: float = 1.0):
    I = np.zeros(ncells(g))
    rc = lib().or_ion_background(ctypes.byref(m), ctypes.byref(g), shape, n0, _p(I, ctypes.c_double))
    if rc:
        raise ValueError("ion background needs an all-periodic grid")
    return I


# ---------------------------------------------------------------- Poisson
def stencil_size(g: Grid) -> int:
    return 27 if g.dim == 3 else 9


def poisson_assemble(m: Map, g: Grid):
    nc = ncells(g)
    A = np.zeros((nc, stencil_size(g)))
    bd = np.zeros(nc)
    rc = lib().or_poisson_assemble(ctypes.byref(m), ctypes.byref(g), _p(A, ctypes.c_double),
                                   _p(bd, ctypes.c_double))
    if rc:
        raise ValueError("unsupported map/boundary combination (%d)" % rc)
    return A, bd


def apply(g: Grid, A, x):
    x = _f64(x)
    y = np.zeros(ncells(g))
    lib().or_apply(ctypes.byref(g), _p(A, ctypes.c_double), _p(x, ctypes.c_double),
                   _p(y, ctypes.c_double))
    return y


def cg(g: Grid, A, b, x0=None, rtol=1e-13, maxit=100000):
    b = _f64(b)
    x = np.zeros(ncells(g)) if x0 is None else _f64(x0).copy()
    rr = ctypes.c_double(0.0)
    it = lib().or_cg(ctypes.byref(g), _p(A, ctypes.c_double), _p(b, ctypes.c_double),
                     _p(x, ctypes.c_double), rtol, maxit, ctypes.byref(rr))
    return x, it, rr.value


def poisson_solve(m: Map, g: Grid, charge, phi0=None, rtol=1e-13, maxit=200000):
    """A phi = -charge - (wall terms); returns (phi, iterations, relative residual)."""
    charge = _f64(charge)
    phi = np.zeros(ncells(g)) if phi0 is None else _f64(phi0).copy()
    rr = ctypes.c_double(0.0)
    it = lib().or_poisson_solve(ctypes.byref(m), ctypes.byref(g), _p(charge, ctypes.c_double),
                                _p(phi, ctypes.c_double), rtol, maxit, ctypes.byref(rr))
    if it < 0:
        raise ValueError("unsupported map/boundary combination (%d)" % it)
    return phi, it, rr.value


def efield(m: Map, g: Grid, phi):
    phi = _f64(phi)
    Ev = np.zeros((nverts(g), 3))
    lib().or_efield(ctypes.byref(m), ctypes.byref(g), _p(phi, ctypes.c_double),
                    _p(Ev, ctypes.c_double))
    return Ev


# ---------------------------------------------------------------- particles
def gather(g: Grid, Ev, cell, off):
    cell = np.ascontiguousarray(cell, dtype=np.int32)
    off = _pts(off)
    Ev = _f64(Ev)
    Ep = np.zeros((cell.size, 3))
    lib().or_gather(ctypes.byref(g), _p(Ev, ctypes.c_double), cell.size, _p(cell, ctypes.c_int32),
                    _p(off, ctypes.c_double), _p(Ep, ctypes.c_double))
    return Ep


def boris(v, E, B, qm, dt):
    v = _pts(v).copy()
    E = _pts(E)
    Bv = _f64(np.asarray(B, dtype=np.float64).reshape(3))
    lib().or_boris(v.shape[0], _p(v, ctypes.c_double), _p(E, ctypes.c_double),
                   _p(Bv, ctypes.c_double), qm, dt)
    return v


def push(m: Map, g: Grid, qm, dt, B, cell, off, vel, Ev):
    """Gather + Boris + map inversion + boundaries, in place on copies.
    Returns (cell, off, vel, (absorbed, outflow))."""
    cell = np.ascontiguousarray(cell, dtype=np.int32).copy()
    off = _pts(off).copy()
    vel = _pts(vel).copy()
    Ev = _f64(Ev)
    Bv = _f64(np.asarray(B, dtype=np.float64).reshape(3))
    counts = (ctypes.c_long * 2)()
    lib().or_push(ctypes.byref(m), ctypes.byref(g), qm, dt, _p(Bv, ctypes.c_double), cell.size,
                  _p(cell, ctypes.c_int32), _p(off, ctypes.c_double), _p(vel, ctypes.c_double),
                  _p(Ev, ctypes.c_double), counts)
    return cell, off, vel, (counts[0], counts[1])


def push_cyclo(m: Map, g: Grid, qm, dt, B, cell, off, vel, Ev):
    """As ``push`` with the cyclotronic velocity step (electric impulse, then
    exact gyration in the uniform B; the position moves by dt times the mean
    velocity of the gyration)."""
    cell = np.ascontiguousarray(cell, dtype=np.int32).copy()
    off = _pts(off).copy()
    vel = _pts(vel).copy()
    Ev = _f64(Ev)
    Bv = _f64(np.asarray(B, dtype=np.float64).reshape(3))
    counts = (ctypes.c_long * 2)()
    lib().or_push_cyclo(ctypes.byref(m), ctypes.byref(g), qm, dt, _p(Bv, ctypes.c_double), cell.size,
                        _p(cell, ctypes.c_int32), _p(off, ctypes.c_double), _p(vel, ctypes.c_double),
                        _p(Ev, ctypes.c_double), counts)
    return cell, off, vel, (counts[0], counts[1])


def cyclotronic(v, E, B, qm, dt):
    """The cyclotronic velocity step alone: (new velocity, mean velocity)."""
    v = _pts(v).copy()
    E = _pts(E)
    Bv = _f64(np.asarray(B, dtype=np.float64).reshape(3))
    vm = np.zeros_like(v)
    lib().or_cyclotronic(v.shape[0], _p(v, ctypes.c_double), _p(E, ctypes.c_double), _p(Bv, ctypes.c_double),
                         qm, dt, _p(vm, ctypes.c_double))
    return v, vm


def push_pc(m: Map, g: Grid, qm, dt, B, cell, off, vel, Ev, kmode=0):
    """As ``push`` with the predictor-corrector position update (Eqs. step2-
    step4): k interpolated from the vertices (kmode 0, the paper's method) or
    evaluated from the map at the point (kmode 1)."""
    cell = np.ascontiguousarray(cell, dtype=np.int32).copy()
    off = _pts(off).copy()
    vel = _pts(vel).copy()
    Ev = _f64(Ev)
    Bv = _f64(np.asarray(B, dtype=np.float64).reshape(3))
    counts = (ctypes.c_long * 2)()
    lib().or_push_pc(ctypes.byref(m), ctypes.byref(g), qm, dt, _p(Bv, ctypes.c_double), cell.size,
                     _p(cell, ctypes.c_int32), _p(off, ctypes.c_double), _p(vel, ctypes.c_double),
                     _p(Ev, ctypes.c_double), int(kmode), counts)
    return cell, off, vel, (counts[0], counts[1])


def face_area(m: Map) -> float:
    return float(lib().or_face_area(ctypes.byref(m)))


def inject(m: Map, g: Grid, n0, vth, w, dt, seed, step, species, cap=1 << 20, with_index=False,
           drift=0.0):
    """Particles injected through the upper face of axis 0 in one step:
    (cell, off (n,3), vel (n,3), number drawn[, draw index of each particle]).
    Particles whose free-streaming start leaves the grid are not kept.  drift:
    speed of the Maxwellian's drift along the inward normal (0: at rest)."""
    cell = np.zeros(cap, dtype=np.int32)
    off = np.zeros((cap, 3))
    vel = np.zeros((cap, 3))
    kidx = np.zeros(cap, dtype=np.int64)
    drawn = ctypes.c_long(0)
    n = lib().or_inject(ctypes.byref(m), ctypes.byref(g), n0, vth, float(drift), w, dt, seed & 0xFFFFFFFF,
                        (seed >> 32) & 0xFFFFFFFF, step, species, cap, _p(cell, ctypes.c_int32),
                        _p(off, ctypes.c_double), _p(vel, ctypes.c_double),
                        _p(kidx, ctypes.c_long), ctypes.byref(drawn))
    out = (cell[:n].copy(), off[:n].copy(), vel[:n].copy(), drawn.value)
    if with_index:
        out = out + (kidx[:n].copy(),)
    return out


def drift_flux(n0, vth, s):
    """Inward flux of a Maxwellian drifting inward at s thermal speeds."""
    return float(lib().or_drift_flux(n0, vth, s))


def wall_flux(m: Map, g: Grid, phi, phib):
    """Discrete flux of E through the lower face of axis 0 held at phib."""
    return float(lib().or_wall_flux(ctypes.byref(m), ctypes.byref(g), _p(_f64(phi), ctypes.c_double), phib))


def _grid_with_wall(g: Grid, value, others_zero):
    """Copy of g with the lower face of axis 0 a Dirichlet wall at `value`
    (and, if others_zero, every other Dirichlet value 0)."""
    bl = list(g.bc_lo)
    bl[0] = DIRICHLET
    pl = [0.0] * 3 if others_zero else list(g.phi_lo)
    ph = [0.0] * 3 if others_zero else list(g.phi_hi)
    pl[0] = value
    return Grid(g.dim, (ctypes.c_int * 3)(*g.n), (ctypes.c_int * 3)(*bl), (ctypes.c_int * 3)(*g.bc_hi),
                (ctypes.c_double * 3)(*pl), (ctypes.c_double * 3)(*ph))


def poisson_solve_floating(m: Map, g: Grid, charge, Qw, phi0=None, phi1=None, rtol=1e-13):
    """Solve with a floating conducting wall at the lower face of axis 0 that
    holds charge Qw (Gauss' law: the flux of E through it equals Qw), by
    superposition: phi = phi_0 + phi_w phi_1, phi_0 the solution with the wall
    at 0, phi_1 the charge-free solution with the wall at 1 and every other
    wall at 0, phi_w = (Qw - F(phi_0)) / F(phi_1).  Returns (phi, phi_w,
    phi_0, phi_1); phi0/phi1 are initial guess and precomputed phi_1."""
    g0 = _grid_with_wall(g, 0.0, False)
    p0, _, _ = poisson_solve(m, g0, charge, phi0, rtol=rtol)
    if phi1 is None:
        g1 = _grid_with_wall(g, 1.0, True)
        phi1, _, _ = poisson_solve(m, g1, np.zeros(ncells(g)), rtol=rtol)
    F0 = wall_flux(m, g0, p0, 0.0)
    F1 = wall_flux(m, g, phi1, 1.0)
    pw = (Qw - F0) / F1
    return p0 + pw * phi1, pw, p0, phi1


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_num_threads(n: int) -> None:
    lib().or_set_num_threads(int(n))


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32), _p(o, ctypes.c_uint32))
    return o


# ---------------------------------------------------------------- grid sums
def charge_from_Q(Qs, species, dim, S1=None, background=None, bg_charge=1.0):
    """Charge per cell: sum_s q_s w_s Q_s (Q_s scaled by 2^-(d S1) when
    integer) plus the fixed background charge.  Eq. (pg) times J_c dV."""
    ch = None
    for Q, sp in zip(Qs, species):
        if Q.dtype == np.uint64:
            # exact integer -> FP64 conversion is a single rounding per cell
            qv = Q.astype(np.float64) * 2.0 ** (-dim * S1)
        else:
            qv = Q
        t = sp["q"] * sp["w"] * qv
        ch = t if ch is None else ch + t
    if background is not None:
        ch = ch + bg_charge * background
    return ch


def field_energy(charge, phi):
    """W_E = 1/2 sum_c (J rho dV)_c phi_c."""
    return 0.5 * float(np.dot(charge, phi))


class OracleSim:
    """The PIC cycle of Sec. II in leap-frog order: gather E^n -> v^{n+1/2} ->
    xi^{n+1} -> boundaries -> deposit -> charge -> phi^{n+1} -> E^{n+1}.

    species: list of dicts with q, m, w and arrays cell (int32), off (n,3),
    vel (n,3) in FP64.  deposit: 'fixed' (integer weights) or 'f64'.  mover:
    'exact' (map inversion) or 'pc' (predictor-corrector, Eqs. step2-step4).
    A FLOATING lower face of axis 0 holds the charge of the particles absorbed
    there (q w per particle, from the start) and floats at phi_wall."""

    def __init__(self, m: Map, g: Grid, species, shape=B2, dt=0.1, B=(0.0, 0.0, 0.0),
                 background=None, deposit="fixed", rtol=1e-13, ke_axes=3, mover="exact", pusher="boris"):
        self.m, self.g, self.sp = m, g, species
        self.shape, self.dt, self.B = shape, dt, np.asarray(B, dtype=np.float64)
        self.bg = background
        self.mode = deposit
        self.S1 = 24 if g.dim == 2 else 16
        self.rtol = rtol
        self.phi = np.zeros(ncells(g))
        self.step_count = 0
        self.ke = None
        self.ke_axes = ke_axes  # velocity components in the kinetic-energy sum
        self.mover = push_pc if mover == "pc" else push
        # cyclotronic: the velocity step resolves the gyration exactly (with the
        # exact position update); the kinetic energy is then that of the
        # velocity at t_n, v + (q/m) E dt / 2, and the initial push-back is the
        # half electric impulse alone
        self.cyclo = pusher == "cyclotronic"
        if self.cyclo:
            self.mover = push_cyclo
        self.floating = g.bc_lo[0] == FLOATING
        self.phi_wall = 0.0
        self.wall_charge = 0.0
        self.phi0 = None
        self.phi1 = None

    def deposit(self):
        if self.mode == "fixed":
            self.Q = [deposit_fixed(self.g, self.shape, self.S1, s["cell"], s["off"]) for s in self.sp]
        else:
            self.Q = [deposit_f64(self.g, self.shape, s["cell"], s["off"]) for s in self.sp]
        self.charge = charge_from_Q(self.Q, self.sp, self.g.dim, self.S1, self.bg)

    def solve(self):
        if self.floating:
            self.wall_charge = sum(s["q"] * s["w"] * s.get("absorbed", 0) for s in self.sp)
            self.phi, self.phi_wall, self.phi0, self.phi1 = poisson_solve_floating(
                self.m, self.g, self.charge, self.wall_charge, self.phi0, self.phi1, rtol=self.rtol)
            self.Ev = efield(self.m, _grid_with_wall(self.g, self.phi_wall, False), self.phi)
            return
        self.phi, self.cg_iters, self.relres = poisson_solve(self.m, self.g, self.charge, self.phi,
                                                             rtol=self.rtol)
        self.Ev = efield(self.m, self.g, self.phi)

    def initialize(self):
        """Deposit, solve, field; then the half-step push-back
        v^{-1/2} = Boris(v^0, E^0, B, -dt/2)."""
        self.deposit()
        self.solve()
        for s in self.sp:
            E = gather(self.g, self.Ev, s["cell"], s["off"])
            s["vel"] = boris(s["vel"], E, np.zeros(3) if self.cyclo else self.B, s["q"] / s["m"], -0.5 * self.dt)

    def step(self):
        ke = 0.0
        self.counts = []
        for s in self.sp:
            v_old = s["vel"].copy()
            if self.cyclo:
                Ep = gather(self.g, self.Ev, s["cell"], s["off"])
                v_mid = v_old + 0.5 * (s["q"] / s["m"]) * self.dt * Ep
            s["cell"], s["off"], s["vel"], cnt = self.mover(self.m, self.g, s["q"] / s["m"], self.dt,
                                                            self.B, s["cell"], s["off"], s["vel"], self.Ev)
            alive = s["cell"] >= 0
            k = self.ke_axes
            if self.cyclo:
                ke += 0.5 * s["m"] * s["w"] * float(np.sum(v_mid[alive, :k] ** 2))
            else:
                ke += 0.5 * s["m"] * s["w"] * float(np.sum(v_old[alive, :k] * s["vel"][alive, :k]))
            self.counts.append(cnt)
            # drop particles that left, then append this step's injection
            s["cell"], s["off"], s["vel"] = s["cell"][alive], s["off"][alive], s["vel"][alive]
            inj = s.get("inject")
            if inj is not None:
                c, o, v, _ = inject(self.m, self.g, inj["n0"], inj["vth"], s["w"], self.dt,
                                    inj["seed"], self.step_count, inj["sid"], drift=inj.get("drift", 0.0))
                s["cell"] = np.concatenate([s["cell"], c])
                s["off"] = np.concatenate([s["off"], o])
                s["vel"] = np.concatenate([s["vel"], v])
                s["injected"] = s.get("injected", 0) + c.size
            s["absorbed"] = s.get("absorbed", 0) + cnt[0]
            s["outflow"] = s.get("outflow", 0) + cnt[1]
        self.ke = ke
        self.deposit()
        self.solve()
        self.step_count += 1

    def field_energy(self):
        """1/2 sum charge phi, plus 1/2 Q_wall phi_wall with a floating wall."""
        return field_energy(self.charge, self.phi) + (0.5 * self.wall_charge * self.phi_wall
                                                      if self.floating else 0.0)
