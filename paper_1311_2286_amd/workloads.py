"""Seeded synthetic workloads: case parameters and particle / field generators.

This module is shared by the tests, the benchmark and the smoke check.  It
holds no step arithmetic of the method (no deposit, gather, push, map
inversion or field solve): it only states the workloads (grid, map, species,
time step) and draws seeded random inputs with the stated distributions.

Loading recipe (uniform plasma in *physical* space with equal macro-weights,
plus the small density perturbation of the Langmuir test): logical positions
are drawn with density proportional to the map's volume factor times
(1 + delta cos(2 pi x/L)).  For the sinusoidal map that factor is
1 + eps * sum_b d/dxi^b prod_k sin(2 pi xi^k) (box units), for the polar-log
map it is proportional to exp(2 xi ln(r_out/r_in)); both are written out below
as the target densities of the draw, by rejection (sinusoidal) or inverse CDF
(polar-log).  Velocities: Maxwellian, N(0, v_th^2) per component, three
components in 2D and 3D.

Random streams: numpy Generator(Philox) keyed by (seed, case, species, chunk),
so every chunk is reproducible on its own and chunks can be drawn in parallel.
"""
from __future__ import annotations

import dataclasses
import math
from concurrent.futures import ThreadPoolExecutor
from typing import List, Optional, Tuple

import numpy as np

IDENTITY, SINUSOIDAL, POLAR_LOG = 0, 1, 2  # map kinds (SPHERICAL_RZ below)
PERIODIC, DIRICHLET, NEUMANN, FLOATING = 0, 1, 2, 3
B1, B2 = 1, 2
FP32, FP64 = 0, 1
BASE_SEED = 1311

MASS_RATIO = 1836.0


@dataclasses.dataclass
class Species:
    name: str
    q: float
    m: float
    vth: float
    ppc: float  # macro-particles per cell of this species (mean)
    count: Optional[int] = None  # overrides ppc * ncells
    w: Optional[float] = None  # macro-weight, for species that start empty
    drift: float = 0.0  # injection: drift along the inward normal, in thermal speeds


@dataclasses.dataclass
class Case:
    name: str
    dim: int
    map_kind: int
    n: Tuple[int, ...]
    L: Tuple[float, ...] = (1.0, 1.0, 1.0)
    eps: float = 0.0
    r_in: float = 1.0
    r_out: float = 60.0
    bc_lo: Tuple[int, ...] = (0, 0, 0)
    bc_hi: Tuple[int, ...] = (0, 0, 0)
    phi_lo: Tuple[float, ...] = (0.0, 0.0, 0.0)
    phi_hi: Tuple[float, ...] = (0.0, 0.0, 0.0)
    dt: float = 0.1
    B: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    species: List[Species] = dataclasses.field(default_factory=list)
    background: bool = False  # fixed neutralising ion background (n0 = 1)
    delta: float = 0.0  # density perturbation amplitude, cos(2 pi x^1 / L_1)
    steps: int = 100
    case_id: int = 0
    # run on the map sampled at the vertices (a tabulated map) instead of the
    # analytic one; particles are still loaded from the analytic map's density
    tabulated: bool = False

    @property
    def ncells(self) -> int:
        return int(np.prod(self.n))

    def volume(self) -> float:
        if self.map_kind == POLAR_LOG:
            return math.pi * (self.r_out ** 2 - self.r_in ** 2)
        return float(np.prod(self.L[: self.dim]))

    def count(self, s: Species) -> int:
        if s.count is not None:
            return int(s.count)
        return int(round(s.ppc * self.ncells))

    def weight(self, s: Species) -> float:
        """Macro-weight w_s = n0 * volume / N_s (n0 = 1), unless given."""
        if s.w is not None:
            return s.w
        return self.volume() / self.count(s)

    def map_args(self):
        return dict(kind=self.map_kind, dim=self.dim, L=tuple(self.L) + (1.0,) * (3 - len(self.L)),
                    eps=self.eps, r_in=self.r_in, r_out=self.r_out)

    def grid_args(self):
        pad = lambda t, v: tuple(t[: self.dim]) + (v,) * (3 - self.dim)
        return dict(n=tuple(self.n), bc_lo=pad(self.bc_lo, 0), bc_hi=pad(self.bc_hi, 0),
                    phi_lo=pad(self.phi_lo, 0.0), phi_hi=pad(self.phi_hi, 0.0))


def vertex_table(case: Case) -> np.ndarray:
    """The case's analytic map at the logical vertices, as a tabulated map's
    vertex coordinates: shape (dim, nverts), vertex i + nv0 (j + nv1 k), nv_a =
    n_a on a periodic axis, n_a + 1 on a bounded one.  Closed forms: identity
    x = L xi; sinusoidal x^a = L_a (xi^a + eps prod_k sin(2 pi xi^k)); polar-log
    (r cos 2 pi eta, r sin 2 pi eta), r = r_in (r_out / r_in)^xi."""
    d = case.dim
    nv = [case.n[a] if case.bc_lo[a] == PERIODIC else case.n[a] + 1 for a in range(d)]
    axes = [np.arange(nv[a]) / case.n[a] for a in range(d)]
    G = [g.ravel() for g in np.meshgrid(*axes[::-1], indexing="ij")[::-1]]  # axis 0 fastest
    if case.map_kind == POLAR_LOG:
        r = case.r_in * (case.r_out / case.r_in) ** G[0]
        return np.stack([r * np.cos(2 * np.pi * G[1]), r * np.sin(2 * np.pi * G[1])])
    P = np.ones_like(G[0])
    if case.map_kind == SINUSOIDAL:
        for a in range(d):
            P = P * np.sin(2 * np.pi * G[a])
    eps = case.eps if case.map_kind == SINUSOIDAL else 0.0
    return np.stack([case.L[a] * (G[a] + eps * P) for a in range(d)])


def table_shift(case: Case) -> Tuple[float, ...]:
    """Shift of x^a per period of each axis of the tabulated map: the box
    length, or 0 for the polar angle (the map closes on itself)."""
    if case.map_kind == POLAR_LOG:
        return (1.0, 0.0)
    return tuple(case.L[: case.dim])


def electrons(vth=1.0, ppc=64.0, count=None):
    return Species("e", -1.0, 1.0, vth, ppc, count)


def ions(vth=1.0 / math.sqrt(MASS_RATIO), ppc=64.0, count=None):
    return Species("i", 1.0, MASS_RATIO, vth, ppc, count)


# ----------------------------------------------------------------------------
# The five workloads.  Where the paper leaves them open: the 3D boxes are N
# cells x 1 Debye length per axis, dt = 0.1 / omega_pe everywhere, and
# particles per cell count both species, split equally.
# ----------------------------------------------------------------------------
def case1(vth=1.0) -> Case:
    """2D periodic Langmuir test: unit square, sinusoidal map eps = 0.1,
    32x32 cells, 64 electrons/cell, fixed ion background, dn/n = 0.01."""
    return Case("langmuir2d", 2, SINUSOIDAL, (32, 32), L=(1.0, 1.0), eps=0.1, dt=0.1,
                species=[electrons(vth, 64.0)], background=True, delta=0.01, steps=200, case_id=1)


def case1_cold() -> Case:
    c = case1(vth=0.0)
    c.name = "langmuir2d_cold"
    return c


def case2() -> Case:
    """3D periodic box 128^3, sinusoidal map eps = 0.05 on all axes, 32 e + 32 i
    per cell (134M), m_i/m_e = 1836, T_i = T_e."""
    return Case("box3d_128", 3, SINUSOIDAL, (128, 128, 128), L=(128.0, 128.0, 128.0), eps=0.05,
                dt=0.1, species=[electrons(1.0, 32.0), ions(ppc=32.0)], delta=0.01, steps=100,
                case_id=2)


def case3() -> Case:
    """2D cylindrical probe: polar-log map r_in = 1, r_out = 60, 512x512 cells,
    100 e + 100 i per cell on average, probe at -5, outer boundary 0."""
    return Case("probe2d_512", 2, POLAR_LOG, (512, 512), r_in=1.0, r_out=60.0,
                bc_lo=(DIRICHLET, PERIODIC), bc_hi=(DIRICHLET, PERIODIC), phi_lo=(-5.0, 0.0),
                phi_hi=(0.0, 0.0), dt=0.1, species=[electrons(1.0, 100.0), ions(ppc=100.0)],
                steps=2000, case_id=3)


def case5() -> Case:
    """3D magnetised box 256x256x128, eps = 0.05, 16 e + 16 i per cell (268M),
    B = 2 z (omega_ce = 2)."""
    return Case("box3d_magnetized", 3, SINUSOIDAL, (256, 256, 128), L=(256.0, 256.0, 128.0),
                eps=0.05, dt=0.1, B=(0.0, 0.0, 2.0),
                species=[electrons(1.0, 16.0), ions(ppc=16.0)], delta=0.01, steps=100, case_id=5)


def planar_wall(n=128, ppc=64.0, case_id=6):
    """The paper's planar-wall test (Sec. "Tests", charging and shielding of a
    conducting planar wall): a 20 x 5 Debye-length box on the identity map,
    n x n cells, a floating absorbing wall at x = 0, phi = 0 and outflow at
    x = L_x, periodic in y; initially empty, filled by flux injection at
    x = L_x of electrons (Maxwellian at rest, v_th = 1) and ions (m_i/m_e = 1836,
    T_i = T_e, drifting toward the wall at 2.1 ion thermal speeds), source
    density 1; omega_pe dt = 0.05.  Macro-weight: ppc particles per cell per
    species at unit density."""
    L = (20.0, 5.0)
    w = L[0] * L[1] / (ppc * n * n)
    e = Species("e", -1.0, 1.0, 1.0, 0.0, count=0, w=w)
    i = Species("i", 1.0, MASS_RATIO, 1.0 / math.sqrt(MASS_RATIO), 0.0, count=0, w=w, drift=2.1)
    return Case("planar_wall_%d" % n, 2, IDENTITY, (n, n), L=L, bc_lo=(FLOATING, PERIODIC),
                bc_hi=(DIRICHLET, PERIODIC), dt=0.05, species=[e, i], steps=24000, case_id=case_id)


def small_case(dim=2, map_kind=SINUSOIDAL, n=None, eps=None, ppc=8.0, two_species=True,
               background=False, B=(0.0, 0.0, 0.0), L=None, dt=0.1, vth_e=1.0, case_id=100):
    """A reduced case with the structure of the workloads above, sized so the
    oracle finishes in seconds, with ragged (non-multiple-of-tile) grids."""
    if n is None:
        n = (40, 24) if dim == 2 else (20, 12, 16)
    if eps is None:
        eps = 0.1 if dim == 2 else 0.05
    if L is None:
        L = tuple(float(v) for v in n)
    sp = [electrons(vth_e, ppc)]
    if two_species:
        sp.append(ions(ppc=ppc))
    return Case("small%dd" % dim, dim, map_kind, tuple(n), L=L, eps=eps, dt=dt, B=B, species=sp,
                background=background, delta=0.01, steps=10, case_id=case_id)


# ----------------------------------------------------------------------------
# Target densities of the draw (see module docstring)
# ----------------------------------------------------------------------------
def _density_sinusoidal(xi: np.ndarray, eps: float, delta: float) -> np.ndarray:
    d = xi.shape[0]
    s = np.sin(2.0 * np.pi * xi)
    c = np.cos(2.0 * np.pi * xi)
    vol = np.ones(xi.shape[1])
    P = np.prod(s, axis=0)
    for b in range(d):
        t = 2.0 * np.pi * c[b]
        for k in range(d):
            if k != b:
                t = t * s[k]
        vol = vol + eps * t
    x1 = xi[0] + eps * P  # first physical coordinate over L_1
    return vol * (1.0 + delta * np.cos(2.0 * np.pi * x1))


def _density_bound(dim: int, eps: float, delta: float) -> float:
    m = 64 if dim == 3 else 256
    g = (np.arange(m) + 0.5) / m
    grids = np.meshgrid(*([g] * dim), indexing="ij")
    xi = np.stack([a.ravel() for a in grids])
    return float(_density_sinusoidal(xi, eps, 0.0).max()) * 1.02 * (1.0 + abs(delta))


def _rng(seed: int, case_id: int, sid: int, chunk: int, purpose: int = 0) -> np.random.Generator:
    key = np.array([seed, (case_id << 40) | (sid << 32) | (purpose << 24) | chunk], dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key))


def _draw_positions(case: Case, rng: np.random.Generator, n: int, bound: float) -> np.ndarray:
    d = case.dim
    if case.map_kind == POLAR_LOG:
        R2 = (case.r_out / case.r_in) ** 2
        u = rng.random(n)
        xi0 = np.log1p(u * (R2 - 1.0)) / np.log(R2)
        return np.stack([xi0, rng.random(n)])
    if case.map_kind == IDENTITY or (case.eps == 0.0 and case.delta == 0.0):
        return rng.random((d, n))
    out = np.empty((d, n))
    filled = 0
    while filled < n:
        m = int((n - filled) * 1.3) + 64
        xi = rng.random((d, m))
        dens = _density_sinusoidal(xi, case.eps, case.delta)
        if np.any(dens > bound):
            raise RuntimeError("density bound violated")
        acc = rng.random(m) * bound < dens
        take = xi[:, acc][:, : n - filled]
        out[:, filled: filled + take.shape[1]] = take
        filled += take.shape[1]
    return out


def _to_cell_offset(case: Case, xi: np.ndarray, dtype):
    d = case.dim
    n = np.asarray(case.n[:d], dtype=np.int64).reshape(d, 1)
    u = xi * n
    ci = np.floor(u).astype(np.int64)
    ci = np.minimum(ci, n - 1)
    off = (u - ci).astype(dtype)
    one_below = np.nextafter(dtype(1.0), dtype(0.0))
    off = np.minimum(off, one_below)
    off = np.maximum(off, dtype(0.0))
    lin = np.zeros(xi.shape[1], dtype=np.int64)
    for a in range(d - 1, -1, -1):
        lin = lin * case.n[a] + ci[a]
    return lin.astype(np.int32), off


CHUNK = 1 << 22


def generate_species(case: Case, sid: int, dtype=np.float32, count: Optional[int] = None,
                     seed: int = BASE_SEED, workers: int = 8):
    """Particles of species `sid`: dict(cell int32 [n], off dtype [d, n],
    vel dtype [3, n], id uint32 [n]).  `count` limits the draw to the first
    `count` particles of the same stream (a bounded sample of the workload)."""
    s = case.species[sid]
    ntot = case.count(s) if count is None else int(count)
    d = case.dim
    nchunks = (ntot + CHUNK - 1) // CHUNK
    cell = np.empty(ntot, dtype=np.int32)
    off = np.empty((d, ntot), dtype=dtype)
    vel = np.empty((3, ntot), dtype=dtype)
    bound = (_density_bound(d, case.eps, case.delta)
             if case.map_kind == SINUSOIDAL and (case.eps != 0.0 or case.delta != 0.0) else 1.0)

    def work(k):
        lo = k * CHUNK
        hi = min(ntot, lo + CHUNK)
        rng = _rng(seed, case.case_id, sid, k)
        xi = _draw_positions(case, rng, hi - lo, bound)
        c, o = _to_cell_offset(case, xi, dtype)
        cell[lo:hi] = c
        off[:, lo:hi] = o
        vel[:, lo:hi] = (rng.standard_normal((3, hi - lo)) * s.vth).astype(dtype)

    if nchunks <= 1 or workers <= 1:
        for k in range(nchunks):
            work(k)
    else:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(work, range(nchunks)))
    return dict(cell=cell, off=off, vel=vel, id=np.arange(ntot, dtype=np.uint32))


def as_dtype(p, dtype):
    """The same particles with offsets / velocities in `dtype`; offsets that
    round up to 1 in the narrower type are kept just below 1."""
    off = p["off"].astype(dtype)
    np.minimum(off, np.nextafter(dtype(1.0), dtype(0.0)), out=off)
    return dict(cell=p["cell"], off=off, vel=p["vel"].astype(dtype), id=p["id"])


def to_oracle(p):
    """SoA generator arrays -> (n, 3) float64 arrays (exact widening)."""
    n = p["cell"].size
    off = np.zeros((n, 3))
    off[:, : p["off"].shape[0]] = p["off"].T.astype(np.float64)
    vel = p["vel"].T.astype(np.float64).copy()
    return dict(cell=p["cell"].copy(), off=off, vel=vel)


# ----------------------------------------------------------------------------
# Synthetic fields for stage tests
# ----------------------------------------------------------------------------
def synthetic_phi(case: Case, seed: int = BASE_SEED, modes: int = 4, noise: float = 0.05):
    """Smooth periodic potential at cell centres plus a little white noise."""
    rng = np.random.Generator(np.random.Philox(seed * 7 + case.case_id))
    d = case.dim
    axes = [(np.arange(case.n[a]) + 0.5) / case.n[a] for a in range(d)]
    grids = np.meshgrid(*axes, indexing="ij")
    phi = np.zeros(grids[0].shape)
    for _ in range(modes):
        k = rng.integers(-2, 3, size=d)
        amp = rng.normal()
        ph = rng.random() * 2 * np.pi
        arg = sum(2 * np.pi * k[a] * grids[a] for a in range(d)) + ph
        phi += amp * np.cos(arg)
    phi += noise * rng.standard_normal(phi.shape)
    # linear cell index i + n0 (j + n1 k): transpose so axis 0 varies fastest
    return np.ascontiguousarray(phi.transpose(tuple(range(d - 1, -1, -1))).ravel())


def synthetic_charge(case: Case, seed: int = BASE_SEED):
    """Random neutral-on-average charge per cell (for solver stage tests)."""
    rng = np.random.Generator(np.random.Philox(seed * 13 + case.case_id))
    q = rng.standard_normal(case.ncells)
    return q


def synthetic_ev(case: Case, nverts: int, dtype=np.float32, seed: int = BASE_SEED, scale=0.5):
    """Random vertex field, components (x, y, z), shape (nverts, 3)."""
    rng = np.random.Generator(np.random.Philox(seed * 17 + case.case_id))
    E = (rng.standard_normal((nverts, 3)) * scale).astype(dtype)
    if case.dim == 2:
        E[:, 2] = 0
    return E


# ----------------------------------------------------------------------------
# Manufactured-solution input of the field solver (Sec. "Field solver",
# Eqs. r, z, mms; Table t1)
# ----------------------------------------------------------------------------
SPHERICAL_RZ = 3
MMS_R1, MMS_R2 = 1.0, 10.0


def spherical_mms_input(n0: int, n1: Optional[int] = None):
    """Right side and exact potential of the paper's spherical r-z test.

    The map is (r, z) = rho (sin t, cos t), rho = r_1 + (r_2 - r_1) xi,
    t = pi (1 - eta), r_1 = 1, r_2 = 10, with the geometric factor Omega = r;
    the potential is phi = sin((r_2 - r_1)^2 xi (1 - xi)) cos(pi eta^2).  The
    right side per cell is Omega J (-lap phi) / (n0 n1) at the cell centre,
    lap the axisymmetric spherical Laplacian written out in (rho, t), and
    J = pi (r_2 - r_1) rho the map's Jacobian (closed form).  Returns
    (charge, exact phi), cell index i + n0 j."""
    n1 = n0 if n1 is None else n1
    D = MMS_R2 - MMS_R1
    A = D * D
    u = (np.arange(n0) + 0.5) / n0
    v = (np.arange(n1) + 0.5) / n1
    u, v = np.meshgrid(u, v, indexing="xy")  # [j, i]: i fastest when raveled
    u, v = u.ravel(), v.ravel()
    arg = A * u * (1 - u)
    sa, ca = np.sin(arg), np.cos(arg)
    ce, se = np.cos(np.pi * v * v), np.sin(np.pi * v * v)
    phi = sa * ce
    rho = MMS_R1 + D * u
    t = np.pi * (1 - v)
    # derivatives in rho and t: d/drho = (1/D) d/dxi, d/dt = -(1/pi) d/deta
    p_r = A * (1 - 2 * u) * ca * ce / D
    p_rr = (-2 * A * ca - A * A * (1 - 2 * u) ** 2 * sa) * ce / (D * D)
    p_t = sa * se * 2 * np.pi * v / np.pi
    p_tt = -sa * (ce * (2 * np.pi * v) ** 2 + se * 2 * np.pi) / (np.pi * np.pi)
    lap = p_rr + 2 * p_r / rho + (p_tt + np.cos(t) / np.sin(t) * p_t) / (rho * rho)
    omega = rho * np.sin(t)
    J = np.pi * D * rho
    return -lap * omega * J / (n0 * n1), phi
