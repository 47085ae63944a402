"""Pins for the oracle's pieces of the paper's planar-wall test (Sec. "Tests",
charging and shielding of a conducting planar wall): flux injection of a
drifting Maxwellian and a floating conducting wall that holds the charge it
absorbed (Gauss' law at the wall).

Expected values, none computed by the routines themselves:
  - the drifting-Maxwellian flux against numerical quadrature of the
    half-range first moment;
  - the sampled normal speeds against the flux-weighted distribution's
    quadrature moments and CDF (Kolmogorov-Smirnov), the count per step
    against its mean, the tangential components against N(0, v_th^2);
  - the floating wall: a charge-free slab is a capacitor with the closed-form
    linear potential phi_w (1 - x / L), phi_w = Q L_x / L_y; with a uniform
    space charge the potential is the quadratic of the 1D problem, reached at
    second order in h; Gauss' law (flux through the wall = its charge) and
    the overall flux balance hold to the solver tolerance."""
import math

import numpy as np
import pytest

import oracle as O

scipy_integrate = pytest.importorskip("scipy.integrate")
scipy_stats = pytest.importorskip("scipy.stats")


def _phi(x):
    return math.exp(-0.5 * x * x) / math.sqrt(2 * math.pi)


@pytest.mark.parametrize("s", [0.0, 0.5, 2.1, 4.0])
def test_drift_flux_is_the_half_range_first_moment(s):
    ref, _ = scipy_integrate.quad(lambda v: v * _phi(v - s), 0.0, np.inf, epsabs=1e-14, epsrel=1e-13)
    assert abs(O.drift_flux(1.0, 1.0, s) - ref) < 1e-12
    assert abs(O.drift_flux(2.0, 0.5, s) - 2.0 * 0.5 * ref) < 1e-12
    if s == 0.0:
        assert abs(O.drift_flux(1.0, 1.0, 0.0) - 1 / math.sqrt(2 * math.pi)) < 1e-15


def _slab(n=(32, 8), L=(20.0, 5.0), floating=True):
    m = O.make_map(O.IDENTITY, 2, L=L)
    g = O.make_grid(n, bc_lo=(O.FLOATING if floating else O.DIRICHLET, O.PERIODIC),
                    bc_hi=(O.DIRICHLET, O.PERIODIC))
    return m, g


def test_drifting_injection_statistics():
    m, g = _slab((16, 8))
    s, vth, w, dt = 2.1, 0.3, 2e-3, 0.05
    lam = O.drift_flux(1.0, vth, s) * O.face_area(m) * dt / w
    vn, vt, counts = [], [], []
    for step in range(400):
        cell, off, vel, drawn = O.inject(m, g, 1.0, vth, w, dt, 99, step, 1, drift=s * vth)
        counts.append(drawn)
        # injected at the upper face of axis 0: inward normal is -x
        vn.append(-vel[:, 0])
        vt.append(vel[:, 1])
    vn = np.concatenate(vn) / vth
    vt = np.concatenate(vt) / vth
    counts = np.array(counts)
    assert abs(counts.mean() - lam) < 4 * math.sqrt(lam / counts.size) + 1.0 / counts.size
    assert np.all(vn > 0)
    # the particles kept are those whose free-streaming start stays in the grid:
    # with these sizes every one of them does
    assert vn.size == counts.sum()
    Z, _ = scipy_integrate.quad(lambda x: x * _phi(x - s), 0, np.inf)
    m1, _ = scipy_integrate.quad(lambda x: x * x * _phi(x - s), 0, np.inf)
    m2, _ = scipy_integrate.quad(lambda x: x ** 3 * _phi(x - s), 0, np.inf)
    mean, var = m1 / Z, m2 / Z - (m1 / Z) ** 2
    n = vn.size
    assert abs(vn.mean() - mean) < 4 * math.sqrt(var / n)
    cdf = np.vectorize(lambda x: scipy_integrate.quad(lambda y: y * _phi(y - s), 0, x)[0] / Z)
    xs = np.sort(vn)
    grid_x = np.linspace(0, xs[-1], 400)
    grid_c = cdf(grid_x)
    ecdf = np.searchsorted(xs, grid_x, side="right") / n
    assert np.max(np.abs(ecdf - grid_c)) < 1.63 / math.sqrt(n)  # KS at 1 %
    assert abs(vt.mean()) < 4 / math.sqrt(n) and abs(vt.var() - 1.0) < 6 * math.sqrt(2.0 / n)


def test_zero_drift_is_the_maxwellian_at_rest():
    m, g = _slab((16, 8))
    a = O.inject(m, g, 1.0, 1.0, 1e-3, 0.05, 5, 3, 0)
    b = O.inject(m, g, 1.0, 1.0, 1e-3, 0.05, 5, 3, 0, drift=0.0)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)


def _centres(g, L):
    n0, n1 = g.n[0], g.n[1]
    c = np.arange(n0 * n1)
    return (c % n0 + 0.5) * L[0] / n0


def test_floating_wall_vacuum_is_a_capacitor():
    L = (20.0, 5.0)
    m, g = _slab((32, 8), L)
    Q = 0.37
    phi, pw, p0, p1 = O.poisson_solve_floating(m, g, np.zeros(32 * 8), Q)
    assert abs(pw - Q * L[0] / L[1]) < 1e-10 * abs(pw)
    x = _centres(g, L)
    assert np.max(np.abs(phi - pw * (1 - x / L[0]))) < 1e-10 * abs(pw)
    gw = O._grid_with_wall(g, pw, False)
    assert abs(O.wall_flux(m, gw, phi, pw) - Q) < 1e-10


def test_floating_wall_with_space_charge_second_order():
    # -phi'' = rho0, E(0) = Q / L_y, phi(L) = 0
    L = (20.0, 5.0)
    rho0, Q = 0.05, -0.8
    errs = []
    for nx in (16, 32, 64):
        m, g = _slab((nx, 4), L)
        dV = (L[0] / nx) * (L[1] / 4)
        charge = np.full(nx * 4, rho0 * dV)
        phi, pw, _, _ = O.poisson_solve_floating(m, g, charge, Q)
        x = _centres(g, L)
        a = -Q / L[1]
        b = rho0 * L[0] ** 2 / 2 - a * L[0]
        exact = -rho0 * x * x / 2 + a * x + b
        errs.append(np.max(np.abs(phi - exact)))
        gw = O._grid_with_wall(g, pw, False)
        assert abs(O.wall_flux(m, gw, phi, pw) - Q) < 1e-9
        # every field line ends on the wall, the right boundary or the charge
        total_charge = charge.sum()
        Aop, bd = O.poisson_assemble(m, gw)
        assert abs(np.sum(O.apply(gw, Aop, phi) + bd) + total_charge) < 1e-8
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs


def test_oracle_sim_wall_charge_is_the_absorbed_charge():
    m, g = _slab((16, 8))
    rng = np.random.default_rng(3)
    n = 400
    cell = rng.integers(0, 16 * 8, n).astype(np.int32)
    cell = np.where(cell % 16 < 3, cell, cell - cell % 16).astype(np.int32)  # near the wall
    off = np.zeros((n, 3))
    off[:, :2] = rng.random((n, 2))
    vel = np.zeros((n, 3))
    vel[:, 0] = -rng.random(n) * 4.0
    sp = [dict(q=-1.0, m=1.0, w=0.01, cell=cell, off=off, vel=vel.copy())]
    osim = O.OracleSim(m, g, sp, dt=0.5, deposit="f64", rtol=1e-12)
    osim.initialize()
    for _ in range(3):
        osim.step()
    absorbed = osim.sp[0]["absorbed"]
    assert absorbed > 0
    assert abs(osim.wall_charge + 0.01 * absorbed) < 1e-15
    assert osim.phi_wall < 0.0
