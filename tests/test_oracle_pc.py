"""Pins for the oracle's predictor-corrector position update (Sec. "Particle
mover", Eqs. step2-step4; k carried by the b1 vertex weights, Eq. step3).

Expected values and properties, none of them computed by the routine itself:
  - on the identity map k is constant, so the update is the exact straight
    line: it equals the exact-inversion mover (pinned in test_oracle_mover);
  - with k taken from the map at the point (kmode 1) the scheme is the
    midpoint rule for d xi/dt = k(xi) v: one step is off the exact logical
    characteristic x^-1(x(xi) + dt v) by O(dt^3), a run to a fixed time by
    O(dt^2) (second order, the property the paper restores with it);
  - with k interpolated from the vertices (kmode 0, the paper's method) the
    step differs from kmode 1 by dt times the O(h^2) error of bilinear
    interpolation."""
import numpy as np

import oracle as O


def _particles(g, dim, n, rng):
    cells = int(np.prod(g.n[:dim]))
    cell = rng.integers(0, cells, n).astype(np.int32)
    off = np.zeros((n, 3))
    off[:, :dim] = rng.random((n, dim))
    return cell, off


def _xi(g, dim, cell, off):
    n = list(g.n[:dim])
    idx = np.zeros((cell.size, dim))
    c = cell.astype(np.int64)
    for a in range(dim):
        idx[:, a] = c % n[a]
        c //= n[a]
    return (idx + off[:, :dim]) / np.array(n)


def _periodic_dist(a, b):
    d = a - b
    return np.abs(d - np.round(d))


def test_identity_map_is_the_straight_line():
    rng = np.random.default_rng(1)
    for dim, n, L in ((2, (12, 10), (3.0, 2.0)), (3, (6, 5, 4), (1.0, 2.0, 1.5))):
        m = O.make_map(O.IDENTITY, dim, L=L)
        g = O.make_grid(n)
        cell, off = _particles(g, dim, 300, rng)
        vel = rng.normal(size=(300, 3))
        nv = int(np.prod(n))
        Ev = rng.normal(size=(nv, 3))
        B = (0.0, 0.0, 0.7)
        a = O.push(m, g, -1.0, 0.05, B, cell, off, vel, Ev)
        b = O.push_pc(m, g, -1.0, 0.05, B, cell, off, vel, Ev)
        assert np.array_equal(a[2], b[2])
        xa, xb = _xi(g, dim, a[0], a[1]), _xi(g, dim, b[0], b[1])
        assert _periodic_dist(xa, xb).max() < 1e-14


def _exact_and_pc(m, g, dim, cell, off, vel, dt, kmode):
    nv = int(np.prod(g.n[:dim]))
    E0 = np.zeros((nv, 3))
    ex = O.push(m, g, -1.0, dt, (0.0, 0.0, 0.0), cell, off, vel, E0)
    pc = O.push_pc(m, g, -1.0, dt, (0.0, 0.0, 0.0), cell, off, vel, E0, kmode=kmode)
    return _xi(g, dim, ex[0], ex[1]), _xi(g, dim, pc[0], pc[1])


def test_one_step_error_is_third_order_in_dt():
    rng = np.random.default_rng(2)
    for dim, eps, n in ((2, 0.1, (32, 32)), (3, 0.05, (16, 16, 16))):
        m = O.make_map(O.SINUSOIDAL, dim, eps=eps)
        g = O.make_grid(n)
        cell, off = _particles(g, dim, 400, rng)
        vel = rng.normal(size=(400, 3))
        errs = []
        for dt in (0.016, 0.008, 0.004):
            ex, pc = _exact_and_pc(m, g, dim, cell, off, vel, dt, kmode=1)
            errs.append(np.median(_periodic_dist(ex, pc).max(axis=1)))
        r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
        assert 6.5 < r1 < 9.5 and 6.5 < r2 < 9.5, (dim, errs, r1, r2)


def test_run_to_fixed_time_is_second_order():
    # free streaming (no field): the exact trajectory is x(t) = x0 + v t
    rng = np.random.default_rng(3)
    m = O.make_map(O.SINUSOIDAL, 2, eps=0.1)
    g = O.make_grid((32, 32))
    cell0, off0 = _particles(g, 2, 200, rng)
    vel0 = rng.normal(size=(200, 3)) * 0.5
    nv = 32 * 32
    E0 = np.zeros((nv, 3))
    T = 0.2
    ex = O.push(m, g, -1.0, T, (0.0, 0.0, 0.0), cell0, off0, vel0, E0)  # exact: one inversion
    x_ex = _xi(g, 2, ex[0], ex[1])
    errs = []
    for nsteps in (10, 20, 40):
        cell, off, vel = cell0, off0, vel0
        for _ in range(nsteps):
            cell, off, vel, _c = O.push_pc(m, g, -1.0, T / nsteps, (0.0, 0.0, 0.0), cell, off, vel, E0,
                                           kmode=1)
        errs.append(np.median(_periodic_dist(x_ex, _xi(g, 2, cell, off)).max(axis=1)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.7 and 3.3 < r2 < 4.7, (errs, r1, r2)


def test_vertex_interpolation_error_is_second_order_in_h():
    rng = np.random.default_rng(4)
    m = O.make_map(O.SINUSOIDAL, 2, eps=0.1)
    xi = rng.random((300, 2))
    vel = rng.normal(size=(300, 3))
    dt = 0.004
    diffs = []
    for nc in (16, 32, 64):
        g = O.make_grid((nc, nc))
        u = xi * nc
        idx = np.floor(u)
        cell = (idx[:, 0] + nc * idx[:, 1]).astype(np.int32)
        off = np.zeros((300, 3))
        off[:, :2] = u - idx
        E0 = np.zeros((nc * nc, 3))
        a = O.push_pc(m, g, -1.0, dt, (0.0, 0.0, 0.0), cell, off, vel, E0, kmode=0)
        b = O.push_pc(m, g, -1.0, dt, (0.0, 0.0, 0.0), cell, off, vel, E0, kmode=1)
        diffs.append(np.median(_periodic_dist(_xi(g, 2, a[0], a[1]), _xi(g, 2, b[0], b[1])).max(axis=1)))
    r1, r2 = diffs[0] / diffs[1], diffs[1] / diffs[2]
    assert 3.0 < r1 < 5.0 and 3.0 < r2 < 5.0, (diffs, r1, r2)


def test_bounded_axis_boundaries_match_the_exact_mover_counts():
    # polar-log annulus: particles that leave through a wall are tombstoned
    # with the same codes; for small steps the two movers agree on who leaves
    rng = np.random.default_rng(5)
    m = O.make_map(O.POLAR_LOG, 2, r_in=1.0, r_out=10.0)
    g = O.make_grid((32, 32), bc_lo=(O.DIRICHLET, O.PERIODIC), bc_hi=(O.DIRICHLET, O.PERIODIC))
    cell, off = _particles(g, 2, 500, rng)
    off[:, 0] = np.where(cell % 32 == 0, 0.05, off[:, 0])
    vel = rng.normal(size=(500, 3)) * 3.0
    Ev = np.zeros((33 * 32, 3))
    a = O.push(m, g, -1.0, 0.01, (0.0, 0.0, 0.0), cell, off, vel, Ev)
    b = O.push_pc(m, g, -1.0, 0.01, (0.0, 0.0, 0.0), cell, off, vel, Ev)
    assert a[3][0] > 0
    same = (a[0] < 0) == (b[0] < 0)
    assert same.mean() > 0.99
    both = (a[0] >= 0) & (b[0] >= 0)
    xa, xb = _xi(g, 2, a[0][both], a[1][both]), _xi(g, 2, b[0][both], b[1][both])
    assert _periodic_dist(xa, xb).max() < 1e-3
