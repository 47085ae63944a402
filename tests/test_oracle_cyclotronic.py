"""Pins for the oracle's cyclotronic velocity step (Sec. "Particle mover":
with a uniform background B the gyration is resolved exactly, so the time
step need not resolve omega_c; Sec. "Tests" runs at omega_ce dt ~ 1): the
velocity takes the electric impulse (q/m) E dt, then the particle gyrates
exactly in B over dt.

Expected values, none computed by the routine itself:
  - B = 0: the leap-frog step (equal to the Boris push with B = 0);
  - pure B at omega_c dt = 2.3 (Boris would turn by 2 atan(1.15) = 1.71 per
    step): after 40 steps the velocity and the position (through the hybrid
    mover on the identity map) are those of the exact helix, written out here;
  - uniform E parallel to B: the positions of the exact uniformly accelerated
    motion (leap-frog with the half-impulse start is exact for a constant force);
  - uniform E perpendicular to B at omega_c dt = 2.3: the mean velocity over
    many steps is the E x B drift E x B / B^2 (no secular error);
  - uniform E perpendicular to B: the orbit converges to the exact one
    (drift plus gyration) at second order in dt at a fixed time."""
import numpy as np

import oracle as O


def _box(n=(64, 64, 64), L=(200.0, 200.0, 200.0)):
    m = O.make_map(O.IDENTITY, 3, L=L)
    g = O.make_grid(n)
    return m, g


def _one(m, g, xi):
    n = np.array(g.n[:3])
    u = np.asarray(xi) * n
    idx = np.floor(u).astype(int)
    cell = np.array([idx[0] + n[0] * (idx[1] + n[1] * idx[2])], dtype=np.int32)
    off = np.zeros((1, 3))
    off[0] = u - idx
    return cell, off


def _x(g, L, cell, off):
    n = np.array(g.n[:3])
    c = int(cell[0])
    idx = np.array([c % n[0], (c // n[0]) % n[1], c // (n[0] * n[1])])
    return (idx + off[0]) / n * np.array(L)


def test_zero_field_b_is_leap_frog():
    rng = np.random.default_rng(0)
    v = rng.normal(size=(50, 3))
    E = rng.normal(size=(50, 3))
    v1, vm = O.cyclotronic(v, E, (0.0, 0.0, 0.0), -1.3, 0.07)
    v2 = O.boris(v, E, (0.0, 0.0, 0.0), -1.3, 0.07)
    np.testing.assert_allclose(v1, v2, atol=1e-14)
    np.testing.assert_allclose(vm, v1, atol=0)


def test_pure_gyration_is_exact_at_large_omega_dt():
    L = (200.0, 200.0, 200.0)
    m, g = _box(L=L)
    qm, Bz, dt = -1.0, 23.0, 0.1  # omega = -23, theta = -2.3
    B = (0.0, 0.0, Bz)
    v0 = np.array([[1.3, -0.4, 0.25]])
    x0 = np.array([100.3, 99.1, 50.7])
    cell, off = _one(m, g, x0 / np.array(L))
    vel = v0.copy()
    Ev = np.zeros((O.nverts(g), 3))
    w = qm * Bz
    for k in range(40):
        cell, off, vel, _ = O.push_cyclo(m, g, qm, dt, B, cell, off, vel, Ev)
    t = 40 * dt
    vp = np.array([v0[0, 0], v0[0, 1], 0.0])
    vxb = np.cross(vp, [0.0, 0.0, 1.0])
    v_exact = vp * np.cos(w * t) + vxb * np.sin(w * t) + np.array([0.0, 0.0, v0[0, 2]])
    x_exact = x0 + vp * np.sin(w * t) / w + vxb * (1 - np.cos(w * t)) / w + np.array([0.0, 0.0, v0[0, 2] * t])
    np.testing.assert_allclose(vel[0], v_exact, atol=1e-12)
    np.testing.assert_allclose(_x(g, L, cell, off), x_exact, atol=1e-10)


def test_parallel_field_gives_the_exact_accelerated_motion():
    L = (200.0, 200.0, 200.0)
    m, g = _box(L=L)
    qm, dt = 1.0, 0.1
    B = (0.0, 0.0, 5.0)
    Ez = 0.3
    Ev = np.zeros((O.nverts(g), 3))
    Ev[:, 2] = Ez
    v0 = np.array([[0.0, 0.0, -1.0]])
    x0 = np.array([100.0, 100.0, 100.0])
    cell, off = _one(m, g, x0 / np.array(L))
    vel, _ = O.cyclotronic(v0, np.array([[0.0, 0.0, Ez]]), (0.0, 0.0, 0.0), qm, -0.5 * dt)  # half impulse back
    for k in range(30):
        cell, off, vel, _ = O.push_cyclo(m, g, qm, dt, B, cell, off, vel, Ev)
    t = 30 * dt
    x_exact = x0 + np.array([0.0, 0.0, v0[0, 2] * t + 0.5 * qm * Ez * t * t])
    np.testing.assert_allclose(_x(g, L, cell, off), x_exact, atol=1e-10)


def test_e_cross_b_drift_has_no_secular_error():
    qm, Bz, dt, Ex = 1.0, 23.0, 0.1, 0.4  # theta = 2.3
    B = (0.0, 0.0, Bz)
    v = np.array([[0.7, -0.2, 0.0]])
    E = np.array([[Ex, 0.0, 0.0]])
    u_drift = np.cross([Ex, 0.0, 0.0], B) / Bz ** 2
    disp = np.zeros(3)
    N = 2000
    for k in range(N):
        v, vm = O.cyclotronic(v, E, B, qm, dt)
        disp += vm[0] * dt
    mean_v = disp / (N * dt)
    # the gyration about the drift contributes at most 2 r_L / (N dt)
    r_l = (np.linalg.norm(v[0] - u_drift) + qm * Ex * dt) / (qm * Bz)
    assert np.all(np.abs(mean_v - u_drift) <= 2 * r_l / (N * dt) + 1e-12), (mean_v, u_drift)


def test_second_order_convergence_to_the_exact_orbit():
    # uniform E perpendicular to B: the exact orbit is the E x B drift plus a
    # gyration about it; the scheme, started with v(0-) = v0 - (q/m) E dt / 2,
    # converges to it at second order at a fixed time (error ratio 4)
    qm, Bz, Ex = 1.0, 2.0, 0.3
    B = (0.0, 0.0, Bz)
    w = qm * Bz
    v0 = np.array([0.5, -0.8, 0.2])
    u_e = np.cross([Ex, 0.0, 0.0], B) / Bz ** 2
    T = 1.0
    r = v0 - u_e
    rp = np.array([r[0], r[1], 0.0])
    rxb = np.cross(rp, [0.0, 0.0, 1.0])
    x_exact = u_e * T + rp * np.sin(w * T) / w + rxb * (1 - np.cos(w * T)) / w + np.array([0.0, 0.0, r[2] * T])
    errs = []
    for dt in (0.1, 0.05, 0.025):
        E = np.array([[Ex, 0.0, 0.0]])
        v = (v0 - 0.5 * qm * dt * E[0])[None, :]
        x = np.zeros(3)
        for k in range(int(round(T / dt))):
            v, vm = O.cyclotronic(v, E, B, qm, dt)
            x += dt * vm[0]
        errs.append(np.abs(x - x_exact).max())
    ratio = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(ratio - 4.0) < 0.3), (errs, ratio)
