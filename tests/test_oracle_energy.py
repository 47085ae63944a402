"""Pins for the oracle's energy diagnostics (Sec. "Tests": the energy
histories of the runs): the field energy W_E = 1/2 sum_c (J rho dV)_c phi_c and
the leap-frog kinetic energy KE = 1/2 sum m w v^{n-1/2} . v^{n+1/2}.

Expected values are closed forms, none computed by the routines under test:
  - W_E of one Fourier mode on the identity map from the eigenvalue of the
    discrete 5-point Laplacian, 4 sin^2(pi h / L) / h^2;
  - W_E of a vacuum capacitor (a floating wall holding charge Q facing a
    grounded wall) as 1/2 Q^2 / C, which is also the energy 1/2 int |E|^2 of
    the uniform field between the plates;
  - KE under a uniform acceleration a from the exact leap-frog velocities:
    v^{n-1/2} . v^{n+1/2} = |v(t_n)|^2 - |a dt / 2|^2 with v(t_n) = v0 + a t_n.
Each fails for a dropped factor 1/2, a sign flip, or (for KE) the velocity of
a neighbouring half step in place of the product."""
import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("L,n,axis", [((1.0, 1.0), (16, 16), 0), ((3.0, 2.0), (24, 10), 1)])
def test_field_energy_of_one_mode(L, n, axis):
    m = O.make_map(O.IDENTITY, 2, L=L)
    g = O.make_grid(n)
    i, j = np.meshgrid(np.arange(n[0]), np.arange(n[1]), indexing="ij")
    xi = ((i if axis == 0 else j) + 0.5) / n[axis]
    dV = L[0] * L[1] / (n[0] * n[1])
    # charge per cell J rho dV = dV cos(2 pi x / L_axis); cell index c = i + n0 j
    charge = (dV * np.cos(2 * np.pi * xi)).T.reshape(-1)
    phi, _, _ = O.poisson_solve(m, g, charge)
    h = L[axis] / n[axis]
    lam = 4.0 * np.sin(np.pi * h / L[axis]) ** 2 / h ** 2
    # phi = cos / lam, so W_E = 1/2 dV sum cos^2 / lam = L0 L1 / (4 lam)
    np.testing.assert_allclose(phi, charge / dV / lam, rtol=0, atol=1e-12 / lam)
    we = O.field_energy(charge, phi)
    assert abs(we - L[0] * L[1] / (4 * lam)) < 1e-12 * we
    # the continuum value (2 pi / L)^2 in place of lam is approached at second order
    cont = L[0] * L[1] / (4 * (2 * np.pi / L[axis]) ** 2)
    assert abs(we / cont - 1) < 0.5 * (np.pi * h / L[axis]) ** 2


def test_field_energy_of_a_charged_floating_wall():
    # no particles: the wall holds Q (absorbed earlier) and faces the grounded
    # wall at x = L_x across vacuum -- a plate capacitor of capacitance
    # C = L_y / L_x per unit depth, energy 1/2 Q^2 / C = 1/2 (Q / L_y)^2 L_x L_y
    L, n, Q = (20.0, 5.0), (32, 8), 3.0
    m = O.make_map(O.IDENTITY, 2, L=L)
    g = O.make_grid(n, bc_lo=(O.FLOATING, O.PERIODIC), bc_hi=(O.DIRICHLET, O.PERIODIC))
    empty = dict(q=1.0, m=1.0, w=1.0, cell=np.zeros(0, np.int32), off=np.zeros((0, 3)),
                 vel=np.zeros((0, 3)), absorbed=3)
    sim = O.OracleSim(m, g, [empty], dt=0.1)
    sim.deposit()
    sim.solve()
    assert abs(sim.wall_charge - Q) < 1e-15
    ref = 0.5 * Q * Q * L[0] / L[1]
    assert abs(sim.field_energy() - ref) < 1e-10 * ref


def test_kinetic_energy_under_uniform_acceleration():
    # identity map, Dirichlet walls phi(0) = V, phi(L_x) = 0, periodic y: the
    # vacuum potential is linear and E_x = V / L_x exactly; the particles'
    # own charge is negligible (tiny weight), so every one of them is
    # uniformly accelerated by a = (q/m) E and leap-frog is exact.
    L, n, V, dt = (16.0, 4.0), (16, 4), -8.0, 0.1
    m = O.make_map(O.IDENTITY, 2, L=L)
    g = O.make_grid(n, bc_lo=(O.DIRICHLET, O.PERIODIC), bc_hi=(O.DIRICHLET, O.PERIODIC),
                    phi_lo=(V, 0.0))
    rng = np.random.Generator(np.random.Philox(11))
    N, q, mass, w = 400, -1.0, 1.0, 1e-20
    cell = (rng.integers(6, 10, N) + n[0] * rng.integers(0, n[1], N)).astype(np.int32)
    off = np.zeros((N, 3))
    off[:, :2] = rng.random((N, 2))
    v0 = 0.3 * rng.standard_normal((N, 3))
    sp = dict(q=q, m=mass, w=w, cell=cell, off=off, vel=v0.copy())
    sim = O.OracleSim(m, g, [sp], dt=dt)
    sim.initialize()
    a = np.array([q / mass * V / L[0], 0.0, 0.0])
    b2 = float(np.sum((0.5 * a * dt) ** 2))
    for k in range(6):
        sim.step()
        assert sim.counts[0] == (0, 0)
        vn = v0 + a * (k * dt)  # v(t_k): the product spans t_k -/+ dt/2
        ref = 0.5 * mass * w * float(np.sum(np.sum(vn * vn, axis=1) - b2))
        assert abs(sim.ke - ref) < 1e-10 * abs(ref), (k, sim.ke, ref)
        # and the stored velocity is v(t_k + dt/2)
        np.testing.assert_allclose(sim.sp[0]["vel"], vn + 0.5 * a * dt, rtol=0, atol=1e-11)
