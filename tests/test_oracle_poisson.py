"""Pins for the oracle's Poisson operator and solve (Eq. poiscurv, Sec. II.B
field solver) and the vertex electric field.

Pins: operator symmetry / null space, an FFT solve of the undistorted periodic
problem, manufactured solutions with second-order convergence (error ratio
-> 4 per doubling, Table I), the paper's own spherical r-z manufactured
solution (Eqs. r, z, mms with Omega = r), and the exact vacuum solution of the
cylindrical probe (phi linear in xi between the walls)."""
import math

import numpy as np
import pytest

import oracle as O
from _golden import paper_value


def cell_centres(n):
    d = len(n)
    axes = [(np.arange(n[a]) + 0.5) / n[a] for a in range(d)]
    G = np.meshgrid(*axes, indexing="ij")
    # linear index i + n0 (j + n1 k): flatten in Fortran order
    xi = np.zeros((int(np.prod(n)), 3))
    for a in range(d):
        xi[:, a] = G[a].ravel(order="F")
    return xi


def dense(g, A):
    nc = O.ncells(g)
    M = np.zeros((nc, nc))
    for c in range(nc):
        e = np.zeros(nc)
        e[c] = 1.0
        M[:, c] = O.apply(g, A, e)
    return M


@pytest.mark.parametrize("dim,n,eps", [(2, (6, 5), 0.1), (3, (4, 3, 5), 0.05)])
def test_operator_symmetric_negative_semidefinite_with_constant_null_space(dim, n, eps):
    L = (1.0,) * dim
    m = O.make_map(O.SINUSOIDAL, dim, L, eps)
    g = O.make_grid(n)
    A, bd = O.poisson_assemble(m, g)
    M = dense(g, A)
    np.testing.assert_allclose(M, M.T, atol=1e-12 * np.abs(M).max())
    np.testing.assert_allclose(M @ np.ones(M.shape[0]), 0.0, atol=1e-12 * np.abs(M).max())
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    assert ev.max() < 1e-10 * np.abs(ev).max()
    assert np.sum(np.abs(ev) < 1e-10 * np.abs(ev).max()) == 1  # only the constant
    # 9-point (2D) / 19-point (3D) couplings: no corner entries in 3D
    if dim == 3:
        corner = [0, 2, 6, 8, 18, 20, 24, 26]
        assert np.all(A[:, corner] == 0.0)


def test_undistorted_periodic_solve_matches_fft():
    n = (16, 12)
    L = (3.0, 2.0)
    m = O.make_map(O.IDENTITY, 2, L)
    g = O.make_grid(n)
    rng = np.random.default_rng(0)
    charge = rng.standard_normal(n[0] * n[1])
    charge -= charge.mean()
    phi, it, rr = O.poisson_solve(m, g, charge, rtol=1e-14)
    # FFT: A = sum_i c_i (shift+ + shift- - 2), c_i = (L0 L1 / L_i^2) dV / h_i^2
    h = [1.0 / n[0], 1.0 / n[1]]
    dV = h[0] * h[1]
    c = [L[0] * L[1] / L[a] ** 2 * dV / h[a] ** 2 for a in range(2)]
    b = -charge.reshape(n[1], n[0])  # [j, i]
    kx = np.fft.fftfreq(n[0]) * n[0]
    ky = np.fft.fftfreq(n[1]) * n[1]
    lam = (c[0] * (2 * np.cos(2 * np.pi * kx / n[0]) - 2))[None, :] + \
          (c[1] * (2 * np.cos(2 * np.pi * ky / n[1]) - 2))[:, None]
    bh = np.fft.fft2(b)
    lam[0, 0] = 1.0
    ph = bh / lam
    ph[0, 0] = 0.0
    ref = np.real(np.fft.ifft2(ph)).ravel()
    ref -= ref.mean()  # J constant: J-weighted mean = plain mean
    np.testing.assert_allclose(phi, ref, atol=1e-11 * np.abs(ref).max())


def _mms_errors(make_case, sizes):
    errs = []
    for N in sizes:
        m, g, phi_ex, charge = make_case(N)
        phi, it, rr = O.poisson_solve(m, g, charge, rtol=1e-12)
        assert rr < 1e-11
        e = phi - phi_ex
        errs.append(math.sqrt(np.mean(e ** 2)))
    return np.array(errs)


def _sinusoidal_case(N):
    L, eps = 1.0, 0.1
    m = O.make_map(O.SINUSOIDAL, 2, (L, L), eps)
    g = O.make_grid((N, N))
    xi = cell_centres((N, N))
    x, _, _, J = O.map_eval(m, xi)
    phi = np.sin(2 * np.pi * x[:, 0] / L) * np.cos(2 * np.pi * x[:, 1] / L)
    rho = 8 * np.pi ** 2 / L ** 2 * phi
    charge = rho * J / N ** 2
    phi_ex = phi - np.sum(J * phi) / np.sum(J)
    return m, g, phi_ex, charge


def _polar_case(N):
    ri, ro = 1.0, 60.0
    m = O.make_map(O.POLAR_LOG, 2, r_in=ri, r_out=ro)
    g = O.make_grid((N, N), bc_lo=(O.DIRICHLET, 0), bc_hi=(O.DIRICHLET, 0))
    xi = cell_centres((N, N))
    x, _, _, J = O.map_eval(m, xi)
    r = np.hypot(x[:, 0], x[:, 1])
    th = np.arctan2(x[:, 1], x[:, 0])
    k = np.pi / (ro - ri)
    S = np.sin(k * (r - ri))
    S1 = k * np.cos(k * (r - ri))
    S2 = -k * k * S
    lap = (S2 + S1 / r - S / r ** 2) * np.cos(th)
    charge = -lap * J / N ** 2
    return m, g, S * np.cos(th), charge


def _paper_mms_case(N):
    # Eqs. (r), (z): r = rho sin(pi (1 - eta)), z = rho cos(pi (1 - eta)),
    # rho = r1 + (r2 - r1) xi; Omega = r; Eq. (mms):
    # phi = sin((r2 - r1)^2 xi (1 - xi)) cos(pi eta^2).  Boundary values:
    # phi = 0 at xi = 0, 1; d phi / d eta = 0 at eta = 0, 1 (the symmetry axis).
    r1, r2 = 1.0, 10.0
    D = r2 - r1
    A = D * D
    m = O.make_map(O.SPHERICAL_RZ, 2, r_in=r1, r_out=r2, omega=1)
    g = O.make_grid((N, N), bc_lo=(O.DIRICHLET, O.NEUMANN), bc_hi=(O.DIRICHLET, O.NEUMANN))
    xi = cell_centres((N, N))
    x, _, _, J = O.map_eval(m, xi)
    u, v = xi[:, 0], xi[:, 1]
    arg = A * u * (1 - u)
    ce = np.cos(np.pi * v ** 2)
    se = np.sin(np.pi * v ** 2)
    phi = np.sin(arg) * ce
    p_u = A * (1 - 2 * u) * np.cos(arg) * ce
    p_uu = (-2 * A * np.cos(arg) - A * A * (1 - 2 * u) ** 2 * np.sin(arg)) * ce
    p_v = -np.sin(arg) * se * 2 * np.pi * v
    p_vv = -np.sin(arg) * (ce * (2 * np.pi * v) ** 2 + se * 2 * np.pi)
    rho_s = r1 + D * u
    th = np.pi * (1 - v)
    # spherical Laplacian of phi(rho, theta), axisymmetric
    p_r = p_u / D
    p_rr = p_uu / D ** 2
    p_t = -p_v / np.pi
    p_tt = p_vv / np.pi ** 2
    lap = p_rr + 2 * p_r / rho_s + (p_tt + np.cos(th) / np.sin(th) * p_t) / rho_s ** 2
    Om = x[:, 0]
    charge = -lap * Om * J / N ** 2
    return m, g, phi, charge


@pytest.mark.parametrize("make_case,sizes", [(_sinusoidal_case, (16, 32, 64, 128)),
                                             (_polar_case, (16, 32, 64, 128))])
def test_manufactured_solutions_second_order(make_case, sizes):
    errs = _mms_errors(make_case, sizes)
    ratios = errs[:-1] / errs[1:]
    assert abs(ratios[-1] - 4.0) < 0.25, (errs, ratios)


def test_paper_spherical_mms_ratio_tends_to_four():
    # Table t1's error ratios (tests/golden): second order, 4.0 from 256^2 on;
    # the absolute L2 values depend on a norm the paper does not state (parity
    # unpinned).  Here 32^2 .. 256^2: the ratio of the last refinement matches
    # the paper's 256^2 value, the one before its 128^2 value.
    errs = _mms_errors(_paper_mms_case, (32, 64, 128, 256))
    ratios = errs[:-1] / errs[1:]
    assert abs(ratios[-1] - paper_value("mms_error_ratio_256")) < 0.15, (errs, ratios)
    assert abs(ratios[-2] - paper_value("mms_error_ratio_128")) < 0.3, (errs, ratios)


def test_probe_vacuum_solution_and_field_are_exact():
    # zero charge, phi(xi=0) = -5, phi(xi=1) = 0: the operator has constant
    # coefficients in xi (conformal map), so phi = -5 (1 - xi) exactly and
    # E_r = -5 / (r ln(r_out / r_in)).
    ri, ro = 1.0, 60.0
    n = (32, 16)
    m = O.make_map(O.POLAR_LOG, 2, r_in=ri, r_out=ro)
    g = O.make_grid(n, bc_lo=(O.DIRICHLET, 0), bc_hi=(O.DIRICHLET, 0), phi_lo=(-5.0, 0),
                    phi_hi=(0.0, 0))
    phi, it, rr = O.poisson_solve(m, g, np.zeros(n[0] * n[1]), rtol=1e-15)
    xi = cell_centres(n)
    np.testing.assert_allclose(phi, -5 * (1 - xi[:, 0]), atol=1e-12)
    Ev = O.efield(m, g, phi)
    nv0 = n[0] + 1
    vi = np.arange(nv0 * n[1])
    vx, vy = vi % nv0, vi // nv0
    xv = np.zeros((vi.size, 3))
    xv[:, 0] = vx / n[0]
    xv[:, 1] = vy / n[1]
    x, *_ = O.map_eval(m, xv)
    r = np.hypot(x[:, 0], x[:, 1])
    Er = -5 / (r * math.log(ro / ri))
    np.testing.assert_allclose(Ev[:, 0], Er * x[:, 0] / r, atol=1e-11)
    np.testing.assert_allclose(Ev[:, 1], Er * x[:, 1] / r, atol=1e-11)


def test_efield_identity_map_is_cartesian_staggered_gradient():
    n = (8, 6)
    L = (4.0, 3.0)
    m = O.make_map(O.IDENTITY, 2, L)
    g = O.make_grid(n)
    phi = np.random.default_rng(1).standard_normal(48)
    Ev = O.efield(m, g, phi).reshape(6, 8, 3)
    P = phi.reshape(6, 8)
    dx, dy = L[0] / 8, L[1] / 6
    for j in range(6):
        for i in range(8):
            # vertex (i, j) sits between cells i-1, i and j-1, j
            gx = 0.5 * ((P[j, i] - P[j, i - 1]) + (P[j - 1, i] - P[j - 1, i - 1])) / dx
            gy = 0.5 * ((P[j, i] - P[j - 1, i]) + (P[j, i - 1] - P[j - 1, i - 1])) / dy
            assert abs(Ev[j, i, 0] + gx) < 1e-12 and abs(Ev[j, i, 1] + gy) < 1e-12


def test_efield_linear_potential_exact_on_distorted_map():
    # phi linear in physical x on a bounded, orthogonal stretched map.
    n = (12, 10)
    m = O.make_map(O.IDENTITY, 2, (2.0, 5.0))
    g = O.make_grid(n, bc_lo=(O.DIRICHLET, O.DIRICHLET), bc_hi=(O.DIRICHLET, O.DIRICHLET),
                    phi_lo=(0.0, 0.0), phi_hi=(0.0, 0.0))
    # phi = 3 x at cell centres (x = 2 xi): the x-walls carry phi 0 and 6, but the
    # y-walls see a non-constant value -- so test only interior vertices.
    xi = cell_centres(n)
    phi = 3 * 2 * xi[:, 0]
    Ev = O.efield(m, g, phi).reshape(11, 13, 3)
    assert np.allclose(Ev[1:-1, 1:-1, 0], -3.0, atol=1e-12)
    assert np.allclose(Ev[1:-1, 1:-1, 1], 0.0, atol=1e-12)
