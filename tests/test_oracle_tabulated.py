"""Pins for the oracle's tabulated map (Sec. "Curvilinear formulation": the
map known at the cell vertices, its metric coefficients from finite
differences of it).

Expected values, none computed by the tabulated map itself:
  - maps whose Jacobi matrix is multilinear (affine maps; quadratic terms
    xi_a^2 and products xi_a xi_b; the triple product in 3D): the centred and
    one-sided differences are exact and so is the multilinear blend of the
    vertex matrices, so x at the vertices and j, J, k everywhere equal the
    closed forms written out here;
  - on a periodic axis the tabulated map continues by whole periods;
  - the analytic sinusoidal map sampled at the vertices: J and the solver
    coefficients converge to the analytic ones at second order in h (error
    ratio 4 per doubling);
  - Poisson solves and the predictor-corrector mover on the sampled map
    converge at second order to those on the analytic map;
  - the inverse of the tabulated map (the piecewise multilinear interpolant
    of the vertex coordinates): round trips to 1e-12, an affine map inverted
    exactly (also beyond its walls, where the boundary cells' polynomials
    continue), and the hybrid mover with this inversion within O(h^2) of the
    mover on the analytic map."""
import numpy as np
import pytest

import oracle as O
from _mms import cell_centres


def _vertices(n, periodic):
    dim = len(n)
    nv = [(n[a] if periodic[a] else n[a] + 1) for a in range(dim)]
    axes = [np.arange(nv[a]) / n[a] for a in range(dim)]
    G = np.meshgrid(*axes, indexing="ij")
    xi = np.zeros((int(np.prod(nv)), 3))
    for a in range(dim):
        xi[:, a] = G[a].ravel(order="F")
    return xi


def _poly_map(dim):
    """x = A xi + b + quadratic and product terms, its Jacobi matrix."""
    rng = np.random.default_rng(40 + dim)
    A = np.eye(dim) * 2.0 + 0.3 * rng.standard_normal((dim, dim))
    b = rng.standard_normal(dim)
    cq = 0.2 * rng.standard_normal((dim, dim))  # c[a, k] xi_k^2 in x^a
    cp = 0.2 * rng.standard_normal(dim)         # c[a] xi_0 xi_1 in x^a
    ct = 0.1 * rng.standard_normal(dim)         # c[a] xi_0 xi_1 xi_2 in x^a (3D)

    def x_of(xi):
        xi = xi[:, :dim]
        x = xi @ A.T + b + (xi ** 2) @ cq.T + np.outer(xi[:, 0] * xi[:, 1], cp)
        if dim == 3:
            x += np.outer(xi[:, 0] * xi[:, 1] * xi[:, 2], ct)
        return x

    def j_of(xi):
        xi = xi[:, :dim]
        n = xi.shape[0]
        j = np.repeat(A[None], n, axis=0) + 2 * cq[None] * xi[:, None, :]
        j[:, :, 0] += np.outer(xi[:, 1], cp)
        j[:, :, 1] += np.outer(xi[:, 0], cp)
        if dim == 3:
            j[:, :, 0] += np.outer(xi[:, 1] * xi[:, 2], ct)
            j[:, :, 1] += np.outer(xi[:, 0] * xi[:, 2], ct)
            j[:, :, 2] += np.outer(xi[:, 0] * xi[:, 1], ct)
        return j

    return x_of, j_of


@pytest.mark.parametrize("dim,n", [(2, (7, 5)), (3, (4, 5, 3))])
def test_multilinear_jacobian_maps_are_exact(dim, n):
    x_of, j_of = _poly_map(dim)
    per = (0,) * dim
    xv = _vertices(n, per)
    m = O.make_tabulated_map(dim, n, per, x_of(xv).T)
    x, jac, k, J = O.map_eval(m, xv)
    np.testing.assert_allclose(x[:, :dim], x_of(xv), atol=1e-13)
    rng = np.random.default_rng(3)
    pts = np.zeros((500, 3))
    pts[:, :dim] = rng.random((500, dim))
    pts[:5, :dim] = 1.0  # the far corner: one-sided differences only
    x, jac, k, J = O.map_eval(m, pts)
    je = j_of(pts)
    np.testing.assert_allclose(jac[:, :dim, :dim], je, atol=1e-12)
    np.testing.assert_allclose(J, np.linalg.det(je), rtol=1e-12)
    np.testing.assert_allclose(k[:, :dim, :dim], np.linalg.inv(je), atol=1e-11)


def test_periodic_axes_continue_by_whole_periods():
    L = (2.0, 3.0)
    m = O.make_map(O.SINUSOIDAL, 2, L, 0.1)
    n = (12, 10)
    t = O.make_tabulated_map(2, n, (1, 1), O.sample_map_vertices(m, n, (1, 1)), L=L)
    rng = np.random.default_rng(5)
    pts = np.zeros((200, 3))
    pts[:, :2] = rng.random((200, 2))
    x0, j0, _, _ = O.map_eval(t, pts)
    for sh in ((1, 0), (0, 1), (-1, 2)):
        q = pts.copy()
        q[:, :2] += sh
        x1, j1, _, _ = O.map_eval(t, q)
        np.testing.assert_allclose(x1[:, :2], x0[:, :2] + np.array(sh) * np.array(L), atol=1e-12)
        np.testing.assert_allclose(j1, j0, atol=1e-12)


def _face_points(n):
    xi = cell_centres(n)
    xi[:, 0] += 0.5 / n[0]
    return xi


@pytest.mark.parametrize("dim,eps", [(2, 0.1), (3, 0.05)])
def test_sampled_sinusoidal_metric_converges_second_order(dim, eps):
    m = O.make_map(O.SINUSOIDAL, dim, (1.0,) * dim, eps)
    errJ, errA = [], []
    sizes = (16, 32, 64) if dim == 3 else (32, 64, 128)
    for N in sizes:
        n = (N,) * dim
        t = O.make_tabulated_map(dim, n, (1,) * dim, O.sample_map_vertices(m, n, (1,) * dim))
        xi = _face_points(n)
        errJ.append(np.abs(O.map_eval(t, xi)[3] - O.map_eval(m, xi)[3]).max())
        errA.append(np.abs(O.coef_eval(t, xi) - O.coef_eval(m, xi)).max())
    for e in (np.array(errJ), np.array(errA)):
        r = e[:-1] / e[1:]
        assert abs(r[-1] - 4.0) < 0.3 and np.all(r > 3.3), (e, r)


def _solve_pair(N, kind):
    if kind == "sinusoidal":
        m = O.make_map(O.SINUSOIDAL, 2, (1.0, 1.0), 0.1)
        per = (1, 1)
        g = O.make_grid((N, N))
        xi = cell_centres((N, N))
        _, _, _, J = O.map_eval(m, xi)
        charge = np.cos(2 * np.pi * xi[:, 0]) * np.sin(4 * np.pi * xi[:, 1]) * J / N ** 2
        charge -= charge.mean()
    else:
        m = O.make_map(O.POLAR_LOG, 2, r_in=1.0, r_out=60.0)
        per = (0, 1)
        g = O.make_grid((N, N), bc_lo=(O.DIRICHLET, 0), bc_hi=(O.DIRICHLET, 0), phi_lo=(-5.0, 0))
        xi = cell_centres((N, N))
        _, _, _, J = O.map_eval(m, xi)
        charge = 1e-3 * np.sin(np.pi * xi[:, 0]) * J / N ** 2
    # the polar map closes on itself around the axis: no shift per period
    L = (1.0, 1.0) if kind == "sinusoidal" else (1.0, 0.0)
    t = O.make_tabulated_map(2, (N, N), per, O.sample_map_vertices(m, (N, N), per), L=L)
    pa = O.poisson_solve(m, g, charge, rtol=1e-13)[0]
    pt = O.poisson_solve(t, g, charge, rtol=1e-13)[0]
    return np.abs(pt - pa).max() / np.abs(pa).max()


@pytest.mark.parametrize("kind", ["sinusoidal", "polar"])
def test_solve_on_the_sampled_map_converges_second_order(kind):
    e = np.array([_solve_pair(N, kind) for N in (16, 32, 64)])
    r = e[:-1] / e[1:]
    assert abs(r[-1] - 4.0) < 0.3 and np.all(r > 3.0), (e, r)


def test_pc_mover_on_the_sampled_map_converges_second_order():
    m = O.make_map(O.SINUSOIDAL, 2, (1.0, 1.0), 0.1)
    rng = np.random.default_rng(9)
    npart = 400
    xi0 = rng.random((npart, 2))
    vel = np.zeros((npart, 3))
    vel[:, :2] = rng.normal(size=(npart, 2))
    errs = []
    for N in (32, 64, 128):
        n = (N, N)
        g = O.make_grid(n)
        t = O.make_tabulated_map(2, n, (1, 1), O.sample_map_vertices(m, n, (1, 1)))
        u = xi0 * N
        idx = np.floor(u).astype(np.int64)
        cell = (idx[:, 0] + N * idx[:, 1]).astype(np.int32)
        off = np.zeros((npart, 3))
        off[:, :2] = u - idx
        Ev = np.zeros((N * N, 3))
        res = []
        for mm in (m, t):
            c, o, _, _ = O.push_pc(mm, g, -1.0, 0.05, (0.0, 0.0, 0.0), cell, off, vel, Ev)
            ci = np.stack([c % N, c // N], axis=1)
            res.append((ci + o[:, :2]) / N)
        d = res[1] - res[0]
        d -= np.round(d)
        errs.append(np.abs(d).max())
    e = np.array(errs)
    r = e[:-1] / e[1:]
    assert abs(r[-1] - 4.0) < 0.3 and np.all(r > 3.0), (e, r)


def test_inverse_of_the_tabulated_map():
    # round trip inside the grid, from a nearby old position, on the sampled
    # sinusoidal map (periodic) and the sampled annulus (walls); an affine map
    # is inverted exactly (closed form A^-1 (x - b))
    rng = np.random.default_rng(11)
    m = O.make_map(O.SINUSOIDAL, 2, (1.0, 1.0), 0.1)
    t = O.make_tabulated_map(2, (24, 20), (1, 1), O.sample_map_vertices(m, (24, 20), (1, 1)))
    xi = np.zeros((400, 3))
    xi[:, :2] = rng.random((400, 2))
    x = O.map_eval(t, xi)[0]
    old = xi.copy()
    old[:, :2] += rng.normal(scale=0.05, size=(400, 2))
    back = O.map_invert(t, x, old)
    dd = back[:, :2] - xi[:, :2]
    assert np.abs(dd - np.round(dd)).max() < 1e-12
    A = np.array([[2.0, 0.3], [-0.4, 1.5]])
    bvec = np.array([0.2, -0.1])
    n = (7, 5)
    xv = _vertices(n, (0, 0))
    ta = O.make_tabulated_map(2, n, (0, 0), (xv[:, :2] @ A.T + bvec).T)
    pts = np.zeros((300, 3))
    pts[:, :2] = rng.random((300, 2)) * 1.2 - 0.1  # some beyond the walls: the extended map
    y = np.zeros((300, 3))
    y[:, :2] = pts[:, :2] @ A.T + bvec
    inv = O.map_invert(ta, y, np.full((300, 3), 0.5))
    np.testing.assert_allclose(inv[:, :2], pts[:, :2], atol=1e-12)


def test_exact_mover_on_the_sampled_map_converges_second_order():
    # the hybrid mover with exact inversion of the tabulated (piecewise
    # multilinear) map tends to the mover on the analytic map as h^2: the
    # difference is that of the interpolation error of x at the old and the
    # new position, O(h^2) but oscillating on the grid scale, so the bar is
    # the envelope: err N^2 about constant, a factor >= 8 over two doublings
    m = O.make_map(O.SINUSOIDAL, 2, (1.0, 1.0), 0.1)
    rng = np.random.default_rng(12)
    npart = 400
    xi0 = rng.random((npart, 2))
    vel = np.zeros((npart, 3))
    vel[:, :2] = rng.normal(size=(npart, 2))
    errs = []
    for N in (32, 64, 128):
        n = (N, N)
        g = O.make_grid(n)
        t = O.make_tabulated_map(2, n, (1, 1), O.sample_map_vertices(m, n, (1, 1)))
        u = xi0 * N
        idx = np.floor(u).astype(np.int64)
        cell = (idx[:, 0] + N * idx[:, 1]).astype(np.int32)
        off = np.zeros((npart, 3))
        off[:, :2] = u - idx
        Ev = np.zeros((N * N, 3))
        res = []
        for mm in (m, t):
            c, o, _, _ = O.push(mm, g, -1.0, 0.05, (0.0, 0.0, 0.0), cell, off, vel, Ev)
            ci = np.stack([c % N, c // N], axis=1)
            res.append((ci + o[:, :2]) / N)
        d = res[1] - res[0]
        d -= np.round(d)
        errs.append(np.abs(d).max())
    e = np.array(errs)
    scaled = e * np.array([32, 64, 128]) ** 2
    assert e[0] / e[-1] >= 8 and scaled.max() <= 2 * scaled.min(), (e, scaled)
