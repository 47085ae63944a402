"""Pins for the oracle's maps and metrics (Sec. II.A, Eqs. map, jcov, jcon, jac,
gcon, map2) and its map inversion.  Every expected value here is a closed form
derived from the map's formula, not a re-evaluation of the oracle's code."""
import math

import numpy as np
import pytest

import oracle as O
from _golden import paper_value

pytestmark = pytest.mark.filterwarnings("ignore")


def rand_xi(n, d, seed=0):
    r = np.random.default_rng(seed).random((n, d))
    out = np.zeros((n, 3))
    out[:, :d] = r
    return out


def test_sinusoidal_2d_jacobian_closed_form():
    # x = xi + eps s(2 pi xi) s(2 pi eta), y = eta + eps s s  (Eq. map2):
    # det = 1 + 2 pi eps sin 2 pi (xi + eta) by the matrix-determinant lemma.
    eps = 0.1
    m = O.make_map(O.SINUSOIDAL, 2, (1.0, 1.0), eps)
    xi = rand_xi(500, 2)
    _, _, _, J = O.map_eval(m, xi)
    ref = 1 + 2 * np.pi * eps * np.sin(2 * np.pi * (xi[:, 0] + xi[:, 1]))
    np.testing.assert_allclose(J, ref, rtol=0, atol=1e-14)
    # physical scaling L^2
    m2 = O.make_map(O.SINUSOIDAL, 2, (3.0, 5.0), eps)
    _, _, _, J2 = O.map_eval(m2, xi)
    np.testing.assert_allclose(J2, 15.0 * ref, rtol=1e-14)


def test_cell_size_ratio_printed_in_paper():
    # the paper gives the largest-to-smallest cell size ratio of the eps = 0.1
    # map to one decimal (tests/golden); J ranges over [1 - 2 pi eps, 1 + 2 pi eps]
    m = O.make_map(O.SINUSOIDAL, 2, (1.0, 1.0), 0.1)
    g = (np.arange(400) + 0.5) / 400
    X, Y = np.meshgrid(g, g, indexing="ij")
    xi = np.stack([X.ravel(), Y.ravel(), 0 * X.ravel()], axis=1)
    _, _, _, J = O.map_eval(m, xi)
    ratio = J.max() / J.min()
    assert abs(ratio - (1 + 0.2 * np.pi) / (1 - 0.2 * np.pi)) < 2e-3
    assert round(ratio, 1) == paper_value("cell_size_ratio_eps_0.1")


def test_sinusoidal_3d_jacobian_closed_form_and_singular_eps():
    eps = 0.05
    m = O.make_map(O.SINUSOIDAL, 3, (1.0, 1.0, 1.0), eps)
    xi = rand_xi(500, 3, 1)
    _, _, _, J = O.map_eval(m, xi)
    s = np.sin(2 * np.pi * xi)
    c = np.cos(2 * np.pi * xi)
    ref = 1 + 2 * np.pi * eps * (c[:, 0] * s[:, 1] * s[:, 2] + s[:, 0] * c[:, 1] * s[:, 2] +
                                 s[:, 0] * s[:, 1] * c[:, 2])
    np.testing.assert_allclose(J, ref, atol=1e-14)
    # range of J: the bracket is at most 2/sqrt 3 in modulus (all three angles
    # equal with tan^2 = 2), so J in [0.637, 1.363] at eps = 0.05 and the map
    # folds at eps = sqrt(3) / (4 pi) = 0.1378.
    bound = 2 / math.sqrt(3)
    assert J.min() >= 1 - 2 * np.pi * eps * bound - 1e-12
    assert J.max() <= 1 + 2 * np.pi * eps * bound + 1e-12
    th = math.atan(math.sqrt(2.0))
    xi_max = np.array([[th / (2 * np.pi)] * 3])
    _, _, _, Jm = O.map_eval(m, xi_max)
    assert abs(Jm[0] - (1 + 2 * np.pi * eps * bound)) < 1e-14
    assert abs(Jm[0] - 1.363) < 1e-3
    assert abs(math.sqrt(3) / (4 * np.pi) - 0.1378) < 1e-4


@pytest.mark.parametrize("kind,dim,L,eps", [(O.SINUSOIDAL, 2, (1.0, 1.0), 0.12),
                                            (O.SINUSOIDAL, 3, (4.0, 2.0, 3.0), 0.05),
                                            (O.POLAR_LOG, 2, (1.0, 1.0), 0.0),
                                            (O.IDENTITY, 3, (2.0, 3.0, 5.0), 0.0),
                                            (O.SPHERICAL_RZ, 2, (1.0, 1.0), 0.0)])
def test_jacobi_matrix_matches_finite_differences_and_inverse(kind, dim, L, eps):
    m = O.make_map(kind, dim, L, eps, r_in=1.0, r_out=10.0)
    xi = rand_xi(64, dim, 2) * 0.9 + 0.05
    xi[:, dim:] = 0
    x, j, k, J = O.map_eval(m, xi)
    h = 1e-6
    for b in range(dim):
        e = np.zeros(3)
        e[b] = h
        xp, *_ = O.map_eval(m, xi + e)
        xm, *_ = O.map_eval(m, xi - e)
        fd = (xp - xm) / (2 * h)
        np.testing.assert_allclose(j[:, :dim, b], fd[:, :dim], rtol=1e-7, atol=1e-7 * max(L))
    jk = np.einsum("nab,nbc->nac", j[:, :dim, :dim], k[:, :dim, :dim])
    np.testing.assert_allclose(jk, np.broadcast_to(np.eye(dim), jk.shape), atol=1e-12)
    np.testing.assert_allclose(J, np.linalg.det(j[:, :dim, :dim]), rtol=1e-12)


def test_sherman_morrison_inverse_closed_form():
    # box units: j = I + eps 1 grad(P)^T -> k = I - (eps / J) 1 grad(P)^T
    eps = 0.05
    m = O.make_map(O.SINUSOIDAL, 3, (1.0, 1.0, 1.0), eps)
    xi = rand_xi(100, 3, 3)
    _, _, k, J = O.map_eval(m, xi)
    s = np.sin(2 * np.pi * xi)
    c = np.cos(2 * np.pi * xi)
    gP = 2 * np.pi * np.stack([c[:, 0] * s[:, 1] * s[:, 2], s[:, 0] * c[:, 1] * s[:, 2],
                               s[:, 0] * s[:, 1] * c[:, 2]], axis=1)
    ref = np.eye(3)[None] - (eps / J)[:, None, None] * np.ones((1, 3, 1)) * gP[:, None, :]
    np.testing.assert_allclose(k, ref, atol=1e-13)


def test_polar_log_is_conformal_with_constant_coefficients():
    # r = r_in R^xi, theta = 2 pi eta:  J = 2 pi ln R r^2, J g^11 = 2 pi / ln R,
    # J g^22 = ln R / (2 pi), J g^12 = 0.
    m = O.make_map(O.POLAR_LOG, 2, r_in=1.0, r_out=60.0)
    xi = rand_xi(200, 2, 4)
    x, _, _, J = O.map_eval(m, xi)
    r = np.hypot(x[:, 0], x[:, 1])
    lnR = math.log(60.0)
    np.testing.assert_allclose(J, 2 * np.pi * lnR * r ** 2, rtol=1e-13)
    a = O.coef_eval(m, xi)
    np.testing.assert_allclose(a[:, 0, 0], 2 * np.pi / lnR, rtol=1e-12)
    np.testing.assert_allclose(a[:, 1, 1], lnR / (2 * np.pi), rtol=1e-12)
    np.testing.assert_allclose(a[:, 0, 1], 0.0, atol=1e-12)
    assert abs(2 * np.pi / lnR - 1.5346) < 1e-4 and abs(lnR / (2 * np.pi) - 0.6516) < 1e-4


def test_coefficient_is_J_times_contravariant_metric():
    m = O.make_map(O.SINUSOIDAL, 2, (2.0, 3.0), 0.1)
    xi = rand_xi(50, 2, 5)
    _, j, _, J = O.map_eval(m, xi)
    a = O.coef_eval(m, xi)
    for p in range(50):
        jj = j[p, :2, :2]
        g_cov = jj.T @ jj  # Eq. gcov
        ref = J[p] * np.linalg.inv(g_cov)  # g^ij is the inverse of g_ij
        np.testing.assert_allclose(a[p, :2, :2], ref, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("dim,eps,L", [(2, 0.15, (1.0, 1.0)), (3, 0.05, (7.0, 5.0, 3.0)),
                                       (2, 0.1, (32.0, 24.0))])
def test_inversion_round_trip(dim, eps, L):
    m = O.make_map(O.SINUSOIDAL, dim, L, eps)
    xi = rand_xi(2000, dim, 6) * 3 - 1  # unbounded logical positions
    xi[:, dim:] = 0
    x, *_ = O.map_eval(m, xi)
    back = O.map_invert(m, x)
    np.testing.assert_allclose(back[:, :dim], xi[:, :dim], atol=1e-13)


def test_inversion_polar_and_free_streaming_invariant():
    m = O.make_map(O.POLAR_LOG, 2, r_in=1.0, r_out=60.0)
    xi = rand_xi(500, 2, 7)
    x, *_ = O.map_eval(m, xi)
    back = O.map_invert(m, x, xi)
    np.testing.assert_allclose(back[:, :2], xi[:, :2], atol=1e-13)
    # 2D sinusoidal map: x - y = L (xi - eta) exactly, so free streaming
    # conserves xi - eta - (x - y)/L along the physical straight line.
    L = 1.0
    m = O.make_map(O.SINUSOIDAL, 2, (L, L), 0.1)
    xi0 = rand_xi(300, 2, 8)
    x0, *_ = O.map_eval(m, xi0)
    v = np.random.default_rng(9).normal(size=(300, 3))
    v[:, 2] = 0
    for t in (0.05, 0.5, 3.0):
        xi_t = O.map_invert(m, x0 + t * v)
        lhs = xi_t[:, 0] - xi_t[:, 1]
        rhs = (x0[:, 0] + t * v[:, 0] - x0[:, 1] - t * v[:, 1]) / L
        np.testing.assert_allclose(lhs, rhs, atol=1e-13)
