"""Pins for the oracle's charge deposit (Eqs. pg, Wpc, b2 with the continuous
order-2 B-spline; CIC variant) and the fixed neutralising background.

Expected values come from exact rational arithmetic (Python Fractions), from
integer identities (total charge), from the spline's moments, or from the
Gauss-Legendre rule's known exactness -- never from the oracle itself."""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def frac_rint(x: Fraction) -> int:
    """Round-half-even of an exact rational."""
    fl = x.numerator // x.denominator
    rem = x - fl
    if rem > Fraction(1, 2):
        return fl + 1
    if rem < Fraction(1, 2):
        return fl
    return fl if fl % 2 == 0 else fl + 1


def exact_weights(shape, S1, f):
    """Integer per-axis weights from the exact value of f (a float)."""
    F = Fraction(f)
    one = 1 << S1
    if shape == O.B2:
        L = frac_rint((1 - F) ** 2 * Fraction(1 << (S1 - 1)))
        R = frac_rint(F ** 2 * Fraction(1 << (S1 - 1)))
        return [L, one - L - R, R]
    g = F - Fraction(1, 2)
    if g >= 0:
        R = frac_rint(g * one)
        return [0, one - R, R]
    Lw = frac_rint(-g * one)
    return [Lw, one - Lw, 0]


def random_particles(g, n, seed, f32=True):
    rng = np.random.default_rng(seed)
    d = g.dim
    nc = O.ncells(g)
    cell = rng.integers(0, nc, n).astype(np.int32)
    off = np.zeros((n, 3))
    o = rng.random((n, d))
    if f32:
        o = o.astype(np.float32).astype(np.float64)
    off[:, :d] = o
    return cell, off


@pytest.mark.parametrize("dim,shape", [(2, O.B2), (2, O.B1), (3, O.B2), (3, O.B1)])
def test_total_charge_is_exact_integer(dim, shape):
    n = (13, 7) if dim == 2 else (6, 5, 7)
    g = O.make_grid(n)
    S1 = 24 if dim == 2 else 16
    cell, off = random_particles(g, 5000, 1)
    Q = O.deposit_fixed(g, shape, S1, cell, off)
    total = sum(int(q) for q in Q)
    assert total == 5000 * (1 << (dim * S1))


@pytest.mark.parametrize("dim", [2, 3])
def test_permutation_invariance_bitwise(dim):
    n = (9, 11) if dim == 2 else (5, 6, 4)
    g = O.make_grid(n)
    S1 = 24 if dim == 2 else 16
    cell, off = random_particles(g, 3000, 2)
    Q1 = O.deposit_fixed(g, O.B2, S1, cell, off)
    perm = np.random.default_rng(3).permutation(3000)
    Q2 = O.deposit_fixed(g, O.B2, S1, cell[perm], off[perm])
    assert np.array_equal(Q1, Q2)


@pytest.mark.parametrize("shape", [O.B2, O.B1])
def test_brute_force_three_particles_against_exact_rationals(shape):
    g = O.make_grid((5, 4, 6))
    S1 = 16
    cell, off = random_particles(g, 3, 4)
    Q = O.deposit_fixed(g, shape, S1, cell, off)
    ref = np.zeros(O.ncells(g), dtype=object)
    ref[:] = 0
    for p in range(3):
        c = int(cell[p])
        idx = [c % 5, (c // 5) % 4, c // 20]
        w = [exact_weights(shape, S1, off[p, a]) for a in range(3)]
        for oz in range(3):
            for oy in range(3):
                for ox in range(3):
                    t = [(idx[0] + ox - 1) % 5, (idx[1] + oy - 1) % 4, (idx[2] + oz - 1) % 6]
                    ref[t[0] + 5 * (t[1] + 4 * t[2])] += w[0][ox] * w[1][oy] * w[2][oz]
    assert [int(q) for q in Q] == list(ref)


def test_cell_centre_weights_and_face_continuity():
    g = O.make_grid((8,) * 2)
    S1 = 24
    # particle at a cell centre: b2 weights (1/8, 3/4, 1/8) per axis
    Q = O.deposit_fixed(g, O.B2, S1, np.array([3 + 8 * 4], np.int32), np.array([[0.5, 0.5, 0]]))
    one = 1 << S1
    w = [one // 8, 3 * one // 4, one // 8]
    Qm = Q.reshape(8, 8)  # [j, i]
    for a in range(3):
        for b in range(3):
            assert int(Qm[3 + a, 2 + b]) == w[a] * w[b]
    # continuity: f -> 1 in cell i equals f = 0 in cell i + 1
    f_hi = np.nextafter(1.0, 0.0)
    for shape in (O.B2, O.B1):
        Qa = O.deposit_fixed(g, shape, S1, np.array([2 + 8 * 2], np.int32), np.array([[f_hi, 0.3, 0]]))
        Qb = O.deposit_fixed(g, shape, S1, np.array([3 + 8 * 2], np.int32), np.array([[0.0, 0.3, 0]]))
        assert np.array_equal(Qa, Qb)


def test_spline_moments():
    # 1D (second axis fixed at the cell centre): zeroth moment 1 and first
    # moment about the particle 0 for both shapes (partition of unity, linear
    # reproduction); second moment exactly 1/4 cell^2 for b2 at any offset
    # (quadratic reproduction).  For CIC to cell centres the second moment is
    # (1 - |g|) g^2 + |g| (1 - |g|)^2 = |g| (1 - |g|), g = f - 1/2.
    g = O.make_grid((16, 4))
    S1 = 24
    one = float(1 << S1) ** 2
    rng = np.random.default_rng(5)
    for f in rng.random(50):
        f = float(np.float32(f))
        cell = np.array([7 + 16 * 1], np.int32)
        off = np.array([[f, 0.5, 0.0]])
        for shape in (O.B2, O.B1):
            Q = O.deposit_fixed(g, shape, S1, cell, off).reshape(4, 16).sum(axis=0) / one
            xc = np.arange(16) + 0.5
            xp = 7 + f
            m0 = Q.sum()
            m1 = (Q * (xc - xp)).sum()
            m2 = (Q * (xc - xp) ** 2).sum()
            assert abs(m0 - 1) < 1e-15
            assert abs(m1) < 3 * 2.0 ** -S1
            gg = abs(f - 0.5)
            ref2 = 0.25 if shape == O.B2 else gg * (1 - gg)
            assert abs(m2 - ref2) < 8 * 2.0 ** -S1


def test_plain_f64_deposit_matches_fixed_within_quantisation():
    g = O.make_grid((10, 9, 8))
    cell, off = random_particles(g, 2000, 6)
    S1 = 16
    Qi = O.deposit_fixed(g, O.B2, S1, cell, off).astype(np.float64) * 2.0 ** (-3 * S1)
    Qf = O.deposit_f64(g, O.B2, cell, off)
    assert abs(Qf.sum() - 2000) < 1e-9
    # per particle per target at most 3 half-units of 2^-S1 per factor
    assert np.max(np.abs(Qi - Qf)) < 2000 * 27 * 3 * 2.0 ** -S1


def test_bounded_axis_folds_ghost_targets():
    g = O.make_grid((6, 5), bc_lo=(O.DIRICHLET, 0), bc_hi=(O.DIRICHLET, 0))
    cell, off = random_particles(g, 500, 7)
    Q = O.deposit_fixed(g, O.B2, 24, cell, off)
    assert sum(int(q) for q in Q) == 500 << 48


def test_gauss_legendre_8_exactness():
    x, w = O.gl8()
    assert abs(w.sum() - 2.0) < 1e-15
    for k in range(16):
        ref = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - ref) < 1e-14


@pytest.mark.parametrize("shape", [O.B2, O.B1])
def test_background_total_is_physical_volume(shape):
    # sum_c I_c = n0 * int J = n0 * volume (partition of unity of the shape)
    m = O.make_map(O.SINUSOIDAL, 2, (3.0, 2.0), 0.1)
    g = O.make_grid((16, 12))
    I = O.ion_background(m, g, shape, n0=1.0)
    assert abs(I.sum() - 6.0) < 1e-13
    # undistorted map: every cell holds exactly n0 dV
    m0 = O.make_map(O.IDENTITY, 2, (3.0, 2.0), 0.0)
    I0 = O.ion_background(m0, g, shape, n0=1.0)
    np.testing.assert_allclose(I0, 6.0 / 192, rtol=1e-13)


def _spline_ft(shape, k):
    """Fourier transform at wavenumber k (radians per cell) of the unit-area
    B-spline of the deposit: the box function convolved with itself once (b1,
    the CIC hat) or twice (b2), so sinc(k/2)^2 resp. ^3."""
    s = np.sinc(k / (2.0 * np.pi))  # numpy's sinc is sin(pi x) / (pi x)
    return s ** (3 if shape == O.B2 else 2)


@pytest.mark.parametrize("shape", [O.B2, O.B1])
def test_background_per_cell_closed_form_2d(shape):
    # Sinusoidal map (Eq. map2) in box units: J = 1 + 2 pi eps sin 2 pi (xi + eta),
    # a single Fourier mode.  The shape is even, so its integral against
    # sin(theta_c + k u) is sin(theta_c) times the spline's transform at k:
    #   I_c = n0 dV [1 + 2 pi eps sin 2 pi (xi_c + eta_c) * prod_a FT(2 pi h_a)]
    # with (xi_c, eta_c) the cell centre and h_a = 1 / n_a in box units.  A node
    # set shifted by half a cell, a wrong spline order or a dropped Jacobian
    # factor all move I_c by far more than the tolerance.
    L, eps, n = (3.0, 2.0), 0.1, (16, 12)
    m = O.make_map(O.SINUSOIDAL, 2, L, eps)
    g = O.make_grid(n)
    I = O.ion_background(m, g, shape, n0=1.7)
    i, j = np.meshgrid(np.arange(n[0]), np.arange(n[1]), indexing="ij")
    xc, yc = (i + 0.5) / n[0], (j + 0.5) / n[1]
    damp = _spline_ft(shape, 2 * np.pi / n[0]) * _spline_ft(shape, 2 * np.pi / n[1])
    dV = L[0] * L[1] / (n[0] * n[1])
    ref = 1.7 * dV * (1.0 + 2 * np.pi * eps * np.sin(2 * np.pi * (xc + yc)) * damp)
    # cell c = i + n0 j
    got = I.reshape(n[1], n[0]).T
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=0)


def test_background_per_cell_closed_form_3d():
    # 3D map x^i = L (xi^i + eps s1 s2 s3): J = 1 + 2 pi eps (c1 s2 s3 + s1 c2 s3
    # + s1 s2 c3) in box units; each term is a product of one cosine and two
    # sines of the three axes, so every axis contributes its factor FT(2 pi h_a).
    eps, n = 0.05, (6, 5, 4)
    m = O.make_map(O.SINUSOIDAL, 3, (1.0, 1.0, 1.0), eps)
    g = O.make_grid(n)
    I = O.ion_background(m, g, O.B2, n0=1.0)
    i, j, k = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij")
    a = [2 * np.pi * (i + 0.5) / n[0], 2 * np.pi * (j + 0.5) / n[1], 2 * np.pi * (k + 0.5) / n[2]]
    s, c = [np.sin(t) for t in a], [np.cos(t) for t in a]
    P = c[0] * s[1] * s[2] + s[0] * c[1] * s[2] + s[0] * s[1] * c[2]
    damp = np.prod([_spline_ft(O.B2, 2 * np.pi / nn) for nn in n])
    ref = (1.0 + 2 * np.pi * eps * P * damp) / (n[0] * n[1] * n[2])
    got = I.reshape(n[2], n[1], n[0]).transpose(2, 1, 0)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=0)
