"""Pins for the oracle's gather (Eqs. vvp, Wvp, b1), Boris / leap-frog push
(Eqs. step1, step1a), position update with map inversion, and its
counter-based RNG.

Expected values: closed-form trajectories (uniform E, pure B, E x B drift),
free streaming, the interpolant's exactness on linear data, a separately
written Cartesian PIC (identity map), and published Philox4x32-10 known-answer
vectors."""
import math

import numpy as np
import pytest

import oracle as O


def test_philox_known_answer_vectors():
    # Random123 known-answer vectors for Philox4x32-10.
    kat = [
        ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
        ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
        ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
         [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
    ]
    for ctr, key, ref in kat:
        assert list(O.philox4x32_10(ctr, key)) == ref


def test_gather_reproduces_uniform_and_linear_fields():
    n = (7, 5)
    g = O.make_grid(n, bc_lo=(O.DIRICHLET, O.DIRICHLET), bc_hi=(O.DIRICHLET, O.DIRICHLET))
    nv = (8, 6)
    vi = np.arange(48)
    vx, vy = vi % 8, vi // 8
    rng = np.random.default_rng(0)
    cell = rng.integers(0, 35, 400).astype(np.int32)
    off = np.zeros((400, 3))
    off[:, :2] = rng.random((400, 2))
    Ev = np.zeros((48, 3))
    Ev[:, 0] = 0.3 + 1.5 * vx - 0.7 * vy
    Ev[:, 1] = -2.0
    Ev[:, 2] = 0.25 * vy
    Ep = O.gather(g, Ev, cell, off)
    X = cell % 7 + off[:, 0]
    Y = cell // 7 + off[:, 1]
    np.testing.assert_allclose(Ep[:, 0], 0.3 + 1.5 * X - 0.7 * Y, atol=1e-13)
    np.testing.assert_allclose(Ep[:, 1], -2.0, atol=1e-14)
    np.testing.assert_allclose(Ep[:, 2], 0.25 * Y, atol=1e-14)


def test_boris_pure_magnetic_rotation():
    B = np.array([0.0, 0.0, 2.0])
    qm, dt = -1.0, 0.1
    v = np.array([[1.0, 0.5, 0.3]])
    th = 2 * math.atan(abs(qm) * 2.0 * dt / 2)
    ang0 = math.atan2(v[0, 1], v[0, 0])
    for k in range(1, 200):
        v = O.boris(v, np.zeros((1, 3)), B, qm, dt)
        assert abs(np.linalg.norm(v) - math.sqrt(1.25 + 0.09)) < 1e-13
        ang = math.atan2(v[0, 1], v[0, 0])
        # electron (q/m < 0) gyrates counter-clockwise about +z
        d = (ang - ang0 - k * th + math.pi) % (2 * math.pi) - math.pi
        assert abs(d) < 1e-11
        assert abs(v[0, 2] - 0.3) < 1e-15


def test_boris_exb_drift():
    B = np.array([0.0, 0.0, 2.0])
    E = np.array([[0.3, 0.0, 0.0]])
    qm, dt = 1.0, 0.05
    v = np.array([[0.0, 0.0, 0.0]])
    vs = []
    for _ in range(20000):
        v = O.boris(v, E, B, qm, dt)
        vs.append(v[0].copy())
    mean = np.mean(vs, axis=0)
    drift = np.cross(E[0], B) / np.dot(B, B)
    np.testing.assert_allclose(mean[:2], drift[:2], atol=2e-3)


@pytest.mark.parametrize("kind,eps,L", [(O.IDENTITY, 0.0, (3.0, 2.0)),
                                        (O.SINUSOIDAL, 0.12, (3.0, 2.0))])
def test_uniform_field_leapfrog_trajectory_is_exact(kind, eps, L):
    # leap-frog with the half-step push-back is exact for constant acceleration:
    # x(t_n) = x0 + v0 t + a t^2 / 2, on any map (the position update is done in
    # physical space and mapped back).
    n = (12, 9)
    m = O.make_map(kind, 2, L, eps)
    g = O.make_grid(n)
    Ev = np.zeros((108, 3))
    Ev[:, 0] = 0.4
    Ev[:, 1] = -0.25
    rng = np.random.default_rng(3)
    npart = 200
    cell = rng.integers(0, 108, npart).astype(np.int32)
    off = np.zeros((npart, 3))
    off[:, :2] = rng.random((npart, 2))
    v0 = np.zeros((npart, 3))
    v0[:, :2] = rng.normal(size=(npart, 2)) * 0.5
    qm, dt = -1.0, 0.1
    xi0 = np.stack([(cell % 12 + off[:, 0]) / 12, (cell // 12 + off[:, 1]) / 9, 0 * off[:, 0]], 1)
    x0, *_ = O.map_eval(m, xi0)
    a = qm * np.array([0.4, -0.25, 0.0])
    vel = O.boris(v0, np.tile([0.4, -0.25, 0], (npart, 1)), np.zeros(3), qm, -0.5 * dt)
    for k in range(1, 31):
        cell, off, vel, _ = O.push(m, g, qm, dt, np.zeros(3), cell, off, vel, Ev)
        t = k * dt
        xi = np.stack([(cell % 12 + off[:, 0]) / 12, (cell // 12 + off[:, 1]) / 9, 0 * off[:, 0]], 1)
        x, *_ = O.map_eval(m, xi)
        ref = x0 + v0 * t + 0.5 * a * t * t
        d = (x - ref)[:, :2]
        d -= np.round(d / np.array(L)) * np.array(L)
        assert np.max(np.abs(d)) < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_free_streaming_matches_one_shot_inversion(dim):
    n = (10, 8) if dim == 2 else (6, 5, 7)
    L = tuple(float(v) for v in n)
    eps = 0.1 if dim == 2 else 0.05
    m = O.make_map(O.SINUSOIDAL, dim, L, eps)
    g = O.make_grid(n)
    nc = int(np.prod(n))
    rng = np.random.default_rng(4)
    npart = 300
    cell = rng.integers(0, nc, npart).astype(np.int32)
    off = np.zeros((npart, 3))
    off[:, :dim] = rng.random((npart, dim))
    vel = np.zeros((npart, 3))
    vel[:, :dim] = rng.normal(size=(npart, dim))
    Ev = np.zeros((nc, 3))

    def xi_of(cell, off):
        idx = []
        c = cell.copy()
        for a in range(dim):
            idx.append(c % n[a])
            c = c // n[a]
        xi = np.zeros((cell.size, 3))
        for a in range(dim):
            xi[:, a] = (idx[a] + off[:, a]) / n[a]
        return xi

    x0, *_ = O.map_eval(m, xi_of(cell, off))
    c, o, v = cell, off, vel
    dt = 0.1
    for k in range(1, 21):
        c, o, v, _ = O.push(m, g, -1.0, dt, np.zeros(3), c, o, v, Ev)
    xi_direct = O.map_invert(m, x0 + 20 * dt * vel)
    xi_direct[:, :dim] -= np.floor(xi_direct[:, :dim])
    d = xi_of(c, o)[:, :dim] - xi_direct[:, :dim]
    d -= np.round(d)
    assert np.max(np.abs(d)) < 1e-12
    np.testing.assert_array_equal(v, vel)


def _cartesian_pic(n, L, cell, off, vel, qm, w, q, dt, steps):
    """Independent periodic 2D Cartesian PIC in plain numpy: b2 deposit to cell
    centres, FFT solve of the 5-point Laplacian, vertex field from averaged
    cell-pair differences, CIC gather, leap-frog x += v dt."""
    nx, ny = n
    dx, dy = L[0] / nx, L[1] / ny
    X = (cell % nx + off[:, 0]) * dx
    Y = (cell // nx + off[:, 1]) * dy
    V = vel.copy()

    def b2w(f):
        return np.stack([0.5 * (1 - f) ** 2, 0.75 - (f - 0.5) ** 2, 0.5 * f ** 2])

    def fields(X, Y):
        ix = np.floor(X / dx).astype(int)
        iy = np.floor(Y / dy).astype(int)
        fx = X / dx - ix
        fy = Y / dy - iy
        wx, wy = b2w(fx), b2w(fy)
        rho = np.zeros((ny, nx))
        for a in range(3):
            for b in range(3):
                np.add.at(rho, ((iy + b - 1) % ny, (ix + a - 1) % nx), wx[a] * wy[b])
        rho = q * w * rho / (dx * dy) + 1.0  # neutralising background n0 = 1
        kx = np.fft.fftfreq(nx) * nx
        ky = np.fft.fftfreq(ny) * ny
        lam = ((2 * np.cos(2 * np.pi * kx / nx) - 2) / dx ** 2)[None, :] + \
              ((2 * np.cos(2 * np.pi * ky / ny) - 2) / dy ** 2)[:, None]
        lam[0, 0] = 1.0
        ph = np.fft.fft2(-rho) / lam
        ph[0, 0] = 0.0
        phi = np.real(np.fft.ifft2(ph))
        P = phi
        Pm = np.roll(P, 1, axis=1)
        Pmm = np.roll(np.roll(P, 1, axis=1), 1, axis=0)
        P0m = np.roll(P, 1, axis=0)
        Ex = -0.5 * ((P - Pm) + (P0m - Pmm)) / dx
        Ey = -0.5 * ((P - P0m) + (Pm - Pmm)) / dy
        E = np.zeros((X.size, 2))
        for a in range(2):
            for b in range(2):
                wgt = (fx if a else 1 - fx) * (fy if b else 1 - fy)
                E[:, 0] += wgt * Ex[(iy + b) % ny, (ix + a) % nx]
                E[:, 1] += wgt * Ey[(iy + b) % ny, (ix + a) % nx]
        return E, phi

    E, phi = fields(X, Y)
    V[:, :2] -= 0.5 * dt * qm * E
    for _ in range(steps):
        V[:, :2] += dt * qm * E
        X = (X + dt * V[:, 0]) % L[0]
        Y = (Y + dt * V[:, 1]) % L[1]
        E, phi = fields(X, Y)
    return X, Y, V, phi


def test_identity_map_reduces_to_cartesian_pic():
    n = (16, 8)
    L = (4.0, 2.0)
    m = O.make_map(O.IDENTITY, 2, L)
    g = O.make_grid(n)
    rng = np.random.default_rng(5)
    npart = 2000
    cell = rng.integers(0, 128, npart).astype(np.int32)
    off = np.zeros((npart, 3))
    off[:, :2] = rng.random((npart, 2))
    vel = np.zeros((npart, 3))
    vel[:, :2] = rng.normal(size=(npart, 2))
    w = L[0] * L[1] / npart
    sp = [dict(q=-1.0, m=1.0, w=w, cell=cell.copy(), off=off.copy(), vel=vel.copy())]
    nc = 128
    background = np.full(nc, L[0] * L[1] / nc)
    sim = O.OracleSim(m, g, sp, shape=O.B2, dt=0.1, background=background, deposit="f64",
                      rtol=1e-14)
    sim.initialize()
    for _ in range(8):
        sim.step()
    X, Y, V, phi = _cartesian_pic(n, L, cell, off, vel, -1.0, w, -1.0, 0.1, 8)
    s = sim.sp[0]
    Xo = (s["cell"] % 16 + s["off"][:, 0]) * L[0] / 16
    Yo = (s["cell"] // 16 + s["off"][:, 1]) * L[1] / 8
    dx = (Xo - X + L[0] / 2) % L[0] - L[0] / 2
    dy = (Yo - Y + L[1] / 2) % L[1] - L[1] / 2
    assert np.max(np.abs(dx)) < 1e-10 and np.max(np.abs(dy)) < 1e-10
    np.testing.assert_allclose(s["vel"][:, :2], V[:, :2], atol=1e-10)
    np.testing.assert_allclose(sim.phi, phi.ravel() - phi.mean(), atol=1e-10)
