"""Flux injection of the oracle: the Maxwellian source at the outer boundary of
the probe problems (Sec. "Tests": the plasma is supplied by injecting a
Maxwellian flux through the outer boundary), pinned by what kinetic theory of
a half-Maxwellian flux fixes:
  - the mean number injected per step is lambda = n0 v_th / sqrt(2 pi) A dt / w;
  - the inward normal velocity is Rayleigh distributed: mean v_th sqrt(pi/2),
    P(v_n > a) = exp(-a^2 / 2 v_th^2); tangential components are N(0, v_th^2);
  - with no field, from an empty slab, the density at depth s after time T is
    n0/2 erfc(s / (sqrt(2) v_th T)): the steady value n0/2 (only the inward
    half of the Maxwellian is present) reached from the face inwards."""
import math

import numpy as np

import oracle as O

N0, VTH = 1.0, 1.0


def _slab(n=(40, 8), L=(40.0, 8.0)):
    m = O.make_map(O.IDENTITY, 2, L=L)
    g = O.make_grid(n, bc_lo=(1, 0), bc_hi=(1, 0))
    return m, g


def _lam(area, dt, w, vth=VTH):
    return N0 * vth / math.sqrt(2 * math.pi) * area * dt / w


def test_face_area():
    assert O.face_area(O.make_map(O.IDENTITY, 2, L=(40.0, 8.0))) == 8.0
    assert O.face_area(O.make_map(O.IDENTITY, 3, L=(4.0, 3.0, 5.0))) == 15.0
    m = O.make_map(O.POLAR_LOG, 2, r_in=1.0, r_out=60.0)
    assert abs(O.face_area(m) - 2 * math.pi * 60.0) < 1e-12


def test_count_mean_is_lambda():
    m, g = _slab()
    dt, w = 0.1, 0.37
    lam = _lam(8.0, dt, w)
    counts = np.array([O.inject(m, g, N0, VTH, w, dt, seed=11, step=k, species=0, cap=16)[3]
                       for k in range(4000)])
    fl = math.floor(lam)
    assert set(np.unique(counts).tolist()) <= {fl, fl + 1}
    p = lam - fl
    assert abs(counts.mean() - lam) < 4 * math.sqrt(p * (1 - p) / counts.size)
    # a larger lambda: floor(lambda) always, plus the Bernoulli remainder
    w2 = 8.0 * 0.1 * N0 * VTH / math.sqrt(2 * math.pi) / 12.25
    c2 = np.array([O.inject(m, g, N0, VTH, w2, dt, seed=3, step=k, species=1, cap=64)[3]
                   for k in range(2000)])
    assert set(np.unique(c2).tolist()) <= {12, 13}
    assert abs(c2.mean() - 12.25) < 4 * math.sqrt(0.25 * 0.75 / c2.size)


def _one_big_injection(m, g, area, dt, lam_target, seed=5, vth=VTH):
    w = N0 * vth / math.sqrt(2 * math.pi) * area * dt / lam_target
    cell, off, vel, drawn, k = O.inject(m, g, N0, vth, w, dt, seed=seed, step=0, species=0,
                                        cap=1 << 20, with_index=True)
    return cell, off, vel, drawn, k


def test_velocity_distribution_of_a_half_maxwellian_flux():
    m, g = _slab()
    dt = 0.1
    cell, off, vel, drawn, k = _one_big_injection(m, g, 8.0, dt, 200000.5)
    n = cell.size
    assert n == drawn  # nothing leaves the slab during the free-streaming start
    assert np.array_equal(k, np.arange(n))
    vn = -vel[:, 0]
    assert np.all(vn > 0)
    sd = VTH * math.sqrt((4 - math.pi) / 2)
    assert abs(vn.mean() - VTH * math.sqrt(math.pi / 2)) < 4 * sd / math.sqrt(n)
    for a in (0.5, 1.0, 2.0):
        p = math.exp(-a * a / 2)
        assert abs(np.mean(vn > a) - p) < 4 * math.sqrt(p * (1 - p) / n)
    for c in (1, 2):
        assert abs(vel[:, c].mean()) < 4 * VTH / math.sqrt(n)
        assert abs(vel[:, c].var() - VTH ** 2) < 4 * VTH ** 2 * math.sqrt(2.0 / n)
    # tangential position uniform; depth = U dt v_n with U uniform on (0, 1)
    y = (cell // 40 + off[:, 1]) / 8.0
    h, _ = np.histogram(y, bins=16, range=(0, 1))
    assert np.all(np.abs(h - n / 16) < 5 * math.sqrt(n / 16))
    x = (cell % 40 + off[:, 0]) * 1.0
    u = (40.0 - x) / (dt * vn)
    assert np.all((u > 0) & (u < 1 + 1e-9))
    h, _ = np.histogram(u, bins=10, range=(0, 1))
    assert np.all(np.abs(h - n / 10) < 5 * math.sqrt(n / 10))


def test_polar_injection_is_radially_inward_at_the_outer_circle():
    m = O.make_map(O.POLAR_LOG, 2, r_in=1.0, r_out=60.0)
    g = O.make_grid((64, 48), bc_lo=(1, 0), bc_hi=(1, 0))
    dt = 0.1
    cell, off, vel, drawn, k = _one_big_injection(m, g, 2 * math.pi * 60.0, dt, 50000.0, seed=9)
    n = cell.size
    xi = np.zeros((n, 3))
    xi[:, 0] = (cell % 64 + off[:, 0]) / 64
    xi[:, 1] = (cell // 64 + off[:, 1]) / 48
    x, *_ = O.map_eval(m, xi)
    r = np.hypot(x[:, 0], x[:, 1])
    assert np.all(r < 60.0) and np.all(r > 60.0 - dt * 8.0)
    # v_r is taken along the particle's own radial direction, which differs
    # from that of its entry point by O(dt v_t / r_out)
    vr = (vel[:, 0] * x[:, 0] + vel[:, 1] * x[:, 1]) / r
    assert abs(-vr.mean() - VTH * math.sqrt(math.pi / 2)) < 5 * VTH / math.sqrt(n) + 2e-3
    th = np.mod(np.arctan2(x[:, 1], x[:, 0]) / (2 * math.pi), 1.0)
    h, _ = np.histogram(th, bins=12, range=(0, 1))
    assert np.all(np.abs(h - n / 12) < 5 * math.sqrt(n / 12))


def test_free_streaming_density_from_an_empty_slab():
    n, L = (40, 8), (40.0, 8.0)
    m, g = _slab(n, L)
    dt, K, w = 0.1, 300, 2e-3
    nv = (n[0] + 1) * n[1]
    E0 = np.zeros((nv, 3))
    cell = np.zeros(0, dtype=np.int32)
    off = np.zeros((0, 3))
    vel = np.zeros((0, 3))
    absorbed = 0
    for k in range(K):
        if cell.size:
            cell, off, vel, cnt = O.push(m, g, -1.0, dt, (0.0, 0.0, 0.0), cell, off, vel, E0)
            assert cnt[1] == 0  # nothing moves outwards
            absorbed += cnt[0]
            alive = cell >= 0
            cell, off, vel = cell[alive], off[alive], vel[alive]
        c, o, v, _ = O.inject(m, g, N0, VTH, w, dt, seed=21, step=k, species=0)
        cell = np.concatenate([cell, c])
        off = np.concatenate([off, o])
        vel = np.concatenate([vel, v])
    T = K * dt
    s = L[0] - (cell % n[0] + off[:, 0]) * (L[0] / n[0])
    edges = np.arange(0.0, 22.0, 2.0)
    h, _ = np.histogram(s, bins=edges)
    area = 2.0 * L[1]
    for b in range(h.size):
        ss = np.linspace(edges[b], edges[b + 1], 201)
        expect = np.mean([0.5 * N0 * math.erfc(t / (math.sqrt(2) * VTH * T)) for t in ss])
        mean_count = expect * area / w
        assert abs(h[b] - mean_count) < 5 * math.sqrt(mean_count), (b, h[b], mean_count)
    # the fast tail has reached the far wall and was absorbed there
    assert absorbed > 0
