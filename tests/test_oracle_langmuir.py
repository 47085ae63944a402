"""The Langmuir-frequency pin: a cold plasma on the distorted map of the 2D
Langmuir workload oscillates at the plasma frequency.  Leap-frog shifts it to
(2/dt) asin(dt/2) = 1.000417 at omega_pe dt = 0.1; the finite-grid correction
at k h = 2 pi / 32 is a few tenths of a percent.  Also checks the loader's
distributions (uniform physical density, Maxwellian variance)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1311_2286_amd import workloads as W


def run_oracle_case(case, steps, shape=O.B2):
    m = O.make_map(**case.map_args())
    g = O.make_grid(**case.grid_args())
    sp = []
    for sid, s in enumerate(case.species):
        p = W.to_oracle(W.generate_species(case, sid, dtype=np.float64))
        sp.append(dict(q=s.q, m=s.m, w=case.weight(s), **p))
    bg = O.ion_background(m, g, shape) if case.background else None
    sim = O.OracleSim(m, g, sp, shape=shape, dt=case.dt, background=bg, rtol=1e-12)
    sim.initialize()
    n = case.n
    xi = np.zeros((case.ncells, 3))
    ii = np.arange(case.ncells)
    xi[:, 0] = (ii % n[0] + 0.5) / n[0]
    xi[:, 1] = (ii // n[0] + 0.5) / n[1]
    x, _, _, J = O.map_eval(m, xi)
    weight = np.cos(2 * np.pi * x[:, 0] / case.L[0]) * J / case.ncells
    amps = [float(np.dot(sim.phi, weight))]
    totals = []
    for _ in range(steps):
        sim.step()
        amps.append(float(np.dot(sim.phi, weight)))
        totals.append(sum(int(q) for q in sim.Q[0]))
    return np.array(amps), totals, sim


def fit_frequency(a, dt):
    t = np.arange(a.size) * dt
    best = None
    for w in np.linspace(0.9, 1.1, 4001):
        M = np.stack([np.cos(w * t), np.sin(w * t), np.ones_like(t)], axis=1)
        coef, res, *_ = np.linalg.lstsq(M, a, rcond=None)
        r = np.sum((M @ coef - a) ** 2)
        if best is None or r < best[0]:
            best = (r, w)
    return best[1]


def test_cold_langmuir_oscillates_at_omega_pe():
    case = W.case1_cold()
    amps, totals, sim = run_oracle_case(case, case.steps)
    w = fit_frequency(amps, case.dt)
    w_lf = (2 / case.dt) * math.asin(case.dt / 2)
    assert abs(w_lf - 1.000417) < 1e-6
    assert abs(w / w_lf - 1) < 0.01, w
    # total deposited charge is an exact integer identity every step
    N = case.count(case.species[0])
    assert all(t == N << 48 for t in totals)


def test_loader_distributions():
    case = W.case1()
    p = W.generate_species(case, 0, dtype=np.float64)
    m = O.make_map(**case.map_args())
    o = W.to_oracle(p)
    n = case.n
    xi = np.zeros((o["cell"].size, 3))
    xi[:, 0] = (o["cell"] % n[0] + o["off"][:, 0]) / n[0]
    xi[:, 1] = (o["cell"] // n[0] + o["off"][:, 1]) / n[1]
    x, *_ = O.map_eval(m, xi)
    # physical density: uniform in y, 1 + 0.01 cos(2 pi x) in x
    N = x.shape[0]
    hy, _ = np.histogram(x[:, 1] % 1.0, bins=16, range=(0, 1))
    expect = N / 16
    assert np.max(np.abs(hy - expect)) < 5 * math.sqrt(expect)
    c1 = np.mean(np.cos(2 * np.pi * x[:, 0]))
    assert abs(c1 - 0.005) < 4 / math.sqrt(2 * N)
    v2 = np.mean(np.sum(o["vel"] ** 2, axis=1))
    assert abs(v2 - 3.0) < 3 * math.sqrt(6.0 / N) * 3
