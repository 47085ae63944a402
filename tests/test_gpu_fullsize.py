"""Parity at the full size of the benchmark workload (3D periodic box, 128^3
cells, 32 electrons + 32 ions per cell: 134,217,728 particles, FP32 particles
with the fixed-point b2 deposit), in the launch configuration the benchmark
times (tiles of 8^3 cells, work items of at most 16,384 particles).

Checked against the oracle where it can afford the full size, else on samples
it computes one by one, else through properties:
  - deposit of every particle: Q bit-exact against the oracle's fixed-point
    deposit of the same positions, per species (all 2,097,152 cells);
  - charge per cell within 1e-14 relative of the oracle's sum q w Q;
  - Poisson solve: the GPU potential solves the oracle's own discrete system
    (its residual in the oracle's operator below 1e-9 of the right side) --
    a full oracle solve at this size takes minutes;
  - vertex field of a synthetic potential within 1e-6 of its maximum;
  - one push in a synthetic vertex field: 32,768 particles per species, drawn
    at random, against the oracle's push of the same particles (positions
    2e-5 cell, velocities 2e-5 (|v| + |q/m E dt|)), and the exact total of
    the deposit after the push (N 2^{3 S1})."""
import time

import numpy as np
import pytest

import oracle as O
from paper_1311_2286_amd import workloads as W
from _helpers import gpu_sim, oracle_objects, logical_cells, periodic_diff

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def C():
    from paper_1311_2286_amd import cpic
    return cpic


def say(t0, msg):
    print("[fullsize %6.1f s] %s" % (time.time() - t0, msg), flush=True)


def test_box3d_128_full_size():
    t0 = time.time()
    case = W.case2()
    assert case.n == (128, 128, 128) and sum(case.count(s) for s in case.species) == 134217728
    sim, parts = gpu_sim(case, precision=0, shape=2, track_ids=True, mg_rtol=1e-10, mg_max_cycles=60,
                         sort_every=4)
    m, g = oracle_objects(case)
    S1 = 16
    say(t0, "loaded %d particles" % sum(p["cell"].size for p in parts))

    # deposit: every cell, bit-exact
    sim.stage(C().STAGE_DEPOSIT)
    charge_o = np.zeros(case.ncells)
    for sid, s in enumerate(case.species):
        o = W.to_oracle(parts[sid])
        Qo = O.deposit_fixed(g, 2, S1, o["cell"], o["off"])
        Qg = sim.get_field(C().FIELD_Q, sid)
        assert np.array_equal(Qg, Qo), sid
        assert int(Qo.astype(object).sum()) == parts[sid]["cell"].size << (3 * S1)
        charge_o += s.q * case.weight(s) * Qo.astype(np.float64) * 2.0 ** (-3 * S1)
        del o, Qo, Qg
        say(t0, "deposit of species %d bit-exact" % sid)
    sim.stage(C().STAGE_CHARGE)
    ch = sim.get_field(C().FIELD_CHARGE)
    assert np.max(np.abs(ch - charge_o)) <= 1e-14 * np.max(np.abs(charge_o))

    # solve: residual of the GPU potential in the oracle's operator
    sim.stage(C().STAGE_SOLVE)
    d = sim.diag()
    assert d.mg_relres <= 1e-10, d.mg_relres
    phi = sim.get_field(C().FIELD_PHI)
    A, bd = O.poisson_assemble(m, g)
    b = -charge_o - bd
    b -= b.mean()  # periodic: the solvable part of the right side
    r = b - O.apply(g, A, phi)
    rel = np.linalg.norm(r) / np.linalg.norm(b)
    assert rel <= 1e-9, rel
    del A, bd, b, r
    say(t0, "solve: residual in the oracle's operator %.2e (%d iterations)" % (rel, d.mg_cycles))

    # vertex field of a synthetic potential
    phis = W.synthetic_phi(case)
    sim.set_field(C().FIELD_PHI, phis)
    sim.stage(C().STAGE_EFIELD)
    Eg = sim.get_field(C().FIELD_EV)[:, :3].astype(np.float64)
    Eo = O.efield(m, g, phis)
    assert np.max(np.abs(Eg - Eo)) <= 1e-6 * np.max(np.abs(Eo))
    del Eg, Eo
    say(t0, "vertex field")

    # one push in a synthetic field, sampled particles against the oracle
    nv = sim.field_bytes(C().FIELD_EV) // 4 // 4
    E = W.synthetic_ev(case, nv, dtype=np.float32)
    Ebuf = np.zeros((nv, 4), dtype=np.float32)
    Ebuf[:, :3] = E[:, :3]
    sim.set_field(C().FIELD_EV, Ebuf)
    sim.stage(C().STAGE_PUSH)
    E64 = Ebuf[:, :3].astype(np.float64)
    dg = sim.diag()
    rng = np.random.default_rng(1311)
    for sid, s in enumerate(case.species):
        n = parts[sid]["cell"].size
        pick = np.sort(rng.choice(n, 32768, replace=False))
        sub = {k: (v[..., pick] if k in ("off", "vel") else v[pick]) for k, v in parts[sid].items()}
        o = W.to_oracle(sub)
        cell, off, vel, cnt = O.push(m, g, s.q / s.m, case.dt, case.B, o["cell"], o["off"], o["vel"], E64)
        got = sim.get_particles(sid)
        where = np.full(n, -1, dtype=np.int64)
        where[got["id"].astype(np.int64)] = np.arange(got["id"].size)
        at = where[parts[sid]["id"][pick].astype(np.int64)]
        assert np.all(at >= 0)
        pg = logical_cells(case, got["cell"][at], got["off"][:, at].astype(np.float64))
        po = logical_cells(case, cell, off)
        dpos = np.abs(periodic_diff(case, pg, po))
        vg = got["vel"][:, at].T.astype(np.float64)
        Eo = O.gather(g, E64, o["cell"], o["off"])
        scale = np.abs(o["vel"]) + np.abs(s.q / s.m * Eo * case.dt)
        dv = np.abs(vg - vel)
        assert dpos.max() < 2e-5, dpos.max()
        assert np.all(dv <= 2e-5 * (scale + 1e-3)), (dv / (scale + 1e-3)).max()
        assert C().qsum(dg, sid) == n << (3 * S1)
        del got, where
        say(t0, "push of species %d: %d sampled particles, max |dxi| %.2e cell" % (sid, pick.size, dpos.max()))
    assert dg.newton_failed == 0
    sim.close()
