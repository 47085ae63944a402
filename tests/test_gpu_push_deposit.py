"""GPU parity of the deposit made by the timed kernel itself: the fused
gather + push + map inversion + boundaries + deposit (CPIC_STAGE_PUSH, and the
step), whose deposit goes through the tile's LDS window, its flush with global
integer atomics, far deposits of particles that left the window, the FP64
fallback kernel, the injection kernel and the extra work items of particles
appended since the last sort.

Bar: bit-exact.  After the push, Q_s of every species equals the oracle's
fixed-point deposit (Eqs. pg, Wpc, b2; CIC) of the live particles at the
positions the GPU moved them to, read back through cpic_get_particles -- the
same positions on both sides.  A misplaced window flush or far deposit keeps
the total but fails this."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_1311_2286_amd import workloads as W
from _helpers import gpu_sim, oracle_objects

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def C():
    from paper_1311_2286_amd import cpic
    return cpic


def probe_case(n=(48, 40), ppc=6.0):
    return W.Case("probe_small", 2, W.POLAR_LOG, n, r_in=1.0, r_out=10.0,
                  bc_lo=(W.DIRICHLET, W.PERIODIC), bc_hi=(W.DIRICHLET, W.PERIODIC),
                  phi_lo=(-5.0, 0.0), phi_hi=(0.0, 0.0), dt=0.1,
                  species=[W.electrons(1.0, ppc), W.ions(ppc=ppc)], case_id=9)


CASES = {
    "2d_sin": lambda: W.small_case(dim=2, n=(40, 24), ppc=8.0),
    "3d_sin": lambda: W.small_case(dim=3, n=(20, 12, 16), ppc=4.0),
    "2d_tiny": lambda: W.small_case(dim=2, n=(6, 4), L=(6.0, 4.0), ppc=20.0),
    "3d_tiny": lambda: W.small_case(dim=3, n=(4, 6, 2), L=(4.0, 6.0, 2.0), ppc=20.0),
    "3d_mag": lambda: W.small_case(dim=3, n=(16, 16, 10), ppc=4.0, B=(0.0, 0.0, 2.0)),
    # particles crossing ~4 cells per step: deposits outside the tile window
    "3d_fast": lambda: W.small_case(dim=3, n=(20, 12, 16), eps=0.05, ppc=4.0, L=(0.5, 0.3, 0.4),
                                    vth_e=1.0, case_id=120),
    # J_min = 0.057 and fast electrons: some updates go to the FP64 fallback
    "2d_fallback": lambda: W.small_case(dim=2, n=(40, 24), eps=0.15, ppc=6.0, L=(1.0, 1.0), vth_e=0.2,
                                        case_id=121),
    # walls: absorption at the probe, outflow at the outer wall
    "2d_probe": probe_case,
    # the probe on its tabulated map, Newton on the interpolant: updates that
    # leave the LDS window or cross a wall go to the FP64 fallback kernel
    "2d_probe_tab": lambda: dataclasses.replace(probe_case(), tabulated=True, case_id=122),
    "3d_sin_tab": lambda: dataclasses.replace(W.small_case(dim=3, n=(20, 12, 16), ppc=4.0, case_id=123),
                                              tabulated=True),
}
# cases whose position update is Newton on a tabulated map
NEWTON_TAB = ("2d_probe_tab", "3d_sin_tab")


def live_deposit(case, sim, g, shape, sid):
    p = sim.get_particles(sid)
    live = p["cell"] >= 0
    o = W.to_oracle({"cell": p["cell"][live], "off": p["off"][:, live], "vel": p["vel"][:, live]})
    S1 = 24 if case.dim == 2 else 16
    return O.deposit_fixed(g, shape, S1, o["cell"], o["off"]), int(live.sum())


@pytest.mark.parametrize("shape", [2, 1])
@pytest.mark.parametrize("name", sorted(CASES))
def test_push_deposit_bit_exact(name, shape):
    case = CASES[name]()
    kw = {"mover": C().MOVER_NEWTON} if name in NEWTON_TAB else {}
    sim, parts = gpu_sim(case, precision=0, shape=shape, **kw)
    nv = sim.field_bytes(C().FIELD_EV) // 4 // (4 if case.dim == 3 else 2)
    E = W.synthetic_ev(case, nv, dtype=np.float32)
    ec = 4 if case.dim == 3 else 2
    Ebuf = np.zeros((nv, ec), dtype=np.float32)
    Ebuf[:, : case.dim] = E[:, : case.dim]
    sim.set_field(C().FIELD_EV, Ebuf)
    sim.stage(C().STAGE_PUSH)
    _, g = oracle_objects(case)
    d = sim.diag()
    for sid in range(len(case.species)):
        Qo, nlive = live_deposit(case, sim, g, shape, sid)
        Qg = sim.get_field(C().FIELD_Q, sid)
        assert np.array_equal(Qg, Qo), (name, sid, int(np.sum(Qg != Qo)))
        assert nlive == d.count[sid]
    if name == "3d_fast":
        assert d.far_deposits > 0
    if name in ("2d_fallback", "2d_probe_tab"):
        assert d.newton_fallback > 0
    if name == "2d_probe":
        assert sum(d.absorbed[:2]) + sum(d.outflow[:2]) > 0
    sim.close()


@pytest.mark.parametrize("shape", [2, 1])
@pytest.mark.parametrize("name", ["2d_probe", "3d_fast", "3d_sin"])
def test_steps_deposit_bit_exact(name, shape):
    # whole steps with a tile sort every 4 steps; the probe injects at its
    # outer wall, so between sorts its appended particles are moved and
    # deposited by the extra work items
    case = CASES[name]()
    inject = name == "2d_probe"
    sim, parts = gpu_sim(case, precision=0, shape=shape, sort_every=4, inject=inject, seed=3,
                         capacity_factor=1.6 if inject else 1.0, mg_rtol=1e-10)
    sim.initialize()
    _, g = oracle_objects(case)
    for k in range(6):
        sim.step(1)
        d = sim.diag()
        for sid in range(len(case.species)):
            Qo, nlive = live_deposit(case, sim, g, shape, sid)
            assert np.array_equal(sim.get_field(C().FIELD_Q, sid), Qo), (name, k, sid)
            assert nlive == d.count[sid]
    if inject:
        assert d.injected[0] > 0 and max(d.sorts[:2]) <= 3
    if name == "3d_fast":
        assert d.far_deposits > 0
    sim.close()


def test_injection_through_a_transverse_wall():
    # identity map with a bounded transverse axis: an injected particle's entry
    # flight (a random fraction of the step from the face) can leave through
    # the side wall at once.  Such particles are never live: the live count,
    # the deposit and the run sorted every step agree with the run sorted
    # every 4 steps, and the oracle's injection (which drops them) gives the
    # same injected count.
    case = W.Case("slab", 2, W.IDENTITY, (24, 6), L=(6.0, 1.5), bc_lo=(W.DIRICHLET, W.DIRICHLET),
                  bc_hi=(W.DIRICHLET, W.DIRICHLET), dt=0.1,
                  species=[W.electrons(1.0, 64.0)], case_id=31)
    a, _ = gpu_sim(case, precision=0, inject=True, seed=21, capacity_factor=4.0, sort_every=1)
    b, _ = gpu_sim(case, precision=0, inject=True, seed=21, capacity_factor=4.0, sort_every=4)
    a.initialize()
    b.initialize()
    m, g = oracle_objects(case)
    s = case.species[0]
    inj_o = 0
    for k in range(8):
        a.step(1)
        b.step(1)
        c, *_ = O.inject(m, g, 1.0, s.vth, case.weight(s), case.dt, 21, k, 0)
        inj_o += c.size
        da, db = a.diag(), b.diag()
        assert da.count[0] == db.count[0] and da.injected[0] == db.injected[0] == inj_o, k
        assert da.inject_lost[0] == db.inject_lost[0]
        assert np.array_equal(a.get_field(C().FIELD_Q, 0), b.get_field(C().FIELD_Q, 0)), k
        Qo, nlive = live_deposit(case, b, g, 2, 0)
        assert nlive == db.count[0]
        assert np.array_equal(b.get_field(C().FIELD_Q, 0), Qo), k
    assert db.inject_lost[0] > 0
    a.close()
    b.close()
