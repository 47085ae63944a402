"""GPU tests of the tile sort that follows a step: the particle, FP64 fallback
and injection kernels of that step count the particles' new tiles themselves
(the sort then runs no histogram pass).

Bars:
  - after a step that sorts a species, it is stored in non-decreasing tile
    order, every identifier once, the live count that of the diagnostics;
  - a species whose particles drift less than a cell between sorts is sorted
    less often than sort_every asks (ions against electrons), with bitwise
    the same physics as sorting every species every step (FP32 path);
  - FP32 path (integer deposit, per-particle arithmetic): a run that sorts
    every step and a run that never sorts give bitwise the same particles
    (matched by identifier) and potential, with particles fast enough to leave
    their tile's neighbourhood in one step and some left to the FP64 fallback;
  - probe with flux injection and absorption: the live count follows
    injected - absorbed - outflow exactly."""
import numpy as np
import pytest

from paper_1311_2286_amd import workloads as W
from _helpers import gpu_sim, by_id

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


TILE = {2: (16, 16, 1), 3: (8, 8, 8)}


def tiles_of(case, cell):
    n = list(case.n) + [1] * (3 - case.dim)
    T = TILE[case.dim]
    nt = [(n[a] + T[a] - 1) // T[a] for a in range(3)]
    i = cell % n[0]
    j = (cell // n[0]) % n[1]
    k = cell // (n[0] * n[1])
    return i // T[0] + nt[0] * (j // T[1] + nt[1] * (k // T[2]))


def check_sorted_storage(case, sim, species=None):
    d = sim.diag()
    for sid in (range(len(case.species)) if species is None else species):
        p = sim.get_particles(sid)
        assert p["cell"].size == d.count[sid]
        assert np.all(p["cell"] >= 0)
        t = tiles_of(case, p["cell"].astype(np.int64))
        assert np.all(np.diff(t) >= 0), sid
        assert np.unique(p["id"]).size == p["id"].size


def fast_case(dim):
    if dim == 3:
        # cell size 0.025, electron thermal displacement 4 cells per step: the
        # tail leaves the 8-cell tile's neighbourhood in one step
        return W.small_case(dim=3, n=(20, 12, 16), eps=0.05, ppc=4.0, L=(0.5, 0.3, 0.4),
                            vth_e=1.0, case_id=120)
    # strong distortion (J_min = 0.057) and fast electrons: some FP32 Newton
    # solves are left to the FP64 fallback
    return W.small_case(dim=2, n=(40, 24), eps=0.15, ppc=6.0, L=(1.0, 1.0), vth_e=0.2, case_id=121)


@pytest.mark.parametrize("dim", [3, 2])
def test_sort_every_step_is_bitwise_no_sort(dim):
    case = fast_case(dim)
    a, _ = gpu_sim(case, precision=0, sort_every=1)
    b, _ = gpu_sim(case, precision=0, sort_every=1 << 20)
    a.initialize()
    b.initialize()
    for k in range(4):
        before = list(a.diag().sorts)
        a.step(1)
        b.step(1)
        after = list(a.diag().sorts)
        check_sorted_storage(case, a, [s for s in range(len(case.species)) if after[s] > before[s]])
        assert np.array_equal(a.get_field(C().FIELD_PHI), b.get_field(C().FIELD_PHI)), k
        for sid in range(len(case.species)):
            pa, pb = by_id(a.get_particles(sid)), by_id(b.get_particles(sid))
            for f in ("id", "cell", "off", "vel"):
                assert np.array_equal(pa[f], pb[f]), (k, sid, f)
    d = a.diag()
    assert d.newton_fallback == b.diag().newton_fallback
    if dim == 3:
        assert d.far_deposits > 0
    else:
        assert d.newton_fallback > 0
    a.close()
    b.close()


def test_slow_species_sort_less_often_with_the_same_physics():
    case = W.small_case(dim=3, n=(20, 12, 16), ppc=4.0, case_id=122)
    a, _ = gpu_sim(case, precision=0, sort_every=2)
    b, _ = gpu_sim(case, precision=0, sort_every=1)
    a.initialize()
    b.initialize()
    for k in range(12):
        before = list(a.diag().sorts)
        a.step(1)
        b.step(1)
        after = list(a.diag().sorts)
        check_sorted_storage(case, a, [s for s in range(2) if after[s] > before[s]])
        assert np.array_equal(a.get_field(C().FIELD_PHI), b.get_field(C().FIELD_PHI)), k
    d = a.diag()
    # electrons (v_th 1, dt 0.1, unit cells): up to every second step; ions
    # (43 times slower) not again within 12 steps after the initial sort
    assert d.sorts[0] >= 4, list(d.sorts)
    assert d.sorts[1] < d.sorts[0], list(d.sorts)
    for sid in range(2):
        pa, pb = by_id(a.get_particles(sid)), by_id(b.get_particles(sid))
        for f in ("id", "cell", "off", "vel"):
            assert np.array_equal(pa[f], pb[f]), (sid, f)
    a.close()
    b.close()


def probe_case():
    return W.Case("probe_small", 2, W.POLAR_LOG, (48, 40), r_in=1.0, r_out=10.0,
                  bc_lo=(W.DIRICHLET, W.PERIODIC), bc_hi=(W.DIRICHLET, W.PERIODIC),
                  phi_lo=(-5.0, 0.0), phi_hi=(0.0, 0.0), dt=0.1,
                  species=[W.electrons(1.0, 6.0), W.ions(ppc=6.0)], case_id=9)


@pytest.mark.parametrize("precision", [0, 1])
def test_probe_sorted_counts_follow_injection_and_absorption(precision):
    case = probe_case()
    sim, parts = gpu_sim(case, precision=precision, inject=True, seed=5, capacity_factor=1.6)
    sim.initialize()
    n0 = [p["cell"].size for p in parts]
    for k in range(5):
        sim.step(1)
        d = sim.diag()
        for sid in range(len(case.species)):
            # the counters run from the start
            assert d.count[sid] == n0[sid] + d.injected[sid] - d.absorbed[sid] - d.outflow[sid], (k, sid)
        check_sorted_storage(case, sim)
    assert d.injected[0] > 0 and d.absorbed[0] + d.outflow[0] > 0
    sim.close()


def test_injecting_species_between_sorts_bitwise_the_same():
    # an injecting species sorted every 4 steps (its appended particles moved
    # by the extra work item in between) gives bitwise the run sorted every step
    case = probe_case()
    a, _ = gpu_sim(case, precision=0, inject=True, seed=9, capacity_factor=1.6, sort_every=1)
    b, _ = gpu_sim(case, precision=0, inject=True, seed=9, capacity_factor=1.6, sort_every=4)
    a.initialize()
    b.initialize()
    for k in range(9):
        a.step(1)
        b.step(1)
        assert np.array_equal(a.get_field(C().FIELD_PHI), b.get_field(C().FIELD_PHI)), k
        da, db = a.diag(), b.diag()
        assert list(da.count) == list(db.count) and list(da.injected) == list(db.injected), k
        assert abs(da.kinetic - db.kinetic) <= 1e-12 * abs(da.kinetic), k
        for sid in range(len(case.species)):
            # the run sorted less often still holds the particles that left
            # since its last sort (cell < 0): compare the live ones
            ga, gb = a.get_particles(sid), b.get_particles(sid)
            assert np.all(ga["cell"] >= 0)
            live = gb["cell"] >= 0
            assert int(live.sum()) == da.count[sid] == db.count[sid], (k, sid)
            gb = {f: (v[..., live] if f in ("off", "vel") else v[live]) for f, v in gb.items()}
            pa, pb = by_id(ga), by_id(gb)
            for f in ("id", "cell", "off", "vel"):
                assert np.array_equal(pa[f], pb[f]), (k, sid, f)
    db = b.diag()
    assert db.injected[0] > 0 and max(db.sorts[:2]) <= 4, list(db.sorts)
    a.close()
    b.close()
