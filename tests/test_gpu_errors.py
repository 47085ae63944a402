"""GPU tests of the library's checked error paths and of run-to-run
determinism, through the C ABI.

  - CPIC_E_OVERFLOW: host particles crowding one 3^d block of cells (2^16 of
    them, whose fixed-point deposit could pass 64 bits) are refused and the
    simulation keeps its particles; a deposit that does wrap (device input,
    which skips the host check: 2^16 particles at a cell centre with the CIC
    shape each put exactly 2^48 into that cell) is reported by the diagnostics
    and by cpic_sync through the exact charge total, and further steps are
    refused until new particles are loaded;
  - CPIC_E_NONFINITE: a NaN in a host field is refused before anything is
    copied; one that reaches the potential from device memory is reported by
    the diagnostics and by cpic_sync;
  - the number of solver iterations a step launches, and which species it
    sorts, come from the record of an earlier step that the host waits for:
    a run stepped without any synchronisation gives bitwise the potential,
    particles and iteration counts of a run synchronised after every step,
    also when the iteration cap binds."""
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


def box(n=(8, 8, 8), shape=2):
    sim = C().Sim(C().MAP_IDENTITY, 3, n, L=tuple(float(x) for x in n), shape=shape, precision=0, dt=0.1,
                  mg_rtol=1e-10, mg_max_cycles=30, track_ids=True)
    sim.add_species(-1.0, 1.0, 1e-3, 1 << 17)
    return sim


def crowd(n, cell, count, spread=False):
    """count particles in `cell` (or spread over its 3x3x3 block), at the centre."""
    rng = np.random.default_rng(3)
    if spread:
        i, j, k = cell % n[0], (cell // n[0]) % n[1], cell // (n[0] * n[1])
        o = rng.integers(-1, 2, size=(3, count))
        cells = ((i + o[0]) % n[0] + n[0] * (((j + o[1]) % n[1]) + n[1] * ((k + o[2]) % n[2]))).astype(np.int32)
    else:
        cells = np.full(count, cell, dtype=np.int32)
    off = np.full((3, count), 0.5, dtype=np.float32)
    vel = np.zeros((3, count), dtype=np.float32)
    return cells, off, vel


def test_crowded_host_particles_are_refused_and_the_sim_kept():
    n = (8, 8, 8)
    sim = box(n)
    base = crowd(n, 100, 1000, spread=True)
    sim.set_particles(0, *base)
    before = by_id(sim.get_particles(0))
    for spread in (False, True):
        with pytest.raises(C().CpicError) as e:
            sim.set_particles(0, *crowd(n, 200, 1 << 16, spread=spread))
        assert e.value.status == C().E_OVERFLOW
        after = by_id(sim.get_particles(0))
        for f in ("cell", "off", "vel", "id"):
            assert np.array_equal(before[f], after[f])
    # one fewer than the bound is accepted, and its deposit is exact
    sim.set_particles(0, *crowd(n, 200, (1 << 16) - 1, spread=True))
    sim.stage(C().STAGE_DEPOSIT)
    d = sim.diag()
    assert C().qsum(d, 0) == ((1 << 16) - 1) << 48
    sim.close()


def test_wrapped_deposit_is_reported():
    import torch
    n = (8, 8, 8)
    sim = box(n, shape=1)
    cells, off, vel = crowd(n, 73, 1 << 16)
    dev = [torch.from_numpy(a).cuda() for a in (cells, off, vel)]
    sim.set_particles(0, *dev)  # device input: no host headroom check
    sim.stage(C().STAGE_DEPOSIT)
    Q = sim.get_field(C().FIELD_Q, 0)
    assert int(Q[73]) == 0  # 2^16 x 2^48 wrapped to zero
    with pytest.raises(C().CpicError) as e:
        sim.diag()
    assert e.value.status == C().E_OVERFLOW
    with pytest.raises(C().CpicError) as e:
        sim.sync()
    assert e.value.status == C().E_OVERFLOW
    # new particles clear it
    cells, off, vel = crowd(n, 73, 100)
    sim.set_particles(0, cells, off, vel)
    sim.stage(C().STAGE_DEPOSIT)
    assert C().qsum(sim.diag(), 0) == 100 << 48
    sim.close()


def test_wrapped_deposit_refuses_steps():
    import torch
    n = (8, 8, 8)
    sim = box(n, shape=1)
    cells, off, vel = crowd(n, 9, 1 << 16)
    sim.set_particles(0, *[torch.from_numpy(a).cuda() for a in (cells, off, vel)])
    sim.initialize()  # deposits, solves, pushes back half a step
    with pytest.raises(C().CpicError) as e:
        sim.sync()
    assert e.value.status == C().E_OVERFLOW
    with pytest.raises(C().CpicError) as e:
        sim.step(1)
    assert e.value.status == C().E_OVERFLOW
    sim.close()


def test_non_finite_fields():
    import torch
    case = W.small_case(dim=2, n=(40, 24), ppc=4.0)
    sim, parts = gpu_sim(case, precision=0, mg_rtol=1e-10)
    sim.initialize()
    phi0 = sim.get_field(C().FIELD_PHI)
    bad = phi0.copy()
    bad[17] = np.nan
    with pytest.raises(C().CpicError) as e:
        sim.set_field(C().FIELD_PHI, bad)
    assert e.value.status == C().E_NONFINITE
    assert np.array_equal(sim.get_field(C().FIELD_PHI), phi0)
    ev = sim.get_field(C().FIELD_EV)
    ev[3, 1] = np.inf
    with pytest.raises(C().CpicError) as e:
        sim.set_field(C().FIELD_EV, ev)
    assert e.value.status == C().E_NONFINITE
    sim.diag()  # still healthy
    # from device memory the value gets in; the checks report it
    t = torch.from_numpy(bad).cuda()
    st = sim.lib.cpic_set_field(sim.h, C().FIELD_PHI, 0, C()._ptr(t), t.numel() * 8, 1)
    assert st == 0
    with pytest.raises(C().CpicError) as e:
        sim.diag()
    assert e.value.status == C().E_NONFINITE
    with pytest.raises(C().CpicError) as e:
        sim.sync()
    assert e.value.status == C().E_NONFINITE
    sim.set_field(C().FIELD_PHI, phi0)
    sim.diag()
    sim.close()


@pytest.mark.parametrize("cap", [30, 3])
def test_unsynchronised_run_is_bitwise_the_synchronised_one(cap):
    # rtol 1e-9 needs more than 3 iterations per solve: with cap 3 every step
    # stops at the launched count, which must not depend on host timing
    case = W.small_case(dim=3, n=(20, 12, 16), ppc=4.0, case_id=130)
    a, _ = gpu_sim(case, precision=0, mg_rtol=1e-9, mg_max_cycles=cap, sort_every=2)
    b, _ = gpu_sim(case, precision=0, mg_rtol=1e-9, mg_max_cycles=cap, sort_every=2)
    a.initialize()
    b.initialize()
    a.step(12)  # no synchronisation between steps
    cyc = []
    for _ in range(12):
        b.step(1)
        cyc.append(b.diag().mg_cycles)
    da, db = a.diag(), b.diag()
    assert da.mg_cycles == db.mg_cycles and da.mg_relres == db.mg_relres
    assert list(da.sorts) == list(db.sorts)
    assert np.array_equal(a.get_field(C().FIELD_PHI), b.get_field(C().FIELD_PHI))
    for sid in range(len(case.species)):
        pa, pb = by_id(a.get_particles(sid)), by_id(b.get_particles(sid))
        for f in ("id", "cell", "off", "vel"):
            assert np.array_equal(pa[f], pb[f]), (sid, f)
    if cap == 3:
        assert max(cyc) == 3 and da.mg_relres > 1e-9
    a.close()
    b.close()
