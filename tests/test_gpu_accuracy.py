"""Error of the timed configuration against the FP64 oracle.

The benchmark runs the FP32 / fixed-point path with the Poisson solve stopped
at a relative residual of 4e-6 (at most 10 iterations per solve, launched as
one more than the solve of two steps before needed) and a tile sort every 4
steps.  This runs the same settings on the benchmark's recipe at a size the
oracle finishes in seconds (the 3D sinusoidal box, eps = 0.05, one Debye
length per cell, 32 electrons + 32 ions per cell, 24^3 cells) and on the 2D
Langmuir workload, from the same initial state as the oracle (its FP32
particles converted exactly), and states after each step:
  - rho: charge per cell, max |difference| / max |oracle|;
  - phi, E (vertex field): the same;
  - W_E: relative difference of the field energy;
  - trajectories: largest |difference| of the logical positions, in cells.
Two oracles: the FP64 particle path with the same fixed-point deposit rule
(this isolates FP32 arithmetic and the solver tolerance) and the plain FP64
path with the unquantised FP64 deposit (adds the quantisation of the weights
to 2^-S1: S1 = 16 per axis in 3D, 24 in 2D).

Bars: phi and E within 1e-5 of the oracle with the same deposit rule (the
FP32 path's field accuracy; the solve's tolerance is the largest term, and
4e-6 keeps the fields below 1e-5 where 1e-5 reached 1.35e-5 on the Langmuir
case); the plain-FP64 differences are reported."""
import numpy as np
import pytest

import oracle as O
from paper_1311_2286_amd import workloads as W
from _helpers import gpu_sim, oracle_objects, oracle_species, by_id, logical_cells, periodic_diff

pytestmark = pytest.mark.gpu

BENCH = dict(mg_rtol=4e-6, mg_max_cycles=10, sort_every=4)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def C():
    from paper_1311_2286_amd import cpic
    return cpic


def box24():
    n = (24, 24, 24)
    return W.Case("box3d_24", 3, W.SINUSOIDAL, n, L=tuple(float(v) for v in n), eps=0.05, dt=0.1,
                  species=[W.electrons(1.0, 32.0), W.ions(ppc=32.0)], delta=0.01, case_id=2)


def errors(case, sim, osim, ids):
    rel = lambda a, b: float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
    e = {}
    e["rho"] = rel(sim.get_field(C().FIELD_CHARGE), osim.charge)
    e["phi"] = rel(sim.get_field(C().FIELD_PHI), osim.phi)
    Ev = sim.get_field(C().FIELD_EV)[:, : case.dim].astype(np.float64)
    e["E"] = rel(Ev, osim.Ev[:, : case.dim])
    we = sim.diag().field_energy
    e["W_E"] = abs(we - osim.field_energy()) / abs(osim.field_energy())
    worst = 0.0
    for sid in range(len(case.species)):
        got = by_id(sim.get_particles(sid))
        o = osim.sp[sid]
        pg = logical_cells(case, got["cell"], got["off"].astype(np.float64))
        po = logical_cells(case, o["cell"], o["off"])
        worst = max(worst, float(np.abs(periodic_diff(case, pg, po)).max()))
    e["traj_cells"] = worst
    return e


@pytest.mark.parametrize("name", ["box3d_24", "langmuir2d"])
def test_bench_settings_error_against_the_oracle(name):
    case = box24() if name == "box3d_24" else W.case1()
    sim, parts = gpu_sim(case, precision=0, **BENCH)
    m, g = oracle_objects(case)
    bg = O.ion_background(m, g, 2) if case.background else None
    ax = 3 if case.dim == 3 else 2
    fixed = O.OracleSim(m, g, oracle_species(case, parts), dt=case.dt, background=bg, deposit="fixed",
                        rtol=1e-13, ke_axes=ax)
    plain = O.OracleSim(m, g, oracle_species(case, parts), dt=case.dt, background=bg, deposit="f64",
                        rtol=1e-13, ke_axes=ax)
    sim.initialize()
    fixed.initialize()
    plain.initialize()
    worst = {"fixed": {}, "plain": {}}
    for k in range(6):
        sim.step(1)
        fixed.step()
        plain.step()
        for tag, osim in (("fixed", fixed), ("plain", plain)):
            e = errors(case, sim, osim, None)
            for key, v in e.items():
                worst[tag][key] = max(worst[tag].get(key, 0.0), v)
        print("[accuracy %s] step %d vs fixed-deposit oracle %s; vs plain FP64 %s; cycles %d relres %.1e"
              % (name, k + 1, {k_: "%.1e" % v for k_, v in errors(case, sim, fixed, None).items()},
                 {k_: "%.1e" % v for k_, v in errors(case, sim, plain, None).items()},
                 sim.diag().mg_cycles, sim.diag().mg_relres), flush=True)
    assert worst["fixed"]["phi"] <= 1e-5, worst
    assert worst["fixed"]["E"] <= 1e-5, worst
    assert worst["fixed"]["traj_cells"] <= 1e-4, worst
    sim.close()
