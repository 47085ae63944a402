"""GPU tests of the serving loop (cpic_server_* in include/cpic.h): independent
2D periodic sinusoidal-map cases (the paper's distorted-mesh test setting,
Eq. map2) of different grids, perturbation amplitudes and temperatures,
admitted by slot and HBM budget and advanced together on per-slot streams;
cases of one grid and map step together, their field phases batched.

Bars:
  - a case's result is the same run alone, in a mix with other cases, and as
    a plain simulation outside the server: field energy, exact charge sums,
    counts and the final potential bitwise, kinetic energy to 1e-13 relative
    (its FP64 per-work-item sums follow the order of particles inside a tile,
    which the tile sort does not fix);
  - the same with batching turned off (CPIC_SERVER_NO_BATCH);
  - the budget is never exceeded, cases that do not fit wait for memory and
    then complete; a case larger than the whole budget fails with
    CPIC_E_BUDGET without disturbing the others."""
import os

import numpy as np
import pytest

from paper_1311_2286_amd import workloads as W

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


def serving_case(n, eps, ppc, vth, case_id):
    return W.Case("serve_%d" % case_id, 2, W.SINUSOIDAL, (n, n), L=(float(n), float(n)), eps=eps,
                  dt=0.1, species=[W.electrons(vth, ppc)], background=True, delta=0.01,
                  case_id=case_id)


def descs(case):
    c = C()
    m = c.make_map_desc(case.map_kind, case.dim, case.L, case.eps)
    g = c.make_grid_desc(case.n, shape=c.SHAPE_B2, precision=c.FP32, dt=case.dt, background=True,
                         background_n0=1.0, mg_rtol=1e-10, mg_max_cycles=40, sort_every=4)
    sp = [c.make_species_desc(s.q, s.m, case.weight(s)) for s in case.species]
    parts = [W.generate_species(case, sid, dtype=np.float32) for sid in range(len(case.species))]
    return m, g, sp, parts


CASES = [serving_case(32, 0.10, 16.0, 1.0, 401), serving_case(48, 0.05, 12.0, 0.7, 402),
         serving_case(64, 0.15, 8.0, 1.5, 403)]
NSTEPS = 12


def run_server(case_list, slots, budget, want_phi=True):
    prepared = [descs(case) for case in case_list]
    srv = C().Server(budget, slots)
    tickets = [srv.submit(m, g, sp, parts, NSTEPS, want_phi=want_phi) for m, g, sp, parts in prepared]
    for _ in range(100000):
        if srv.pump(8):
            break
    res = [srv.poll(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    return res, stats


def same(a, b):
    for f in ("status", "steps", "field_energy", "count", "qsum_lo", "qsum_hi", "absorbed",
              "outflow", "injected", "pushes"):
        assert a[f] == b[f], (f, a[f], b[f])
    assert abs(a["kinetic"] - b["kinetic"]) <= 1e-13 * abs(a["kinetic"])
    assert np.array_equal(a["phi"], b["phi"])


def test_case_result_is_the_same_alone_in_a_mix_and_outside_the_server():
    A = CASES[0]
    alone, st1 = run_server([A], slots=1, budget=1 << 30)
    assert alone[0]["status"] == 0 and alone[0]["steps"] == NSTEPS
    mixed, st2 = run_server([CASES[2], A, CASES[1]], slots=3, budget=1 << 30)
    assert all(r["status"] == 0 for r in mixed)
    same(alone[0], mixed[1])
    assert st2["completed"] == 3 and st2["step_samples"] == 3 * NSTEPS
    assert st2["pushes"] == sum(r["pushes"] for r in mixed)
    assert 0 < st2["step_p50_ms"] <= st2["step_p99_ms"]
    # the same case as a plain simulation
    c = C()
    m, g, sp, parts = descs(A)
    sim = c.Sim(A.map_kind, 2, A.n, L=A.L, eps=A.eps, dt=A.dt, background=True, mg_rtol=1e-10,
                mg_max_cycles=40, sort_every=4)
    sim.add_species(A.species[0].q, A.species[0].m, A.weight(A.species[0]), parts[0]["cell"].size)
    sim.set_particles(0, parts[0]["cell"], parts[0]["off"], parts[0]["vel"])
    sim.initialize()
    sim.step(NSTEPS)
    d = sim.diag()
    assert abs(d.kinetic - alone[0]["kinetic"]) <= 1e-13 * abs(d.kinetic)
    assert d.field_energy == alone[0]["field_energy"]
    assert np.array_equal(sim.get_field(c.FIELD_PHI), alone[0]["phi"])
    sim.close()


def test_admission_by_budget_and_a_case_that_never_fits():
    # three cases of the same size (different seeds); a budget of 1.5 cases
    # lets one run at a time although three slots are free
    same_size = [serving_case(64, 0.15, 8.0, 1.5, 410 + k) for k in range(3)]
    _, st = run_server(same_size[:1], slots=1, budget=1 << 30, want_phi=False)
    one = st["peak_bytes"]
    budget = int(one * 1.5)
    res, st = run_server(same_size, slots=3, budget=budget, want_phi=False)
    assert all(r["status"] == 0 for r in res)
    assert st["peak_bytes"] <= budget and st["completed"] == 3
    assert st["peak_active"] == 1
    # with room for all three they run together
    res, st = run_server(same_size, slots=3, budget=4 * one, want_phi=False)
    assert all(r["status"] == 0 for r in res) and st["peak_active"] == 3
    # a case larger than the whole budget fails; the others complete
    big = serving_case(256, 0.05, 16.0, 1.0, 404)
    res, st = run_server([CASES[0], big, CASES[1]], slots=2, budget=budget, want_phi=False)
    assert res[0]["status"] == 0 and res[2]["status"] == 0
    assert res[1]["status"] == -4  # CPIC_E_BUDGET
    assert st["failed"] == 1 and st["completed"] == 2


def test_tabulated_map_case_is_copied_at_submit_and_matches_a_plain_run():
    # a case on a map known at its vertices (the sinusoidal map sampled there),
    # moved by the predictor-corrector update; the vertex table is overwritten
    # right after submit: the server works from its own copy
    c = C()
    case = serving_case(48, 0.10, 12.0, 1.0, 420)
    vt = np.ascontiguousarray(W.vertex_table(case))
    m = c.make_map_desc(c.MAP_TABULATED, 2, W.table_shift(case), vertices=vt)
    g = c.make_grid_desc(case.n, shape=c.SHAPE_B2, precision=c.FP32, dt=case.dt, background=True,
                         background_n0=1.0, mg_rtol=1e-10, mg_max_cycles=40, sort_every=4, mover=c.MOVER_PC)
    sp = [c.make_species_desc(s.q, s.m, case.weight(s)) for s in case.species]
    parts = [W.generate_species(case, 0, dtype=np.float32)]
    srv = c.Server(1 << 30, 2)
    t = srv.submit(m, g, sp, parts, NSTEPS, want_phi=True)
    vt[:] = np.nan
    for _ in range(100000):
        if srv.pump(8):
            break
    res = srv.poll(t)
    srv.close()
    assert res["status"] == 0 and res["steps"] == NSTEPS
    sim = c.Sim(c.MAP_TABULATED, 2, case.n, L=W.table_shift(case), dt=case.dt, background=True, mg_rtol=1e-10,
                mg_max_cycles=40, sort_every=4, mover=c.MOVER_PC, vertices=W.vertex_table(case))
    sim.add_species(case.species[0].q, case.species[0].m, case.weight(case.species[0]), parts[0]["cell"].size)
    sim.set_particles(0, parts[0]["cell"], parts[0]["off"], parts[0]["vel"])
    sim.initialize()
    sim.step(NSTEPS)
    d = sim.diag()
    assert abs(d.kinetic - res["kinetic"]) <= 1e-13 * abs(d.kinetic)
    assert d.field_energy == res["field_energy"]
    assert np.array_equal(sim.get_field(c.FIELD_PHI), res["phi"])
    sim.close()


def test_batched_server_equals_unbatched():
    # four cases of one grid and map (different seeds and temperatures) step
    # as one batch group; a fifth of another grid steps alone
    group = [serving_case(48, 0.10, 12.0, v, 430 + k) for k, v in enumerate((1.0, 0.7, 1.3, 0.9))]
    mix = group + [CASES[0]]
    res_b, st_b = run_server(mix, slots=5, budget=1 << 30)
    os.environ["CPIC_SERVER_NO_BATCH"] = "1"
    try:
        res_u, st_u = run_server(mix, slots=5, budget=1 << 30)
    finally:
        del os.environ["CPIC_SERVER_NO_BATCH"]
    print("[server] batched steps %d / %d, p50 %.3f ms vs %.3f ms" %
          (st_b["batched_steps"], st_u["batched_steps"], st_b["step_p50_ms"], st_u["step_p50_ms"]), flush=True)
    assert all(r["status"] == 0 for r in res_b + res_u)
    for a, b in zip(res_b, res_u):
        same(a, b)
    assert st_b["batched_steps"] == len(group) * NSTEPS and st_u["batched_steps"] == 0


def test_requests_admitted_while_others_run_equal_alone():
    # continuous batching: requests arrive while others are running (two of
    # them join the batch group of a running case mid-way through its steps);
    # every result equals the case served alone
    group = [serving_case(48, 0.10, 12.0, v, 440 + k) for k, v in enumerate((1.0, 0.8, 1.2))]
    other = serving_case(32, 0.05, 16.0, 1.0, 445)
    alone = [run_server([c], slots=1, budget=1 << 30)[0][0] for c in group + [other]]
    srv = C().Server(1 << 30, 4)
    prepared = [descs(c) for c in group + [other]]
    tickets = [srv.submit(*prepared[0], NSTEPS, want_phi=True)]
    srv.pump(3)  # the first case is 3 steps in when the others arrive
    assert srv.poll(tickets[0]) is None
    tickets.append(srv.submit(*prepared[3], NSTEPS, want_phi=True))
    srv.pump(2)
    tickets += [srv.submit(*p, NSTEPS, want_phi=True) for p in prepared[1:3]]
    for _ in range(100000):
        if srv.pump(1):
            break
    res = [srv.poll(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    order = [0, 3, 1, 2]
    for r, k in zip(res, order):
        assert r["status"] == 0
        same(r, alone[k])
    # the late members stepped together with the first while it ran
    assert stats["batched_steps"] > 0
