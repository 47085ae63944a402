"""GPU parity of tabulated maps (CPIC_MAP_TABULATED: the map known at the
vertices, its metric by finite differences; Sec. "Curvilinear formulation")
against the oracle's tabulated map, through the C ABI.

Bars: charge 1e-14 relative, potential 1e-9 of its maximum, vertex field 1e-6
(FP32 storage) / 1e-10 (FP64) of its maximum -- as for the analytic maps;
pushes as for the analytic maps (FP32 1e-5 cell and 1e-5 (|v| + |q/m E dt|),
FP64 1e-12); three FP64 steps: potential 1e-10, positions 1e-10 cell.
Cases: the 2D and 3D sinusoidal maps (periodic, mixed terms) and the
polar-log annulus with walls, each sampled at its vertices.  The GPU solve on
the sampled map converges at second order (or faster) in h to the solve on
the analytic map (difference ratio at least 3.5 per doubling).  Tables that fold, or that are not
orthogonal at walls, are refused at creation.  Pushes with the Newton
mover (inverting the multilinear interpolant of the vertex coordinates) match
the oracle's inversion of the same map, one push in FP32 and FP64 and three
full FP64 steps; the predictor-corrector mover on tabulated maps is in its own
tests."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_1311_2286_amd import workloads as W
from _helpers import check_push, gpu_sim, oracle_objects, oracle_species

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


def probe_case(n=(48, 40)):
    return W.Case("probe_tab", 2, W.POLAR_LOG, n, r_in=1.0, r_out=10.0,
                  bc_lo=(W.DIRICHLET, W.PERIODIC), bc_hi=(W.DIRICHLET, W.PERIODIC),
                  phi_lo=(-5.0, 0.0), phi_hi=(0.0, 0.0), dt=0.1,
                  species=[W.electrons(1.0, 4.0), W.ions(ppc=4.0)], case_id=160)


CASES = {
    "2d_sin": lambda: dataclasses.replace(W.small_case(dim=2, n=(40, 24), ppc=8.0, case_id=161), tabulated=True),
    "3d_sin": lambda: dataclasses.replace(W.small_case(dim=3, n=(20, 12, 16), ppc=4.0, case_id=162),
                                          tabulated=True),
    "probe": lambda: dataclasses.replace(probe_case(), tabulated=True),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precision", [0, 1])
def test_charge_solve_and_field(name, precision):
    case = CASES[name]()
    sim, parts = gpu_sim(case, precision=precision, mg_rtol=1e-12, mover=C().MOVER_PC)
    sim.stage(C().STAGE_DEPOSIT)
    sim.stage(C().STAGE_CHARGE)
    sim.stage(C().STAGE_SOLVE)
    sim.stage(C().STAGE_EFIELD)
    m, g = oracle_objects(case)
    osim = O.OracleSim(m, g, oracle_species(case, parts), dt=case.dt,
                       deposit="fixed" if precision == 0 else "f64", rtol=1e-13, mover="pc")
    osim.deposit()
    ch = sim.get_field(C().FIELD_CHARGE)
    assert np.max(np.abs(ch - osim.charge)) <= 1e-14 * np.max(np.abs(osim.charge)) + 1e-300
    jc = sim.get_field(C().FIELD_JC)
    _, _, _, Jo = O.map_eval(m, _centres(case.n))
    assert np.max(np.abs(jc - Jo)) <= 1e-13 * np.max(np.abs(Jo))
    osim.solve()
    phi = sim.get_field(C().FIELD_PHI)
    print("[tabulated] %s p%d phi %.2e" % (name, precision, np.max(np.abs(phi - osim.phi)) / np.max(np.abs(osim.phi))))
    assert np.max(np.abs(phi - osim.phi)) <= 1e-9 * np.max(np.abs(osim.phi))
    d = sim.diag()
    assert d.mg_relres <= 1e-12 and d.mg_cycles > 0
    Ev = sim.get_field(C().FIELD_EV)[:, : case.dim].astype(np.float64)
    tol = 1e-6 if precision == 0 else 1e-10
    Emax = np.max(np.abs(osim.Ev))
    assert np.max(np.abs(Ev - osim.Ev[:, : case.dim])) <= tol * Emax
    sim.close()


def _centres(n):
    d = len(n)
    axes = [(np.arange(n[a]) + 0.5) / n[a] for a in range(d)]
    G = [g.ravel() for g in np.meshgrid(*axes[::-1], indexing="ij")[::-1]]
    xi = np.zeros((G[0].size, 3))
    for a in range(d):
        xi[:, a] = G[a]
    return xi


def _solve(case, charge):
    cp = C()
    kind, L, vertices = case.map_kind, case.L, None
    if case.tabulated:
        kind, L, vertices = cp.MAP_TABULATED, W.table_shift(case), W.vertex_table(case)
    sim = cp.Sim(kind, case.dim, case.n, L=L, eps=case.eps, r_in=case.r_in, r_out=case.r_out,
                 bc_lo=case.bc_lo, bc_hi=case.bc_hi, phi_lo=case.phi_lo, phi_hi=case.phi_hi,
                 precision=cp.FP64, mg_rtol=1e-12, mg_max_cycles=80, vertices=vertices)
    try:
        sim.set_field(cp.FIELD_CHARGE, charge)
        sim.stage(cp.STAGE_SOLVE)
        assert sim.diag().mg_relres <= 1e-12
        return sim.get_field(cp.FIELD_PHI)
    finally:
        sim.close()


@pytest.mark.parametrize("kind", ["sinusoidal", "polar"])
def test_solve_converges_to_the_analytic_map(kind):
    errs = []
    for N in (32, 64, 128):
        if kind == "sinusoidal":
            case = W.small_case(dim=2, n=(N, N), ppc=1.0, case_id=163)
        else:
            case = probe_case((N, N))
        xi = _centres(case.n)
        # a smooth charge, the same on both maps (neutral on the periodic one)
        charge = np.cos(2 * np.pi * xi[:, 0]) * np.sin(4 * np.pi * xi[:, 1]) / N ** 2
        if kind == "sinusoidal":
            charge -= charge.mean()
        pa = _solve(case, charge)
        pt = _solve(dataclasses.replace(case, tabulated=True), charge)
        errs.append(np.max(np.abs(pt - pa)) / np.max(np.abs(pa)))
    e = np.array(errs)
    r = e[:-1] / e[1:]
    # at least second order (the annulus, whose potential is close to the
    # vacuum solution linear in xi, converges faster: ratio about 8)
    assert np.all(r > 3.5), (e, r)


def _create(case, vertices, L=None):
    cp = C()
    return cp.Sim(cp.MAP_TABULATED, case.dim, case.n, L=L or W.table_shift(case), bc_lo=case.bc_lo,
                  bc_hi=case.bc_hi, phi_lo=case.phi_lo, precision=cp.FP64, vertices=vertices)


def test_tables_that_fold_or_skew_at_walls_are_refused():
    cp = C()
    case = CASES["2d_sin"]()
    v = W.vertex_table(case)
    v[0, 5] += 2.5 * (v[0, 6] - v[0, 5])  # a vertex moved past its neighbour's neighbour
    with pytest.raises(cp.CpicError) as e:
        _create(case, v)
    assert e.value.status == -2
    # a sheared annulus: the radial lines lean, not orthogonal to the walls
    pc = probe_case()
    v = W.vertex_table(pc)
    nv0 = pc.n[0] + 1
    i = np.arange(v.shape[1]) % nv0
    th = 0.6 * i / pc.n[0]
    x, y = v[0].copy(), v[1].copy()
    v[0], v[1] = x * np.cos(th) - y * np.sin(th), x * np.sin(th) + y * np.cos(th)
    with pytest.raises(cp.CpicError) as e:
        _create(pc, v)
    assert e.value.status == -9
    # the unsheared table is accepted
    _create(pc, W.vertex_table(pc)).close()


PUSH_CASES = {
    "2d_sin": lambda: dataclasses.replace(W.small_case(dim=2, n=(40, 24), ppc=8.0, case_id=164), tabulated=True),
    "3d_sin": lambda: dataclasses.replace(W.small_case(dim=3, n=(20, 12, 16), ppc=4.0, case_id=165),
                                          tabulated=True),
    "probe": lambda: dataclasses.replace(probe_case(), tabulated=True, case_id=166),
}


@pytest.mark.parametrize("name", sorted(PUSH_CASES))
@pytest.mark.parametrize("precision", [0, 1])
def test_newton_push_on_the_tabulated_map(name, precision):
    # the hybrid mover inverting the tabulated map (its multilinear
    # interpolant) by Newton, against the oracle's inversion of the same map;
    # bars as for the analytic maps
    from _helpers import by_id, logical_cells, periodic_diff
    case = PUSH_CASES[name]()
    sim, parts = gpu_sim(case, precision=precision, mover=C().MOVER_NEWTON)
    ec = 4 if case.dim == 3 else 2
    nv = sim.field_bytes(C().FIELD_EV) // (4 if precision == 0 else 8) // ec
    E = W.synthetic_ev(case, nv, dtype=np.float64 if precision else np.float32)
    Ebuf = np.zeros((nv, ec), dtype=E.dtype)
    Ebuf[:, : case.dim] = E[:, : case.dim]
    sim.set_field(C().FIELD_EV, Ebuf)
    sim.stage(C().STAGE_PUSH)
    m, g = oracle_objects(case)
    E64 = np.zeros((nv, 3))
    E64[:, : case.dim] = Ebuf[:, : case.dim].astype(np.float64)
    d = sim.diag()
    for sid, s in enumerate(case.species):
        o = W.to_oracle(parts[sid])
        cell, off, vel, cnt = O.push(m, g, s.q / s.m, case.dt, case.B, o["cell"], o["off"], o["vel"], E64)
        assert (d.absorbed[sid], d.outflow[sid]) == cnt
        got = by_id(sim.get_particles(sid, cap=parts[sid]["cell"].size))
        alive = cell >= 0
        gl = got["cell"] >= 0
        assert np.array_equal(gl, alive)
        Eo = O.gather(g, E64, o["cell"], o["off"])
        check_push(case, precision, "tabulated newton %s sid %d" % (name, sid), got["cell"][gl],
                   got["off"][:, gl], got["vel"][:, gl], cell[alive], off[alive], vel[alive],
                   o["vel"][alive], (s.q / s.m * case.dt) * Eo[alive])
    assert d.newton_failed == 0
    sim.close()


def test_newton_three_steps_fp64_match_the_oracle():
    from _helpers import by_id, logical_cells, periodic_diff
    case = PUSH_CASES["2d_sin"]()
    sim, parts = gpu_sim(case, precision=1, mover=C().MOVER_NEWTON, mg_rtol=1e-13)
    m, g = oracle_objects(case)
    osim = O.OracleSim(m, g, oracle_species(case, parts), dt=case.dt, deposit="f64", rtol=1e-13, ke_axes=2)
    sim.initialize()
    osim.initialize()
    for k in range(3):
        sim.step(1)
        osim.step()
        phi = sim.get_field(C().FIELD_PHI)
        rel = np.max(np.abs(phi - osim.phi)) / np.max(np.abs(osim.phi))
        print("[tabulated newton 3 steps] k %d phi %.2e" % (k, rel))
        assert rel < 1e-10, k
    for sid in range(len(case.species)):
        got = by_id(sim.get_particles(sid))
        o = osim.sp[sid]
        order = np.argsort(parts[sid]["id"])
        pg = logical_cells(case, got["cell"], got["off"].astype(np.float64))
        po = logical_cells(case, o["cell"][order], o["off"][order])
        dmax = np.abs(periodic_diff(case, pg, po)).max()
        print("[tabulated newton 3 steps] sid %d dpos %.2e" % (sid, dmax))
        assert dmax < 1e-10
    sim.close()
