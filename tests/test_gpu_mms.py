"""GPU field solve of the paper's manufactured-solution test (Sec. "Field
solver", Eqs. r, z, mms; Table t1): the spherical r-z map with the geometric
factor Omega = r, Dirichlet walls at rho = r_1, r_2 and Neumann walls on the
symmetry axis.

Bars:
  - parity: the GPU solve of the same right side matches the oracle's
    conjugate-gradient solution of the same discrete system within 1e-8 of its
    maximum, on a ragged grid (48 x 40) and a square one (64^2);
  - convergence: the error against Eq. mms (RMS over the cell centres) is
    Table t1's L2 error within 10 % on every grid from 64^2 to 2048^2, and
    falls by the paper's ratios on doubling (its 4.1 at 128^2 within 0.3, 4.0
    from 256^2 on within 0.15);
  - the geometric solver's iteration count stays bounded as the grid is
    refined (flexible CG with a point-smoothed V-cycle on rediscretised coarse
    operators: more iterations than the paper's, growing slowly);
  - the variational solver (CPIC_MG_BOXMG: coarse operators P^T A P, zebra
    line relaxation) meets Table t1's iteration counts: at most 6 iterations
    to rtol 1e-10 on every grid from 128^2 to 2048^2, with the same solution;
  - Table t4's flatness (Test B, the charging sphere on this map): over a
    sequence of solves whose right sides change like a PIC run's (each solve
    from the last solution), the average iteration count stays within one of
    its value on the coarsest grid from 32^2 to 256^2, and within Table t4's
    range of 8 to 9 or below.  The right side stands in for Test B's particle
    charge: the manufactured charge with 7 % cell-to-cell noise (about the
    relative noise of 230 particles per cell), redrawn for every solve."""
import numpy as np
import pytest

import oracle as O
from _golden import paper_value
from _mms import R1, R2, spherical_mms

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def gpu_solve(n0, n1, charge, rtol, max_cycles=60, method=0):
    from paper_1311_2286_amd import cpic
    sim = cpic.Sim(cpic.MAP_SPHERICAL_RZ, 2, (n0, n1), r_in=R1, r_out=R2, omega=1,
                   bc_lo=(cpic.BC_DIRICHLET, cpic.BC_NEUMANN), bc_hi=(cpic.BC_DIRICHLET, cpic.BC_NEUMANN),
                   precision=cpic.FP64, mg_rtol=rtol, mg_max_cycles=max_cycles, mg_method=method)
    try:
        sim.set_field(cpic.FIELD_CHARGE, charge)
        sim.stage(cpic.STAGE_SOLVE)
        phi = sim.get_field(cpic.FIELD_PHI)
        d = sim.diag()
        return phi, d.mg_cycles, d.mg_relres
    finally:
        sim.close()


@pytest.mark.parametrize("method", [0, 2])
@pytest.mark.parametrize("n", [(48, 40), (64, 64)])
def test_spherical_solve_matches_oracle(n, method):
    m, g, _, charge = spherical_mms(*n)
    ref, it, rr = O.poisson_solve(m, g, charge, rtol=1e-13)
    assert rr < 1e-12
    phi, cycles, relres = gpu_solve(n[0], n[1], charge, 1e-12, method=method)
    assert relres <= 1e-12 and 0 < cycles < 60, (relres, cycles)
    err = np.max(np.abs(phi - ref)) / np.max(np.abs(ref))
    assert err <= 1e-8, err


def test_species_are_refused_on_the_solve_only_map():
    from paper_1311_2286_amd import cpic
    sim = cpic.Sim(cpic.MAP_SPHERICAL_RZ, 2, (16, 16), r_in=R1, r_out=R2, omega=1,
                   bc_lo=(cpic.BC_DIRICHLET, cpic.BC_NEUMANN), bc_hi=(cpic.BC_DIRICHLET, cpic.BC_NEUMANN))
    with pytest.raises(cpic.CpicError):
        sim.add_species(-1.0, 1.0, 1.0, 100, pbc_lo=(cpic.PBC_ABSORB,) * 2, pbc_hi=(cpic.PBC_ABSORB,) * 2)
    sim.close()


def test_second_order_convergence_and_bounded_iterations():
    sizes = (64, 128, 256, 512, 1024, 2048)
    errs, cycles = [], []
    for N in sizes:
        _, _, exact, charge = spherical_mms(N)
        phi, c, relres = gpu_solve(N, N, charge, 1e-10)
        assert relres <= 1e-10, (N, relres, c)
        errs.append(np.sqrt(np.mean((phi - exact) ** 2)))
        cycles.append(c)
    errs = np.array(errs)
    for N, e in zip(sizes, errs):
        ref = paper_value("mms_l2_%d" % N)
        assert abs(e - ref) < 0.1 * ref, (N, e, ref)
    ratios = errs[:-1] / errs[1:]
    print("MMS L2 errors", errs, "ratios", ratios, "cycles", cycles)
    assert abs(ratios[0] - paper_value("mms_error_ratio_128")) < 0.3, ratios
    for r in ratios[1:]:
        assert abs(r - paper_value("mms_error_ratio_256")) < 0.15, ratios
    assert max(cycles) <= min(cycles) + 6, cycles
    # the geometric preconditioner's strength on this operator (rows scale
    # with r): 12, 12, 13, 14, 15, 16 iterations measured from 64^2 to 2048^2;
    # a weakened preconditioner (e.g. reduced-precision stencil copies of its
    # small rows) shows up here first
    assert cycles[-1] <= 16, cycles


def test_boxmg_iterations_meet_table_t1():
    bar = paper_value("mms_iterations_max")
    out = []
    for N in (128, 256, 512, 1024, 2048):
        _, _, exact, charge = spherical_mms(N)
        phi, c, relres = gpu_solve(N, N, charge, 1e-10, method=2)
        e = np.sqrt(np.mean((phi - exact) ** 2))
        out.append((N, c, relres, e))
        print("[boxmg] %d^2: %d iterations, relres %.2e, L2 error %.3e" % (N, c, relres, e), flush=True)
        assert relres <= 1e-10, (N, relres, c)
        assert c <= bar, (N, c)
        ref = paper_value("mms_l2_%d" % N)
        assert abs(e - ref) < 0.1 * ref, (N, e, ref)


def test_boxmg_iterations_flat_like_table_t4():
    from paper_1311_2286_amd import cpic
    means = []
    for N in (32, 64, 128, 256):
        _, _, _, charge = spherical_mms(N)
        rng = np.random.default_rng(1311 + N)
        sim = cpic.Sim(cpic.MAP_SPHERICAL_RZ, 2, (N, N), r_in=R1, r_out=R2, omega=1,
                       bc_lo=(cpic.BC_DIRICHLET, cpic.BC_NEUMANN), bc_hi=(cpic.BC_DIRICHLET, cpic.BC_NEUMANN),
                       phi_lo=(-2.5, 0.0), precision=cpic.FP64, mg_rtol=1e-10, mg_max_cycles=40, mg_method=2)
        its = []
        try:
            for k in range(12):
                sim.set_field(cpic.FIELD_CHARGE, charge * (1.0 + 0.07 * rng.standard_normal(charge.size)))
                sim.stage(cpic.STAGE_SOLVE)
                d = sim.diag()
                assert d.mg_relres <= 1e-10, (N, k, d.mg_relres)
                its.append(d.mg_cycles)
        finally:
            sim.close()
        means.append(float(np.mean(its[2:])))
        print("[boxmg] Test B stand-in %d^2: iterations %s" % (N, its), flush=True)
    assert max(means) - means[0] <= 1.0, means
    assert max(means) <= paper_value("testb_iterations_max"), means
