"""GPU test of the preconditioner's FP16 stencil copies at extreme physical
scales.  The flexible-CG solve (Sec. "Field solver") preconditions with an
FP32 V-cycle whose levels above the one-workgroup tail read the stencil from
FP16 copies scaled per level by a power of two (largest coefficient below 1).
The scale keeps the copies inside FP16's range whatever the units: a box
whose lengths are multiplied by 2^-20 or by 1e-5 or 1e5 (the 3D stencil
scales with the cell size) must solve the same discrete system as the FP64
oracle (potential 1e-9 of its maximum after a solve to residual 1e-12) in
the iterations the unscaled box takes (the same with a power-of-two factor,
whose copies carry the same mantissas; within one otherwise)."""
import numpy as np
import pytest

import oracle as O
from paper_1311_2286_amd import workloads as W
from _helpers import gpu_sim, oracle_objects, oracle_species

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


def solve(scale):
    n = (32, 32, 32)
    case = W.small_case(dim=3, n=n, L=tuple(scale * v for v in n), ppc=1.0, case_id=601)
    sim, parts = gpu_sim(case, precision=0, mg_rtol=1e-12)
    for st in (C().STAGE_DEPOSIT, C().STAGE_CHARGE, C().STAGE_SOLVE):
        sim.stage(st)
    phi = sim.get_field(C().FIELD_PHI)
    d = sim.diag()
    sim.close()
    m, g = oracle_objects(case)
    osim = O.OracleSim(m, g, oracle_species(case, parts), dt=case.dt, deposit="fixed", rtol=1e-13)
    osim.deposit()
    osim.solve()
    rel = np.max(np.abs(phi - osim.phi)) / np.max(np.abs(osim.phi))
    print("[scale] %g: %d iterations, relres %.2e, phi rel %.2e" % (scale, d.mg_cycles, d.mg_relres, rel),
          flush=True)
    return d, rel


def test_fp16_stencil_copies_at_extreme_scales():
    d1, rel1 = solve(1.0)
    assert d1.mg_relres <= 1e-12 and rel1 <= 1e-9
    for scale in (2.0 ** -20, 1e-5, 1e5):
        d, rel = solve(scale)
        assert d.mg_relres <= 1e-12, (scale, d.mg_relres)
        assert rel <= 1e-9, (scale, rel)
        if scale == 2.0 ** -20:
            assert d.mg_cycles == d1.mg_cycles, (scale, d.mg_cycles, d1.mg_cycles)
        else:
            assert abs(d.mg_cycles - d1.mg_cycles) <= 1, (scale, d.mg_cycles, d1.mg_cycles)
