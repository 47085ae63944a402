"""cpic_get_diag_noalloc (the diagnostics in the library's per-device scratch
array, for callers that cannot allocate) against cpic_get_diag, through the C
ABI.  Bar: bit-identical output structures and equal status codes, on two
calls in a row where the second simulation is smaller (fewer cells, fewer
species) than the first -- the scratch keeps the first call's contents, so
anything read before it is written would show -- and a non-finite potential
reported by the first call must not leak into the second."""
import ctypes

import numpy as np
import pytest

from paper_1311_2286_amd import workloads as W
from _helpers import gpu_sim

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


def both(sim):
    """(status, raw bytes) of cpic_get_diag_noalloc then cpic_get_diag."""
    out = []
    for fn in (sim.lib.cpic_get_diag_noalloc, sim.lib.cpic_get_diag):
        d = C().Diag()
        st = fn(sim.h, ctypes.byref(d))
        out.append((st, ctypes.string_at(ctypes.addressof(d), ctypes.sizeof(d)), d))
    return out


def sims():
    big = W.small_case(dim=3, n=(20, 12, 16), ppc=4.0, case_id=150)
    small = W.small_case(dim=2, n=(40, 24), ppc=6.0, two_species=False, background=True, case_id=151)
    a, _ = gpu_sim(big, precision=0, mg_rtol=1e-8)
    b, _ = gpu_sim(small, precision=0, mg_rtol=1e-8)
    return a, b


def test_noalloc_diag_equals_get_diag_on_two_calls():
    a, b = sims()
    for sim in (a, b):
        sim.initialize()
        sim.step(3)
    for sim, nsp in ((a, 2), (b, 1)):
        (s1, r1, d1), (s0, r0, d0) = both(sim)
        assert s1 == s0 == 0
        assert r1 == r0
        assert d1.nspecies == nsp and d1.field_energy > 0
        for sid in range(nsp):
            assert C().qsum(d1, sid) == d1.count[sid] << 48
    a.close()
    b.close()


def test_noalloc_diag_reports_and_clears_non_finite():
    import torch
    a, b = sims()
    for sim in (a, b):
        sim.initialize()
        sim.step(1)
    phi = a.get_field(C().FIELD_PHI)
    phi[5] = np.nan
    t = torch.from_numpy(phi).cuda()
    assert a.lib.cpic_set_field(a.h, C().FIELD_PHI, 0, C()._ptr(t), t.numel() * 8, 1) == 0
    (s1, r1, _), (s0, r0, _) = both(a)
    assert s1 == s0 == C().E_NONFINITE and r1 == r0
    # the next call, on a smaller healthy simulation, starts from a cleared count
    (s1, r1, _), (s0, r0, _) = both(b)
    assert s1 == s0 == 0 and r1 == r0
    a.close()
    b.close()
