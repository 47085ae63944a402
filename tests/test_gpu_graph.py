"""Graph mode (cpic_set_graphs): steps replayed from recorded HIP graphs give
the results of the ordinary path, step after step, across tile sorts and both
particle-buffer parities, with ordinary synchronising calls between the
replays.  Both simulations run on a torch stream of default priority (the null
stream cannot be captured).

Bars, FP32 path (integer deposit): potential, vertex field, field energy,
counts, exact charge sums and every particle (matched by identifier) bitwise;
kinetic energy to 1e-13 relative (its FP64 per-work-item sums follow the
order of particles inside a tile, which the tile sort does not fix).  FP64
path (FP64 atomic deposit, rounding order free): 1e-11 relative throughout."""
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


def _close(x, y, tol):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if tol == 0:
        return np.array_equal(x, y)
    return np.max(np.abs(x - y)) <= tol * max(np.max(np.abs(x)), 1e-300)


def _same(a, b, exact):
    tol = 0 if exact else 1e-11
    da, db = a.diag(), b.diag()
    assert da.step == db.step
    assert abs(da.kinetic - db.kinetic) <= (1e-13 if exact else tol) * abs(da.kinetic)
    assert _close(da.field_energy, db.field_energy, tol)
    for sid in range(da.nspecies):
        assert da.count[sid] == db.count[sid]
        if exact:
            assert (da.qsum_lo[sid], da.qsum_hi[sid]) == (db.qsum_lo[sid], db.qsum_hi[sid])
    assert _close(a.get_field(C().FIELD_PHI), b.get_field(C().FIELD_PHI), tol)
    assert _close(a.get_field(C().FIELD_EV), b.get_field(C().FIELD_EV), tol)
    return db


@pytest.mark.parametrize("name,precision", [("2d", 0), ("3d", 0), ("2d", 1), ("3d_cyclotronic", 0)])
def test_graph_steps_are_bitwise_the_ordinary_steps(name, precision):
    import torch
    st = torch.cuda.Stream()
    pusher = 0
    if name == "2d":
        case = W.small_case(dim=2, n=(40, 24), ppc=8.0)
    elif name == "3d":
        case = W.small_case(dim=3, n=(20, 12, 16), ppc=4.0)
    else:
        # the cyclotronic variant of the particle kernel, omega_ce dt = 2
        case = W.small_case(dim=3, n=(20, 12, 16), ppc=4.0, B=(0.0, 0.0, 20.0))
        pusher = C().PUSH_CYCLOTRONIC
    a, _ = gpu_sim(case, precision=precision, sort_every=3, mg_rtol=1e-9, stream=st.cuda_stream, pusher=pusher)
    b, _ = gpu_sim(case, precision=precision, sort_every=3, mg_rtol=1e-9, stream=st.cuda_stream, pusher=pusher)
    b.set_graphs(True)
    a.initialize()
    b.initialize()
    for k in range(8):
        a.step(1)
        b.step(1)
        db = _same(a, b, precision == 0)
    # variants: sort or not x buffer parity x cycles launched, and the first
    # (not extrapolated) step: graphs were recorded and reused
    assert 3 <= db.step_graphs < 8, db.step_graphs
    a.step(7)
    b.step(7)
    _same(a, b, precision == 0)
    for sid in range(len(case.species)):
        pa, pb = by_id(a.get_particles(sid)), by_id(b.get_particles(sid))
        assert np.array_equal(pa["id"], pb["id"])
        assert np.array_equal(pa["cell"], pb["cell"])
        for f in ("off", "vel"):
            assert _close(pa[f], pb[f], 0 if precision == 0 else 1e-11), f
    a.close()
    b.close()
