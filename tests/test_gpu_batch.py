"""GPU tests of batched stepping (cpic_step_batch in include/cpic.h): the field
phases of several simulations of one grid shape (charge, right side, the
flexible-CG solve with its FP32 V-cycle preconditioner, vertex field) run as
one launch per kernel over all of them, the case index in the grid's z extent.

Bar: bitwise (also when the batch's field phase is replayed as a captured
HIP graph).  The batched kernels compute for each case exactly what its own
launch computes, so after the same steps every case's potential, vertex field,
charge, exact deposits, solver cycles and residual and its particles (matched
by id: the order inside a tile after a sort is the atomics') equal those of
the same case stepped alone; kinetic energy to 1e-13 relative (its FP64
per-work-item sums follow the particle order inside a tile).  Each case's
solve stops at its own convergence inside the shared launches, so cases that
need different cycle counts are batched together on purpose."""
import ctypes

import numpy as np
import pytest

from paper_1311_2286_amd import workloads as W
from _helpers import gpu_sim

pytestmark = pytest.mark.gpu

STEPS = 6


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def C():
    from paper_1311_2286_amd import cpic
    return cpic


def variants(dim, k0, n=None, bc=None):
    """Cases of one grid shape and map with different seeds, density
    perturbations and temperatures (so their solves converge in different
    cycle counts)."""
    out = []
    for k, (delta, vth) in enumerate([(0.01, 1.0), (0.08, 0.6), (0.002, 1.6)]):
        c = W.small_case(dim, n=n, vth_e=vth, case_id=k0 + k)
        c.delta = delta
        if bc is not None:
            c.map_kind = W.IDENTITY
            c.eps = 0.0
            c.bc_lo, c.bc_hi, c.phi_lo, c.phi_hi = bc
        out.append(c)
    return out


def make(case, graphs=False, **kw):
    args = dict(precision=0, mg_rtol=1e-10, mg_max_cycles=40, sort_every=2)
    args.update(kw)
    sim, _ = gpu_sim(case, **args)
    sim.initialize()
    if graphs:
        sim.set_graphs(True)
    return sim


def state(sim, case):
    c = C()
    d = sim.diag()
    out = dict(phi=sim.get_field(c.FIELD_PHI), ev=sim.get_field(c.FIELD_EV),
               charge=sim.get_field(c.FIELD_CHARGE), diag=d)
    out["Q"] = [sim.get_field(c.FIELD_Q, sid) for sid in range(len(case.species))]
    parts = []
    for sid in range(len(case.species)):
        g = sim.get_particles(sid)
        o = np.argsort(g["id"], kind="stable")
        parts.append({k: (v[..., o] if k in ("off", "vel") else v[o]) for k, v in g.items()})
    out["parts"] = parts
    return out


def same_state(a, b, tag):
    for k in ("phi", "ev", "charge"):
        assert np.array_equal(a[k], b[k]), (tag, k)
    for sid, (qa, qb) in enumerate(zip(a["Q"], b["Q"])):
        assert np.array_equal(qa, qb), (tag, "Q", sid)
    for sid, (pa, pb) in enumerate(zip(a["parts"], b["parts"])):
        for k in pa:
            assert np.array_equal(pa[k], pb[k]), (tag, "particles", sid, k)
    da, db = a["diag"], b["diag"]
    for f in ("step", "field_energy", "mg_relres", "mg_cycles", "newton_fallback", "far_deposits",
              "newton_failed"):
        assert getattr(da, f) == getattr(db, f), (tag, f, getattr(da, f), getattr(db, f))
    for f in ("count", "absorbed", "outflow", "qsum_lo", "qsum_hi", "sorts"):
        assert list(getattr(da, f)) == list(getattr(db, f)), (tag, f)
    assert abs(da.kinetic - db.kinetic) <= 1e-13 * abs(db.kinetic), (tag, da.kinetic, db.kinetic)


def run_pair(cases, batched_expected, steps=STEPS, **kw):
    c = C()
    alone = [make(case, **kw) for case in cases]
    for _ in range(steps):
        for s in alone:
            s.step(1)
    ref = [state(s, case) for s, case in zip(alone, cases)]
    for s in alone:
        s.close()
    sims = [make(case, **kw) for case in cases]
    for _ in range(steps):
        assert c.step_batch(sims) == [0] * len(sims)
    got = [state(s, case) for s, case in zip(sims, cases)]
    for s in sims:
        s.close()
    for k, (a, b, case) in enumerate(zip(got, ref, cases)):
        print("[batch] %s case %d: cycles %d relres %.3e batched %d" %
              (case.name, k, a["diag"].mg_cycles, a["diag"].mg_relres, a["diag"].batched_steps), flush=True)
        same_state(a, b, "%s/%d" % (case.name, k))
        if batched_expected is not None:
            assert a["diag"].batched_steps == (steps if batched_expected else 0)
        assert b["diag"].batched_steps == 0
    return got


def test_batch_2d_sinusoidal_equals_alone():
    got = run_pair(variants(2, 501), True)
    # the cases converge in different cycle counts inside the shared launches
    assert len({g["diag"].mg_cycles for g in got}) > 1 or len({g["diag"].mg_relres for g in got}) > 1


def test_batch_3d_sinusoidal_equals_alone():
    run_pair(variants(3, 511), True)


def test_batch_2d_walls_equals_alone():
    D, P = W.DIRICHLET, W.PERIODIC
    bc = ((D, P), (D, P), (0.0, 0.0), (1.0, 0.0))
    run_pair(variants(2, 521, n=(48, 40), bc=bc), True)


def test_different_shapes_step_one_by_one():
    cases = [W.small_case(2, case_id=531), W.small_case(2, n=(48, 24), case_id=532)]
    run_pair(cases, False)


def test_different_maps_give_the_same_results():
    # the same grid, maps of different distortion: batched when their solves
    # restrict alike, else stepped one by one; the same results either way
    cases = variants(2, 541)
    cases[1].eps = 0.02
    cases[2].eps = 0.15
    run_pair(cases, None)


def test_vcycle_cases_step_one_by_one():
    run_pair(variants(2, 545)[:2], False, mg_method=1)


def test_refused_case_is_left_out_and_keeps_its_state():
    c = C()
    cases = variants(2, 551)
    ref = [make(case) for case in cases[:2]]
    for s in ref:
        s.step(2)
    want = [state(s, case) for s, case in zip(ref, cases)]
    for s in ref:
        s.close()
    # the middle one is not initialised: cpic_step would refuse it
    sims = [make(cases[0]), gpu_sim(cases[2], precision=0, mg_rtol=1e-10, mg_max_cycles=40, sort_every=2)[0],
            make(cases[1])]
    arr = (ctypes.c_void_p * 3)(*[s.h for s in sims])
    for _ in range(2):
        status = (ctypes.c_int * 3)()
        rc = c.load().cpic_step_batch(arr, 3, status)
        assert rc == c.E_STATE and list(status) == [0, c.E_STATE, 0]
    got = [state(sims[0], cases[0]), state(sims[2], cases[1])]
    for s in sims:
        s.close()
    for a, b in zip(got, want):
        same_state(a, b, "refused")
        assert a["diag"].batched_steps == 2


def test_duplicate_and_empty_batches_are_rejected():
    c = C()
    s = make(variants(2, 561)[0])
    arr = (ctypes.c_void_p * 2)(s.h, s.h)
    assert c.load().cpic_step_batch(arr, 2, None) == c.E_ARG
    assert c.load().cpic_step_batch(arr, 0, None) == c.E_ARG
    assert s.diag().step == 0
    s.close()


def test_batch_signature_and_set_stream():
    torch = pytest.importorskip("torch")
    c = C()
    a, b = variants(2, 571)[:2]
    sa, sb = make(a), make(b)
    other = make(W.small_case(2, n=(48, 24), case_id=573))
    vc = make(a, mg_method=1)
    assert sa.batch_signature() == sb.batch_signature() != 0
    assert other.batch_signature() not in (0, sa.batch_signature())
    assert vc.batch_signature() == 0
    # on different streams they step one by one; moved onto one, batched
    s1 = torch.cuda.Stream()
    sb.set_stream(s1.cuda_stream)
    assert c.step_batch([sa, sb]) == [0, 0]
    assert sa.diag().batched_steps == 0
    sb.set_stream(sa.stream)
    assert c.step_batch([sa, sb]) == [0, 0]
    assert sa.diag().batched_steps == 1 and sb.diag().batched_steps == 1
    for s in (sa, sb, other, vc):
        s.close()


def test_step_ready():
    # ready while the step two before has completed on the device: the first
    # two steps never wait; after a synchronisation every step is ready
    torch = pytest.importorskip("torch")
    s = make(variants(2, 591)[0])
    assert s.step_ready()
    s.step(1)
    assert s.step_ready()
    for _ in range(4):
        s.step(1)
        r = s.step_ready()
        assert r in (True, False)
    torch.cuda.synchronize()
    s.diag()
    assert s.step_ready()
    s.close()


def test_batch_with_graphs_equals_alone():
    # graph mode on a created stream: a batch's field phase is captured once
    # per sequence and replayed as one graph launch per step
    torch = pytest.importorskip("torch")
    st = torch.cuda.Stream()
    run_pair(variants(2, 581), True, steps=8, stream=st.cuda_stream, graphs=True)
    run_pair(variants(3, 585), True, steps=8, stream=st.cuda_stream, graphs=True)
