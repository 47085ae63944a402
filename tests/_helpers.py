"""Shared helpers of the GPU tests: build a library simulation and the oracle
from the same seeded workload."""
import numpy as np

import oracle as O
from paper_1311_2286_amd import workloads as W


def gpu_sim(case, precision=0, shape=2, track_ids=True, mg_rtol=1e-12, mg_max_cycles=80,
            sort_every=1, count=None, capacity_factor=1.0, inject=False, seed=0, stream=None, mover=0,
            pusher=0, mg_method=0):
    """inject: every species gets flux injection at the outer wall with
    n0 = 1 and its own thermal speed, keyed by `seed`."""
    from paper_1311_2286_amd import cpic as C
    dt = np.float64 if precision == C.FP64 else np.float32
    pbc_lo = tuple(0 if b == 0 else C.PBC_ABSORB for b in case.bc_lo)
    pbc_hi = tuple(0 if b == 0 else C.PBC_OUTFLOW for b in case.bc_hi)
    kind, L, vertices = case.map_kind, case.L, None
    if case.tabulated:
        kind, L, vertices = C.MAP_TABULATED, W.table_shift(case), W.vertex_table(case)
    sim = C.Sim(kind, case.dim, case.n, L=L, eps=case.eps, r_in=case.r_in,
                r_out=case.r_out, bc_lo=case.bc_lo, bc_hi=case.bc_hi, phi_lo=case.phi_lo,
                phi_hi=case.phi_hi, shape=shape, precision=precision, dt=case.dt, B0=case.B,
                background=case.background, mg_rtol=mg_rtol, mg_max_cycles=mg_max_cycles,
                sort_every=sort_every, track_ids=track_ids, stream=stream, mover=mover, vertices=vertices,
                pusher=pusher, mg_method=mg_method)
    parts = []
    for sid, s in enumerate(case.species):
        p = W.generate_species(case, sid, dtype=dt, count=count)
        cap = max(1, int(p["cell"].size * capacity_factor))
        sim.add_species(s.q, s.m, case.weight(s), cap, pbc_lo=pbc_lo, pbc_hi=pbc_hi,
                        inject=dict(n0=1.0, vth=s.vth, drift=s.drift * s.vth) if inject else None, seed=seed)
        sim.set_particles(sid, p["cell"], p["off"], p["vel"], p["id"])
        parts.append(p)
    return sim, parts


def oracle_objects(case):
    g = O.make_grid(**case.grid_args())
    if case.tabulated:
        per = [int(case.bc_lo[a] == W.PERIODIC) for a in range(case.dim)]
        m = O.make_tabulated_map(case.dim, case.n, per, W.vertex_table(case), L=W.table_shift(case))
        return m, g
    return O.make_map(**case.map_args()), g


def oracle_species(case, parts):
    sp = []
    for sid, s in enumerate(case.species):
        sp.append(dict(q=s.q, m=s.m, w=case.weight(s), **W.to_oracle(parts[sid])))
    return sp


def by_id(g):
    o = np.argsort(g["id"], kind="stable")
    return dict(cell=g["cell"][o], off=g["off"][:, o], vel=g["vel"][:, o], id=g["id"][o])


def logical_cells(case, cell, off):
    """(n_particles, dim) positions in cell units (i + f, ...) from linear cell
    index and offsets given as (dim, n) or (n, 3)."""
    d = case.dim
    if off.shape[0] != d and off.shape[-1] == 3:
        off = off[:, :d].T
    pos = np.zeros((cell.size, d))
    c = cell.astype(np.int64)
    for a in range(d):
        pos[:, a] = c % case.n[a] + off[a]
        c = c // case.n[a]
    return pos


def periodic_diff(case, a, b):
    d = a - b
    for ax in range(case.dim):
        if case.bc_lo[ax] == 0:
            n = case.n[ax]
            d[:, ax] -= np.round(d[:, ax] / n) * n
    return d


def check_push(case, precision, tag, got_cell, got_off, got_vel, cell, off, vel, vel0, acc_dt,
               pos_tol=1e-5, vel_tol=1e-5):
    """One push from identical states, GPU against oracle, particle by
    particle (the same particles, in the same order, on both sides).
    Positions: largest |difference| in cells <= pos_tol (FP32) or 1e-12
    (FP64).  Velocities: |dv| <= vel_tol (|v0| + |q/m E dt|) per particle
    (FP32), 1e-12 (FP64), vector norms.  Returns the two measured maxima."""
    pg = logical_cells(case, got_cell, got_off.astype(np.float64))
    po = logical_cells(case, cell, off)
    dpos = float(np.abs(periodic_diff(case, pg, po)).max()) if cell.size else 0.0
    dvv = got_vel.T.astype(np.float64) - vel
    if case.dim == 2 and not any(case.B):
        dvv[:, 2] = 0.0  # v_z is not advanced without a magnetic field in 2D
    scale = np.linalg.norm(vel0, axis=1) + np.linalg.norm(acc_dt, axis=1)
    rv = float((np.linalg.norm(dvv, axis=1) / scale).max()) if cell.size else 0.0
    print("[push %s p%d] max |dxi| %.2e cell, max |dv| / (|v| + |a dt|) %.2e" % (tag, precision, dpos, rv))
    pt, vt = (pos_tol, vel_tol) if precision == 0 else (1e-12, 1e-12)
    assert dpos <= pt, (tag, dpos)
    assert rv <= vt, (tag, rv)
    return dpos, rv
