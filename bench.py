#!/usr/bin/env python3
"""Benchmark: particle pushes/s of the curvilinear PIC step on one MI355X.

Default workload: the 3D periodic box (128^3 cells, sinusoidal map eps = 0.05
on all axes, 32 electrons + 32 ions per cell = 134,217,728 particles,
m_i/m_e = 1836, T_i = T_e), FP32 particles with the 64-bit fixed-point
deposit, order-2 B-spline deposit; the plain FP64 path is timed on the same
workload beside it.  A step is one full PIC cycle (particle kernel: gather +
push + Newton map inversion + boundaries + deposit; charge; multigrid solve;
vertex field; tile sort).  Inputs are resident in HBM before the timed region.

Prints one JSON line: the throughput over whole steps, the per-phase split,
the particle kernel against the HBM roofline, the FP64 path beside it and the
oracle timed on the host cores."""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "particle_kernel_box3d_128_traffic.md")
KERNEL_SOURCES = ["paper_1311_2286_amd/csrc/particles.hip", "paper_1311_2286_amd/csrc/common.hpp",
                  "paper_1311_2286_amd/csrc/kernels.hpp"]
METRIC = "particle pushes/s (gather+push+map-invert+deposit) FP32 vs FP64; p50/p99 step ms"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def workload(name):
    from paper_1311_2286_amd import workloads as W
    return {"box3d_128": W.case2, "langmuir2d": W.case1, "box3d_magnetized": W.case5,
            "probe2d_512": W.case3}[name]()


def bytes_per_particle(dim, precision, magnetic):
    """Algorithmic HBM bytes per particle push: state read once and written
    once.  FP32: int32 cell + dim FP32 offsets + FP32 velocities (2 in 2D
    without B, else 3).  Plain FP64: the logical position and the velocity,
    dim + 3 (2 in 2D without B) FP64 values -- the library stores the position
    as an int32 cell and FP64 offsets, 8 B more per particle than counted."""
    nv = 3 if (dim == 3 or magnetic) else 2
    if precision == 1:
        return 2 * (8 * dim + 8 * nv)
    return 2 * (4 + 4 * dim + 4 * nv)


def layout_bytes_per_particle(dim, precision, magnetic):
    """Bytes the library's layout moves per particle push (int32 cell kept on
    the FP64 path too)."""
    r = 8 if precision == 1 else 4
    nv = 3 if (dim == 3 or magnetic) else 2
    return 2 * (4 + dim * r + nv * r)


def bytes_per_cell(dim, precision):
    """Per cell per particle-kernel launch: the vertex field read (dim
    components) and the species' deposit written (8 B)."""
    r = 8 if precision == 1 else 4
    return dim * r + 8


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload_name, shape, precision_tag):
    """HBM bytes per particle-kernel launch from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE per dispatch, each scaled by the factor a plain
    copy of known size gives), or None when the summary is absent, covers
    another configuration, or was taken on different kernel sources."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    kv = {}
    with open(TRAFFIC_SUMMARY) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#", "|", "`")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_sha():
        return None
    if kv.get("workload") != workload_name or kv.get("shape") != shape or kv.get("precision") != precision_tag:
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibrate(nbytes, reps):
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters to bytes: each launch reads and writes nbytes."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read_per_launch": nbytes, "copy_bytes_written_per_launch": nbytes,
                      "launches": reps}), flush=True)


_STREAM = None


def make_sim(case, precision, shape, sort_every, mg_rtol, mg_cycles, parts, graphs=False, mover=0, pusher=0,
             track_ids=False):
    """graphs: step in graph mode, on a stream of its own (default priority);
    mover: 0 Newton map inversion, 1 predictor-corrector; pusher: 0 Boris,
    1 cyclotronic."""
    global _STREAM
    import torch
    from paper_1311_2286_amd import cpic as C
    stream = None
    if graphs:
        if _STREAM is None:
            _STREAM = torch.cuda.Stream()
        stream = _STREAM.cuda_stream
    from paper_1311_2286_amd import workloads as W
    kind, L, vertices = case.map_kind, case.L, None
    if case.tabulated:  # the map known at its vertices only
        kind, L, vertices = C.MAP_TABULATED, W.table_shift(case), W.vertex_table(case)
    sim = C.Sim(kind, case.dim, case.n, L=L, eps=case.eps, r_in=case.r_in,
                r_out=case.r_out, bc_lo=case.bc_lo, bc_hi=case.bc_hi, phi_lo=case.phi_lo,
                phi_hi=case.phi_hi, shape=shape, precision=precision, dt=case.dt, B0=case.B,
                background=case.background, mg_rtol=mg_rtol, mg_max_cycles=mg_cycles,
                sort_every=sort_every, track_ids=track_ids, stream=stream, mover=mover, vertices=vertices,
                pusher=pusher)
    del vertices
    if graphs:
        sim.set_graphs(True)
    bounded = any(b != 0 for b in case.bc_lo[: case.dim])
    # the particles cross PCIe once, here (host arrays in, resident in HBM
    # from then on): timed, for the rate that includes the upload
    upload_s, upload_bytes = 0.0, 0
    for sid, s in enumerate(case.species):
        p = parts[sid]
        n = p["cell"].size
        pbc_lo = tuple(0 if b == 0 else C.PBC_ABSORB for b in case.bc_lo)
        pbc_hi = tuple(0 if b == 0 else C.PBC_OUTFLOW for b in case.bc_hi)
        # bounded problems (the probe): Maxwellian flux injection at the outer
        # wall keeps the plasma supplied; room for the particle count to grow
        inject = dict(n0=1.0, vth=s.vth) if bounded else None
        cap = int(n * 1.3) if bounded else n
        sim.add_species(s.q, s.m, case.weight(s), cap, pbc_lo=pbc_lo, pbc_hi=pbc_hi, inject=inject,
                        seed=1311 + sid)
        from paper_1311_2286_amd import workloads as W
        q = W.as_dtype(p, np.float64 if precision == 1 else np.float32)
        torch.cuda.synchronize()
        t_up = time.perf_counter()
        sim.set_particles(sid, q["cell"], q["off"], q["vel"])
        sim.sync()
        upload_s += time.perf_counter() - t_up
        upload_bytes += q["cell"].nbytes + q["off"].nbytes + q["vel"].nbytes
        del q
    sim.upload_s, sim.upload_bytes = upload_s, upload_bytes
    return sim


def run_path(case, parts, precision, shape, steps, warmup, sort_every, mg_rtol, mg_cycles,
             graphs=False, mover=0, pusher=0):
    import torch
    from paper_1311_2286_amd import cpic as C
    t0 = time.time()
    sim = make_sim(case, precision, shape, sort_every, mg_rtol, mg_cycles, parts, graphs, mover, pusher)
    sim.initialize()
    sim.sync()
    log("precision", precision, "set up + initialise %.1f s" % (time.time() - t0))
    if warmup > 0:
        sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    sim.set_timing(True)
    t1 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    tm = sim.get_timing()
    d = sim.diag()
    sim.set_timing(False)
    n_p = sum(p["cell"].size for p in parts)
    if any(b != 0 for b in case.bc_lo[: case.dim]):
        n_p = int(sum(d.count[k] for k in range(d.nspecies)))  # after injection and absorption
    res = dict(wall_s=wall, ms_per_step=1e3 * wall / steps, pushes=n_p,
               upload_s=sim.upload_s, upload_bytes=sim.upload_bytes,
               pushes_per_s=n_p * steps / wall,
               push_ms=float(np.mean(tm["push"])), solve_ms=float(np.mean(tm["solve"])),
               sort_ms=float(np.mean(tm["sort"])),
               p50_step_ms=float(np.percentile(tm["step"], 50)),
               p99_step_ms=float(np.percentile(tm["step"], 99)),
               mg_cycles_last=int(d.mg_cycles), mg_relres_last=float(d.mg_relres),
               newton_fallback=int(d.newton_fallback), newton_failed=int(d.newton_failed),
               far_deposits=int(d.far_deposits))
    nspec = len(parts)
    magnetic = any(case.B)
    bp = bytes_per_particle(case.dim, precision, magnetic)
    bc = bytes_per_cell(case.dim, precision)
    per_launch = (n_p / nspec) * bp + case.ncells * bc
    launch_ms = res["push_ms"] / nspec
    res["kernel_pushes_per_s"] = n_p / (res["push_ms"] * 1e-3)
    res["bytes_per_particle"] = bp
    res["bytes_per_cell"] = bc
    res["bytes_per_launch"] = per_launch
    res["launch_ms"] = launch_ms
    res["achieved_GBs"] = per_launch / (launch_ms * 1e-3) / 1e9
    sim.close()
    torch.cuda.empty_cache()
    return res


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(case, sample, shape, single_sample=1 << 18):
    """The FP64 oracle (gather + Boris + exact map inversion + deposit) on the
    host cores, on the first `sample` particles of each species, with all of
    the oracle's OpenMP threads; and on the first `single_sample` with one."""
    import oracle as O
    from paper_1311_2286_amd import workloads as W
    m = O.make_map(**case.map_args())
    g = O.make_grid(**case.grid_args())
    nv = O.nverts(g)
    E = W.synthetic_ev(case, nv, dtype=np.float64, scale=0.05)
    S1 = 24 if case.dim == 2 else 16
    threads = O.num_threads()

    def run(count):
        t_total, n_total = 0.0, 0
        for sid, s in enumerate(case.species):
            p = W.to_oracle(W.generate_species(case, sid, dtype=np.float32, count=count, workers=16))
            t0 = time.perf_counter()
            cell, off, vel, _ = O.push(m, g, s.q / s.m, case.dt, case.B, p["cell"], p["off"], p["vel"], E)
            O.deposit_fixed(g, shape, S1, cell, off)
            t_total += time.perf_counter() - t0
            n_total += p["cell"].size
            del p, cell, off, vel
        return n_total, t_total

    n_all, t_all = run(sample)
    O.set_num_threads(1)
    try:
        n_one, t_one = run(single_sample)
    finally:
        O.set_num_threads(threads)
    return dict(value=n_all / t_all, unit="particle pushes/s", cores=threads, kind="oracle",
                sample="%d particles per species (first of each seeded stream), one "
                       "gather+push+map-inversion+deposit pass, %.1f s on %d threads"
                       % (sample, t_all, threads),
                single_thread_value=n_one / t_one,
                single_thread_sample="%d particles per species, %.1f s on 1 thread" % (single_sample, t_one),
                cpu_model=_cpu_model())


def cpu_configs(shape):
    """The oracle timed on the host cores for the other configurations (all
    its OpenMP threads): the 2D Langmuir workload whole (65,536 electrons, ion
    background, 200 steps: push, deposit and the FP64 field solve every step);
    one full step of the probe (52M particles: push, deposit, field solve on
    512^2); one push + deposit pass of the magnetised box on an 8.4M-particle
    sample per species (a whole step of 268M particles takes minutes)."""
    import oracle as O
    from paper_1311_2286_amd import workloads as W
    out = {}
    threads = O.num_threads()
    # config 1: the whole run
    case = W.case1()
    m, g = O.make_map(**case.map_args()), O.make_grid(**case.grid_args())
    p = W.generate_species(case, 0, dtype=np.float32, workers=16)
    sp = [dict(q=case.species[0].q, m=case.species[0].m, w=case.weight(case.species[0]), **W.to_oracle(p))]
    t0 = time.perf_counter()
    bg = O.ion_background(m, g, shape)
    osim = O.OracleSim(m, g, sp, shape=shape, dt=case.dt, background=bg, deposit="fixed", rtol=1e-13,
                       ke_axes=2)
    osim.initialize()
    for _ in range(case.steps):
        osim.step()
    t = time.perf_counter() - t0
    out["langmuir2d"] = {"value": p["cell"].size * case.steps / t, "unit": "particle pushes/s", "cores": threads,
                         "sample": "the whole run: %d electrons, %d steps (push, deposit, FP64 solve to 1e-13), "
                                   "%.1f s" % (p["cell"].size, case.steps, t)}
    del osim, sp, p
    # config 3: one full step
    case = W.case3()
    m, g = O.make_map(**case.map_args()), O.make_grid(**case.grid_args())
    nv = O.nverts(g)
    E = W.synthetic_ev(case, nv, dtype=np.float64, scale=0.05)
    t_push, n = 0.0, 0
    Q = []
    for sid, sp_ in enumerate(case.species):
        q = W.to_oracle(W.generate_species(case, sid, dtype=np.float32, workers=16))
        t0 = time.perf_counter()
        cell, off, vel, _ = O.push(m, g, sp_.q / sp_.m, case.dt, case.B, q["cell"], q["off"], q["vel"], E)
        Q.append(O.deposit_fixed(g, shape, 24, cell[cell >= 0], off[cell >= 0]))
        t_push += time.perf_counter() - t0
        n += q["cell"].size
        del q, cell, off, vel
    t0 = time.perf_counter()
    charge = O.charge_from_Q(Q, [dict(q=s_.q, w=case.weight(s_)) for s_ in case.species], 2, 24)
    phi, _, _ = O.poisson_solve(m, g, charge, rtol=1e-10)
    O.efield(m, g, phi)
    t_solve = time.perf_counter() - t0
    out["probe2d_512"] = {"value": n / (t_push + t_solve), "unit": "particle pushes/s", "cores": threads,
                          "sample": "one full step: %d particles pushed and deposited (%.1f s), field solve of "
                                    "512^2 to 1e-10 (%.1f s)" % (n, t_push, t_solve)}
    del Q, charge
    # config 5: push + deposit pass on a sample
    case = W.case5()
    m, g = O.make_map(**case.map_args()), O.make_grid(**case.grid_args())
    E = W.synthetic_ev(case, O.nverts(g), dtype=np.float64, scale=0.05)
    t_all, n = 0.0, 0
    for sid, sp_ in enumerate(case.species):
        q = W.to_oracle(W.generate_species(case, sid, dtype=np.float32, count=1 << 23, workers=16))
        t0 = time.perf_counter()
        cell, off, vel, _ = O.push(m, g, sp_.q / sp_.m, case.dt, case.B, q["cell"], q["off"], q["vel"], E)
        O.deposit_fixed(g, shape, 16, cell, off)
        t_all += time.perf_counter() - t0
        n += q["cell"].size
        del q, cell, off, vel
    out["box3d_magnetized"] = {"value": n / t_all, "unit": "particle pushes/s", "cores": threads,
                               "sample": "%d particles per species (first of each seeded stream), one gather + "
                                         "Boris + map inversion + deposit pass, %.1f s" % (n // 2, t_all)}
    return out


def error_vs_oracle(shape, sort_every, mg_rtol, mg_cycles, steps=6):
    """Error of the timed configuration (FP32 particles, fixed-point deposit,
    the solver at the benchmark's tolerance and iteration cap, the tile sort
    schedule) against the FP64 oracle, from the same initial state, on the
    headline recipe at 24^3 cells (32 e + 32 i per cell): after each step the
    largest relative difference of the charge per cell (rho), the potential
    and the vertex field (to their maxima), of the field energy, and the
    largest trajectory difference in cells; against the oracle with the same
    fixed-point deposit rule and against the plain FP64 oracle (unquantised
    deposit).  Largest over the steps."""
    import oracle as O
    from paper_1311_2286_amd import cpic as C
    from paper_1311_2286_amd import workloads as W
    n = (24, 24, 24)
    case = W.Case("box3d_24", 3, W.SINUSOIDAL, n, L=(24.0, 24.0, 24.0), eps=0.05, dt=0.1,
                  species=[W.electrons(1.0, 32.0), W.ions(ppc=32.0)], delta=0.01, case_id=2)
    parts = [W.generate_species(case, sid, dtype=np.float32) for sid in range(2)]
    sim = make_sim(case, C.FP32, shape, sort_every, mg_rtol, mg_cycles, parts, track_ids=True)
    m, g = O.make_map(**case.map_args()), O.make_grid(**case.grid_args())
    sims = {}
    for tag, dep in (("fixed_deposit_oracle", "fixed"), ("plain_fp64_oracle", "f64")):
        sp = [dict(q=s.q, m=s.m, w=case.weight(s), **W.to_oracle(parts[k])) for k, s in enumerate(case.species)]
        sims[tag] = O.OracleSim(m, g, sp, shape=shape, dt=case.dt, deposit=dep, rtol=1e-13, ke_axes=3)
        sims[tag].initialize()
    sim.initialize()
    rel = lambda a, b: float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
    worst = {tag: {} for tag in sims}
    for _ in range(steps):
        sim.step(1)
        ch, phi = sim.get_field(C.FIELD_CHARGE), sim.get_field(C.FIELD_PHI)
        Ev = sim.get_field(C.FIELD_EV)[:, :3].astype(np.float64)
        we = sim.diag().field_energy
        got = []
        for sid in range(2):
            gp = sim.get_particles(sid)
            o = np.argsort(gp["id"])
            c = gp["cell"][o].astype(np.int64)
            got.append(np.stack([c % n[0] + gp["off"][0][o], (c // n[0]) % n[1] + gp["off"][1][o],
                                 c // (n[0] * n[1]) + gp["off"][2][o]], axis=1))
        for tag, osim in sims.items():
            osim.step()
            e = {"rho": rel(ch, osim.charge), "phi": rel(phi, osim.phi), "E": rel(Ev, osim.Ev[:, :3]),
                 "W_E": abs(we - osim.field_energy()) / abs(osim.field_energy())}
            tr = 0.0
            for sid in range(2):
                oc = osim.sp[sid]["cell"].astype(np.int64)
                oo = osim.sp[sid]["off"]
                po = np.stack([oc % n[0] + oo[:, 0], (oc // n[0]) % n[1] + oo[:, 1],
                               oc // (n[0] * n[1]) + oo[:, 2]], axis=1)
                dd = got[sid] - po
                dd -= np.round(dd / np.array(n)) * np.array(n)
                tr = max(tr, float(np.abs(dd).max()))
            e["trajectory_cells"] = tr
            for k, v in e.items():
                worst[tag][k] = max(worst[tag].get(k, 0.0), v)
    sim.close()
    out = {"workload": "box3d recipe at 24^3 (eps 0.05, 32 e + 32 i per cell), %d steps, FP32 path at the "
                       "benchmark's solver settings (rtol %g, at most %d iterations) and sort schedule"
                       % (steps, mg_rtol, mg_cycles), "largest_over_steps": worst}
    return out


def serving_requests(nreq, seed=1311):
    """The serving stream: 2D periodic sinusoidal-map cases, eps ~ U[0, 0.15],
    L = N, grid from {32^2, 64^2, 128^2, 256^2}, 16..128 electrons per cell
    on a fixed ion background, v_th ~ U[0.5, 2], dt = 0.1."""
    from paper_1311_2286_amd import workloads as W
    rng = np.random.default_rng(seed)
    out = []
    for k in range(nreq):
        n = int(rng.choice([32, 64, 128, 256]))
        eps = float(rng.uniform(0.0, 0.15))
        ppc = int(rng.integers(16, 129))
        vth = float(rng.uniform(0.5, 2.0))
        out.append(W.Case("serve_%d" % k, 2, W.SINUSOIDAL, (n, n), L=(float(n), float(n)), eps=eps,
                          dt=0.1, species=[W.electrons(vth, float(ppc))], background=True,
                          delta=0.01, case_id=1000 + k))
    return out


def serving_descs(case, mg_rtol, mg_cycles):
    from paper_1311_2286_amd import cpic as C
    from paper_1311_2286_amd import workloads as W
    m = C.make_map_desc(case.map_kind, case.dim, case.L, case.eps)
    g = C.make_grid_desc(case.n, shape=C.SHAPE_B2, precision=C.FP32, dt=case.dt, background=True,
                         background_n0=1.0, mg_rtol=mg_rtol, mg_max_cycles=mg_cycles, sort_every=4)
    sp = [C.make_species_desc(s.q, s.m, case.weight(s)) for s in case.species]
    parts = [W.generate_species(case, sid, dtype=np.float32, workers=16)
             for sid in range(len(case.species))]
    return m, g, sp, parts


def run_serving(nreq, nsteps, budget, slots, load, mg_rtol, mg_cycles, seed=1311):
    """Poisson arrivals at rate load / tau (tau: mean service time of a case
    alone, measured first on a sample of the requests); every request is
    submitted when its arrival time has passed, and the server is pumped one
    iteration at a time.  Returns the served throughput and latencies."""
    from paper_1311_2286_amd import cpic as C
    reqs = serving_requests(nreq, seed)
    t0 = time.time()
    prepared = [serving_descs(c, mg_rtol, mg_cycles) for c in reqs]
    log("serving: generated %d requests (%d particles) in %.1f s"
        % (nreq, sum(p[3][0]["cell"].size for p in prepared), time.time() - t0))
    # tau: each of a sample of requests alone
    sample = list(range(0, nreq, max(1, nreq // 4)))[:4]
    taus = []
    for k in sample:
        srv = C.Server(budget, 1)
        t = srv.submit(*prepared[k], nsteps)
        while not srv.pump(16):
            pass
        taus.append(srv.poll(t)["service_ms"] / 1e3)
        srv.close()
    tau = float(np.mean(taus))
    rate = load / tau
    rng = np.random.default_rng(seed + 1)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=nreq))
    srv = C.Server(budget, slots)
    tickets = []
    t_start = time.perf_counter()
    k = 0
    while True:
        now = time.perf_counter() - t_start
        while k < nreq and arrivals[k] <= now:
            tickets.append(srv.submit(*prepared[k], nsteps))
            k += 1
        idle = srv.pump(1)
        if idle and k == nreq:
            break
        if idle:
            time.sleep(max(0.0, min(0.01, arrivals[k] - (time.perf_counter() - t_start))))
    wall = time.perf_counter() - t_start
    res = [srv.poll(t) for t in tickets]
    st = srv.stats()
    srv.close()
    lat = [r["queue_ms"] + r["service_ms"] for r in res]
    ok = sum(1 for r in res if r["status"] == 0)
    return {"requests": nreq, "completed": ok, "steps_per_request": nsteps, "load": load,
            "tau_s": tau, "arrival_rate_per_s": rate, "wall_s": wall,
            "pushes": st["pushes"], "pushes_per_s": st["pushes"] / wall,
            "step_p50_ms": st["step_p50_ms"], "step_p99_ms": st["step_p99_ms"],
            "request_latency_p50_s": float(np.percentile(lat, 50)) / 1e3,
            "request_latency_p99_s": float(np.percentile(lat, 99)) / 1e3,
            "peak_active": st["peak_active"], "peak_bytes": st["peak_bytes"],
            "batched_case_steps": st["batched_steps"],
            "budget_bytes": budget, "slots": slots}


def extra_workload(name, shape_name, precision, steps, warmup, sort_every, mg_rtol, mg_cycles, mover=0,
                   tabulated=False, pusher=0):
    """Throughput of another workload (same fields as the headline path);
    tabulated: on its map sampled at the vertices (a tabulated map)."""
    from paper_1311_2286_amd import cpic as C
    from paper_1311_2286_amd import workloads as W
    import dataclasses
    import torch
    case = workload(name)
    if tabulated:
        case = dataclasses.replace(case, tabulated=True)
    shape = C.SHAPE_B2 if shape_name == "b2" else C.SHAPE_B1
    t0 = time.time()
    parts = [W.generate_species(case, sid, dtype=np.float64 if precision == C.FP64 else np.float32,
                                workers=16) for sid in range(len(case.species))]
    log("%s: generated %d particles in %.1f s" % (name, sum(p["cell"].size for p in parts),
                                                  time.time() - t0))
    r = run_path(case, parts, precision, shape, steps, warmup, sort_every, mg_rtol, mg_cycles, mover=mover,
                 pusher=pusher)
    del parts
    torch.cuda.empty_cache()
    out = {"workload": "%s%s, %s deposit, %s%s" % (name, ", tabulated map" if tabulated else "", shape_name.upper(),
                                                  "FP64" if precision else "FP32",
                                                  (", predictor-corrector mover" if mover else "")
                                                  + (", cyclotronic step" if pusher else "")),
           "particles": r["pushes"], "steps": steps, "pushes_per_s": r["pushes_per_s"],
           "ms_per_step": r["ms_per_step"], "p50_step_ms": r["p50_step_ms"], "p99_step_ms": r["p99_step_ms"],
           "particle_kernel_pushes_per_s": r["kernel_pushes_per_s"], "achieved_GBs": r["achieved_GBs"],
           "frac": r["achieved_GBs"] / HBM_PEAK_GBS, "bytes_per_launch": r["bytes_per_launch"],
           "launch_ms": r["launch_ms"], "phase_ms": {"particles": r["push_ms"], "field": r["solve_ms"],
                                                     "sort": r["sort_ms"]},
           "mg_cycles_last": r["mg_cycles_last"], "mg_relres_last": r["mg_relres_last"]}
    log(name, json.dumps(out))
    return out


def mover_timing(steps=200, dts=(0.001, 0.002, 0.004, 0.01, 0.025, 0.05)):
    """The paper's mover-timing test (Sec. "Particle mover", Tables t2 and t3):
    unit square, sinusoidal map with eps = 0 and 0.1, 64^2 cells, 100 electrons
    per cell (v_th = 1), fixed fields, periodic boundaries.  Times the particle
    stage (gather, push, position update, boundaries, deposit) per particle and
    step for both position updates, the tile sort (every step) beside it;
    normalised like the tables, to the Newton mover at eps = 0, dt = 0.001."""
    from paper_1311_2286_amd import cpic as C
    from paper_1311_2286_amd import workloads as W
    import torch
    rows = []
    for mover in (C.MOVER_NEWTON, C.MOVER_PC):
        for eps in (0.0, 0.1):
            case = W.Case("mover64", 2, W.SINUSOIDAL, (64, 64), L=(1.0, 1.0), eps=eps,
                          species=[W.electrons(1.0, 100.0)], case_id=170)
            p = W.generate_species(case, 0, dtype=np.float32)
            for dt in dts:
                sim = C.Sim(W.SINUSOIDAL, 2, (64, 64), L=(1.0, 1.0), eps=eps, dt=dt, precision=C.FP32,
                            mover=mover)
                try:
                    sim.add_species(-1.0, 1.0, 1.0 / p["cell"].size, p["cell"].size)
                    sim.set_particles(0, p["cell"], p["off"], p["vel"])
                    nv = sim.field_bytes(C.FIELD_EV) // 8
                    sim.set_field(C.FIELD_EV, W.synthetic_ev(case, nv, scale=0.5)[:, :2].copy())
                    st = torch.cuda.current_stream()
                    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
                    push_ms = sort_ms = 0.0
                    for k in range(steps + 5):
                        ev[0].record(st)
                        sim.stage(C.STAGE_PUSH)
                        ev[1].record(st)
                        sim.stage(C.STAGE_SORT)
                        ev[2].record(st)
                        st.synchronize()
                        if k >= 5:
                            push_ms += ev[0].elapsed_time(ev[1])
                            sort_ms += ev[1].elapsed_time(ev[2])
                    d = sim.diag()
                    rows.append({"mover": "newton" if mover == C.MOVER_NEWTON else "predictor-corrector",
                                 "eps": eps, "dt": dt,
                                 "ns_per_particle_step": 1e6 * push_ms / steps / p["cell"].size,
                                 "sort_ns_per_particle_step": 1e6 * sort_ms / steps / p["cell"].size,
                                 "newton_fallback": int(d.newton_fallback),
                                 "far_deposits": int(d.far_deposits)})
                finally:
                    sim.close()
            del p
    ref = rows[0]["ns_per_particle_step"]
    for r in rows:
        r["normalised"] = r["ns_per_particle_step"] / ref
    ratio = {}
    for mv in ("newton", "predictor-corrector"):
        t = {(r["eps"], r["dt"]): r["ns_per_particle_step"] for r in rows if r["mover"] == mv}
        ratio[mv] = {str(dt): t[(0.1, dt)] / t[(0.0, dt)] for dt in dts}
    out = {"workload": "mover timing: unit square, sinusoidal map eps 0 / 0.1, 64^2 cells, 100 e/cell "
                       "(409,600), v_th 1, fixed fields, periodic, %d steps per point, FP32" % steps,
           "rows": rows, "eps_0.1_over_eps_0": ratio}
    log("mover", json.dumps(ratio))
    return out


def field_solve_anisotropic(N=2048, stretches=(10.0, 40.0), rtol=1e-10):
    """The field solve on strongly anisotropic grids: identity map, N^2 cells,
    box 1 x Ly (face-coefficient ratio Ly^2), Dirichlet walls, a smooth right
    side, zero initial guess; the preconditioner relaxes along lines there."""
    from paper_1311_2286_amd import cpic as C
    import torch
    xi = (np.arange(N) + 0.5) / N
    u, v = np.meshgrid(xi, xi, indexing="xy")
    charge = (np.sin(3 * np.pi * u) * np.sin(5 * np.pi * v)).ravel() / N ** 2
    rows = []
    for Ly, method in [(ly, m) for m in (0, C.MG_BOXMG) for ly in stretches]:
        cap, times = 400, []
        for attempt in range(2):
            sim = C.Sim(C.MAP_IDENTITY, 2, (N, N), L=(1.0, Ly), bc_lo=(1, 1), bc_hi=(1, 1), precision=C.FP64,
                        mg_rtol=rtol, mg_max_cycles=cap, mg_method=method)
            try:
                sim.set_field(C.FIELD_CHARGE, charge)
                for r in range(3 if attempt else 1):
                    sim.set_field(C.FIELD_PHI, np.zeros(N * N))
                    sim.sync()
                    t0 = time.perf_counter()
                    sim.stage(C.STAGE_SOLVE)
                    sim.sync()
                    times.append(time.perf_counter() - t0)
                d = sim.diag()
            finally:
                sim.close()
            cap = d.mg_cycles + 1
        rows.append({"grid": "%d^2" % N, "box": [1.0, Ly], "coefficient_ratio": Ly * Ly,
                     "method": "boxmg" if method else "fcg", "cycles": d.mg_cycles,
                     "relres": d.mg_relres, "solve_ms": 1e3 * float(np.median(times[1:]))})
        log("aniso", json.dumps(rows[-1]))
    torch.cuda.empty_cache()
    return {"workload": "field solve on stretched grids (identity map, Dirichlet walls), rtol %g" % rtol,
            "grids": rows}


def field_solve_mms(sizes=(1024, 2048, 4096), rtol=1e-10, reps=3, method=0):
    """The field solve alone on the paper's manufactured-solution test (spherical
    r-z map, Omega = r, Eq. mms; Table t1's grids and tolerance): cycles, time
    per solve from a zero initial guess and the RMS error against Eq. mms.
    Each grid is solved once to learn its cycle count, then timed with one
    cycle of slack, as the time step launches its solves."""
    from paper_1311_2286_amd import cpic as C
    from paper_1311_2286_amd import workloads as W
    import torch
    out = []
    for N in sizes:
        charge, exact = W.spherical_mms_input(N)
        zeros = np.zeros(N * N)
        row = {"grid": "%d^2" % N}
        cap = 60
        for attempt in range(2):
            sim = C.Sim(W.SPHERICAL_RZ, 2, (N, N), r_in=W.MMS_R1, r_out=W.MMS_R2, omega=1,
                        bc_lo=(C.BC_DIRICHLET, C.BC_NEUMANN), bc_hi=(C.BC_DIRICHLET, C.BC_NEUMANN),
                        precision=C.FP64, mg_rtol=rtol, mg_max_cycles=cap, mg_method=method)
            try:
                sim.set_field(C.FIELD_CHARGE, charge)
                times = []
                for r in range(reps if attempt else 1):
                    sim.set_field(C.FIELD_PHI, zeros)
                    sim.sync()
                    t0 = time.perf_counter()
                    sim.stage(C.STAGE_SOLVE)
                    sim.sync()
                    times.append(time.perf_counter() - t0)
                d = sim.diag()
                phi = sim.get_field(C.FIELD_PHI)
            finally:
                sim.close()
            if attempt == 0:
                cap = d.mg_cycles + 1
                continue
            row.update({"cycles": d.mg_cycles, "relres": d.mg_relres, "launched_cycles": cap,
                        "solve_ms": 1e3 * float(np.median(times)),
                        "l2_error": float(np.sqrt(np.mean((phi - exact) ** 2)))})
        del charge, exact, zeros
        torch.cuda.empty_cache()
        log("mms", json.dumps(row))
        out.append(row)
    how = ("one FP32 V(2,2) cycle per iteration (point Chebyshev smoother, rediscretised coarse operators)"
           if method == 0 else "one FP32 V(1,2) cycle per iteration with variational coarse operators and zebra "
                               "line relaxation (CPIC_MG_BOXMG)")
    return {"workload": "field solve of the spherical r-z manufactured solution (Omega = r), FCG with "
                        "%s, rtol %g, from a zero initial guess" % (how, rtol),
            "grids": out}


def extra_table(C):
    """The other workloads: name -> (workload, shape, precision, steps, mover,
    tabulated map, pusher)."""
    return {
        "box3d_128_b1": ("box3d_128", "b1", C.FP32, 10, 0, False, 0),
        "box3d_128_b1_fp64": ("box3d_128", "b1", C.FP64, 10, 0, False, 0),
        "box3d_128_pc": ("box3d_128", "b2", C.FP32, 10, C.MOVER_PC, False, 0),
        "box3d_128_tabulated": ("box3d_128", "b2", C.FP32, 10, 0, True, 0),
        "box3d_128_tabulated_pc": ("box3d_128", "b2", C.FP32, 10, C.MOVER_PC, True, 0),
        "probe2d_512": ("probe2d_512", "b2", C.FP32, 200, 0, False, 0),
        "box3d_magnetized": ("box3d_magnetized", "b2", C.FP32, 10, 0, False, 0),
        "box3d_magnetized_cyclotronic": ("box3d_magnetized", "b2", C.FP32, 10, 0, False, C.PUSH_CYCLOTRONIC)}


def run_extra(C, key, args, steps=None):
    if key in ("field_solve_mms", "field_solve_mms_boxmg"):
        sizes = tuple(int(v) for v in args.mms_sizes.split(","))
        return field_solve_mms(sizes=sizes, method=C.MG_BOXMG if key.endswith("boxmg") else 0)
    if key == "field_solve_anisotropic":
        return field_solve_anisotropic()
    if key == "mover_timing":
        return mover_timing()
    name, shp, prec, n, mover, tab, push = extra_table(C)[key]
    # the probe is timed in its injected steady state: the last 200 of the
    # configuration's 2,000 steps
    warm = 1800 if name == "probe2d_512" else 2
    return extra_workload(name, shp, prec, steps or n, warm, args.sort_every, args.mg_rtol, args.mg_cycles,
                          mover, tab, push)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="box3d_128")
    ap.add_argument("--shape", default="b2", choices=["b2", "b1"])
    ap.add_argument("--sort-every", type=int, default=4)
    # relative residual 4e-6: far below the particle noise of the charge density
    # (about 1/sqrt(32) per cell here) and small enough that phi and E stay within
    # 1e-5 of the FP64 oracle (with 1e-5, E reached 1.35e-5 on the 2D Langmuir
    # case); the cap is not reached in practice
    ap.add_argument("--mg-rtol", type=float, default=4e-6)
    ap.add_argument("--mg-cycles", type=int, default=10)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    # about 10-20 s of oracle work on the box's 16 host threads
    ap.add_argument("--cpu-sample", type=int, default=24 << 20)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (B1 deposit, probe, magnetised box)")
    ap.add_argument("--only-extra", default=None,
                    help="only run this one of the other workloads (e.g. box3d_128_tabulated) and print its "
                         "result")
    ap.add_argument("--mms-sizes", default="1024,2048,4096",
                    help="grids of --only-extra field_solve_mms / field_solve_mms_boxmg")
    ap.add_argument("--copy-calibrate", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--serve", action="store_true",
                    help="only run the serving stream (64 requests, 500 steps each)")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-steps", type=int, default=500)
    ap.add_argument("--serve-load", type=float, default=8.0,
                    help="arrival rate in units of 1 / (mean service time alone)")
    ap.add_argument("--serve-budget-gib", type=float, default=1.0,
                    help="HBM budget of the serving stream's cases")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; "
              "rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibrate:
        copy_calibrate(1 << 30, 5)
        return
    if args.only_extra:
        from paper_1311_2286_amd import cpic as C
        C.load()
        print(json.dumps({"workload": args.only_extra,
                          "result": run_extra(C, args.only_extra, args, args.steps)}), flush=True)
        return
    if args.serve:
        from paper_1311_2286_amd import cpic as C
        C.load()
        budget = int(args.serve_budget_gib * (1 << 30))
        sv = run_serving(args.serve_requests, args.serve_steps, budget, 32, args.serve_load,
                         args.mg_rtol, args.mg_cycles)
        print(json.dumps({"metric": "served particle pushes/s; p50/p99 step ms", "value": sv["pushes_per_s"],
                          "unit": "particle pushes/s", "n_gpus": 1, "higher_is_better": True,
                          "dtype": "f32", "data": "synthetic",
                          "config": {"workload": "serving stream: %d requests, 2D periodic sinusoidal "
                                                 "maps, grids 32^2..256^2, %d steps each, HBM budget "
                                                 "%g GiB, 32 slots" % (args.serve_requests,
                                                                       args.serve_steps,
                                                                       args.serve_budget_gib)},
                          "serving": sv}), flush=True)
        return
    from paper_1311_2286_amd import cpic as C
    from paper_1311_2286_amd import workloads as W
    C.load()
    case = workload(args.workload)
    shape = C.SHAPE_B2 if args.shape == "b2" else C.SHAPE_B1
    t0 = time.time()
    parts = [W.generate_species(case, sid, dtype=np.float64 if not args.no_fp64 else np.float32,
                                workers=16) for sid in range(len(case.species))]
    log("generated %d particles in %.1f s" % (sum(p["cell"].size for p in parts), time.time() - t0))
    r32 = run_path(case, parts, C.FP32, shape, args.steps, args.warmup, args.sort_every,
                   args.mg_rtol, args.mg_cycles)
    log("fp32", json.dumps(r32))
    r64 = None
    if not args.no_fp64:
        r64 = run_path(case, parts, C.FP64, shape, args.steps, args.warmup, args.sort_every,
                       args.mg_rtol, args.mg_cycles)
        log("fp64", json.dumps(r64))
    del parts
    cpu = None
    errors = None
    if not args.no_cpu:
        cpu = cpu_baseline(case, args.cpu_sample, shape)
        log("cpu", json.dumps(cpu))
        try:
            cpu["other_configs"] = cpu_configs(shape)
        except Exception as e:  # reported, never fatal for the headline line
            cpu["other_configs"] = {"error": repr(e)}
        log("cpu configs", json.dumps(cpu["other_configs"]))
        try:
            errors = error_vs_oracle(shape, args.sort_every, args.mg_rtol, args.mg_cycles)
        except Exception as e:
            errors = {"error": repr(e)}
        log("errors", json.dumps(errors))
    extra = {}
    if not args.no_extra:
        for key in extra_table(C):
            try:
                extra[key] = run_extra(C, key, args)
            except Exception as e:  # reported, never fatal for the headline line
                extra[key] = {"error": repr(e)}
        try:
            extra["field_solve_mms"] = field_solve_mms()
        except Exception as e:
            extra["field_solve_mms"] = {"error": repr(e)}
        try:
            extra["field_solve_mms_boxmg"] = field_solve_mms(method=C.MG_BOXMG)
        except Exception as e:
            extra["field_solve_mms_boxmg"] = {"error": repr(e)}
        try:
            extra["field_solve_anisotropic"] = field_solve_anisotropic()
        except Exception as e:
            extra["field_solve_anisotropic"] = {"error": repr(e)}
        try:
            extra["mover_timing"] = mover_timing()
        except Exception as e:
            extra["mover_timing"] = {"error": repr(e)}
        # the serving stream, shortened: 32 requests of 200 steps under a 4 GiB budget
        try:
            sv = run_serving(32, 200, 4 << 30, 32, 8.0, args.mg_rtol, args.mg_cycles)
            sv["workload"] = ("serving stream: 32 requests, 2D periodic sinusoidal maps, grids 32^2..256^2, "
                              "200 steps each, Poisson arrivals at 8 / (mean service time alone), HBM budget "
                              "4 GiB, 32 slots; same-shape cases batched")
            extra["serving"] = sv
        except Exception as e:
            extra["serving"] = {"error": repr(e)}
    n_p = r32["pushes"]
    out = {
        "metric": METRIC,
        "value": r32["pushes_per_s"],
        "unit": "particle pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %dD periodic sinusoidal map eps=%g, %s cells, %s, %d particles, "
                               "%s deposit, FP32 particles + int64 fixed-point deposit, dt=%g"
                               % (case.name, case.dim, case.eps, "x".join(map(str, case.n)),
                                  " + ".join("%g %s/cell" % (s.ppc, s.name) for s in case.species),
                                  n_p, args.shape.upper(), case.dt),
                   "sort_every": args.sort_every, "mg_rtol": args.mg_rtol,
                   "mg_max_cycles": args.mg_cycles},
        "p50_step_ms": r32["p50_step_ms"],
        "p99_step_ms": r32["p99_step_ms"],
        "particle_kernel_pushes_per_s": r32["kernel_pushes_per_s"],
        "phase_ms": {"particles": r32["push_ms"], "field": r32["solve_ms"], "sort": r32["sort_ms"]},
        "roofline": {"bound": "hbm", "achieved": r32["achieved_GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": r32["achieved_GBs"] / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload, args.shape, "fp32"),
                     "kernel": "particle_kernel (one launch per species)",
                     "bytes_per_launch": r32["bytes_per_launch"],
                     "launch_ms": r32["launch_ms"]},
        "cpu_baseline": cpu,
        "error_vs_oracle": errors,
        # the particles' one upload from host arrays (pageable numpy), not in
        # the timed steps: its rate and the pushes/s of the timed steps with it
        "host_upload": {"bytes": r32["upload_bytes"], "s": r32["upload_s"],
                        "GB_per_s": r32["upload_bytes"] / max(r32["upload_s"], 1e-12) / 1e9,
                        "pushes_per_s_with_upload": r32["pushes"] * args.steps / (r32["wall_s"] + r32["upload_s"])},
    }
    if r64 is not None:
        out["fp64_path"] = {"value": r64["pushes_per_s"], "unit": "particle pushes/s",
                            "ms_per_step": r64["ms_per_step"], "p50_step_ms": r64["p50_step_ms"],
                            "p99_step_ms": r64["p99_step_ms"],
                            "particle_kernel_pushes_per_s": r64["kernel_pushes_per_s"],
                            "achieved_GBs": r64["achieved_GBs"],
                            "frac": r64["achieved_GBs"] / HBM_PEAK_GBS,
                            "bytes_per_launch": r64["bytes_per_launch"],
                            "bytes_per_particle": r64["bytes_per_particle"],
                            "layout_bytes_per_particle": layout_bytes_per_particle(case.dim, 1, any(case.B)),
                            "launch_ms": r64["launch_ms"],
                            "phase_ms": {"particles": r64["push_ms"], "field": r64["solve_ms"],
                                         "sort": r64["sort_ms"]}}
    out["diagnostics"] = {k: r32[k] for k in ("mg_cycles_last", "mg_relres_last", "newton_fallback",
                                              "newton_failed", "far_deposits")}
    if extra:
        out["other_workloads"] = extra
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
