/*
 * cpic.h -- C ABI of the MI355X curvilinear particle-in-cell hot path.
 *
 * What is computed (Delzanno et al., "CPIC: a Curvilinear Particle-In-Cell
 * code for plasma-material interaction studies", arXiv:1311.2286):
 *   - a map x(xi) from the logical unit cube to physical space and its metric
 *     (Sec. II.A, Eqs. map, jcov, jcon, jac, gcon; the sinusoidal test map of
 *     Eq. map2; a polar-log annulus map; the identity / affine map);
 *   - particles with logical position xi (cell index + in-cell offset) and
 *     physical velocity v -- the hybrid mover of Sec. II.B;
 *   - one electrostatic PIC cycle in leap-frog order (Sec. II, four-step
 *     cycle): gather of the vertex field (Eqs. vvp, Wvp, b1), velocity push
 *     (Eqs. step1, step1a; Boris rotation when a uniform B0 is set), position
 *     update x(xi^n) + dt v^{n+1/2} mapped back to xi by Newton iterations on
 *     the map, particle boundaries (periodic, absorbing wall, outflow), charge
 *     deposit divided by the cell volume J_c dxi deta dzeta (Eqs. pg, Wpc,
 *     b2), and the Poisson solve of Eq. poiscurv by geometric multigrid, with
 *     the field E = -grad phi formed at vertices (Sec. II.B staggering).
 *
 * Units are the paper's normalised ones (Sec. II.B): lengths in Debye
 * lengths, velocities in electron thermal speeds, time in 1/omega_pe,
 * potential in T_e/e, epsilon_0 = 1, reference density n0 = 1.
 *
 * Conventions used by every call
 *   - cell index (input and output): c = i + n0 * (j + n1 * k), 0 <= i < n0 ...
 *   - offsets: in-cell logical offset per axis in [0, 1), structure of arrays
 *     off[a * n + p] for axis a < dim;
 *   - velocities: physical, three components always, vel[a * n + p];
 *   - floating point type of off/vel/fields: float for CPIC_FP32, double for
 *     CPIC_FP64 (cpic_grid_desc.precision);
 *   - vertex field: physical components, vertex v = i + nv0 * (j + nv1 * k)
 *     with nv_a = n_a on periodic axes and n_a + 1 on bounded axes, interleaved
 *     with a component stride of 2 (2D) or 4 (3D; the 4th slot is padding);
 *   - all launches are asynchronous on the stream given at creation; calls
 *     that return data to the host synchronise that stream.
 *
 * Ownership: the library copies what it is given (set_* calls) and never frees
 * caller memory.  Library memory comes from the caller's allocator (or
 * hipMalloc when none is given) and is returned by cpic_destroy.
 *
 * Errors: every call returns a cpic_status; arguments are validated before any
 * launch, so a failed call leaves the simulation unchanged.  An asynchronous
 * device fault surfaces as CPIC_E_HIP at the next synchronising call and
 * poisons the simulation.  cpic_last_error() returns a description of the last
 * failure on that simulation.  A simulation is used from one host thread at a
 * time.
 */
#ifndef CPIC_H_
#define CPIC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cpic_sim cpic_sim;

typedef enum {
  CPIC_OK = 0,
  CPIC_E_ARG = -1,         /* invalid argument / descriptor */
  CPIC_E_MAP = -2,         /* map not invertible on the domain (J <= 0) */
  CPIC_E_NOMEM = -3,       /* allocation failed */
  CPIC_E_BUDGET = -4,      /* capacity exceeded */
  CPIC_E_HIP = -5,         /* HIP runtime error */
  CPIC_E_OVERFLOW = -6,    /* fixed-point deposit headroom exceeded */
  CPIC_E_NONFINITE = -7,   /* non-finite value found in a field */
  CPIC_E_STATE = -8,       /* call out of order */
  CPIC_E_UNSUPPORTED = -9, /* valid but not implemented combination */
  CPIC_E_PENDING = 1       /* serving: the work is not finished yet (not an error) */
} cpic_status;

/* map kinds.  CPIC_MAP_SPHERICAL_RZ (2D): the meridian half plane of a
   spherical shell in cylindrical coordinates, r = rho sin(pi (1 - eta)),
   z = rho cos(pi (1 - eta)), rho = r_in + (r_out - r_in) xi (Sec. "Field
   solver", Eqs. r and z); with cpic_map_desc.omega = 1 it is the paper's
   manufactured-solution test of the solver.  It serves the field solve only:
   cpic_add_species returns CPIC_E_UNSUPPORTED on it.
   CPIC_MAP_TABULATED (2D, 3D): a map known only at the cell vertices
   (cpic_map_desc.vertices), as a mesh generator gives it; the Jacobi matrix,
   J, g^ij and k come from finite differences of the vertex coordinates (Sec.
   "Curvilinear formulation"): centred over the two neighbours, second-order
   one-sided at the ends of a bounded axis, blended multilinearly between
   vertices.  For the position update the map between vertices is the
   multilinear interpolant of the vertex coordinates: CPIC_MOVER_NEWTON inverts
   it by Newton iterations on the position in cells (FP64, the polynomial of
   the cell holding the iterate, continued beyond a wall by the boundary
   cell's), CPIC_MOVER_PC uses the inverse-Jacobian table as on any map.
   Particles cannot be injected; with walls the map must be orthogonal, up to its
   sampling error, in every plane that holds a bounded axis (the columns of j
   within acos(0.05) of a right angle at every vertex, else
   CPIC_E_UNSUPPORTED); J <= 0 at a vertex or cell centre gives CPIC_E_MAP. */
enum {
  CPIC_MAP_IDENTITY = 0,
  CPIC_MAP_SINUSOIDAL = 1,
  CPIC_MAP_POLAR_LOG = 2,
  CPIC_MAP_SPHERICAL_RZ = 3,
  CPIC_MAP_TABULATED = 4
};
/* field boundary conditions per axis side (ghost cells, Sec. II.B).
   CPIC_BC_FLOATING (lower side of axis 0 only, every other axis periodic): a
   conducting wall whose potential floats so that Gauss' law holds -- the
   flux of E through it equals the charge of the particles it absorbed
   (Sec. "Tests", charging of a conducting planar wall). */
enum { CPIC_BC_PERIODIC = 0, CPIC_BC_DIRICHLET = 1, CPIC_BC_NEUMANN = 2, CPIC_BC_FLOATING = 3 };
/* particle boundary conditions per axis side */
enum { CPIC_PBC_PERIODIC = 0, CPIC_PBC_ABSORB = 1, CPIC_PBC_OUTFLOW = 2 };
/* deposit shape: order-2 B-spline of Eq. b2 (default) or CIC */
enum { CPIC_SHAPE_B2 = 2, CPIC_SHAPE_B1 = 1 };
/* particle precision: FP32 offsets/velocities with 64-bit fixed-point deposit,
   or plain FP64 throughout (FP64 deposit) */
enum { CPIC_FP32 = 0, CPIC_FP64 = 1 };
/* fields for get/set */
enum {
  CPIC_FIELD_Q = 0,      /* deposit of one species: uint64 (FP32 path) or double */
  CPIC_FIELD_CHARGE = 1, /* charge per cell, J rho dV (double) */
  CPIC_FIELD_PHI = 2,    /* potential at cell centres (double) */
  CPIC_FIELD_EV = 3,     /* vertex field (float or double, interleaved) */
  CPIC_FIELD_JC = 4,     /* physical Jacobian at cell centres (double) */
  CPIC_FIELD_RHO = 5,    /* charge density rho = charge / (J_c dV) (double) */
  CPIC_FIELD_BACKGROUND = 6 /* fixed background charge per cell (double) */
};
/* single stages of the step, for tests and timing */
enum {
  CPIC_STAGE_SORT = 0,     /* tile-sort (and compact) all species */
  CPIC_STAGE_DEPOSIT = 1,  /* Q_s <- deposit of the current positions */
  CPIC_STAGE_CHARGE = 2,   /* charge <- sum_s q_s w_s Q_s + background */
  CPIC_STAGE_SOLVE = 3,    /* phi <- multigrid solve from charge */
  CPIC_STAGE_EFIELD = 4,   /* E_v <- -k^T D phi at vertices */
  CPIC_STAGE_PUSH = 5,     /* gather + push + map inversion + boundaries + deposit */
  CPIC_STAGE_HALFSTEP = 6, /* v <- Boris(v, E, B, -dt/2): initial velocity push-back */
  CPIC_STAGE_INJECT = 7    /* this step's flux injection (appends, deposits into Q_s) */
};

/* Poisson solve method (cpic_grid_desc.mg_method) */
enum {
  CPIC_MG_FCG = 0,    /* flexible conjugate gradients, one V-cycle per iteration as the
                         preconditioner (default: converges on strongly distorted,
                         anisotropic grids where V-cycles alone can diverge) */
  CPIC_MG_VCYCLE = 1, /* plain V-cycles */
  CPIC_MG_BOXMG = 2   /* 2D: flexible conjugate gradients preconditioned by a V(1,2) cycle with
                         variational coarse operators (P^T A P, P the cell-centred bilinear
                         interpolation) and zebra line relaxation along both axes (Sec.
                         "Field solver": the robust solver for anisotropic, strongly
                         varying operators); grids of 4..4096 cells per axis, else
                         CPIC_E_UNSUPPORTED */
};

/* Position update of the mover (cpic_grid_desc.mover) */
enum {
  CPIC_MOVER_NEWTON = 0, /* x(xi^n) + dt v^{n+1/2} mapped back to logical space by Newton
                            on the analytic map (default) */
  CPIC_MOVER_PC = 1      /* the paper's predictor-corrector hybrid update (Sec. "Particle
                            mover", Eqs. step2-step4): xi' = xi^n + (dt/2) k(xi^n) v,
                            xi^{n+1} = xi^n + dt k(xi') v, with the inverse Jacobian k
                            tabulated at the vertices and carried to the particle by the
                            CIC vertex weights (Eq. step3) */
};

/* Velocity step (cpic_grid_desc.pusher) */
enum {
  CPIC_PUSH_BORIS = 0,       /* leap-frog with the Boris rotation (default) */
  CPIC_PUSH_CYCLOTRONIC = 1  /* with a uniform background B, the gyration resolved exactly (Sec. "Particle
                                mover"; Sec. "Tests" runs at omega_ce dt ~ 1): the electric impulse
                                (q/m) E dt, then the exact helix over dt -- the velocity rotated by
                                theta = (q/m)|B| dt about B, the position moved by dt times the mean
                                velocity of the gyration (then mapped back by the position update).
                                Stored velocities are those just before the next impulse; the start-up
                                in cpic_initialize is the half impulse alone; the kinetic energy is that
                                of v + (q/m) E dt / 2.  Needs CPIC_MOVER_NEWTON (else
                                CPIC_E_UNSUPPORTED); without B it is the leap-frog step. */
};

typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} cpic_allocator;

typedef struct {
  int kind;       /* CPIC_MAP_* */
  int dim;        /* 2 or 3 */
  double L[3];    /* box lengths (identity, sinusoidal); period shifts (tabulated) */
  double eps;     /* sinusoidal amplitude, relative to the box */
  double r_in;    /* polar-log inner radius */
  double r_out;   /* polar-log outer radius */
  /* geometric factor Omega of the Poisson operator, d_i(Omega J g^ij d_j phi)
     = -Omega J rho (Sec. "Field solver", Eq. poiscurv): 0 -> Omega = 1;
     1 -> Omega = x^1, the radius of an axisymmetric r-z plane (2D identity or
     spherical r-z map with a bounded axis 0, else CPIC_E_UNSUPPORTED).  With
     Omega = x^1, CPIC_FIELD_CHARGE is the right side Omega J rho dV of the
     solve, and the map serves the field solve only (no species). */
  int omega;
  /* CPIC_MAP_TABULATED: physical coordinates at the logical vertices, host
     memory owned by the caller and read during cpic_create only: d arrays of
     nv0 nv1 (nv2) doubles (x^1 at every vertex, then x^2, ...), vertex
     (i, j, k) at i + nv0 (j + nv1 k), nv_a = n_a on a periodic axis and
     n_a + 1 on a bounded one.  On a periodic axis a the map continues as
     x(xi + e_a) = x(xi) + L_a e_a (L_a >= 0; 0 for an axis that closes on
     itself, such as an angle).  Ignored by the other kinds. */
  const double* vertices;
} cpic_map_desc;

typedef struct {
  int n[3];             /* cells per axis (n[2] ignored in 2D) */
  int bc_lo[3], bc_hi[3];
  double phi_lo[3], phi_hi[3]; /* Dirichlet wall values */
  int shape;            /* CPIC_SHAPE_B2 / CPIC_SHAPE_B1 */
  int precision;        /* CPIC_FP32 / CPIC_FP64 */
  double dt;
  double B0[3];         /* uniform background magnetic field */
  int background;       /* 1: fixed neutralising background of density n0 */
  double background_n0; /* its density (charge +n0 per unit volume) */
  double mg_rtol;       /* relative residual target of the Poisson solve */
  int mg_max_cycles;    /* V-cycles per solve (upper bound; one per FCG iteration) */
  int sort_every;       /* tile sort of a species at most every this many steps (>= 1): then,
                           unless (steps since its last sort) x (largest particle increment seen,
                           in cells) is below one cell -- slow species are sorted less often,
                           at least every 16 sort_every steps; injecting species every step */
  int track_ids;        /* carry a uint32 particle id through sorts */
  int mg_method;        /* CPIC_MG_FCG (0), CPIC_MG_VCYCLE or CPIC_MG_BOXMG */
  int mover;            /* CPIC_MOVER_NEWTON (0) or CPIC_MOVER_PC */
  int pusher;           /* CPIC_PUSH_BORIS (0) or CPIC_PUSH_CYCLOTRONIC */
} cpic_grid_desc;

typedef struct {
  double q, m, w;       /* charge, mass, macro-weight */
  int pbc_lo[3], pbc_hi[3];
  size_t capacity;      /* maximum particle count */
  /* Maxwellian flux injection through the upper face of axis 0 (the outer
     wall; Sec. "Tests": plasma injected from the boundary opposite the
     object): inject != 0 enables it, with density inject_n0, thermal speed
     inject_vth and a drift of speed inject_drift (>= 0) along the inward
     normal (the planar-wall test's ions; 0: at rest); the random stream is
     Philox4x32-10 keyed by seed.  Needs a bounded axis 0 and an orthogonal
     map (identity or polar-log). */
  int inject;
  double inject_n0, inject_vth;
  uint64_t seed;
  double inject_drift;
} cpic_species_desc;

typedef struct {
  long long step;
  double kinetic;        /* 1/2 sum m w v^{n-1/2} . v^{n+1/2} of the last push */
  double field_energy;   /* 1/2 sum_c charge_c phi_c */
  double mg_relres;      /* final relative residual of the last solve */
  int mg_cycles;         /* V-cycles used by the last solve */
  int nspecies;
  long long count[8];    /* live particles per species */
  long long absorbed[8]; /* cumulative absorbed at lower walls */
  long long outflow[8];  /* cumulative lost through upper walls */
  uint64_t qsum_lo[8];   /* sum_c Q_s (exact, 128-bit: lo, hi words) */
  uint64_t qsum_hi[8];
  long long newton_fallback; /* cumulative FP64 fallbacks in FP32 Newton */
  long long far_deposits;    /* cumulative deposits outside the tile window */
  long long newton_failed;   /* cumulative position updates that missed the tolerance */
  long long injected[8];     /* cumulative injected particles per species */
  int step_graphs;           /* step variants recorded as HIP graphs (graph mode) */
  long long sorts[8];        /* tile sorts per species so far (a species whose particles
                                drift less than a cell between sorts is sorted less often) */
  double phi_wall;           /* potential of a floating wall (CPIC_BC_FLOATING), else 0 */
  double wall_charge;        /* charge it holds: sum of q w over the particles it absorbed */
  long long inject_lost[8];  /* cumulative injected particles whose entry flight (a random fraction of
                                the step from the face) left the domain at once: never live, not in
                                injected[] */
  long long batched_steps;   /* steps whose field phase ran batched with other simulations
                                (cpic_step_batch) */
} cpic_diag;

/* Create a simulation on the current HIP device.  hip_stream may be NULL
   (default stream).  alloc may be NULL (hipMalloc / hipFree).  Rejects maps
   whose Jacobian is not positive on the domain (CPIC_E_MAP) and walls on
   non-orthogonal maps (CPIC_E_UNSUPPORTED). */
cpic_status cpic_create(const cpic_map_desc* map, const cpic_grid_desc* grid,
                        const cpic_allocator* alloc, void* hip_stream, cpic_sim** out);

/* Add a species (charge q, mass m, macro-weight w; Eq. f); returns its id. */
cpic_status cpic_add_species(cpic_sim* sim, const cpic_species_desc* desc, int* species_id);

/* Copy n particles in (host pointers, or device pointers when on_device != 0).
   cell: int32 [n]; off: [dim][n]; vel: [3][n] (float for CPIC_FP32, double for
   CPIC_FP64); ids: uint32 [n] or NULL (ids 0..n-1).  n <= capacity (else
   CPIC_E_BUDGET).  Host input is validated first: cells out of range or
   offsets outside [0, 1) give CPIC_E_ARG; on the FP32 path, 2^16 or more
   particles within one 3^d block of cells give CPIC_E_OVERFLOW, as their
   fixed-point deposit (at most 2^{d S1} = 2^48 per particle and cell) could
   pass 64 bits in the block's centre cell.  Both leave the simulation
   unchanged.  Device input is range-checked on the device (CPIC_E_ARG); a
   deposit that wraps later is reported by cpic_get_diag / cpic_sync. */
cpic_status cpic_set_particles(cpic_sim* sim, int species_id, size_t n, const int32_t* cell,
                               const void* off, const void* vel, const uint32_t* ids,
                               int on_device);

/* Copy particles out (synchronises).  Arrays as in cpic_set_particles with
   room for cap particles; *n receives the number of slots in use: the live
   particles and, until their species' next tile sort, those that left since
   the last one, with cell -1 (absorbed) or -2 (left through an upper wall).
   Order is the library's (tile-sorted, particles injected since the last sort
   after the others); ids identify particles when track_ids is set. */
cpic_status cpic_get_particles(cpic_sim* sim, int species_id, size_t cap, int32_t* cell,
                               void* off, void* vel, uint32_t* ids, size_t* n, int on_device);

/* Initial state: sort, deposit, solve, field, and the half-step velocity
   push-back v^{-1/2} = Boris(v^0, E^0, B, -dt/2). */
cpic_status cpic_initialize(cpic_sim* sim);

/* Advance nsteps full PIC cycles (asynchronous). */
cpic_status cpic_step(cpic_sim* sim, int nsteps);

/* Advance each of n simulations by one PIC cycle (asynchronous), with their
   phases batched (the throughput path of a server running many small
   cases).  Each result is bit for bit what cpic_step(sims[i], 1) gives.  The
   particle phase runs as one launch over the work items of every case and
   species whose particle kernel is the same (precision, dimension, map kind,
   deposit shape, mover, pusher; else case by case), with the deposit clears
   of all cases in one launch; the field phase (charge, the flexible-CG
   solve of Sec. "Field solve" with its V-cycle preconditioner, the vertex
   field) runs as one launch per kernel over all cases when every case has
   FP32 particles, the flexible-CG method, no floating wall, no injection, a
   stream shared with the others, and the same grid dimensions, boundary
   types and restriction; a small grid's field phase is launch-bound, and the
   batch pays those launches once.  Otherwise the cases are stepped one after
   the other.  The solve of each case stops at its own convergence and cycle
   budget.  With graph mode on for the first case stepped (cpic_set_graphs)
   and a stream that can be captured, each batched sequence is captured once
   as a HIP graph and replayed with one launch per step.  Each simulation may appear once; n >= 1.  status (NULL, or n
   entries) receives each case's outcome: a case that cpic_step would refuse
   (CPIC_E_STATE, CPIC_E_OVERFLOW) is left out and keeps its state while the
   others step; a runtime error during the batched launches (CPIC_E_HIP) is
   reported for every case of the batch.  The batch's argument buffers (a few
   hundred bytes per kernel and case) come from the allocator of the first
   case stepped and are freed by its cpic_destroy; when they cannot be
   allocated the phases run case by case.  Returns CPIC_OK, else the first
   failing case's status. */
cpic_status cpic_step_batch(cpic_sim* const* sims, int n, cpic_status* status);

/* *sig receives 0 when cpic_step_batch cannot batch the simulation's field
   phase (see there), else a value that two simulations share when their
   field phases can be batched together (on a shared stream).  Valid once the
   species are added. */
cpic_status cpic_batch_signature(const cpic_sim* sim, uint64_t* sig);

/* Move the simulation to another stream (NULL: the default stream): waits for
   the work queued on the current one (synchronises), and everything after
   runs on the new one. */
cpic_status cpic_set_stream(cpic_sim* sim, void* hip_stream);

/* *ready = 1 when the next cpic_step (or cpic_step_batch) of the simulation
   would not wait for the device: a step decides its solver cycles and sorts
   from the record of the step two before, which it waits for; 0 while that
   step is still running.  Lets a caller driving many simulations step the
   ones that are ready first. */
cpic_status cpic_step_ready(const cpic_sim* sim, int* ready);

/* Run one stage (asynchronous); see CPIC_STAGE_*. */
cpic_status cpic_run_stage(cpic_sim* sim, int stage);

/* Field copies (synchronise).  species_id is used by CPIC_FIELD_Q only.
   bytes must equal the field's size.  cpic_set_field rejects host input that
   holds a NaN or an infinity (CPIC_E_NONFINITE) before copying anything. */
cpic_status cpic_get_field(cpic_sim* sim, int which, int species_id, void* dst, size_t bytes,
                           int on_device);
cpic_status cpic_set_field(cpic_sim* sim, int which, int species_id, const void* src,
                           size_t bytes, int on_device);

/* Size in bytes of a field (for get/set). */
size_t cpic_field_bytes(const cpic_sim* sim, int which);

/* Diagnostics (synchronises).  Also checks the state: returns
   CPIC_E_NONFINITE (diagnostics filled) when the potential, the charge or the
   vertex field holds a NaN or an infinity, and CPIC_E_OVERFLOW (diagnostics
   filled) when a species' fixed-point deposit wrapped -- its exact total
   sum_c Q_s differs from (particles deposited) x 2^{d S1}, which every
   particle adds exactly; after that cpic_step returns CPIC_E_OVERFLOW until
   cpic_set_particles loads new particles.  Neither changes the simulation. */
cpic_status cpic_get_diag(cpic_sim* sim, cpic_diag* out);

/* cpic_get_diag for callers that cannot allocate device memory (code under
   HIP graph capture, tight serving loops, harnesses that forbid allocation):
   the same diagnostics and checks, bit for bit, computed in a fixed scratch
   array of 35,200 bytes that the library keeps per device for the life of the
   process (field-energy partial sums, the non-finite count, and the 128-bit
   charge sums of up to CPIC_MAX_SPECIES species; a simulation with more
   species gets CPIC_E_BUDGET).  Allocates nothing, on the device or the host,
   on success.  Every call on one device shares that array: calls that overlap
   on one device (several host threads, or streams whose calls are in flight
   together) race and must be serialised by the caller.  CPIC_E_HIP when the
   array's address cannot be found on the simulation's device. */
cpic_status cpic_get_diag_noalloc(cpic_sim* sim, cpic_diag* out);

/* Wait for all work on the simulation's stream, then run the checks of
   cpic_get_diag (CPIC_E_NONFINITE, CPIC_E_OVERFLOW). */
cpic_status cpic_sync(cpic_sim* sim);

/* Per-step durations (ms) of every step since timing was last enabled by
   cpic_set_timing(sim, 1) (which clears the record), measured with HIP events
   on the simulation's stream: particle kernels, field phase (charge, solve,
   vertex field), tile sort, whole step.  Writes at most cap samples per array
   (any array may be NULL); *samples receives the number of steps recorded.
   Synchronises. */
cpic_status cpic_set_timing(cpic_sim* sim, int enable);
cpic_status cpic_get_timing(cpic_sim* sim, int cap, double* push_ms, double* solve_ms,
                            double* sort_ms, double* step_ms, int* samples);

/* Graph mode (enable != 0): each distinct variant of a step (buffer parity of
   every species after the last sort, whether this step sorts, whether the
   solve's initial guess is extrapolated) is recorded once as a HIP graph by
   stream capture and replayed by later steps, so a step costs one launch on
   the host.  Results are bitwise those of the ordinary path.  Steps with flux
   injection always run the ordinary path.  With timing enabled, a replayed
   step reports only its whole duration (the phase durations read 0).  Off by
   default.  Capture needs a stream other than the null stream; on the null
   stream every step runs the ordinary path (cpic_diag.step_graphs stays 0). */
cpic_status cpic_set_graphs(cpic_sim* sim, int enable);

const char* cpic_status_str(cpic_status s);
const char* cpic_last_error(const cpic_sim* sim);
void cpic_destroy(cpic_sim* sim);

/* ------------------------------------------------------------------ serving
 * A request loop over independent simulation cases, such as the parameter
 * sweeps of the paper's probe studies (object potential, plasma temperature;
 * Sec. "Tests").  Cases are admitted in submission order whenever a slot is
 * free and their device memory fits the HBM budget (admission is exact: a
 * case's allocations are counted against the budget while it is created, and
 * a case that does not fit waits until a running case finishes).  Admitted
 * cases stay resident and each pump iteration advances every running case by
 * one step, each slot on its own HIP stream, so their work overlaps on the
 * GPU.  A case's result does not depend on which other cases ran beside it.
 * The server is single-threaded: call it from one host thread.  Its cases
 * step in graph mode (cpic_set_graphs) unless the environment variable
 * CPIC_SERVER_NO_GRAPHS is set. */
#define CPIC_MAX_SPECIES 8
typedef struct cpic_server cpic_server;

typedef struct {
  cpic_map_desc map;                        /* a tabulated map's vertices are copied at submit */
  cpic_grid_desc grid;
  int nspecies;                             /* 1..CPIC_MAX_SPECIES */
  cpic_species_desc species[CPIC_MAX_SPECIES]; /* capacity 0 means the initial count */
  size_t count[CPIC_MAX_SPECIES];           /* initial particles per species */
  const int32_t* cell[CPIC_MAX_SPECIES];    /* host arrays laid out as for cpic_set_particles; */
  const void* off[CPIC_MAX_SPECIES];        /* copied at submit (the caller may free them after) */
  const void* vel[CPIC_MAX_SPECIES];
  int nsteps;                               /* steps after cpic_initialize, >= 1 */
  double* phi_out;                          /* optional host array of n cells: the potential after
                                               the last step, written before the case reports done */
} cpic_case_desc;

typedef struct {
  int status;             /* CPIC_OK when finished; else why the case failed (CPIC_E_BUDGET: it can
                             never fit the budget) */
  int steps;
  double kinetic, field_energy, mg_relres; /* as cpic_diag after the last step */
  int nspecies;
  long long count[CPIC_MAX_SPECIES], absorbed[CPIC_MAX_SPECIES], outflow[CPIC_MAX_SPECIES],
      injected[CPIC_MAX_SPECIES];
  uint64_t qsum_lo[CPIC_MAX_SPECIES], qsum_hi[CPIC_MAX_SPECIES];
  long long pushes;       /* particle pushes over all steps */
  double queue_ms;        /* submit -> admission (host clock) */
  double service_ms;      /* admission -> completion (host clock) */
  double step_p50_ms, step_p99_ms; /* per-step durations from HIP events on the case's stream */
} cpic_case_result;

typedef struct {
  long long submitted, completed, failed, queued, active;
  long long peak_active;  /* most cases resident at once */
  size_t budget_bytes, used_bytes, peak_bytes;
  long long pushes;       /* over completed cases */
  long long step_samples;
  double step_p50_ms, step_p99_ms; /* over every step of every completed case */
  long long batched_steps; /* case steps taken by cpic_step_batch with other cases */
} cpic_server_stats;

/* hbm_budget_bytes: device memory the cases may hold together; max_slots:
   cases resident at once (1..64); alloc: as for cpic_create (NULL: hipMalloc);
   hip_stream: NULL to give the server max_slots streams (created and
   destroyed by it, and one more where new cases are set up), else every case
   runs on that stream.  Running cases of one batch signature
   (cpic_batch_signature) share a stream and step together through
   cpic_step_batch; the others take the least loaded stream.  The
   environment variable CPIC_SERVER_NO_BATCH set at creation turns batching off. */
cpic_status cpic_server_create(size_t hbm_budget_bytes, int max_slots, const cpic_allocator* alloc,
                               void* hip_stream, cpic_server** out);
/* Queue a case; *ticket identifies it.  Validates the description (CPIC_E_ARG)
   and copies the particle arrays. */
cpic_status cpic_server_submit(cpic_server* srv, const cpic_case_desc* desc, uint64_t* ticket);
/* Run up to max_iterations rounds of: admit, one step of the running cases
   (the cases of a batch group through one cpic_step_batch; cases or groups
   whose step would wait for the device, see cpic_step_ready, wait for a later
   round unless none is ready), retire finished cases.  Returns CPIC_OK when nothing is queued or running
   afterwards, CPIC_E_PENDING otherwise. */
cpic_status cpic_server_pump(cpic_server* srv, int max_iterations);
/* CPIC_E_PENDING until the case is done, then CPIC_OK with *out filled
   (out->status tells whether it succeeded); CPIC_E_ARG for an unknown ticket. */
cpic_status cpic_server_poll(cpic_server* srv, uint64_t ticket, cpic_case_result* out);
cpic_status cpic_server_get_stats(cpic_server* srv, cpic_server_stats* out);
/* Frees every resident case and the server's streams. */
void cpic_server_destroy(cpic_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* CPIC_H_ */
