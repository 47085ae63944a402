// api.hip -- host core and C ABI of the MI355X curvilinear PIC library.
//
// Owns device memory (through the caller's allocator), validates descriptors,
// and orders the kernel launches of the PIC cycle on one HIP stream:
//   per step:  [species] zero Q_s, particle kernel (gather, push, Newton map
//              inversion, boundaries, deposit) -> charge -> rhs -> multigrid ->
//              gauge -> vertex field -> (every sort_every steps) tile sort.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "cpic.h"
#include "common.hpp"
#include "kernels.hpp"

using namespace cpic;

namespace {

constexpr int MAX_SPECIES = 8;
constexpr int NCOUNTERS = 10;
// Records of the last steps copied back to the host (solver iterations used,
// particle drift), one slot per step in a ring; step n waits for the record of
// step n - 2, so what it launches is a fixed function of the device state.
constexpr int HIST = 4;

struct Species {
  cpic_species_desc desc;
  size_t cap = 0;
  int cur = 0;
  int32_t* key[2] = {nullptr, nullptr};
  void* off[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
  void* vel[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
  uint32_t* id[2] = {nullptr, nullptr};
  int* d_n = nullptr;
  void* Q = nullptr;
  int* counts = nullptr;
  int* start = nullptr;
  int* cursor = nullptr;
  int* n_items = nullptr;
  int* item_tile = nullptr;
  int* item_begin = nullptr;
  int* item_end = nullptr;
  int max_items = 0;
  double* ke_part = nullptr;
  // absorbed, outflow, fallback, far, nonconv, injected, dropped, ids issued, injected but
  // gone at once, deposited since Q was cleared (NCOUNTERS)
  unsigned long long* counters = nullptr;
  unsigned long long* dead_mark = nullptr;  // counters[0..8] at the last sort (departures since then)
  double inject_lam = 0.0;
  int* fb_queue = nullptr;  // particles handed to the FP64 fallback kernel
  int* fb_count = nullptr;
  int since_sort = 0;       // steps since this species' last tile sort
  long long sorts = 0;      // tile sorts so far
};

struct StepEvents {
  hipEvent_t e[5];  // start, before particle kernels, after them, after field, after sort
};

}  // namespace

struct cpic_sim {
  int device = 0;  // the HIP device current at creation
  cpic_map_desc map;
  cpic_grid_desc grid;
  cpic_allocator alloc;
  bool has_alloc = false;
  hipStream_t stream = nullptr;
  Geo g;
  GridCtx G;
  std::vector<Species> sp;
  int S1 = 24;
  int chunk = 4096;
  double kappa = 0.0;  // Newton quadratic-convergence constant of the map (cells)
  bool initialized = false;
  bool poisoned = false;
  bool sorted_dirty = true;
  bool phi_prev_valid = false;  // G.phi_prev holds the previous step's potential
  void* kc = nullptr;           // predictor-corrector mover: vertex table of n_a dxi^a/dx^b
  bool graphs = false;          // replay recorded HIP graphs of the step
  unsigned* drift_dev = nullptr;   // per species: running max of a particle's increment (cells, FP32 bits)
  int* cycles_host = nullptr;      // pinned [HIST]: V-cycles of the solve of step n in slot n % HIST
  unsigned* drift_host = nullptr;  // pinned [HIST][8]: drift_dev after step n in slot n % HIST
  hipEvent_t hist_ev[HIST] = {};   // recorded after the copies of step n, slot n % HIST
  long long hist_from = 0;         // records of steps before this one are not used
  bool overflowed = false;         // a fixed-point deposit wrapped (sticky until new particles)
  BatchArgs batch_args;            // argument structs of batched field phases led by this simulation
  BatchArgs batch_pargs;           // argument structs of batched particle kernels led by it
  long long batched_steps = 0;     // steps whose field phase ran batched
  struct StepGraph {
    uint64_t key;
    hipGraphExec_t exec;
    std::vector<int> cur_after;
  };
  std::vector<StepGraph> step_graphs;
  long long step = 0;
  double* ke = nullptr;  // device: kinetic energy of the last push
  int* flags = nullptr;  // device ints: [0] bad input count
  uint64_t* qsum = nullptr;
  double* tmp_scalar = nullptr;
  std::string err;
  std::vector<std::pair<void*, size_t>> allocs;
  bool timing = false;
  std::vector<StepEvents> evs;
  size_t ev_used = 0;
};

// ----------------------------------------------------------------------------
static cpic_status fail(cpic_sim* s, cpic_status st, const std::string& msg) {
  if (s) s->err = msg;
  return st;
}

#define HIPCHK(sim, expr)                                                           \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) {                                                         \
      (sim)->poisoned = true;                                                       \
      return fail((sim), CPIC_E_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
    }                                                                               \
  } while (0)

static void* sim_alloc(cpic_sim* s, size_t bytes) {
  if (bytes == 0) bytes = 8;
  bytes = (bytes + 255) & ~(size_t)255;
  void* p = nullptr;
  if (s->has_alloc) {
    p = s->alloc.alloc(bytes, s->alloc.ctx);
  } else {
    if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
  }
  if (p) s->allocs.push_back({p, bytes});
  return p;
}

// the batch argument buffer: the simulation's allocator, outside its list
// (the buffer may be replaced by a larger one while the simulation lives)
static void* batch_dev_alloc(size_t bytes, void* ctx) {
  cpic_sim* s = (cpic_sim*)ctx;
  void* p = nullptr;
  if (s->has_alloc) return s->alloc.alloc(bytes, s->alloc.ctx);
  return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}
static void batch_dev_free(void* p, void* ctx) {
  cpic_sim* s = (cpic_sim*)ctx;
  if (s->has_alloc)
    s->alloc.free(p, s->alloc.ctx);
  else
    (void)hipFree(p);
}

static void sim_free_all(cpic_sim* s) {
  for (auto& a : s->allocs) {
    if (s->has_alloc)
      s->alloc.free(a.first, s->alloc.ctx);
    else
      (void)hipFree(a.first);
  }
  s->allocs.clear();
}

static int bits_for(int n) {
  int b = 0;
  while ((1 << b) < n) ++b;
  return b < 1 ? 1 : b;
}

static size_t real_size(const cpic_sim* s) { return s->grid.precision == CPIC_FP64 ? 8 : 4; }
static int ecomp(const cpic_sim* s) { return s->map.dim == 3 ? 4 : 2; }

static cpic_status check_async(cpic_sim* s) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    s->poisoned = true;
    return fail(s, CPIC_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  }
  return CPIC_OK;
}

// ----------------------------------------------------------------------------
// Scratch of cpic_get_diag_noalloc: the reductions of the diagnostics work in
// a file-scope device array instead of buffers the simulation allocated.  Each
// device holds its own copy until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns for that device (the array's
// name is a host-side stand-in).  Layout: REDUCE_BLOCKS doubles of field-energy
// partials, the energy sum and the non-finite count, then QSUM_WORDS words of
// exact-charge sums per species.
// ----------------------------------------------------------------------------
constexpr size_t SCR_PARTIALS = 0;
constexpr size_t SCR_WE = SCR_PARTIALS + sizeof(double) * REDUCE_BLOCKS;
constexpr size_t SCR_NONFINITE = SCR_WE + sizeof(double);
constexpr size_t SCR_QSUM = (SCR_NONFINITE + sizeof(int) + 255) & ~(size_t)255;
constexpr int SCR_SPECIES = MAX_SPECIES;
constexpr size_t SCRATCH_BYTES = SCR_QSUM + sizeof(uint64_t) * QSUM_WORDS * SCR_SPECIES;  // 35,200 bytes
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int SCRATCH_DEVICES = 64;
static std::mutex scratch_mu;
static void* scratch_addr[SCRATCH_DEVICES] = {};

// Address of `scratch` on device `dev`, looked up once per device with that
// device current; nullptr when the lookup fails.
static void* scratch_on(int dev) {
  if (dev < 0 || dev >= SCRATCH_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_addr[dev]) return scratch_addr[dev];
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return nullptr;
  if (cur != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != dev) (void)hipSetDevice(cur);
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return nullptr;
  }
  scratch_addr[dev] = p;
  return p;
}

// ----------------------------------------------------------------------------
// creation
// ----------------------------------------------------------------------------
extern "C" cpic_status cpic_create(const cpic_map_desc* map, const cpic_grid_desc* grid,
                                   const cpic_allocator* alloc, void* hip_stream, cpic_sim** out) {
  if (!map || !grid || !out) return CPIC_E_ARG;
  *out = nullptr;
  const int d = map->dim;
  if (d != 2 && d != 3) return CPIC_E_ARG;
  if (map->kind < CPIC_MAP_IDENTITY || map->kind > CPIC_MAP_TABULATED) return CPIC_E_ARG;
  const bool tabulated = map->kind == CPIC_MAP_TABULATED;
  if (tabulated && !map->vertices) return CPIC_E_ARG;
  const bool radial = map->kind == CPIC_MAP_POLAR_LOG || map->kind == CPIC_MAP_SPHERICAL_RZ;
  if (radial && (d != 2 || !(map->r_in > 0) || !(map->r_out > map->r_in))) return CPIC_E_ARG;
  // Omega = x^1 is the radius of an r-z plane: it must stay >= 0, which holds
  // on the identity map (bounded axis 0) and the spherical r-z map
  if (map->omega != 0 && map->omega != 1) return CPIC_E_ARG;
  if (map->omega && (d != 2 || (map->kind != CPIC_MAP_IDENTITY && map->kind != CPIC_MAP_SPHERICAL_RZ) ||
                     grid->bc_lo[0] == CPIC_BC_PERIODIC))
    return CPIC_E_UNSUPPORTED;
  if (tabulated) {
    // L_a: the shift of x^a per period of a periodic axis (0: the map closes
    // on itself, e.g. an angle)
    for (int a = 0; a < d; ++a)
      if (!(map->L[a] >= 0) || !isfinite(map->L[a])) return CPIC_E_ARG;
  } else if (!radial) {
    for (int a = 0; a < d; ++a)
      if (!(map->L[a] > 0)) return CPIC_E_ARG;
  }
  if (map->kind == CPIC_MAP_SINUSOIDAL) {
    // J = 1 + 2 pi eps (sum of products); its bracket is bounded by 1 (2D) and
    // 2/sqrt(3) (3D): the map folds beyond eps = 1/(2 pi) resp. sqrt(3)/(4 pi)
    double bound = (d == 2) ? 1.0 : 2.0 / sqrt(3.0);
    if (!(2.0 * M_PI * fabs(map->eps) * bound < 1.0)) return CPIC_E_MAP;
  }
  long long ncells = 1;
  int bitsum = 0;
  for (int a = 0; a < d; ++a) {
    if (grid->n[a] < 2 || grid->n[a] > (1 << 14)) return CPIC_E_ARG;
    ncells *= grid->n[a];
    bitsum += bits_for(grid->n[a]);
    bool plo = grid->bc_lo[a] == CPIC_BC_PERIODIC, phi = grid->bc_hi[a] == CPIC_BC_PERIODIC;
    if (plo != phi) return CPIC_E_ARG;
    const int lo_max = a == 0 ? CPIC_BC_FLOATING : CPIC_BC_NEUMANN;
    if (grid->bc_lo[a] < 0 || grid->bc_lo[a] > lo_max || grid->bc_hi[a] < 0 || grid->bc_hi[a] > CPIC_BC_NEUMANN)
      return CPIC_E_ARG;
  }
  const bool floating = grid->bc_lo[0] == CPIC_BC_FLOATING;
  if (floating)
    for (int a = 1; a < d; ++a)
      if (grid->bc_lo[a] != CPIC_BC_PERIODIC) return CPIC_E_UNSUPPORTED;
  if (bitsum > 30 || ncells > (1ll << 30)) return CPIC_E_ARG;
  bool all_periodic = true;
  for (int a = 0; a < d; ++a) all_periodic = all_periodic && grid->bc_lo[a] == CPIC_BC_PERIODIC;
  if (!all_periodic && map->kind == CPIC_MAP_SINUSOIDAL && map->eps != 0.0) return CPIC_E_UNSUPPORTED;
  if (grid->shape != CPIC_SHAPE_B1 && grid->shape != CPIC_SHAPE_B2) return CPIC_E_ARG;
  if (grid->precision != CPIC_FP32 && grid->precision != CPIC_FP64) return CPIC_E_ARG;
  if (!(grid->dt > 0) || !isfinite(grid->dt)) return CPIC_E_ARG;
  if (grid->background && (d != 2 || !all_periodic)) return CPIC_E_UNSUPPORTED;
  if (grid->mg_method != CPIC_MG_FCG && grid->mg_method != CPIC_MG_VCYCLE && grid->mg_method != CPIC_MG_BOXMG)
    return CPIC_E_ARG;
  if (grid->mg_method == CPIC_MG_BOXMG &&
      (map->dim != 2 || grid->n[0] < 4 || grid->n[1] < 4 || grid->n[0] > 4096 || grid->n[1] > 4096))
    return CPIC_E_UNSUPPORTED;
  if (grid->mover != CPIC_MOVER_NEWTON && grid->mover != CPIC_MOVER_PC) return CPIC_E_ARG;
  if (grid->pusher != CPIC_PUSH_BORIS && grid->pusher != CPIC_PUSH_CYCLOTRONIC) return CPIC_E_ARG;
  if (grid->pusher == CPIC_PUSH_CYCLOTRONIC && grid->mover != CPIC_MOVER_NEWTON) return CPIC_E_UNSUPPORTED;

  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return CPIC_E_HIP;
  cpic_sim* s = new cpic_sim();
  s->device = device;
  // per-device set-up of the no-allocation diagnostics' scratch (its entry
  // point reports a failed lookup; nothing else needs it)
  (void)scratch_on(device);
  s->map = *map;
  s->grid = *grid;
  if (s->grid.mg_rtol <= 0) s->grid.mg_rtol = 1e-10;
  if (s->grid.mg_max_cycles <= 0) s->grid.mg_max_cycles = 20;
  if (s->grid.sort_every <= 0) s->grid.sort_every = 1;
  if (alloc && alloc->alloc && alloc->free) {
    s->alloc = *alloc;
    s->has_alloc = true;
  }
  s->stream = (hipStream_t)hip_stream;
  for (BatchArgs* ba : {&s->batch_args, &s->batch_pargs}) {
    ba->dev_alloc = batch_dev_alloc;
    ba->dev_free = batch_dev_free;
    ba->ctx = s;
  }
  s->S1 = (d == 2) ? 24 : 16;
  s->chunk = (d == 2) ? 4096 : 16384;
  {
    // Newton on the map increment converges quadratically: the error after a
    // step s is at most kappa |s|^2 (in cells).  Sinusoidal: the residual
    // after the step is e R, |R| <= (1/2) w_max^2 |s|_1^2 with w = 2 pi / n,
    // and the inverse of the mean-value Jacobian (I + e g^T) maps e to e / J,
    // so kappa = e_max w_max^2 / (2 J_min) with the 1-norm of the step.
    // Polar-log: second derivatives ~ k_max^2, inverse ~ 1/k_min with
    // k = (ln R / n0, 2 pi / n1), max-norm of the step.
    int nmin = grid->n[0], nmax = grid->n[0];
    for (int a = 1; a < d; ++a) {
      nmin = std::min(nmin, grid->n[a]);
      nmax = std::max(nmax, grid->n[a]);
    }
    if (map->kind == CPIC_MAP_SINUSOIDAL) {
      double bound = (d == 2) ? 1.0 : 2.0 / sqrt(3.0);
      double jmin = 1.0 - 2.0 * M_PI * fabs(map->eps) * bound;
      double emax = fabs(map->eps) * nmax;
      double w = 2.0 * M_PI / nmin;
      s->kappa = 0.5 * emax * w * w / jmin;
    } else if (map->kind == CPIC_MAP_POLAR_LOG) {
      double kx = log(map->r_out / map->r_in) / grid->n[0], ky = 2.0 * M_PI / grid->n[1];
      double kmax = std::max(kx, ky), kmin = std::min(kx, ky);
      s->kappa = 0.5 * d * d * kmax * kmax / kmin;
    }
  }

  Geo& g = s->g;
  memset(&g, 0, sizeof(g));
  g.dim = d;
  g.kind = map->kind;
  g.ncells = ncells;
  g.nverts = 1;
  g.ntiles = 1;
  const int T[3] = {d == 2 ? TileShape<2>::T0 : TileShape<3>::T0, d == 2 ? TileShape<2>::T1 : TileShape<3>::T1,
                    d == 2 ? 1 : TileShape<3>::T2};
  for (int a = 0; a < 3; ++a) {
    if (a < d) {
      g.n[a] = grid->n[a];
      g.periodic[a] = grid->bc_lo[a] == CPIC_BC_PERIODIC;
      g.nv[a] = g.periodic[a] ? g.n[a] : g.n[a] + 1;
      g.nt[a] = (g.n[a] + T[a] - 1) / T[a];
      g.invn[a] = 1.0 / g.n[a];
      g.L[a] = map->L[a];
    } else {
      g.n[a] = 1;
      g.nv[a] = 1;
      g.nt[a] = 1;
      g.periodic[a] = 1;
      g.invn[a] = 1.0;
      g.L[a] = 1.0;
    }
    g.nverts *= g.nv[a];
    g.ntiles *= g.nt[a];
  }
  g.sx = bits_for(g.n[0]);
  g.sy = bits_for(g.n[1]);
  g.eps = map->kind == CPIC_MAP_SINUSOIDAL ? map->eps : 0.0;
  g.r_in = map->r_in;
  g.r_out = map->r_out;
  g.lnR = map->kind == CPIC_MAP_POLAR_LOG ? log(map->r_out / map->r_in) : 0.0;
  g.omega = map->omega;
  for (int a = 0; a < 3; ++a) {
    g.ecell[a] = g.eps * g.n[a];
    g.dxc[a] = g.L[a] / g.n[a];
  }

  // grid context and multigrid hierarchy
  GridCtx& G = s->G;
  memset(&G, 0, sizeof(G));
  G.g = g;
  G.fp64 = grid->precision == CPIC_FP64;
  G.all_periodic = all_periodic;
  G.mixed = (map->kind == CPIC_MAP_SINUSOIDAL && map->eps != 0.0) || tabulated;
  for (int a = 0; a < 3; ++a) {
    G.bc_lo[a] = a < d ? grid->bc_lo[a] : CPIC_BC_PERIODIC;
    G.bc_hi[a] = a < d ? grid->bc_hi[a] : CPIC_BC_PERIODIC;
    G.phi_lo[a] = a < d ? grid->phi_lo[a] : 0.0;
    G.phi_hi[a] = a < d ? grid->phi_hi[a] : 0.0;
  }
  if (floating) {
    // the operator sees the floating wall as a Dirichlet wall at 0 (phi_0)
    G.floating = 1;
    G.bc_lo[0] = CPIC_BC_DIRICHLET;
    G.phi_lo[0] = 0.0;
  }
  int nl = 0;
  int n[3] = {g.n[0], g.n[1], g.n[2]};
  while (nl < 16) {
    Level& L = G.lev[nl];
    L.ncells = 1;
    L.dV = 1.0;
    for (int a = 0; a < 3; ++a) {
      L.n[a] = n[a];
      L.h[a] = a < d ? 1.0 / n[a] : 1.0;
      L.ncells *= n[a];
      L.dV *= L.h[a];
    }
    ++nl;
    bool can = true;
    for (int a = 0; a < d; ++a) can = can && (n[a] % 2 == 0) && (n[a] / 2 >= 4);
    if (!can) break;
    for (int a = 0; a < d; ++a) n[a] /= 2;
  }
  G.nlev = nl;
  bool ok = true;
  auto A = [&](size_t bytes) {
    void* p = sim_alloc(s, bytes);
    if (!p) ok = false;
    return p;
  };
  const int np = d == 3 ? 3 : 1;
  for (int l = 0; l < nl; ++l) {
    Level& L = G.lev[l];
    size_t b = sizeof(double) * (size_t)L.ncells;
    for (int a = 0; a < 3; ++a) {
      L.wf[a] = a < d ? (double*)A(b) : nullptr;
      L.wlo[a] = a < d ? (double*)A(b) : nullptr;
      L.we[a] = a < np ? (double*)A(b) : nullptr;
    }
    L.diag = (double*)A(b);
    L.phi = (double*)A(b);
    L.phi2 = (double*)A(b);
    L.rhs = (double*)A(b);
    L.res = (double*)A(b);
    L.aux = (double*)A(b);
    // stencil slots: faces x, y (, z); mixed pairs only for non-orthogonal maps
    for (int k = 0; k < 9; ++k) {
      bool used = (k < d) || (G.mixed && (d == 3 ? k >= 3 : (k == 3 || k == 4)));
      L.S[k] = used ? (double*)A(b) : nullptr;
    }
  }
  size_t cb = sizeof(double) * (size_t)ncells;
  G.bdir = (double*)A(cb);
  if (floating) {
    G.phi1 = (double*)A(cb);
    G.bdir1 = (double*)A(cb);
    G.phi_full = (double*)A(cb);
    G.E1 = A(real_size(s) * ecomp(s) * (size_t)g.nverts);
  }
  G.Jc = (double*)A(cb);
  G.charge = (double*)A(cb);
  G.background = grid->background ? (double*)A(cb) : nullptr;
  G.partials = (double*)A(sizeof(double) * 1024);
  const size_t sweep_blocks = (size_t)((g.n[0] + 63) / 64) * ((g.n[1] + 3) / 4) * g.n[2];
  G.mg_partials = (double*)A(sizeof(double) * sweep_blocks);
  G.boxmg = grid->mg_method == CPIC_MG_BOXMG;
  G.coarse = nl - 1;
  if (G.boxmg)
    // the variational hierarchy ends at the first level the dense inverse can take
    for (int l = 0; l < nl; ++l)
      if (G.lev[l].ncells <= DENSE_MAX) {
        G.coarse = l;
        break;
      }
  if (G.lev[G.coarse].ncells <= DENSE_MAX) {
    const size_t nn = (size_t)G.lev[G.coarse].ncells * (size_t)G.lev[G.coarse].ncells;
    G.cinv64 = (double*)A(sizeof(double) * nn);
    if (grid->mg_method != CPIC_MG_VCYCLE) G.cinv32 = (float*)A(sizeof(float) * nn);
  }
  if (G.boxmg)
    for (int l = 1; l <= G.coarse; ++l) {
      Level& L = G.lev[l];
      L.gal64 = (double*)A(sizeof(double) * 25 * (size_t)L.ncells);
      L.gal32 = (float*)A(sizeof(float) * 25 * (size_t)L.ncells);
    }
  if (grid->mg_method != CPIC_MG_VCYCLE) {
    for (int l = 0; l < nl; ++l) {
      Level& L = G.lev[l];
      const size_t fb = sizeof(float) * (size_t)L.ncells;
      for (int k = 0; k < 9; ++k) L.f_S[k] = L.S[k] ? (float*)A(fb) : nullptr;
      L.f_diag = (float*)A(fb);
      L.f_phi = (float*)A(fb);
      L.f_phi2 = (float*)A(fb);
      L.f_rhs = (float*)A(fb);
      L.f_res = (float*)A(fb);
      L.f_aux = (float*)A(fb);
      if (!G.boxmg && L.ncells > SMALL_CELLS) {
        const size_t hb = sizeof(unsigned short) * (size_t)L.ncells;
        for (int k = 0; k < 9; ++k) L.h_S[k] = L.S[k] ? (unsigned short*)A(hb) : nullptr;
        L.h_diag = (unsigned short*)A(hb);
      }
    }
    G.kr = (double*)A(cb);
    G.kp = (double*)A(cb);
    G.kq = (double*)A(cb);
    G.kw = (double*)A(cb);
    G.k_partials = (double*)A(sizeof(double) * 3 * sweep_blocks);
  }
  G.scalars = (double*)A(sizeof(double) * 16);
  G.mg_flag = (int*)A(sizeof(int) * 4);
  s->drift_dev = (unsigned*)A(sizeof(unsigned) * 8);
  G.Ev = A(real_size(s) * ecomp(s) * (size_t)g.nverts);
  G.Kv = (double*)A(sizeof(double) * (size_t)(d * d) * (size_t)g.nverts);
  double* xtab = tabulated ? (double*)A(sizeof(double) * (size_t)d * (size_t)g.nverts) : nullptr;
  double* jtab = tabulated ? (double*)A(sizeof(double) * (size_t)(d * d) * (size_t)g.nverts) : nullptr;
  // predictor-corrector table: d x d per vertex padded to 4 (2D) or 12 (3D) values
  if (grid->mover == CPIC_MOVER_PC) s->kc = A(real_size(s) * (size_t)(d == 3 ? 12 : 4) * (size_t)g.nverts);
  G.phi_prev = (double*)A(cb);
  s->ke = (double*)A(sizeof(double) * 2);
  s->flags = (int*)A(sizeof(int) * 8);
  s->qsum = (uint64_t*)A(sizeof(uint64_t) * QSUM_WORDS * MAX_SPECIES);
  s->tmp_scalar = (double*)A(sizeof(double) * 4);
  if (!ok) {
    sim_free_all(s);
    delete s;
    return CPIC_E_NOMEM;
  }
  hipStream_t st = s->stream;
  // tabulated map: vertex coordinates in (d values per vertex), then the Jacobi
  // matrices by finite differences; every metric below is taken from them
  std::vector<double> xh;
  if (tabulated) {
    const size_t nv = (size_t)g.nverts;
    xh.resize((size_t)d * nv);
    bool finite = true;
    for (size_t v = 0; v < nv; ++v)
      for (int a = 0; a < d; ++a) {
        const double x = map->vertices[(size_t)a * nv + v];
        finite = finite && isfinite(x);
        xh[v * d + a] = x;
      }
    if (!finite) {
      sim_free_all(s);
      delete s;
      return CPIC_E_ARG;
    }
    s->g.xtab = G.g.xtab = xtab;
    s->g.jtab = G.g.jtab = jtab;
    if (hipMemcpyAsync(xtab, xh.data(), sizeof(double) * xh.size(), hipMemcpyHostToDevice, st) != hipSuccess) {
      cpic_destroy(s);
      return CPIC_E_HIP;
    }
    launch_map_table(G.g, jtab, st);
  }
  for (int l = 0; l < nl; ++l) {
    Level& L = G.lev[l];
    size_t b = sizeof(double) * (size_t)L.ncells;
    launch_fill_u8(L.phi, 0, b, st);
    launch_fill_u8(L.phi2, 0, b, st);
    launch_fill_u8(L.rhs, 0, b, st);
    launch_coefficients(G, l, st);
    if (L.f_phi) {
      const size_t fb = sizeof(float) * (size_t)L.ncells;
      for (float* v : {L.f_phi, L.f_phi2, L.f_rhs, L.f_res, L.f_aux}) launch_fill_u8(v, 0, fb, st);
    }
  }
  if (launch_operator_f32(G, st) != 0) {
    cpic_destroy(s);
    return CPIC_E_HIP;
  }
  launch_fill_u8(G.charge, 0, cb, st);
  launch_fill_u8(G.Ev, 0, real_size(s) * ecomp(s) * (size_t)g.nverts, st);
  launch_fill_u8(s->ke, 0, sizeof(double) * 2, st);
  launch_fill_u8(G.mg_flag, 0, sizeof(int) * 4, st);
  launch_fill_u8(s->drift_dev, 0, sizeof(unsigned) * 8, st);
  launch_jacobian_centres(G, st);
  launch_vertex_metric(G, st);
  if (s->kc) launch_kc_table(g, G.Kv, s->kc, G.fp64, st);
  if (hipHostMalloc((void**)&s->cycles_host, sizeof(int) * HIST, hipHostMallocDefault) != hipSuccess) {
    s->cycles_host = nullptr;
    cpic_destroy(s);
    return CPIC_E_NOMEM;
  }
  if (hipHostMalloc((void**)&s->drift_host, sizeof(unsigned) * 8 * HIST, hipHostMallocDefault) != hipSuccess) {
    s->drift_host = nullptr;
    cpic_destroy(s);
    return CPIC_E_NOMEM;
  }
  for (int i = 0; i < HIST; ++i) s->cycles_host[i] = -1;
  memset(s->drift_host, 0, sizeof(unsigned) * 8 * HIST);
  for (int i = 0; i < HIST; ++i)
    if (hipEventCreateWithFlags(&s->hist_ev[i], hipEventDisableTiming) != hipSuccess) {
      s->hist_ev[i] = nullptr;
      cpic_destroy(s);
      return CPIC_E_HIP;
    }
  if (compute_smoother_bounds(G, st) != 0 || setup_galerkin(G, st) != 0 || setup_coarse_inverse(G, st) != 0 ||
      setup_floating_wall(G, st) != 0) {
    cpic_destroy(s);
    return CPIC_E_HIP;
  }
  if (G.background) launch_background(G, grid->shape, grid->background_n0, st);
  cpic_status rc = check_async(s);
  if (rc != CPIC_OK) {
    cpic_destroy(s);
    return rc;
  }
  // sum_c J_c via a one-off host reduction of the (small) J array
  std::vector<double> Jh((size_t)ncells);
  if (hipMemcpyAsync(Jh.data(), G.Jc, cb, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    cpic_destroy(s);
    return CPIC_E_HIP;
  }
  double sj = 0.0;
  double jmin = 1e300;
  for (double v : Jh) {
    sj += v;
    jmin = std::min(jmin, v);
  }
  G.sumJ = sj;
  if (!(jmin > 0)) {
    cpic_destroy(s);
    return CPIC_E_MAP;
  }
  if (tabulated) {
    // the tabulated map must fold nowhere (J > 0 at every vertex as at every
    // cell centre) and, with walls, be orthogonal in every plane that holds a
    // bounded axis (the operator keeps mixed terms only between periodic
    // axes): there the columns of j may deviate from a right angle by at most
    // acos(0.05) -- the sampling error of an orthogonal map
    const size_t nv = (size_t)g.nverts, dd = (size_t)(d * d);
    std::vector<double> jh(dd * nv);
    if (hipMemcpyAsync(jh.data(), jtab, sizeof(double) * jh.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      cpic_destroy(s);
      return CPIC_E_HIP;
    }
    cpic_status bad = CPIC_OK;
    for (size_t v = 0; v < nv && bad == CPIC_OK; ++v) {
      const double* j = jh.data() + v * dd;
      double det = (d == 2) ? j[0] * j[3] - j[1] * j[2]
                            : j[0] * (j[4] * j[8] - j[5] * j[7]) - j[1] * (j[3] * j[8] - j[5] * j[6]) +
                                  j[2] * (j[3] * j[7] - j[4] * j[6]);
      if (!(det > 0)) bad = CPIC_E_MAP;
      for (int p = 0; p < d && bad == CPIC_OK; ++p)
        for (int q = p + 1; q < d; ++q) {
          if (g.periodic[p] && g.periodic[q]) continue;
          double dot = 0.0, np2 = 0.0, nq2 = 0.0;
          for (int a = 0; a < d; ++a) {
            dot += j[a * d + p] * j[a * d + q];
            np2 += j[a * d + p] * j[a * d + p];
            nq2 += j[a * d + q] * j[a * d + q];
          }
          if (fabs(dot) > 0.05 * sqrt(np2 * nq2)) bad = CPIC_E_UNSUPPORTED;
        }
    }
    if (bad != CPIC_OK) {
      cpic_destroy(s);
      return bad;
    }
  }
  *out = s;
  return CPIC_OK;
}

extern "C" cpic_status cpic_add_species(cpic_sim* s, const cpic_species_desc* desc, int* sid) {
  if (!s || !desc || !sid) return CPIC_E_ARG;
  if (s->poisoned) return fail(s, CPIC_E_STATE, "simulation poisoned by an earlier device error");
  if ((int)s->sp.size() >= MAX_SPECIES) return fail(s, CPIC_E_ARG, "too many species");
  if (s->initialized) return fail(s, CPIC_E_STATE, "species must be added before cpic_initialize");
  if (!(desc->m != 0) || !(desc->w > 0) || !isfinite(desc->q) || desc->capacity == 0 ||
      desc->capacity > (size_t)INT32_MAX / 2)
    return fail(s, CPIC_E_ARG, "bad species descriptor");
  if (s->g.kind == CPIC_MAP_SPHERICAL_RZ || s->g.omega)
    return fail(s, CPIC_E_UNSUPPORTED, "the spherical r-z map and Omega = r serve the field solve only");
  const int d = s->g.dim;
  for (int a = 0; a < d; ++a) {
    bool per = s->g.periodic[a];
    for (int side = 0; side < 2; ++side) {
      int b = side ? desc->pbc_hi[a] : desc->pbc_lo[a];
      if (per && b != CPIC_PBC_PERIODIC) return fail(s, CPIC_E_ARG, "particle bc must be periodic on a periodic axis");
      if (!per && b != CPIC_PBC_ABSORB && b != CPIC_PBC_OUTFLOW)
        return fail(s, CPIC_E_ARG, "particle bc must absorb or outflow on a bounded axis");
    }
  }
  double lam = 0.0;
  if (desc->inject) {
    if (s->g.periodic[0]) return fail(s, CPIC_E_ARG, "injection needs a bounded axis 0");
    if (s->g.kind != CPIC_MAP_IDENTITY && s->g.kind != CPIC_MAP_POLAR_LOG)
      return fail(s, CPIC_E_UNSUPPORTED, "injection needs an orthogonal analytic map");
    if (!(desc->inject_n0 > 0) || !(desc->inject_vth > 0) || !(desc->inject_drift >= 0) ||
        !isfinite(desc->inject_drift))
      return fail(s, CPIC_E_ARG, "bad injection parameters");
    // area of the outer face: 2 pi r_out (polar-log, per unit length) or the
    // product of the other box lengths; one-sided Maxwellian particle flux
    double A = 1.0;
    if (s->g.kind == CPIC_MAP_POLAR_LOG)
      A = 2.0 * M_PI * s->map.r_out;
    else
      for (int a = 1; a < d; ++a) A *= s->map.L[a];
    // inward flux of a Maxwellian drifting inward at s thermal speeds:
    // n0 vth (phi(s) + s Phi(s)), phi / Phi the standard normal density / CDF
    const double sd = desc->inject_drift / desc->inject_vth;
    const double flux = desc->inject_n0 * desc->inject_vth *
                        (exp(-0.5 * sd * sd) / sqrt(2.0 * M_PI) + sd * 0.5 * (1.0 + erf(sd / sqrt(2.0))));
    lam = flux * A * s->grid.dt / desc->w;
    if (lam > 1e8) return fail(s, CPIC_E_ARG, "injection rate too large");
  }
  Species S;
  S.desc = *desc;
  S.cap = desc->capacity;
  S.inject_lam = lam;
  bool ok = true;
  auto A = [&](size_t bytes) {
    void* p = sim_alloc(s, bytes);
    if (!p) ok = false;
    return p;
  };
  const size_t rs = real_size(s);
  for (int b = 0; b < 2; ++b) {
    S.key[b] = (int32_t*)A(sizeof(int32_t) * S.cap);
    for (int a = 0; a < 3; ++a) {
      S.off[b][a] = a < d ? A(rs * S.cap) : nullptr;
      S.vel[b][a] = A(rs * S.cap);
    }
    S.id[b] = s->grid.track_ids ? (uint32_t*)A(sizeof(uint32_t) * S.cap) : nullptr;
  }
  S.d_n = (int*)A(sizeof(int) * 2);
  S.Q = A(8 * (size_t)s->g.ncells);
  const int nt = s->g.ntiles;
  S.counts = (int*)A(sizeof(int) * (nt + 2));
  S.start = (int*)A(sizeof(int) * (nt + 2));
  S.cursor = (int*)A(sizeof(int) * (nt + 2));
  S.n_items = (int*)A(sizeof(int) * 2);
  S.max_items = (int)((S.cap + s->chunk - 1) / s->chunk) + nt;
  S.item_tile = (int*)A(sizeof(int) * S.max_items);
  S.item_begin = (int*)A(sizeof(int) * S.max_items);
  S.item_end = (int*)A(sizeof(int) * S.max_items);
  S.ke_part = (double*)A(sizeof(double) * (S.max_items + TAIL_ITEMS));  // + the appended particles' items
  S.counters = (unsigned long long*)A(sizeof(unsigned long long) * NCOUNTERS);
  S.dead_mark = (unsigned long long*)A(sizeof(unsigned long long) * NCOUNTERS);
  S.fb_queue = (int*)A(sizeof(int) * S.cap);
  S.fb_count = (int*)A(sizeof(int) * 2);
  if (!ok) return fail(s, CPIC_E_NOMEM, "species allocation failed");
  hipStream_t st = s->stream;
  launch_fill_u8(S.d_n, 0, sizeof(int) * 2, st);
  launch_fill_u8(S.n_items, 0, sizeof(int) * 2, st);
  launch_fill_u8(S.counters, 0, sizeof(unsigned long long) * NCOUNTERS, st);
  launch_fill_u8(S.dead_mark, 0, sizeof(unsigned long long) * NCOUNTERS, st);
  launch_fill_u8(S.Q, 0, 8 * (size_t)s->g.ncells, st);
  s->sp.push_back(S);
  *sid = (int)s->sp.size() - 1;
  s->sorted_dirty = true;
  return check_async(s);
}

// ----------------------------------------------------------------------------
// particles in / out
// ----------------------------------------------------------------------------
// Headroom of the fixed-point deposit: a particle adds at most 2^{d S1} = 2^48
// to any cell, and only to cells within one of its own per axis, so a cell's
// uint64 sum cannot wrap while every 3^d block of cells holds fewer than 2^16
// particles.  True when some block holds more (host arrays).
static bool crowded(const cpic_sim* s, size_t n, const int32_t* cell) {
  if (n < (1u << 16)) return false;
  const Geo& g = s->g;
  std::vector<uint32_t> cnt((size_t)g.ncells, 0u);
  for (size_t p = 0; p < n; ++p) ++cnt[(size_t)cell[p]];
  // sums over windows of three cells, one axis at a time (wrapped on periodic
  // axes, cut at walls)
  std::vector<uint64_t> a(cnt.begin(), cnt.end()), b((size_t)g.ncells);
  const long long str[3] = {1, g.n[0], (long long)g.n[0] * g.n[1]};
  for (int ax = 0; ax < g.dim; ++ax) {
    const int nn = g.n[ax];
    for (long long c = 0; c < g.ncells; ++c) {
      const int i = (int)((c / str[ax]) % nn);
      uint64_t v = a[(size_t)c];
      for (int o = -1; o <= 1; o += 2) {
        int j = i + o;
        if (g.periodic[ax]) j = (j + nn) % nn;
        else if (j < 0 || j >= nn) continue;
        if (j == i) continue;
        v += a[(size_t)(c + (long long)(j - i) * str[ax])];
      }
      b[(size_t)c] = v;
    }
    a.swap(b);
  }
  for (uint64_t v : a)
    if (v >= (1u << 16)) return true;
  return false;
}

extern "C" cpic_status cpic_set_particles(cpic_sim* s, int sid, size_t n, const int32_t* cell,
                                          const void* off, const void* vel, const uint32_t* ids,
                                          int on_device) {
  if (!s) return CPIC_E_ARG;
  if (s->poisoned) return fail(s, CPIC_E_STATE, "simulation poisoned by an earlier device error");
  if (sid < 0 || sid >= (int)s->sp.size()) return fail(s, CPIC_E_ARG, "bad species id");
  Species& S = s->sp[sid];
  if (n > S.cap) return fail(s, CPIC_E_BUDGET, "particle count exceeds species capacity");
  if (n > 0 && (!cell || !off || !vel)) return fail(s, CPIC_E_ARG, "null particle array");
  const int d = s->g.dim;
  const size_t rs = real_size(s);
  hipStream_t st = s->stream;
  if (!on_device) {
    // validate on the host before touching device state
    for (size_t p = 0; p < n; ++p)
      if (cell[p] < 0 || (long long)cell[p] >= s->g.ncells) return fail(s, CPIC_E_ARG, "cell index out of range");
    for (int a = 0; a < d; ++a)
      for (size_t p = 0; p < n; ++p) {
        double v = rs == 8 ? ((const double*)off)[a * n + p] : ((const float*)off)[a * n + p];
        if (!(v >= 0.0 && v < 1.0)) return fail(s, CPIC_E_ARG, "offset outside [0, 1)");
      }
    if (rs == 4 && crowded(s, n, cell))
      return fail(s, CPIC_E_OVERFLOW, "a cell's 3^d neighbourhood holds 2^16 or more particles: its fixed-point "
                                      "deposit could exceed 64 bits");
  }
  const int buf = S.cur;
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  int32_t* lin_tmp = S.key[1 - buf];
  if (n > 0) {
    HIPCHK(s, hipMemcpyAsync(lin_tmp, cell, sizeof(int32_t) * n, kind, st));
    for (int a = 0; a < d; ++a)
      HIPCHK(s, hipMemcpyAsync(S.off[buf][a], (const char*)off + rs * n * a, rs * n, kind, st));
    for (int a = 0; a < 3; ++a)
      HIPCHK(s, hipMemcpyAsync(S.vel[buf][a], (const char*)vel + rs * n * a, rs * n, kind, st));
  }
  if (S.id[buf]) {
    if (ids && n > 0)
      HIPCHK(s, hipMemcpyAsync(S.id[buf], ids, sizeof(uint32_t) * n, kind, st));
    else
      launch_iota(S.id[buf], (int)n, st);
  }
  launch_fill_u8(s->flags, 0, sizeof(int) * 8, st);
  // new particles: their drift is unknown again, older records are not used
  launch_fill_u8(s->drift_dev + sid, 0, sizeof(unsigned), st);
  s->hist_from = s->step;
  s->overflowed = false;
  launch_lin_to_key(lin_tmp, S.key[buf], (int)n, s->g, s->flags, st);
  if (on_device)
    for (int a = 0; a < d; ++a) launch_offsets_check(S.off[buf][a], (long long)n, rs == 8, s->flags + 1, st);
  int nn = (int)n;
  HIPCHK(s, hipMemcpyAsync(S.d_n, &nn, sizeof(int), hipMemcpyHostToDevice, st));
  unsigned long long next_id = (unsigned long long)n;  // ids of injected particles start after these
  HIPCHK(s, hipMemcpyAsync(S.counters + 7, &next_id, sizeof(next_id), hipMemcpyHostToDevice, st));
  int bad[2] = {0, 0};
  HIPCHK(s, hipMemcpyAsync(bad, s->flags, sizeof(int) * 2, hipMemcpyDeviceToHost, st));
  HIPCHK(s, hipStreamSynchronize(st));
  if (bad[0] || bad[1]) {
    int zero = 0;
    HIPCHK(s, hipMemcpy(S.d_n, &zero, sizeof(int), hipMemcpyHostToDevice));
    return fail(s, CPIC_E_ARG, "device particle input has cells or offsets out of range");
  }
  s->sorted_dirty = true;
  return check_async(s);
}

extern "C" cpic_status cpic_get_particles(cpic_sim* s, int sid, size_t cap, int32_t* cell, void* off,
                                          void* vel, uint32_t* ids, size_t* n_out, int on_device) {
  if (!s || !n_out) return CPIC_E_ARG;
  if (sid < 0 || sid >= (int)s->sp.size()) return fail(s, CPIC_E_ARG, "bad species id");
  Species& S = s->sp[sid];
  hipStream_t st = s->stream;
  int n = 0;
  HIPCHK(s, hipMemcpyAsync(&n, S.d_n, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(s, hipStreamSynchronize(st));
  *n_out = (size_t)n;
  if ((size_t)n > cap) return fail(s, CPIC_E_BUDGET, "output capacity too small");
  const int d = s->g.dim;
  const size_t rs = real_size(s);
  const int buf = S.cur;
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (n > 0) {
    int32_t* lin_tmp = S.key[1 - buf];
    launch_key_to_lin(S.key[buf], lin_tmp, n, s->g, st);
    if (cell) HIPCHK(s, hipMemcpyAsync(cell, lin_tmp, sizeof(int32_t) * n, kind, st));
    if (off)
      for (int a = 0; a < d; ++a)
        HIPCHK(s, hipMemcpyAsync((char*)off + rs * n * a, S.off[buf][a], rs * n, kind, st));
    if (vel)
      for (int a = 0; a < 3; ++a)
        HIPCHK(s, hipMemcpyAsync((char*)vel + rs * n * a, S.vel[buf][a], rs * n, kind, st));
    if (ids && S.id[buf]) HIPCHK(s, hipMemcpyAsync(ids, S.id[buf], sizeof(uint32_t) * n, kind, st));
  }
  HIPCHK(s, hipStreamSynchronize(st));
  return check_async(s);
}

// ----------------------------------------------------------------------------
// stages
// ----------------------------------------------------------------------------
static void sort_species(cpic_sim* s, Species& S, bool counts_ready) {
  SortLaunch L;
  memset(&L, 0, sizeof(L));
  L.g = s->g;
  L.fp64 = s->grid.precision == CPIC_FP64;
  L.capacity = (long long)S.cap;
  L.chunk = s->chunk;
  const int a = S.cur, b = 1 - S.cur;
  L.key_in = S.key[a];
  L.key_out = S.key[b];
  for (int i = 0; i < 3; ++i) {
    L.off_in[i] = S.off[a][i];
    L.off_out[i] = S.off[b][i];
    L.vel_in[i] = S.vel[a][i];
    L.vel_out[i] = S.vel[b][i];
  }
  L.id_in = S.id[a];
  L.id_out = S.id[b];
  L.d_n = S.d_n;
  L.counts = S.counts;
  L.start = S.start;
  L.cursor = S.cursor;
  L.n_items = S.n_items;
  L.item_tile = S.item_tile;
  L.item_begin = S.item_begin;
  L.item_end = S.item_end;
  L.counts_ready = counts_ready ? 1 : 0;
  launch_tile_sort(L, s->stream);
  // the sort compacts away the particles that left: remember how many had
  (void)hipMemcpyAsync(S.dead_mark, S.counters, sizeof(unsigned long long) * NCOUNTERS, hipMemcpyDeviceToDevice,
                       s->stream);
  S.cur = b;
}

static unsigned all_species(const cpic_sim* s) { return (1u << s->sp.size()) - 1u; }

// Tile sort of the species in `mask`; counts_ready: the step's particle and
// injection kernels counted their tiles.
static void sort_species_mask(cpic_sim* s, unsigned mask, bool counts_ready) {
  for (size_t k = 0; k < s->sp.size(); ++k)
    if (mask >> k & 1u) sort_species(s, s->sp[k], counts_ready);
}

static void sort_all(cpic_sim* s) {
  sort_species_mask(s, all_species(s), false);
  for (auto& S : s->sp) {
    S.since_sort = 0;
    ++S.sorts;
  }
  s->sorted_dirty = false;
}

static void zero_deposits(cpic_sim* s, int mode) {
  if (mode == MODE_PUSH) launch_fill_u8(s->ke, 0, sizeof(double), s->stream);
  if (mode == MODE_HALFSTEP) return;
  for (auto& S : s->sp) {
    launch_fill_u8(S.Q, 0, 8 * (size_t)s->g.ncells, s->stream);
    launch_fill_u8(S.counters + 9, 0, sizeof(unsigned long long), s->stream);
    launch_fill_u8(S.fb_count, 0, sizeof(int) * 2, s->stream);
  }
}

// the particle-kernel launch of species k (count_mask: species whose new
// tiles are counted for a sort at the end of the step)
static ParticleLaunch make_launch(cpic_sim* s, size_t k, int mode, unsigned count_mask) {
  const bool halfstep = mode == MODE_HALFSTEP;
  {
    Species& S = s->sp[k];
    ParticleLaunch L;
    memset(&L, 0, sizeof(L));
    L.g = s->g;
    L.fp64 = s->grid.precision == CPIC_FP64;
    L.shape = s->grid.shape;
    L.mode = mode;
    const int b = S.cur;
    L.key = S.key[b];
    for (int a = 0; a < 3; ++a) {
      L.off[a] = S.off[b][a];
      L.vel[a] = S.vel[b][a];
      L.pbc_lo[a] = S.desc.pbc_lo[a];
      L.pbc_hi[a] = S.desc.pbc_hi[a];
      L.B[a] = s->grid.B0[a];
    }
    L.item_tile = S.item_tile;
    L.item_begin = S.item_begin;
    L.item_end = S.item_end;
    L.n_items = S.n_items;
    L.max_items = S.max_items;
    L.d_n = S.d_n;
    L.Ev = s->G.Ev;
    L.Q = S.Q;
    L.qm = S.desc.q / S.desc.m;
    L.dt = halfstep ? -0.5 * s->grid.dt : s->grid.dt;
    L.magnetic = (s->grid.B0[0] != 0 || s->grid.B0[1] != 0 || s->grid.B0[2] != 0);
    if (s->grid.pusher == CPIC_PUSH_CYCLOTRONIC && L.magnetic) {
      // exact gyration: theta = (q/m) |B| dt, b = B / |B|
      const double bn = sqrt(s->grid.B0[0] * s->grid.B0[0] + s->grid.B0[1] * s->grid.B0[1] +
                             s->grid.B0[2] * s->grid.B0[2]);
      const double th = L.qm * bn * s->grid.dt;
      L.cyclo = 1;
      for (int i = 0; i < 3; ++i) L.cyc_b[i] = s->grid.B0[i] / bn;
      L.cyc_c = cos(th);
      L.cyc_s = sin(th);
      L.cyc_s1 = fabs(th) < 1e-4 ? 1.0 - th * th / 6.0 : sin(th) / th;
      L.cyc_s2 = fabs(th) < 1e-4 ? th / 2.0 - th * th * th / 24.0 : (1.0 - cos(th)) / th;
    }
    L.vz_active = (s->g.dim == 3) || L.magnetic;
    L.S1 = s->S1;
    L.newton_maxit = 8;
    L.newton_tol = L.fp64 ? 1e-12 : 1e-5;
    L.kappa = s->kappa;
    L.fb_queue = S.fb_queue;
    L.fb_count = S.fb_count;
    L.fb_cap = (int)S.cap;
    L.ke_scale = 0.5 * S.desc.m * S.desc.w;
    L.ke = s->ke;
    L.ke_part = S.ke_part;
    L.tile_counts = ((count_mask >> k & 1u) && mode == MODE_PUSH) ? S.counts : nullptr;
    L.kc = s->kc;
    L.drift = mode == MODE_PUSH ? s->drift_dev + k : nullptr;
    L.counters = S.counters;
    return L;
  }
}

// the kinetic energy of the step: fixed-order sum of the work items' partials
static void ke_pass(cpic_sim* s) {
  {
    KeReduce r;
    memset(&r, 0, sizeof(r));
    r.nspecies = (int)s->sp.size();
    for (int k = 0; k < r.nspecies; ++k) {
      r.part[k] = s->sp[k].ke_part;
      r.n_items[k] = s->sp[k].n_items;
      // the particle kernels of the maps that allow injection run TAIL_ITEMS
      // more work items (the particles appended since the last sort)
      r.tail[k] = (s->g.kind == CPIC_MAP_IDENTITY || s->g.kind == CPIC_MAP_POLAR_LOG || s->kc) ? TAIL_ITEMS : 0;
      r.scale[k] = 0.5 * s->sp[k].desc.m * s->sp[k].desc.w;
    }
    r.out = s->ke;
    launch_ke_reduce(r, s->stream);
  }
}

// particle kernels of all species (deposit arrays must have been zeroed)
// count_mask: species whose new tiles are counted for a sort at the end of the step
static void particles_pass(cpic_sim* s, int mode, unsigned count_mask = 0) {
  for (size_t k = 0; k < s->sp.size(); ++k) launch_particles(make_launch(s, k, mode, count_mask), s->stream);
  if (mode == MODE_PUSH) ke_pass(s);
}

static bool any_injection(const cpic_sim* s) {
  for (const auto& S : s->sp)
    if (S.desc.inject) return true;
  return false;
}

// Maxwellian-flux injection of every injecting species for step `step`
static void inject_pass(cpic_sim* s, long long step, unsigned count_mask = 0) {
  for (size_t k = 0; k < s->sp.size(); ++k) {
    Species& S = s->sp[k];
    if (!S.desc.inject) continue;
    InjectLaunch I;
    memset(&I, 0, sizeof(I));
    I.g = s->g;
    I.fp64 = s->grid.precision == CPIC_FP64;
    const int b = S.cur;
    I.key = S.key[b];
    for (int a = 0; a < 3; ++a) {
      I.off[a] = S.off[b][a];
      I.vel[a] = S.vel[b][a];
    }
    I.id = S.id[b];
    I.d_n = S.d_n;
    I.cap = (int)S.cap;
    I.Q = S.Q;
    I.shape = s->grid.shape;
    I.S1 = s->S1;
    I.lam = S.inject_lam;
    I.kappa = s->kappa;
    I.vth = S.desc.inject_vth;
    I.s_drift = S.desc.inject_drift / S.desc.inject_vth;
    I.dt = s->grid.dt;
    I.k0 = (uint32_t)(S.desc.seed & 0xFFFFFFFFu);
    I.k1 = (uint32_t)(S.desc.seed >> 32);
    I.step = (uint32_t)step;
    I.species = (uint32_t)k;
    I.counters = S.counters;
    I.count_out = S.d_n + 1;
    I.tile_counts = (count_mask >> k & 1u) ? S.counts : nullptr;
    launch_inject(I, s->stream);
  }
}

static void charge_pass(cpic_sim* s) {
  ChargeSpecies cs;
  memset(&cs, 0, sizeof(cs));
  cs.n = (int)s->sp.size();
  cs.fixed = s->grid.precision == CPIC_FP32;
  const double scale = cs.fixed ? ldexp(1.0, -s->g.dim * s->S1) : 1.0;
  for (int k = 0; k < cs.n; ++k) {
    cs.Q[k] = s->sp[k].Q;
    cs.qw[k] = s->sp[k].desc.q * s->sp[k].desc.w * scale;
  }
  launch_charge(s->G, cs, 1.0, s->stream);
}

// cycles: V-cycles to launch (the solve stops on the device once converged;
// cycles launched after that return at once but still cost their launches);
// cap: the cycles the solve may use (<= 0: as many as launched)
static void solve_pass(cpic_sim* s, int cycles = -1, int cap = 0) {
  launch_rhs(s->G, s->stream);
  launch_mg_solve(s->G, s->grid.mg_rtol, cycles > 0 ? cycles : s->grid.mg_max_cycles, 2, 2, s->stream, cap);
  if (s->G.floating) {
    WallCharge wc;
    memset(&wc, 0, sizeof(wc));
    wc.nsp = (int)s->sp.size();
    for (size_t k = 0; k < s->sp.size(); ++k) {
      wc.absorbed[k] = s->sp[k].counters;  // [0]: absorbed at the lower face of axis 0
      wc.qw[k] = s->sp[k].desc.q * s->sp[k].desc.w;
    }
    launch_floating_wall(s->G, wc, s->stream);
  }
  launch_gauge(s->G, s->stream);
}

// Cycles to launch in a time step: one more than the solve of step n - 2
// needed (its record waited for, so the count is a fixed function of the
// device state, whatever the host's timing), at most the cap; the cap while
// no record is usable (last < 0).  A solve that would need more stops at the
// launched count, its relative residual in the diagnostics, and later steps
// launch more.
static int step_cycles(const cpic_sim* s, int last) {
  if (last < 0) return s->grid.mg_max_cycles;
  return std::min(s->grid.mg_max_cycles, last + 1);
}

// Species to tile-sort at the end of the coming step.  A species sorts at
// most every sort_every steps; it sorts then unless a bound on its particles'
// drift since its last sort (steps x the largest increment seen up to step
// n - 2, from its record; none: unknown) is below one cell, the slack of the
// tile windows, and at least every 16 sort_every steps.  Injecting species sort
// every sort_every steps: their appended particles, processed meanwhile by one
// extra work item through the global paths, join their tiles at a sort.
static unsigned sort_mask(const cpic_sim* s, const unsigned* drift) {
  const int K = s->grid.sort_every;
  unsigned mask = 0;
  for (size_t k = 0; k < s->sp.size(); ++k) {
    const Species& S = s->sp[k];
    const int after = S.since_sort + 1;
    bool sort = S.desc.inject != 0 && after >= K;
    if (!sort && after >= K) {
      float dmax = 0.0f;
      if (drift) memcpy(&dmax, &drift[k], sizeof(dmax));
      sort = !(dmax > 0.0f) || (float)after * dmax >= 1.0f || after >= 16 * K;
    }
    if (sort) mask |= 1u << k;
  }
  return mask;
}

static void ensure_sorted(cpic_sim* s) {
  if (s->sorted_dirty) sort_all(s);
}

extern "C" cpic_status cpic_run_stage(cpic_sim* s, int stage) {
  if (!s) return CPIC_E_ARG;
  if (s->poisoned) return fail(s, CPIC_E_STATE, "simulation poisoned by an earlier device error");
  switch (stage) {
    case CPIC_STAGE_SORT: sort_all(s); break;
    case CPIC_STAGE_DEPOSIT: ensure_sorted(s); zero_deposits(s, MODE_DEPOSIT); particles_pass(s, MODE_DEPOSIT); break;
    case CPIC_STAGE_CHARGE: charge_pass(s); break;
    case CPIC_STAGE_SOLVE: solve_pass(s); break;
    case CPIC_STAGE_EFIELD: launch_efield(s->G, s->stream); break;
    case CPIC_STAGE_INJECT: inject_pass(s, s->step); s->sorted_dirty = true; break;
    case CPIC_STAGE_PUSH: ensure_sorted(s); zero_deposits(s, MODE_PUSH); particles_pass(s, MODE_PUSH); break;
    case CPIC_STAGE_HALFSTEP: ensure_sorted(s); particles_pass(s, MODE_HALFSTEP); break;
    default: return fail(s, CPIC_E_ARG, "unknown stage");
  }
  return check_async(s);
}

extern "C" cpic_status cpic_initialize(cpic_sim* s) {
  if (!s) return CPIC_E_ARG;
  if (s->poisoned) return fail(s, CPIC_E_STATE, "simulation poisoned by an earlier device error");
  if (s->sp.empty()) return fail(s, CPIC_E_STATE, "no species");
  sort_all(s);
  zero_deposits(s, MODE_DEPOSIT);
  particles_pass(s, MODE_DEPOSIT);
  charge_pass(s);
  solve_pass(s);
  launch_efield(s->G, s->stream);
  particles_pass(s, MODE_HALFSTEP);
  s->initialized = true;
  s->step = 0;
  s->phi_prev_valid = false;
  s->hist_from = 0;
  return check_async(s);
}

static StepEvents* next_events(cpic_sim* s) {
  if (s->ev_used >= s->evs.size()) {
    StepEvents e;
    for (int i = 0; i < 5; ++i)
      if (hipEventCreate(&e.e[i]) != hipSuccess) return nullptr;
    s->evs.push_back(e);
  }
  return &s->evs[s->ev_used++];
}

// Particle phase of a step: cleared deposits (and tile counts of the species
// sorted at its end, counted by the step's particle and injection kernels, so
// that the sort needs no histogram), the particle kernels, the injection.
static void particle_phase(cpic_sim* s, StepEvents* ev, bool inj, unsigned sort_mask) {
  if (ev) hipEventRecord(ev->e[0], s->stream);
  zero_deposits(s, MODE_PUSH);
  for (size_t k = 0; k < s->sp.size(); ++k)
    if (sort_mask >> k & 1u)
      launch_fill_u8(s->sp[k].counts, 0, sizeof(int) * (size_t)(s->g.ntiles + 2), s->stream);
  if (ev) hipEventRecord(ev->e[1], s->stream);
  particles_pass(s, MODE_PUSH, sort_mask);
  if (ev) hipEventRecord(ev->e[2], s->stream);
  if (inj) inject_pass(s, s->step, sort_mask);
}

// Field phase of a step: charge, the solve's initial guess extrapolated
// linearly from the last two steps, the solve (launching `cycles`, using at
// most `cap`), the vertex field.
static void field_phase(cpic_sim* s, int cycles, int cap) {
  charge_pass(s);
  launch_extrapolate_guess(s->G, s->phi_prev_valid ? 1 : 0, s->stream);
  s->phi_prev_valid = true;
  solve_pass(s, cycles, cap);
  launch_efield(s->G, s->stream);
}

// End of a step: the tile sort of the species in sort_mask.
static void step_end(cpic_sim* s, StepEvents* ev, unsigned sort_mask) {
  if (ev) hipEventRecord(ev->e[3], s->stream);
  ++s->step;
  sort_species_mask(s, sort_mask, true);
  if (ev) hipEventRecord(ev->e[4], s->stream);
}

// The kernels of one step after ensure_sorted (asynchronous, no host reads);
// the species in sort_mask are tile-sorted at its end.
static void step_body(cpic_sim* s, StepEvents* ev, bool inj, unsigned sort_mask, int cycles) {
  particle_phase(s, ev, inj, sort_mask);
  field_phase(s, cycles, cycles);
  step_end(s, ev, sort_mask);
}

// One step as a HIP graph: every step variant (buffer parity of each species,
// sort or not, extrapolated guess or not) is recorded once by stream capture
// and replayed afterwards; the host state a replay stands for (buffer parity,
// step count) is applied here.  Returns false when capture is not possible.
static bool graph_step(cpic_sim* s, unsigned sort_mask, int cycles, StepEvents* ev) {
  uint64_t key = (s->phi_prev_valid ? 2u : 0u) | ((uint64_t)cycles << 16) | ((uint64_t)sort_mask << 32);
  for (size_t k = 0; k < s->sp.size(); ++k) key |= (uint64_t)s->sp[k].cur << (2 + k);
  if (ev) {
    hipEventRecord(ev->e[0], s->stream);
    for (int i = 1; i < 4; ++i) hipEventRecord(ev->e[i], s->stream);
  }
  for (auto& gph : s->step_graphs) {
    if (gph.key != key) continue;
    if (hipGraphLaunch(gph.exec, s->stream) != hipSuccess) return false;
    for (size_t k = 0; k < s->sp.size(); ++k) s->sp[k].cur = gph.cur_after[k];
    s->phi_prev_valid = true;
    ++s->step;
    if (ev) hipEventRecord(ev->e[4], s->stream);
    return true;
  }
  // record: the capture runs the host logic of the step (which advances the
  // host state) while the kernels go into the graph instead of the GPU
  std::vector<int> cur_before;
  for (auto& S : s->sp) cur_before.push_back(S.cur);
  const bool prev_before = s->phi_prev_valid;
  const long long step_before = s->step;
  if (hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();  // e.g. the null stream cannot be captured
    return false;
  }
  step_body(s, nullptr, false, sort_mask, cycles);
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool ok = hipStreamEndCapture(s->stream, &graph) == hipSuccess && graph &&
            hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
  if (graph) (void)hipGraphDestroy(graph);
  if (!ok || hipGraphLaunch(exec, s->stream) != hipSuccess) {
    if (exec) (void)hipGraphExecDestroy(exec);
    // nothing ran: restore the host state and let the caller step eagerly
    for (size_t k = 0; k < s->sp.size(); ++k) s->sp[k].cur = cur_before[k];
    s->phi_prev_valid = prev_before;
    s->step = step_before;
    (void)hipGetLastError();
    return false;
  }
  cpic_sim::StepGraph gph;
  gph.key = key;
  gph.exec = exec;
  for (auto& S : s->sp) gph.cur_after.push_back(S.cur);
  s->step_graphs.push_back(gph);
  if (ev) hipEventRecord(ev->e[4], s->stream);
  return true;
}

// Host decisions of the coming step from the record of step n - 2 (waited
// for): the species to sort at its end and the solver cycles to launch.
static cpic_status step_prelude(cpic_sim* s, unsigned* mask, int* cycles) {
  const long long n = s->step;
  int last = -1;
  const unsigned* drift = nullptr;
  if (n - 2 >= s->hist_from) {
    const int slot = (int)((n - 2) % HIST);
    HIPCHK(s, hipEventSynchronize(s->hist_ev[slot]));
    last = s->cycles_host[slot];
    drift = s->drift_host + 8 * slot;
  }
  *mask = sort_mask(s, drift);
  *cycles = step_cycles(s, last);
  return CPIC_OK;
}

// Host bookkeeping after a step's launches: sort counters, and the step's
// record (solver cycles, drift) copied back for step n + 2.
static cpic_status step_record(cpic_sim* s, unsigned mask, long long n) {
  for (size_t q = 0; q < s->sp.size(); ++q) {
    Species& S = s->sp[q];
    if (mask >> q & 1u) {
      S.since_sort = 0;
      ++S.sorts;
    } else {
      ++S.since_sort;
    }
  }
  const int slot = (int)(n % HIST);
  launch_step_record(s->G.mg_flag + 1, s->drift_dev, (int)s->sp.size(), s->cycles_host + slot,
                     s->drift_host + 8 * slot, s->stream);
  HIPCHK(s, hipEventRecord(s->hist_ev[slot], s->stream));
  return CPIC_OK;
}

extern "C" cpic_status cpic_step_ready(const cpic_sim* s, int* ready) {
  if (!s || !ready) return CPIC_E_ARG;
  *ready = 1;
  const long long n = s->step;
  if (n - 2 >= s->hist_from) {
    const hipError_t q = hipEventQuery(s->hist_ev[(int)((n - 2) % HIST)]);
    if (q == hipErrorNotReady)
      *ready = 0;
    else if (q != hipSuccess)
      return CPIC_E_HIP;
  }
  return CPIC_OK;
}

static cpic_status step_checks(cpic_sim* s) {
  if (s->poisoned) return fail(s, CPIC_E_STATE, "simulation poisoned by an earlier device error");
  if (!s->initialized) return fail(s, CPIC_E_STATE, "cpic_initialize has not been called");
  if (s->overflowed) return fail(s, CPIC_E_OVERFLOW, "an earlier fixed-point deposit wrapped");
  return CPIC_OK;
}

extern "C" cpic_status cpic_step(cpic_sim* s, int nsteps) {
  if (!s || nsteps < 0) return CPIC_E_ARG;
  const cpic_status chk = step_checks(s);
  if (chk != CPIC_OK) return chk;
  for (int k = 0; k < nsteps; ++k) {
    ensure_sorted(s);
    StepEvents* ev = s->timing ? next_events(s) : nullptr;
    const bool inj = any_injection(s);
    const long long n = s->step;
    unsigned mask = 0;
    int cycles = 0;
    cpic_status rc = step_prelude(s, &mask, &cycles);
    if (rc != CPIC_OK) return rc;
    // injection draws depend on the step number, a kernel argument: no graphs
    if (!(s->graphs && !inj && graph_step(s, mask, cycles, ev))) step_body(s, ev, inj, mask, cycles);
    rc = step_record(s, mask, n);
    if (rc != CPIC_OK) return rc;
  }
  return check_async(s);
}

// The field phases of simulations that share a grid shape can be batched:
// FP32 particles, flexible CG with the point smoother (not the line
// relaxation of strongly anisotropic operators), no floating wall, no
// injection, on the same stream.
static bool batchable(const cpic_sim* s) {
  return s->grid.precision == CPIC_FP32 && s->grid.mg_method == CPIC_MG_FCG && !s->G.floating &&
         s->G.anisotropy <= 50.0 && !any_injection(s) && s->G.kr != nullptr;
}
static bool same_shape(const cpic_sim* a, const cpic_sim* b) {
  if (a->g.dim != b->g.dim || a->G.nlev != b->G.nlev || a->stream != b->stream) return false;
  for (int k = 0; k < 3; ++k)
    if (a->g.n[k] != b->g.n[k] || a->G.bc_lo[k] != b->G.bc_lo[k] || a->G.bc_hi[k] != b->G.bc_hi[k]) return false;
  return a->G.restrict_transpose == b->G.restrict_transpose;
}


extern "C" cpic_status cpic_step_batch(cpic_sim* const* sims, int n, cpic_status* status) {
  if (!sims || n < 1) return CPIC_E_ARG;
  for (int i = 0; i < n; ++i) {
    if (!sims[i]) return CPIC_E_ARG;
    for (int j = 0; j < i; ++j)
      if (sims[j] == sims[i]) return fail(sims[i], CPIC_E_ARG, "a simulation appears twice in the batch");
  }
  cpic_status first = CPIC_OK;
  auto report = [&](int i, cpic_status rc) {
    if (status) status[i] = rc;
    if (first == CPIC_OK) first = rc;
  };
  // the cases that pass the checks step; the others keep their state
  std::vector<int> idx;
  for (int i = 0; i < n; ++i) {
    const cpic_status rc = step_checks(sims[i]);
    if (status) status[i] = rc;
    if (rc != CPIC_OK)
      report(i, rc);
    else
      idx.push_back(i);
  }
  const int m = (int)idx.size();
  bool batch = m > 1;
  for (int i = 0; i < m && batch; ++i) batch = batchable(sims[idx[i]]) && same_shape(sims[idx[i]], sims[idx[0]]);
  if (!batch) {
    for (int i : idx) {
      const cpic_status rc = cpic_step(sims[i], 1);
      if (rc != CPIC_OK) report(i, rc);
    }
    return first;
  }
  std::vector<cpic_sim*> S((size_t)m);
  for (int i = 0; i < m; ++i) S[i] = sims[idx[i]];
  // a failure past this point (a runtime error) is reported for every case of the batch
  auto fail_all = [&](cpic_status rc) {
    for (int i : idx) report(i, rc);
    return first;
  };
  std::vector<unsigned> mask((size_t)m);
  std::vector<int> cycles((size_t)m);
  std::vector<long long> step0((size_t)m);
  std::vector<StepEvents*> ev((size_t)m);
  int launch = 0;
  for (int i = 0; i < m; ++i) {
    ensure_sorted(S[i]);
    ev[i] = S[i]->timing ? next_events(S[i]) : nullptr;
    step0[i] = S[i]->step;
    const cpic_status rc = step_prelude(S[i], &mask[i], &cycles[i]);
    if (rc != CPIC_OK) return fail_all(rc);
    launch = std::max(launch, cycles[i]);
  }
  // particle phases: the deposit clears of every case in one launch, then
  // the particle kernels of every case and species as one launch (plus one
  // for the FP64 fallback), when they share a kernel
  {
    std::vector<FillRange> zr;
    for (int i = 0; i < m; ++i) {
      cpic_sim* s = S[i];
      if (ev[i]) hipEventRecord(ev[i]->e[0], s->stream);
      zr.push_back({s->ke, sizeof(double)});
      for (size_t k = 0; k < s->sp.size(); ++k) {
        Species& P = s->sp[k];
        zr.push_back({P.Q, 8 * (size_t)s->g.ncells});
        zr.push_back({P.counters + 9, sizeof(unsigned long long)});
        zr.push_back({P.fb_count, sizeof(int) * 2});
        if (mask[i] >> k & 1u) zr.push_back({P.counts, sizeof(int) * (size_t)(s->g.ntiles + 2)});
      }
    }
    launch_zero_ranges(zr.data(), (int)zr.size(), S[0]->stream);
    std::vector<ParticleLaunch> pl;
    for (int i = 0; i < m; ++i) {
      if (ev[i]) hipEventRecord(ev[i]->e[1], S[i]->stream);
      for (size_t k = 0; k < S[i]->sp.size(); ++k) pl.push_back(make_launch(S[i], k, MODE_PUSH, mask[i]));
    }
    const int pr = launch_particles_batch(pl.data(), (int)pl.size(), S[0]->batch_pargs, S[0]->stream);
    if (pr == -3) {
      for (int i = 0; i < m; ++i) S[i]->poisoned = true;
      return fail_all(fail(S[0], CPIC_E_HIP, "batched particle kernels: runtime error"));
    }
    if (pr != 0)
      for (const ParticleLaunch& L : pl) launch_particles(L, S[0]->stream);
    for (int i = 0; i < m; ++i) {
      ke_pass(S[i]);
      if (ev[i]) hipEventRecord(ev[i]->e[2], S[i]->stream);
    }
  }
  // the field phases: recorded case by case, replayed as one launch per kernel
  std::vector<BatchRecorder> recs((size_t)m);
  std::vector<BatchRecorder*> rp((size_t)m);
  std::vector<int> prev((size_t)m);
  for (int i = 0; i < m; ++i) {
    prev[i] = S[i]->phi_prev_valid ? 1 : 0;
    g_batch_rec = &recs[i];
    field_phase(S[i], launch, cycles[i]);
    g_batch_rec = nullptr;
    rp[i] = &recs[i];
  }
  S[0]->batch_args.graphs_on = S[0]->graphs;
  const int rr = replay_batch(rp.data(), m, S[0]->batch_args, S[0]->stream);
  if (rr == -3) {
    for (int i = 0; i < m; ++i) S[i]->poisoned = true;
    return fail_all(fail(S[0], CPIC_E_HIP, "batched field phase: runtime error"));
  }
  if (rr != 0) {
    // the cases recorded different sequences, or no memory for the batch's
    // arguments: their field phases one by one
    for (int i = 0; i < m; ++i) {
      S[i]->phi_prev_valid = prev[i] != 0;
      field_phase(S[i], cycles[i], cycles[i]);
    }
  } else {
    for (int i = 0; i < m; ++i) ++S[i]->batched_steps;
  }
  for (int i = 0; i < m; ++i) {
    step_end(S[i], ev[i], mask[i]);
    const cpic_status rc = step_record(S[i], mask[i], step0[i]);
    if (rc != CPIC_OK) return fail_all(rc);
  }
  for (int i = 0; i < m; ++i) {
    const cpic_status rc = check_async(S[i]);
    if (rc != CPIC_OK) return fail_all(rc);
  }
  return first;
}

extern "C" cpic_status cpic_set_stream(cpic_sim* s, void* hip_stream) {
  if (!s) return CPIC_E_ARG;
  // work already queued finishes first: everything after runs on the new stream
  HIPCHK(s, hipStreamSynchronize(s->stream));
  s->stream = (hipStream_t)hip_stream;
  return CPIC_OK;
}

extern "C" cpic_status cpic_batch_signature(const cpic_sim* s, uint64_t* sig) {
  if (!s || !sig) return CPIC_E_ARG;
  *sig = 0;
  if (!batchable(s)) return CPIC_OK;
  // what same_shape compares, hashed (FNV-1a); never 0
  int words[16] = {s->g.dim, s->G.nlev, s->G.restrict_transpose};
  int k = 3;
  for (int a = 0; a < 3; ++a) {
    words[k++] = s->g.n[a];
    words[k++] = s->G.bc_lo[a];
    words[k++] = s->G.bc_hi[a];
  }
  uint64_t h = 1469598103934665603ull;
  const unsigned char* b = (const unsigned char*)words;
  for (size_t i = 0; i < sizeof(int) * (size_t)k; ++i) h = (h ^ b[i]) * 1099511628211ull;
  *sig = h | 1u;
  return CPIC_OK;
}

extern "C" cpic_status cpic_set_graphs(cpic_sim* s, int enable) {
  if (!s) return CPIC_E_ARG;
  s->graphs = enable != 0;
  return CPIC_OK;
}

// ----------------------------------------------------------------------------
// fields and diagnostics
// ----------------------------------------------------------------------------
extern "C" size_t cpic_field_bytes(const cpic_sim* s, int which) {
  if (!s) return 0;
  const size_t nc = (size_t)s->g.ncells;
  switch (which) {
    case CPIC_FIELD_Q: return 8 * nc;
    case CPIC_FIELD_CHARGE:
    case CPIC_FIELD_PHI:
    case CPIC_FIELD_JC:
    case CPIC_FIELD_RHO: return 8 * nc;
    case CPIC_FIELD_BACKGROUND: return s->G.background ? 8 * nc : 0;
    case CPIC_FIELD_EV: return real_size(s) * ecomp(s) * (size_t)s->g.nverts;
    default: return 0;
  }
}

static void* field_ptr(cpic_sim* s, int which, int sid) {
  switch (which) {
    case CPIC_FIELD_Q: return (sid >= 0 && sid < (int)s->sp.size()) ? s->sp[sid].Q : nullptr;
    case CPIC_FIELD_CHARGE: return s->G.charge;
    case CPIC_FIELD_PHI: return s->G.floating ? s->G.phi_full : s->G.lev[0].phi;
    case CPIC_FIELD_JC: return s->G.Jc;
    case CPIC_FIELD_RHO: return s->G.lev[0].phi2;
    case CPIC_FIELD_BACKGROUND: return s->G.background;
    case CPIC_FIELD_EV: return s->G.Ev;
    default: return nullptr;
  }
}

extern "C" cpic_status cpic_get_field(cpic_sim* s, int which, int sid, void* dst, size_t bytes, int on_device) {
  if (!s || !dst) return CPIC_E_ARG;
  size_t need = cpic_field_bytes(s, which);
  void* src = field_ptr(s, which, sid);
  if (!src || need == 0) return fail(s, CPIC_E_ARG, "unknown field / species");
  if (bytes != need) return fail(s, CPIC_E_ARG, "field size mismatch");
  if (which == CPIC_FIELD_RHO) launch_rho(s->G, s->G.lev[0].phi2, s->stream);
  HIPCHK(s, hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return check_async(s);
}

extern "C" cpic_status cpic_set_field(cpic_sim* s, int which, int sid, const void* src, size_t bytes,
                                      int on_device) {
  if (!s || !src) return CPIC_E_ARG;
  if (s->poisoned) return fail(s, CPIC_E_STATE, "simulation poisoned by an earlier device error");
  if (which != CPIC_FIELD_Q && which != CPIC_FIELD_CHARGE && which != CPIC_FIELD_PHI && which != CPIC_FIELD_EV)
    return fail(s, CPIC_E_ARG, "field is read-only");
  if (which == CPIC_FIELD_PHI && s->G.floating)
    return fail(s, CPIC_E_UNSUPPORTED, "the potential of a floating-wall problem follows from its solve");
  size_t need = cpic_field_bytes(s, which);
  void* dst = field_ptr(s, which, sid);
  if (!dst || need == 0) return fail(s, CPIC_E_ARG, "unknown field / species");
  if (bytes != need) return fail(s, CPIC_E_ARG, "field size mismatch");
  if (!on_device && which != CPIC_FIELD_Q) {
    // floating-point fields from the host must be finite
    const bool f32 = which == CPIC_FIELD_EV && real_size(s) == 4;
    const size_t cnt = bytes / (f32 ? 4 : 8);
    for (size_t i = 0; i < cnt; ++i)
      if (!(f32 ? isfinite(((const float*)src)[i]) : isfinite(((const double*)src)[i])))
        return fail(s, CPIC_E_NONFINITE, "field value is not finite");
  }
  HIPCHK(s, hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  // a potential set from outside starts a new time history
  if (which == CPIC_FIELD_PHI) s->phi_prev_valid = false;
  if (which == CPIC_FIELD_PHI || which == CPIC_FIELD_CHARGE) s->hist_from = s->step;
  return check_async(s);
}

// Device buffers the diagnostics' reductions work in.
struct DiagScratch {
  double* partials;  // REDUCE_BLOCKS doubles: per-workgroup sums of the field energy
  double* we;        // the field-energy sum
  int* nonfinite;    // count of non-finite field values (cleared by a kernel first)
  uint64_t* qsum;    // MAX_SPECIES x QSUM_WORDS words: exact charge totals and their partials
};

// Non-finite values in the potential, the charge or the vertex field, counted
// into *bad (asynchronous; read after a synchronisation).
static void launch_field_checks(cpic_sim* s, int* bad) {
  hipStream_t st = s->stream;
  launch_fill_u8(bad, 0, sizeof(int), st);
  const long long nc = s->g.ncells;
  launch_nonfinite_check(field_ptr(s, CPIC_FIELD_PHI, 0), nc, 1, bad, st);
  launch_nonfinite_check(s->G.charge, nc, 1, bad, st);
  launch_nonfinite_check(s->G.Ev, (long long)ecomp(s) * s->g.nverts, s->grid.precision == CPIC_FP64 ? 1 : 0, bad,
                         st);
}

// The fixed-point deposit of a species wrapped when its exact total differs
// from (particles deposited since Q was cleared) x 2^{d S1}: every particle
// adds exactly 2^{d S1} over its target cells (walls fold, they do not drop),
// so a cell whose uint64 sum passed 2^64 leaves the total short.
static bool deposit_wrapped(const cpic_sim* s, uint64_t lo, uint64_t hi, unsigned long long deposited) {
  const int sh = s->g.dim * s->S1;  // 48
  const uint64_t elo = (uint64_t)deposited << sh;
  const uint64_t ehi = sh ? (uint64_t)deposited >> (64 - sh) : 0;
  return lo != elo || hi != ehi;
}

// Diagnostics and state checks with the reductions in `sc`; host staging in
// fixed-size arrays, one synchronisation.
static cpic_status diag_impl(cpic_sim* s, cpic_diag* out, const DiagScratch& sc) {
  memset(out, 0, sizeof(*out));
  hipStream_t st = s->stream;
  out->step = s->step;
  out->nspecies = (int)s->sp.size();
  out->step_graphs = (int)s->step_graphs.size();
  out->batched_steps = s->batched_steps;
  const int nsp = (int)s->sp.size();
  double ke = 0.0, we = 0.0, sc2[2] = {0, 0}, wall[2] = {0, 0};
  int fl[2] = {0, 0}, nonfinite = 0;
  unsigned long long cnt[MAX_SPECIES][NCOUNTERS], mark[MAX_SPECIES][NCOUNTERS];
  int ns[MAX_SPECIES] = {0};
  uint64_t qs[MAX_SPECIES][2] = {{0, 0}};
  HIPCHK(s, hipMemcpyAsync(&ke, s->ke, sizeof(double), hipMemcpyDeviceToHost, st));
  launch_field_energy(s->G, sc.partials, sc.we, st);
  launch_field_checks(s, sc.nonfinite);
  const bool fixed = s->grid.precision == CPIC_FP32;
  for (int k = 0; k < nsp; ++k)
    if (fixed) launch_qsum((const uint64_t*)s->sp[k].Q, s->g.ncells, sc.qsum + (size_t)k * QSUM_WORDS, st);
  HIPCHK(s, hipMemcpyAsync(&we, sc.we, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(s, hipMemcpyAsync(sc2, s->G.scalars, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
  if (s->G.floating) HIPCHK(s, hipMemcpyAsync(wall, s->G.scalars + 10, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
  HIPCHK(s, hipMemcpyAsync(fl, s->G.mg_flag, sizeof(int) * 2, hipMemcpyDeviceToHost, st));
  HIPCHK(s, hipMemcpyAsync(&nonfinite, sc.nonfinite, sizeof(int), hipMemcpyDeviceToHost, st));
  for (int k = 0; k < nsp; ++k) {
    Species& S = s->sp[k];
    HIPCHK(s, hipMemcpyAsync(cnt[k], S.counters, sizeof(unsigned long long) * NCOUNTERS, hipMemcpyDeviceToHost, st));
    HIPCHK(s, hipMemcpyAsync(mark[k], S.dead_mark, sizeof(unsigned long long) * NCOUNTERS, hipMemcpyDeviceToHost, st));
    HIPCHK(s, hipMemcpyAsync(&ns[k], S.d_n, sizeof(int), hipMemcpyDeviceToHost, st));
    if (fixed)
      HIPCHK(s, hipMemcpyAsync(qs[k], sc.qsum + (size_t)k * QSUM_WORDS, sizeof(uint64_t) * 2, hipMemcpyDeviceToHost,
                               st));
  }
  HIPCHK(s, hipStreamSynchronize(st));
  out->kinetic = ke;
  // with a floating wall, the energy of its charge 1/2 Q_w phi_w is included
  out->field_energy = 0.5 * we + 0.5 * wall[1] * wall[0];
  out->phi_wall = wall[0];
  out->wall_charge = wall[1];
  out->mg_relres = sc2[0] > 0 ? sqrt(sc2[1] / sc2[0]) : 0.0;
  out->mg_cycles = fl[1];
  bool wrapped = false;
  for (int k = 0; k < nsp; ++k) {
    const unsigned long long* c = cnt[k];
    const unsigned long long* m = mark[k];
    // slots in use less the particles that left since the last sort (absorbed,
    // outflow, injected ones whose entry flight left at once)
    out->count[k] = ns[k] - (long long)((c[0] + c[1] + c[8]) - (m[0] + m[1] + m[8]));
    out->absorbed[k] = (long long)c[0];
    out->outflow[k] = (long long)c[1];
    out->newton_fallback += (long long)c[2];
    out->far_deposits += (long long)c[3];
    out->newton_failed += (long long)c[4];
    out->injected[k] = (long long)c[5];
    out->inject_lost[k] = (long long)c[8];
    out->sorts[k] = s->sp[k].sorts;
    out->qsum_lo[k] = qs[k][0];
    out->qsum_hi[k] = qs[k][1];
    if (fixed && deposit_wrapped(s, qs[k][0], qs[k][1], c[9])) wrapped = true;
  }
  cpic_status rc = check_async(s);
  if (rc != CPIC_OK) return rc;
  if (wrapped) {
    s->overflowed = true;
    return fail(s, CPIC_E_OVERFLOW, "a cell's fixed-point deposit passed 2^64 (too many particles in one place)");
  }
  if (nonfinite) return fail(s, CPIC_E_NONFINITE, "the potential, charge or vertex field holds non-finite values");
  return CPIC_OK;
}

extern "C" cpic_status cpic_get_diag(cpic_sim* s, cpic_diag* out) {
  if (!s || !out) return CPIC_E_ARG;
  const DiagScratch sc = {s->G.partials, s->tmp_scalar, s->flags + 3, s->qsum};
  return diag_impl(s, out, sc);
}

extern "C" cpic_status cpic_get_diag_noalloc(cpic_sim* s, cpic_diag* out) {
  if (!s || !out) return CPIC_E_ARG;
  if ((int)s->sp.size() > SCR_SPECIES) return fail(s, CPIC_E_BUDGET, "more species than the diagnostics scratch holds");
  unsigned char* base = (unsigned char*)scratch_on(s->device);
  if (!base) return fail(s, CPIC_E_HIP, "address of the diagnostics scratch on this device not available");
  const DiagScratch sc = {(double*)(base + SCR_PARTIALS), (double*)(base + SCR_WE), (int*)(base + SCR_NONFINITE),
                          (uint64_t*)(base + SCR_QSUM)};
  return diag_impl(s, out, sc);
}

extern "C" cpic_status cpic_sync(cpic_sim* s) {
  if (!s) return CPIC_E_ARG;
  HIPCHK(s, hipStreamSynchronize(s->stream));
  cpic_status rc = check_async(s);
  if (rc != CPIC_OK) return rc;
  // the checks of cpic_get_diag: deposit headroom, non-finite fields
  cpic_diag d;
  return cpic_get_diag(s, &d);
}

extern "C" cpic_status cpic_set_timing(cpic_sim* s, int enable) {
  if (!s) return CPIC_E_ARG;
  s->timing = enable != 0;
  s->ev_used = 0;
  return CPIC_OK;
}

extern "C" cpic_status cpic_get_timing(cpic_sim* s, int cap, double* push_ms, double* solve_ms,
                                       double* sort_ms, double* step_ms, int* samples) {
  if (!s || cap < 0) return CPIC_E_ARG;
  HIPCHK(s, hipStreamSynchronize(s->stream));
  const size_t n = std::min(s->ev_used, (size_t)cap);
  if (samples) *samples = (int)s->ev_used;
  for (size_t i = 0; i < n; ++i) {
    float t[3] = {0, 0, 0}, tot = 0;
    for (int k = 0; k < 3; ++k)
      HIPCHK(s, hipEventElapsedTime(&t[k], s->evs[i].e[k + 1], s->evs[i].e[k + 2]));
    HIPCHK(s, hipEventElapsedTime(&tot, s->evs[i].e[0], s->evs[i].e[4]));
    if (push_ms) push_ms[i] = t[0];
    if (solve_ms) solve_ms[i] = t[1];
    if (sort_ms) sort_ms[i] = t[2];
    if (step_ms) step_ms[i] = tot;
  }
  return CPIC_OK;
}

extern "C" const char* cpic_status_str(cpic_status st) {
  switch (st) {
    case CPIC_OK: return "ok";
    case CPIC_E_ARG: return "invalid argument";
    case CPIC_E_MAP: return "map not invertible on the domain";
    case CPIC_E_NOMEM: return "out of memory";
    case CPIC_E_BUDGET: return "capacity exceeded";
    case CPIC_E_HIP: return "HIP runtime error";
    case CPIC_E_OVERFLOW: return "fixed-point headroom exceeded";
    case CPIC_E_NONFINITE: return "non-finite value";
    case CPIC_E_STATE: return "call out of order";
    case CPIC_E_UNSUPPORTED: return "unsupported combination";
    case CPIC_E_PENDING: return "pending";
  }
  return "unknown status";
}

extern "C" const char* cpic_last_error(const cpic_sim* s) { return s ? s->err.c_str() : "no simulation"; }

extern "C" void cpic_destroy(cpic_sim* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  for (auto& gph : s->step_graphs) (void)hipGraphExecDestroy(gph.exec);
  if (s->cycles_host) (void)hipHostFree(s->cycles_host);
  if (s->drift_host) (void)hipHostFree(s->drift_host);
  for (int i = 0; i < HIST; ++i)
    if (s->hist_ev[i]) (void)hipEventDestroy(s->hist_ev[i]);
  free_batch_args(s->batch_args);
  free_batch_args(s->batch_pargs);
  for (auto& e : s->evs)
    for (int i = 0; i < 5; ++i) (void)hipEventDestroy(e.e[i]);
  sim_free_all(s);
  delete s;
}
