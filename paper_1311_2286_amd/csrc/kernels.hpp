// kernels.hpp -- launch descriptors and launchers shared by the kernel files
// and the host core (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "common.hpp"

namespace cpic {

struct ParticleLaunch {
  Geo g;
  int fp64;
  int shape;
  int mode;
  int32_t* key;
  void* off[3];
  void* vel[3];
  const int* item_tile;
  const int* item_begin;
  const int* item_end;
  const int* n_items;
  int max_items;
  const int* d_n;   // live count, appended (injected) particles included
  const void* Ev;
  void* Q;
  int pbc_lo[3], pbc_hi[3];
  double qm, dt;
  double B[3];
  int magnetic, vz_active;
  // cyclotronic velocity step (PUSH): b = B/|B| and, with theta = qm |B| dt,
  // cos, sin, sin(theta)/theta and (1 - cos(theta))/theta
  int cyclo;
  double cyc_b[3], cyc_c, cyc_s, cyc_s1, cyc_s2;
  int S1;
  int newton_maxit;
  double newton_tol;
  double kappa;
  int* fb_queue;  // FP64 fallback queue (capacity = species capacity)
  int* fb_count;  // zeroed before each push
  int fb_cap;
  double ke_scale;
  double* ke;
  double* ke_part;  // [max_items] per-item kinetic energy sums (PUSH)
  int* tile_counts; // when set: per-tile counts of the new positions for the next sort
  const void* kc;   // when set: predictor-corrector mover with this vertex table (R, D x D per vertex)
  unsigned* drift;  // PUSH: running maximum of the particles' increments (cells, FP32 bits)
  unsigned long long* counters;
};

// work items of the particles appended (injected) since a species' last sort:
// the kernels of maps that allow injection split them over this many items
constexpr int TAIL_ITEMS = 64;

struct KeReduce {
  int nspecies;
  const double* part[8];
  const int* n_items[8];
  int tail[8];  // the per-item sums hold this many more slots: the appended particles' items
  double scale[8];
  double* out;
};

struct SortLaunch {
  Geo g;
  int fp64;
  long long capacity;
  int chunk;
  const int32_t* key_in;
  int32_t* key_out;
  const void* off_in[3];
  void* off_out[3];
  const void* vel_in[3];
  void* vel_out[3];
  const uint32_t* id_in;
  uint32_t* id_out;
  int* d_n;
  int* counts;  // ntiles + 2
  int counts_ready;  // counts already made by the step's kernels (else a histogram pass)
  int* start;   // ntiles + 2
  int* cursor;  // ntiles + 2
  int* n_items;
  int* item_tile;
  int* item_begin;
  int* item_end;
};

struct InjectLaunch {
  Geo g;
  int fp64;
  int32_t* key;
  void* off[3];
  void* vel[3];
  uint32_t* id;
  int* d_n;
  int cap;
  void* Q;
  int shape;
  int S1;
  double lam, vth, dt, kappa;
  double s_drift;  // inward drift of the injected Maxwellian in thermal speeds
  uint32_t k0, k1, step, species;
  unsigned long long* counters;
  int* count_out;
  int* tile_counts;
};

int launch_particles(const ParticleLaunch& L, hipStream_t st);
void launch_kc_table(const Geo& g, const double* Kv, void* kc, int fp64, hipStream_t st);
void launch_ke_reduce(const KeReduce& r, hipStream_t st);
int launch_inject(const InjectLaunch& I, hipStream_t st);
int launch_tile_sort(const SortLaunch& S, hipStream_t st);
void launch_lin_to_key(const int32_t* lin, int32_t* key, int n, const Geo& g, int* bad, hipStream_t st);
void launch_key_to_lin(const int32_t* key, int32_t* lin, int n, const Geo& g, hipStream_t st);
void launch_iota(uint32_t* id, int n, hipStream_t st);
void launch_offsets_check(const void* o, long long n, int fp64, int* bad, hipStream_t st);
void launch_fill_u8(void* p, unsigned char v, size_t bytes, hipStream_t st);
// zeroes n ranges of 4-byte-aligned memory (sizes multiples of 4) in as few
// launches as possible (32 ranges per launch)
struct FillRange {
  void* p;
  size_t bytes;
};
void launch_zero_ranges(const FillRange* r, int n, hipStream_t st);
// copies the step's record (cycles_dev[0], drift_dev[0 .. nsp)) into pinned
// host memory
void launch_step_record(const int* cycles_dev, const unsigned* drift_dev, int nsp, int* cycles_host,
                        unsigned* drift_host, hipStream_t st);

// ---------------------------------------------------------------- grid side
// One multigrid level: cell-centred grid, coefficient arrays (FP64).
struct Level {
  int n[3];
  long long ncells;
  double h[3];
  double dV;
  double* wf[3];     // upper-face coefficient of each cell, a^{aa} dV / h_a^2
  double* wlo[3];    // lower wall-face coefficient (bounded axes, cells at i_a = 0)
  double* we[3];     // mixed-term coefficient at the upper corner edge, pairs (01, 02, 12)
  // explicit operator, upper half of the symmetric stencil: S[k][c] couples c
  // and c + o_k, o = (+x, +y, +z, +x+y, +x-y, +x+z, +x-z, +y+z, +y-z)
  double* S[9];
  double* diag;
  double* phi;
  double* phi2;      // ping-pong
  double* rhs;
  double* res;
  double* aux;       // Chebyshev direction; coarsest-level solver vector
  double lam_max;    // upper bound of the spectrum of D^-1 A (host)
  // FP32 copy of the operator and the V-cycle vectors, for the preconditioner
  // of the flexible-CG solve (null with plain V-cycles); on level 0, f_phi is
  // the preconditioned residual z and f_rhs the FP32 copy of the residual
  float* f_S[9];
  float* f_diag;
  float* f_phi;
  float* f_phi2;
  float* f_rhs;
  float* f_res;
  float* f_aux;
  // FP16 copy of the operator scaled by 2^-e (largest magnitude at most 1),
  // h_inv = 2^e: the preconditioner's smoothing and residual on the levels of
  // more than a few hundred cells, where they are bound by memory traffic
  // (null elsewhere)
  unsigned short* h_S[9];
  unsigned short* h_diag;
  float h_inv;
  // variational coarse operator (levels >= 1 of CPIC_MG_BOXMG, 2D): 25
  // coefficients per cell, offset-major, FP64 and its FP32 copy
  double* gal64;
  float* gal32;
};

struct GridCtx {
  Geo g;
  int nlev;
  Level lev[16];
  int bc_lo[3], bc_hi[3];
  double phi_lo[3], phi_hi[3];
  int mixed;          // the map has non-zero mixed metric terms
  int all_periodic;
  double* bdir;       // wall contribution to the operator (level 0)
  double* Jc;         // physical J at cell centres (level 0)
  double sumJ;        // host copy
  double* charge;
  double* background;
  double* partials;   // reduction scratch (>= 1024 doubles)
  double* mg_partials; // per-block residual sums of the level-0 sweep grid
  double* scalars;    // device scalars: [0] |b|^2 [1] |r|^2 [2] sumJphi [3] mean [4..] misc
  int* mg_flag;       // [0] converged [1] cycles done
  void* Ev;           // vertex field (float or double, interleaved)
  double* Kv;         // inverse Jacobian at vertices, d x d row-major (FP64)
  double* phi_prev;   // level-0 potential of the previous step
  // flexible conjugate gradients around the V-cycle (null when plain V-cycles)
  // floating conducting wall at the lower face of axis 0 (the operator sees it
  // as a Dirichlet wall at 0; the potential is phi_0 + phi_w phi_1)
  int floating;
  double* phi1;       // charge-free potential of the wall at 1, every other wall at 0
  double* bdir1;      // its wall term
  void* E1;           // its vertex field (particle precision)
  double* phi_full;   // phi_0 + phi_w phi_1 (the potential); scalars [10] phi_w [11] Q_w [12] F(phi_1)
  double anisotropy;      // largest ratio of a level-0 cell's face coefficients
  int restrict_transpose; // restriction = transpose of the prolongation (else summing)
  int boxmg;              // preconditioner: variational coarse operators + zebra line relaxation (2D)
  int coarse;             // the solver's coarsest level (nlev - 1; with boxmg the first of <= DENSE_MAX cells)
  double* cinv64;     // dense inverse of the coarsest operator (<= DENSE_MAX cells), or null
  float* cinv32;      // its FP32 copy (flexible-CG preconditioner)
  double* kr;         // residual b - A x
  double* kp;         // search direction
  double* kq;         // A p
  double* kw;         // A z
  double* k_partials; // 3 x level-0 sweep blocks
  int fp64;
};

void launch_coefficients(const GridCtx& G, int level, hipStream_t st);
void launch_jacobian_centres(const GridCtx& G, hipStream_t st);
void launch_background(const GridCtx& G, int shape, double n0, hipStream_t st);
struct ChargeSpecies {
  int n;
  const void* Q[8];
  double qw[8];  // q_s w_s (times 2^-d S1 for integer deposits)
  int fixed;
};
void launch_charge(const GridCtx& G, const ChargeSpecies& cs, double bg_charge, hipStream_t st);
void launch_rhs(const GridCtx& G, hipStream_t st);
// cap: the cycles this solve may use (<= 0: max_cycles); a solve launched with
// more cycles than its cap stops at the cap on the device
int launch_mg_solve(const GridCtx& G, double rtol, int max_cycles, int nu1, int nu2, hipStream_t st, int cap = 0);
int compute_smoother_bounds(GridCtx& G, hipStream_t st);
// FP32 (and, where allocated, scaled FP16) copies of every level's operator;
// waits for the stream; -1 on a HIP error
int launch_operator_f32(GridCtx& G, hipStream_t st);
int setup_coarse_inverse(GridCtx& G, hipStream_t st);
int setup_floating_wall(GridCtx& G, hipStream_t st);
// coarse operators P^T A P of the CPIC_MG_BOXMG hierarchy (set-up, before the coarse inverse)
int setup_galerkin(GridCtx& G, hipStream_t st);
// charge of a floating wall: sum over species of q w (particles it absorbed)
struct WallCharge {
  int nsp;
  const unsigned long long* absorbed[8];
  double qw[8];
};
void launch_floating_wall(const GridCtx& G, const WallCharge& wc, hipStream_t st);
// levels of at most this many cells are smoothed inside one workgroup (the
// V-cycle's tail kernel)
constexpr int SMALL_CELLS = 512;
constexpr int DENSE_MAX = 640;  // coarsest levels up to this many cells are solved by a dense inverse
// operators more anisotropic than this (face-coefficient ratio within a cell)
// use the transpose of the prolongation as restriction
constexpr double ANISO_TRANSPOSE = 4.0;
void launch_extrapolate_guess(const GridCtx& G, int extrapolate, hipStream_t st);
void launch_gauge(const GridCtx& G, hipStream_t st);
void launch_vertex_metric(const GridCtx& G, hipStream_t st);
void launch_map_table(const Geo& g, double* jtab, hipStream_t st);
void launch_efield(const GridCtx& G, hipStream_t st);
void launch_rho(const GridCtx& G, double* rho, hipStream_t st);
// deterministic reductions use a fixed grid of REDUCE_BLOCKS workgroups
constexpr int REDUCE_BLOCKS = 256;
// sum_c charge_c phi_c into *out; partials: REDUCE_BLOCKS doubles of scratch
void launch_field_energy(const GridCtx& G, double* partials, double* out, hipStream_t st);
// exact 128-bit sum of Q[0..n) into out2[0] (low word), out2[1] (high word);
// out2 holds QSUM_WORDS words (the per-workgroup partials follow the result)
constexpr int QSUM_WORDS = 2 + 2 * REDUCE_BLOCKS;
void launch_qsum(const uint64_t* Q, long long n, uint64_t* out2, hipStream_t st);
// adds the number of non-finite entries of x (double when fp64, else float) to *bad
void launch_nonfinite_check(const void* x, long long n, int fp64, int* bad, hipStream_t st);

// ---------------------------------------------------------------------------
// Batched field phase (serving).  Every launch of the field phase (charge,
// extrapolated guess, right side, the flexible-CG solve with its FP32 V-cycle,
// gauge, vertex field) goes through one launcher per kernel.  Without a
// recorder it launches at once.  With the calling thread's recorder set, it
// records the kernel's kind, grid, block and argument struct instead.
// Simulations of the same grid shape record the same sequence, in which the
// arguments differ (pointers, per-case scalars); replay_batch() then runs each
// record as ONE launch over all of them: the grid's z extent times the number
// of cases, the case index in blockIdx.z / z, every case's argument struct
// read from one device buffer.  Each case computes exactly what its own launch
// would: its kernels see their own block coordinates.
// ---------------------------------------------------------------------------
struct BatchRec {
  int kind;
  dim3 grid, block;
  std::vector<unsigned char> args;
};
struct BatchRecorder {
  std::vector<BatchRec> recs;
  bool unsupported = false;  // a launch without a batched form was attempted while recording
};
extern thread_local BatchRecorder* g_batch_rec;
// records a launch that has no batched form (the batch falls back to per-case steps)
inline bool batch_unsupported() {
  if (!g_batch_rec) return false;
  g_batch_rec->unsupported = true;
  return true;
}
// Device buffer of one batch's argument structs, with the host copy they are
// assembled in, the last uploaded contents, and two pinned upload buffers used
// in turn (each reused only after the event recorded behind its last copy).
struct BatchArgs {
  // device allocation of the buffer (the owning simulation's allocator)
  void* (*dev_alloc)(size_t bytes, void* ctx) = nullptr;
  void (*dev_free)(void* p, void* ctx) = nullptr;
  void* ctx = nullptr;
  void* dev = nullptr;
  size_t bytes = 0;
  std::vector<unsigned char> staging, uploaded;
  void* pinned[2] = {nullptr, nullptr};
  void* pinned_dev[2] = {nullptr, nullptr};  // their addresses for kernels
  hipEvent_t copied[2] = {nullptr, nullptr};
  size_t pinned_bytes = 0;
  int slot = 0;
  // replayed sequences captured as HIP graphs (keyed by the sequence's kernels
  // and grids, the case count and the buffer), when graphs_on
  bool graphs_on = false;
  std::vector<std::pair<uint64_t, hipGraphExec_t>> graphs;
};
// Replays the recorded sequences of n cases as batched launches on st.
// Returns 0; -1 (nothing launched) when the sequences differ or a case
// recorded an unsupported launch; -2 (nothing launched) when the argument
// buffers could not be allocated; -3 on a runtime error.
int replay_batch(BatchRecorder* const* cases, int n, BatchArgs& ba, hipStream_t st);
// Brings ba.staging to ba.dev (stream-ordered; grows the buffers, uploads only
// when the contents changed).  0; -2 allocation failed (nothing queued); -3
// runtime error.
int batch_upload(BatchArgs& ba, hipStream_t st);
// The particle kernels of n launches of one kind (the same template: precision,
// dimension, map, mover, shape, pusher, mode) as one launch over all their
// work items, then one fallback launch: 0; -1 the launches differ (nothing
// queued); -2 / -3 as batch_upload.  The argument buffer is ba's.
int launch_particles_batch(const ParticleLaunch* L, int n, BatchArgs& ba, hipStream_t st);
void free_batch_args(BatchArgs& ba);

}  // namespace cpic
