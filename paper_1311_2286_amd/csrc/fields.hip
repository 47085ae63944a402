// fields.hip -- grid-side kernels of the curvilinear PIC hot path (FP64):
// metric coefficients, fixed background, charge, Poisson solve by geometric
// multigrid, gauge, vertex field, diagnostics reductions.
//
// Discrete operator (Eq. poiscurv multiplied by J and integrated over a cell;
// second order, conservative, ghost-cell boundaries):
//   (A phi)_c = sum_a [ w_a(c+) (phi_{c+e_a} - phi_c) + w_a(c-) (phi_{c-e_a} - phi_c) ]
//             - sum_{pairs i<j} sum_{4 edges e around c} W_e (u_c D_j phi + w_c D_i phi)_e
// with face weights w = a^{ii} dV / h_i^2, edge weights W = a^{ij} dV/(h_i h_j),
// a^{ij} = J g^{ij} at the face / edge centre, D_i phi at an edge the mean of
// the two cell differences across i in the 2x2 block around it, and
// u_c, w_c = +-1/2 the position of c in that block.  It is the negative
// Hessian of the discrete energy, hence symmetric (and negative
// semi-definite).  Dirichlet walls: ghost 2 phi_b - phi_in; Neumann: phi_in.
//
// Multigrid: cell-centred V-cycles, damped Jacobi smoothing (even sweep
// counts, ping-pong buffers), residual restricted by summing the 2^d children,
// correction prolonged by (3/4, 1/4) tensor interpolation, coarse operators
// rediscretised from the analytic map at each level, coarsest level solved
// by one workgroup.  Convergence is tested on the device (no host sync); the
// kernels of later cycles return at once once the flag is set.
#include <hip/hip_fp16.h>
#include <string.h>

#include <type_traits>
#include <utility>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace cpic {

// ----------------------------------------------------------------------------
// metric helpers in FP64 (the Jacobi matrix itself is map_jacobi, common.hpp)
// ----------------------------------------------------------------------------
__device__ inline double det3(int d, const double j[3][3]) {
  if (d == 2) return j[0][0] * j[1][1] - j[0][1] * j[1][0];
  return j[0][0] * (j[1][1] * j[2][2] - j[1][2] * j[2][1]) - j[0][1] * (j[1][0] * j[2][2] - j[1][2] * j[2][0]) +
         j[0][2] * (j[1][0] * j[2][1] - j[1][1] * j[2][0]);
}

// inverse Jacobi matrix k = j^{-1} (Eq. jcon) by the adjugate
__device__ inline void inv3(int d, const double j[3][3], double k[3][3], double& J) {
  J = det3(d, j);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) k[a][b] = (a == b) ? 1.0 : 0.0;
  if (d == 2) {
    k[0][0] = j[1][1] / J;
    k[0][1] = -j[0][1] / J;
    k[1][0] = -j[1][0] / J;
    k[1][1] = j[0][0] / J;
    return;
  }
  k[0][0] = (j[1][1] * j[2][2] - j[1][2] * j[2][1]) / J;
  k[0][1] = (j[0][2] * j[2][1] - j[0][1] * j[2][2]) / J;
  k[0][2] = (j[0][1] * j[1][2] - j[0][2] * j[1][1]) / J;
  k[1][0] = (j[1][2] * j[2][0] - j[1][0] * j[2][2]) / J;
  k[1][1] = (j[0][0] * j[2][2] - j[0][2] * j[2][0]) / J;
  k[1][2] = (j[0][2] * j[1][0] - j[0][0] * j[1][2]) / J;
  k[2][0] = (j[1][0] * j[2][1] - j[1][1] * j[2][0]) / J;
  k[2][1] = (j[0][1] * j[2][0] - j[0][0] * j[2][1]) / J;
  k[2][2] = (j[0][0] * j[1][1] - j[0][1] * j[1][0]) / J;
}

// a^{pq} = Omega J g^{pq}, g^{pq} = k^{p r} k^{q r} (Eqs. gcon, poiscurv), with
// the geometric factor Omega = x^1 when g.omega is set, else 1
__device__ inline double coef_pq(const Geo& g, const double* xi, int p, int q) {
  double j[3][3], k[3][3], J, x[3];
  map_jacobi(g, xi, j, x);
  inv3(g.dim, j, k, J);
  double s = 0.0;
  for (int r = 0; r < g.dim; ++r) s += k[p][r] * k[q][r];
  return (g.omega ? x[0] : 1.0) * J * s;
}

// ----------------------------------------------------------------------------
// small helpers
// ----------------------------------------------------------------------------
__device__ inline void lin_to_idx(long long c, const int* n, int* idx) {
  idx[0] = (int)(c % n[0]);
  long long t = c / n[0];
  idx[1] = (int)(t % n[1]);
  idx[2] = (int)(t / n[1]);
}
__device__ inline long long idx_to_lin(const int* idx, const int* n) {
  return (long long)idx[0] + (long long)n[0] * (idx[1] + (long long)n[1] * idx[2]);
}
__device__ inline int wrapi(int v, int n) {
  if (v < 0) return v + n;
  if (v >= n) return v - n;
  return v;
}

__global__ void fill_u8_kernel(unsigned char* p, unsigned char v, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}
__global__ void fill_u64_kernel(unsigned long long* p, unsigned long long v, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

struct ZeroRanges {
  unsigned* p[32];
  unsigned long long words[32];
};
// workgroup row blockIdx.y zeroes range y, grid-stride over its words
__global__ __launch_bounds__(256) void zero_ranges_kernel(ZeroRanges r) {
  unsigned* p = r.p[blockIdx.y];
  const unsigned long long n = r.words[blockIdx.y];
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * blockDim.x)
    p[i] = 0u;
}

void launch_zero_ranges(const FillRange* r, int n, hipStream_t st) {
  for (int b = 0; b < n; b += 32) {
    ZeroRanges z;
    memset(&z, 0, sizeof(z));
    const int m = std::min(32, n - b);
    unsigned long long most = 0;
    for (int i = 0; i < m; ++i) {
      z.p[i] = (unsigned*)r[b + i].p;
      z.words[i] = r[b + i].bytes / 4;
      most = std::max(most, z.words[i]);
    }
    if (most == 0) continue;
    const unsigned bx = (unsigned)std::min<unsigned long long>((most + 255) / 256, 1024);
    hipLaunchKernelGGL(zero_ranges_kernel, dim3(bx, (unsigned)m), dim3(256), 0, st, z);
  }
}

// A step's record for the host (the solver's cycles and the species' drift),
// written into pinned host memory, which the host reads after the event
// recorded behind this launch: one small launch in place of two copies.
__global__ void step_record_kernel(const int* __restrict__ cycles_dev, const unsigned* __restrict__ drift_dev, int nsp,
                                   int* cycles_host, unsigned* drift_host) {
  const int t = threadIdx.x;
  if (t == 0) cycles_host[0] = cycles_dev[0];
  if (t < nsp) drift_host[t] = drift_dev[t];
  __threadfence_system();
}

void launch_step_record(const int* cycles_dev, const unsigned* drift_dev, int nsp, int* cycles_host,
                        unsigned* drift_host, hipStream_t st) {
  hipLaunchKernelGGL(step_record_kernel, dim3(1), dim3(64), 0, st, cycles_dev, drift_dev, nsp, cycles_host,
                     drift_host);
}

void launch_fill_u8(void* p, unsigned char v, size_t bytes, hipStream_t st) {
  if (bytes == 0 || batch_unsupported()) return;
  if (v == 0 && bytes % 8 == 0 && ((uintptr_t)p % 8) == 0) {
    size_t n = bytes / 8;
    unsigned blocks = (unsigned)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks), dim3(256), 0, st, (unsigned long long*)p, 0ull, n);
    return;
  }
  unsigned blocks = (unsigned)((bytes + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_u8_kernel, dim3(blocks), dim3(256), 0, st, (unsigned char*)p, v, bytes);
}

// Block coordinates and grid extent of one case's launch: its own launch, or
// its slice of a batched launch (cases stacked along z).
struct Blk {
  int x, y, z, gx, gy, gz;
};
__device__ inline Blk blk_single() {
  return {(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z, (int)gridDim.x, (int)gridDim.y, (int)gridDim.z};
}
__device__ inline Blk blk_batch(int gz) {
  return {(int)blockIdx.x, (int)blockIdx.y, (int)(blockIdx.z % gz), (int)gridDim.x, (int)gridDim.y, gz};
}

// kinds of the batched field-phase kernels (record tags)
enum BatchKind : int {
  BK_CHARGE = 1, BK_EXTRAP, BK_RHS, BK_SUB, BK_REDP, BK_REDF, BK_RESET, BK_FCGRES, BK_FCGAPPLY, BK_FCGCOEF,
  BK_FCGUPD, BK_SMOOTH_F, BK_SMOOTH_D, BK_RESID_F, BK_RESID_D, BK_RSUM_F, BK_RSUM_D, BK_RTR_F, BK_RTR_D,
  BK_PROL_F, BK_PROL_D, BK_SMALL_F, BK_SMALL_D, BK_EF2F, BK_EF2D, BK_EF3F, BK_EF3D, BK_RESR_F, BK_RESR_D,
  BK_SMOOTH_H, BK_RESR_H, BK_COUNT
};
template <typename T>
constexpr int kind_of(int kf, int kd) {
  return std::is_same<T, float>::value ? kf : kd;
}
template <typename T, typename C>
constexpr int kind_of(int kf, int kd, int kh) {
  return std::is_same<C, __half>::value ? kh : kind_of<T>(kf, kd);
}

// Kernels of the field phase as ops: an argument struct and a body that takes
// the case's block coordinates, launched alone or batched (see kernels.hpp).
template <typename Op>
__global__ __launch_bounds__(256) void op_single256(typename Op::Args a) {
  Op::body(a, blk_single());
}
template <typename Op>
__global__ __launch_bounds__(256) void op_batch256(const typename Op::Args* __restrict__ a, int gz) {
  Op::body(a[blockIdx.z / gz], blk_batch(gz));
}
template <typename Op>
__global__ __launch_bounds__(1024) void op_single1024(typename Op::Args a) {
  Op::body(a, blk_single());
}
template <typename Op>
__global__ __launch_bounds__(1024) void op_batch1024(const typename Op::Args* __restrict__ a, int gz) {
  Op::body(a[blockIdx.z / gz], blk_batch(gz));
}

thread_local BatchRecorder* g_batch_rec = nullptr;

template <typename Op>
static void op_launch(dim3 grid, dim3 block, const typename Op::Args& a, hipStream_t st) {
  if (g_batch_rec) {
    BatchRec r;
    r.kind = Op::KIND;
    r.grid = grid;
    r.block = block;
    r.args.assign((const unsigned char*)&a, (const unsigned char*)&a + sizeof(a));
    g_batch_rec->recs.push_back(std::move(r));
    return;
  }
  if (Op::BOUND == 1024)
    hipLaunchKernelGGL(op_single1024<Op>, grid, block, 0, st, a);
  else
    hipLaunchKernelGGL(op_single256<Op>, grid, block, 0, st, a);
}
template <typename Op>
static void op_replay(dim3 grid, dim3 block, const void* args, int n, hipStream_t st) {
  const dim3 g(grid.x, grid.y, grid.z * (unsigned)n);
  if (Op::BOUND == 1024)
    hipLaunchKernelGGL(op_batch1024<Op>, g, block, 0, st, (const typename Op::Args*)args, (int)grid.z);
  else
    hipLaunchKernelGGL(op_batch256<Op>, g, block, 0, st, (const typename Op::Args*)args, (int)grid.z);
}

// ----------------------------------------------------------------------------
// coefficients
// ----------------------------------------------------------------------------
// T: type of the operator coefficients (FP64; FP32 for the V-cycle used as a
// preconditioner of the flexible-CG solve)
// C: the storage type of the explicit stencil (T, or FP16 scaled by a power
// of two for the preconditioner's multi-workgroup levels: the stencil then
// holds 2^-e times the coefficients and cinv = 2^e)
template <typename T, typename C = T>
struct LevelArgsT {
  int dim;
  int n[3];
  int periodic[3];
  int dir[3][2];  // Dirichlet flags [axis][lo, hi]
  double h[3];
  double dV;
  int mixed;
  const double* wf[3];
  const double* wlo[3];
  const double* we[3];
  const C* S[9];
  const C* diag;
  T cinv;
};

template <typename T, typename C>
__device__ __forceinline__ T coef_val(C v) {
  if constexpr (std::is_same<C, __half>::value)
    return (T)__half2float(v);
  else
    return (T)v;
}
// diagonal of the operator at cell c
template <typename T, typename C>
__device__ __forceinline__ T diag_at(const LevelArgsT<T, C>& a, int c) {
  if constexpr (std::is_same<C, T>::value)
    return a.diag[c];
  else
    return coef_val<T>(a.diag[c]) * a.cinv;
}
using LevelArgs = LevelArgsT<double>;

static LevelArgs level_args(const GridCtx& G, int l) {
  const Level& L = G.lev[l];
  LevelArgs a;
  a.dim = G.g.dim;
  a.mixed = G.mixed;
  a.dV = L.dV;
  for (int i = 0; i < 3; ++i) {
    a.n[i] = L.n[i];
    a.periodic[i] = G.g.periodic[i];
    a.dir[i][0] = G.bc_lo[i] == BC_DIRICHLET;
    a.dir[i][1] = G.bc_hi[i] == BC_DIRICHLET;
    a.h[i] = L.h[i];
    a.wf[i] = L.wf[i];
    a.wlo[i] = L.wlo[i];
    a.we[i] = L.we[i];
  }
  for (int k = 0; k < 9; ++k) a.S[k] = L.S[k];
  a.diag = L.diag;
  a.cinv = 1.0;
  return a;
}

// the FP32 copy of a level's operator
static LevelArgsT<float> level_args_f32(const GridCtx& G, int l) {
  const LevelArgs d = level_args(G, l);
  const Level& L = G.lev[l];
  LevelArgsT<float> a;
  a.dim = d.dim;
  a.mixed = d.mixed;
  a.dV = d.dV;
  for (int i = 0; i < 3; ++i) {
    a.n[i] = d.n[i];
    a.periodic[i] = d.periodic[i];
    a.dir[i][0] = d.dir[i][0];
    a.dir[i][1] = d.dir[i][1];
    a.h[i] = d.h[i];
    a.wf[i] = d.wf[i];
    a.wlo[i] = d.wlo[i];
    a.we[i] = d.we[i];
  }
  for (int k = 0; k < 9; ++k) a.S[k] = L.f_S[k];
  a.diag = L.f_diag;
  a.cinv = 1.0f;
  return a;
}

// the FP16 copy of a level's operator (null diag when the level has none)
static LevelArgsT<float, __half> level_args_h(const GridCtx& G, int l) {
  const LevelArgsT<float> f = level_args_f32(G, l);
  const Level& L = G.lev[l];
  LevelArgsT<float, __half> a;
  a.dim = f.dim;
  a.mixed = f.mixed;
  a.dV = f.dV;
  for (int i = 0; i < 3; ++i) {
    a.n[i] = f.n[i];
    a.periodic[i] = f.periodic[i];
    a.dir[i][0] = f.dir[i][0];
    a.dir[i][1] = f.dir[i][1];
    a.h[i] = f.h[i];
    a.wf[i] = f.wf[i];
    a.wlo[i] = f.wlo[i];
    a.we[i] = f.we[i];
  }
  for (int k = 0; k < 9; ++k) a.S[k] = (const __half*)L.h_S[k];
  a.diag = (const __half*)L.h_diag;
  a.cinv = L.h_inv;
  return a;
}

template <typename T> static LevelArgsT<T> level_args_t(const GridCtx& G, int l);
template <> LevelArgsT<double> level_args_t<double>(const GridCtx& G, int l) { return level_args(G, l); }
template <> LevelArgsT<float> level_args_t<float>(const GridCtx& G, int l) { return level_args_f32(G, l); }

// the V-cycle vectors of a level in precision T
template <typename T>
struct LevelVec {
  T* phi;
  T* phi2;
  T* rhs;
  T* res;
  T* aux;
};
template <typename T> static LevelVec<T> level_vec(const GridCtx& G, int l);
template <> LevelVec<double> level_vec<double>(const GridCtx& G, int l) {
  const Level& L = G.lev[l];
  return {L.phi, L.phi2, L.rhs, L.res, L.aux};
}
template <> LevelVec<float> level_vec<float>(const GridCtx& G, int l) {
  const Level& L = G.lev[l];
  return {L.f_phi, L.f_phi2, L.f_rhs, L.f_res, L.f_aux};
}

__global__ void coef_kernel(Geo g, LevelArgs a, double* wf0, double* wf1, double* wf2, double* wl0,
                            double* wl1, double* wl2, double* we0, double* we1, double* we2) {
  long long nc = (long long)a.n[0] * a.n[1] * a.n[2];
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  int idx[3];
  lin_to_idx(c, a.n, idx);
  double* wf[3] = {wf0, wf1, wf2};
  double* wl[3] = {wl0, wl1, wl2};
  double* we[3] = {we0, we1, we2};
  const int d = a.dim;
  for (int ax = 0; ax < d; ++ax) {
    double xi[3];
    for (int b = 0; b < 3; ++b) xi[b] = (b < d) ? (idx[b] + 0.5) * a.h[b] : 0.0;
    xi[ax] = (idx[ax] + 1) * a.h[ax];
    wf[ax][c] = coef_pq(g, xi, ax, ax) * a.dV / (a.h[ax] * a.h[ax]);
    double lo = 0.0;
    if (!a.periodic[ax] && idx[ax] == 0) {
      xi[ax] = 0.0;
      lo = coef_pq(g, xi, ax, ax) * a.dV / (a.h[ax] * a.h[ax]);
    }
    wl[ax][c] = lo;
  }
  int pi[3] = {0, 0, 1}, pj[3] = {1, 2, 2};
  int np = (d == 3) ? 3 : 1;
  for (int p = 0; p < np; ++p) {
    double W = 0.0;
    // mixed terms only in planes of two periodic axes: with walls the map must
    // be orthogonal in the planes that hold a bounded axis
    if (a.mixed && a.periodic[pi[p]] && a.periodic[pj[p]]) {
      double xi[3];
      for (int b = 0; b < 3; ++b) xi[b] = (b < d) ? (idx[b] + 0.5) * a.h[b] : 0.0;
      xi[pi[p]] = (idx[pi[p]] + 1) * a.h[pi[p]];
      xi[pj[p]] = (idx[pj[p]] + 1) * a.h[pj[p]];
      W = coef_pq(g, xi, pi[p], pj[p]) * a.dV / (a.h[pi[p]] * a.h[pj[p]]);
    }
    we[p][c] = W;
  }
}

// diag of A and (level 0) the wall term bdir
__global__ void diag_kernel(LevelArgs a, double* diag, double* bdir, double plo0, double plo1,
                            double plo2, double phi0, double phi1, double phi2) {
  long long nc = (long long)a.n[0] * a.n[1] * a.n[2];
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  int idx[3];
  lin_to_idx(c, a.n, idx);
  const int d = a.dim;
  const double plo[3] = {plo0, plo1, plo2}, phi_[3] = {phi0, phi1, phi2};
  double dg = 0.0, bd = 0.0;
  for (int ax = 0; ax < d; ++ax) {
    // upper face
    if (a.periodic[ax] || idx[ax] < a.n[ax] - 1) {
      dg -= a.wf[ax][c];
    } else if (a.dir[ax][1]) {
      dg -= 2.0 * a.wf[ax][c];
      bd += 2.0 * a.wf[ax][c] * phi_[ax];
    }
    // lower face
    if (a.periodic[ax] || idx[ax] > 0) {
      int nb[3] = {idx[0], idx[1], idx[2]};
      nb[ax] = wrapi(idx[ax] - 1, a.n[ax]);
      dg -= a.wf[ax][idx_to_lin(nb, a.n)];
    } else if (a.dir[ax][0]) {
      dg -= 2.0 * a.wlo[ax][c];
      bd += 2.0 * a.wlo[ax][c] * plo[ax];
    }
  }
  if (a.mixed) {
    int pi[3] = {0, 0, 1}, pj[3] = {1, 2, 2};
    int np = (d == 3) ? 3 : 1;
    for (int p = 0; p < np; ++p) {
      int i = pi[p], j = pj[p];
      for (int si = 0; si < 2; ++si)
        for (int sj = 0; sj < 2; ++sj) {
          int b[3] = {idx[0], idx[1], idx[2]};
          b[i] = wrapi(idx[i] - si, a.n[i]);
          b[j] = wrapi(idx[j] - sj, a.n[j]);
          double W = a.we[p][idx_to_lin(b, a.n)];
          double sg = (si == sj) ? 1.0 : -1.0;
          dg -= 0.5 * W * sg;
        }
    }
  }
  diag[c] = dg;
  if (bdir) bdir[c] = bd;
}

// Explicit stencil from the face / edge weights.  The energy's face terms
// couple c and c + e_a with w_a(c).  An edge term W (D_i phi)(D_j phi) over
// the 2x2 block with lower corner b couples the diagonal pair (b, b+e_i+e_j)
// with +W/2 and the anti-diagonal pair (b+e_j, b+e_i) with -W/2; face pairs of
// the block get no mixed contribution.  Upper-half storage:
//   S[a](c)       = w_a(c)                (a = x, y, z; zero across a wall)
//   S[+i+j](c)    =  W_ij(c) / 2
//   S[+i-j](c)    = -W_ij(c - e_j) / 2
__global__ void stencil_kernel(LevelArgs a, double* S0, double* S1, double* S2, double* S3, double* S4,
                               double* S5, double* S6, double* S7, double* S8) {
  long long nc = (long long)a.n[0] * a.n[1] * a.n[2];
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  int idx[3];
  lin_to_idx(c, a.n, idx);
  double* S[9] = {S0, S1, S2, S3, S4, S5, S6, S7, S8};
  const int d = a.dim;
  for (int ax = 0; ax < d; ++ax) {
    bool wall = !a.periodic[ax] && idx[ax] == a.n[ax] - 1;
    S[ax][c] = wall ? 0.0 : a.wf[ax][c];
  }
  if (!a.mixed) return;
  // pairs (i, j) -> (diagonal slot, anti-diagonal slot)
  const int pi[3] = {0, 0, 1}, pj[3] = {1, 2, 2};
  const int np = (d == 3) ? 3 : 1;
  for (int p = 0; p < np; ++p) {
    const int i = pi[p], j = pj[p];
    int b[3] = {idx[0], idx[1], idx[2]};
    b[j] = wrapi(idx[j] - 1, a.n[j]);
    double Wd = a.we[p][c];
    double Wa = a.we[p][idx_to_lin(b, a.n)];
    const int sd = (d == 3) ? 3 + 2 * p : 3, sa = (d == 3) ? 4 + 2 * p : 4;
    S[sd][c] = 0.5 * Wd;
    S[sa][c] = -0.5 * Wa;
  }
}

void launch_coefficients(const GridCtx& G, int l, hipStream_t st) {
  const Level& L = G.lev[l];
  LevelArgs a = level_args(G, l);
  unsigned blocks = (unsigned)((L.ncells + 255) / 256);
  hipLaunchKernelGGL(coef_kernel, dim3(blocks), dim3(256), 0, st, G.g, a, L.wf[0], L.wf[1], L.wf[2],
                     L.wlo[0], L.wlo[1], L.wlo[2], L.we[0], L.we[1], L.we[2]);
  hipLaunchKernelGGL(diag_kernel, dim3(blocks), dim3(256), 0, st, a, L.diag, l == 0 ? G.bdir : nullptr,
                     G.phi_lo[0], G.phi_lo[1], G.phi_lo[2], G.phi_hi[0], G.phi_hi[1], G.phi_hi[2]);
  hipLaunchKernelGGL(stencil_kernel, dim3(blocks), dim3(256), 0, st, a, L.S[0], L.S[1], L.S[2], L.S[3],
                     L.S[4], L.S[5], L.S[6], L.S[7], L.S[8]);
}

__global__ void jc_kernel(Geo g, double* Jc) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ncells) return;
  int idx[3];
  lin_to_idx(c, g.n, idx);
  double xi[3];
  for (int b = 0; b < 3; ++b) xi[b] = (b < g.dim) ? (idx[b] + 0.5) * g.invn[b] : 0.0;
  double j[3][3];
  map_jacobi(g, xi, j, nullptr);
  Jc[c] = det3(g.dim, j);
}

void launch_jacobian_centres(const GridCtx& G, hipStream_t st) {
  unsigned blocks = (unsigned)((G.g.ncells + 255) / 256);
  hipLaunchKernelGGL(jc_kernel, dim3(blocks), dim3(256), 0, st, G.g, G.Jc);
}

// ----------------------------------------------------------------------------
// fixed background: I_c = n0 * int S(xi - xi_c) J(xi) dxi (deposit's shape S),
// Gauss-Legendre, 8 nodes on each half cell of the 3-cell support.  2D only.
// ----------------------------------------------------------------------------
__constant__ double GL_NODE[8] = {-0.96028985649753623, -0.79666647741362674, -0.52553240991632899,
                                  -0.18343464249564980, 0.18343464249564980,  0.52553240991632899,
                                  0.79666647741362674,  0.96028985649753623};
__constant__ double GL_WGT[8] = {0.10122853629037626, 0.22238103445337447, 0.31370664587788729,
                                 0.36268378337836198, 0.36268378337836198, 0.31370664587788729,
                                 0.22238103445337447, 0.10122853629037626};

__device__ inline double shape_val(int shape, double u) {
  double a = fabs(u);
  if (shape == SHAPE_B2) {
    if (a < 0.5) return 0.75 - u * u;
    if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
    return 0.0;
  }
  return a < 1.0 ? 1.0 - a : 0.0;
}

__global__ void background_kernel(Geo g, int shape, double n0, double* I) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ncells) return;
  int idx[3];
  lin_to_idx(c, g.n, idx);
  double sum = 0.0;
  for (int qy = 0; qy < 48; ++qy) {
    double uy = -1.25 + 0.5 * (qy / 8) + 0.25 * GL_NODE[qy % 8];
    double wy = 0.25 * GL_WGT[qy % 8] * shape_val(shape, uy);
    if (wy == 0.0) continue;
    for (int qx = 0; qx < 48; ++qx) {
      double ux = -1.25 + 0.5 * (qx / 8) + 0.25 * GL_NODE[qx % 8];
      double wx = 0.25 * GL_WGT[qx % 8] * shape_val(shape, ux);
      if (wx == 0.0) continue;
      double xi[3] = {(idx[0] + 0.5 + ux) * g.invn[0], (idx[1] + 0.5 + uy) * g.invn[1], 0.0};
      double j[3][3];
      map_jacobi(g, xi, j, nullptr);
      sum += wx * wy * det3(2, j);
    }
  }
  I[c] = n0 * sum * g.invn[0] * g.invn[1];
}

void launch_background(const GridCtx& G, int shape, double n0, hipStream_t st) {
  unsigned blocks = (unsigned)((G.g.ncells + 127) / 128);
  hipLaunchKernelGGL(background_kernel, dim3(blocks), dim3(128), 0, st, G.g, shape, n0, G.background);
}

// ----------------------------------------------------------------------------
// charge per cell: sum_s q_s w_s Q_s (integer Q scaled by 2^-d S1) + background
// ----------------------------------------------------------------------------
struct charge_kernelOp {
  static constexpr int KIND = BK_CHARGE, BOUND = 256;
  struct Args {
    long long nc;
    ChargeSpecies cs;
    const double* bg;
    double bgq;
    double* charge;
  };
  static __device__ void body(const Args& k_, const Blk& b_) {
    long long nc = k_.nc;
    const ChargeSpecies& cs = k_.cs;
    const double* bg = k_.bg;
    double bgq = k_.bgq;
    double* charge = k_.charge;

  long long c = (long long)b_.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  double s = 0.0;
  for (int k = 0; k < cs.n; ++k) {
    double q = cs.fixed ? (double)((const unsigned long long*)cs.Q[k])[c] : ((const double*)cs.Q[k])[c];
    double t = cs.qw[k] * q;
    s = (k == 0) ? t : s + t;
  }
  if (bg) s = s + bgq * bg[c];
  charge[c] = s;

  }
};

void launch_charge(const GridCtx& G, const ChargeSpecies& cs, double bg_charge, hipStream_t st) {
  unsigned blocks = (unsigned)((G.g.ncells + 255) / 256);
  op_launch<charge_kernelOp>(dim3(blocks), dim3(256), charge_kernelOp::Args{G.g.ncells, cs, G.background, bg_charge, G.charge}, st);
}

// ----------------------------------------------------------------------------
// deterministic reductions: fixed grid of 256 blocks, fixed-order tree
// ----------------------------------------------------------------------------
constexpr int RED_BLOCKS = REDUCE_BLOCKS;
// the field phase's sums over the level-0 cells (right side, |b|^2, gauge):
// four workgroups per CU keep enough loads in flight for HBM; G.partials holds
// this many partial sums
constexpr int FIELD_RED_BLOCKS = 1024;

__device__ inline double block_sum(double v) {
  __shared__ double sh[16];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int nthreads = blockDim.x * blockDim.y * blockDim.z;
  const int lane = tid & 63, w = tid >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (tid == 0) {
    const int nw = (nthreads + 63) / 64;
    for (int i = 0; i < nw; ++i) s += sh[i];
  }
  return s;  // valid in thread 0
}

// Workgroups are dealt to the eight XCDs round-robin in launch order.  The
// stencil kernels below take their tile from a remapped index instead, so that
// each XCD walks a contiguous run of tiles (whole z-planes in order) and finds
// the neighbour rows and planes it reads in its own L2.  That pays only while
// three planes of the stencil's arrays fit in one XCD's 4 MB L2: planes of at
// most XCD_PLANE_TILES tiles (16,384 cells: 3 x 44 B x 16,384 = 2.2 MB in
// FP32); larger planes keep the launch order, which spreads every plane over
// all eight L2s.  The map is a bijection (identity unless the tile count
// divides by eight); `blk` is the logical tile number, which orders the
// per-block partial sums as before.
constexpr int XCD_PLANE_TILES = 64;
struct Tile3 {
  int bx, by, bz, blk;
};
__device__ inline Tile3 xcd_tile(const Blk& B) {
  const int gx = B.gx, gy = B.gy;
  const int nb = gx * gy * B.gz;
  const int b = B.x + gx * (B.y + gy * B.z);
  const int t = ((nb & 7) == 0 && gx * gy <= XCD_PLANE_TILES) ? (b & 7) * (nb >> 3) + (b >> 3) : b;
  Tile3 r;
  r.bx = t % gx;
  r.by = (t / gx) % gy;
  r.bz = t / (gx * gy);
  r.blk = t;
  return r;
}
__device__ inline Tile3 xcd_tile() { return xcd_tile(blk_single()); }


// kind 0: sum a*b; kind 1: sum a; kind 2: sum a*a
struct reduce_partial_kernelOp {
  static constexpr int KIND = BK_REDP, BOUND = 256;
  struct Args {
    const double* a;
    const double* b;
    long long n;
    int kind;
    double* partials;
    const int* flag;
  };
  static __device__ void body(const Args& k_, const Blk& b_) {
    const double* a = k_.a;
    const double* b = k_.b;
    long long n = k_.n;
    int kind = k_.kind;
    double* partials = k_.partials;
    const int* flag = k_.flag;

  if (flag && flag[0]) return;
  // grid-stride, four running sums (four loads in flight), added pairwise
  const long long stride = (long long)b_.gx * blockDim.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  auto term = [&](long long i) {
    const double x = a[i];
    return (kind == 0) ? x * b[i] : (kind == 1 ? x : x * x);
  };
  long long i = (long long)b_.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] += term(i + u * stride);
  }
  for (; i < n; i += stride) acc[0] += term(i);
  const double s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  double t = block_sum(s);
  if (threadIdx.x == 0) partials[b_.x] = t;

  }
};

// op 0: out = sum; op 1: MG convergence test vs scalars[0] (|b|^2):
//   sets flag[0] when sum <= rtol^2 |b|^2 (or |b| == 0), counts cycles in flag[1]
struct reduce_final_kernelOp {
  static constexpr int KIND = BK_REDF, BOUND = 1024;
  struct Args {
    const double* partials;
    int nb;
    double* out;
    int op;
    double rtol2;
    const double* bnorm2;
    int* flag;
    int count_cycle;
  };
  static __device__ void body(const Args& k_, const Blk& b_) {
    const double* partials = k_.partials;
    int nb = k_.nb;
    double* out = k_.out;
    int op = k_.op;
    double rtol2 = k_.rtol2;
    const double* bnorm2 = k_.bnorm2;
    int* flag = k_.flag;
    int count_cycle = k_.count_cycle;

  if (op == 1 && flag[0]) return;
  double s;
  strided_sums<1, 8>(partials, 0, nb, &s);
  // fixed-order: each thread's strided sums, then the block tree
  double t = block_sum(s);
  if (threadIdx.x == 0) {
    *out = t;
    if (op == 1) {
      if (count_cycle) flag[1] += 1;
      if (t <= rtol2 * (*bnorm2) || *bnorm2 == 0.0) flag[0] = 1;
      if (count_cycle && flag[1] >= flag[2]) flag[0] = 1;  // the solve's cycle budget is spent
    }
  }

  }
};

// blocks: the number of partial sums, which partials must hold
static void reduce(const double* a, const double* b, long long n, int kind, double* partials, double* out,
                   hipStream_t st, int blocks = FIELD_RED_BLOCKS) {
  op_launch<reduce_partial_kernelOp>(dim3(blocks), dim3(256), reduce_partial_kernelOp::Args{a, b, n, kind, partials, (const int*)nullptr}, st);
  op_launch<reduce_final_kernelOp>(dim3(1), dim3(256), reduce_final_kernelOp::Args{partials, blocks, out, 0, 0.0, (const double*)nullptr, (int*)nullptr, 0}, st);
}

// ----------------------------------------------------------------------------
// right-hand side: b = -charge - bdir, projected to zero sum when singular
// ----------------------------------------------------------------------------
struct rhs_kernelOp {
  static constexpr int KIND = BK_RHS, BOUND = 256;
  struct Args {
    long long nc;
    const double* charge;
    const double* bdir;
    double* rhs;
  };
  static __device__ void body(const Args& k_, const Blk& b_) {
    long long nc = k_.nc;
    const double* charge = k_.charge;
    const double* bdir = k_.bdir;
    double* rhs = k_.rhs;

  long long c = (long long)b_.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  rhs[c] = -charge[c] - bdir[c];

  }
};
struct sub_scalar_kernelOp {
  static constexpr int KIND = BK_SUB, BOUND = 256;
  struct Args {
    long long n;
    double* x;
    const double* s;
    double scale;
  };
  static __device__ void body(const Args& k_, const Blk& b_) {
    long long n = k_.n;
    double* x = k_.x;
    const double* s = k_.s;
    double scale = k_.scale;

  long long c = (long long)b_.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  x[c] -= (*s) * scale;

  }
};

void launch_rhs(const GridCtx& G, hipStream_t st) {
  const Level& L = G.lev[0];
  unsigned blocks = (unsigned)((L.ncells + 255) / 256);
  op_launch<rhs_kernelOp>(dim3(blocks), dim3(256), rhs_kernelOp::Args{L.ncells, G.charge, G.bdir, L.rhs}, st);
  if (G.all_periodic) {
    reduce(L.rhs, nullptr, L.ncells, 1, G.partials, G.scalars + 3, st);
    op_launch<sub_scalar_kernelOp>(dim3(blocks), dim3(256), sub_scalar_kernelOp::Args{L.ncells, L.rhs, G.scalars + 3, 1.0 / (double)L.ncells}, st);
  }
}

// ----------------------------------------------------------------------------
// operator
// ----------------------------------------------------------------------------
// (A phi)_c from the explicit stencil: diag, the upper-half coefficients of c
// and, by symmetry, those stored at the lower neighbours.  Across a wall the
// lower neighbour term is absent and the upper coefficient is zero.
template <typename T, typename TV, typename C>
__device__ inline T apply_A(const LevelArgsT<T, C>& a, const TV* __restrict__ phi_in, const int* idx, long long cl) {
  const int c = (int)cl;
  const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
  const int sy = n0, sz = n0 * n1;
  const int dxp = idx[0] + 1 < n0 ? 1 : (a.periodic[0] ? 1 - n0 : 0);
  const int dxm = idx[0] > 0 ? -1 : (a.periodic[0] ? n0 - 1 : 0);
  const int dyp = (idx[1] + 1 < n1 ? 1 : (a.periodic[1] ? 1 - n1 : 0)) * sy;
  const int dym = (idx[1] > 0 ? -1 : (a.periodic[1] ? n1 - 1 : 0)) * sy;
  struct Rd {
    const TV* p;
    __device__ T operator[](long long i) const { return (T)p[i]; }
  } phi{phi_in};
  T acc = coef_val<T>(a.diag[c]) * phi[c];
  acc += coef_val<T>(a.S[0][c]) * phi[c + dxp];
  if (dxm) acc += coef_val<T>(a.S[0][c + dxm]) * phi[c + dxm];
  acc += coef_val<T>(a.S[1][c]) * phi[c + dyp];
  if (dym) acc += coef_val<T>(a.S[1][c + dym]) * phi[c + dym];
  if (a.dim == 3) {
    const int dzp = (idx[2] + 1 < n2 ? 1 : (a.periodic[2] ? 1 - n2 : 0)) * sz;
    const int dzm = (idx[2] > 0 ? -1 : (a.periodic[2] ? n2 - 1 : 0)) * sz;
    acc += coef_val<T>(a.S[2][c]) * phi[c + dzp];
    if (dzm) acc += coef_val<T>(a.S[2][c + dzm]) * phi[c + dzm];
    if (a.mixed) {
      acc += coef_val<T>(a.S[3][c]) * phi[c + dxp + dyp] + coef_val<T>(a.S[3][c + dxm + dym]) * phi[c + dxm + dym];
      acc += coef_val<T>(a.S[4][c]) * phi[c + dxp + dym] + coef_val<T>(a.S[4][c + dxm + dyp]) * phi[c + dxm + dyp];
      acc += coef_val<T>(a.S[5][c]) * phi[c + dxp + dzp] + coef_val<T>(a.S[5][c + dxm + dzm]) * phi[c + dxm + dzm];
      acc += coef_val<T>(a.S[6][c]) * phi[c + dxp + dzm] + coef_val<T>(a.S[6][c + dxm + dzp]) * phi[c + dxm + dzp];
      acc += coef_val<T>(a.S[7][c]) * phi[c + dyp + dzp] + coef_val<T>(a.S[7][c + dym + dzm]) * phi[c + dym + dzm];
      acc += coef_val<T>(a.S[8][c]) * phi[c + dyp + dzm] + coef_val<T>(a.S[8][c + dym + dzp]) * phi[c + dym + dzp];
    }
  } else if (a.mixed) {
    acc += coef_val<T>(a.S[3][c]) * phi[c + dxp + dyp] + coef_val<T>(a.S[3][c + dxm + dym]) * phi[c + dxm + dym];
    acc += coef_val<T>(a.S[4][c]) * phi[c + dxp + dym] + coef_val<T>(a.S[4][c + dxm + dyp]) * phi[c + dxm + dyp];
  }
  if constexpr (!std::is_same<C, T>::value) acc *= a.cinv;
  return acc;
}

// One smoothing step on a 3D launch grid (x threads along i, blockIdx.y/z
// along j, k):  r = rhs - A phi,  dn = cr r / diag + cd dprev,  out = phi + dn
// (and dout = dn when requested).  cd = 0 is a damped Jacobi sweep; the
// Chebyshev steps of the multigrid smoother use the three-term recurrence.
// With partials != null the squared residual of the input is summed per block
// (fixed order) for the convergence test.
// levels of at least this many cells take two cells per thread in the FP32
// smoothing sweeps
constexpr long long SMOOTH_ZP_CELLS = 1 << 20;
template <typename T, typename C = T>
struct smooth_kernelOp {
  static constexpr int KIND = kind_of<T, C>(BK_SMOOTH_F, BK_SMOOTH_D, BK_SMOOTH_H), BOUND = 256;
  // at most ZP cells per thread along z (Args::zp of them; the launch grid's
  // z extent is ceil(n2 / zp)): two on the large FP32 levels, so that each
  // wave has twice the loads in flight; one on the others, whose few blocks
  // need every thread, and on the FP64 sweeps, whose per-block partial sums
  // the plain V-cycles read
  static constexpr int ZP = sizeof(T) == 4 ? 2 : 1;
  struct Args {
    LevelArgsT<T, C> a;
    const T* phi;
    const T* rhs;
    T* out;
    double cr;
    double cd;
    const T* dprev;
    T* dout;
    const int* flag;
    double* partials;
    int zp;
  };
  static __device__ void body(const Args& k_, const Blk& b_) {
    const LevelArgsT<T, C>& a = k_.a;
    const T* __restrict__ phi = k_.phi;
    const T* __restrict__ rhs = k_.rhs;
    T* out = k_.out;
    double cr = k_.cr;
    double cd = k_.cd;
    const T* dprev = k_.dprev;
    T* dout = k_.dout;
    const int* flag = k_.flag;
    double* partials = k_.partials;

  if (flag[0]) return;
  const Tile3 T3 = xcd_tile(b_);
  const int i = T3.bx * blockDim.x + threadIdx.x;
  const int j = T3.by * blockDim.y + threadIdx.y;
  double rr = 0.0;
  if (i < a.n[0] && j < a.n[1]) {
    // the residuals of the thread's cells first, then the stores
    T r[ZP];
    int cz[ZP];
#pragma unroll
    for (int z = 0; z < ZP; ++z) {
      const int k = T3.bz * k_.zp + z;
      cz[z] = -1;
      r[z] = (T)0;
      if (z < k_.zp && k < a.n[2]) {
        const int idx[3] = {i, j, k};
        cz[z] = i + a.n[0] * (j + a.n[1] * k);
        r[z] = rhs[cz[z]] - apply_A(a, phi, idx, cz[z]);
      }
    }
#pragma unroll
    for (int z = 0; z < ZP; ++z) {
      const int c = cz[z];
      if (c < 0) continue;
      T dn = (T)cr * r[z] / diag_at(a, c);
      if (dprev) dn += (T)cd * dprev[c];
      out[c] = phi[c] + dn;
      if (dout) dout[c] = dn;
      rr += (double)r[z] * (double)r[z];
    }
  }
  if (partials) {
    double t = block_sum(rr);
    if (threadIdx.x == 0 && threadIdx.y == 0)
      partials[T3.blk] = t;
  }

  }
};

// Line relaxation on segments (anisotropic operators): every thread owns a
// run of LINE_SEG consecutive cells along axis `ax`; the residual
// r = rhs - A phi of the whole operator is formed for them, the tridiagonal
// part of A along the axis restricted to the run is solved by Thomas
// elimination (couplings to cells outside the run stay in r: block Jacobi over
// runs), and out = phi + omega delta.  Sweeps along every axis in turn smooth
// the error along whichever direction couples strongly, the role line
// relaxation plays in the paper's solver on anisotropic problems.  Residuals,
// diagonals and couplings go through LDS, so that every global access is
// coalesced: along axis 0 the workgroup's runs cover one contiguous range of
// cells (runs of 16 stored at a stride of 17 words, free of bank conflicts);
// along the other axes the threads of a workgroup take adjacent columns.
constexpr int LINE_SEG = 8;
constexpr int LINE_PAD = LINE_SEG + 1;
constexpr double LINE_OMEGA = 1.0;
// line relaxation replaces the Chebyshev smoother of the preconditioner once
// the operator's anisotropy (largest ratio of a cell's face coefficients)
// exceeds this; below it the cheaper point smoother wins in time
constexpr double LINE_ANISO = 50.0;

template <typename T>
__device__ inline void line_thomas(const T* lr_in, const T* ld, const T* lu, T* lr_out, int len, int step) {
  // lower coupling of cell m = upper coupling of cell m - 1 (symmetric A)
  T cp[LINE_SEG], dp[LINE_SEG];
  T prev_cp = (T)0, prev_dp = (T)0, lo = (T)0;
#pragma unroll
  for (int m = 0; m < LINE_SEG; ++m) {
    if (m < len) {
      const T den = ld[m * step] - lo * prev_cp;
      const T up = lu[m * step];
      cp[m] = up / den;
      dp[m] = (lr_in[m * step] - lo * prev_dp) / den;
      prev_cp = cp[m];
      prev_dp = dp[m];
      lo = up;
    }
  }
  T next = (T)0;
#pragma unroll
  for (int m = LINE_SEG - 1; m >= 0; --m) {
    if (m < len) {
      next = dp[m] - cp[m] * next;
      lr_out[m * step] = next;
    }
  }
}

// runs along axis 0
template <typename T>
__global__ __launch_bounds__(256) void line_x_kernel(LevelArgsT<T> a, const T* __restrict__ phi,
                                                     const T* __restrict__ rhs, T* out, T omega, const int* flag) {
  __shared__ T lr[256 * LINE_PAD], ld[256 * LINE_PAD], lu[256 * LINE_PAD];
  if (flag[0]) return;
  const int n0 = a.n[0], n1 = a.n[1];
  const long long nrows = (long long)n1 * a.n[2];
  const int nseg = (n0 + LINE_SEG - 1) / LINE_SEG;
  const long long total = (long long)nseg * nrows;
  const long long t0 = (long long)blockIdx.x * 256;
  const long long t1 = min(t0 + 255, total - 1);  // last run of the workgroup
  const long long row0 = t0 / nseg, row1 = t1 / nseg;
  const int s0 = (int)(t0 % nseg), s1 = (int)(t1 % nseg);
  const long long cfirst = row0 * n0 + (long long)s0 * LINE_SEG;
  const long long cend = row1 * n0 + min(n0, (s1 + 1) * LINE_SEG);
  for (long long c = cfirst + threadIdx.x; c < cend; c += 256) {
    const long long row = c / n0;
    const int i = (int)(c - row * n0);
    const int idx[3] = {i, (int)(row % n1), (int)(row / n1)};
    const int m = i % LINE_SEG;
    const long long run = (row - row0) * nseg + i / LINE_SEG - s0;
    const int o = (int)run * LINE_PAD + m;
    lr[o] = rhs[c] - apply_A(a, phi, idx, c);
    ld[o] = a.diag[c];
    lu[o] = (m + 1 < LINE_SEG && i + 1 < n0) ? (T)a.S[0][c] : (T)0;
  }
  __syncthreads();
  const long long t = t0 + threadIdx.x;
  if (t <= t1) {
    const int sg = (int)(t % nseg);
    const int len = min(LINE_SEG, n0 - sg * LINE_SEG);
    const int o = threadIdx.x * LINE_PAD;
    line_thomas(lr + o, ld + o, lu + o, lr + o, len, 1);
  }
  __syncthreads();
  for (long long c = cfirst + threadIdx.x; c < cend; c += 256) {
    const long long row = c / n0;
    const int i = (int)(c - row * n0);
    const long long run = (row - row0) * nseg + i / LINE_SEG - s0;
    out[c] = phi[c] + omega * lr[(int)run * LINE_PAD + i % LINE_SEG];
  }
}

// runs along axis 1 or 2: thread = column (adjacent along axis 0)
template <typename T>
__global__ __launch_bounds__(256) void line_yz_kernel(LevelArgsT<T> a, int ax, const T* __restrict__ phi,
                                                      const T* __restrict__ rhs, T* out, T omega,
                                                      const int* flag) {
  __shared__ T lr[LINE_SEG * 256], ld[LINE_SEG * 256], lu[LINE_SEG * 256];
  if (flag[0]) return;
  const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
  const int nax = a.n[ax];
  const int nseg = (nax + LINE_SEG - 1) / LINE_SEG;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)n0 * nseg * (ax == 1 ? n2 : n1);
  const bool live = t < total;
  int idx[3] = {0, 0, 0};
  if (live) {
    idx[0] = (int)(t % n0);
    const long long r = t / n0;
    if (ax == 1) {
      idx[1] = (int)(r % nseg) * LINE_SEG;
      idx[2] = (int)(r / nseg);
    } else {
      idx[1] = (int)(r % n1);
      idx[2] = (int)(r / n1) * LINE_SEG;
    }
  }
  const int start = idx[ax];
  const int len = live ? min(LINE_SEG, nax - start) : 0;
  const long long stride = ax == 1 ? (long long)n0 : (long long)n0 * n1;
  const long long c0 = idx[0] + (long long)n0 * (idx[1] + (long long)n1 * idx[2]);
  const int tx = threadIdx.x;
  for (int m = 0; m < len; ++m) {
    const long long c = c0 + m * stride;
    int id[3] = {idx[0], idx[1], idx[2]};
    id[ax] = start + m;
    lr[m * 256 + tx] = rhs[c] - apply_A(a, phi, id, c);
    ld[m * 256 + tx] = a.diag[c];
    lu[m * 256 + tx] = (m + 1 < len) ? (T)a.S[ax][c] : (T)0;
  }
  if (len > 0) line_thomas(lr + tx, ld + tx, lu + tx, lr + tx, len, 256);
  for (int m = 0; m < len; ++m) {
    const long long c = c0 + m * stride;
    out[c] = phi[c] + omega * lr[m * 256 + tx];
  }
}

// Gershgorin bound of D^-1 A per cell: sum over off-diagonal |A_cj| / |A_cc|
// (same neighbour pattern as apply_A); 1 + its maximum bounds the spectrum.
__global__ __launch_bounds__(256) void gershgorin_kernel(LevelArgs a, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= a.n[0] || j >= a.n[1]) return;
  const int idx[3] = {i, j, k};
  const int c = i + a.n[0] * (j + a.n[1] * k);
  const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
  const int sy = n0, sz = n0 * n1;
  const int dxm = idx[0] > 0 ? -1 : (a.periodic[0] ? n0 - 1 : 0);
  const int dym = (idx[1] > 0 ? -1 : (a.periodic[1] ? n1 - 1 : 0)) * sy;
  const int dxp = idx[0] + 1 < n0 ? 1 : (a.periodic[0] ? 1 - n0 : 0);
  const int dyp = (idx[1] + 1 < n1 ? 1 : (a.periodic[1] ? 1 - n1 : 0)) * sy;
  double s = fabs(a.S[0][c]) + (dxm ? fabs(a.S[0][c + dxm]) : 0.0) + fabs(a.S[1][c]) +
             (dym ? fabs(a.S[1][c + dym]) : 0.0);
  if (a.dim == 3) {
    const int dzm = (idx[2] > 0 ? -1 : (a.periodic[2] ? n2 - 1 : 0)) * sz;
    const int dzp = (idx[2] + 1 < n2 ? 1 : (a.periodic[2] ? 1 - n2 : 0)) * sz;
    s += fabs(a.S[2][c]) + (dzm ? fabs(a.S[2][c + dzm]) : 0.0);
    if (a.mixed) {
      s += fabs(a.S[3][c]) + fabs(a.S[3][c + dxm + dym]) + fabs(a.S[4][c]) + fabs(a.S[4][c + dxm + dyp]);
      s += fabs(a.S[5][c]) + fabs(a.S[5][c + dxm + dzm]) + fabs(a.S[6][c]) + fabs(a.S[6][c + dxm + dzp]);
      s += fabs(a.S[7][c]) + fabs(a.S[7][c + dym + dzm]) + fabs(a.S[8][c]) + fabs(a.S[8][c + dym + dzp]);
    }
  } else if (a.mixed) {
    s += fabs(a.S[3][c]) + fabs(a.S[3][c + dxm + dym]) + fabs(a.S[4][c]) + fabs(a.S[4][c + dxm + dyp]);
  }
  out[c] = s / fabs(a.diag[c]);
}

// residual r = rhs - A phi (coalesced pass over the fine level)
template <typename T>
struct residual_kernelOp {
  static constexpr int KIND = kind_of<T>(BK_RESID_F, BK_RESID_D), BOUND = 256;
  struct Args {
    LevelArgsT<T> a;
    const T* phi;
    const T* rhs;
    T* res;
    const int* flag;
  };
  static __device__ void body(const Args& k_, const Blk& b_) {
    const LevelArgsT<T>& a = k_.a;
    const T* __restrict__ phi = k_.phi;
    const T* __restrict__ rhs = k_.rhs;
    T* res = k_.res;
    const int* flag = k_.flag;

  if (flag[0]) return;
  const Tile3 T3 = xcd_tile(b_);
  const int i = T3.bx * blockDim.x + threadIdx.x;
  const int j = T3.by * blockDim.y + threadIdx.y;
  const int k = T3.bz;
  if (i >= a.n[0] || j >= a.n[1]) return;
  const int idx[3] = {i, j, k};
  const int c = i + a.n[0] * (j + a.n[1] * k);
  res[c] = rhs[c] - apply_A(a, phi, idx, c);

  }
};

// The first Chebyshev step of a smoothing that starts from a zero guess needs
// no residual: phi2 = aux = cr r / diag (then the step from phi2 follows).
// Kernels that produce the right side r of such a level apply it as they
// write r, which saves that step's pass over the level.
struct FirstSweep {
  const float* diag;  // null: not applied
  float* phi2;
  float* aux;
  float cr;
  __device__ inline void apply(int c, float r) const {
    const float d = cr * r / diag[c];
    phi2[c] = d;
    aux[c] = d;
  }
};
template <typename T>
struct FirstSweepT {
  const T* diag;
  T* phi2;
  T* aux;
  double cr;
};

// Two restrictions.  Summing the 2^d children's residuals is the cheaper and,
// on near-isotropic grids, the faster one; but with the bilinear prolongation
// it makes the V-cycle non-symmetric, and flexible CG can then stall on
// strongly anisotropic operators.  There the transpose of the prolongation is
// used, which makes the V-cycle symmetric and keeps the conjugate-gradient
// convergence guarantee (the choice is made once, at set-up).
//
// Residual of the fine level summed over each coarse cell's children (the
// summing restriction); coarse phi = 0, or with fs.diag set the coarse
// level's first Chebyshev step from zero.  Threads take fine cells as the
// residual kernel does (64 x 4 per workgroup, consecutive i in a wave, so
// every load is coalesced), each the two cells of a column pair in z (3D);
// the pairs along i add by a lane shuffle, along j through LDS.  Fixed
// summation order: bitwise reproducible.
template <typename T, typename CT = T>
struct resrestrict_kernelOp {
  static constexpr int KIND = kind_of<T, CT>(BK_RESR_F, BK_RESR_D, BK_RESR_H), BOUND = 256;
  struct Args {
    LevelArgsT<T, CT> a;
    const T* phi;
    const T* rhs;
    int nc0;
    int nc1;
    T* crhs;
    T* cphi;
    FirstSweepT<T> fs;
    const int* flag;
  };
  static __device__ void body(const Args& k_, const Blk& b_) {
    if (k_.flag[0]) return;
    const LevelArgsT<T, CT>& a = k_.a;
    const int i = b_.x * 64 + threadIdx.x, j = b_.y * 4 + threadIdx.y, K = b_.z;
    T s = (T)0;
    if (i < a.n[0] && j < a.n[1]) {
      const int nz = a.dim == 3 ? 2 : 1;
      for (int dz = 0; dz < nz; ++dz) {
        const int k = a.dim == 3 ? 2 * K + dz : 0;
        const int idx[3] = {i, j, k};
        const int c = i + a.n[0] * (j + a.n[1] * k);
        s += k_.rhs[c] - apply_A(a, k_.phi, idx, c);
      }
    }
    s += __shfl_xor(s, 1, 64);
    __shared__ T row[4][64];
    row[threadIdx.y][threadIdx.x] = s;
    __syncthreads();
    if ((threadIdx.x & 1) || (threadIdx.y & 1) || i >= a.n[0] || j >= a.n[1]) return;
    s += row[threadIdx.y + 1][threadIdx.x];
    const int I0 = i >> 1, I1 = j >> 1;
    const int C = I0 + k_.nc0 * (I1 + k_.nc1 * K);
    k_.crhs[C] = s;
    if (k_.fs.diag) {
      const T d = (T)k_.fs.cr * s / k_.fs.diag[C];
      k_.fs.phi2[C] = d;
      k_.fs.aux[C] = d;
    } else {
      k_.cphi[C] = (T)0;
    }
  }
};

// summing restriction of a residual array (multi-workgroup levels)
template <typename T>
struct restrict_sum_kernelOp {
  static constexpr int KIND = kind_of<T>(BK_RSUM_F, BK_RSUM_D), BOUND = 256;
  struct Args {
    int dim;
    int nf0;
    int nf1;
    const T* res;
    int nc0;
    int nc1;
    T* crhs;
    T* cphi;
    const int* flag;
  };
  static __device__ void body(const Args& k_, const Blk& b_) {
    int dim = k_.dim;
    int nf0 = k_.nf0;
    int nf1 = k_.nf1;
    const T* __restrict__ res = k_.res;
    int nc0 = k_.nc0;
    int nc1 = k_.nc1;
    T* crhs = k_.crhs;
    T* cphi = k_.cphi;
    const int* flag = k_.flag;

  if (flag[0]) return;
  const int I0 = b_.x * blockDim.x + threadIdx.x, I1 = b_.y * blockDim.y + threadIdx.y;
  const int I2 = b_.z;
  if (I0 >= nc0 || I1 >= nc1) return;
  const int C = I0 + nc0 * (I1 + nc1 * I2);
  const int f = 2 * I0 + nf0 * (2 * I1 + nf1 * (dim == 3 ? 2 * I2 : 0));
  T s = res[f] + res[f + 1] + res[f + nf0] + res[f + nf0 + 1];
  if (dim == 3) {
    const int fz = f + nf0 * nf1;
    s += res[fz] + res[fz + 1] + res[fz + nf0] + res[fz + nf0 + 1];
  }
  crhs[C] = s;
  cphi[C] = (T)0;

  }
};

// Transpose of the prolongation:  Per axis, coarse
// cell I receives from fine cells 2I and 2I+1 with weight 3/4 and from 2I-1
// and 2I+2 with weight 1/4; at a wall the prolongation's ghost (-e Dirichlet,
// +e Neumann) folds the outer 1/4 back onto I.  Weights multiply over axes.
template <typename T>
__device__ inline int restrict_taps(const LevelArgsT<T>& fa, int ax, int I, int nc, int* f, T* w) {
  const int nf = fa.n[ax];
  if (ax >= fa.dim) {
    f[0] = 0;
    w[0] = (T)1;
    return 1;
  }
  int k = 0;
  T in_lo = (T)0.75, in_hi = (T)0.75;
  if (I > 0 || fa.periodic[ax]) {
    f[k] = wrapi(2 * I - 1, nf);
    w[k++] = (T)0.25;
  } else {
    in_lo += fa.dir[ax][0] ? (T)-0.25 : (T)0.25;
  }
  if (I < nc - 1 || fa.periodic[ax]) {
    f[k] = wrapi(2 * I + 2, nf);
    w[k++] = (T)0.25;
  } else {
    in_hi += fa.dir[ax][1] ? (T)-0.25 : (T)0.25;
  }
  f[k] = 2 * I;
  w[k++] = in_lo;
  f[k] = 2 * I + 1;
  w[k++] = in_hi;
  return k;
}

template <typename T>
__device__ inline T restrict_transpose(const LevelArgsT<T>& fa, const T* __restrict__ res, const int* cn,
                                       const int* I) {
  int fx[4], fy[4], fz[4];
  T wx[4], wy[4], wz[4];
  const int kx = restrict_taps(fa, 0, I[0], cn[0], fx, wx);
  const int ky = restrict_taps(fa, 1, I[1], cn[1], fy, wy);
  const int kz = restrict_taps(fa, 2, I[2], cn[2], fz, wz);
  T s = (T)0;
  for (int c = 0; c < kz; ++c)
    for (int b = 0; b < ky; ++b) {
      const T wyz = wy[b] * wz[c];
      const int row = fa.n[0] * (fy[b] + fa.n[1] * fz[c]);
      for (int a = 0; a < kx; ++a) s += wx[a] * wyz * res[fx[a] + row];
    }
  return s;
}

// coarse rhs = P^T (fine residual); coarse phi = 0
template <typename T>
struct restrict_kernelOp {
  static constexpr int KIND = kind_of<T>(BK_RTR_F, BK_RTR_D), BOUND = 256;
  struct Args {
    LevelArgsT<T> fa;
    const T* res;
    int nc0;
    int nc1;
    int nc2;
    T* crhs;
    T* cphi;
    const int* flag;
  };
  static __device__ void body(const Args& k_, const Blk& b_) {
    const LevelArgsT<T>& fa = k_.fa;
    const T* __restrict__ res = k_.res;
    int nc0 = k_.nc0;
    int nc1 = k_.nc1;
    int nc2 = k_.nc2;
    T* crhs = k_.crhs;
    T* cphi = k_.cphi;
    const int* flag = k_.flag;

  if (flag[0]) return;
  const int I0 = b_.x * blockDim.x + threadIdx.x, I1 = b_.y * blockDim.y + threadIdx.y;
  const int I2 = b_.z;
  if (I0 >= nc0 || I1 >= nc1) return;
  const int cn[3] = {nc0, nc1, nc2};
  const int I[3] = {I0, I1, I2};
  const int C = I0 + nc0 * (I1 + nc1 * I2);
  crhs[C] = restrict_transpose(fa, res, cn, I);
  cphi[C] = (T)0;

  }
};

// (3/4, 1/4)-tensor interpolation of the coarse correction at fine cell idx
template <typename T>
__device__ inline T prolong_cell(const LevelArgsT<T>& fa, const T* __restrict__ cphi, const int* cn,
                                 const int* idx) {
  const int d = fa.dim;
  int I[3] = {idx[0] >> 1, idx[1] >> 1, idx[2] >> 1};
  int J[3];
  T sgn[3];
  for (int ax = 0; ax < 3; ++ax) {
    J[ax] = I[ax];
    sgn[ax] = (T)1;
    if (ax >= d) continue;
    int step = (idx[ax] & 1) ? 1 : -1;
    int v = I[ax] + step;
    if (fa.periodic[ax]) {
      J[ax] = wrapi(v, cn[ax]);
    } else if (v < 0 || v >= cn[ax]) {
      // ghost of the correction: homogeneous Dirichlet -> -e, Neumann -> e
      J[ax] = I[ax];
      int dirw = (v < 0) ? fa.dir[ax][0] : fa.dir[ax][1];
      sgn[ax] = dirw ? (T)-1 : (T)1;
    } else {
      J[ax] = v;
    }
  }
  T acc = (T)0;
  const int nz = (d == 3) ? 2 : 1;
  for (int tz = 0; tz < nz; ++tz)
    for (int ty = 0; ty < 2; ++ty)
      for (int tx = 0; tx < 2; ++tx) {
        int t[3] = {tx, ty, tz};
        int K[3];
        T w = (T)1;
        for (int ax = 0; ax < 3; ++ax) {
          if (ax >= d) {
            K[ax] = 0;
            continue;
          }
          K[ax] = t[ax] ? J[ax] : I[ax];
          w *= t[ax] ? (T)0.25 * sgn[ax] : (T)0.75;
        }
        acc += w * cphi[K[0] + cn[0] * (K[1] + cn[1] * K[2])];
      }
  return acc;
}

template <typename T>
struct prolong_kernelOp {
  static constexpr int KIND = kind_of<T>(BK_PROL_F, BK_PROL_D), BOUND = 256;
  struct Args {
    LevelArgsT<T> fa;
    T* phi;
    const T* cphi;
    int nc0;
    int nc1;
    int nc2;
    const int* flag;
    int zp;  // fine cells per thread along z (1 or 2; the grid's z extent is ceil(n2 / zp))
  };
  static __device__ void body(const Args& k_, const Blk& b_) {
    const LevelArgsT<T>& fa = k_.fa;
    T* phi = k_.phi;
    const T* __restrict__ cphi = k_.cphi;
    int nc0 = k_.nc0;
    int nc1 = k_.nc1;
    int nc2 = k_.nc2;
    const int* flag = k_.flag;

  if (flag[0]) return;
  const int cn[3] = {nc0, nc1, nc2};
  const int i = (int)(b_.x * blockDim.x + threadIdx.x), j = (int)(b_.y * blockDim.y + threadIdx.y);
  if (i >= fa.n[0] || j >= fa.n[1]) return;
  T e[2];
  int cz[2] = {-1, -1};
#pragma unroll
  for (int dz = 0; dz < 2; ++dz) {
    const int k = (int)b_.z * k_.zp + dz;
    e[dz] = (T)0;
    if (dz < k_.zp && k < fa.n[2]) {
      const int idx[3] = {i, j, k};
      cz[dz] = i + fa.n[0] * (j + fa.n[1] * k);
      e[dz] = prolong_cell(fa, cphi, cn, idx);
    }
  }
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
    if (cz[dz] >= 0) phi[cz[dz]] += e[dz];

  }
};

// The V-cycle below level ls (all levels of at most SMALL_CELLS cells) in one
// workgroup: smoothing, restriction, coarsest solve (conjugate gradients, in
// LDS by one wavefront when the level is small enough), prolongation, with
// workgroup barriers between the phases.  Each phase costs a few L2 round
// trips, so only levels of a few hundred cells are worth keeping here.
constexpr int MAX_SMALL = 8;
constexpr int COARSE_LDS = 384;  // coarsest levels up to this many cells are solved in LDS
template <typename T>
struct SmallLevels {
  int nl;
  int transpose;  // restriction: transpose of the prolongation (else summing)
  const T* cinv;  // dense inverse of the coarsest operator (column-major), or null
  LevelArgsT<T> a[MAX_SMALL];
  T* phi[MAX_SMALL];
  T* phi2[MAX_SMALL];
  T* rhs[MAX_SMALL];
  T* res[MAX_SMALL];
  T* aux[MAX_SMALL];
};

// sum over the workgroup, returned to every thread
__device__ inline double block_allsum(double v) {
  __shared__ double sh[16];
  __shared__ double tot;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) s += sh[i];
    tot = s;
  }
  __syncthreads();
  return tot;
}

// Coarsest-level solve inside one workgroup: Jacobi-preconditioned conjugate
// gradients on -A (A is negative semi-definite) until |r|^2 <= tol2 |b|^2 or
// maxit iterations; singular (all-periodic) problems are solved on
// the zero-mean subspace and the result shifted to zero mean.
template <typename T>
__device__ inline void block_cg(const LevelArgsT<T>& a, T* x, const T* b, T* r, T* p, T* q, int maxit, int singular,
                                double tol2) {
  const int nc = a.n[0] * a.n[1] * a.n[2];
  double bmean = 0.0;
  if (singular) {
    double s = 0.0;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) s += b[c];
    bmean = block_allsum(s) / nc;
  }
  double rz = 0.0, bb = 0.0;
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    int idx[3] = {c % a.n[0], (c / a.n[0]) % a.n[1], c / (a.n[0] * a.n[1])};
    double bc = b[c] - bmean;
    double rc = bc - apply_A(a, x, idx, c);
    r[c] = rc;
    double z = rc / a.diag[c];
    p[c] = z;
    rz += rc * z;
    bb += bc * bc;
  }
  rz = block_allsum(rz);
  bb = block_allsum(bb);
  for (int it = 0; it < maxit; ++it) {
    double pq = 0.0;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
      int idx[3] = {c % a.n[0], (c / a.n[0]) % a.n[1], c / (a.n[0] * a.n[1])};
      double qc = apply_A(a, p, idx, c);
      q[c] = qc;
      pq += p[c] * qc;
    }
    pq = block_allsum(pq);
    if (pq == 0.0) break;
    const double alpha = rz / pq;
    double rr = 0.0, rz2 = 0.0;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
      x[c] += alpha * p[c];
      double rc = r[c] - alpha * q[c];
      r[c] = rc;
      rr += rc * rc;
      rz2 += rc * rc / a.diag[c];
    }
    rr = block_allsum(rr);
    rz2 = block_allsum(rz2);
    if (rr <= tol2 * bb || rz == 0.0) break;
    const double beta = rz2 / rz;
    rz = rz2;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) p[c] = r[c] / a.diag[c] + beta * p[c];
    __syncthreads();
  }
  if (singular) {
    double s = 0.0;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) s += x[c];
    const double mean = block_allsum(s) / nc;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) x[c] -= mean;
  }
  __syncthreads();
}

// The same Jacobi-preconditioned CG run by one wavefront (lanes 0..63) on
// vectors held in LDS: reductions are lane shuffles and no workgroup barrier is
// needed between iterations.  LDS accesses of one wavefront complete in issue
// order; the fences keep the compiler from reordering them across phases.
__device__ inline double wave_allsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <typename T>
__device__ inline void wave_cg(const LevelArgsT<T>& a, T* x, const T* b, T* r, T* p, T* q, int maxit, int singular,
                               double tol2) {
  const int nc = a.n[0] * a.n[1] * a.n[2];
  const int lane = threadIdx.x & 63;
  double bmean = 0.0;
  if (singular) {
    double s = 0.0;
    for (int c = lane; c < nc; c += 64) s += b[c];
    bmean = wave_allsum(s) / nc;
  }
  double rz = 0.0, bb = 0.0;
  for (int c = lane; c < nc; c += 64) {
    int idx[3] = {c % a.n[0], (c / a.n[0]) % a.n[1], c / (a.n[0] * a.n[1])};
    double bc = b[c] - bmean;
    double rc = bc - apply_A(a, x, idx, c);
    r[c] = rc;
    double z = rc / a.diag[c];
    p[c] = z;
    rz += rc * z;
    bb += bc * bc;
  }
  rz = wave_allsum(rz);
  bb = wave_allsum(bb);
  wave_sync();
  for (int it = 0; it < maxit; ++it) {
    double pq = 0.0;
    for (int c = lane; c < nc; c += 64) {
      int idx[3] = {c % a.n[0], (c / a.n[0]) % a.n[1], c / (a.n[0] * a.n[1])};
      double qc = apply_A(a, p, idx, c);
      q[c] = qc;
      pq += p[c] * qc;
    }
    pq = wave_allsum(pq);
    if (pq == 0.0) break;
    const double alpha = rz / pq;
    double rr = 0.0, rz2 = 0.0;
    for (int c = lane; c < nc; c += 64) {
      x[c] += alpha * p[c];
      double rc = r[c] - alpha * q[c];
      r[c] = rc;
      rr += rc * rc;
      rz2 += rc * rc / a.diag[c];
    }
    rr = wave_allsum(rr);
    rz2 = wave_allsum(rz2);
    if (rr <= tol2 * bb || rz == 0.0) break;
    const double beta = rz2 / rz;
    rz = rz2;
    wave_sync();
    for (int c = lane; c < nc; c += 64) p[c] = r[c] / a.diag[c] + beta * p[c];
    wave_sync();
  }
  if (singular) {
    double s = 0.0;
    for (int c = lane; c < nc; c += 64) s += x[c];
    const double mean = wave_allsum(s) / nc;
    for (int c = lane; c < nc; c += 64) x[c] -= mean;
  }
  wave_sync();
}

template <typename T>
__device__ inline void block_smooth(const LevelArgsT<T>& a, const T* phi, const T* rhs, T* out, T omega) {
  const int nc = a.n[0] * a.n[1] * a.n[2];
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    int idx[3] = {c % a.n[0], (c / a.n[0]) % a.n[1], c / (a.n[0] * a.n[1])};
    const T r = rhs[c] - apply_A(a, phi, idx, c);
    out[c] = phi[c] + omega * r / a.diag[c];
  }
  __syncthreads();
}

template <typename T>
struct small_vcycle_kernelOp {
  static constexpr int KIND = kind_of<T>(BK_SMALL_F, BK_SMALL_D), BOUND = 1024;
  struct Args {
    SmallLevels<T> S;
    int nu1;
    int nu2;
    double coarse_tol2;
    int singular;
    const int* flag;
  };
  static __device__ void body(const Args& k_, const Blk& b_) {
    const SmallLevels<T>& S = k_.S;
    int nu1 = k_.nu1;
    int nu2 = k_.nu2;
    double coarse_tol2 = k_.coarse_tol2;
    int singular = k_.singular;
    const int* flag = k_.flag;

  if (flag[0]) return;
  const T omega = (T)0.8;
  const int last = S.nl - 1;
  for (int l = 0; l < last; ++l) {
    const LevelArgsT<T>& a = S.a[l];
    for (int s = 0; s < nu1; s += 2) {
      block_smooth(a, S.phi[l], S.rhs[l], S.phi2[l], omega);
      block_smooth(a, S.phi2[l], S.rhs[l], S.phi[l], omega);
    }
    const LevelArgsT<T>& ca = S.a[l + 1];
    const int ncc = ca.n[0] * ca.n[1] * ca.n[2];
    // the residual of every fine cell at once, then the coarse right side
    // from it (the summing restriction adds the children x fastest, then y, z)
    const int nc = a.n[0] * a.n[1] * a.n[2];
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
      int idx[3] = {c % a.n[0], (c / a.n[0]) % a.n[1], c / (a.n[0] * a.n[1])};
      S.res[l][c] = S.rhs[l][c] - apply_A(a, S.phi[l], idx, c);
    }
    __syncthreads();
    for (int C = threadIdx.x; C < ncc; C += blockDim.x) {
      int I[3] = {C % ca.n[0], (C / ca.n[0]) % ca.n[1], C / (ca.n[0] * ca.n[1])};
      T r;
      if (S.transpose) {
        r = restrict_transpose(a, S.res[l], ca.n, I);
      } else {
        r = (T)0;
        const int nz = (a.dim == 3) ? 2 : 1;
        for (int sz = 0; sz < nz; ++sz)
          for (int sy = 0; sy < 2; ++sy)
            for (int sx = 0; sx < 2; ++sx)
              r += S.res[l][2 * I[0] + sx + a.n[0] * (2 * I[1] + sy + a.n[1] * ((a.dim == 3) ? 2 * I[2] + sz : 0))];
      }
      S.rhs[l + 1][C] = r;
      S.phi[l + 1][C] = 0.0;
    }
    __syncthreads();
  }
  {
    const LevelArgsT<T>& a = S.a[last];
    const int ncl = a.n[0] * a.n[1] * a.n[2];
    const int maxit = min(2000, 2 * ncl + 20);
    if (S.cinv) {
      // exact coarsest solve by the precomputed inverse (the pseudo-inverse on
      // the zero-mean space when singular): x_i = sum_j Minv_ij b_j
      __shared__ T lb[DENSE_MAX];
      double bmean = 0.0;
      if (singular) {
        double sb = 0.0;
        for (int c = threadIdx.x; c < ncl; c += blockDim.x) sb += (double)S.rhs[last][c];
        bmean = block_allsum(sb) / ncl;
      }
      for (int c = threadIdx.x; c < ncl; c += blockDim.x) lb[c] = (T)((double)S.rhs[last][c] - bmean);
      __syncthreads();
      // the workgroup's threads split the columns into ng groups (thread
      // i + ncl g takes rows i, columns j = g mod ng), so that each thread has
      // ncl / ng loads to wait for instead of ncl; the groups' sums are added
      // in group order
      const int ng = ncl <= (int)blockDim.x ? (int)blockDim.x / ncl : 1;
      __shared__ T part[1024];
      for (int t = threadIdx.x; t < ncl * ng; t += blockDim.x) {
        const int i = t % ncl, g = t / ncl;
        // eight running sums, so that eight loads of the inverse are in flight
        T acc[8] = {(T)0, (T)0, (T)0, (T)0, (T)0, (T)0, (T)0, (T)0};
        int j = g;
        for (; j + 7 * ng < ncl; j += 8 * ng) {
#pragma unroll
          for (int u = 0; u < 8; ++u) acc[u] += S.cinv[(size_t)(j + u * ng) * ncl + i] * lb[j + u * ng];
        }
        for (; j < ncl; j += ng) acc[0] += S.cinv[(size_t)j * ncl + i] * lb[j];
        part[t] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
      }
      __syncthreads();
      for (int i = threadIdx.x; i < ncl; i += blockDim.x) {
        T acc = part[i];
        for (int g = 1; g < ng; ++g) acc += part[i + ncl * g];
        S.phi[last][i] = acc;
      }
      __syncthreads();
    } else if (ncl <= COARSE_LDS) {
      // coarsest level held in LDS: operator, potential, right side, CG vectors
      __shared__ T lphi[COARSE_LDS], lrhs[COARSE_LDS], ldiag[COARSE_LDS];
      __shared__ T lr[COARSE_LDS], lp[COARSE_LDS], lq[COARSE_LDS];
      __shared__ T lS[9][COARSE_LDS];
      LevelArgsT<T> la = a;
      for (int c = threadIdx.x; c < ncl; c += blockDim.x) {
        lphi[c] = S.phi[last][c];
        lrhs[c] = S.rhs[last][c];
        ldiag[c] = a.diag[c];
        for (int k = 0; k < 9; ++k)
          if (a.S[k]) lS[k][c] = a.S[k][c];
      }
      la.diag = ldiag;
      for (int k = 0; k < 9; ++k) la.S[k] = a.S[k] ? lS[k] : nullptr;
      __syncthreads();
      if (threadIdx.x < 64) wave_cg(la, lphi, lrhs, lr, lp, lq, maxit, singular, coarse_tol2);
      __syncthreads();
      for (int c = threadIdx.x; c < ncl; c += blockDim.x) S.phi[last][c] = lphi[c];
      __syncthreads();
    } else {
      block_cg(a, S.phi[last], S.rhs[last], S.res[last], S.aux[last], S.phi2[last], maxit, singular, coarse_tol2);
    }
  }
  for (int l = last - 1; l >= 0; --l) {
    const LevelArgsT<T>& a = S.a[l];
    const LevelArgsT<T>& ca = S.a[l + 1];
    const int nc = a.n[0] * a.n[1] * a.n[2];
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
      int idx[3] = {c % a.n[0], (c / a.n[0]) % a.n[1], c / (a.n[0] * a.n[1])};
      S.phi[l][c] += prolong_cell(a, S.phi[l + 1], ca.n, idx);
    }
    __syncthreads();
    for (int s = 0; s < nu2; s += 2) {
      block_smooth(a, S.phi[l], S.rhs[l], S.phi2[l], omega);
      block_smooth(a, S.phi2[l], S.rhs[l], S.phi[l], omega);
    }
  }

  }
};

__global__ void residual_norm_kernel(LevelArgs a, const double* __restrict__ phi,
                                     const double* __restrict__ rhs, double* partials,
                                     const int* flag) {
  if (flag[0]) return;
  const Tile3 T3 = xcd_tile();
  const int i = T3.bx * blockDim.x + threadIdx.x;
  const int j = T3.by * blockDim.y + threadIdx.y;
  const int k = T3.bz;
  double rr = 0.0;
  if (i < a.n[0] && j < a.n[1]) {
    const int idx[3] = {i, j, k};
    const int c = i + a.n[0] * (j + a.n[1] * k);
    double r = rhs[c] - apply_A(a, phi, idx, c);
    rr = r * r;
  }
  double t = block_sum(rr);
  if (threadIdx.x == 0 && threadIdx.y == 0)
    partials[T3.blk] = t;
}

// start of a solve: not converged, no cycle done, at most `cap` cycles (a
// solve launched with more, as a batch of cases launches the largest count,
// stops at its own)
struct mg_reset_kernelOp {
  static constexpr int KIND = BK_RESET, BOUND = 256;
  struct Args {
    int* flag;
    int cap;
  };
  static __device__ void body(const Args& k_, const Blk& b_) {
    int* flag = k_.flag;
    flag[0] = 0;
    flag[1] = 0;
    flag[2] = k_.cap;
  }
};

static dim3 grid3(const Level& L) {
  return dim3((unsigned)((L.n[0] + 63) / 64), (unsigned)((L.n[1] + 3) / 4), (unsigned)L.n[2]);
}
static const dim3 BLOCK3(64, 4, 1);

template <typename T> static const T* coarse_inverse(const GridCtx& G);
template <> const double* coarse_inverse<double>(const GridCtx& G) { return G.cinv64; }
template <> const float* coarse_inverse<float>(const GridCtx& G) { return G.cinv32; }

// column j of the coarsest operator, A e_j (one workgroup per column)
__global__ __launch_bounds__(256) void dense_operator_kernel(LevelArgs a, double* M) {
  __shared__ double e[DENSE_MAX];
  const int n = a.n[0] * a.n[1] * a.n[2];
  const int j = blockIdx.x;
  for (int c = threadIdx.x; c < n; c += blockDim.x) e[c] = c == j ? 1.0 : 0.0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int idx[3] = {i % a.n[0], (i / a.n[0]) % a.n[1], i / (a.n[0] * a.n[1])};
    M[(size_t)j * n + i] = apply_A(a, (const double*)e, idx, i);
  }
}

// Dense inverse of the coarsest operator (at set-up, on the host by
// Gauss-Jordan elimination with partial pivoting).  Singular (all-periodic)
// problems: A has the constant null vector 1 and 1^T A = 0, so
// B = A - beta 1 1^T is invertible and for zero-sum b the solution of B x = b
// has zero sum and solves A x = b.  The inverse is stored in FP64 and FP32.
void launch_dense_galerkin(const GridCtx& G, double* M, hipStream_t st);
int setup_coarse_inverse(GridCtx& G, hipStream_t st) {
  if (!G.cinv64) return 0;
  const int l = G.coarse;
  const int n = (int)G.lev[l].ncells;
  LevelArgs a = level_args(G, l);
  if (G.boxmg)
    launch_dense_galerkin(G, G.cinv64, st);
  else
    hipLaunchKernelGGL(dense_operator_kernel, dim3(n), dim3(256), 0, st, a, G.cinv64);
  std::vector<double> M((size_t)n * n), Inv((size_t)n * n, 0.0);
  if (hipMemcpyAsync(M.data(), G.cinv64, sizeof(double) * M.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return -1;
  if (G.all_periodic) {
    double dsum = 0.0;
    for (int i = 0; i < n; ++i) dsum += M[(size_t)i * n + i];
    const double beta = dsum / n / n;  // B's eigenvalue on 1 is -beta n, about the mean diagonal
    for (double& v : M) v -= beta;
  }
  // row-major working copy (A symmetric, so the column-major M reads the same)
  for (int i = 0; i < n; ++i) Inv[(size_t)i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(M[(size_t)r * n + c]) > fabs(M[(size_t)piv * n + c])) piv = r;
    if (M[(size_t)piv * n + c] == 0.0) return -1;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(M[(size_t)piv * n + k], M[(size_t)c * n + k]);
        std::swap(Inv[(size_t)piv * n + k], Inv[(size_t)c * n + k]);
      }
    const double inv = 1.0 / M[(size_t)c * n + c];
    for (int k = 0; k < n; ++k) {
      M[(size_t)c * n + k] *= inv;
      Inv[(size_t)c * n + k] *= inv;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = M[(size_t)r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        M[(size_t)r * n + k] -= f * M[(size_t)c * n + k];
        Inv[(size_t)r * n + k] -= f * Inv[(size_t)c * n + k];
      }
    }
  }
  // column-major storage for the device (thread i reads row i along j):
  // element (i, j) at j * n + i
  std::vector<double> T64((size_t)n * n);
  std::vector<float> T32((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      T64[(size_t)j * n + i] = Inv[(size_t)i * n + j];
      T32[(size_t)j * n + i] = (float)Inv[(size_t)i * n + j];
    }
  if (hipMemcpyAsync(G.cinv64, T64.data(), sizeof(double) * T64.size(), hipMemcpyHostToDevice, st) != hipSuccess)
    return -1;
  if (G.cinv32 &&
      hipMemcpyAsync(G.cinv32, T32.data(), sizeof(float) * T32.size(), hipMemcpyHostToDevice, st) != hipSuccess)
    return -1;
  return hipStreamSynchronize(st) == hipSuccess ? 0 : -1;
}

static int first_small_level(const GridCtx& G) {
  int ls = G.nlev - 1;
  while (ls > 0 && G.lev[ls - 1].ncells <= SMALL_CELLS && G.nlev - (ls - 1) <= MAX_SMALL) --ls;
  return ls;
}

// nu (even) Chebyshev smoothing steps on level l, targeting the upper part
// [lam_max / 8, lam_max] of the spectrum of D^-1 A (the modes the coarse grid
// cannot represent), lam_max from the Gershgorin bound; phi and phi2 alternate
// and the result ends in phi.  With partials != null the last step sums the
// squared residual of its input.
template <typename T>
static T* chebyshev(const GridCtx& G, int l, int nu, double* partials, hipStream_t st,
                   double* first_partials = nullptr, double rtol2 = 0.0, bool first_done = false,
                   T* start = nullptr) {
  const Level& L = G.lev[l];
  const LevelArgsT<T> a = level_args_t<T>(G, l);
  const LevelVec<T> v = level_vec<T>(G, l);
  const int zp = L.ncells >= SMOOTH_ZP_CELLS ? smooth_kernelOp<T>::ZP : 1;
  const dim3 gr(grid3(L).x, grid3(L).y, (unsigned)((L.n[2] + zp - 1) / zp));
  const double lmax = L.lam_max, lmin = L.lam_max / 8.0;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
  double rho = 1.0 / sigma;
  // the sweeps alternate between the start buffer (phi unless given) and the
  // other one; first_done: the step from the zero guess was taken by the
  // kernel that wrote the right side (phi2 and aux hold it)
  T* A = start ? start : v.phi;
  T* B = A == v.phi ? v.phi2 : v.phi;
  for (int s = first_done ? 1 : 0; s < nu; ++s) {
    const T* in = (s & 1) ? B : A;
    T* out = (s & 1) ? A : B;
    double cr, cd;
    if (s == 0) {
      cr = 1.0 / theta;
      cd = 0.0;
    } else {
      const double rn = 1.0 / (2.0 * sigma - rho);
      cr = 2.0 * rn / delta;
      cd = rn * rho;
      rho = rn;
    }
    const bool last = s + 1 == nu;
    double* pp = last ? partials : (s == 0 ? first_partials : nullptr);
    const T* dprev = s == 0 ? nullptr : v.aux;
    T* dout = last ? nullptr : v.aux;
    bool done = false;
    if constexpr (sizeof(T) == 4) {
      if (L.h_diag) {
        const LevelArgsT<float, __half> ah = level_args_h(G, l);
        op_launch<smooth_kernelOp<float, __half>>(gr, BLOCK3, typename smooth_kernelOp<float, __half>::Args{ah, in, (const T*)v.rhs, out, cr, cd, dprev, dout, (const int*)G.mg_flag, pp, zp}, st);
        done = true;
      }
    }
    if (!done)
      op_launch<smooth_kernelOp<T>>(gr, BLOCK3, typename smooth_kernelOp<T>::Args{a, in, (const T*)v.rhs, out, cr, cd, dprev, dout, (const int*)G.mg_flag, pp, zp}, st);
    if (s == 0 && first_partials) {
      // the residual entering the first step is the solve's initial residual:
      // stop here when the initial guess already meets the tolerance
      const int nblk = (int)(gr.x * gr.y * gr.z);
      op_launch<reduce_final_kernelOp>(dim3(1), dim3(1024), reduce_final_kernelOp::Args{(const double*)first_partials, nblk, G.scalars + 1, 1, rtol2, (const double*)(G.scalars + 0), G.mg_flag, 0}, st);
    }
  }
  return (nu & 1) ? B : A;
}

// Largest ratio of a cell's face coefficients (w_a = J g^aa dV / h_a^2) on
// level 0: the operator's anisotropy.
__global__ __launch_bounds__(256) void anisotropy_kernel(LevelArgs a, unsigned* out) {
  const long long nc = (long long)a.n[0] * a.n[1] * a.n[2];
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  double wmax = 0.0, wmin = 1e300;
  for (int ax = 0; ax < a.dim; ++ax) {
    const double w = a.wf[ax][c];
    wmax = fmax(wmax, w);
    wmin = fmin(wmin, w);
  }
  if (wmin > 0.0) atomicMax(out, __float_as_uint((float)(wmax / wmin)));
}

// Upper spectral bound of D^-1 A on every level (once, at set-up), and the
// restriction: the transpose of the prolongation on operators whose face
// coefficients differ by more than ANISO_TRANSPOSE within a cell.
int compute_smoother_bounds(GridCtx& G, hipStream_t st) {
  {
    const Level& L = G.lev[0];
    unsigned* tmp = (unsigned*)G.mg_flag + 3;  // scratch word ([2] is the cycle budget of a solve)
    launch_fill_u8(tmp, 0, sizeof(unsigned), st);
    hipLaunchKernelGGL(anisotropy_kernel, dim3((unsigned)((L.ncells + 255) / 256)), dim3(256), 0, st, level_args(G, 0),
                       tmp);
    unsigned bits = 0;
    if (hipMemcpyAsync(&bits, tmp, sizeof(bits), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return -1;
    float ratio;
    memcpy(&ratio, &bits, sizeof(ratio));
    G.anisotropy = ratio;
    G.restrict_transpose = ratio > ANISO_TRANSPOSE ? 1 : 0;
  }
  for (int l = 0; l < G.nlev; ++l) {
    Level& L = G.lev[l];
    LevelArgs a = level_args(G, l);
    hipLaunchKernelGGL(gershgorin_kernel, grid3(L), BLOCK3, 0, st, a, L.res);
    std::vector<double> h((size_t)L.ncells);
    if (hipMemcpyAsync(h.data(), L.res, sizeof(double) * (size_t)L.ncells, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return -1;
    double m = 0.0;
    for (double v : h) m = v > m ? v : m;
    L.lam_max = 1.0 + m;
  }
  return 0;
}

// phi <- 2 phi - prev, prev <- old phi (linear extrapolation in time of the
// initial guess); with extrapolate = 0 only prev <- phi.
struct extrapolate_kernelOp {
  static constexpr int KIND = BK_EXTRAP, BOUND = 256;
  struct Args {
    long long n;
    double* phi;
    double* prev;
    int extrapolate;
  };
  static __device__ void body(const Args& k_, const Blk& b_) {
    long long n = k_.n;
    double* phi = k_.phi;
    double* prev = k_.prev;
    int extrapolate = k_.extrapolate;

  long long c = (long long)b_.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const double t = phi[c];
  if (extrapolate) phi[c] = 2.0 * t - prev[c];
  prev[c] = t;

  }
};

void launch_extrapolate_guess(const GridCtx& G, int extrapolate, hipStream_t st) {
  const Level& L = G.lev[0];
  unsigned blocks = (unsigned)((L.ncells + 255) / 256);
  op_launch<extrapolate_kernelOp>(dim3(blocks), dim3(256), extrapolate_kernelOp::Args{L.ncells, L.phi, G.phi_prev, extrapolate}, st);
}

// nu sweeps of segment line relaxation along every axis (phi -> phi2 -> phi ...;
// nu * dim is even, so the result is back in phi)
template <typename T>
static void line_sweeps(const GridCtx& G, int l, int nu, bool reverse, hipStream_t st) {
  if (batch_unsupported()) return;
  const Level& L = G.lev[l];
  const LevelArgsT<T> a = level_args_t<T>(G, l);
  const LevelVec<T> v = level_vec<T>(G, l);
  const int d = G.g.dim;
  int k = 0;
  for (int s = 0; s < nu; ++s)
    for (int q = 0; q < d; ++q, ++k) {
      const int ax = reverse ? d - 1 - q : q;
      const T* in = (k & 1) ? v.phi2 : v.phi;
      T* out = (k & 1) ? v.phi : v.phi2;
      const long long nseg = (L.n[ax] + LINE_SEG - 1) / LINE_SEG;
      const long long nthreads = nseg * (L.ncells / L.n[ax]);
      const dim3 blocks((unsigned)((nthreads + 255) / 256));
      if (ax == 0)
        hipLaunchKernelGGL(line_x_kernel<T>, blocks, dim3(256), 0, st, a, in, (const T*)v.rhs, out, (T)LINE_OMEGA,
                           (const int*)G.mg_flag);
      else
        hipLaunchKernelGGL(line_yz_kernel<T>, blocks, dim3(256), 0, st, a, ax, in, (const T*)v.rhs, out,
                           (T)LINE_OMEGA, (const int*)G.mg_flag);
    }
}

// whether the smoothing of a multi-workgroup level is the segment line
// relaxation (FP32 preconditioner of an anisotropic operator)
static bool line_level(const GridCtx& G, int nu, bool fp32) {
  const int nl = G.g.dim == 2 ? nu / 2 : nu;
  return fp32 && G.anisotropy > LINE_ANISO && nl > 0 && (nl * G.g.dim) % 2 == 0;
}
static int first_small_level(const GridCtx& G);
template <typename T>
static FirstSweepT<T> first_sweep(const GridCtx& G, int l, int nu) {
  FirstSweepT<T> f;
  memset(&f, 0, sizeof(f));
  if (l >= first_small_level(G) || nu < 1 || line_level(G, nu, sizeof(T) == 4)) return f;
  const LevelVec<T> v = level_vec<T>(G, l);
  const double lmax = G.lev[l].lam_max, lmin = lmax / 8.0;
  f.diag = level_args_t<T>(G, l).diag;
  f.phi2 = v.phi2;
  f.aux = v.aux;
  f.cr = 1.0 / (0.5 * (lmax + lmin));
  return f;
}

// the smoother of a multi-workgroup level: segment line relaxation for the
// preconditioner of an anisotropic operator (its summed residual is not
// needed there), Chebyshev otherwise
template <typename T>
static T* smooth_level(const GridCtx& G, int l, int nu, bool post, double* partials, hipStream_t st,
                       double* first_partials = nullptr, double rtol2 = 0.0, bool first_done = false,
                       T* start = nullptr) {
  if constexpr (sizeof(T) == 4) {
    // one sweep along every axis in place of two point-smoothing steps (2D;
    // in 3D two, so that the result ends in phi), the post-smoothing in
    // reverse axis order so that the V-cycle stays symmetric
    const int nl = G.g.dim == 2 ? nu / 2 : nu;
    const T* phi = level_vec<T>(G, l).phi;
    if (G.anisotropy > LINE_ANISO && !partials && !first_partials && nl > 0 && (nl * G.g.dim) % 2 == 0 &&
        (!start || start == phi)) {
      line_sweeps<T>(G, l, nl, post, st);
      return level_vec<T>(G, l).phi;
    }
  }
  return chebyshev<T>(G, l, nu, partials, st, first_partials, rtol2, first_done, start);
}

// One V-cycle from level l in precision T.  With partials != null, the last
// smoothing sweep on level 0 also sums the squared residual (of its input) per
// block.
// Returns the buffer holding the level's result (phi, or phi2 after an odd
// number of sweeps).
template <typename T>
static T* vcycle(const GridCtx& G, int l, int nu1, int nu2, double* partials, hipStream_t st,
                 double* first_partials = nullptr, double rtol2 = 0.0, bool first_done = false) {
  const int ls = first_small_level(G);
  if (l >= ls) {
    SmallLevels<T> S;
    memset(&S, 0, sizeof(S));
    S.nl = G.nlev - l;
    S.cinv = coarse_inverse<T>(G);
    S.transpose = G.restrict_transpose;
    for (int k = 0; k < S.nl; ++k) {
      const LevelVec<T> v = level_vec<T>(G, l + k);
      S.a[k] = level_args_t<T>(G, l + k);
      S.phi[k] = v.phi;
      S.phi2[k] = v.phi2;
      S.rhs[k] = v.rhs;
      S.res[k] = v.res;
      S.aux[k] = v.aux;
    }
    // Inside a V-cycle the coarsest level needs only a modest relative residual
    // (1e-6); when it is the whole grid of an FP64 solve it is solved to 1e-13.
    const double coarse_tol2 = (l == 0 && S.nl == 1 && sizeof(T) == 8) ? 1e-26 : 1e-12;
    op_launch<small_vcycle_kernelOp<T>>(dim3(1), dim3(1024), typename small_vcycle_kernelOp<T>::Args{S, nu1, nu2, coarse_tol2, G.all_periodic, (const int*)G.mg_flag}, st);
    return S.phi[0];
  }
  const Level& L = G.lev[l];
  const LevelArgsT<T> a = level_args_t<T>(G, l);
  const LevelVec<T> v = level_vec<T>(G, l);
  const dim3 gr = grid3(L);
  T* cur = smooth_level<T>(G, l, nu1, false, nullptr, st, first_partials, rtol2, first_done);
  const Level& C = G.lev[l + 1];
  const LevelVec<T> cv = level_vec<T>(G, l + 1);
  bool coarse_first = false;
  if (G.restrict_transpose) {
    op_launch<residual_kernelOp<T>>(gr, BLOCK3, typename residual_kernelOp<T>::Args{a, (const T*)cur, (const T*)v.rhs, v.res, (const int*)G.mg_flag}, st);
    op_launch<restrict_kernelOp<T>>(grid3(C), BLOCK3, typename restrict_kernelOp<T>::Args{a, (const T*)v.res, C.n[0], C.n[1], C.n[2], cv.rhs, cv.phi, (const int*)G.mg_flag}, st);
  } else {
    // residual and summing restriction in one pass, with the coarse level's
    // first smoothing step from its zero guess
    const FirstSweepT<T> fs = first_sweep<T>(G, l + 1, nu1);
    coarse_first = fs.diag != nullptr;
    const dim3 rg((unsigned)((L.n[0] + 63) / 64), (unsigned)((L.n[1] + 3) / 4), (unsigned)C.n[2]);
    bool done = false;
    if constexpr (sizeof(T) == 4) {
      if (L.h_diag) {
        const LevelArgsT<float, __half> ah = level_args_h(G, l);
        op_launch<resrestrict_kernelOp<float, __half>>(rg, dim3(64, 4, 1), typename resrestrict_kernelOp<float, __half>::Args{ah, (const T*)cur, (const T*)v.rhs, C.n[0], C.n[1], cv.rhs, cv.phi, fs, (const int*)G.mg_flag}, st);
        done = true;
      }
    }
    if (!done)
      op_launch<resrestrict_kernelOp<T>>(rg, dim3(64, 4, 1), typename resrestrict_kernelOp<T>::Args{a, (const T*)cur, (const T*)v.rhs, C.n[0], C.n[1], cv.rhs, cv.phi, fs, (const int*)G.mg_flag}, st);
  }
  const T* ce = vcycle<T>(G, l + 1, nu1, nu2, nullptr, st, nullptr, 0.0, coarse_first);
  {
    // two fine cells per thread along z on large levels (more loads in flight)
    const int zp = L.ncells >= SMOOTH_ZP_CELLS ? 2 : 1;
    const dim3 pg(gr.x, gr.y, (unsigned)((L.n[2] + zp - 1) / zp));
    op_launch<prolong_kernelOp<T>>(pg, BLOCK3, typename prolong_kernelOp<T>::Args{a, cur, ce, C.n[0], C.n[1], C.n[2], (const int*)G.mg_flag, zp}, st);
  }
  return smooth_level<T>(G, l, nu2, true, partials, st, nullptr, 0.0, false, cur);
}

// ----------------------------------------------------------------------------
// Flexible conjugate gradients, truncated to one previous direction, with one
// V-cycle (zero initial guess) as the preconditioner.  The V-cycle is not a
// symmetric operator (summing restriction, bilinear prolongation), which the
// flexible form tolerates; the outer iteration removes the few modes a
// V-cycle alone amplifies on strongly distorted, anisotropic grids.  The
// V-cycle runs on the FP32 copy of the hierarchy (it only has to approximate
// A^-1); the outer iteration keeps x, r and the operator in FP64, so the
// attainable residual is that of FP64.  Per iteration k (A symmetric,
// p_{k-1} . r_k = 0 by the choice of alpha):
//   z = V(r), w = A z,
//   beta = -(q_{k-1} . z) / (p_{k-1} . q_{k-1})          (0 on the first),
//   p = z + beta p_{k-1},  q = A p = w + beta q_{k-1},
//   p . q = z . w + 2 beta (q_{k-1} . z) + beta^2 (p_{k-1} . q_{k-1}),
//   alpha = (z . r) / (p . q),  x += alpha p,  r -= alpha q.
// Level 0's FP32 vectors hold z (phi) and the FP32 copy of r (rhs).
// Device scalars: [4] z.w  [5] q.z  [6] z.r  [7] p.q  [8] alpha  [9] beta.
// ----------------------------------------------------------------------------
struct fcg_residual_kernelOp {
  static constexpr int KIND = BK_FCGRES, BOUND = 256;
  struct Args {
    LevelArgs a;
    const double* x;
    const double* b;
    double* r;
    float* r32;
    float* z;
    double* partials;
    const int* flag;
    FirstSweep fs;
    int zp;  // cells per thread along z (1 or 2; the grid's z extent is ceil(n2 / zp))
  };
  static __device__ void body(const Args& k_, const Blk& b_) {
    const LevelArgs& a = k_.a;
    const double* __restrict__ x = k_.x;
    const double* __restrict__ b = k_.b;
    double* r = k_.r;
    float* r32 = k_.r32;
    float* z = k_.z;
    double* partials = k_.partials;
    const int* flag = k_.flag;

  if (flag[0]) return;
  const Tile3 T3 = xcd_tile(b_);
  const int i = T3.bx * blockDim.x + threadIdx.x;
  const int j = T3.by * blockDim.y + threadIdx.y;
  double rr = 0.0;
  if (i < a.n[0] && j < a.n[1]) {
    double vz[2];
    int cz[2] = {-1, -1};
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
      const int k = T3.bz * k_.zp + dz;
      vz[dz] = 0.0;
      if (dz < k_.zp && k < a.n[2]) {
        const int idx[3] = {i, j, k};
        cz[dz] = i + a.n[0] * (j + a.n[1] * k);
        vz[dz] = b[cz[dz]] - apply_A(a, x, idx, cz[dz]);
      }
    }
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
      const int c = cz[dz];
      if (c < 0) continue;
      const double v = vz[dz];
      r[c] = v;
      r32[c] = (float)v;
      if (k_.fs.diag)
        k_.fs.apply(c, (float)v);
      else
        z[c] = 0.0f;
      rr += v * v;
    }
  }
  const double t = block_sum(rr);
  if (threadIdx.x == 0 && threadIdx.y == 0) partials[T3.blk] = t;

  }
};

// w = A z and the block sums of z.w, q.z (first iteration: 0), z.r
struct fcg_apply_kernelOp {
  static constexpr int KIND = BK_FCGAPPLY, BOUND = 256;
  struct Args {
    LevelArgs a;
    const float* z;
    const double* r;
    const double* q;
    double* w;
    double* partials;
    int nblk;
    int first;
    const int* flag;
    int zp;  // cells per thread along z (1 or 2)
  };
  static __device__ void body(const Args& k_, const Blk& b_) {
    const LevelArgs& a = k_.a;
    const float* __restrict__ z = k_.z;
    const double* __restrict__ r = k_.r;
    const double* __restrict__ q = k_.q;
    double* w = k_.w;
    double* partials = k_.partials;
    int nblk = k_.nblk;
    int first = k_.first;
    const int* flag = k_.flag;

  if (flag[0]) return;
  const Tile3 T3 = xcd_tile(b_);
  const int i = T3.bx * blockDim.x + threadIdx.x;
  const int j = T3.by * blockDim.y + threadIdx.y;
  double zw = 0.0, qz = 0.0, zr = 0.0;
  if (i < a.n[0] && j < a.n[1]) {
    double wz[2];
    int cz[2] = {-1, -1};
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
      const int k = T3.bz * k_.zp + dz;
      wz[dz] = 0.0;
      if (dz < k_.zp && k < a.n[2]) {
        const int idx[3] = {i, j, k};
        cz[dz] = i + a.n[0] * (j + a.n[1] * k);
        wz[dz] = apply_A(a, z, idx, cz[dz]);
      }
    }
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
      const int c = cz[dz];
      if (c < 0) continue;
      const double wc = wz[dz];
      const double zc = (double)z[c];
      w[c] = wc;
      zw += zc * wc;
      qz += first ? 0.0 : q[c] * zc;
      zr += zc * r[c];
    }
  }
  const int blk = T3.blk;
  double t = block_sum(zw);
  if (threadIdx.x == 0 && threadIdx.y == 0) partials[blk] = t;
  t = block_sum(qz);
  if (threadIdx.x == 0 && threadIdx.y == 0) partials[nblk + blk] = t;
  t = block_sum(zr);
  if (threadIdx.x == 0 && threadIdx.y == 0) partials[2 * nblk + blk] = t;

  }
};

// one workgroup: the three sums (fixed order), then beta, p.q and alpha
struct fcg_coef_kernelOp {
  static constexpr int KIND = BK_FCGCOEF, BOUND = 1024;
  struct Args {
    const double* partials;
    int nblk;
    double* sc;
    int first;
    const int* flag;
  };
  static __device__ void body(const Args& k_, const Blk& b_) {
    const double* __restrict__ partials = k_.partials;
    int nblk = k_.nblk;
    double* sc = k_.sc;
    int first = k_.first;
    const int* flag = k_.flag;

  if (flag[0]) return;
  double v[3], s[3];
  strided_sums<3, 4>(partials, nblk, nblk, s);
  for (int m = 0; m < 3; ++m) v[m] = block_sum(s[m]);
  if (threadIdx.x == 0) {
    const double zw = v[0], qz = v[1], zr = v[2];
    const double pq_prev = sc[7];
    const double beta = (first || pq_prev == 0.0) ? 0.0 : -qz / pq_prev;
    const double pq = zw + 2.0 * beta * qz + beta * beta * pq_prev;
    sc[4] = zw;
    sc[5] = qz;
    sc[6] = zr;
    sc[7] = pq;
    // A and the V-cycle are both negative definite (on the zero-mean space
    // when singular), so p.q and z.r share their sign; p.q = 0 only once r = 0
    sc[8] = pq != 0.0 ? zr / pq : 0.0;
    sc[9] = beta;
  }

  }
};

// p, q, x, r updated; the FP32 copy of r and a cleared z for the next V-cycle;
// block sums of |r|^2
struct fcg_update_kernelOp {
  static constexpr int KIND = BK_FCGUPD, BOUND = 256;
  struct Args {
    LevelArgs a;
    const double* sc;
    const float* z;  // the preconditioner's result
    float* z0;       // its level-0 start buffer: cleared (zero guess) unless fs takes the first step
    double* p;
    const double* w;
    double* q;
    double* x;
    double* r;
    float* r32;
    int first;
    double* partials;
    const int* flag;
    FirstSweep fs;
    int zp;  // cells per thread along z (1 or 2)
  };
  static __device__ void body(const Args& k_, const Blk& b_) {
    const LevelArgs& a = k_.a;
    const double* __restrict__ sc = k_.sc;
    const float* z = k_.z;
    double* p = k_.p;
    const double* __restrict__ w = k_.w;
    double* q = k_.q;
    double* x = k_.x;
    double* r = k_.r;
    float* r32 = k_.r32;
    int first = k_.first;
    double* partials = k_.partials;
    const int* flag = k_.flag;

  if (flag[0]) return;
  const int i = b_.x * blockDim.x + threadIdx.x;
  const int j = b_.y * blockDim.y + threadIdx.y;
  double rr = 0.0;
  const double alpha = sc[8], beta = sc[9];
  for (int dz = 0; dz < k_.zp; ++dz) {
    const int k = b_.z * k_.zp + dz;
    if (i >= a.n[0] || j >= a.n[1] || k >= a.n[2]) continue;
    const int c = i + a.n[0] * (j + a.n[1] * k);
    const double zc = (double)z[c];
    const double pc = first ? zc : zc + beta * p[c];
    const double qc = first ? w[c] : w[c] + beta * q[c];
    p[c] = pc;
    q[c] = qc;
    x[c] += alpha * pc;
    const double rc = r[c] - alpha * qc;
    r[c] = rc;
    r32[c] = (float)rc;
    if (k_.fs.diag)
      k_.fs.apply(c, (float)rc);
    else
      k_.z0[c] = 0.0f;
    rr += rc * rc;
  }
  const double t = block_sum(rr);
  if (threadIdx.x == 0 && threadIdx.y == 0) partials[b_.x + b_.gx * (b_.y + b_.gy * b_.z)] = t;

  }
};

static void boxmg_vcycle(const GridCtx& G, int l, hipStream_t st);
static int launch_fcg_solve(const GridCtx& G, double rtol2, int max_iter, int nu1, int nu2, hipStream_t st) {
  const Level& L = G.lev[0];
  LevelArgs a = level_args(G, 0);
  // the level-0 kernels of the iteration: two cells per thread along z on
  // large grids (more loads in flight per wave)
  const int zp = L.ncells >= SMOOTH_ZP_CELLS ? 2 : 1;
  const dim3 gr(grid3(L).x, grid3(L).y, (unsigned)((L.n[2] + zp - 1) / zp));
  const int nblk = (int)(gr.x * gr.y * gr.z);
  // the preconditioner's first smoothing step on level 0 (zero guess) is taken
  // by the kernels that write its right side
  FirstSweep fs;
  memset(&fs, 0, sizeof(fs));
  if (!G.boxmg) {
    const FirstSweepT<float> f = first_sweep<float>(G, 0, nu1);
    fs.diag = f.diag;
    fs.phi2 = f.phi2;
    fs.aux = f.aux;
    fs.cr = (float)f.cr;
  }
  op_launch<fcg_residual_kernelOp>(gr, BLOCK3, fcg_residual_kernelOp::Args{a, (const double*)L.phi, (const double*)L.rhs, G.kr, L.f_rhs, L.f_phi, G.mg_partials, (const int*)G.mg_flag, fs, zp}, st);
  op_launch<reduce_final_kernelOp>(dim3(1), dim3(1024), reduce_final_kernelOp::Args{(const double*)G.mg_partials, nblk, G.scalars + 1, 1, rtol2, (const double*)(G.scalars + 0), G.mg_flag, 0}, st);
  for (int it = 0; it < max_iter; ++it) {
    const int first = it == 0;
    // z: the preconditioner's result (level 0's FP32 phi, or phi2 after an
    // odd number of sweeps)
    const float* z = L.f_phi;
    if (G.boxmg)
      boxmg_vcycle(G, 0, st);
    else
      z = vcycle<float>(G, 0, nu1, nu2, nullptr, st, nullptr, 0.0, fs.diag != nullptr);
    op_launch<fcg_apply_kernelOp>(gr, BLOCK3, fcg_apply_kernelOp::Args{a, z, (const double*)G.kr, (const double*)G.kq, G.kw, G.k_partials, nblk, first, (const int*)G.mg_flag, zp}, st);
    op_launch<fcg_coef_kernelOp>(dim3(1), dim3(1024), fcg_coef_kernelOp::Args{(const double*)G.k_partials, nblk, G.scalars, first, (const int*)G.mg_flag}, st);
    op_launch<fcg_update_kernelOp>(gr, BLOCK3, fcg_update_kernelOp::Args{a, (const double*)G.scalars, z, L.f_phi, G.kp, (const double*)G.kw, G.kq, L.phi, G.kr, L.f_rhs, first, G.mg_partials, (const int*)G.mg_flag, fs, zp}, st);
    op_launch<reduce_final_kernelOp>(dim3(1), dim3(1024), reduce_final_kernelOp::Args{(const double*)G.mg_partials, nblk, G.scalars + 1, 1, rtol2, (const double*)(G.scalars + 0), G.mg_flag, 1}, st);
  }
  return max_iter;
}

// FP32 copy of every level's operator (the preconditioner's hierarchy)
__global__ void to_f32_kernel(long long n, const double* __restrict__ src, float* dst) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) dst[c] = (float)src[c];
}

// largest magnitude of an array (as the bits of a non-negative float, whose
// order is that of the unsigned integers)
__global__ void absmax_kernel(long long n, const double* __restrict__ src, unsigned* out) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  float m = c < n ? (float)fabs(src[c]) : 0.0f;
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0 && m > 0.0f) atomicMax(out, __float_as_uint(m));
}

// smallest magnitude of an array (bits of a non-negative float; *out starts
// at +inf)
__global__ void absmin_kernel(long long n, const double* __restrict__ src, unsigned* out) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  float m = c < n ? (float)fabs(src[c]) : __int_as_float(0x7f800000);
  for (int o = 32; o > 0; o >>= 1) m = fminf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMin(out, __float_as_uint(m));
}

__global__ void to_f16_kernel(long long n, const double* __restrict__ src, double scale, __half* dst) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) dst[c] = __float2half_rn((float)(src[c] * scale));
}

// largest ratio of two diagonal entries of a level for its FP16 stencil copy
constexpr float HALF_ROW_RANGE = 64.0f;

int launch_operator_f32(GridCtx& G, hipStream_t st) {
  for (int l = 0; l < G.nlev; ++l) {
    Level& L = G.lev[l];
    if (!L.f_diag) continue;
    const unsigned blocks = (unsigned)((L.ncells + 255) / 256);
    hipLaunchKernelGGL(to_f32_kernel, dim3(blocks), dim3(256), 0, st, L.ncells, (const double*)L.diag, L.f_diag);
    for (int k = 0; k < 9; ++k)
      if (L.S[k] && L.f_S[k])
        hipLaunchKernelGGL(to_f32_kernel, dim3(blocks), dim3(256), 0, st, L.ncells, (const double*)L.S[k], L.f_S[k]);
    if (!L.h_diag) continue;
    // scale 2^-e with 2^e the smallest power of two at or above the largest
    // coefficient: FP16 keeps 11 bits of every coefficient above 2^-14 of it.
    // Operators whose rows differ in scale by more than HALF_ROW_RANGE (the
    // diagonal's range: e.g. the axisymmetric r-z plane, rows ~ r) keep the
    // FP32 stencil: the small rows' coefficients would lose their precision
    // relative to their own row, and the preconditioner its strength
    unsigned* tmp = (unsigned*)G.mg_flag + 3;
    unsigned bits = 0, dbits = 0;
    const unsigned inf_bits = 0x7f800000u;
    if (hipMemcpyAsync(tmp, &inf_bits, sizeof(unsigned), hipMemcpyHostToDevice, st) != hipSuccess) return -1;
    hipLaunchKernelGGL(absmin_kernel, dim3(blocks), dim3(256), 0, st, L.ncells, (const double*)L.diag, tmp);
    if (hipMemcpyAsync(&dbits, tmp, sizeof(dbits), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return -1;
    launch_fill_u8(tmp, 0, sizeof(unsigned), st);
    hipLaunchKernelGGL(absmax_kernel, dim3(blocks), dim3(256), 0, st, L.ncells, (const double*)L.diag, tmp);
    if (hipMemcpyAsync(&bits, tmp, sizeof(bits), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return -1;
    float dmin, dmax;
    memcpy(&dmin, &dbits, sizeof(dmin));
    memcpy(&dmax, &bits, sizeof(dmax));
    if (!(dmin > 0.0f) || !(dmax <= HALF_ROW_RANGE * dmin)) {
      L.h_diag = nullptr;  // (the copies stay allocated, unused)
      continue;
    }
    for (int k = 0; k < 9; ++k)
      if (L.S[k]) hipLaunchKernelGGL(absmax_kernel, dim3(blocks), dim3(256), 0, st, L.ncells, (const double*)L.S[k], tmp);
    if (hipMemcpyAsync(&bits, tmp, sizeof(bits), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return -1;
    float amax;
    memcpy(&amax, &bits, sizeof(amax));
    int e = 0;
    if (amax > 0.0f && std::isfinite(amax)) {
      (void)frexp((double)amax, &e);  // amax = m 2^e, 1/2 <= m < 1
    }
    const double scale = ldexp(1.0, -e);
    L.h_inv = (float)ldexp(1.0, e);
    hipLaunchKernelGGL(to_f16_kernel, dim3(blocks), dim3(256), 0, st, L.ncells, (const double*)L.diag, scale,
                       (__half*)L.h_diag);
    for (int k = 0; k < 9; ++k)
      if (L.S[k] && L.h_S[k])
        hipLaunchKernelGGL(to_f16_kernel, dim3(blocks), dim3(256), 0, st, L.ncells, (const double*)L.S[k], scale,
                           (__half*)L.h_S[k]);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Solve A phi = rhs on level 0 (phi holds the initial guess; the plain
// V-cycles need nu1 + nu2 even, so that their result lands in phi).  Returns the
// number of cycles launched; the number executed is in mg_flag[1].  With the
// Krylov vectors present each cycle is one flexible-CG iteration and the test
// uses the updated residual; with plain V-cycles the test after a cycle uses
// the residual entering its last sweep (an upper bound of the final one in
// practice).
int launch_mg_solve(const GridCtx& G, double rtol, int max_cycles, int nu1, int nu2, hipStream_t st, int cap) {
  const Level& L = G.lev[0];
  LevelArgs a = level_args(G, 0);
  const dim3 gr = grid3(L);
  const int nblk = (int)(gr.x * gr.y * gr.z);
  op_launch<mg_reset_kernelOp>(dim3(1), dim3(1), mg_reset_kernelOp::Args{G.mg_flag, cap > 0 ? cap : max_cycles}, st);
  // |b|^2
  op_launch<reduce_partial_kernelOp>(dim3(FIELD_RED_BLOCKS), dim3(256), reduce_partial_kernelOp::Args{L.rhs, (const double*)nullptr, L.ncells, 2, G.partials, (const int*)nullptr}, st);
  op_launch<reduce_final_kernelOp>(dim3(1), dim3(256), reduce_final_kernelOp::Args{G.partials, FIELD_RED_BLOCKS, G.scalars + 0, 0, 0.0, (const double*)nullptr, (int*)nullptr, 0}, st);
  const double rtol2 = rtol * rtol;
  if (G.kr) return launch_fcg_solve(G, rtol2, max_cycles, nu1, nu2, st);
  if (batch_unsupported()) return max_cycles;
  const bool small = first_small_level(G) == 0;
  if (small) {
    // initial residual (on a multi-workgroup level 0 the first smoothing step
    // of the first cycle computes it)
    hipLaunchKernelGGL(residual_norm_kernel, gr, BLOCK3, 0, st, a, L.phi, L.rhs, G.mg_partials, G.mg_flag);
    op_launch<reduce_final_kernelOp>(dim3(1), dim3(1024), reduce_final_kernelOp::Args{G.mg_partials, nblk, G.scalars + 1, 1, rtol2, G.scalars + 0, G.mg_flag, 0}, st);
  }
  for (int cyc = 0; cyc < max_cycles; ++cyc) {
    if (small) {
      vcycle<double>(G, 0, nu1, nu2, nullptr, st);
      hipLaunchKernelGGL(residual_norm_kernel, gr, BLOCK3, 0, st, a, L.phi, L.rhs, G.mg_partials, G.mg_flag);
    } else {
      vcycle<double>(G, 0, nu1, nu2, G.mg_partials, st, cyc == 0 ? G.mg_partials : nullptr, rtol2);
    }
    op_launch<reduce_final_kernelOp>(dim3(1), dim3(1024), reduce_final_kernelOp::Args{G.mg_partials, nblk, G.scalars + 1, 1, rtol2, G.scalars + 0, G.mg_flag, 1}, st);
  }
  return max_cycles;
}

template <typename R>
__global__ void axpy_scalar_kernel(long long n, const R* __restrict__ x, const double* __restrict__ a, R* y) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += (R)(*a) * x[i];
}

// periodic problems: shift phi so that its J-weighted mean is zero
void launch_gauge(const GridCtx& G, hipStream_t st) {
  if (!G.all_periodic) return;
  const Level& L = G.lev[0];
  reduce(G.Jc, L.phi, L.ncells, 0, G.partials, G.scalars + 2, st);
  unsigned blocks = (unsigned)((L.ncells + 255) / 256);
  op_launch<sub_scalar_kernelOp>(dim3(blocks), dim3(256), sub_scalar_kernelOp::Args{L.ncells, L.phi, G.scalars + 2, 1.0 / G.sumJ}, st);
}

// ----------------------------------------------------------------------------
// vertex field E_v = -k(xi_v)^T (D phi)_v (physical components)
// ----------------------------------------------------------------------------
__device__ inline double phi_ghost(const Geo& g, const int* bclo, const int* bchi, const double* plo,
                                   const double* phh, const double* phi, const int* in_idx) {
  int idx[3] = {in_idx[0], in_idx[1], in_idx[2]};
  double sgn = 1.0, add = 0.0;
  for (int a = 0; a < g.dim; ++a) {
    const int n = g.n[a];
    if (idx[a] >= 0 && idx[a] < n) continue;
    if (g.periodic[a]) {
      idx[a] = wrapi(idx[a], n);
      continue;
    }
    bool lo = idx[a] < 0;
    idx[a] = lo ? 0 : n - 1;
    int bct = lo ? bclo[a] : bchi[a];
    if (bct == BC_DIRICHLET) {
      // ghost = 2 phi_b - phi_in (applied to the value after the other axes)
      add = sgn * 2.0 * (lo ? plo[a] : phh[a]) + add * 1.0;
      sgn = -sgn;
    }
  }
  return add + sgn * phi[idx_to_lin(idx, g.n)];
}

// Tabulated map: the Jacobi matrix at every vertex by finite differences of
// the vertex coordinates (Sec. "Curvilinear formulation"): centred over the
// two neighbours, second-order one-sided over three vertices at the ends of a
// bounded axis; across a periodic seam the neighbour carries a whole period.
__device__ inline double tab_coord(const Geo& g, int a, int i, int jj, int k) {
  int iv[3] = {i, jj, k};
  double per = 0.0;
  long long v = 0, stride = 1;
  for (int b = 0; b < g.dim; ++b) {
    int t = iv[b];
    if (g.periodic[b]) {
      if (t < 0) {
        t += g.n[b];
        if (b == a) per = -1.0;
      } else if (t >= g.n[b]) {
        t -= g.n[b];
        if (b == a) per = 1.0;
      }
    }
    v += stride * t;
    stride *= g.nv[b];
  }
  return g.xtab[v * g.dim + a] + per * g.L[a];
}

__global__ __launch_bounds__(256) void map_table_kernel(Geo g, double* jtab) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= g.nverts) return;
  const int d = g.dim;
  int iv[3] = {(int)(v % g.nv[0]), (int)((v / g.nv[0]) % g.nv[1]), d == 3 ? (int)(v / ((long long)g.nv[0] * g.nv[1])) : 0};
  for (int b = 0; b < d; ++b) {
    const double half_n = 0.5 * g.n[b];
    int lo[3] = {iv[0], iv[1], iv[2]}, hi[3] = {iv[0], iv[1], iv[2]}, far[3] = {iv[0], iv[1], iv[2]};
    const bool interior = g.periodic[b] || (iv[b] > 0 && iv[b] < g.n[b]);
    const int s = interior ? 0 : (iv[b] == 0 ? 1 : -1);  // one-sided: direction into the domain
    if (interior) {
      lo[b] = iv[b] - 1;
      hi[b] = iv[b] + 1;
    } else {
      hi[b] = iv[b] + s;
      far[b] = iv[b] + 2 * s;
    }
    for (int a = 0; a < d; ++a) {
      double dv;
      if (interior) {
        dv = (tab_coord(g, a, hi[0], hi[1], hi[2]) - tab_coord(g, a, lo[0], lo[1], lo[2])) * half_n;
      } else {
        dv = s * (-3.0 * tab_coord(g, a, iv[0], iv[1], iv[2]) + 4.0 * tab_coord(g, a, hi[0], hi[1], hi[2]) -
                  tab_coord(g, a, far[0], far[1], far[2])) * half_n;
      }
      jtab[v * d * d + a * d + b] = dv;
    }
  }
}

void launch_map_table(const Geo& g, double* jtab, hipStream_t st) {
  const unsigned blocks = (unsigned)((g.nverts + 255) / 256);
  hipLaunchKernelGGL(map_table_kernel, dim3(blocks), dim3(256), 0, st, g, jtab);
}

// Inverse Jacobian k = j^-1 of the map at every vertex (FP64, row-major d x d),
// computed once: the vertex field reuses it every step.
__global__ __launch_bounds__(256) void vertex_metric_kernel(Geo g, double* Kv) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= g.nv[0] || y >= g.nv[1]) return;
  const int d = g.dim;
  const long long v = x + (long long)g.nv[0] * (y + (long long)g.nv[1] * z);
  double xi[3] = {x * g.invn[0], y * g.invn[1], (d == 3) ? z * g.invn[2] : 0.0};
  double j[3][3], k[3][3], J;
  map_jacobi(g, xi, j, nullptr);
  inv3(d, j, k, J);
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) Kv[v * d * d + a * d + b] = k[a][b];
}

void launch_vertex_metric(const GridCtx& G, hipStream_t st) {
  const Geo& g = G.g;
  dim3 gr((unsigned)((g.nv[0] + 63) / 64), (unsigned)((g.nv[1] + 3) / 4), (unsigned)(g.dim == 3 ? g.nv[2] : 1));
  hipLaunchKernelGGL(vertex_metric_kernel, gr, dim3(64, 4, 1), 0, st, g, G.Kv);
}

struct FieldBC {
  int bclo[3], bchi[3];
  double plo[3], phh[3];
};

// E_v = -k^T D phi at vertex (x, y, z): D_a is the difference across axis a of
// the 2^d cells around the vertex, averaged over the 2^(d-1) cell pairs.
// Vertices whose cells are all inside the grid (or wrap periodically) read phi
// directly; the others go through the boundary ghosts.  Both paths sum the
// pairs in the same order.
template <int d, typename R>
struct efield_kernelOp {
  static constexpr int KIND = (d == 3 ? kind_of<R>(BK_EF3F, BK_EF3D) : kind_of<R>(BK_EF2F, BK_EF2D)), BOUND = 256;
  struct Args {
    Geo g;
    FieldBC bc;
    const double* phi;
    const double* Kv;
    R* Ev;
  };
  static __device__ void body(const Args& k_, const Blk& b_) {
    const Geo& g = k_.g;
    const FieldBC& bc = k_.bc;
    const double* __restrict__ phi = k_.phi;
    const double* __restrict__ Kv = k_.Kv;
    R* Ev = k_.Ev;

  const int x = b_.x * blockDim.x + threadIdx.x, y = b_.y * blockDim.y + threadIdx.y;
  const int z = b_.z;
  if (x >= g.nv[0] || y >= g.nv[1]) return;
  const int vi[3] = {x, y, z};
  const long long v = x + (long long)g.nv[0] * (y + (long long)g.nv[1] * z);
  // cell index below (lo) and above (hi) the vertex on every axis
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  bool interior = true;
#pragma unroll
  for (int a = 0; a < d; ++a) {
    const int n = g.n[a];
    lo[a] = vi[a] - 1;
    hi[a] = vi[a];
    if (g.periodic[a]) {
      if (lo[a] < 0) lo[a] += n;
      if (hi[a] >= n) hi[a] -= n;
    } else {
      interior = interior && lo[a] >= 0 && hi[a] < n;
    }
  }
  double D[3] = {0.0, 0.0, 0.0};
  constexpr int npair = 1 << (d - 1);
#pragma unroll
  for (int a = 0; a < d; ++a) {
    double s = 0.0;
#pragma unroll
    for (int comb = 0; comb < npair; ++comb) {
      int cp[3] = {0, 0, 0}, cm[3] = {0, 0, 0};
      int bit = 0;
#pragma unroll
      for (int b = 0; b < d; ++b) {
        if (b == a) {
          cp[b] = interior ? hi[b] : vi[b];
          cm[b] = interior ? lo[b] : vi[b] - 1;
        } else {
          const int sb = (comb >> bit) & 1;
          ++bit;
          cp[b] = cm[b] = interior ? (sb ? hi[b] : lo[b]) : vi[b] - 1 + sb;
        }
      }
      if (interior)
        s += phi[cp[0] + g.n[0] * (cp[1] + g.n[1] * cp[2])] - phi[cm[0] + g.n[0] * (cm[1] + g.n[1] * cm[2])];
      else
        s += phi_ghost(g, bc.bclo, bc.bchi, bc.plo, bc.phh, phi, cp) -
             phi_ghost(g, bc.bclo, bc.bchi, bc.plo, bc.phh, phi, cm);
    }
    D[a] = s / (npair * g.invn[a]);
  }
  const double* k = Kv + v * d * d;
  constexpr int EC = (d == 3) ? 4 : 2;
#pragma unroll
  for (int b = 0; b < d; ++b) {
    double e = 0.0;
#pragma unroll
    for (int a = 0; a < d; ++a) e -= k[a * d + b] * D[a];
    Ev[v * EC + b] = (R)e;
  }
  if (d == 3) Ev[v * EC + 3] = (R)0;

  }
};

void launch_efield(const GridCtx& G, hipStream_t st) {
  const Geo& g = G.g;
  FieldBC bc;
  for (int a = 0; a < 3; ++a) {
    bc.bclo[a] = G.bc_lo[a];
    bc.bchi[a] = G.bc_hi[a];
    bc.plo[a] = G.phi_lo[a];
    bc.phh[a] = G.phi_hi[a];
  }
  dim3 gr((unsigned)((g.nv[0] + 63) / 64), (unsigned)((g.nv[1] + 3) / 4), (unsigned)(g.dim == 3 ? g.nv[2] : 1));
  const dim3 bl(64, 4, 1);
  if (g.dim == 3) {
    if (G.fp64)
      op_launch<efield_kernelOp<3, double>>(gr, bl, efield_kernelOp<3, double>::Args{g, bc, G.lev[0].phi, G.Kv, (double*)G.Ev}, st);
    else
      op_launch<efield_kernelOp<3, float>>(gr, bl, efield_kernelOp<3, float>::Args{g, bc, G.lev[0].phi, G.Kv, (float*)G.Ev}, st);
  } else {
    if (G.fp64)
      op_launch<efield_kernelOp<2, double>>(gr, bl, efield_kernelOp<2, double>::Args{g, bc, G.lev[0].phi, G.Kv, (double*)G.Ev}, st);
    else
      op_launch<efield_kernelOp<2, float>>(gr, bl, efield_kernelOp<2, float>::Args{g, bc, G.lev[0].phi, G.Kv, (float*)G.Ev}, st);
  }
  if (G.floating && !batch_unsupported()) {
    // E of phi_0 (wall at 0) plus phi_w times E of phi_1
    const long long n = (long long)g.nverts * (g.dim == 3 ? 4 : 2);
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (G.fp64)
      hipLaunchKernelGGL(axpy_scalar_kernel<double>, dim3(blocks), dim3(256), 0, st, n, (const double*)G.E1,
                         (const double*)(G.scalars + 10), (double*)G.Ev);
    else
      hipLaunchKernelGGL(axpy_scalar_kernel<float>, dim3(blocks), dim3(256), 0, st, n, (const float*)G.E1,
                         (const double*)(G.scalars + 10), (float*)G.Ev);
  }
}

// ----------------------------------------------------------------------------
// Floating conducting wall at the lower face of axis 0 (Sec. "Tests": the
// planar wall charges with the particles it absorbs and Gauss' law holds
// there).  By superposition phi = phi_0 + phi_w phi_1: phi_0 solves the
// problem with the wall at 0, phi_1 the charge-free problem with the wall at
// 1 and every other wall at 0, and phi_w = (Q_w - F(phi_0)) / F(phi_1), where
// F is the discrete flux of E through the wall, sum over its cells of
// 2 w_lo (phi_b - phi_c), and Q_w the absorbed charge.
// ----------------------------------------------------------------------------
__device__ inline double wall_flux_sum(const LevelArgs& a, const double* phi, double phib) {
  const int nw = a.n[1] * a.n[2];
  double f = 0.0;
  for (int t = threadIdx.x; t < nw; t += blockDim.x) {
    const int c = a.n[0] * t;  // cell (0, j, k)
    f += 2.0 * a.wlo[0][c] * (phib - phi[c]);
  }
  return block_sum(f);
}

__global__ __launch_bounds__(1024) void wall_flux_kernel(LevelArgs a, const double* __restrict__ phi, double phib,
                                                         double* out) {
  const double f = wall_flux_sum(a, phi, phib);
  if (threadIdx.x == 0) *out = f;
}

__global__ __launch_bounds__(1024) void floating_wall_kernel(LevelArgs a, const double* __restrict__ phi0,
                                                             WallCharge wc, double* sc) {
  const double F0 = wall_flux_sum(a, phi0, 0.0);
  if (threadIdx.x == 0) {
    double Q = 0.0;
    for (int s = 0; s < wc.nsp; ++s) Q += wc.qw[s] * (double)wc.absorbed[s][0];
    sc[10] = (Q - F0) / sc[12];
    sc[11] = Q;
  }
}

__global__ void phi_full_kernel(long long n, const double* __restrict__ phi0, const double* __restrict__ phi1,
                                const double* __restrict__ sc, double* out) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) out[c] = phi0[c] + sc[10] * phi1[c];
}

void launch_floating_wall(const GridCtx& G, const WallCharge& wc, hipStream_t st) {
  if (batch_unsupported()) return;
  const Level& L = G.lev[0];
  hipLaunchKernelGGL(floating_wall_kernel, dim3(1), dim3(1024), 0, st, level_args(G, 0), (const double*)L.phi, wc,
                     G.scalars);
  const unsigned blocks = (unsigned)((L.ncells + 255) / 256);
  hipLaunchKernelGGL(phi_full_kernel, dim3(blocks), dim3(256), 0, st, L.ncells, (const double*)L.phi,
                     (const double*)G.phi1, (const double*)G.scalars, G.phi_full);
}

// At set-up: phi_1, its vertex field and F(phi_1).
int setup_floating_wall(GridCtx& G, hipStream_t st) {
  if (!G.floating) return 0;
  Level& L = G.lev[0];
  const LevelArgs a = level_args(G, 0);
  const size_t cb = sizeof(double) * (size_t)L.ncells;
  const unsigned blocks = (unsigned)((L.ncells + 255) / 256);
  // wall term of a unit potential on the floating wall alone (the diagonal
  // written to the scratch vector aux is the operator's own)
  hipLaunchKernelGGL(diag_kernel, dim3(blocks), dim3(256), 0, st, a, L.aux, G.bdir1, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0);
  // charge-free solve: rhs = -bdir1 (phi_full serves as the zero charge)
  launch_fill_u8(G.phi_full, 0, cb, st);
  launch_fill_u8(L.phi, 0, cb, st);
  GridCtx G1 = G;
  G1.bdir = G.bdir1;
  G1.charge = G.phi_full;
  launch_rhs(G1, st);
  launch_mg_solve(G1, 1e-13, 200, 2, 2, st);
  if (hipMemcpyAsync(G.phi1, L.phi, cb, hipMemcpyDeviceToDevice, st) != hipSuccess) return -1;
  launch_fill_u8(L.phi, 0, cb, st);
  // its vertex field, with the wall at 1 and every other wall at 0
  GridCtx G2 = G;
  G2.floating = 0;
  G2.lev[0].phi = G.phi1;
  G2.Ev = G.E1;
  for (int ax = 0; ax < 3; ++ax) G2.phi_lo[ax] = G2.phi_hi[ax] = 0.0;
  G2.phi_lo[0] = 1.0;
  launch_efield(G2, st);
  hipLaunchKernelGGL(wall_flux_kernel, dim3(1), dim3(1024), 0, st, a, (const double*)G.phi1, 1.0, G.scalars + 12);
  double F1 = 0.0;
  if (hipMemcpyAsync(&F1, G.scalars + 12, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return -1;
  // a unit wall potential drives a positive flux into a charge-free domain
  if (!(F1 > 0.0)) return -1;
  launch_fill_u8(G.phi_full, 0, cb, st);
  launch_fill_u8(G.scalars + 10, 0, 2 * sizeof(double), st);
  return 0;
}

__global__ void rho_kernel(long long nc, double dV, const double* charge, const double* Jc, double* rho) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  rho[c] = charge[c] / (Jc[c] * dV);
}

void launch_rho(const GridCtx& G, double* rho, hipStream_t st) {
  unsigned blocks = (unsigned)((G.g.ncells + 255) / 256);
  hipLaunchKernelGGL(rho_kernel, dim3(blocks), dim3(256), 0, st, G.g.ncells, G.lev[0].dV, G.charge, G.Jc, rho);
}

void launch_field_energy(const GridCtx& G, double* partials, double* out, hipStream_t st) {
  reduce(G.charge, G.floating ? G.phi_full : G.lev[0].phi, G.g.ncells, 0, partials, out, st, RED_BLOCKS);
  // W_E = 1/2 sum charge phi: the factor is applied by the host
}

// exact 128-bit sum of a uint64 array: per-block (lo, hi) partials, then one block
__global__ __launch_bounds__(256) void qsum_kernel(const unsigned long long* Q, long long n,
                                                   unsigned long long* part) {
  __shared__ unsigned long long slo[256], shi[256];
  unsigned long long lo = 0, hi = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    unsigned long long v = Q[i];
    unsigned long long s = lo + v;
    hi += (s < lo) ? 1ull : 0ull;
    lo = s;
  }
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long L = 0, H = 0;
    for (int t = 0; t < (int)blockDim.x; ++t) {
      unsigned long long s = L + slo[t];
      H += shi[t] + ((s < L) ? 1ull : 0ull);
      L = s;
    }
    part[2 * blockIdx.x] = L;
    part[2 * blockIdx.x + 1] = H;
  }
}
__global__ void qsum_final_kernel(const unsigned long long* part, int nb, unsigned long long* out) {
  unsigned long long L = 0, H = 0;
  for (int b = 0; b < nb; ++b) {
    unsigned long long s = L + part[2 * b];
    H += part[2 * b + 1] + ((s < L) ? 1ull : 0ull);
    L = s;
  }
  out[0] = L;
  out[1] = H;
}

void launch_qsum(const uint64_t* Q, long long n, uint64_t* out2, hipStream_t st) {
  // out2 must have room for 2 + 2 * RED_BLOCKS words (partials follow the result)
  unsigned long long* part = (unsigned long long*)out2 + 2;
  hipLaunchKernelGGL(qsum_kernel, dim3(RED_BLOCKS), dim3(256), 0, st, (const unsigned long long*)Q, n, part);
  hipLaunchKernelGGL(qsum_final_kernel, dim3(1), dim3(1), 0, st, part, RED_BLOCKS, (unsigned long long*)out2);
}

// Count of non-finite entries of x[0..n) (NaN or infinite) added to *bad.
template <typename T>
__global__ __launch_bounds__(256) void nonfinite_kernel(const T* __restrict__ x, long long n, int* bad) {
  int cnt = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    cnt += isfinite(x[i]) ? 0 : 1;
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(bad, cnt);
}
void launch_nonfinite_check(const void* x, long long n, int fp64, int* bad, hipStream_t st) {
  if (n <= 0) return;
  const long long want = (n + 255) / 256;
  const unsigned blocks = (unsigned)(want < RED_BLOCKS ? want : RED_BLOCKS);
  if (fp64)
    hipLaunchKernelGGL(nonfinite_kernel<double>, dim3(blocks), dim3(256), 0, st, (const double*)x, n, bad);
  else
    hipLaunchKernelGGL(nonfinite_kernel<float>, dim3(blocks), dim3(256), 0, st, (const float*)x, n, bad);
}

}  // namespace cpic

namespace cpic {

// ----------------------------------------------------------------------------
// Variational coarse operators and zebra line relaxation (2D)
// ----------------------------------------------------------------------------
// The paper's solver (Sec. "Field solver") builds its coarse operators
// variationally, A_{l+1} = P^T A_l P, and relaxes along grid lines where the
// operator is anisotropic.  Here the two serve as the preconditioner of the
// flexible-CG solve (CPIC_MG_BOXMG, 2D).  P is the cell-centred bilinear
// interpolation of prolong_cell (per axis 3/4 from the own coarse cell and 1/4
// from the neighbour on the fine cell's side; at a wall the neighbour is the
// ghost of the correction, -e behind a Dirichlet wall and e behind a Neumann
// one) and the restriction is its transpose.  With them every coarse operator
// couples a cell with the 5 x 5 block around it: 25 coefficients per cell,
// stored offset-major, coef[o * ncells + c] for the offset (dx, dy) with
// o = dx + 2 + 5 (dy + 2).  The smoother is line Gauss-Seidel in zebra order:
// every line along x, then every line along y, the lines of one colour at a
// time.  The colour count is the smallest that leaves the lines of a colour
// uncoupled (2 for the 9-point level 0, 4 for the 25-point coarse levels), so
// the lines of a colour are relaxed together, one wave per line.

constexpr int GAL_NO = 25;

// interpolation of fine index x along one axis of nc coarse cells: weight wp
// from the own coarse cell p = x / 2, wq from the neighbour q on x's side
// (wrapped on a periodic axis; -1 with wq = 0 behind a wall)
struct GalP {
  int p, q;
  double wp, wq;
};
__device__ inline GalP gal_p(int x, int nc, int periodic, int dir_lo, int dir_hi) {
  GalP r;
  r.p = x >> 1;
  int q = r.p + ((x & 1) ? 1 : -1);
  r.wp = 0.75;
  r.wq = 0.25;
  if (q < 0 || q >= nc) {
    if (periodic) {
      q = q < 0 ? q + nc : q - nc;
    } else {
      r.wp += (q < 0 ? dir_lo : dir_hi) ? -0.25 : 0.25;
      r.wq = 0.0;
      q = -1;
    }
  }
  r.q = q;
  return r;
}

// weight of fine index x in the interpolation from coarse cell I
__device__ inline double gal_w(int x, int I, int nc, int periodic, int dir_lo, int dir_hi) {
  const GalP g = gal_p(x, nc, periodic, dir_lo, dir_hi);
  return (g.p == I ? g.wp : 0.0) + (g.q == I ? g.wq : 0.0);
}

// Coefficient A(c, c + (dx, dy)) of a 2D level: from the 9-point upper-half
// stencil (level 0: diag, S[0] +x, S[1] +y, S[3] +x+y, S[4] +x-y; the lower
// half read at the neighbour) or from 25 offset-major coefficients.  Zero
// when the neighbour lies behind a wall.
template <typename T>
struct Stencil2 {
  int n0, n1, per0, per1;
  const T* diag;
  const T* S[5];  // +x, +y, (unused), +x+y, +x-y
  const T* g25;   // 25 offset-major coefficients, or null for the 9-point form
  __device__ inline bool nb(int i, int j, int dx, int dy, int* c) const {
    int x = i + dx, y = j + dy;
    if (x < 0 || x >= n0) {
      if (!per0) return false;
      x = x < 0 ? x + n0 : x - n0;
    }
    if (y < 0 || y >= n1) {
      if (!per1) return false;
      y = y < 0 ? y + n1 : y - n1;
    }
    *c = x + n0 * y;
    return true;
  }
  __device__ inline T coef(int i, int j, int dx, int dy) const {
    int t;
    if (!nb(i, j, dx, dy, &t)) return (T)0;
    const int c = i + n0 * j;
    if (g25) return g25[(size_t)(dx + 2 + 5 * (dy + 2)) * ((size_t)n0 * n1) + c];
    if (dx == 0 && dy == 0) return diag[c];
    // the pair (c, t) is stored at its lower cell
    const T* s = nullptr;
    int at = c;
    if (dy == 0) {
      s = S[0];
      at = dx > 0 ? c : t;
    } else if (dx == 0) {
      s = S[1];
      at = dy > 0 ? c : t;
    } else if (dx == dy) {
      s = S[3];
      at = dx > 0 ? c : t;
    } else {
      s = S[4];
      at = dx > 0 ? c : t;
    }
    return s ? s[at] : (T)0;
  }
};

template <typename T>
static Stencil2<T> stencil2(const GridCtx& G, int l);
template <>
Stencil2<double> stencil2<double>(const GridCtx& G, int l) {
  const Level& L = G.lev[l];
  Stencil2<double> s;
  s.n0 = L.n[0];
  s.n1 = L.n[1];
  s.per0 = G.g.periodic[0];
  s.per1 = G.g.periodic[1];
  s.diag = L.diag;
  for (int k = 0; k < 5; ++k) s.S[k] = L.S[k];
  s.g25 = l > 0 ? L.gal64 : nullptr;
  return s;
}
template <>
Stencil2<float> stencil2<float>(const GridCtx& G, int l) {
  const Level& L = G.lev[l];
  Stencil2<float> s;
  s.n0 = L.n[0];
  s.n1 = L.n[1];
  s.per0 = G.g.periodic[0];
  s.per1 = G.g.periodic[1];
  s.diag = L.f_diag;
  for (int k = 0; k < 5; ++k) s.S[k] = L.f_S[k];
  s.g25 = l > 0 ? L.gal32 : nullptr;
  return s;
}

// A_{l+1} = P^T A_l P, one thread per coarse cell I: every fine cell f that I
// interpolates to (a 4 x 4 block), every coupling (f, g) of the fine operator,
// every coarse cell J that interpolates to g.  Offsets J - I are taken in
// [-2, 2] (on a periodic axis of 4 coarse cells +2 and -2 name the same cell
// and the coupling is kept under -2).
template <int FR>
__global__ __launch_bounds__(256) void galerkin_kernel(Stencil2<double> A, int nc0, int nc1, int dlo0, int dhi0,
                                                       int dlo1, int dhi1, double* out) {
  const int C = blockIdx.x * blockDim.x + threadIdx.x;
  if (C >= nc0 * nc1) return;
  const int I0 = C % nc0, I1 = C / nc0;
  double acc[GAL_NO];
  for (int o = 0; o < GAL_NO; ++o) acc[o] = 0.0;
  for (int ty = -1; ty <= 2; ++ty) {
    int fy = 2 * I1 + ty;
    if (fy < 0 || fy >= A.n1) {
      if (!A.per1) continue;
      fy = fy < 0 ? fy + A.n1 : fy - A.n1;
    }
    const double wy = gal_w(fy, I1, nc1, A.per1, dlo1, dhi1);
    if (wy == 0.0) continue;
    for (int tx = -1; tx <= 2; ++tx) {
      int fx = 2 * I0 + tx;
      if (fx < 0 || fx >= A.n0) {
        if (!A.per0) continue;
        fx = fx < 0 ? fx + A.n0 : fx - A.n0;
      }
      const double wf = gal_w(fx, I0, nc0, A.per0, dlo0, dhi0) * wy;
      if (wf == 0.0) continue;
      for (int oy = -FR; oy <= FR; ++oy)
        for (int ox = -FR; ox <= FR; ++ox) {
          const double a = A.coef(fx, fy, ox, oy);
          if (a == 0.0) continue;
          int g;
          A.nb(fx, fy, ox, oy, &g);
          const GalP px = gal_p(g % A.n0, nc0, A.per0, dlo0, dhi0);
          const GalP py = gal_p(g / A.n0, nc1, A.per1, dlo1, dhi1);
          const int jx[2] = {px.p, px.q}, jy[2] = {py.p, py.q};
          const double wx[2] = {px.wp, px.wq}, wyy[2] = {py.wp, py.wq};
          for (int b = 0; b < 2; ++b) {
            if (wyy[b] == 0.0) continue;
            int dy = jy[b] - I1;
            if (A.per1) dy = ((dy + 2) % nc1 + nc1) % nc1 - 2;
            for (int q = 0; q < 2; ++q) {
              if (wx[q] == 0.0) continue;
              int dx = jx[q] - I0;
              if (A.per0) dx = ((dx + 2) % nc0 + nc0) % nc0 - 2;
              acc[dx + 2 + 5 * (dy + 2)] += wf * a * wx[q] * wyy[b];
            }
          }
        }
    }
  }
  const size_t nc = (size_t)nc0 * nc1;
  for (int o = 0; o < GAL_NO; ++o) out[(size_t)o * nc + C] = acc[o];
}

__global__ void f64_to_f32_kernel(long long n, const double* __restrict__ a, float* b) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

int setup_galerkin(GridCtx& G, hipStream_t st) {
  if (!G.boxmg) return 0;
  for (int l = 0; l < G.coarse; ++l) {
    const Level& C = G.lev[l + 1];
    const Stencil2<double> A = stencil2<double>(G, l);
    const unsigned blocks = (unsigned)((C.ncells + 255) / 256);
    const int d0 = G.bc_lo[0] == BC_DIRICHLET, e0 = G.bc_hi[0] == BC_DIRICHLET;
    const int d1 = G.bc_lo[1] == BC_DIRICHLET, e1 = G.bc_hi[1] == BC_DIRICHLET;
    if (l == 0)
      hipLaunchKernelGGL(galerkin_kernel<1>, dim3(blocks), dim3(256), 0, st, A, C.n[0], C.n[1], d0, e0, d1, e1,
                         C.gal64);
    else
      hipLaunchKernelGGL(galerkin_kernel<2>, dim3(blocks), dim3(256), 0, st, A, C.n[0], C.n[1], d0, e0, d1, e1,
                         C.gal64);
    const long long n = (long long)GAL_NO * C.ncells;
    hipLaunchKernelGGL(f64_to_f32_kernel, dim3((unsigned)std::min<long long>((n + 255) / 256, 4096)), dim3(256), 0,
                       st, n, (const double*)C.gal64, C.gal32);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// column j of the coarsest operator of the variational hierarchy, A e_j (one
// workgroup per column)
__global__ __launch_bounds__(256) void dense_galerkin_kernel(Stencil2<double> A, double* M) {
  const int n = A.n0 * A.n1;
  const int j = blockIdx.x;
  const int R = A.g25 ? 2 : 1;  // a single-level hierarchy keeps the 9-point level 0
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int i0 = i % A.n0, i1 = i / A.n0;
    double s = 0.0;
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        int t;
        if (A.nb(i0, i1, dx, dy, &t) && t == j) s += A.coef(i0, i1, dx, dy);
      }
    M[(size_t)j * n + i] = s;
  }
}
void launch_dense_galerkin(const GridCtx& G, double* M, hipStream_t st) {
  const int l = G.coarse;
  hipLaunchKernelGGL(dense_galerkin_kernel, dim3((unsigned)G.lev[l].ncells), dim3(256), 0, st,
                     stencil2<double>(G, l), M);
}

// ---- one wave per line: partitioned elimination + cyclic reduction ---------
// The line's tridiagonal system (the couplings along the line; every other
// coupling stays in the residual) is split into K segments of consecutive
// cells, one per lane (K a power of two, at most 64, segments of at least two
// cells).  Each lane eliminates its segment's interior rows, leaving them in
// terms of the segment's first and last unknowns; the first and last rows of
// all segments form a tridiagonal system of 2K rows (cyclic on a periodic
// line), solved by parallel cyclic reduction; the interior follows.  Element i
// of segment k sits at LDS index i + k (one pad word per segment keeps the
// lanes' strided accesses on different banks).
constexpr int LINE_MAXN = 4096;
constexpr int LINE_LDS_WORDS = 3 * (LINE_MAXN + 64) + 4 * 128;

struct LineSeg {
  int K, m, rem;
  __device__ inline int start(int k) const { return k * m + (k < rem ? k : rem); }
  __device__ inline int seg(int i) const {
    const int big = rem * (m + 1);
    return i < big ? i / (m + 1) : rem + (i - big) / m;
  }
};

template <typename T, bool G25>
struct LineRelaxArgs {
  Stencil2<T> A;
  T* x;
  const T* rhs;
  int axis;   // 0: lines along x (one per row j), 1: along y (one per column i)
  int color;  // this launch relaxes the lines color, color + ncolor, ...
  int ncolor;
  const int* flag;
};

template <typename T, bool G25>
__global__ __launch_bounds__(64) void line_relax_kernel(LineRelaxArgs<T, G25> k) {
  if (k.flag[0]) return;
  extern __shared__ float lds[];
  const Stencil2<T>& A = k.A;
  const int ax = k.axis;
  const int n = ax == 0 ? A.n0 : A.n1;          // cells along the line
  const int line = k.color + k.ncolor * blockIdx.x;  // the cross coordinate
  const int per = ax == 0 ? A.per0 : A.per1;
  const int lane = threadIdx.x;
  LineSeg S;
  S.K = 1;
  while (S.K * 2 <= 64 && S.K * 4 <= n) S.K *= 2;
  S.m = n / S.K;
  S.rem = n % S.K;
  const int stride = n + S.K;
  float* Rv = lds;               // rhs, then h
  float* Dv = lds + stride;      // diagonal, then f
  float* Uv = lds + 2 * stride;  // upper coupling, then g
  float* red = lds + 3 * stride; // reduced system: a, b, c, d of 2K rows
  // residual b - A x of every cell of the line and its line couplings
  for (int t = lane; t < n; t += 64) {
    const int i = ax == 0 ? t : line, j = ax == 0 ? line : t;
    const int c = i + A.n0 * j;
    T r = k.rhs[c];
    constexpr int R = G25 ? 2 : 1;
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        int nbc;
        if (!A.nb(i, j, dx, dy, &nbc)) continue;
        r -= A.coef(i, j, dx, dy) * k.x[nbc];
      }
    const int p = t + S.seg(t);
    Rv[p] = (float)r;
    Dv[p] = (float)A.coef(i, j, 0, 0);
    // coupling to the next cell of the line (zero at the end of a bounded line)
    Uv[p] = (float)(ax == 0 ? A.coef(i, j, 1, 0) : A.coef(i, j, 0, 1));
  }
  __syncthreads();
  // this lane's segment [s, e]; its boundary rows before elimination
  const int K = S.K;
  float ra[2] = {0.f, 0.f}, rb[2], rc[2], rd[2];
  const int s = S.start(lane), e = S.start(lane + 1) - 1;
  const int ps = s + lane, pe = e + lane;
  if (lane < K) {
    // a_i = coupling to the previous cell = U of the previous cell
    const int prev = s > 0 ? s - 1 : n - 1;
    ra[0] = (s > 0 || per) ? Uv[prev + S.seg(prev)] : 0.f;
    rb[0] = Dv[ps];
    rc[0] = Uv[ps];
    rd[0] = Rv[ps];
    ra[1] = Uv[pe - 1];  // segments hold at least two cells
    rb[1] = Dv[pe];
    rc[1] = (e < n - 1 || per) ? Uv[pe] : 0.f;
    rd[1] = Rv[pe];
    if (e - s >= 2) {
      // forward over the interior rows s+1 .. e-1 (fill-in on x_s):
      // f_i x_s + x_i + g_i x_{i+1} = h_i
      float a = Uv[ps];  // coupling of row s+1 to row s
      float fp = 0.f, gp = 0.f, hp = 0.f;
      for (int i = s + 1; i < e; ++i) {
        const int p = i + lane;
        const float b = Dv[p], c = Uv[p], d = Rv[p];
        float f, g, h;
        if (i == s + 1) {
          const float im = 1.f / b;
          f = a * im;
          g = c * im;
          h = d * im;
        } else {
          const float im = 1.f / (b - a * gp);
          f = -a * fp * im;
          g = c * im;
          h = (d - a * hp) * im;
        }
        Dv[p] = f;
        Uv[p] = g;
        Rv[p] = h;
        fp = f;
        gp = g;
        hp = h;
        a = c;
      }
      // backward: x_i = h'_i - f'_i x_s - g'_i x_e
      float fn = fp, gn = gp, hn = hp;  // row e-1 as is
      for (int i = e - 2; i > s; --i) {
        const int p = i + lane;
        const float g = Uv[p];
        const float h = Rv[p] - g * hn, f = Dv[p] - g * fn, gg = -g * gn;
        Rv[p] = h;
        Dv[p] = f;
        Uv[p] = gg;
        fn = f;
        gn = gg;
        hn = h;
      }
      // first and last rows in terms of x_{prev}, x_s, x_e, x_{next}
      const float f1 = Dv[ps + 1], g1 = Uv[ps + 1], h1 = Rv[ps + 1];
      rd[0] -= rc[0] * h1;
      rb[0] -= rc[0] * f1;
      rc[0] = -rc[0] * g1;
      const float fe = Dv[pe - 1], ge = Uv[pe - 1], he = Rv[pe - 1];
      rd[1] -= ra[1] * he;
      rb[1] -= ra[1] * ge;
      ra[1] = -ra[1] * fe;
    }
  }
  // parallel cyclic reduction over the 2K boundary rows (row 2k: x_s of
  // segment k, row 2k+1: its x_e), cyclic indices
  const int M = 2 * K;
  float* RA = red;
  float* RB = red + 128;
  float* RC = red + 256;
  float* RD = red + 384;
  if (lane < K)
    for (int q = 0; q < 2; ++q) {
      RA[2 * lane + q] = ra[q];
      RB[2 * lane + q] = rb[q];
      RC[2 * lane + q] = rc[q];
      RD[2 * lane + q] = rd[q];
    }
  __syncthreads();
  for (int off = 1; off < M; off *= 2) {
    float na[2], nbv[2], nc[2], nd[2];
    if (lane < K)
      for (int q = 0; q < 2; ++q) {
        const int r = 2 * lane + q;
        const int im = (r - off + M) % M, ip = (r + off) % M;
        const float k1 = RA[r] / RB[im], k2 = RC[r] / RB[ip];
        na[q] = -k1 * RA[im];
        nc[q] = -k2 * RC[ip];
        nbv[q] = RB[r] - k1 * RC[im] - k2 * RA[ip];
        nd[q] = RD[r] - k1 * RD[im] - k2 * RD[ip];
      }
    __syncthreads();
    if (lane < K)
      for (int q = 0; q < 2; ++q) {
        const int r = 2 * lane + q;
        RA[r] = na[q];
        RB[r] = nbv[q];
        RC[r] = nc[q];
        RD[r] = nd[q];
      }
    __syncthreads();
  }
  // couplings now reach 2K rows away: the row itself
  float xs = 0.f, xe = 0.f;
  if (lane < K) {
    xs = RD[2 * lane] / (RB[2 * lane] + RA[2 * lane] + RC[2 * lane]);
    xe = RD[2 * lane + 1] / (RB[2 * lane + 1] + RA[2 * lane + 1] + RC[2 * lane + 1]);
  }
  // corrections of the segment (the interior from the eliminated rows)
  if (lane < K)
    for (int i = s; i <= e; ++i) {
      float dlt;
      if (i == s)
        dlt = xs;
      else if (i == e)
        dlt = xe;
      else {
        const int p = i + lane;
        dlt = Rv[p] - Dv[p] * xs - Uv[p] * xe;
      }
      const int c = ax == 0 ? i + A.n0 * line : line + A.n0 * i;
      k.x[c] += (T)dlt;
    }
}

// residual of a 25-point level
__global__ __launch_bounds__(256) void residual25_kernel(Stencil2<float> A, const float* __restrict__ x,
                                                         const float* __restrict__ rhs, float* res, const int* flag) {
  if (flag[0]) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= A.n0 * A.n1) return;
  const int i = c % A.n0, j = c / A.n0;
  float r = rhs[c];
  for (int dy = -2; dy <= 2; ++dy)
    for (int dx = -2; dx <= 2; ++dx) {
      int t;
      if (!A.nb(i, j, dx, dy, &t)) continue;
      r -= A.coef(i, j, dx, dy) * x[t];
    }
  res[c] = r;
}

// x = Cinv rhs on the coarsest level (one workgroup)
__global__ __launch_bounds__(1024) void dense_solve_kernel(int n, const float* __restrict__ cinv,
                                                           const float* __restrict__ rhs, float* x, const int* flag) {
  if (flag[0]) return;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    float s = 0.f;
    for (int j = 0; j < n; ++j) s += cinv[(size_t)j * n + i] * rhs[j];
    x[i] = s;
  }
}

// colours of the lines along `axis` on a level: the smallest count c >= 2 R
// (R the stencil's reach across lines) that divides the line count when the
// cross axis is periodic (lines 0 and n - 1 are then neighbours)
static int line_colors(int nlines, int per, int reach) {
  for (int c = 2 * reach; c < nlines; ++c)
    if (!per || nlines % c == 0) return c;
  return nlines;
}

static void line_sweep(const GridCtx& G, int l, int axis, bool reverse, hipStream_t st) {
  const Level& L = G.lev[l];
  const int nl = axis == 0 ? L.n[1] : L.n[0];  // number of lines
  const int per = axis == 0 ? G.g.periodic[1] : G.g.periodic[0];
  const int reach = l > 0 ? 2 : 1;
  const int nc = line_colors(nl, per, reach);
  const int n = axis == 0 ? L.n[0] : L.n[1];
  const size_t lds = sizeof(float) * (3 * (size_t)(n + 64) + 4 * 128);
  for (int q = 0; q < nc; ++q) {
    const int col = reverse ? nc - 1 - q : q;
    const unsigned lines = (unsigned)((nl - col + nc - 1) / nc);
    if (l > 0) {
      LineRelaxArgs<float, true> a{stencil2<float>(G, l), L.f_phi, L.f_rhs, axis, col, nc, G.mg_flag};
      hipLaunchKernelGGL((line_relax_kernel<float, true>), dim3(lines), dim3(64), lds, st, a);
    } else {
      LineRelaxArgs<float, false> a{stencil2<float>(G, l), L.f_phi, L.f_rhs, axis, col, nc, G.mg_flag};
      hipLaunchKernelGGL((line_relax_kernel<float, false>), dim3(lines), dim3(64), lds, st, a);
    }
  }
}

// one relaxation: lines along x, then along y (post-smoothing: the reverse)
static void line_relax(const GridCtx& G, int l, bool post, hipStream_t st) {
  if (!post) {
    line_sweep(G, l, 0, false, st);
    line_sweep(G, l, 1, false, st);
  } else {
    line_sweep(G, l, 1, true, st);
    line_sweep(G, l, 0, true, st);
  }
}

// V(1,2) cycle of the variational hierarchy on the FP32 vectors (level 0:
// z = f_phi, zero on entry, from r = f_rhs): one relaxation before the coarse
// correction, two after (on the spherical r-z test, 5 flexible-CG iterations to
// 1e-10 at 1024^2 where V(1,1) takes 7 and V(2,2) 5 at a third more work)
static void boxmg_vcycle(const GridCtx& G, int l, hipStream_t st) {
  const Level& L = G.lev[l];
  if (l == G.coarse) {
    if (G.cinv32) {
      hipLaunchKernelGGL(dense_solve_kernel, dim3(1), dim3(1024), 0, st, (int)L.ncells, (const float*)G.cinv32,
                         (const float*)L.f_rhs, L.f_phi, (const int*)G.mg_flag);
    } else {
      for (int s = 0; s < 4; ++s) line_relax(G, l, s & 1, st);
    }
    return;
  }
  line_relax(G, l, false, st);
  const Level& C = G.lev[l + 1];
  const LevelArgsT<float> fa = level_args_f32(G, l);
  if (l == 0) {
    op_launch<residual_kernelOp<float>>(grid3(L), BLOCK3, residual_kernelOp<float>::Args{fa, (const float*)L.f_phi, (const float*)L.f_rhs, L.f_res, (const int*)G.mg_flag}, st);
  } else {
    hipLaunchKernelGGL(residual25_kernel, dim3((unsigned)((L.ncells + 255) / 256)), dim3(256), 0, st,
                       stencil2<float>(G, l), (const float*)L.f_phi, (const float*)L.f_rhs, L.f_res,
                       (const int*)G.mg_flag);
  }
  op_launch<restrict_kernelOp<float>>(grid3(C), BLOCK3, restrict_kernelOp<float>::Args{fa, (const float*)L.f_res, C.n[0], C.n[1], C.n[2], C.f_rhs, C.f_phi, (const int*)G.mg_flag}, st);
  boxmg_vcycle(G, l + 1, st);
  op_launch<prolong_kernelOp<float>>(grid3(L), BLOCK3, prolong_kernelOp<float>::Args{fa, L.f_phi, (const float*)C.f_phi, C.n[0], C.n[1], C.n[2], (const int*)G.mg_flag, 1}, st);
  line_relax(G, l, true, st);
  line_relax(G, l, true, st);
}

// ----------------------------------------------------------------------------
// replay of recorded field phases as batched launches (see kernels.hpp)
// ----------------------------------------------------------------------------
static void replay_one(int kind, dim3 g, dim3 b, const void* a, int n, hipStream_t st) {
  switch (kind) {
    case BK_CHARGE: op_replay<charge_kernelOp>(g, b, a, n, st); break;
    case BK_EXTRAP: op_replay<extrapolate_kernelOp>(g, b, a, n, st); break;
    case BK_RHS: op_replay<rhs_kernelOp>(g, b, a, n, st); break;
    case BK_SUB: op_replay<sub_scalar_kernelOp>(g, b, a, n, st); break;
    case BK_REDP: op_replay<reduce_partial_kernelOp>(g, b, a, n, st); break;
    case BK_REDF: op_replay<reduce_final_kernelOp>(g, b, a, n, st); break;
    case BK_RESET: op_replay<mg_reset_kernelOp>(g, b, a, n, st); break;
    case BK_FCGRES: op_replay<fcg_residual_kernelOp>(g, b, a, n, st); break;
    case BK_FCGAPPLY: op_replay<fcg_apply_kernelOp>(g, b, a, n, st); break;
    case BK_FCGCOEF: op_replay<fcg_coef_kernelOp>(g, b, a, n, st); break;
    case BK_FCGUPD: op_replay<fcg_update_kernelOp>(g, b, a, n, st); break;
    case BK_SMOOTH_F: op_replay<smooth_kernelOp<float>>(g, b, a, n, st); break;
    case BK_SMOOTH_D: op_replay<smooth_kernelOp<double>>(g, b, a, n, st); break;
    case BK_RESID_F: op_replay<residual_kernelOp<float>>(g, b, a, n, st); break;
    case BK_RESID_D: op_replay<residual_kernelOp<double>>(g, b, a, n, st); break;
    case BK_RSUM_F: op_replay<restrict_sum_kernelOp<float>>(g, b, a, n, st); break;
    case BK_RSUM_D: op_replay<restrict_sum_kernelOp<double>>(g, b, a, n, st); break;
    case BK_RTR_F: op_replay<restrict_kernelOp<float>>(g, b, a, n, st); break;
    case BK_RTR_D: op_replay<restrict_kernelOp<double>>(g, b, a, n, st); break;
    case BK_PROL_F: op_replay<prolong_kernelOp<float>>(g, b, a, n, st); break;
    case BK_PROL_D: op_replay<prolong_kernelOp<double>>(g, b, a, n, st); break;
    case BK_SMALL_F: op_replay<small_vcycle_kernelOp<float>>(g, b, a, n, st); break;
    case BK_SMALL_D: op_replay<small_vcycle_kernelOp<double>>(g, b, a, n, st); break;
    case BK_EF2F: op_replay<efield_kernelOp<2, float>>(g, b, a, n, st); break;
    case BK_EF2D: op_replay<efield_kernelOp<2, double>>(g, b, a, n, st); break;
    case BK_EF3F: op_replay<efield_kernelOp<3, float>>(g, b, a, n, st); break;
    case BK_EF3D: op_replay<efield_kernelOp<3, double>>(g, b, a, n, st); break;
    case BK_RESR_F: op_replay<resrestrict_kernelOp<float>>(g, b, a, n, st); break;
    case BK_RESR_H: op_replay<resrestrict_kernelOp<float, __half>>(g, b, a, n, st); break;
    case BK_SMOOTH_H: op_replay<smooth_kernelOp<float, __half>>(g, b, a, n, st); break;
    case BK_RESR_D: op_replay<resrestrict_kernelOp<double>>(g, b, a, n, st); break;
    default: break;
  }
}

// The argument buffer's copy from pinned host memory (read by the kernel
// through its device address) to the device buffer: launching it costs the
// host a few microseconds, an asynchronous copy call several times that.
__global__ __launch_bounds__(256) void args_copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                        long long n16) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n16; i += (long long)gridDim.x * 256)
    dst[i] = src[i];
}

int batch_upload(BatchArgs& ba, hipStream_t st) {
  const size_t total = ba.staging.size();
  if (total > ba.bytes || total > ba.pinned_bytes) {
    // larger buffers; the old ones may still be read by work in flight on st
    if (hipStreamSynchronize(st) != hipSuccess) return -3;
    free_batch_args(ba);
    const size_t want = total + total / 2 + 4096;
    ba.dev = ba.dev_alloc ? ba.dev_alloc(want, ba.ctx) : nullptr;
    if (!ba.dev) return -2;
    ba.bytes = want;
    for (int k = 0; k < 2; ++k) {
      if (hipHostMalloc(&ba.pinned[k], want, hipHostMallocDefault) != hipSuccess) {
        ba.pinned[k] = nullptr;
        free_batch_args(ba);
        return -2;
      }
      if (hipHostGetDevicePointer(&ba.pinned_dev[k], ba.pinned[k], 0) != hipSuccess) ba.pinned_dev[k] = nullptr;
      if (hipEventCreateWithFlags(&ba.copied[k], hipEventDisableTiming) != hipSuccess) {
        ba.copied[k] = nullptr;
        free_batch_args(ba);
        return -2;
      }
      if (hipEventRecord(ba.copied[k], st) != hipSuccess) return -3;
    }
    ba.pinned_bytes = want;
  }
  // most steps bring the same contents as the last one: upload on change
  // (stream-ordered, so launches still in flight read the previous contents)
  if (ba.uploaded != ba.staging) {
    const int k = ba.slot;
    ba.slot ^= 1;
    if (hipEventSynchronize(ba.copied[k]) != hipSuccess) return -3;
    memcpy(ba.pinned[k], ba.staging.data(), total);
    // whole 16-byte words: both buffers hold at least total + 4096 bytes
    const long long n16 = (long long)((total + 15) / 16);
    if (n16 == 0) {
      // nothing to copy
    } else if (ba.pinned_dev[k] && (((uintptr_t)ba.pinned_dev[k] | (uintptr_t)ba.dev) & 15) == 0) {
      const unsigned blocks = (unsigned)std::min<long long>(64, (n16 + 255) / 256);
      hipLaunchKernelGGL(args_copy_kernel, dim3(blocks), dim3(256), 0, st, (const uint4*)ba.pinned_dev[k],
                         (uint4*)ba.dev, n16);
      if (hipGetLastError() != hipSuccess) return -3;
    } else if (hipMemcpyAsync(ba.dev, ba.pinned[k], total, hipMemcpyHostToDevice, st) != hipSuccess) {
      return -3;
    }
    if (hipEventRecord(ba.copied[k], st) != hipSuccess) return -3;
    ba.uploaded = ba.staging;
  }
  return 0;
}

int replay_batch(BatchRecorder* const* cases, int n, BatchArgs& ba, hipStream_t st) {
  if (n < 1) return 0;
  const BatchRecorder& r0 = *cases[0];
  // every case must have recorded the same sequence of launches
  for (int c = 0; c < n; ++c) {
    const BatchRecorder& rc = *cases[c];
    if (rc.unsupported || rc.recs.size() != r0.recs.size()) return -1;
    for (size_t i = 0; i < rc.recs.size(); ++i) {
      const BatchRec &a = rc.recs[i], &b = r0.recs[i];
      if (a.kind != b.kind || a.args.size() != b.args.size() || a.grid.x != b.grid.x || a.grid.y != b.grid.y ||
          a.grid.z != b.grid.z || a.block.x != b.block.x || a.block.y != b.block.y || a.block.z != b.block.z)
        return -1;
      // the batched grid stacks the cases along z
      if ((size_t)a.grid.z * (size_t)n > 65535) return -1;
    }
  }
  // argument structs: record i of every case as an array Args[n] (the kernel
  // indexes it with the struct's own size), each array 16-byte aligned
  std::vector<size_t> offs(r0.recs.size());
  size_t total = 0;
  for (size_t i = 0; i < r0.recs.size(); ++i) {
    total = (total + 15) & ~(size_t)15;
    offs[i] = total;
    total += r0.recs[i].args.size() * (size_t)n;
  }
  ba.staging.assign(total, 0);
  for (size_t i = 0; i < r0.recs.size(); ++i) {
    const size_t sz = r0.recs[i].args.size();
    for (int c = 0; c < n; ++c) memcpy(ba.staging.data() + offs[i] + sz * (size_t)c, cases[c]->recs[i].args.data(), sz);
  }
  const int up = batch_upload(ba, st);
  if (up != 0) return up;
  if (ba.graphs_on) {
    // one graph launch per step instead of one launch per kernel: the graph
    // holds the launches (their arguments are read from the buffer, uploaded
    // above), so it serves every step with the same sequence
    uint64_t key = 1469598103934665603ull;
    auto mix = [&key](uint64_t v) { key = (key ^ v) * 1099511628211ull; };
    mix((uint64_t)n);
    mix((uint64_t)(uintptr_t)ba.dev);
    for (const BatchRec& rec : r0.recs) {
      mix((uint64_t)rec.kind);
      mix(((uint64_t)rec.grid.x << 32) ^ ((uint64_t)rec.grid.y << 16) ^ rec.grid.z);
      mix(((uint64_t)rec.block.x << 32) ^ ((uint64_t)rec.block.y << 16) ^ rec.block.z);
      mix((uint64_t)rec.args.size());
    }
    for (const auto& g : ba.graphs)
      if (g.first == key) return hipGraphLaunch(g.second, st) == hipSuccess ? 0 : -3;
    if (ba.graphs.size() < 64 && hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      for (size_t i = 0; i < r0.recs.size(); ++i) {
        const BatchRec& rec = r0.recs[i];
        replay_one(rec.kind, rec.grid, rec.block, (const unsigned char*)ba.dev + offs[i], n, st);
      }
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      const bool ok = hipStreamEndCapture(st, &graph) == hipSuccess && graph &&
                      hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
      if (graph) (void)hipGraphDestroy(graph);
      if (ok && hipGraphLaunch(exec, st) == hipSuccess) {
        ba.graphs.push_back({key, exec});
        return 0;
      }
      // nothing ran: launch directly
      if (exec) (void)hipGraphExecDestroy(exec);
    }
    (void)hipGetLastError();  // e.g. the null stream cannot be captured
  }
  for (size_t i = 0; i < r0.recs.size(); ++i) {
    const BatchRec& rec = r0.recs[i];
    replay_one(rec.kind, rec.grid, rec.block, (const unsigned char*)ba.dev + offs[i], n, st);
  }
  return 0;
}

void free_batch_args(BatchArgs& ba) {
  if (ba.dev && ba.dev_free) ba.dev_free(ba.dev, ba.ctx);
  ba.dev = nullptr;
  ba.bytes = 0;
  for (int k = 0; k < 2; ++k) {
    if (ba.pinned[k]) (void)hipHostFree(ba.pinned[k]);
    if (ba.copied[k]) (void)hipEventDestroy(ba.copied[k]);
    ba.pinned[k] = nullptr;
    ba.pinned_dev[k] = nullptr;
    ba.copied[k] = nullptr;
  }
  ba.pinned_bytes = 0;
  ba.slot = 0;
  ba.uploaded.clear();
  for (auto& g : ba.graphs) (void)hipGraphExecDestroy(g.second);
  ba.graphs.clear();
}

}  // namespace cpic
