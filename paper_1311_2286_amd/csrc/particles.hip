// particles.hip -- particle kernels of the curvilinear PIC hot path for CDNA4.
//
//   particle_kernel : one workgroup per work item (a contiguous run of the
//                     particles of one 16^2 / 8^3 cell tile).  Per particle:
//                     gather of the vertex field (Eqs. vvp, Wvp, b1), Boris /
//                     leap-frog velocity update (Eqs. step1, step1a), position
//                     update x(xi^n) + dt v^{n+1/2} mapped back to xi by
//                     Newton on the map increment, particle boundaries, and
//                     the charge deposit (Eqs. pg, Wpc, b2) into an LDS window
//                     of the tile plus G cells, flushed to HBM with atomics.
//   tile sort       : counting sort of the particle arrays by tile (histogram,
//                     scan into work items, scatter), dropping dead particles.
//
// Particles are structure-of-arrays; a tile's particles are contiguous after a
// sort, so every workgroup streams its run with coalesced loads and stores.
#include <cstring>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace cpic {

// ----------------------------------------------------------------------------
// wave-level helpers (wave64)
// ----------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Aggregated atomicAdd of 1 per active lane onto counters[key]: lanes sharing a
// key are served by one atomic; each active lane gets old value + its rank.
// Must be called by all lanes of the wave.
__device__ inline int agg_inc(int* counters, int key, bool active) {
  int out = 0;
  bool pending = active;
  const int lane = __lane_id();
  while (true) {
    unsigned long long pm = __ballot(pending);
    if (pm == 0ull) break;
    int leader = __ffsll((unsigned long long)pm) - 1;
    int lkey = __shfl(key, leader, 64);
    bool mine = pending && key == lkey;
    unsigned long long mm = __ballot(mine);
    int base = 0;
    if (lane == leader) base = atomicAdd(&counters[lkey], __popcll(mm));
    base = __shfl(base, leader, 64);
    if (mine) {
      out = base + __popcll(mm & ((1ull << lane) - 1ull));
      pending = false;
    }
  }
  return out;
}

// ----------------------------------------------------------------------------
// field gather: CIC weights (1 - f, f) over the 2^D vertices of the cell
// ----------------------------------------------------------------------------
template <int D, typename R>
__device__ inline void gather_E(const R* __restrict__ Ev, const Geo& g, const int* idx, const R* f,
                                R* E) {
  constexpr int EC = (D == 3) ? 4 : 2;
  E[0] = E[1] = E[2] = (R)0;
  int vx0 = idx[0], vx1 = idx[0] + 1;
  if (vx1 >= g.nv[0]) vx1 -= g.nv[0];
  int vy0 = idx[1], vy1 = idx[1] + 1;
  if (vy1 >= g.nv[1]) vy1 -= g.nv[1];
  R wx[2] = {(R)1 - f[0], f[0]};
  R wy[2] = {(R)1 - f[1], f[1]};
  if (D == 2) {
    const int vxs[2] = {vx0, vx1}, vys[2] = {vy0, vy1};
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        long long v = (long long)vxs[a] + (long long)g.nv[0] * vys[b];
        const R* e = Ev + v * EC;
        R w = wx[a] * wy[b];
        E[0] += w * e[0];
        E[1] += w * e[1];
      }
  } else {
    int vz0 = idx[2], vz1 = idx[2] + 1;
    if (vz1 >= g.nv[2]) vz1 -= g.nv[2];
    R wz[2] = {(R)1 - f[2], f[2]};
    const int vxs[2] = {vx0, vx1}, vys[2] = {vy0, vy1}, vzs[2] = {vz0, vz1};
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          long long v = (long long)vxs[a] + (long long)g.nv[0] * (vys[b] + (long long)g.nv[1] * vzs[c]);
          const R* e = Ev + v * EC;
          R w = wx[a] * wy[b] * wz[c];
          E[0] += w * e[0];
          E[1] += w * e[1];
          E[2] += w * e[2];
        }
  }
}

template <typename R>
__device__ inline void boris_push(R* v, const R* E, const R* B, R qm, R dt, bool magnetic) {
  R h = (R)0.5 * dt * qm;
  R vm0 = v[0] + h * E[0], vm1 = v[1] + h * E[1], vm2 = v[2] + h * E[2];
  if (magnetic) {
    R t0 = h * B[0], t1 = h * B[1], t2 = h * B[2];
    R tt = t0 * t0 + t1 * t1 + t2 * t2;
    R p0 = vm0 + (vm1 * t2 - vm2 * t1);
    R p1 = vm1 + (vm2 * t0 - vm0 * t2);
    R p2 = vm2 + (vm0 * t1 - vm1 * t0);
    R sc = (R)2 / ((R)1 + tt);
    R s0 = sc * t0, s1 = sc * t1, s2 = sc * t2;
    vm0 += p1 * s2 - p2 * s1;
    vm1 += p2 * s0 - p0 * s2;
    vm2 += p0 * s1 - p1 * s0;
  }
  v[0] = vm0 + h * E[0];
  v[1] = vm1 + h * E[1];
  v[2] = vm2 + h * E[2];
}

// Globalised FP64 inversion for the rare particles that plain Newton does not
// settle: the physical displacement is split into m equal parts (continuation)
// so that each part moves the particle by at most a quarter cell in logical
// space, and each part is solved by Newton from the end of the previous one.
// Tabulated map, the mover's view: between vertices the map is the
// multilinear interpolant of the vertex coordinates (piecewise multilinear,
// continuous).  x and J = dx/du at u (cells) from the cell holding u; on a
// bounded axis the boundary cell's polynomial continues beyond the wall.
template <int D>
__device__ inline void tab_cell_xj(const Geo& g, const double* u, double* x, double (*J)[3]) {
  int base[3] = {0, 0, 0};
  double f[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    int c = (int)floor(u[a]);
    if (!g.periodic[a]) c = min(max(c, 0), g.n[a] - 1);
    base[a] = c;
    f[a] = u[a] - c;
    x[a] = 0.0;
#pragma unroll
    for (int b = 0; b < D; ++b) J[a][b] = 0.0;
  }
#pragma unroll
  for (int corner = 0; corner < (1 << D); ++corner) {
    double w = 1.0, dw[3] = {1.0, 1.0, 1.0}, per[3] = {0.0, 0.0, 0.0};
    long long v = 0, stride = 1;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int up = (corner >> a) & 1;
      int i = base[a] + up;
      const double wa = up ? f[a] : 1.0 - f[a];
#pragma unroll
      for (int b = 0; b < D; ++b) dw[b] *= (b == a) ? (up ? 1.0 : -1.0) : wa;
      w *= wa;
      if (g.periodic[a]) {
        int r = i % g.n[a];
        if (r < 0) r += g.n[a];
        per[a] = (double)((i - r) / g.n[a]);
        i = r;
      }
      v += stride * i;
      stride *= g.nv[a];
    }
    const double* xv = g.xtab + v * D;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double xa = xv[a] + per[a] * g.L[a];
      x[a] += w * xa;
#pragma unroll
      for (int b = 0; b < D; ++b) J[a][b] += dw[b] * xa;
    }
  }
}

// x^{-1}(x(u0) + disp) on a tabulated map by Newton on the position u in cells
// (each iteration with the polynomial of the cell holding u, a step of at most
// one cell per axis); d = u - u0.  Converged once a step is below 1e-9 cell.
template <int D>
__device__ inline bool move_tab(const Geo& g, const int* idx, const double* f0, const double* disp, int maxit,
                                double* d) {
  double u0[3] = {0.0, 0.0, 0.0}, u[3], tgt[3], x[3], J[3][3];
#pragma unroll
  for (int a = 0; a < D; ++a) u0[a] = idx[a] + f0[a];
  tab_cell_xj<D>(g, u0, x, J);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    u[a] = u0[a];
    tgt[a] = a < D ? x[a] + disp[a] : 0.0;
  }
  bool conv = false;
  for (int it = 0; it < maxit; ++it) {
    if (it > 0) tab_cell_xj<D>(g, u, x, J);
    double r[3] = {0.0, 0.0, 0.0}, du[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < D; ++a) r[a] = tgt[a] - x[a];
    if (D == 2) {
      const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      du[0] = (J[1][1] * r[0] - J[0][1] * r[1]) / det;
      du[1] = (J[0][0] * r[1] - J[1][0] * r[0]) / det;
    } else {
      const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1], c01 = J[0][2] * J[2][1] - J[0][1] * J[2][2],
                   c02 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
      const double c10 = J[1][2] * J[2][0] - J[1][0] * J[2][2], c11 = J[0][0] * J[2][2] - J[0][2] * J[2][0],
                   c12 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
      const double c20 = J[1][0] * J[2][1] - J[1][1] * J[2][0], c21 = J[0][1] * J[2][0] - J[0][0] * J[2][1],
                   c22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      const double det = J[0][0] * c00 + J[0][1] * c10 + J[0][2] * c20;
      du[0] = (c00 * r[0] + c01 * r[1] + c02 * r[2]) / det;
      du[1] = (c10 * r[0] + c11 * r[1] + c12 * r[2]) / det;
      du[2] = (c20 * r[0] + c21 * r[1] + c22 * r[2]) / det;
    }
    double big = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) big = fmax(big, fabs(du[a]));
    if (!(big < 1e30)) break;  // singular cell: not converged
    const double sc = big > 1.0 ? 1.0 / big : 1.0;
#pragma unroll
    for (int a = 0; a < D; ++a) u[a] += sc * du[a];
    if (big < 1e-9) {
      conv = true;
      break;
    }
  }
#pragma unroll
  for (int a = 0; a < D; ++a) d[a] = u[a] - u0[a];
  return conv;
}

// Cyclotronic velocity step (a uniform B): the electric impulse, then the
// exact rotation by theta about b; vm receives the mean velocity of the
// gyration over the step (the position moves by dt vm).  c, s, s1, s2: cos,
// sin, sin(theta)/theta, (1 - cos(theta))/theta.
template <typename R>
__device__ __forceinline__ void cyclotronic_step(R* v, const R* E, R qm, R dt, const R* b, R c, R s, R s1, R s2,
                                                 R* vm) {
#pragma unroll
  for (int a = 0; a < 3; ++a) v[a] += qm * E[a] * dt;
  const R vpar = v[0] * b[0] + v[1] * b[1] + v[2] * b[2];
  R vp[3], w[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) vp[a] = v[a] - vpar * b[a];
  w[0] = vp[1] * b[2] - vp[2] * b[1];
  w[1] = vp[2] * b[0] - vp[0] * b[2];
  w[2] = vp[0] * b[1] - vp[1] * b[0];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    vm[a] = vpar * b[a] + vp[a] * s1 + w[a] * s2;
    v[a] = vpar * b[a] + vp[a] * c + w[a] * s;
  }
}

// The mean velocity of the last cyclotronic step from the velocity it left,
// rotating that back by theta (for a position update redone in FP64).
template <typename R>
__device__ __forceinline__ void cyclotronic_mean(const R* vn, const R* b, R c, R s, R s1, R s2, R* vm) {
  const R vpar = vn[0] * b[0] + vn[1] * b[1] + vn[2] * b[2];
  R u[3], uxb[3], vp[3], w[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) u[a] = vn[a] - vpar * b[a];
  uxb[0] = u[1] * b[2] - u[2] * b[1];
  uxb[1] = u[2] * b[0] - u[0] * b[2];
  uxb[2] = u[0] * b[1] - u[1] * b[0];
#pragma unroll
  for (int a = 0; a < 3; ++a) vp[a] = u[a] * c - uxb[a] * s;
  w[0] = vp[1] * b[2] - vp[2] * b[1];
  w[1] = vp[2] * b[0] - vp[0] * b[2];
  w[2] = vp[0] * b[1] - vp[1] * b[0];
#pragma unroll
  for (int a = 0; a < 3; ++a) vm[a] = vpar * b[a] + vp[a] * s1 + w[a] * s2;
}

template <int D, int MAP>
__device__ __forceinline__ bool move_fallback(const Geo& g, const int* idx, const double* f0,
                                              const double* disp, double kappa, double* d) {
  if constexpr (MAP == MAP_TABULATED) return move_tab<D>(g, idx, f0, disp, 96, d);
  double dt0[3] = {0.0, 0.0, 0.0};
  double J = 1.0;
  double est[3] = {0.0, 0.0, 0.0};
  if (MAP == MAP_SINUSOIDAL)
    newton_sinusoidal<D, double>(g, idx, f0, disp, est, 0.0, 0.0, 1, J);
  else
    newton_polar<double>(g, idx, f0, disp, est, 0.0, 0.0, 1, J);
  double mx = 0.0;
  for (int a = 0; a < D; ++a) mx = fmax(mx, fabs(est[a]));
  int m = (int)ceil(mx / 0.25);
  m = m < 1 ? 1 : (m > 256 ? 256 : m);
  bool ok = true;
  for (int k = 0; k < m; ++k) {
    double fb[3] = {0.0, 0.0, 0.0}, part[3] = {0.0, 0.0, 0.0}, dd[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < D; ++a) {
      fb[a] = f0[a] + dt0[a];
      part[a] = disp[a] / m;
    }
    bool c;
    if (MAP == MAP_SINUSOIDAL)
      c = newton_sinusoidal<D, double>(g, idx, fb, part, dd, 1e-12, kappa, 24, J);
    else
      c = newton_polar<double>(g, idx, fb, part, dd, 1e-12, kappa, 24, J);
    ok = ok && c;
    for (int a = 0; a < D; ++a) dt0[a] += dd[a];
  }
  for (int a = 0; a < D; ++a) d[a] = dt0[a];
  return ok;
}

// Newton on the map increment in the particle's precision.  Returns false
// when it does not converge or (FP32 only) when the cell is strongly
// compressed (J < 0.25 in box units): such particles are handed to the FP64
// fallback kernel.  inv_dxc: n_a / L_a.
template <int D, int MAP, typename R>
__device__ __forceinline__ bool move_delta(const Geo& g, const int* idx, const R* f, const R* v,
                                           R dt, const R* inv_dxc, int maxit, R tol, R kappa, R* d) {
  if (MAP == MAP_IDENTITY) {
#pragma unroll
    for (int a = 0; a < D; ++a) d[a] = dt * v[a] * inv_dxc[a];
    return true;
  }
  bool conv;
  R J0 = (R)1;
  if (MAP == MAP_SINUSOIDAL) {
    R r[D];
#pragma unroll
    for (int a = 0; a < D; ++a) r[a] = dt * v[a] * inv_dxc[a];
    conv = newton_sinusoidal<D, R>(g, idx, f, r, d, tol, kappa, maxit, J0);
  } else {
    R vdt[2] = {dt * v[0], dt * v[1]};
    conv = newton_polar<R>(g, idx, f, vdt, d, tol, kappa, maxit, J0);
  }
  // FP32 residuals lose about 1/J of their accuracy: strongly stretched cells
  // (J < 1/4 of the undistorted cell at the start or at any iterate) go to
  // the FP64 fallback
  const bool low_j = std::is_same<R, float>::value && J0 < (R)0.25;
  return conv && !low_j;
}

// LDS window of vertex data of a tile: its vertices and a one-cell halo
template <int D> struct FieldWindow {
  static constexpr int E0 = TileShape<D>::T0 + 3, E1 = TileShape<D>::T1 + 3, E2 = (D == 3) ? TileShape<D>::T2 + 3 : 1;
  static constexpr int N = E0 * E1 * E2;
  static constexpr int C = D;  // packed components per vertex
};

__device__ inline int wrap_local(int v, int origin, int n, bool periodic) {
  int l = v - origin;
  if (periodic) l = l < -n / 2 ? l + n : (l >= n - n / 2 ? l - n : l);
  return l;
}

// values per vertex in the kc table: D x D padded to a multiple of 4
template <int D> constexpr int KC_STRIDE = D == 3 ? 12 : 4;

// Inverse Jacobian in cells per unit length, kc_ab = n_a dxi^a/dx^b, carried
// from the vertex table to the point (cell cidx, offset cf) by the CIC vertex
// weights (Eq. step3 with the b1 weights of Eq. Wvp).  Vertex n of a periodic
// axis is vertex 0.
template <int D, typename R>
__device__ __forceinline__ void kc_interp(const Geo& g, const R* __restrict__ kc, const int* cidx, const R* cf,
                                          R* k) {
#pragma unroll
  for (int e = 0; e < D * D; ++e) k[e] = (R)0;
#pragma unroll
  for (int corner = 0; corner < (1 << D); ++corner) {
    long long v = 0;
    R w = (R)1;
#pragma unroll
    for (int ax = D - 1; ax >= 0; --ax) {
      const int c = (corner >> ax) & 1;
      int vi = cidx[ax] + c;
      if (vi >= g.nv[ax]) vi -= g.nv[ax];
      v = v * g.nv[ax] + vi;
      w *= c ? cf[ax] : (R)1 - cf[ax];
    }
    R kv[KC_STRIDE<D>];
    using V4 = typename std::conditional<std::is_same<R, float>::value, float4, double4>::type;
    const V4* src = reinterpret_cast<const V4*>(kc + v * KC_STRIDE<D>);
#pragma unroll
    for (int q = 0; q < KC_STRIDE<D> / 4; ++q) {
      const V4 t = src[q];
      kv[4 * q + 0] = t.x;
      kv[4 * q + 1] = t.y;
      kv[4 * q + 2] = t.z;
      kv[4 * q + 3] = t.w;
    }
#pragma unroll
    for (int e = 0; e < D * D; ++e) k[e] += w * kv[e];
  }
}

// kc at (cidx, cf) from the tile's LDS copy of the table (D x D values per
// vertex, the window of the field: the tile and a one-cell halo); false when a
// vertex of the cell lies outside it.  Same weights and summation order as
// kc_interp, so both give identical sums.
template <int D, typename R>
__device__ __forceinline__ bool kc_interp_window(const R* __restrict__ kwin, const Geo& g, const int* origin,
                                                 const int* cidx, const R* cf, R* k) {
  using FW = FieldWindow<D>;
  const int Ew[3] = {FW::E0, FW::E1, FW::E2};
  int l[3] = {0, 0, 0};
  bool in = true;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    l[a] = wrap_local(cidx[a], origin[a] - 1, g.n[a], g.periodic[a] != 0);
    in = in && l[a] >= 0 && l[a] + 1 < Ew[a];
  }
  if (!in) return false;
  constexpr int KD = D * D;
  const R* k0 = kwin + KD * (l[0] + FW::E0 * (l[1] + FW::E1 * l[2]));
#pragma unroll
  for (int e = 0; e < KD; ++e) k[e] = (R)0;
#pragma unroll
  for (int corner = 0; corner < (1 << D); ++corner) {
    R w = (R)1;
    int off = 0;
#pragma unroll
    for (int ax = D - 1; ax >= 0; --ax) {
      const int c = (corner >> ax) & 1;
      w *= c ? cf[ax] : (R)1 - cf[ax];
      off += c * (ax == 0 ? 1 : (ax == 1 ? FW::E0 : FW::E0 * FW::E1));
    }
#pragma unroll
    for (int e = 0; e < KD; ++e) k[e] += w * k0[KD * off + e];
  }
  return true;
}

// Tabulated map, FP32 Newton on the tile's LDS copy of the vertex coordinates
// (the window of the field: the tile and a one-cell halo; coordinates relative
// to the tile's first vertex, so FP32 keeps about 1e-6 of a cell).  Positions
// are window cells w = u - (origin - 1).  Returns false, leaving d alone, when
// an iterate leaves the window or crosses a bounded axis' wall, or when eight
// iterations do not settle it below 2e-6 cell (about the FP32 resolution of
// w): the FP64 inversion on the global table (move_tab) then moves the
// particle.  Each iteration uses the polynomial of the cell holding w.
template <int D>
__device__ inline bool tab_window_xj(const float* __restrict__ xwin, const Geo& g, const int* origin,
                                     const float* w, float* x, float (*J)[3]) {
  using FW = FieldWindow<D>;
  const int Ew[3] = {FW::E0, FW::E1, FW::E2};
  int c[3] = {0, 0, 0};
  float f[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const float fl = floorf(w[a]);
    c[a] = (int)fl;
    f[a] = w[a] - fl;
    if (c[a] < 0 || c[a] + 1 >= Ew[a]) return false;
    if (!g.periodic[a]) {
      const int gc = origin[a] - 1 + c[a];
      if (gc < 0 || gc >= g.n[a]) return false;
    }
    x[a] = 0.f;
#pragma unroll
    for (int b = 0; b < D; ++b) J[a][b] = 0.f;
  }
  const float* x0 = xwin + D * (c[0] + FW::E0 * (c[1] + FW::E1 * c[2]));
#pragma unroll
  for (int corner = 0; corner < (1 << D); ++corner) {
    float wt = 1.f, dw[3] = {1.f, 1.f, 1.f};
    int off = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int up = (corner >> a) & 1;
      const float wa = up ? f[a] : 1.f - f[a];
#pragma unroll
      for (int b = 0; b < D; ++b) dw[b] *= (b == a) ? (up ? 1.f : -1.f) : wa;
      wt *= wa;
      off += up * (a == 0 ? 1 : (a == 1 ? FW::E0 : FW::E0 * FW::E1));
    }
    const float* xv = x0 + D * off;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      x[a] += wt * xv[a];
#pragma unroll
      for (int b = 0; b < D; ++b) J[a][b] += dw[b] * xv[a];
    }
  }
  return true;
}

template <int D>
__device__ inline bool move_tab_window(const float* __restrict__ xwin, const Geo& g, const int* origin,
                                       const int* idx, const float* f, const float* disp, float* d) {
  using FW = FieldWindow<D>;
  const int Ew[3] = {FW::E0, FW::E1, FW::E2};
  float w0[3] = {0.f, 0.f, 0.f}, w[3] = {0.f, 0.f, 0.f}, x[3], J[3][3], tgt[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const int l = wrap_local(idx[a], origin[a] - 1, g.n[a], g.periodic[a] != 0);
    if (l < 0 || l + 1 >= Ew[a]) return false;
    w0[a] = (float)l + f[a];
    w[a] = w0[a];
  }
  if (!tab_window_xj<D>(xwin, g, origin, w0, x, J)) return false;
#pragma unroll
  for (int a = 0; a < D; ++a) tgt[a] = x[a] + disp[a];
  for (int it = 0; it < 8; ++it) {
    if (it > 0 && !tab_window_xj<D>(xwin, g, origin, w, x, J)) return false;
    float r[3] = {0.f, 0.f, 0.f}, du[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < D; ++a) r[a] = tgt[a] - x[a];
    if (D == 2) {
      const float det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      du[0] = (J[1][1] * r[0] - J[0][1] * r[1]) / det;
      du[1] = (J[0][0] * r[1] - J[1][0] * r[0]) / det;
    } else {
      const float c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1], c01 = J[0][2] * J[2][1] - J[0][1] * J[2][2],
                  c02 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
      const float c10 = J[1][2] * J[2][0] - J[1][0] * J[2][2], c11 = J[0][0] * J[2][2] - J[0][2] * J[2][0],
                  c12 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
      const float c20 = J[1][0] * J[2][1] - J[1][1] * J[2][0], c21 = J[0][1] * J[2][0] - J[0][0] * J[2][1],
                  c22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      const float det = J[0][0] * c00 + J[0][1] * c10 + J[0][2] * c20;
      du[0] = (c00 * r[0] + c01 * r[1] + c02 * r[2]) / det;
      du[1] = (c10 * r[0] + c11 * r[1] + c12 * r[2]) / det;
      du[2] = (c20 * r[0] + c21 * r[1] + c22 * r[2]) / det;
    }
    float big = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a) big = fmaxf(big, fabsf(du[a]));
    if (!(big < 1e30f)) return false;
    const float sc = big > 1.f ? 1.f / big : 1.f;
#pragma unroll
    for (int a = 0; a < D; ++a) w[a] += sc * du[a];
    if (big < 2e-6f) {
#pragma unroll
      for (int a = 0; a < D; ++a) d[a] = w[a] - w0[a];
      return true;
    }
  }
  return false;
}

// Predictor-corrector position update (Eqs. step2-step4) in cells:
//   predictor  u' = (idx + f) + (dt/2) kc(idx, f) v,
//   corrector  d  = dt kc(u') v,
// the predictor point wrapped on periodic axes and clamped into the grid on
// bounded ones for the interpolation of kc.
template <int D, typename R, bool WIN>
__device__ __forceinline__ void move_pc(const Geo& g, const R* __restrict__ kc, const R* __restrict__ kwin,
                                        const int* origin, const int* idx, const R* f, const R* v, R dt, R* d) {
  R k[D * D];
  if (!(WIN && kc_interp_window<D, R>(kwin, g, origin, idx, f, k))) kc_interp<D, R>(g, kc, idx, f, k);
  int pidx[3] = {0, 0, 0};
  R pf[3] = {(R)0, (R)0, (R)0};
  const R h = (R)0.5 * dt;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    R s = (R)0;
#pragma unroll
    for (int b = 0; b < D; ++b) s += k[a * D + b] * v[b];
    const R u = (R)idx[a] + f[a] + h * s;
    const R fl = floor(u);
    int i = (int)fl;
    R fr = u - fl;
    const int n = g.n[a];
    if (g.periodic[a]) {
      i %= n;
      if (i < 0) i += n;
    } else if (u < (R)0) {
      i = 0;
      fr = (R)0;
    } else if (i >= n) {
      i = n - 1;
      fr = (R)1;
    }
    pidx[a] = i;
    pf[a] = fr;
  }
  if (!(WIN && kc_interp_window<D, R>(kwin, g, origin, pidx, pf, k))) kc_interp<D, R>(g, kc, pidx, pf, k);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    R s = (R)0;
#pragma unroll
    for (int b = 0; b < D; ++b) s += k[a * D + b] * v[b];
    d[a] = dt * s;
  }
}

// New cell and offset from cell idx, offset f and increment d (cells), with
// the particle boundaries.  Returns 0 (alive), -1 (absorbed: a wall with an
// absorbing condition) or -2 (left through an outflow wall).
template <int D, typename R>
__device__ __forceinline__ int place_particle(const Geo& g, const int* pbc_lo, const int* pbc_hi,
                                              int* idx, R* f, const R* d, int* shift = nullptr) {
  int dead = 0;
#pragma unroll
  for (int ax = 0; ax < D; ++ax) {
    R u = f[ax] + d[ax];
    R fl = floor(u);
    R nf = u - fl;
    int sh = (int)fl;
    if (nf >= (R)1) {
      nf = (R)0;
      sh += 1;
    }
    int ni = idx[ax] + sh;
    if (shift) shift[ax] = sh;
    const int n = g.n[ax];
    if (g.periodic[ax]) {
      // one period at most in the common case; a division only beyond it
      ni = ni < 0 ? ni + n : (ni >= n ? ni - n : ni);
      if ((unsigned)ni >= (unsigned)n) {
        ni %= n;
        if (ni < 0) ni += n;
      }
    } else if (ni < 0) {
      dead = (pbc_lo[ax] == PBC_ABSORB) ? -1 : -2;
    } else if (ni >= n) {
      dead = (pbc_hi[ax] == PBC_ABSORB) ? -1 : -2;
    }
    idx[ax] = ni;
    f[ax] = nf;
  }
  return dead;
}

// Element i of a particle array.  For 4-byte elements the byte offset is a
// 32-bit unsigned value (species capacities stay below 2^30), so each access
// takes the scalar base + 32-bit vector offset form and needs no 64-bit
// address arithmetic of its own.
template <typename T>
__device__ __forceinline__ T& pel(T* base, int i) {
  if constexpr (sizeof(T) == 4)
    return *(T*)((char*)base + (unsigned)i * 4u);
  else
    return base[i];
}

template <typename R>
struct PartArgs {
  int32_t* key;
  R* off0;
  R* off1;
  R* off2;
  R* v0;
  R* v1;
  R* v2;
  const int* item_tile;
  const int* item_begin;
  const int* item_end;
  const int* n_items;
  const int* d_n;  // live count, particles appended since the last sort included
  const R* Ev;
  const R* kc;  // predictor-corrector mover: n_a dxi^a/dx^b at every vertex (row-major D x D,
                // padded to KC_STRIDE<D> values so a vertex is whole 16-byte loads)
  void* Q;
  Geo g;
  int pbc_lo[3], pbc_hi[3];
  R qm, dt;
  R B[3];
  int magnetic;
  int vz_active;
  int cyclo;  // cyclotronic velocity step: constants of the exact gyration
  R cyc_b[3], cyc_c, cyc_s, cyc_s1, cyc_s2;
  int mode;
  int S1;
  int newton_maxit;
  R newton_tol;
  R kappa;
  R inv_dxc[3];
  double ke_scale;
  double* ke;
  double* ke_part;
  int* tcount;  // when set (steps followed by a tile sort): live particles per new tile, dead last
  unsigned* drift;  // PUSH: running maximum of a particle's increment (cells, FP32 bits)
  // [0] absorbed, [1] outflow, [2] FP64 fallbacks, [3] far deposits, [4] missed tolerance,
  // [5] injected, [6] dropped for capacity, [7] next identifier, [8] injected particles whose
  // entry flight left the domain, [9] particles deposited since Q was last cleared
  unsigned long long* counters;
  int* fb_queue;  // particles left to the FP64 fallback kernel
  int* fb_count;
  int fb_cap;
};

// lcell: when set, the particle's cell in deposit-window coordinates
// (idx - origin + G, wrapped), known from the gather's field-window index.
template <int D, int SHAPE, typename R, bool FIXED, typename QT>
__device__ __forceinline__ void deposit_particle(const Geo& g, const int* origin, QT* win, void* Qg,
                                        const int* idx, const R* f, int S1,
                                        unsigned long long& far, const int* lcell = nullptr) {
  using TS = TileShape<D>;
  typedef typename std::conditional<FIXED, uint32_t, R>::type WT;
  const int Wd[3] = {TS::W0, TS::W1, TS::W2};
  // per axis: weights of cells i-1, i, i+1
  WT w[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a >= D) {
      w[a][0] = w[a][2] = (WT)0;
      w[a][1] = (WT)1;
      continue;
    }
    if (FIXED) {
      uint32_t wi[3];
      weights_fixed<SHAPE>((double)f[a], S1, wi);
      w[a][0] = (WT)wi[0];
      w[a][1] = (WT)wi[1];
      w[a][2] = (WT)wi[2];
    } else {
      R wr[3];
      weights_real<SHAPE, R>(f[a], wr);
      w[a][0] = (WT)wr[0];
      w[a][1] = (WT)wr[1];
      w[a][2] = (WT)wr[2];
    }
  }
  // Common case: the targets are consecutive window cells (no wall folding
  // and inside the window), so one base address serves every target and the
  // offsets are compile-time constants.  b2 has 3 targets per axis starting at
  // i - 1; b1 has 2, starting at i - 1 when its lower weight is the non-zero
  // one (f < 1/2) and at i otherwise.
  constexpr int NT = (SHAPE == SHAPE_B2) ? 3 : 2;
  WT wt[3][NT];
  int lo[3];
  bool fast = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int sft = -1;
    if (SHAPE == SHAPE_B2 || a >= D) {
#pragma unroll
      for (int o = 0; o < NT; ++o) wt[a][o] = w[a][o];
      if (a >= D) sft = 0;
    } else {
      const bool upper = (f[a] >= (R)0.5);  // same split as the b1 weight rule
      sft = upper ? 0 : -1;
      wt[a][0] = upper ? w[a][1] : w[a][0];
      wt[a][1] = upper ? w[a][2] : w[a][1];
    }
    if (a >= D) {
      lo[a] = 0;
      continue;
    }
    const int n = g.n[a];
    int l;
    if (lcell) {
      l = lcell[a];
      if (!g.periodic[a]) fast = fast && idx[a] + sft >= 0 && idx[a] + sft + NT - 1 <= n - 1;
    } else {
      l = idx[a] - origin[a] + TS::G;
      if (g.periodic[a]) {
        if (l < 0) l += n;
        else if (l >= Wd[a]) l -= n;
      } else {
        fast = fast && idx[a] + sft >= 0 && idx[a] + sft + NT - 1 <= n - 1;
      }
    }
    l += sft;
    fast = fast && l >= 0 && l + NT - 1 <= Wd[a] - 1;
    lo[a] = l;
  }
  if (fast) {
    QT* base = win + (lo[0] + TS::W0 * (lo[1] + TS::W1 * lo[2]));
    constexpr int NZ = (D == 3) ? NT : 1;
#pragma unroll
    for (int oz = 0; oz < NZ; ++oz)
#pragma unroll
      for (int oy = 0; oy < NT; ++oy) {
        // b2 weights are at most 3/4 of 2^S1 (S1 = 16 in 3D), so the product
        // of two fits 32 bits and the 24-bit multiplier is exact; a b1 weight
        // reaches 2^S1 and takes the 64-bit product
        typedef typename std::conditional<FIXED, unsigned long long, R>::type PT;
        PT wyz;
        if (FIXED) {
          if (D == 3 && SHAPE == SHAPE_B2)
            wyz = (PT)(uint32_t)__umul24((uint32_t)wt[1][oy], (uint32_t)wt[2][oz]);
          else if (D == 3)
            wyz = (PT)wt[1][oy] * (PT)wt[2][oz];
          else
            wyz = (PT)wt[1][oy];
        } else {
          wyz = (D == 3) ? (PT)(wt[1][oy] * wt[2][oz]) : (PT)wt[1][oy];
        }
#pragma unroll
        for (int ox = 0; ox < NT; ++ox) {
          QT val;
          if (FIXED)
            val = (QT)((unsigned long long)wt[0][ox] * wyz);
          else
            val = (QT)(wt[0][ox] * wyz);
          atomicAdd(base + (ox + TS::W0 * (oy + TS::W1 * oz)), val);
        }
      }
    return;
  }
  // general case (walls, a particle near the window edge, tiny periodic grids
  // whose window overlaps itself): per-target window indices
  int tl[3][3];
  bool inwin = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a >= D) {
      tl[a][0] = tl[a][1] = tl[a][2] = 0;
      continue;
    }
    const int n = g.n[a];
#pragma unroll
    for (int o = 0; o < 3; ++o) {
      int t = idx[a] + o - 1;
      if (g.periodic[a]) {
        t = t < 0 ? t + n : (t >= n ? t - n : t);
      } else {
        t = t < 0 ? 0 : (t >= n ? n - 1 : t);
      }
      int l = t - origin[a] + TS::G;
      if (g.periodic[a]) l = l < 0 ? l + n : (l >= Wd[a] ? l - n : l);
      tl[a][o] = l;
      inwin = inwin && l >= 0 && l < Wd[a];
    }
  }
  constexpr int NZ = (D == 3) ? 3 : 1;
  if (inwin) {
#pragma unroll 1
    for (int oz = 0; oz < NZ; ++oz) {
      const int az = (D == 3) ? oz : 1;
#pragma unroll
      for (int oy = 0; oy < 3; ++oy)
#pragma unroll
        for (int ox = 0; ox < 3; ++ox) {
          QT val;
          if (FIXED) {
            if (D == 3)
              val = (QT)((unsigned long long)w[0][ox] * (unsigned long long)w[1][oy] * (unsigned long long)w[2][az]);
            else
              val = (QT)((unsigned long long)w[0][ox] * (unsigned long long)w[1][oy]);
          } else {
            val = (QT)(w[0][ox] * w[1][oy] * w[2][az]);
          }
          if (val == (QT)0) continue;
          atomicAdd(&win[tl[0][ox] + TS::W0 * (tl[1][oy] + TS::W1 * tl[2][az])], val);
        }
    }
    return;
  }
  // some target outside the window (particle drifted since the last sort):
  // those go straight to HBM
#pragma unroll 1
  for (int oz = 0; oz < NZ; ++oz) {
    const int az = (D == 3) ? oz : 1;
#pragma unroll 1
    for (int oy = 0; oy < 3; ++oy)
#pragma unroll 1
      for (int ox = 0; ox < 3; ++ox) {
        QT val;
        if (FIXED) {
          unsigned long long p = (unsigned long long)w[0][ox] * (unsigned long long)w[1][oy];
          if (D == 3) p *= (unsigned long long)w[2][az];
          val = (QT)p;
        } else {
          val = (QT)(w[0][ox] * w[1][oy] * w[2][az]);
        }
        if (val == (QT)0) continue;
        const int o3[3] = {ox, oy, az};
        int lt[3], t[3];
        bool in = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          lt[a] = tl[a][o3[a]];
          in = in && lt[a] >= 0 && lt[a] < Wd[a];
          int v = (a < D) ? idx[a] + o3[a] - 1 : 0;
          const int n = g.n[a];
          if (a < D) v = g.periodic[a] ? (v < 0 ? v + n : (v >= n ? v - n : v)) : (v < 0 ? 0 : (v >= n ? n - 1 : v));
          t[a] = v;
        }
        if (in) {
          atomicAdd(&win[lt[0] + TS::W0 * (lt[1] + TS::W1 * lt[2])], val);
        } else {
          long long c = (long long)t[0] + (long long)g.n[0] * (t[1] + (long long)g.n[1] * t[2]);
          atomicAdd(&((QT*)Qg)[c], val);
          ++far;
        }
      }
  }
}

// Tile of a particle's new cell, counted for the next tile sort.  Staying in
// this tile (the common case) is not counted here: the workgroup derives it
// at the end from its particle count and the other bins.  A neighbouring
// tile (wrapping on periodic axes) goes to the workgroup's bins, a farther
// one straight into the global count (and bin TB_FAR).
// new-tile bins of a workgroup: 27 tiles around its own (dx + 3 dy + 9 dz,
// offsets + 1), dead, farther tiles, particles left to the FP64 fallback
constexpr int TB_OWN = 13, TB_DEAD = 27, TB_FAR = 28, TB_FALLBACK = 29, TB_N = 30;

template <int D>
__device__ __forceinline__ void count_new_tile(const Geo& g, const int* idx, int tci, int tcj, int tck,
                                               int* tbins, int* tcount) {
  using TS = TileShape<D>;
  const int tn[3] = {idx[0] / TS::T0, idx[1] / TS::T1, (D == 3) ? idx[2] / TS::T2 : 0};
  const int tc[3] = {tci, tcj, tck};
  int b = 0, mul = 1;
  bool near = true;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    int dd = tn[ax] - tc[ax];
    if (g.periodic[ax]) {
      const int nt = g.nt[ax];
      if (dd > 1) dd -= nt;
      if (dd < -1) dd += nt;
    }
    near = near && dd >= -1 && dd <= 1;
    b += (dd + 1) * mul;
    mul *= 3;
  }
  if (near) {
    if (b != TB_OWN) atomicAdd(&tbins[b], 1);
  } else {
    atomicAdd(&tcount[tn[0] + g.nt[0] * (tn[1] + g.nt[1] * tn[2])], 1);
    atomicAdd(&tbins[TB_FAR], 1);
  }
}

// Vertex-field window of a tile: vertices origin-1 .. origin+T+1 per axis, so
// that particles up to one cell outside the tile (drift since the last sort)
// gather from LDS.  Components are packed (2 in 2D, 3 in 3D; the padding slot
// of the global array is not staged).
// Same weights and summation order as gather_E, so both give identical sums.
// lout: the cell's local index in the field window (vertex origin - 1 is 0)
template <int D, typename R>
__device__ __forceinline__ bool gather_E_window(const R* __restrict__ ewin, const Geo& g, const int* origin,
                                                const int* idx, const R* f, R* E, int* lout) {
  using FW = FieldWindow<D>;
  const int Ew[3] = {FW::E0, FW::E1, FW::E2};
  int l[3] = {0, 0, 0};
  bool in = true;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    l[a] = wrap_local(idx[a], origin[a] - 1, g.n[a], g.periodic[a] != 0);
    in = in && l[a] >= 0 && l[a] + 1 < Ew[a];
    lout[a] = l[a];
  }
  if (!in) return false;
  // all 2^D vertices are loaded first (one base address, constant offsets),
  // so the LDS latency is paid once per particle
  const R* e0 = ewin + FW::C * (l[0] + FW::E0 * (l[1] + FW::E1 * l[2]));
  constexpr int NZ = (D == 3) ? 2 : 1;
  R ev[NZ][2][2][FW::C];
#pragma unroll
  for (int z = 0; z < NZ; ++z)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int k = 0; k < FW::C; ++k) ev[z][b][c][k] = e0[FW::C * (c + FW::E0 * (b + FW::E1 * z)) + k];
  R wx[2] = {(R)1 - f[0], f[0]};
  R wy[2] = {(R)1 - f[1], f[1]};
  E[0] = E[1] = E[2] = (R)0;
  if (D == 2) {
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        R w = wx[c] * wy[b];
        E[0] += w * ev[0][b][c][0];
        E[1] += w * ev[0][b][c][1];
      }
  } else {
    R wz[2] = {(R)1 - f[D - 1], f[D - 1]};
#pragma unroll
    for (int z = 0; z < NZ; ++z)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          R w = wx[c] * wy[b] * wz[z];
          E[0] += w * ev[z][b][c][0];
          E[1] += w * ev[z][b][c][1];
          E[2] += w * ev[z][b][c][FW::C - 1];
        }
  }
  return true;
}

// Slot range of the t-th of the TAIL_ITEMS work items that share the particles
// appended since the last sort: [end of the last sorted item, live count).
template <typename R>
__device__ inline void tail_range(const PartArgs<R>& a, int nit, int t, int& begin, int& end) {
  const int b0 = nit > 0 ? a.item_end[nit - 1] : 0;
  const int total = *a.d_n - b0;
  const int per = (total + TAIL_ITEMS - 1) / TAIL_ITEMS;
  begin = b0 + min(total, t * per);
  end = b0 + min(total, (t + 1) * per);
}

// CYC: the cyclotronic velocity step (a uniform B) in place of Boris.
// One work item (a tile's particles, or a slice of those appended since the
// last sort) per workgroup; launched alone (particle_kernel) or for many
// simulations at once (particle_kernel_batch).
template <int D, int MAP, int SHAPE, typename R, bool FIXED, bool CYC>
__device__ __forceinline__ void particle_body(const PartArgs<R>& a, const int item) {
  using TS = TileShape<D>;
  using FW = FieldWindow<D>;
  constexpr int EC = (D == 3) ? 4 : 2;  // components per vertex in the global array
  typedef typename std::conditional<FIXED, unsigned long long, double>::type QT;
  __shared__ QT win[TS::WIN];
  __shared__ R ewin[FW::N * FW::C];
  // predictor-corrector (FP32): the k table of the same window in LDS
  constexpr bool KWIN = MAP == MAP_TABLE_PC && std::is_same<R, float>::value;
  constexpr int KD = D * D;
  __shared__ R kwin[KWIN ? FW::N * KD : 1];
  // tabulated map, FP32: the window's vertex coordinates (D per vertex),
  // relative to the tile's first vertex
  constexpr bool XWIN = MAP == MAP_TABULATED && std::is_same<R, float>::value;
  __shared__ float xwin[XWIN ? FW::N * D : 1];
  __shared__ double red_d[8];
  __shared__ unsigned long long red_u[8][6];
  __shared__ int tbins[TB_N];  // new tiles of the particles (see count_new_tile)

  // maps that allow injection: TAIL_ITEMS more work items share the particles
  // appended since the last sort (they follow the sorted ones), through the
  // global gather and deposit paths, so an injecting species need not sort
  // every step
  constexpr bool TAIL = MAP == MAP_IDENTITY || MAP == MAP_POLAR_LOG || MAP == MAP_TABLE_PC;
  const Geo& g = a.g;
  int tile, begin, end;
  if constexpr (TAIL) {
    const int nit = *a.n_items;
    if (item >= nit + TAIL_ITEMS) return;
    if (item < nit) {
      tile = a.item_tile[item];
      begin = a.item_begin[item];
      end = a.item_end[item];
    } else {
      tile = 0;
      tail_range(a, nit, item - nit, begin, end);
      if (begin >= end) {
        if (threadIdx.x == 0 && a.mode == MODE_PUSH) a.ke_part[item] = 0.0;
        return;
      }
    }
  } else {
    if (item >= *a.n_items) return;
    tile = a.item_tile[item];
    begin = a.item_begin[item];
    end = a.item_end[item];
  }
  int origin[3];
  origin[0] = (tile % g.nt[0]) * TS::T0;
  origin[1] = ((tile / g.nt[0]) % g.nt[1]) * TS::T1;
  origin[2] = (D == 3) ? (tile / (g.nt[0] * g.nt[1])) * TS::T2 : 0;

  const bool deposit = a.mode != MODE_HALFSTEP;
  const bool tcount = a.tcount != nullptr && a.mode == MODE_PUSH;
  if (deposit)
    for (int s = threadIdx.x; s < TS::WIN; s += blockDim.x) win[s] = (QT)0;
  if (threadIdx.x < TB_N) tbins[threadIdx.x] = 0;
  const int tci = tile % g.nt[0], tcj = (tile / g.nt[0]) % g.nt[1], tck = tile / (g.nt[0] * g.nt[1]);
  if (a.mode != MODE_DEPOSIT) {
    // stage the vertex field of the tile and a one-cell halo
    double xref[3] = {0.0, 0.0, 0.0};
    if constexpr (XWIN) {
      // the tile's first vertex (always inside the grid)
      long long v0 = 0;
#pragma unroll
      for (int ax = D - 1; ax >= 0; --ax) v0 = v0 * g.nv[ax] + origin[ax];
#pragma unroll
      for (int ax = 0; ax < D; ++ax) xref[ax] = g.xtab[v0 * D + ax];
    }
    for (int s = threadIdx.x; s < FW::N; s += blockDim.x) {
      const int l0 = s % FW::E0, l1 = (s / FW::E0) % FW::E1, l2 = s / (FW::E0 * FW::E1);
      const int lv[3] = {l0, l1, l2};
      long long v = 0;
      bool ok = true;
      double shift[3] = {0.0, 0.0, 0.0};  // period shifts of the wrapped vertex
#pragma unroll
      for (int ax = D - 1; ax >= 0; --ax) {
        int x = origin[ax] - 1 + lv[ax];
        const int nv = g.nv[ax];
        if (g.periodic[ax]) {
          // x lies in [-1, n + 2]; grids narrower than the window wrap more than once
          while (x < 0) {
            x += nv;
            shift[ax] -= g.L[ax];
          }
          while (x >= nv) {
            x -= nv;
            shift[ax] += g.L[ax];
          }
        } else {
          ok = ok && x >= 0 && x < nv;
        }
        v = v * nv + x;
      }
      if (ok) {
        if constexpr (XWIN) {
#pragma unroll
          for (int ax = 0; ax < D; ++ax) xwin[s * D + ax] = (float)(g.xtab[v * D + ax] + shift[ax] - xref[ax]);
        }
#pragma unroll
        for (int c = 0; c < FW::C; ++c) ewin[s * FW::C + c] = a.Ev[v * EC + c];
        if constexpr (KWIN) {
#pragma unroll
          for (int e = 0; e < KD; ++e) kwin[s * KD + e] = a.kc[v * KC_STRIDE<D> + e];
        }
      }
    }
  }
  __syncthreads();

  double ke = 0.0;
  unsigned long long absorbed = 0, outflow = 0, far = 0, ndep = 0;
  float dmax = 0.0f;  // largest increment of this thread's particles (cells)


  // The state of the thread's next particle is loaded while the current one
  // is processed, so each wave keeps two particles' loads in flight.
  const bool need_v = a.mode != MODE_DEPOSIT;
  int p = begin + (int)threadIdx.x;
  int nkey = -1;
  R nf0 = (R)0, nf1 = (R)0, nf2 = (R)0, nv0 = (R)0, nv1 = (R)0, nv2 = (R)0;
  if (p < end) {
    nkey = pel(a.key, p);
    nf0 = pel(a.off0, p);
    nf1 = pel(a.off1, p);
    if (D == 3) nf2 = pel(a.off2, p);
    if (need_v) {
      nv0 = pel(a.v0, p);
      nv1 = pel(a.v1, p);
      if (a.vz_active) nv2 = pel(a.v2, p);
    }
  }
  for (; p < end; p += (int)blockDim.x) {
    const int key = nkey;
    R f[3] = {nf0, nf1, nf2};
    R v[3] = {nv0, nv1, nv2};
    const int pn = p + (int)blockDim.x;
    if (pn < end) {
      nkey = pel(a.key, pn);
      nf0 = pel(a.off0, pn);
      nf1 = pel(a.off1, pn);
      if (D == 3) nf2 = pel(a.off2, pn);
      if (need_v) {
        nv0 = pel(a.v0, pn);
        nv1 = pel(a.v1, pn);
        if (a.vz_active) nv2 = pel(a.v2, pn);
      }
    }
    if (key < 0) {
      if (tcount) atomicAdd(&tbins[TB_DEAD], 1);
      continue;
    }
    int idx[3] = {key_i(key, g), key_j(key, g), (D == 3) ? key_k(key, g) : 0};
    // the new cell in deposit-window coordinates, when the field window served
    // the gather: its local index + G - 1 + the cell shift of the move
    int lcell[3] = {0, 0, 0};
    bool have_l = false;

    if (need_v) {
      R E[3];
      int le[3] = {0, 0, 0};
      have_l = gather_E_window<D, R>(ewin, g, origin, idx, f, E, le);
      if (!have_l) gather_E<D, R>(a.Ev, g, idx, f, E);
      R vo0 = v[0], vo1 = v[1], vo2 = v[2];
      if (CYC && a.mode == MODE_PUSH) {
        // cyclotronic step: exact gyration; the position moves with the mean
        // velocity of the gyration, which takes v's place once v is stored
        R vm[3];
        cyclotronic_step<R>(v, E, a.qm, a.dt, a.cyc_b, a.cyc_c, a.cyc_s, a.cyc_s1, a.cyc_s2, vm);
        pel(a.v0, p) = v[0];
        pel(a.v1, p) = v[1];
        if (a.vz_active) pel(a.v2, p) = v[2];
        // kinetic energy of the velocity at t_n: before the impulse plus half of it
        const R h = (R)0.5 * a.qm * a.dt;
        const R m0 = vo0 + h * E[0], m1 = vo1 + h * E[1], m2 = vo2 + h * E[2];
        ke += (double)(m0 * m0 + m1 * m1 + m2 * m2);
        v[0] = vm[0];
        v[1] = vm[1];
        v[2] = vm[2];
      } else {
        // Boris (the cyclotronic start-up is the half impulse alone)
        boris_push<R>(v, E, a.B, a.qm, a.dt, a.magnetic != 0 && !CYC);
        pel(a.v0, p) = v[0];
        pel(a.v1, p) = v[1];
        if (a.vz_active) pel(a.v2, p) = v[2];
        if (a.mode == MODE_HALFSTEP) continue;
        ke += (double)(vo0 * v[0] + vo1 * v[1] + vo2 * v[2]);
      }

      R d[3] = {(R)0, (R)0, (R)0};
      bool conv;
      if constexpr (MAP == MAP_TABLE_PC) {
        move_pc<D, R, KWIN>(g, a.kc, kwin, origin, idx, f, v, a.dt, d);
        conv = true;
      } else if constexpr (MAP == MAP_TABULATED) {
        bool done = false;
        if constexpr (XWIN) {
          const float disp32[3] = {(float)a.dt * (float)v[0], (float)a.dt * (float)v[1], (float)a.dt * (float)v[2]};
          float d32[3] = {0.f, 0.f, 0.f};
          const float f32[3] = {(float)f[0], (float)f[1], (float)f[2]};
          if (move_tab_window<D>(xwin, g, origin, idx, f32, disp32, d32)) {
#pragma unroll
            for (int ax = 0; ax < D; ++ax) d[ax] = (R)d32[ax];
            conv = true;
            done = true;
          }
        }
        if (!done) {
          if constexpr (XWIN) {
            // the FP64 fallback kernel inverts it on the global table (kept out
            // of this kernel, whose registers it would otherwise set)
            conv = false;
          } else {
            double f64[3] = {(double)f[0], (double)f[1], (double)f[2]}, disp[3], dd[3];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) disp[ax] = (double)a.dt * (double)v[ax];
            conv = move_tab<D>(g, idx, f64, disp, 16, dd);
#pragma unroll
            for (int ax = 0; ax < D; ++ax) d[ax] = (R)dd[ax];
          }
        }
      } else
        conv = move_delta<D, MAP, R>(g, idx, f, v, a.dt, a.inv_dxc, a.newton_maxit, a.newton_tol,
                                        a.kappa, d);
      if (!conv) {
        // rare: the FP64 fallback kernel moves, deposits and counts this particle
        int slot = atomicAdd(a.fb_count, 1);
        if (slot < a.fb_cap) a.fb_queue[slot] = p;
        if (tcount) atomicAdd(&tbins[TB_FALLBACK], 1);
        continue;
      }
#pragma unroll
      for (int ax = 0; ax < D; ++ax) dmax = fmaxf(dmax, fabsf((float)d[ax]));
      int sh[3] = {0, 0, 0};
      int dead = place_particle<D, R>(g, a.pbc_lo, a.pbc_hi, idx, f, d, sh);
#pragma unroll
      for (int ax = 0; ax < D; ++ax) lcell[ax] = le[ax] + TS::G - 1 + sh[ax];
      if (dead) {
        pel(a.key, p) = dead;
        absorbed += dead == -1 ? 1 : 0;
        outflow += dead == -2 ? 1 : 0;
        if (tcount) atomicAdd(&tbins[TB_DEAD], 1);
        continue;
      }
      pel(a.key, p) = make_key(idx[0], idx[1], idx[2], g);
      if (tcount) count_new_tile<D>(g, idx, tci, tcj, tck, tbins, a.tcount);
      pel(a.off0, p) = f[0];
      pel(a.off1, p) = f[1];
      if (D == 3) pel(a.off2, p) = f[2];
    }
    deposit_particle<D, SHAPE, R, FIXED, QT>(g, origin, win, a.Q, idx, f, a.S1, far, have_l ? lcell : nullptr);
    ++ndep;
  }

  if (deposit) {
    __syncthreads();
    for (int s = threadIdx.x; s < TS::WIN; s += blockDim.x) {
      QT val = win[s];
      if (val == (QT)0) continue;
      int lx = s % TS::W0;
      int ly = (s / TS::W0) % TS::W1;
      int lz = s / (TS::W0 * TS::W1);
      int l[3] = {lx, ly, lz};
      int t[3] = {0, 0, 0};
      bool ok = true;
#pragma unroll
      for (int ax = 0; ax < D; ++ax) {
        int v = origin[ax] - TS::G + l[ax];
        const int n = g.n[ax];
        if (g.periodic[ax]) {
          while (v < 0) v += n;
          while (v >= n) v -= n;
        } else if (v < 0 || v >= n) {
          ok = false;
        }
        t[ax] = v;
      }
      if (!ok) continue;
      long long c = (long long)t[0] + (long long)g.n[0] * (t[1] + (long long)g.n[1] * t[2]);
      atomicAdd(&((QT*)a.Q)[c], val);
    }
  }

  if (tcount) {
    __syncthreads();
    if (threadIdx.x == 0) {
      int other = 0;
      for (int b = 0; b < TB_N; ++b) other += b == TB_OWN ? 0 : tbins[b];
      // the item's bounds are read again rather than kept live across the loop
      int nb;
      if constexpr (TAIL) {
        const int nit = *a.n_items;
        if (item < nit) {
          nb = a.item_end[item] - a.item_begin[item];
        } else {
          int b0, e0;
          tail_range(a, nit, item - nit, b0, e0);
          nb = e0 - b0;
        }
      } else {
        nb = a.item_end[item] - a.item_begin[item];
      }
      tbins[TB_OWN] = nb - other;
    }
    __syncthreads();
    if (threadIdx.x < 27) {
      const int c = tbins[threadIdx.x];
      if (c) {
        const int dd[3] = {(int)threadIdx.x % 3 - 1, ((int)threadIdx.x / 3) % 3 - 1, (int)threadIdx.x / 9 - 1};
        const int tc[3] = {tci, tcj, tck};
        int t[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const int nt = g.nt[ax];
          t[ax] = tc[ax] + dd[ax];
          t[ax] = t[ax] < 0 ? t[ax] + nt : (t[ax] >= nt ? t[ax] - nt : t[ax]);
        }
        atomicAdd(&a.tcount[t[0] + g.nt[0] * (t[1] + g.nt[1] * t[2])], c);
      }
    } else if (threadIdx.x == TB_DEAD && tbins[TB_DEAD]) {
      atomicAdd(&a.tcount[g.ntiles], tbins[TB_DEAD]);
    }
  }

  // block sums of the diagnostics
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (a.drift && a.mode == MODE_PUSH) {
    for (int o = 32; o > 0; o >>= 1) dmax = fmaxf(dmax, __shfl_xor(dmax, o, 64));
    // non-negative floats order like their bit patterns
    if (lane == 0 && dmax > 0.0f) atomicMax(a.drift, __float_as_uint(dmax));
  }
  double kes = wave_sum(ke);
  unsigned long long cs[6] = {wave_sum_u64(absorbed), wave_sum_u64(outflow), 0ull, wave_sum_u64(far),
                              0ull, deposit ? wave_sum_u64(ndep) : 0ull};
  if (lane == 0) {
    red_d[wv] = kes;
    for (int i = 0; i < 6; ++i) red_u[wv][i] = cs[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) / 64;
    double s = 0.0;
    unsigned long long u[6] = {0, 0, 0, 0, 0, 0};
    for (int w = 0; w < nw; ++w) {
      s += red_d[w];
      for (int i = 0; i < 6; ++i) u[i] += red_u[w][i];
    }
    // per-item slot, summed in a fixed order afterwards (deterministic energy)
    if (a.mode == MODE_PUSH) a.ke_part[item] = s;
    for (int i = 0; i < 5; ++i)
      if (u[i]) atomicAdd(&a.counters[i], u[i]);
    if (u[5]) atomicAdd(&a.counters[9], u[5]);
  }
}

// Threads per workgroup of the particle kernel: 512 for the 3D
// predictor-corrector and tabulated-map Newton kernels, whose LDS windows
// (about 78 and 46 KB) leave room for two such workgroups per CU, so that a
// CU keeps 16 waves in flight (8 and 12 with 256-thread workgroups); 256 for
// the others.
template <int D, int MAP>
constexpr int pk_threads() {
  return (D == 3 && (MAP == MAP_TABLE_PC || MAP == MAP_TABULATED)) ? 512 : 256;
}
// Waves per SIMD the register allocation aims at: four for the 3D kernels of
// 512-thread workgroups (two per CU), five for the other FP32 kernels, two
// for FP64.
template <int D, int MAP, bool FIXED>
constexpr int pk_waves() {
  return !FIXED ? 2 : (D == 3 && (MAP == MAP_TABLE_PC || MAP == MAP_TABULATED)) ? 4 : 5;
}

template <int D, int MAP, int SHAPE, typename R, bool FIXED, bool CYC>
__global__ __launch_bounds__((pk_threads<D, MAP>())) __attribute__((amdgpu_waves_per_eu(pk_waves<D, MAP, FIXED>(), 8))) void particle_kernel(
    PartArgs<R> a) {
  particle_body<D, MAP, SHAPE, R, FIXED, CYC>(a, blockIdx.x);
}

// The work items of several simulations (or species) in one launch: entry e
// owns the workgroups base[e] .. base[e + 1] - 1, with its own arguments.
template <int D, int MAP, int SHAPE, typename R, bool FIXED, bool CYC>
__global__ __launch_bounds__((pk_threads<D, MAP>())) __attribute__((amdgpu_waves_per_eu(pk_waves<D, MAP, FIXED>(), 8))) void particle_kernel_batch(
    const PartArgs<R>* __restrict__ A, const int* __restrict__ base, int n) {
  const int b = (int)blockIdx.x;
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (base[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  particle_body<D, MAP, SHAPE, R, FIXED, CYC>(A[lo], b - base[lo]);
}

// Deposit of one particle straight into HBM (global atomics): used for the
// few particles handled outside the tile kernel (FP64 fallback, injection).
template <int D, typename R, bool FIXED>
__device__ inline void deposit_global(const Geo& g, int shape, int S1, const int* idx, const R* f,
                                      void* Q) {
  typedef typename std::conditional<FIXED, unsigned long long, double>::type QT;
  QT w[3][3];
  int tg[3][3];
  for (int ax = 0; ax < 3; ++ax) {
    if (ax >= D) {
      w[ax][0] = w[ax][2] = (QT)0;
      w[ax][1] = (QT)1;
      tg[ax][0] = tg[ax][1] = tg[ax][2] = 0;
      continue;
    }
    if (FIXED) {
      uint32_t wi[3];
      if (shape == SHAPE_B2)
        weights_fixed<SHAPE_B2>((double)f[ax], S1, wi);
      else
        weights_fixed<SHAPE_B1>((double)f[ax], S1, wi);
      for (int o = 0; o < 3; ++o) w[ax][o] = (QT)wi[o];
    } else {
      R wr[3];
      if (shape == SHAPE_B2)
        weights_real<SHAPE_B2, R>(f[ax], wr);
      else
        weights_real<SHAPE_B1, R>(f[ax], wr);
      for (int o = 0; o < 3; ++o) w[ax][o] = (QT)wr[o];
    }
    const int n = g.n[ax];
    for (int o = 0; o < 3; ++o) {
      int t = idx[ax] + o - 1;
      if (g.periodic[ax])
        t = t < 0 ? t + n : (t >= n ? t - n : t);
      else
        t = t < 0 ? 0 : (t >= n ? n - 1 : t);
      tg[ax][o] = t;
    }
  }
  const int nz = (D == 3) ? 3 : 1;
  for (int oz = 0; oz < nz; ++oz) {
    const int az = (D == 3) ? oz : 1;
    for (int oy = 0; oy < 3; ++oy)
      for (int ox = 0; ox < 3; ++ox) {
        QT val;
        if (FIXED) {
          unsigned long long p = (unsigned long long)w[0][ox] * (unsigned long long)w[1][oy];
          if (D == 3) p *= (unsigned long long)w[2][az];
          val = (QT)p;
        } else {
          val = w[0][ox] * w[1][oy] * w[2][az];
        }
        if (val == (QT)0) continue;
        long long c = (long long)tg[0][ox] + (long long)g.n[0] * (tg[1][oy] + (long long)g.n[1] * tg[2][az]);
        atomicAdd(&((QT*)Q)[c], val);
      }
  }
}

// Particles whose position update was left by the tile kernel: globalised FP64
// Newton (continuation over the physical displacement), boundaries, deposit.
// Their new velocity is already stored.
template <int D, int MAP, typename R, bool FIXED>
__device__ __forceinline__ void fallback_body(const PartArgs<R>& a, int shape) {
  const Geo& g = a.g;
  const int n = min(*a.fb_count, a.fb_cap);
  unsigned long long done = 0, failed = 0, absorbed = 0, outflow = 0, ndep = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int p = a.fb_queue[i];
    const int key = a.key[p];
    int idx[3] = {key_i(key, g), key_j(key, g), (D == 3) ? key_k(key, g) : 0};
    double f[3] = {(double)a.off0[p], (double)a.off1[p], (D == 3) ? (double)a.off2[p] : 0.0};
    double v[3] = {(double)a.v0[p], (double)a.v1[p], a.vz_active ? (double)a.v2[p] : 0.0};
    if (a.cyclo) {
      // the displacement of a cyclotronic step: the mean velocity of the gyration
      const double b[3] = {(double)a.cyc_b[0], (double)a.cyc_b[1], (double)a.cyc_b[2]};
      double vn[3] = {v[0], v[1], v[2]};
      cyclotronic_mean<double>(vn, b, (double)a.cyc_c, (double)a.cyc_s, (double)a.cyc_s1, (double)a.cyc_s2, v);
    }
    double disp[3] = {0.0, 0.0, 0.0}, d[3] = {0.0, 0.0, 0.0};
    for (int ax = 0; ax < D; ++ax)
      disp[ax] = (MAP == MAP_SINUSOIDAL) ? (double)a.dt * v[ax] / g.dxc[ax] : (double)a.dt * v[ax];
    bool ok = move_fallback<D, MAP>(g, idx, f, disp, (double)a.kappa, d);
    ++done;
    failed += ok ? 0 : 1;
    if (a.drift) {
      float m = 0.0f;
      for (int ax = 0; ax < D; ++ax) m = fmaxf(m, (float)fabs(d[ax]));
      atomicMax(a.drift, __float_as_uint(m));
    }
    int dead = place_particle<D, double>(g, a.pbc_lo, a.pbc_hi, idx, f, d);
    if (dead) {
      a.key[p] = dead;
      absorbed += dead == -1 ? 1 : 0;
      outflow += dead == -2 ? 1 : 0;
      if (a.tcount) atomicAdd(&a.tcount[g.ntiles], 1);
      continue;
    }
    if (a.tcount) {
      using TS = TileShape<D>;
      atomicAdd(&a.tcount[idx[0] / TS::T0 + g.nt[0] * (idx[1] / TS::T1 + g.nt[1] * ((D == 3) ? idx[2] / TS::T2 : 0))],
                1);
    }
    R fr[3];
    for (int ax = 0; ax < 3; ++ax) {
      R r = (R)f[ax];
      if (r >= (R)1) r = std::is_same<R, float>::value ? (R)0.99999994f : (R)f[ax];
      fr[ax] = r;
    }
    a.key[p] = make_key(idx[0], idx[1], idx[2], g);
    a.off0[p] = fr[0];
    a.off1[p] = fr[1];
    if (D == 3) a.off2[p] = fr[2];
    deposit_global<D, R, FIXED>(g, shape, a.S1, idx, fr, a.Q);
    ++ndep;
  }
  if (done) {
    atomicAdd(&a.counters[2], done);
    if (failed) atomicAdd(&a.counters[4], failed);
    if (absorbed) atomicAdd(&a.counters[0], absorbed);
    if (outflow) atomicAdd(&a.counters[1], outflow);
    if (ndep) atomicAdd(&a.counters[9], ndep);
  }
}

// Workgroups of the fallback launch (grid-stride over the queue, whose length
// only the device knows): one per CU, so that a step with many FP64 updates
// (the tabulated map's window failures) spreads them over the whole GPU; a
// batched launch, whose entries are small cases, takes fewer per entry.
constexpr int FB_BLOCKS = 256;
constexpr int FB_BATCH_BLOCKS = 64;

template <int D, int MAP, typename R, bool FIXED>
__global__ __launch_bounds__(256) void fallback_kernel(PartArgs<R> a, int shape) {
  fallback_body<D, MAP, R, FIXED>(a, shape);
}
// one row of workgroups (blockIdx.y) per entry
template <int D, int MAP, typename R, bool FIXED>
__global__ __launch_bounds__(256) void fallback_kernel_batch(const PartArgs<R>* __restrict__ A, int shape) {
  fallback_body<D, MAP, R, FIXED>(A[blockIdx.y], shape);
}

// ----------------------------------------------------------------------------
// injection of a Maxwellian at rest through the upper face of axis 0 (the
// outer wall): per step floor(lambda) + Bernoulli(frac lambda) particles,
// lambda = n0 v_th / sqrt(2 pi) A dt / w.  Each: uniform tangential logical
// position on the face, inward normal speed v_th sqrt(-2 ln u) (flux-weighted
// half-Maxwellian), tangential components N(0, v_th^2) by Box-Muller, and a
// free flight over a uniform fraction of the step from the face, mapped back
// to xi by Newton on the map increment.  FP64 throughout (few particles).
// Random numbers: Philox4x32-10, key (seed), counter (step, k, species, use).
// Particles are appended after the live ones; their charge is deposited with
// global atomics (they join a tile at the next sort).
// ----------------------------------------------------------------------------
template <typename R>
struct InjectArgs {
  Geo g;
  int32_t* key;
  R* off[3];
  R* vel[3];
  uint32_t* id;
  const int* d_n;
  int cap;
  void* Q;
  int shape;
  int S1;
  double lam, vth, dt, kappa;
  double s_drift;  // inward drift of the injected Maxwellian in thermal speeds (0: at rest)
  uint32_t k0, k1, step, species;
  unsigned long long* counters;  // [5] injected, [6] dropped for capacity, [7] next identifier,
                                 // [8] entry flight left the domain, [9] deposited
  int* count_out;
  int* tcount;  // when set: the injected particles' tiles are counted for the next sort
};

__device__ inline int injection_count(double lam, uint32_t k0, uint32_t k1, uint32_t step,
                                      uint32_t species) {
  uint32_t r[4];
  philox4x32_10(step, 0xFFFFFFFFu, species, 2u, k0, k1, r);
  double fl = floor(lam);
  return (int)fl + (unit_open(r[0]) < lam - fl ? 1 : 0);
}

// Inward normal speed (thermal units) of injected particle k: distributed as
// w exp(-(w - s)^2 / 2) on w > 0 (flux-weighted drifting Maxwellian).  s = 0:
// sqrt(-2 ln u).  s > 0: proposals from N(s + delta, 1), delta the inverse of
// the distribution's mode 2 / (s + sqrt(s^2 + 4)), each kept with probability
// delta w exp(1 - delta w) (the target over proposal ratio, scaled to a
// maximum of 1); attempt t draws from counter (step, k, species, 3 + t), at
// most 64 attempts.
__device__ inline double inject_normal_speed(double s, uint32_t k0, uint32_t k1, uint32_t step, uint32_t k,
                                             uint32_t species, double u_rayleigh) {
  if (s <= 0.0) return sqrt(-2.0 * log(u_rayleigh));
  const double delta = 2.0 / (s + sqrt(s * s + 4.0)), mu = s + delta;
  double w = mu;
  for (uint32_t t = 0; t < 64; ++t) {
    uint32_t r[4];
    philox4x32_10(step, k, species, 3u + t, k0, k1, r);
    double sn, cs;
    sincospi(2.0 * unit_open(r[1]), &sn, &cs);
    w = mu + sqrt(-2.0 * log(unit_open(r[0]))) * cs;
    if (w > 0.0 && unit_open(r[2]) < delta * w * exp(1.0 - delta * w)) return w;
  }
  return w > 0.0 ? w : mu;
}

template <int D, int MAP, typename R, bool FIXED>
__global__ __launch_bounds__(256) void inject_kernel(InjectArgs<R> a) {
  const Geo& g = a.g;
  const int count = injection_count(a.lam, a.k0, a.k1, a.step, a.species);
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0) *a.count_out = count;
  if (k >= count) return;
  const int base = *a.d_n;
  const long long slot = (long long)base + k;
  if (slot >= a.cap) {
    atomicAdd(&a.counters[6], 1ull);
    return;
  }
  uint32_t ra[4], rb[4];
  philox4x32_10(a.step, (uint32_t)k, a.species, 0u, a.k0, a.k1, ra);
  philox4x32_10(a.step, (uint32_t)k, a.species, 1u, a.k0, a.k1, rb);
  double xi_f[3] = {1.0, unit_open(ra[0]), (D == 3) ? unit_open(rb[1]) : 0.0};
  double vn = a.vth * inject_normal_speed(a.s_drift, a.k0, a.k1, a.step, (uint32_t)k, a.species, unit_open(ra[1]));
  double rho = sqrt(-2.0 * log(unit_open(ra[2])));
  double sn, cs;
  sincospi(2.0 * unit_open(ra[3]), &sn, &cs);
  double t1 = a.vth * rho * cs, t2 = a.vth * rho * sn;
  double frac = unit_open(rb[0]);
  double j[3][3], xf[3];
  map_jacobi(g, xi_f, j, xf);
  double e[3][3];
  for (int b = 0; b < 3; ++b) {
    double nrm = sqrt(j[0][b] * j[0][b] + j[1][b] * j[1][b] + j[2][b] * j[2][b]);
    for (int c = 0; c < 3; ++c) e[b][c] = j[c][b] / nrm;
  }
  double v[3];
  for (int c = 0; c < 3; ++c) v[c] = -vn * e[0][c] + t1 * e[1][c];
  if (D == 2)
    v[2] += t2;
  else
    for (int c = 0; c < 3; ++c) v[c] += t2 * e[2][c];
  // base: upper face of the last cell along axis 0
  int idx[3] = {g.n[0] - 1, 0, 0};
  double f[3] = {1.0, 0.0, 0.0};
  for (int ax = 1; ax < D; ++ax) {
    double u = xi_f[ax] * g.n[ax];
    int i = (int)floor(u);
    if (i > g.n[ax] - 1) i = g.n[ax] - 1;
    idx[ax] = i;
    f[ax] = u - i;
  }
  double disp[3] = {0.0, 0.0, 0.0};
  for (int c = 0; c < D; ++c) disp[c] = (MAP == MAP_IDENTITY) ? frac * a.dt * v[c] / g.dxc[c] : frac * a.dt * v[c];
  double d[3] = {0.0, 0.0, 0.0};
  if (MAP == MAP_IDENTITY) {
    for (int c = 0; c < D; ++c) d[c] = disp[c];
  } else {
    double J;
    bool ok = (MAP == MAP_POLAR_LOG) ? newton_polar<double>(g, idx, f, disp, d, 1e-12, a.kappa, 24, J)
                                     : newton_sinusoidal<D, double>(g, idx, f, disp, d, 1e-12, a.kappa, 24, J);
    if (!ok) move_fallback<D, MAP>(g, idx, f, disp, a.kappa, d);
  }
  int dead = 0;
  R fo[3];
  for (int ax = 0; ax < D; ++ax) {
    double u = f[ax] + d[ax];
    double fl = floor(u);
    int ni = idx[ax] + (int)fl;
    double nf = u - fl;
    const int n = g.n[ax];
    if (g.periodic[ax]) {
      ni %= n;
      if (ni < 0) ni += n;
    } else if (ni < 0 || ni >= n) {
      dead = 1;
    }
    idx[ax] = ni;
    R r = (R)nf;
    if (r >= (R)1) r = (R)0.99999994;  // keep the stored offset inside [0, 1)
    fo[ax] = r;
  }
  for (int ax = D; ax < 3; ++ax) fo[ax] = (R)0;
  // identifiers follow the draw index k, so they do not depend on scheduling
  if (a.id) a.id[slot] = (uint32_t)(a.counters[7] + (unsigned long long)k);
  if (dead) {
    // its slot stays in use until the next sort: counted, so the live count
    // (slots less the departures since the last sort) leaves it out
    a.key[slot] = -2;
    atomicAdd(&a.counters[8], 1ull);
    if (a.tcount) atomicAdd(&a.tcount[g.ntiles], 1);
    return;
  }
  a.key[slot] = make_key(idx[0], idx[1], idx[2], g);
  if (a.tcount) {
    using TS = TileShape<D>;
    atomicAdd(&a.tcount[idx[0] / TS::T0 + g.nt[0] * (idx[1] / TS::T1 + g.nt[1] * ((D == 3) ? idx[2] / TS::T2 : 0))],
              1);
  }
  for (int ax = 0; ax < D; ++ax) a.off[ax][slot] = fo[ax];
  for (int c = 0; c < 3; ++c) a.vel[c][slot] = (R)v[c];
  atomicAdd(&a.counters[5], 1ull);
  atomicAdd(&a.counters[9], 1ull);
  deposit_global<D, R, FIXED>(g, a.shape, a.S1, idx, fo, a.Q);
}

__global__ void inject_finish_kernel(int* d_n, const int* count, int cap, unsigned long long* counters) {
  int n = *d_n + *count;
  *d_n = n < cap ? n : cap;
  counters[7] += (unsigned long long)*count;
}

// ----------------------------------------------------------------------------
// tile sort
// ----------------------------------------------------------------------------
// Each workgroup sorts one chunk of SORT_CHUNK consecutive particles.  Global
// atomics on the tile counters cost a round trip through the memory-side
// cache, so the chunk is first histogrammed in LDS over the tile range it
// spans (particles are nearly tile-sorted: the range is small) and only one
// global atomic per (chunk, tile) is issued.  Chunks spanning more than
// SORT_BINS tiles (the first sort of unsorted input) use per-wave aggregated
// global atomics instead.
constexpr int SORT_CHUNK = 4096;
constexpr int SORT_BINS = 2048;

template <int D>
__device__ inline int tile_or_dead(int k, const Geo& g) {
  return k < 0 ? g.ntiles : tile_of_key<D>(k, g);
}

// block-wide min / max of v (thread 0 broadcasts through LDS)
__device__ inline void block_minmax(int v_min, int v_max, int* out) {
  __shared__ int smin[8], smax[8];
  for (int o = 32; o > 0; o >>= 1) {
    v_min = min(v_min, __shfl_xor(v_min, o, 64));
    v_max = max(v_max, __shfl_xor(v_max, o, 64));
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    smin[w] = v_min;
    smax[w] = v_max;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = smin[0], b = smax[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
      a = min(a, smin[i]);
      b = max(b, smax[i]);
    }
    out[0] = a;
    out[1] = b;
  }
  __syncthreads();
}

template <int D>
__global__ __launch_bounds__(256) void tile_hist_kernel(const int32_t* __restrict__ key,
                                                        const int* __restrict__ d_n, int* counts,
                                                        Geo g) {
  __shared__ int bins[SORT_BINS];
  __shared__ int range[2];
  __shared__ int dead;
  const int n = *d_n;
  const int p0 = blockIdx.x * SORT_CHUNK;
  if (p0 >= n) return;
  const int p1 = min(n, p0 + SORT_CHUNK);
  int tmin = 1 << 30, tmax = -1;
  for (int p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    int k = key[p];
    if (k < 0) continue;
    int t = tile_of_key<D>(k, g);
    tmin = min(tmin, t);
    tmax = max(tmax, t);
  }
  if (threadIdx.x == 0) dead = 0;
  block_minmax(tmin, tmax, range);
  const int lo = range[0];
  if (range[1] - lo < SORT_BINS) {
    for (int b = threadIdx.x; b < SORT_BINS; b += blockDim.x) bins[b] = 0;
    __syncthreads();
    for (int q = p0; q < p1; q += blockDim.x) {
      int p = q + threadIdx.x;
      int k = p < p1 ? key[p] : 0;
      bool live = p < p1 && k >= 0;
      if (p < p1 && k < 0) atomicAdd(&dead, 1);
      agg_inc(bins, live ? tile_of_key<D>(k, g) - lo : 0, live);
    }
    __syncthreads();
    for (int b = threadIdx.x; b <= range[1] - lo; b += blockDim.x)
      if (bins[b]) atomicAdd(&counts[lo + b], bins[b]);
    if (threadIdx.x == 0 && dead) atomicAdd(&counts[g.ntiles], dead);
  } else {
    for (int q = p0; q < p1; q += blockDim.x) {
      int p = q + threadIdx.x;
      bool active = p < p1;
      int t = active ? tile_or_dead<D>(key[p], g) : 0;
      agg_inc(counts, t, active);
    }
  }
}

// Single workgroup: exclusive scan of the tile counts (dead bin last), work
// items of at most `chunk` particles per tile, new live count.
__global__ __launch_bounds__(1024) void tile_scan_kernel(const int* __restrict__ counts, int ntiles,
                                                         int chunk, int* start, int* cursor,
                                                         int* n_items, int* item_tile,
                                                         int* item_begin, int* item_end, int* d_n) {
  __shared__ long long sp[1024];
  __shared__ long long si[1024];
  const int T = blockDim.x;
  const int tid = threadIdx.x;
  const int per = (ntiles + T - 1) / T;
  const int t0 = tid * per;
  const int t1 = min(ntiles, t0 + per);
  long long ps = 0, is = 0;
  for (int t = t0; t < t1; ++t) {
    int c = counts[t];
    ps += c;
    is += (c + chunk - 1) / chunk;
  }
  sp[tid] = ps;
  si[tid] = is;
  __syncthreads();
  for (int o = 1; o < T; o <<= 1) {
    long long a = (tid >= o) ? sp[tid - o] : 0;
    long long b = (tid >= o) ? si[tid - o] : 0;
    __syncthreads();
    sp[tid] += a;
    si[tid] += b;
    __syncthreads();
  }
  long long pbase = sp[tid] - ps;
  long long ibase = si[tid] - is;
  for (int t = t0; t < t1; ++t) {
    int c = counts[t];
    start[t] = (int)pbase;
    cursor[t] = (int)pbase;
    // the tile's particles in k equal parts (a full chunk and a small
    // remainder would cost the remainder a whole workgroup's set-up)
    int k = (c + chunk - 1) / chunk;
    for (int j = 0; j < k; ++j) {
      item_tile[ibase + j] = t;
      item_begin[ibase + j] = (int)(pbase + (long long)j * c / k);
      item_end[ibase + j] = (int)(pbase + (long long)(j + 1) * c / k);
    }
    pbase += c;
    ibase += k;
  }
  if (tid == T - 1) {
    long long alive = sp[T - 1];
    start[ntiles] = (int)alive;
    cursor[ntiles] = (int)alive;
    start[ntiles + 1] = (int)(alive + counts[ntiles]);
    *n_items = (int)si[T - 1];
    *d_n = (int)alive;
  }
}

template <int D, typename R>
__global__ __launch_bounds__(256) void tile_scatter_kernel(
    const int* __restrict__ start, int* cursor, Geo g, const int32_t* __restrict__ key_in,
    int32_t* key_out, const R* __restrict__ o0i, const R* __restrict__ o1i, const R* __restrict__ o2i,
    R* o0o, R* o1o, R* o2o, const R* __restrict__ v0i, const R* __restrict__ v1i,
    const R* __restrict__ v2i, R* v0o, R* v1o, R* v2o, const uint32_t* __restrict__ id_in,
    uint32_t* id_out) {
  __shared__ int bins[SORT_BINS];
  __shared__ int rank[SORT_CHUNK];
  __shared__ int range[2];
  const int n = start[g.ntiles + 1];
  const int p0 = blockIdx.x * SORT_CHUNK;
  if (p0 >= n) return;
  const int p1 = min(n, p0 + SORT_CHUNK);
  int tmin = 1 << 30, tmax = -1;
  for (int p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    int k = key_in[p];
    if (k < 0) continue;
    int t = tile_of_key<D>(k, g);
    tmin = min(tmin, t);
    tmax = max(tmax, t);
  }
  block_minmax(tmin, tmax, range);
  const int lo = range[0];
  const bool local = range[1] - lo < SORT_BINS;
  if (local) {
    for (int b = threadIdx.x; b < SORT_BINS; b += blockDim.x) bins[b] = 0;
    __syncthreads();
    // rank of each particle among the chunk's particles of its tile
    for (int q = p0; q < p1; q += blockDim.x) {
      int p = q + threadIdx.x;
      int k = p < p1 ? key_in[p] : -1;
      bool live = k >= 0;
      int r = agg_inc(bins, live ? tile_of_key<D>(k, g) - lo : 0, live);
      if (p < p1) rank[p - p0] = r;
    }
    __syncthreads();
    // one global reservation per tile present in the chunk
    for (int b = threadIdx.x; b <= range[1] - lo; b += blockDim.x)
      bins[b] = bins[b] ? atomicAdd(&cursor[lo + b], bins[b]) : 0;
    __syncthreads();
  }
  for (int q = p0; q < p1; q += blockDim.x) {
    int p = q + threadIdx.x;
    bool active = p < p1;
    int k = active ? key_in[p] : -1;
    bool live = active && k >= 0;
    int t = live ? tile_of_key<D>(k, g) : 0;
    int dst;
    if (local)
      dst = live ? bins[t - lo] + rank[p - p0] : 0;
    else
      dst = agg_inc(cursor, t, live);
    if (live) {
      key_out[dst] = k;
      o0o[dst] = o0i[p];
      o1o[dst] = o1i[p];
      if (D == 3) o2o[dst] = o2i[p];
      v0o[dst] = v0i[p];
      v1o[dst] = v1i[p];
      v2o[dst] = v2i[p];
      if (id_in) id_out[dst] = id_in[p];
    }
  }
}

// ----------------------------------------------------------------------------
// conversions between the ABI's linear cell index and the packed key
// ----------------------------------------------------------------------------
__global__ void lin_to_key_kernel(const int32_t* __restrict__ lin, int32_t* key, int n, Geo g,
                                  int* bad) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int c = lin[p];
  if (c < 0 || (long long)c >= g.ncells) {
    key[p] = -1;
    atomicAdd(bad, 1);
    return;
  }
  int i = c % g.n[0];
  int j = (c / g.n[0]) % g.n[1];
  int k = c / (g.n[0] * g.n[1]);
  key[p] = make_key(i, j, k, g);
}

__global__ void key_to_lin_kernel(const int32_t* __restrict__ key, int32_t* lin, int n, Geo g) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int k = key[p];
  lin[p] = k < 0 ? k : key_i(k, g) + g.n[0] * (key_j(k, g) + g.n[1] * key_k(k, g));
}

__global__ void iota_kernel(uint32_t* id, int n) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) id[p] = (uint32_t)p;
}

template <typename R>
__global__ void offsets_check_kernel(const R* __restrict__ o, long long n, int* bad) {
  long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  R v = o[p];
  if (!(v >= (R)0 && v < (R)1)) atomicAdd(bad, 1);
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------
template <typename R>
static PartArgs<R> make_part_args(const ParticleLaunch& L) {
  PartArgs<R> a;
  a.key = L.key;
  a.off0 = (R*)L.off[0];
  a.off1 = (R*)L.off[1];
  a.off2 = (R*)L.off[2];
  a.v0 = (R*)L.vel[0];
  a.v1 = (R*)L.vel[1];
  a.v2 = (R*)L.vel[2];
  a.item_tile = L.item_tile;
  a.item_begin = L.item_begin;
  a.item_end = L.item_end;
  a.n_items = L.n_items;
  a.d_n = L.d_n;
  a.Ev = (const R*)L.Ev;
  a.kc = (const R*)L.kc;
  a.Q = L.Q;
  a.g = L.g;
  for (int i = 0; i < 3; ++i) {
    a.pbc_lo[i] = L.pbc_lo[i];
    a.pbc_hi[i] = L.pbc_hi[i];
    a.B[i] = (R)L.B[i];
  }
  a.qm = (R)L.qm;
  a.dt = (R)L.dt;
  a.magnetic = L.magnetic;
  a.cyclo = L.cyclo;
  for (int i = 0; i < 3; ++i) a.cyc_b[i] = (R)L.cyc_b[i];
  a.cyc_c = (R)L.cyc_c;
  a.cyc_s = (R)L.cyc_s;
  a.cyc_s1 = (R)L.cyc_s1;
  a.cyc_s2 = (R)L.cyc_s2;
  a.vz_active = L.vz_active;
  a.mode = L.mode;
  a.S1 = L.S1;
  a.newton_maxit = L.newton_maxit;
  a.newton_tol = (R)L.newton_tol;
  a.kappa = (R)L.kappa;
  for (int i = 0; i < 3; ++i) a.inv_dxc[i] = (R)(1.0 / L.g.dxc[i]);
  a.ke_scale = L.ke_scale;
  a.ke_part = L.ke_part;
  a.tcount = L.tile_counts;
  a.drift = L.drift;
  a.ke = L.ke;
  a.counters = L.counters;
  a.fb_queue = L.fb_queue;
  a.fb_count = L.fb_count;
  a.fb_cap = L.fb_cap;
  return a;
}

// work items of the maps that allow injection: the appended particles' slices
template <int MAP>
constexpr int tail_items() {
  return (MAP == MAP_IDENTITY || MAP == MAP_POLAR_LOG || MAP == MAP_TABLE_PC) ? TAIL_ITEMS : 0;
}

template <int D, int MAP, int SHAPE, typename R>
static void launch_particle_t(const ParticleLaunch& L, hipStream_t st) {
  const PartArgs<R> a = make_part_args<R>(L);
  if (L.max_items <= 0) return;
  constexpr bool FIXED = std::is_same<R, float>::value;
  // the appended particles' items (maps that allow injection)
  const int tail = (MAP == MAP_IDENTITY || MAP == MAP_POLAR_LOG || MAP == MAP_TABLE_PC) ? TAIL_ITEMS : 0;
  if (L.cyclo)
    hipLaunchKernelGGL((particle_kernel<D, MAP, SHAPE, R, FIXED, true>), dim3(L.max_items + tail), dim3((pk_threads<D, MAP>())), 0, st,
                     a);
  else
    hipLaunchKernelGGL((particle_kernel<D, MAP, SHAPE, R, FIXED, false>), dim3(L.max_items + tail), dim3((pk_threads<D, MAP>())), 0, st,
                     a);
  if constexpr (MAP != MAP_IDENTITY && MAP != MAP_TABLE_PC) {
    if (L.mode == MODE_PUSH)
      hipLaunchKernelGGL((fallback_kernel<D, MAP, R, FIXED>), dim3(FB_BLOCKS), dim3(256), 0, st, a, L.shape);
  }
}

template <int D, int MAP, int SHAPE, typename R>
static int launch_particle_batch_t(const ParticleLaunch* Ls, int n, BatchArgs& ba, hipStream_t st) {
  constexpr bool FIXED = std::is_same<R, float>::value;
  constexpr int tail = tail_items<MAP>();
  std::vector<PartArgs<R>> args;
  std::vector<int> base(1, 0);
  for (int i = 0; i < n; ++i) {
    if (Ls[i].max_items <= 0) continue;
    args.push_back(make_part_args<R>(Ls[i]));
    base.push_back(base.back() + Ls[i].max_items + tail);
  }
  if (args.empty()) return 0;
  const size_t off_base = (sizeof(PartArgs<R>) * args.size() + 15) & ~(size_t)15;
  ba.staging.assign(off_base + sizeof(int) * base.size(), 0);
  std::memcpy(ba.staging.data(), args.data(), sizeof(PartArgs<R>) * args.size());
  std::memcpy(ba.staging.data() + off_base, base.data(), sizeof(int) * base.size());
  const int rc = batch_upload(ba, st);
  if (rc != 0) return rc;
  const PartArgs<R>* dA = (const PartArgs<R>*)ba.dev;
  const int* dB = (const int*)((const unsigned char*)ba.dev + off_base);
  const int ne = (int)args.size();
  if (Ls[0].cyclo)
    hipLaunchKernelGGL((particle_kernel_batch<D, MAP, SHAPE, R, FIXED, true>), dim3(base.back()), dim3((pk_threads<D, MAP>())), 0, st,
                       dA, dB, ne);
  else
    hipLaunchKernelGGL((particle_kernel_batch<D, MAP, SHAPE, R, FIXED, false>), dim3(base.back()), dim3((pk_threads<D, MAP>())), 0, st,
                       dA, dB, ne);
  if constexpr (MAP != MAP_IDENTITY && MAP != MAP_TABLE_PC) {
    if (Ls[0].mode == MODE_PUSH)
      hipLaunchKernelGGL((fallback_kernel_batch<D, MAP, R, FIXED>), dim3(FB_BATCH_BLOCKS, ne), dim3(256), 0, st, dA, Ls[0].shape);
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <int D, int MAP, typename R>
static int launch_particle_shape(const ParticleLaunch& L, hipStream_t st, const ParticleLaunch* batch = nullptr,
                                 int n = 0, BatchArgs* ba = nullptr) {
  if (batch) {
    return L.shape == SHAPE_B2 ? launch_particle_batch_t<D, MAP, SHAPE_B2, R>(batch, n, *ba, st)
                               : launch_particle_batch_t<D, MAP, SHAPE_B1, R>(batch, n, *ba, st);
  }
  if (L.shape == SHAPE_B2)
    launch_particle_t<D, MAP, SHAPE_B2, R>(L, st);
  else
    launch_particle_t<D, MAP, SHAPE_B1, R>(L, st);
  return 0;
}

template <typename R>
static int launch_particle_r(const ParticleLaunch& L, hipStream_t st, const ParticleLaunch* B = nullptr, int n = 0,
                             BatchArgs* ba = nullptr) {
  const int D = L.g.dim, M = L.g.kind;
  if (L.kc) {
    if (D == 2) return launch_particle_shape<2, MAP_TABLE_PC, R>(L, st, B, n, ba);
    if (D == 3) return launch_particle_shape<3, MAP_TABLE_PC, R>(L, st, B, n, ba);
    return -1;
  }
  if (M == MAP_TABULATED) {
    if (D == 2) return launch_particle_shape<2, MAP_TABULATED, R>(L, st, B, n, ba);
    if (D == 3) return launch_particle_shape<3, MAP_TABULATED, R>(L, st, B, n, ba);
    return -1;
  }
  if (D == 2) {
    if (M == MAP_IDENTITY) return launch_particle_shape<2, MAP_IDENTITY, R>(L, st, B, n, ba);
    if (M == MAP_SINUSOIDAL) return launch_particle_shape<2, MAP_SINUSOIDAL, R>(L, st, B, n, ba);
    if (M == MAP_POLAR_LOG) return launch_particle_shape<2, MAP_POLAR_LOG, R>(L, st, B, n, ba);
  } else if (D == 3) {
    if (M == MAP_IDENTITY) return launch_particle_shape<3, MAP_IDENTITY, R>(L, st, B, n, ba);
    if (M == MAP_SINUSOIDAL) return launch_particle_shape<3, MAP_SINUSOIDAL, R>(L, st, B, n, ba);
  }
  return -1;
}

// kc = n_a k_ab at every vertex from the FP64 inverse-Jacobian table
template <typename R>
__global__ void kc_table_kernel(long long nverts, int d, const double* __restrict__ Kv, double n0, double n1,
                                double n2, R* kc) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nverts) return;
  const double n[3] = {n0, n1, n2};
  const int stride = d == 3 ? KC_STRIDE<3> : KC_STRIDE<2>;
  for (int e = 0; e < stride; ++e) kc[v * stride + e] = (R)0;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) kc[v * stride + a * d + b] = (R)(n[a] * Kv[v * d * d + a * d + b]);
}

void launch_kc_table(const Geo& g, const double* Kv, void* kc, int fp64, hipStream_t st) {
  const unsigned blocks = (unsigned)((g.nverts + 255) / 256);
  if (fp64)
    hipLaunchKernelGGL(kc_table_kernel<double>, dim3(blocks), dim3(256), 0, st, (long long)g.nverts, g.dim, Kv,
                       (double)g.n[0], (double)g.n[1], (double)g.n[2], (double*)kc);
  else
    hipLaunchKernelGGL(kc_table_kernel<float>, dim3(blocks), dim3(256), 0, st, (long long)g.nverts, g.dim, Kv,
                       (double)g.n[0], (double)g.n[1], (double)g.n[2], (float*)kc);
}

int launch_particles(const ParticleLaunch& L, hipStream_t st) {
  return L.fp64 ? launch_particle_r<double>(L, st) : launch_particle_r<float>(L, st);
}

int launch_particles_batch(const ParticleLaunch* L, int n, BatchArgs& ba, hipStream_t st) {
  if (n < 1) return 0;
  // one template for all: precision, dimension, map (and its mover), shape,
  // pusher and mode must agree
  for (int i = 1; i < n; ++i) {
    const ParticleLaunch &a = L[i], &b = L[0];
    if (a.fp64 != b.fp64 || a.g.dim != b.g.dim || a.g.kind != b.g.kind || (a.kc != nullptr) != (b.kc != nullptr) ||
        a.shape != b.shape || a.cyclo != b.cyclo || a.mode != b.mode)
      return -1;
  }
  return L[0].fp64 ? launch_particle_r<double>(L[0], st, L, n, &ba) : launch_particle_r<float>(L[0], st, L, n, &ba);
}

template <int D, int MAP, typename R>
static void launch_inject_t(const InjectLaunch& I, hipStream_t st) {
  InjectArgs<R> a;
  a.g = I.g;
  a.key = I.key;
  for (int i = 0; i < 3; ++i) {
    a.off[i] = (R*)I.off[i];
    a.vel[i] = (R*)I.vel[i];
  }
  a.id = I.id;
  a.d_n = I.d_n;
  a.cap = I.cap;
  a.Q = I.Q;
  a.shape = I.shape;
  a.S1 = I.S1;
  a.lam = I.lam;
  a.kappa = I.kappa;
  a.vth = I.vth;
  a.s_drift = I.s_drift;
  a.dt = I.dt;
  a.k0 = I.k0;
  a.k1 = I.k1;
  a.step = I.step;
  a.species = I.species;
  a.counters = I.counters;
  a.count_out = I.count_out;
  a.tcount = I.tile_counts;
  const int maxc = (int)floor(I.lam) + 1;
  const unsigned blocks = (unsigned)((maxc + 255) / 256);
  constexpr bool FIXED = std::is_same<R, float>::value;
  hipLaunchKernelGGL((inject_kernel<D, MAP, R, FIXED>), dim3(blocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(inject_finish_kernel, dim3(1), dim3(1), 0, st, I.d_n, (const int*)I.count_out, I.cap,
                     I.counters);
}

template <typename R>
static int launch_inject_r(const InjectLaunch& I, hipStream_t st) {
  if (I.g.dim == 2) {
    if (I.g.kind == MAP_IDENTITY) launch_inject_t<2, MAP_IDENTITY, R>(I, st);
    else if (I.g.kind == MAP_POLAR_LOG) launch_inject_t<2, MAP_POLAR_LOG, R>(I, st);
    else return -1;
  } else {
    if (I.g.kind == MAP_IDENTITY) launch_inject_t<3, MAP_IDENTITY, R>(I, st);
    else return -1;
  }
  return 0;
}

int launch_inject(const InjectLaunch& I, hipStream_t st) {
  return I.fp64 ? launch_inject_r<double>(I, st) : launch_inject_r<float>(I, st);
}

// Kinetic energy of the step: the per-item sums of every species added in a
// fixed order (strided per thread, then a fixed tree), species by species.
__global__ __launch_bounds__(256) void ke_reduce_kernel(KeReduce r) {
  __shared__ double sh[256];
  double total = 0.0;
  for (int k = 0; k < r.nspecies; ++k) {
    const int n = *r.n_items[k] + r.tail[k];
    double t;
    strided_sums<1, 8>(r.part[k], 0, n, &t);
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    total += r.scale[k] * sh[0];
    __syncthreads();
  }
  if (threadIdx.x == 0) *r.out = total;
}

void launch_ke_reduce(const KeReduce& r, hipStream_t st) {
  hipLaunchKernelGGL(ke_reduce_kernel, dim3(1), dim3(256), 0, st, r);
}

int launch_tile_sort(const SortLaunch& S, hipStream_t st) {
  const Geo& g = S.g;
  // one workgroup per chunk of the buffer's capacity (chunks past the live
  // count return at once)
  int blocks = (int)((S.capacity + SORT_CHUNK - 1) / SORT_CHUNK);
  if (blocks < 1) blocks = 1;
  if (!S.counts_ready) {
    launch_fill_u8(S.counts, 0, sizeof(int) * (size_t)(g.ntiles + 2), st);
    if (g.dim == 2)
      hipLaunchKernelGGL(tile_hist_kernel<2>, dim3(blocks), dim3(256), 0, st, S.key_in, S.d_n, S.counts, g);
    else
      hipLaunchKernelGGL(tile_hist_kernel<3>, dim3(blocks), dim3(256), 0, st, S.key_in, S.d_n, S.counts, g);
  }
  hipLaunchKernelGGL(tile_scan_kernel, dim3(1), dim3(1024), 0, st, S.counts, g.ntiles, S.chunk, S.start,
                     S.cursor, S.n_items, S.item_tile, S.item_begin, S.item_end, S.d_n);
#define SCATTER(DD, RR)                                                                            \
  hipLaunchKernelGGL((tile_scatter_kernel<DD, RR>), dim3(blocks), dim3(256), 0, st, S.start, S.cursor, \
                     g, S.key_in, S.key_out, (const RR*)S.off_in[0], (const RR*)S.off_in[1],        \
                     (const RR*)S.off_in[2], (RR*)S.off_out[0], (RR*)S.off_out[1], (RR*)S.off_out[2], \
                     (const RR*)S.vel_in[0], (const RR*)S.vel_in[1], (const RR*)S.vel_in[2],          \
                     (RR*)S.vel_out[0], (RR*)S.vel_out[1], (RR*)S.vel_out[2], S.id_in, S.id_out)
  if (g.dim == 2) {
    if (S.fp64) SCATTER(2, double); else SCATTER(2, float);
  } else {
    if (S.fp64) SCATTER(3, double); else SCATTER(3, float);
  }
#undef SCATTER
  return 0;
}

void launch_lin_to_key(const int32_t* lin, int32_t* key, int n, const Geo& g, int* bad,
                       hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(lin_to_key_kernel, dim3((n + 255) / 256), dim3(256), 0, st, lin, key, n, g, bad);
}
void launch_key_to_lin(const int32_t* key, int32_t* lin, int n, const Geo& g, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(key_to_lin_kernel, dim3((n + 255) / 256), dim3(256), 0, st, key, lin, n, g);
}
void launch_iota(uint32_t* id, int n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(iota_kernel, dim3((n + 255) / 256), dim3(256), 0, st, id, n);
}
void launch_offsets_check(const void* o, long long n, int fp64, int* bad, hipStream_t st) {
  if (n <= 0) return;
  unsigned blocks = (unsigned)((n + 255) / 256);
  if (fp64)
    hipLaunchKernelGGL(offsets_check_kernel<double>, dim3(blocks), dim3(256), 0, st, (const double*)o, n, bad);
  else
    hipLaunchKernelGGL(offsets_check_kernel<float>, dim3(blocks), dim3(256), 0, st, (const float*)o, n, bad);
}

}  // namespace cpic
