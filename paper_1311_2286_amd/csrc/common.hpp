// common.hpp -- internal types and device helpers of the MI355X curvilinear
// PIC library (not part of the public ABI; see include/cpic.h).
//
// Particle cells are kept internally as packed coordinates
//     key = i | j << sx | k << (sx + sy)          (sx, sy = bit widths of n0, n1)
// so that decoding is shifts and masks.  Negative keys mark dead particles
// (-1: absorbed at a lower wall, -2: left through an upper wall).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cpic {

// MAP_SPHERICAL_RZ (the r-z half plane of a spherical shell) serves the field
// solve only: no particle kernel is built for it.  MAP_TABULATED: the map known
// at the vertices only (particles move with the predictor-corrector update)
enum { MAP_IDENTITY = 0, MAP_SINUSOIDAL = 1, MAP_POLAR_LOG = 2, MAP_SPHERICAL_RZ = 3, MAP_TABULATED = 4 };
// particle-kernel variant that moves with the tabulated inverse Jacobian (the
// predictor-corrector update), whatever the map
constexpr int MAP_TABLE_PC = 5;
enum { BC_PERIODIC = 0, BC_DIRICHLET = 1, BC_NEUMANN = 2 };
enum { PBC_PERIODIC = 0, PBC_ABSORB = 1, PBC_OUTFLOW = 2 };
enum { SHAPE_B1 = 1, SHAPE_B2 = 2 };
enum { MODE_PUSH = 0, MODE_DEPOSIT = 1, MODE_HALFSTEP = 2 };

// Tile geometry of the particle kernel: 16x16 cells in 2D, 8x8x8 in 3D, with a
// deposit window of G cells on every side held in LDS.
template <int D> struct TileShape;
template <> struct TileShape<2> {
  static constexpr int T0 = 16, T1 = 16, T2 = 1, G = 2;
  static constexpr int W0 = T0 + 2 * G, W1 = T1 + 2 * G, W2 = 1;
  static constexpr int WIN = W0 * W1;
};
template <> struct TileShape<3> {
  static constexpr int T0 = 8, T1 = 8, T2 = 8, G = 2;
  static constexpr int W0 = T0 + 2 * G, W1 = T1 + 2 * G, W2 = T2 + 2 * G;
  static constexpr int WIN = W0 * W1 * W2;
};

// Everything a kernel needs to know about the grid and the map (by value).
struct Geo {
  int dim;
  int n[3];        // cells per axis (1 on unused axes)
  int nv[3];       // vertices per axis (n on periodic axes, n + 1 on bounded ones)
  int periodic[3]; // 1 if the axis is periodic
  int sx, sy;      // packed-key shifts
  int nt[3];       // tiles per axis
  int ntiles;
  long long ncells, nverts;
  double invn[3];  // 1 / n
  // map
  int kind;
  double L[3];
  double eps;
  double r_in, r_out, lnR;
  int omega;       // 1: geometric factor Omega = x^1 (radius of an axisymmetric r-z plane), else 1
  // tabulated map: x at the vertices (d per vertex) and the Jacobi matrix there
  // from finite differences of it (d x d per vertex, row-major); on a periodic
  // axis a the map continues as x(xi + e_a) = x(xi) + L_a e_a
  const double* xtab;
  const double* jtab;
  double ecell[3]; // eps * n_a: map perturbation in cells of axis a
  double dxc[3];   // L_a / n_a: undistorted cell size
};

__host__ __device__ inline int key_i(int key, const Geo& g) { return key & ((1 << g.sx) - 1); }
__host__ __device__ inline int key_j(int key, const Geo& g) { return (key >> g.sx) & ((1 << g.sy) - 1); }
__host__ __device__ inline int key_k(int key, const Geo& g) { return key >> (g.sx + g.sy); }
__host__ __device__ inline int make_key(int i, int j, int k, const Geo& g) {
  return i | (j << g.sx) | (k << (g.sx + g.sy));
}

template <int D>
__host__ __device__ inline int tile_of_key(int key, const Geo& g) {
  using TS = TileShape<D>;
  int ti = key_i(key, g) / TS::T0;
  int tj = key_j(key, g) / TS::T1;
  int tk = (D == 3) ? key_k(key, g) / TS::T2 : 0;
  return ti + g.nt[0] * (tj + g.nt[1] * tk);
}

// Per thread of a one-dimensional workgroup, the sums over m < M of
// p[m * ld + i] for i = threadIdx.x + k blockDim.x < n, in a fixed order: U
// running sums per array over interleaved strides (U M loads in flight per
// thread instead of one chain of dependent loads), added pairwise at the end.
template <int M, int U>
__device__ inline void strided_sums(const double* __restrict__ p, int ld, int n, double* out) {
  const int B = blockDim.x;
  double a[M][U];
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int u = 0; u < U; ++u) a[m][u] = 0.0;
  int i = threadIdx.x;
  for (; i + (U - 1) * B < n; i += U * B) {
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int u = 0; u < U; ++u) a[m][u] += p[m * (size_t)ld + i + u * B];
  }
  for (; i < n; i += B) {
#pragma unroll
    for (int m = 0; m < M; ++m) a[m][0] += p[m * (size_t)ld + i];
  }
#pragma unroll
  for (int m = 0; m < M; ++m) {
#pragma unroll
    for (int w = 1; w < U; w *= 2)
#pragma unroll
      for (int u = 0; u + w < U; u += 2 * w) a[m][u] += a[m][u + w];
    out[m] = a[m][0];
  }
}

// ---------------------------------------------------------------------------
// Trigonometric helpers.  sin/cos of 2 pi u at the base position: in FP32 the
// hardware instructions, which take their argument in revolutions (valid for
// |u| <= 256; measured largest absolute error 1.3e-7 on [0, 1], the rounding of
// FP32 near 1) -- the Newton residual uses them only multiplied by the small
// increments below, so their error is damped; in FP64, the turn reduced by
// its nearest quarter (exactly) and the increment polynomials below on the
// remainder (|x| <= pi/4), rotated by the quarter.  Increments sin(2 pi u)
// and cos(2 pi u) - 1 for the Newton steps need relative accuracy (their
// error is amplified by the map amplitude over the Jacobian): Taylor
// polynomials in x = 2 pi u, in nested form, of degree 9 and 10 in FP32
// (truncation below 3e-9 for |x| < 0.8) and 19 and 20 in FP64 (below 1e-21),
// without branches; beyond |x| = 0.8 (a move of more than 0.13 of the grid in
// one step) the device library.
// ---------------------------------------------------------------------------
__device__ inline void sincos2pi(float u, float& s, float& c) {
  s = __builtin_amdgcn_sinf(u);
  c = __builtin_amdgcn_cosf(u);
}

__device__ inline void incr2pi(float u, float& sn, float& cm1) {
  const float th = 6.28318530717958648f * u;
  const float t2 = th * th;
  sn = th * (1.0f - t2 * (1.0f / 6.0f) *
                        (1.0f - t2 * (1.0f / 20.0f) * (1.0f - t2 * (1.0f / 42.0f) * (1.0f - t2 * (1.0f / 72.0f)))));
  cm1 = -0.5f * t2 *
        (1.0f - t2 * (1.0f / 12.0f) *
                    (1.0f - t2 * (1.0f / 30.0f) * (1.0f - t2 * (1.0f / 56.0f) * (1.0f - t2 * (1.0f / 90.0f)))));
  if (!(fabsf(th) < 0.8f)) {
    float s, c;
    sincospif(2.0f * u, &s, &c);
    sn = s;
    cm1 = c - 1.0f;
  }
}
// sin x and cos x - 1 for |x| < 0.8 (FP64), in nested form (few live
// constants: the particle kernel keeps its register budget)
__device__ inline void taylor_sin_cm1(double x, double& sn, double& cm1) {
  const double t = x * x;
  sn = x * (1.0 - t * (1.0 / 6.0) *
                      (1.0 - t * (1.0 / 20.0) *
                                 (1.0 - t * (1.0 / 42.0) *
                                            (1.0 - t * (1.0 / 72.0) *
                                                       (1.0 - t * (1.0 / 110.0) *
                                                                  (1.0 - t * (1.0 / 156.0) *
                                                                             (1.0 - t * (1.0 / 210.0) *
                                                                                        (1.0 - t * (1.0 / 272.0) *
                                                                                                   (1.0 - t * (1.0 / 342.0))))))))));
  cm1 = -0.5 * t *
        (1.0 - t * (1.0 / 12.0) *
                   (1.0 - t * (1.0 / 30.0) *
                              (1.0 - t * (1.0 / 56.0) *
                                         (1.0 - t * (1.0 / 90.0) *
                                                    (1.0 - t * (1.0 / 132.0) *
                                                               (1.0 - t * (1.0 / 182.0) *
                                                                          (1.0 - t * (1.0 / 240.0) *
                                                                                     (1.0 - t * (1.0 / 306.0) *
                                                                                                (1.0 - t * (1.0 / 380.0))))))))));
}

__device__ inline void sincos2pi(double u, double& s, double& c) {
  const double q = rint(4.0 * u);                         // nearest quarter turn
  const double x = 6.283185307179586 * fma(-0.25, q, u);  // u - q/4 is exact
  double sr, cm1;
  taylor_sin_cm1(x, sr, cm1);
  const double cr = 1.0 + cm1;
  // rotation by k quarter turns: (s, c) = (sr, cr), (cr, -sr), (-sr, -cr), (-cr, sr)
  const int k = (int)((long long)q & 3);
  const double a = (k & 1) ? cr : sr, b = (k & 1) ? sr : cr;
  s = (k & 2) ? -a : a;
  c = (k == 1 || k == 2) ? -b : b;
}

__device__ inline void incr2pi(double u, double& sn, double& cm1) {
  const double x = 6.283185307179586 * u;
  taylor_sin_cm1(x, sn, cm1);
  if (!(fabs(x) < 0.8)) {
    sn = sinpi(2.0 * u);
    double h = sinpi(u);
    cm1 = -2.0 * h * h;
  }
}

template <typename R> __device__ inline R r_expm1(R x);
template <> __device__ inline float r_expm1<float>(float x) { return expm1f(x); }
template <> __device__ inline double r_expm1<double>(double x) { return expm1(x); }
template <typename R> __device__ inline R r_exp(R x);
template <> __device__ inline float r_exp<float>(float x) { return expf(x); }
template <> __device__ inline double r_exp<double>(double x) { return exp(x); }

// reciprocal for the Newton steps: the hardware approximation (1 ulp) in FP32,
// where the step tolerance is 1e-5 cell; correctly rounded in FP64
__device__ inline float newton_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double newton_rcp(double x) { return 1.0 / x; }

// ---------------------------------------------------------------------------
// Position update: solve x(xi^n + delta h) - x(xi^n) = dt v for delta (in
// cells) by Newton's method on the increment, starting from delta = 0 (whose
// first step is k(xi^n) dt v / h).  Converged when the last Newton step s is
// below tol cells, or when the quadratic-convergence bound kappa s^2 on the
// remaining error is below tol / 4 (kappa = max second derivative over twice
// the smallest Jacobian of the increment map, from the host).  J0 receives
// the smallest (box-unit) Jacobian met: at xi^n and at every Newton iterate.
// ---------------------------------------------------------------------------

// Sinusoidal map, x^a = L_a (xi^a + eps P), P = prod_k sin(2 pi xi^k) (Eq. map2
// and its 3D extension).  In cells of axis a the increment equation reads
//   F_a(delta) = delta_a + e_a [P(xi + delta h) - P(xi)] - r_a = 0,
// e_a = eps n_a, r_a = dt v_a n_a / L_a.  Jacobian I + e g^T with
// g_m = (2 pi / n_m) cos(2 pi xi_m') prod_{k != m} sin(2 pi xi_k'), inverted by
// Sherman-Morrison; 1 + g.e is the box Jacobian at xi'.  Stopping bound:
// after a step s the residual is e R with |R| <= (1/2) w_max^2 (sum |s_a|)^2
// (the second derivatives of P in cells are at most w_max^2, w = 2 pi / n),
// and the mean-value Jacobian, again I + e g^T, maps e R to e R / J, so the
// error is at most kappa (sum |s_a|)^2 with kappa = e_max w_max^2 / (2 J_min).
template <int D, typename R>
__device__ __forceinline__ bool newton_sinusoidal(const Geo& g, const int* idx, const R* f,
                                                  const R* r, R* d, R tol, R kappa, int maxit,
                                                  R& J0) {
  R s[D], c[D], e[D], w[D], invn[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    invn[a] = (R)g.invn[a];
    R phase = ((R)idx[a] + f[a]) * invn[a];
    sincos2pi(phase, s[a], c[a]);
    e[a] = (R)g.ecell[a];
    w[a] = (R)6.28318530717958647692 * invn[a];
  }
  // first step from delta = 0, where F = -r: delta = r - e (g.r) / J
  {
    R gg[D];
    R Jn = (R)1, gr = (R)0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      R t = w[a] * c[a];
#pragma unroll
      for (int k = 0; k < D; ++k)
        if (k != a) t *= s[k];
      gg[a] = t;
      Jn += e[a] * t;
      gr += t * r[a];
    }
    J0 = Jn;
    const R q = gr * newton_rcp(Jn);
    R mx = (R)0, l1 = (R)0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      d[a] = r[a] - e[a] * q;
      mx = fmax(mx, fabs(d[a]));
      l1 += fabs(d[a]);
    }
    if (mx < tol || kappa * l1 * l1 < (R)0.25 * tol) return true;
  }
  for (int it = 1; it < maxit; ++it) {
    R sn[D], cn[D], ds[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      R st, cm1;
      incr2pi(d[a] * invn[a], st, cm1);
      ds[a] = s[a] * cm1 + c[a] * st;
      R dc = c[a] * cm1 - s[a] * st;
      sn[a] = s[a] + ds[a];
      cn[a] = c[a] + dc;
    }
    R dP;
    if (D == 2) {
      dP = ds[0] * sn[1] + s[0] * ds[1];
    } else {
      dP = ds[0] * sn[1] * sn[D - 1] + s[0] * ds[1] * sn[D - 1] + s[0] * s[1] * ds[D - 1];
    }
    R F[D], gg[D];
    R Jn = (R)1, gF = (R)0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      F[a] = d[a] + e[a] * dP - r[a];
      R t = w[a] * cn[a];
#pragma unroll
      for (int k = 0; k < D; ++k)
        if (k != a) t *= sn[k];
      gg[a] = t;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      Jn += e[a] * gg[a];
      gF += gg[a] * F[a];
    }
    J0 = fmin(J0, Jn);
    R q = gF * newton_rcp(Jn);
    R mx = (R)0, l1 = (R)0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      R dd = -(F[a] - e[a] * q);
      d[a] += dd;
      mx = fmax(mx, fabs(dd));
      l1 += fabs(dd);
    }
    if (mx < tol || kappa * l1 * l1 < (R)0.25 * tol) return true;
  }
  return false;
}

// Polar-log map: r = r_in exp(xi ln R), theta = 2 pi eta.  Increment in units
// of r^n:  F = (rho - 1) e(theta') + [e(theta') - e(theta)] - dt v / r^n,
// rho = exp(delta_0 ln R / n0), theta' = theta + 2 pi delta_1 / n1.  The
// Jacobian columns are rho (ln R / n0) e(theta') and rho (2 pi / n1) e_perp.
template <typename R>
__device__ __forceinline__ bool newton_polar(const Geo& g, const int* idx, const R* f, const R* vdt,
                                             R* d, R tol, R kappa, int maxit, R& J0) {
  R invn0 = (R)g.invn[0], invn1 = (R)g.invn[1];
  R lnR = (R)g.lnR;
  R xi0 = ((R)idx[0] + f[0]) * invn0;
  R r0 = (R)g.r_in * r_exp<R>(lnR * xi0);
  R s0, c0;
  sincos2pi(((R)idx[1] + f[1]) * invn1, s0, c0);
  R bx = vdt[0] / r0, by = vdt[1] / r0;
  R kx = lnR * invn0, ky = (R)6.28318530717958647692 * invn1;
  d[0] = d[1] = (R)0;
  J0 = (R)1;
  bool conv = false;
  for (int it = 0; it < maxit; ++it) {
    R rm1 = r_expm1<R>(kx * d[0]);
    R rho = (R)1 + rm1;
    R st, cm1;
    if (it == 0) {
      st = (R)0;
      cm1 = (R)0;
    } else {
      incr2pi(d[1] * invn1, st, cm1);
    }
    R dex = c0 * cm1 - s0 * st, dey = s0 * cm1 + c0 * st;
    R ex = c0 + dex, ey = s0 + dey;
    R Fx = rm1 * ex + dex - bx, Fy = rm1 * ey + dey - by;
    R d0 = -(Fx * ex + Fy * ey) / (rho * kx);
    R d1 = -(-Fx * ey + Fy * ex) / (rho * ky);
    d[0] += d0;
    d[1] += d1;
    R mx = fmax(fabs(d0), fabs(d1));
    if (mx < tol || kappa * mx * mx < (R)0.25 * tol) {
      conv = true;
      break;
    }
  }
  return conv;
}

// ---------------------------------------------------------------------------
// Fixed-point deposit weights: per axis, integers at scale 2^S1 for the cells
// i-1, i, i+1 of a particle at in-cell offset f (exactly representable in
// FP64).  b2:  L = rint(2^(S1-1) (1-f)^2), R = rint(2^(S1-1) f^2),
// C = 2^S1 - L - R.  CIC to cell centres with g = f - 1/2.  Multiplications
// and ldexp are exact or correctly rounded, rint rounds half to even.
// ---------------------------------------------------------------------------
template <int SHAPE>
__device__ inline void weights_fixed(double f, int S1, uint32_t* w) {
  uint32_t one = 1u << S1;
  if (SHAPE == SHAPE_B2) {
    double a = 1.0 - f;
    uint32_t L = (uint32_t)rint(ldexp(a * a, S1 - 1));
    uint32_t R = (uint32_t)rint(ldexp(f * f, S1 - 1));
    w[0] = L;
    w[2] = R;
    w[1] = one - L - R;
  } else {
    double gg = f - 0.5;
    if (gg >= 0.0) {
      uint32_t R = (uint32_t)rint(ldexp(gg, S1));
      w[0] = 0;
      w[1] = one - R;
      w[2] = R;
    } else {
      uint32_t Lw = (uint32_t)rint(ldexp(-gg, S1));
      w[0] = Lw;
      w[1] = one - Lw;
      w[2] = 0;
    }
  }
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter-based RNG used by
// the injection; u = (r + 1/2) 2^-32 maps an output word into (0, 1).
// ---------------------------------------------------------------------------
__device__ inline void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                     uint32_t k1, uint32_t* out) {
  uint32_t c[4] = {c0, c1, c2, c3};
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c[0];
  out[1] = c[1];
  out[2] = c[2];
  out[3] = c[3];
}
__device__ inline double unit_open(uint32_t r) { return ((double)r + 0.5) * (1.0 / 4294967296.0); }

// map x(xi) and Jacobi matrix j[a][b] = dx^a / dxi^b in FP64 (Eqs. map, jcov)
__device__ inline void map_jacobi(const Geo& g, const double* xi, double j[3][3], double* x) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) j[a][b] = (a == b) ? 1.0 : 0.0;
  const int d = g.dim;
  if (g.kind == MAP_TABULATED) {
    // multilinear blend of the values at the 2^d vertices of the cell holding
    // xi; a point beyond a bounded axis is taken on its wall
    int base[3] = {0, 0, 0};
    double f[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d; ++a) {
      double u = xi[a] * g.n[a];
      if (!g.periodic[a]) u = fmin(fmax(u, 0.0), (double)g.n[a]);
      int i = (int)floor(u);
      if (!g.periodic[a] && i > g.n[a] - 1) i = g.n[a] - 1;
      base[a] = i;
      f[a] = u - i;
    }
    for (int a = 0; a < d; ++a) {
      j[a][a] = 0.0;
      if (x) x[a] = 0.0;
    }
    for (int c = 0; c < (1 << d); ++c) {
      double w = 1.0, per[3] = {0.0, 0.0, 0.0};
      long long v = 0, stride = 1;
      for (int a = 0; a < d; ++a) {
        const int up = (c >> a) & 1;
        int i = base[a] + up;
        w *= up ? f[a] : 1.0 - f[a];
        if (g.periodic[a]) {
          int r = i % g.n[a];
          if (r < 0) r += g.n[a];
          per[a] = (double)((i - r) / g.n[a]);
          i = r;
        }
        v += stride * i;
        stride *= g.nv[a];
      }
      const double* xv = g.xtab + v * d;
      const double* jv = g.jtab + v * d * d;
      for (int a = 0; a < d; ++a) {
        if (x) x[a] += w * (xv[a] + per[a] * g.L[a]);
        for (int b = 0; b < d; ++b) j[a][b] += w * jv[a * d + b];
      }
    }
  } else if (g.kind == MAP_IDENTITY) {
    for (int a = 0; a < d; ++a) {
      j[a][a] = g.L[a];
      if (x) x[a] = g.L[a] * xi[a];
    }
  } else if (g.kind == MAP_SINUSOIDAL) {
    double s[3], c[3];
    for (int k = 0; k < d; ++k) sincospi(2.0 * xi[k], &s[k], &c[k]);
    double P = 1.0;
    for (int k = 0; k < d; ++k) P *= s[k];
    for (int b = 0; b < d; ++b) {
      double t = 6.283185307179586 * c[b];
      for (int k = 0; k < d; ++k)
        if (k != b) t *= s[k];
      for (int a = 0; a < d; ++a) j[a][b] = g.L[a] * ((a == b ? 1.0 : 0.0) + g.eps * t);
    }
    if (x)
      for (int a = 0; a < d; ++a) x[a] = g.L[a] * (xi[a] + g.eps * P);
  } else if (g.kind == MAP_SPHERICAL_RZ) {
    // (r, z) = rho (sin t, cos t), rho = r_in + (r_out - r_in) xi^1,
    // t = pi (1 - xi^2) (Sec. "Field solver", Eqs. r and z)
    const double D = g.r_out - g.r_in, rho = g.r_in + D * xi[0];
    double st, ct;
    sincospi(1.0 - xi[1], &st, &ct);
    j[0][0] = D * st;
    j[0][1] = -3.141592653589793 * rho * ct;
    j[1][0] = D * ct;
    j[1][1] = 3.141592653589793 * rho * st;
    if (x) {
      x[0] = rho * st;
      x[1] = rho * ct;
    }
  } else {  // polar-log
    double r = g.r_in * exp(xi[0] * g.lnR);
    double st, ct;
    sincospi(2.0 * xi[1], &st, &ct);
    j[0][0] = r * g.lnR * ct;
    j[0][1] = -6.283185307179586 * r * st;
    j[1][0] = r * g.lnR * st;
    j[1][1] = 6.283185307179586 * r * ct;
    if (x) {
      x[0] = r * ct;
      x[1] = r * st;
    }
  }
}

template <int SHAPE, typename R>
__device__ inline void weights_real(R f, R* w) {
  if (SHAPE == SHAPE_B2) {
    R a = (R)1 - f, b = f - (R)0.5;
    w[0] = (R)0.5 * a * a;
    w[1] = (R)0.75 - b * b;
    w[2] = (R)0.5 * f * f;
  } else {
    R gg = f - (R)0.5;
    if (gg >= (R)0) {
      w[0] = (R)0;
      w[1] = (R)1 - gg;
      w[2] = gg;
    } else {
      w[0] = -gg;
      w[1] = (R)1 + gg;
      w[2] = (R)0;
    }
  }
}

}  // namespace cpic
