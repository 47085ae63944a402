/*
 * oracle.c -- slow, plain, FP64 CPU reference for the electrostatic
 * curvilinear particle-in-cell step of Delzanno et al., "CPIC: a Curvilinear
 * Particle-In-Cell code for plasma-material interaction studies"
 * (arXiv:1311.2286).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * constant with the HIP path.
 *
 * Every routine is the plain definition of the quantity it computes (loops
 * over particles / cells / faces in the order the definition is written), in
 * FP64, built with -O2 -ffp-contract=off (no FMA contraction, no fast-math).
 *
 * Conventions
 *   logical space: unit cube, cell c=(i,j,k) spans [i h, (i+1) h) per axis,
 *   vertices sit at integer multiples of h (Sec. II.B: potential and density
 *   at cell centres, field at vertices).
 *   linear cell index  c = i + n0 (j + n1 k);
 *   vertex counts per axis: n (periodic axis) or n+1 (bounded axis).
 *   points / vectors are passed row-major with 3 components (unused = 0),
 *   3x3 matrices row-major with 9 entries.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

enum { OR_IDENTITY = 0, OR_SINUSOIDAL = 1, OR_POLAR_LOG = 2, OR_SPHERICAL_RZ = 3, OR_TABULATED = 4 };
enum { OR_PERIODIC = 0, OR_DIRICHLET = 1, OR_NEUMANN = 2 };
enum { OR_B1 = 1, OR_B2 = 2 };

typedef struct {
  int kind;
  int dim;
  double L[3];
  double eps;
  double r_in, r_out;
  int omega; /* 0: Omega = 1; 1: Omega = x^1 (cylindrical r) */
  /* OR_TABULATED: the map known at the cell vertices only.  tx holds x^a at
     the vertices, d arrays of tn0 tn1 tn2 values (vertex (i, j, k) at
     i + tn0 (j + tn1 k)); tn_a = n_a vertices on a periodic axis (tper_a = 1),
     where the map continues as x(xi + e_a) = x(xi) + L_a e_a, and n_a + 1 on a
     bounded one. */
  int tn[3];
  int tper[3];
  const double* tx;
} or_map;

typedef struct {
  int dim;
  int n[3];
  int bc_lo[3], bc_hi[3];
  double phi_lo[3], phi_hi[3];
} or_grid;

/* ------------------------------------------------------------------------ */
/* Maps and metrics: Eqs. (map), (jcov), (jcon), (jac), (gcon), (poiscurv).   */
/* ------------------------------------------------------------------------ */

/* Tabulated map (Sec. "Curvilinear formulation": the metric coefficients of
   a map known at the cell vertices come from finite differences of it).
   tab_x: x at vertex iv, whose indices on a periodic axis may lie outside
   [0, n): the table entry of the wrapped vertex plus the whole periods. */
static int tab_cells(const or_map* m, int a) { return m->tper[a] ? m->tn[a] : m->tn[a] - 1; }

static void tab_x(const or_map* m, const int* iv, double* x) {
  int d = m->dim;
  int w[3] = {0, 0, 0};
  double per[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < d; ++a) {
    w[a] = iv[a];
    if (m->tper[a]) {
      int n = m->tn[a];
      int r = ((iv[a] % n) + n) % n;
      per[a] = (double)((iv[a] - r) / n);
      w[a] = r;
    }
  }
  long nv = (long)m->tn[0] * m->tn[1] * (d == 3 ? m->tn[2] : 1);
  long lin = w[0] + (long)m->tn[0] * (w[1] + (long)m->tn[1] * w[2]);
  for (int a = 0; a < 3; ++a) x[a] = 0.0;
  for (int a = 0; a < d; ++a) x[a] = m->tx[a * nv + lin] + per[a] * m->L[a];
}

/* Jacobi matrix at vertex iv: dx/dxi^b by the centred difference over the two
   neighbouring vertices (spacing 2/n_b), and at the two ends of a bounded axis
   by the second-order one-sided difference over three vertices. */
static void tab_jac_vertex(const or_map* m, const int* iv, double j[3][3]) {
  int d = m->dim;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) j[a][b] = (a == b) ? 1.0 : 0.0;
  for (int b = 0; b < d; ++b) {
    int n = tab_cells(m, b);
    int p0[3] = {iv[0], iv[1], iv[2]}, p1[3] = {iv[0], iv[1], iv[2]}, p2[3] = {iv[0], iv[1], iv[2]};
    double x0[3], x1[3], x2[3];
    if (m->tper[b] || (iv[b] > 0 && iv[b] < n)) {
      p0[b] = iv[b] - 1;
      p1[b] = iv[b] + 1;
      tab_x(m, p0, x0);
      tab_x(m, p1, x1);
      for (int a = 0; a < d; ++a) j[a][b] = (x1[a] - x0[a]) * n / 2.0;
    } else {
      int s = (iv[b] == 0) ? 1 : -1; /* direction into the domain */
      p1[b] = iv[b] + s;
      p2[b] = iv[b] + 2 * s;
      tab_x(m, p0, x0);
      tab_x(m, p1, x1);
      tab_x(m, p2, x2);
      for (int a = 0; a < d; ++a) j[a][b] = s * (-3.0 * x0[a] + 4.0 * x1[a] - x2[a]) * n / 2.0;
    }
  }
}

/* Between vertices: x and the Jacobi matrix are the multilinear blends of the
   values at the 2^d vertices of the cell holding xi (weights prod_a (1 - f_a)
   or f_a); a point outside a bounded axis is taken on its wall. */
static void tab_x_jac(const or_map* m, const double* xi, double* x, double j[3][3]) {
  int d = m->dim;
  int base[3] = {0, 0, 0};
  double f[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < d; ++a) {
    int n = tab_cells(m, a);
    double u = xi[a] * n;
    if (!m->tper[a]) {
      if (u < 0.0) u = 0.0;
      if (u > n) u = n;
    }
    int i = (int)floor(u);
    if (!m->tper[a] && i > n - 1) i = n - 1;
    base[a] = i;
    f[a] = u - i;
  }
  for (int a = 0; a < 3; ++a) {
    x[a] = 0.0;
    for (int b = 0; b < 3; ++b) j[a][b] = 0.0;
  }
  int nc = 1 << d;
  for (int c = 0; c < nc; ++c) {
    int iv[3] = {0, 0, 0};
    double w = 1.0;
    for (int a = 0; a < d; ++a) {
      int up = (c >> a) & 1;
      iv[a] = base[a] + up;
      w *= up ? f[a] : 1.0 - f[a];
    }
    double xv[3], jv[3][3];
    tab_x(m, iv, xv);
    tab_jac_vertex(m, iv, jv);
    for (int a = 0; a < d; ++a) {
      x[a] += w * xv[a];
      for (int b = 0; b < d; ++b) j[a][b] += w * jv[a][b];
    }
  }
  for (int a = d; a < 3; ++a) j[a][a] = 1.0;
}

/* x(xi) and the Jacobi matrix j[a][b] = dx^a / dxi^b (Eq. jcov). */
static void map_x_jac(const or_map* m, const double* xi, double* x, double j[3][3]) {
  if (m->kind == OR_TABULATED) {
    tab_x_jac(m, xi, x, j);
    return;
  }
  int d = m->dim;
  for (int a = 0; a < 3; ++a) {
    x[a] = 0.0;
    for (int b = 0; b < 3; ++b) j[a][b] = (a == b) ? 1.0 : 0.0;
  }
  if (m->kind == OR_IDENTITY) {
    for (int a = 0; a < d; ++a) {
      x[a] = m->L[a] * xi[a];
      j[a][a] = m->L[a];
    }
  } else if (m->kind == OR_SINUSOIDAL) {
    /* x^a = L_a (xi^a + eps * prod_k sin(2 pi xi^k)) -- Eq. (map2), same
       product perturbation on every axis in 3D. */
    double s[3], c[3];
    for (int k = 0; k < d; ++k) {
      s[k] = sin(2.0 * OR_PI * xi[k]);
      c[k] = cos(2.0 * OR_PI * xi[k]);
    }
    double P = 1.0;
    for (int k = 0; k < d; ++k) P *= s[k];
    double dP[3];
    for (int b = 0; b < d; ++b) {
      double t = 2.0 * OR_PI * c[b];
      for (int k = 0; k < d; ++k)
        if (k != b) t *= s[k];
      dP[b] = t;
    }
    for (int a = 0; a < d; ++a) {
      x[a] = m->L[a] * (xi[a] + m->eps * P);
      for (int b = 0; b < d; ++b) j[a][b] = m->L[a] * ((a == b ? 1.0 : 0.0) + m->eps * dP[b]);
    }
  } else if (m->kind == OR_POLAR_LOG) {
    double lnR = log(m->r_out / m->r_in);
    double r = m->r_in * exp(xi[0] * lnR);
    double th = 2.0 * OR_PI * xi[1];
    double ct = cos(th), st = sin(th);
    x[0] = r * ct;
    x[1] = r * st;
    j[0][0] = r * lnR * ct;
    j[0][1] = -2.0 * OR_PI * r * st;
    j[1][0] = r * lnR * st;
    j[1][1] = 2.0 * OR_PI * r * ct;
  } else { /* OR_SPHERICAL_RZ, Eqs. (r), (z) */
    double D = m->r_out - m->r_in;
    double rho = m->r_in + D * xi[0];
    double th = OR_PI * (1.0 - xi[1]);
    double st = sin(th), ct = cos(th);
    x[0] = rho * st; /* r */
    x[1] = rho * ct; /* z */
    j[0][0] = D * st;
    j[0][1] = -OR_PI * rho * ct;
    j[1][0] = D * ct;
    j[1][1] = OR_PI * rho * st;
  }
}

static double det_d(int d, double j[3][3]) {
  if (d == 2) return j[0][0] * j[1][1] - j[0][1] * j[1][0];
  return j[0][0] * (j[1][1] * j[2][2] - j[1][2] * j[2][1]) -
         j[0][1] * (j[1][0] * j[2][2] - j[1][2] * j[2][0]) +
         j[0][2] * (j[1][0] * j[2][1] - j[1][1] * j[2][0]);
}

/* k = j^{-1} by the adjugate (Eq. jcon). */
static void inv_d(int d, double j[3][3], double k[3][3]) {
  double J = det_d(d, j);
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

/* Solver coefficient a^{ij} = Omega J g^{ij}, g^{ij} = k^{i g} k^{j g}
   (Eqs. gcon, poiscurv). */
static void coef_at(const or_map* m, const double* xi, double a[3][3]) {
  double x[3], j[3][3], k[3][3];
  int d = m->dim;
  map_x_jac(m, xi, x, j);
  double J = det_d(d, j);
  inv_d(d, j, k);
  double Om = m->omega ? x[0] : 1.0;
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q) {
      double g = 0.0;
      for (int r = 0; r < d; ++r) g += k[p][r] * k[q][r];
      a[p][q] = (p < d && q < d) ? Om * J * g : 0.0;
    }
}

void or_map_eval(const or_map* m, long n, const double* xi, double* x, double* jac, double* kinv,
                 double* J) {
  for (long p = 0; p < n; ++p) {
    double xx[3], j[3][3], k[3][3];
    map_x_jac(m, xi + 3 * p, xx, j);
    inv_d(m->dim, j, k);
    if (x)
      for (int a = 0; a < 3; ++a) x[3 * p + a] = xx[a];
    if (jac)
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) jac[9 * p + 3 * a + b] = j[a][b];
    if (kinv)
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) kinv[9 * p + 3 * a + b] = k[a][b];
    if (J) J[p] = det_d(m->dim, j);
  }
}

void or_coef_eval(const or_map* m, long n, const double* xi, double* a9) {
  for (long p = 0; p < n; ++p) {
    double a[3][3];
    coef_at(m, xi + 3 * p, a);
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s) a9[9 * p + 3 * r + s] = a[r][s];
  }
}

/* ------------------------------------------------------------------------ */
/* Inverse map x -> xi, by methods that do not use Newton iteration.         */
/* ------------------------------------------------------------------------ */

static double sin_product(int d, const double* xi) {
  double P = 1.0;
  for (int k = 0; k < d; ++k) P *= sin(2.0 * OR_PI * xi[k]);
  return P;
}

/* The tabulated map inside one cell (lower vertex `base`, indices taken with
   periodic continuation): x(f) = sum over the cell's 2^d vertices of
   prod_a (1 - f_a or f_a) X_vertex, the multilinear interpolant of the vertex
   coordinates, and its derivative jf[a][b] = dx^a / df_b.  f may lie outside
   [0, 1]: the cell's polynomial extended (used beyond a wall). */
static void tab_cell(const or_map* m, const int* base, const double* f, double* x, double jf[3][3]) {
  int d = m->dim;
  for (int a = 0; a < 3; ++a) {
    x[a] = 0.0;
    for (int b = 0; b < 3; ++b) jf[a][b] = 0.0;
  }
  for (int c = 0; c < (1 << d); ++c) {
    int iv[3] = {0, 0, 0};
    double w = 1.0, dw[3] = {1.0, 1.0, 1.0};
    for (int a = 0; a < d; ++a) {
      int up = (c >> a) & 1;
      iv[a] = base[a] + up;
      double wa = up ? f[a] : 1.0 - f[a];
      for (int b = 0; b < d; ++b) dw[b] *= (b == a) ? (up ? 1.0 : -1.0) : wa;
      w *= wa;
    }
    double xv[3];
    tab_x(m, iv, xv);
    for (int a = 0; a < d; ++a) {
      x[a] += w * xv[a];
      for (int b = 0; b < d; ++b) jf[a][b] += dw[b] * xv[a];
    }
  }
}

/* Inverse of the tabulated map by Newton iterations on the position u in
   cells, starting at xi_old (or the grid centre): each iteration takes the
   cell holding u (on a bounded axis the boundary cell beyond the wall, whose
   polynomial is extended there), solves its linearisation at u and moves u,
   at most one cell per axis per iteration; converged when the step is below
   1e-14 cell. */
static int tab_invert(const or_map* m, const double* x, const double* xi_old, double* xi) {
  int d = m->dim;
  int n[3] = {1, 1, 1};
  double u[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < d; ++a) {
    n[a] = tab_cells(m, a);
    u[a] = xi_old ? xi_old[a] * n[a] : 0.5 * n[a];
  }
  for (int it = 0; it < 500; ++it) {
    int base[3] = {0, 0, 0};
    double f[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d; ++a) {
      int c = (int)floor(u[a]);
      if (!m->tper[a]) c = c < 0 ? 0 : (c > n[a] - 1 ? n[a] - 1 : c);
      base[a] = c;
      f[a] = u[a] - c;
    }
    double xc[3], jf[3][3], k[3][3], du[3];
    tab_cell(m, base, f, xc, jf);
    for (int a = d; a < 3; ++a) jf[a][a] = 1.0;
    inv_d(d, jf, k);
    double big = 0.0;
    for (int a = 0; a < d; ++a) {
      du[a] = 0.0;
      for (int b = 0; b < d; ++b) du[a] += k[a][b] * (x[b] - xc[b]);
      if (fabs(du[a]) > big) big = fabs(du[a]);
    }
    double scale = big > 1.0 ? 1.0 / big : 1.0;
    for (int a = 0; a < d; ++a) u[a] += scale * du[a];
    if (big < 1e-14) {
      for (int a = 0; a < 3; ++a) xi[a] = (a < d) ? u[a] / n[a] : 0.0;
      return 0;
    }
  }
  for (int a = 0; a < 3; ++a) xi[a] = (a < d) ? u[a] / n[a] : 0.0;
  return -1;
}

/* Returns 0 on success.  xi_old is used only to pick the periodic image of the
   angular coordinate of the polar map, and the starting cell of a tabulated
   map's inversion. */
static int map_invert(const or_map* m, const double* x, const double* xi_old, double* xi) {
  int d = m->dim;
  for (int a = 0; a < 3; ++a) xi[a] = 0.0;
  if (m->kind == OR_TABULATED) return tab_invert(m, x, xi_old, xi);
  if (m->kind == OR_IDENTITY) {
    for (int a = 0; a < d; ++a) xi[a] = x[a] / m->L[a];
    return 0;
  }
  if (m->kind == OR_SINUSOIDAL) {
    /* x^a/L_a - xi^a = eps P(xi) = t for every axis, so xi^a = x^a/L_a - t and
       t is the root of g(t) = t - eps P(x/L - t), increasing (g' = J/prod L)
       and bracketed by |t| <= |eps|.  Bisection. */
    double u[3];
    for (int a = 0; a < d; ++a) u[a] = x[a] / m->L[a];
    double lo = -fabs(m->eps), hi = fabs(m->eps);
    if (hi == 0.0) {
      for (int a = 0; a < d; ++a) xi[a] = u[a];
      return 0;
    }
    for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {
      double mid = 0.5 * (lo + hi);
      if (mid == lo || mid == hi) break;
      double p[3];
      for (int a = 0; a < d; ++a) p[a] = u[a] - mid;
      double g = mid - m->eps * sin_product(d, p);
      if (g > 0.0)
        hi = mid;
      else
        lo = mid;
    }
    double t = 0.5 * (lo + hi);
    for (int a = 0; a < d; ++a) xi[a] = u[a] - t;
    return 0;
  }
  if (m->kind == OR_POLAR_LOG) {
    double r = hypot(x[0], x[1]);
    xi[0] = log(r / m->r_in) / log(m->r_out / m->r_in);
    double eta = atan2(x[1], x[0]) / (2.0 * OR_PI);
    if (xi_old) eta += nearbyint(xi_old[1] - eta);
    xi[1] = eta;
    return 0;
  }
  if (m->kind == OR_SPHERICAL_RZ) {
    double rho = hypot(x[0], x[1]);
    double th = atan2(x[0], x[1]);
    xi[0] = (rho - m->r_in) / (m->r_out - m->r_in);
    xi[1] = 1.0 - th / OR_PI;
    return 0;
  }
  return -1;
}

void or_map_invert(const or_map* m, long n, const double* x, const double* xi_old, double* xi) {
#pragma omp parallel for schedule(static)
  for (long p = 0; p < n; ++p) map_invert(m, x + 3 * p, xi_old ? xi_old + 3 * p : 0, xi + 3 * p);
}

/* ------------------------------------------------------------------------ */
/* Grid helpers                                                              */
/* ------------------------------------------------------------------------ */

static long ncells(const or_grid* g) {
  long n = 1;
  for (int a = 0; a < g->dim; ++a) n *= g->n[a];
  return n;
}
static int nvert_axis(const or_grid* g, int a) {
  return (g->bc_lo[a] == OR_PERIODIC) ? g->n[a] : g->n[a] + 1;
}
static long nverts(const or_grid* g) {
  long n = 1;
  for (int a = 0; a < g->dim; ++a) n *= nvert_axis(g, a);
  return n;
}
static void cell_coords(const or_grid* g, long c, int* idx) {
  idx[0] = idx[1] = idx[2] = 0;
  for (int a = 0; a < g->dim; ++a) {
    idx[a] = (int)(c % g->n[a]);
    c /= g->n[a];
  }
}
static long cell_lin(const or_grid* g, const int* idx) {
  long c = 0;
  for (int a = g->dim - 1; a >= 0; --a) c = c * g->n[a] + idx[a];
  return c;
}
static int all_periodic(const or_grid* g) {
  for (int a = 0; a < g->dim; ++a)
    if (g->bc_lo[a] != OR_PERIODIC) return 0;
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Charge deposit, Eqs. (pg), (Wpc), (b2); the order-2 B-spline is taken in   */
/* its standard (continuous, unit-sum) form with the factor 1/2 on the outer  */
/* branch.  Fixed-point rule: per-axis integer weights at scale 2^S1.        */
/* ------------------------------------------------------------------------ */

/* w[0] -> cell i-1, w[1] -> cell i, w[2] -> cell i+1, for in-cell offset f. */
static void w1d_fixed(int shape, int S1, double f, int64_t* w) {
  int64_t one = (int64_t)1 << S1;
  if (shape == OR_B2) {
    double a = 1.0 - f;
    int64_t L = (int64_t)rint(ldexp(a * a, S1 - 1));
    int64_t R = (int64_t)rint(ldexp(f * f, S1 - 1));
    w[0] = L;
    w[2] = R;
    w[1] = one - L - R;
  } else {
    double g = f - 0.5;
    if (g >= 0.0) {
      int64_t R = (int64_t)rint(ldexp(g, S1));
      w[0] = 0;
      w[1] = one - R;
      w[2] = R;
    } else {
      int64_t Lw = (int64_t)rint(ldexp(-g, S1));
      w[0] = Lw;
      w[1] = one - Lw;
      w[2] = 0;
    }
  }
}

static void w1d_f64(int shape, double f, double* w) {
  if (shape == OR_B2) {
    double a = 1.0 - f;
    double b = f - 0.5;
    w[0] = 0.5 * a * a;
    w[1] = 0.75 - b * b;
    w[2] = 0.5 * f * f;
  } else {
    double g = f - 0.5;
    if (g >= 0.0) {
      w[0] = 0.0;
      w[1] = 1.0 - g;
      w[2] = g;
    } else {
      w[0] = -g;
      w[1] = 1.0 + g;
      w[2] = 0.0;
    }
  }
}

/* target cell index along axis a for cell index t (may be -1 or n): periodic
   wrap, bounded axes fold the ghost target back onto the boundary cell. */
static int target_axis(const or_grid* g, int a, int t) {
  int n = g->n[a];
  if (g->bc_lo[a] == OR_PERIODIC) return ((t % n) + n) % n;
  if (t < 0) return 0;
  if (t >= n) return n - 1;
  return t;
}

/* Q[c] += sum_p prod_a w_a(p, c); integer sums are exact and order-free.
   cell_mask (optional) restricts accumulation to cells with mask != 0.
   Returns the number of particles skipped because cell < 0 (dead). */
long or_deposit_fixed(const or_grid* g, int shape, int S1, long np, const int32_t* cell,
                      const double* off, const uint8_t* cell_mask, uint64_t* Q) {
  long nc = ncells(g);
  int d = g->dim;
  long skipped = 0;
  int nthr = 1;
#ifdef _OPENMP
  nthr = omp_get_max_threads();
#endif
  uint64_t* priv = (uint64_t*)calloc((size_t)nthr * (size_t)nc, sizeof(uint64_t));
  if (!priv) return -1;
#pragma omp parallel reduction(+ : skipped)
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    uint64_t* q = priv + (size_t)tid * (size_t)nc;
#pragma omp for schedule(static)
    for (long p = 0; p < np; ++p) {
      if (cell[p] < 0) {
        skipped++;
        continue;
      }
      int idx[3];
      cell_coords(g, cell[p], idx);
      int64_t w[3][3];
      for (int a = 0; a < 3; ++a) {
        w[a][0] = 0;
        w[a][1] = 1;
        w[a][2] = 0;
      }
      for (int a = 0; a < d; ++a) w1d_fixed(shape, S1, off[3 * p + a], w[a]);
      int nk = (d == 3) ? 3 : 1;
      for (int oz = 0; oz < nk; ++oz)
        for (int oy = 0; oy < 3; ++oy)
          for (int ox = 0; ox < 3; ++ox) {
            int t[3];
            t[0] = target_axis(g, 0, idx[0] + ox - 1);
            t[1] = target_axis(g, 1, idx[1] + oy - 1);
            t[2] = (d == 3) ? target_axis(g, 2, idx[2] + oz - 1) : 0;
            uint64_t prod = (uint64_t)w[0][ox] * (uint64_t)w[1][oy];
            if (d == 3) prod *= (uint64_t)w[2][oz];
            long c = cell_lin(g, t);
            if (cell_mask && !cell_mask[c]) continue;
            q[c] += prod;
          }
    }
  }
  for (long c = 0; c < nc; ++c) {
    uint64_t s = 0;
    for (int t = 0; t < nthr; ++t) s += priv[(size_t)t * (size_t)nc + c];
    Q[c] = s;
  }
  free(priv);
  return skipped;
}

/* Unquantised FP64 deposit: Q[c] = sum_p W_pc (particle weight 1). */
long or_deposit_f64(const or_grid* g, int shape, long np, const int32_t* cell, const double* off,
                    double* Q) {
  long nc = ncells(g);
  int d = g->dim;
  long skipped = 0;
  for (long c = 0; c < nc; ++c) Q[c] = 0.0;
  for (long p = 0; p < np; ++p) {
    if (cell[p] < 0) {
      skipped++;
      continue;
    }
    int idx[3];
    cell_coords(g, cell[p], idx);
    double w[3][3];
    for (int a = 0; a < 3; ++a) {
      w[a][0] = 0.0;
      w[a][1] = 1.0;
      w[a][2] = 0.0;
    }
    for (int a = 0; a < d; ++a) w1d_f64(shape, off[3 * p + a], w[a]);
    int nk = (d == 3) ? 3 : 1;
    for (int oz = 0; oz < nk; ++oz)
      for (int oy = 0; oy < 3; ++oy)
        for (int ox = 0; ox < 3; ++ox) {
          int t[3];
          t[0] = target_axis(g, 0, idx[0] + ox - 1);
          t[1] = target_axis(g, 1, idx[1] + oy - 1);
          t[2] = (d == 3) ? target_axis(g, 2, idx[2] + oz - 1) : 0;
          double wt = w[0][ox] * w[1][oy];
          if (d == 3) wt *= w[2][oz];
          Q[cell_lin(g, t)] += wt;
        }
  }
  return skipped;
}

/* ------------------------------------------------------------------------ */
/* Fixed neutralising background: I_c = n0 * int S(xi - xi_c) J(xi) dxi with  */
/* the deposit's own shape S, by 8-point Gauss-Legendre on each half cell.   */
/* ------------------------------------------------------------------------ */

static const double GL8_X[8] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290,
                                -0.1834346424956498, 0.1834346424956498,  0.5255324099163290,
                                0.7966664774136267,  0.9602898564975363};
static const double GL8_W[8] = {0.1012285362903763, 0.2223810344533745, 0.3137066458778873,
                                0.3626837833783620, 0.3626837833783620, 0.3137066458778873,
                                0.2223810344533745, 0.1012285362903763};

void or_gl8(double* x, double* w) {
  for (int i = 0; i < 8; ++i) {
    x[i] = GL8_X[i];
    w[i] = GL8_W[i];
  }
}

static double shape_u(int shape, double u) {
  double a = fabs(u);
  if (shape == OR_B2) {
    if (a < 0.5) return 0.75 - u * u;
    if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
    return 0.0;
  }
  return a < 1.0 ? 1.0 - a : 0.0;
}

int or_ion_background(const or_map* m, const or_grid* g, int shape, double n0, double* I) {
  int d = g->dim;
  if (!all_periodic(g)) return -1;
  long nc = ncells(g);
  double h[3] = {1.0, 1.0, 1.0};
  for (int a = 0; a < d; ++a) h[a] = 1.0 / g->n[a];
  /* 1D nodes in cell units relative to the cell centre: 3 cells x 2 halves x 8 */
  double un[48], uw[48];
  int q = 0;
  for (int o = -1; o <= 1; ++o)
    for (int half = 0; half < 2; ++half) {
      double lo = o - 0.5 + 0.5 * half; /* interval [lo, lo + 0.5] */
      double mid = lo + 0.25;
      for (int k = 0; k < 8; ++k) {
        un[q] = mid + 0.25 * GL8_X[k];
        uw[q] = 0.25 * GL8_W[k];
        ++q;
      }
    }
#pragma omp parallel for schedule(dynamic, 16)
  for (long c = 0; c < nc; ++c) {
    int idx[3];
    cell_coords(g, c, idx);
    double sum = 0.0;
    int nz = (d == 3) ? 48 : 1;
    for (int qz = 0; qz < nz; ++qz)
      for (int qy = 0; qy < 48; ++qy)
        for (int qx = 0; qx < 48; ++qx) {
          double wx = uw[qx] * shape_u(shape, un[qx]);
          double wy = uw[qy] * shape_u(shape, un[qy]);
          double wz = (d == 3) ? uw[qz] * shape_u(shape, un[qz]) : 1.0;
          double wt = wx * wy * wz;
          if (wt == 0.0) continue;
          double xi[3] = {(idx[0] + 0.5 + un[qx]) * h[0], (idx[1] + 0.5 + un[qy]) * h[1],
                          (d == 3) ? (idx[2] + 0.5 + un[qz]) * h[2] : 0.0};
          double x[3], j[3][3];
          map_x_jac(m, xi, x, j);
          sum += wt * det_d(d, j);
        }
    I[c] = n0 * sum * h[0] * h[1] * h[2];
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Poisson operator (Eq. poiscurv times Omega J, integrated over a cell):     */
/*   A = -Hessian of Q(phi),                                                 */
/*   Q = 1/2 sum_faces w_f (phi_+ - phi_-)^2                                 */
/*     + sum_{i<j} sum_{edges} W_e (Delta_i phi)_e (Delta_j phi)_e,           */
/*   w_f = a^{ii}(face) dV / h_i^2,  W_e = a^{ij}(edge) dV / (h_i h_j),      */
/* (Delta_i phi)_e = half the sum of the two differences across axis i in the */
/* 2x2 block of cells around the edge (vertex in 2D).  Symmetric; second      */
/* order; conservative (flux form).  Ghost cells (Sec. II.B): Dirichlet        */
/* phi_g = 2 phi_b - phi_in, Neumann phi_g = phi_in.                          */
/* Stored as a 3^d stencil per row: A[c*S + o], o = (ox+1)+3(oy+1)+9(oz+1).   */
/* bdir[c] collects the boundary-value part, so that (A phi)_c + bdir_c is    */
/* the full discrete operator.                                               */
/* ------------------------------------------------------------------------ */

static int stencil_size(int d) { return d == 3 ? 27 : 9; }
static int off_index(int d, const int* o) {
  return (o[0] + 1) + 3 * (o[1] + 1) + (d == 3 ? 9 * (o[2] + 1) : 0);
}

int or_poisson_assemble(const or_map* m, const or_grid* g, double* A, double* bdir) {
  int d = g->dim;
  long nc = ncells(g);
  int S = stencil_size(d);
  double h[3] = {1.0, 1.0, 1.0};
  for (int a = 0; a < d; ++a) h[a] = 1.0 / g->n[a];
  double dV = h[0] * h[1] * h[2];
  int bounded = !all_periodic(g);
  /* with walls the mixed terms are dropped in every plane that holds a bounded
     axis: accepted only for maps orthogonal there (a tabulated map: up to its
     sampling error) */
  if (bounded && m->kind == OR_SINUSOIDAL && m->eps != 0.0) return -2;
  memset(A, 0, sizeof(double) * (size_t)nc * (size_t)S);
  memset(bdir, 0, sizeof(double) * (size_t)nc);
  for (long c = 0; c < nc; ++c) {
    int idx[3];
    cell_coords(g, c, idx);
    /* faces: the upper face of c on each axis, plus the lower wall face */
    for (int i = 0; i < d; ++i) {
      for (int side = 0; side < 2; ++side) {
        int wall = 0;
        double phib = 0.0;
        int bct;
        if (side == 0) { /* lower face: only if wall */
          if (idx[i] != 0 || g->bc_lo[i] == OR_PERIODIC) continue;
          wall = 1;
          bct = g->bc_lo[i];
          phib = g->phi_lo[i];
        } else {
          if (idx[i] == g->n[i] - 1 && g->bc_hi[i] != OR_PERIODIC) {
            wall = 1;
            bct = g->bc_hi[i];
            phib = g->phi_hi[i];
          }
        }
        double xi[3];
        for (int a = 0; a < 3; ++a) xi[a] = (a < d) ? (idx[a] + 0.5) * h[a] : 0.0;
        xi[i] = (idx[i] + side) * h[i];
        double a9[3][3];
        coef_at(m, xi, a9);
        double w = a9[i][i] * dV / (h[i] * h[i]);
        int o0[3] = {0, 0, 0};
        if (wall) {
          if (bct == OR_DIRICHLET) {
            A[c * S + off_index(d, o0)] -= 2.0 * w;
            bdir[c] += 2.0 * w * phib;
          }
          continue;
        }
        int nb[3] = {idx[0], idx[1], idx[2]};
        nb[i] = (idx[i] + 1) % g->n[i];
        long cn = cell_lin(g, nb);
        int op[3] = {0, 0, 0}, om[3] = {0, 0, 0};
        op[i] = 1;
        om[i] = -1;
        A[c * S + off_index(d, o0)] -= w;
        A[c * S + off_index(d, op)] += w;
        A[cn * S + off_index(d, o0)] -= w;
        A[cn * S + off_index(d, om)] += w;
      }
    }
    /* mixed terms: the corner at (idx_i + 1, idx_j + 1) of c in plane (i,j) */
    for (int i = 0; i < d; ++i)
      for (int j = i + 1; j < d; ++j) {
        if (bounded && (g->bc_lo[i] != OR_PERIODIC || g->bc_lo[j] != OR_PERIODIC)) {
          /* only orthogonal maps are accepted with walls (checked above) */
          continue;
        }
        double xi[3];
        for (int a = 0; a < 3; ++a) xi[a] = (a < d) ? (idx[a] + 0.5) * h[a] : 0.0;
        xi[i] = (idx[i] + 1) * h[i];
        xi[j] = (idx[j] + 1) * h[j];
        double a9[3][3];
        coef_at(m, xi, a9);
        double W = a9[i][j] * dV / (h[i] * h[j]);
        if (W == 0.0) continue;
        long cs[4];
        double ui[4], uj[4];
        int so[4][3];
        for (int s = 0; s < 4; ++s) {
          int si = s & 1, sj = (s >> 1) & 1;
          int t[3] = {idx[0], idx[1], idx[2]};
          t[i] = (idx[i] + si) % g->n[i];
          t[j] = (idx[j] + sj) % g->n[j];
          cs[s] = cell_lin(g, t);
          ui[s] = 0.5 * (2 * si - 1);
          uj[s] = 0.5 * (2 * sj - 1);
          so[s][0] = so[s][1] = so[s][2] = 0;
          so[s][i] = si;
          so[s][j] = sj;
        }
        for (int s = 0; s < 4; ++s)
          for (int t = 0; t < 4; ++t) {
            int o[3];
            for (int a = 0; a < 3; ++a) o[a] = so[t][a] - so[s][a];
            A[cs[s] * S + off_index(d, o)] -= W * (ui[s] * uj[t] + uj[s] * ui[t]);
          }
      }
  }
  return 0;
}

/* y = A x (stencil form, periodic wrap; out-of-domain entries are zero). */
void or_apply(const or_grid* g, const double* A, const double* x, double* y) {
  int d = g->dim;
  long nc = ncells(g);
  int S = stencil_size(d);
#pragma omp parallel for schedule(static)
  for (long c = 0; c < nc; ++c) {
    int idx[3];
    cell_coords(g, c, idx);
    double s = 0.0;
    for (int o = 0; o < S; ++o) {
      double a = A[c * S + o];
      if (a == 0.0) continue;
      int off[3] = {o % 3 - 1, (o / 3) % 3 - 1, (d == 3) ? o / 9 - 1 : 0};
      int t[3];
      int ok = 1;
      for (int k = 0; k < 3; ++k) {
        if (k >= d) {
          t[k] = 0;
          continue;
        }
        int v = idx[k] + off[k];
        if (g->bc_lo[k] == OR_PERIODIC)
          v = ((v % g->n[k]) + g->n[k]) % g->n[k];
        else if (v < 0 || v >= g->n[k])
          ok = 0;
        t[k] = v;
      }
      if (ok) s += a * x[cell_lin(g, t)];
    }
    y[c] = s;
  }
}

static double dot(long n, const double* a, const double* b) {
  double s = 0.0;
  for (long i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* Jacobi-preconditioned conjugate gradients on -A (A is negative
   semi-definite).  Stops when ||b - A x|| <= rtol ||b||. */
int or_cg(const or_grid* g, const double* A, const double* b, double* x, double rtol, int maxit,
          double* relres) {
  long nc = ncells(g);
  int S = stencil_size(g->dim);
  int center = (S == 27) ? 13 : 4;
  double* r = (double*)malloc(sizeof(double) * nc);
  double* z = (double*)malloc(sizeof(double) * nc);
  double* p = (double*)malloc(sizeof(double) * nc);
  double* q = (double*)malloc(sizeof(double) * nc);
  or_apply(g, A, x, q);
  for (long i = 0; i < nc; ++i) r[i] = b[i] - q[i];
  double bn = sqrt(dot(nc, b, b));
  if (bn == 0.0) bn = 1.0;
  for (long i = 0; i < nc; ++i) z[i] = r[i] / A[i * S + center];
  memcpy(p, z, sizeof(double) * nc);
  double rz = dot(nc, r, z);
  int it = 0;
  double rn = sqrt(dot(nc, r, r));
  while (rn > rtol * bn && it < maxit) {
    or_apply(g, A, p, q);
    double alpha = rz / dot(nc, p, q);
    for (long i = 0; i < nc; ++i) {
      x[i] += alpha * p[i];
      r[i] -= alpha * q[i];
    }
    rn = sqrt(dot(nc, r, r));
    ++it;
    if (rn <= rtol * bn) break;
    for (long i = 0; i < nc; ++i) z[i] = r[i] / A[i * S + center];
    double rz2 = dot(nc, r, z);
    double beta = rz2 / rz;
    rz = rz2;
    for (long i = 0; i < nc; ++i) p[i] = z[i] + beta * p[i];
  }
  /* true residual */
  or_apply(g, A, x, q);
  for (long i = 0; i < nc; ++i) r[i] = b[i] - q[i];
  if (relres) *relres = sqrt(dot(nc, r, r)) / bn;
  free(r);
  free(z);
  free(p);
  free(q);
  return it;
}

/* Cell-centre Jacobians (physical) and the full solve: A phi = -charge - bdir;
   all-periodic problems: right side projected to zero sum, and phi shifted so
   that its J-weighted mean is zero.  phi holds the initial guess on entry. */
int or_poisson_solve(const or_map* m, const or_grid* g, const double* charge, double* phi,
                     double rtol, int maxit, double* relres) {
  int d = g->dim;
  long nc = ncells(g);
  int S = stencil_size(d);
  double* A = (double*)malloc(sizeof(double) * (size_t)nc * S);
  double* bd = (double*)malloc(sizeof(double) * nc);
  double* b = (double*)malloc(sizeof(double) * nc);
  int rc = or_poisson_assemble(m, g, A, bd);
  if (rc) {
    free(A);
    free(bd);
    free(b);
    return rc;
  }
  for (long c = 0; c < nc; ++c) b[c] = -charge[c] - bd[c];
  int per = all_periodic(g);
  if (per) {
    double s = 0.0;
    for (long c = 0; c < nc; ++c) s += b[c];
    s /= (double)nc;
    for (long c = 0; c < nc; ++c) b[c] -= s;
  }
  int it = or_cg(g, A, b, phi, rtol, maxit, relres);
  if (per) {
    double sj = 0.0, sp = 0.0;
    double h[3] = {1.0, 1.0, 1.0};
    for (int a = 0; a < d; ++a) h[a] = 1.0 / g->n[a];
    for (long c = 0; c < nc; ++c) {
      int idx[3];
      cell_coords(g, c, idx);
      double xi[3] = {(idx[0] + 0.5) * h[0], (idx[1] + 0.5) * h[1], (idx[2] + 0.5) * h[2]};
      double x[3], j[3][3];
      map_x_jac(m, xi, x, j);
      double J = det_d(d, j);
      sj += J;
      sp += J * phi[c];
    }
    for (long c = 0; c < nc; ++c) phi[c] -= sp / sj;
  }
  free(A);
  free(bd);
  free(b);
  return it;
}

/* ------------------------------------------------------------------------ */
/* Electric field at vertices: E_v = -k(xi_v)^T (D phi)_v, (D_a phi)_v the   */
/* average over the 2^(d-1) cell pairs around v of the difference across a.  */
/* ------------------------------------------------------------------------ */

/* Field flux through the lower face of axis 0 (a conducting wall at
   potential phib): sum over the face cells c of 2 w_c (phib - phi_c), w_c the
   face coefficient a^{00} dV / h_0^2 of the discrete operator -- the discrete
   form of the surface integral of E . n, which Gauss' law sets equal to the
   charge the wall holds. */
double or_wall_flux(const or_map* m, const or_grid* g, const double* phi, double phib) {
  int d = g->dim;
  double h[3] = {1.0, 1.0, 1.0};
  for (int a = 0; a < d; ++a) h[a] = 1.0 / g->n[a];
  double dV = h[0] * h[1] * h[2];
  double F = 0.0;
  for (long c = 0; c < ncells(g); ++c) {
    int idx[3];
    cell_coords(g, c, idx);
    if (idx[0] != 0) continue;
    double xi[3];
    for (int a = 0; a < 3; ++a) xi[a] = (a < d) ? (idx[a] + 0.5) * h[a] : 0.0;
    xi[0] = 0.0;
    double a9[3][3];
    coef_at(m, xi, a9);
    double w = a9[0][0] * dV / (h[0] * h[0]);
    F += 2.0 * w * (phib - phi[c]);
  }
  return F;
}

static double phi_at(const or_grid* g, const double* phi, const int* idx_in) {
  int idx[3] = {idx_in[0], idx_in[1], idx_in[2]};
  for (int a = 0; a < g->dim; ++a) {
    int n = g->n[a];
    if (idx[a] >= 0 && idx[a] < n) continue;
    if (g->bc_lo[a] == OR_PERIODIC) {
      idx[a] = ((idx[a] % n) + n) % n;
      continue;
    }
    int lo = idx[a] < 0;
    int inner[3] = {idx[0], idx[1], idx[2]};
    inner[a] = lo ? 0 : n - 1;
    double pin = phi_at(g, phi, inner);
    int bct = lo ? g->bc_lo[a] : g->bc_hi[a];
    double pb = lo ? g->phi_lo[a] : g->phi_hi[a];
    return bct == OR_DIRICHLET ? 2.0 * pb - pin : pin;
  }
  return phi[cell_lin(g, idx)];
}

void or_efield(const or_map* m, const or_grid* g, const double* phi, double* Ev) {
  int d = g->dim;
  int nv[3] = {1, 1, 1};
  for (int a = 0; a < d; ++a) nv[a] = nvert_axis(g, a);
  long N = nverts(g);
  double h[3] = {1.0, 1.0, 1.0};
  for (int a = 0; a < d; ++a) h[a] = 1.0 / g->n[a];
#pragma omp parallel for schedule(static)
  for (long v = 0; v < N; ++v) {
    int vi[3] = {0, 0, 0};
    long t = v;
    for (int a = 0; a < d; ++a) {
      vi[a] = (int)(t % nv[a]);
      t /= nv[a];
    }
    double D[3] = {0.0, 0.0, 0.0};
    int npair = 1 << (d - 1);
    for (int a = 0; a < d; ++a) {
      double s = 0.0;
      for (int comb = 0; comb < npair; ++comb) {
        int cp[3] = {0, 0, 0}, cm[3] = {0, 0, 0};
        int bit = 0;
        for (int b = 0; b < d; ++b) {
          if (b == a) {
            cp[b] = vi[b];
            cm[b] = vi[b] - 1;
          } else {
            int sb = (comb >> bit) & 1;
            ++bit;
            cp[b] = cm[b] = vi[b] - 1 + sb;
          }
        }
        s += phi_at(g, phi, cp) - phi_at(g, phi, cm);
      }
      D[a] = s / (npair * h[a]);
    }
    double xi[3] = {vi[0] * h[0], vi[1] * h[1], (d == 3) ? vi[2] * h[2] : 0.0};
    double x[3], j[3][3], k[3][3];
    map_x_jac(m, xi, x, j);
    inv_d(d, j, k);
    for (int b = 0; b < 3; ++b) {
      double e = 0.0;
      if (b < d)
        for (int a = 0; a < d; ++a) e -= k[a][b] * D[a];
      Ev[3 * v + b] = e;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Gather (Eqs. vvp, Wvp, b1), Boris push (Eqs. step1, step1a), position     */
/* update x(xi^n) + dt v^{n+1/2} mapped back to logical space, boundaries.   */
/* ------------------------------------------------------------------------ */

static void gather_one(const or_grid* g, const double* Ev, int32_t cell, const double* off,
                       double* E) {
  int d = g->dim;
  int idx[3];
  cell_coords(g, cell, idx);
  int nv[3] = {1, 1, 1};
  for (int a = 0; a < d; ++a) nv[a] = nvert_axis(g, a);
  E[0] = E[1] = E[2] = 0.0;
  int nk = (d == 3) ? 2 : 1;
  for (int cz = 0; cz < nk; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        int cc[3] = {cx, cy, cz};
        double w = 1.0;
        long v = 0;
        for (int a = d - 1; a >= 0; --a) {
          int vi = idx[a] + cc[a];
          if (vi >= nv[a]) vi -= nv[a]; /* periodic: vertex n is vertex 0 */
          v = v * nv[a] + vi;
          w *= cc[a] ? off[a] : 1.0 - off[a];
        }
        for (int b = 0; b < 3; ++b) E[b] += w * Ev[3 * v + b];
      }
}

void or_gather(const or_grid* g, const double* Ev, long np, const int32_t* cell, const double* off,
               double* Ep) {
#pragma omp parallel for schedule(static)
  for (long p = 0; p < np; ++p) gather_one(g, Ev, cell[p], off + 3 * p, Ep + 3 * p);
}

static void cross(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Boris: half electric kick, magnetic rotation, half electric kick.  With
   B = 0 it is the leap-frog kick v += (q/m) E dt. */
static void boris(double* v, const double* E, const double* B, double qm, double dt) {
  double vm[3], t[3], vp[3], c[3], s[3];
  for (int a = 0; a < 3; ++a) {
    vm[a] = v[a] + 0.5 * dt * qm * E[a];
    t[a] = 0.5 * dt * qm * B[a];
  }
  double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  cross(vm, t, c);
  for (int a = 0; a < 3; ++a) {
    vp[a] = vm[a] + c[a];
    s[a] = 2.0 * t[a] / (1.0 + t2);
  }
  cross(vp, s, c);
  for (int a = 0; a < 3; ++a) v[a] = vm[a] + c[a] + 0.5 * dt * qm * E[a];
}

void or_boris(long np, double* v, const double* E, const double* B, double qm, double dt) {
  for (long p = 0; p < np; ++p) boris(v + 3 * p, E + 3 * p, B, qm, dt);
}

/* Cyclotronic step (Sec. "Particle mover": with a uniform background B the
   gyration is resolved exactly, so that the time step need not resolve
   omega_c): the velocity takes the electric impulse (q/m) E dt, then the
   particle gyrates exactly in B for dt.  With w = (q/m)|B|, b = B/|B|,
   v = v_par b + v_perp and theta = w dt:
     v(dt)   = v_par b + v_perp cos(theta) + (v_perp x b) sin(theta),
     x(dt)-x = dt [v_par b + v_perp sin(theta)/theta + (v_perp x b)(1 - cos(theta))/theta].
   vmean receives the bracket (the mean velocity over the step); B = 0 is the
   leap-frog step.  Series for |theta| < 1e-4. */
static void cyclotronic(double* v, const double* E, const double* B, double qm, double dt, double* vmean) {
  for (int a = 0; a < 3; ++a) v[a] += qm * E[a] * dt;
  double bn = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
  if (bn == 0.0) {
    for (int a = 0; a < 3; ++a) vmean[a] = v[a];
    return;
  }
  double b[3] = {B[0] / bn, B[1] / bn, B[2] / bn};
  double th = qm * bn * dt;
  double vpar = v[0] * b[0] + v[1] * b[1] + v[2] * b[2];
  double vp[3], w[3];
  for (int a = 0; a < 3; ++a) vp[a] = v[a] - vpar * b[a];
  cross(vp, b, w);
  double c = cos(th), s = sin(th), s1, s2;
  if (fabs(th) < 1e-4) {
    s1 = 1.0 - th * th / 6.0;
    s2 = th / 2.0 - th * th * th / 24.0;
  } else {
    s1 = s / th;
    s2 = (1.0 - c) / th;
  }
  for (int a = 0; a < 3; ++a) {
    vmean[a] = vpar * b[a] + vp[a] * s1 + w[a] * s2;
    v[a] = vpar * b[a] + vp[a] * c + w[a] * s;
  }
}

void or_cyclotronic(long np, double* v, const double* E, const double* B, double qm, double dt,
                    double* vmean) {
  for (long p = 0; p < np; ++p) cyclotronic(v + 3 * p, E + 3 * p, B, qm, dt, vmean + 3 * p);
}

/* Logical position from absolute xi: returns 0 alive, 1 absorbed at a lower
   wall, 2 left through an upper wall. */
static int place(const or_grid* g, double* xi, int32_t* cell, double* off, int* wall_axis) {
  int d = g->dim;
  int idx[3] = {0, 0, 0};
  for (int a = 0; a < d; ++a) {
    if (g->bc_lo[a] == OR_PERIODIC) {
      xi[a] -= floor(xi[a]);
    } else {
      if (xi[a] < 0.0) {
        *wall_axis = a;
        return 1;
      }
      if (xi[a] >= 1.0) {
        *wall_axis = a;
        return 2;
      }
    }
  }
  for (int a = 0; a < d; ++a) {
    double u = xi[a] * g->n[a];
    double fl = floor(u);
    int ci = (int)fl;
    double f = u - fl;
    if (ci >= g->n[a]) {
      if (g->bc_lo[a] == OR_PERIODIC) {
        ci -= g->n[a];
      } else {
        ci = g->n[a] - 1;
        f = nextafter(1.0, 0.0);
      }
    }
    idx[a] = ci;
    off[a] = f;
  }
  for (int a = d; a < 3; ++a) off[a] = 0.0;
  *cell = (int32_t)cell_lin(g, idx);
  return 0;
}

/* One mover pass for one species: gather E^n at xi^n, v^{n-1/2} -> v^{n+1/2},
   xi^{n+1} = x^{-1}(x(xi^n) + dt v^{n+1/2}), boundaries.  Dead particles get
   cell = -1 (lower wall, absorbed) or -2 (upper wall, outflow).  In 2D v_z is
   pushed as the third component (zero field, rotated only by B).
   counts[0] absorbed, counts[1] outflow. */
/* The hybrid mover with the cyclotronic velocity step: the position update
   maps x(xi^n) + dt vmean back to logical space exactly (vmean the mean
   velocity of the exact gyration over the step). */
int or_push_cyclo(const or_map* m, const or_grid* g, double qm, double dt, const double* B, long np,
                  int32_t* cell, double* off, double* vel, const double* Ev, long* counts) {
  int d = g->dim;
  long absorbed = 0, outflow = 0;
#pragma omp parallel for schedule(static) reduction(+ : absorbed, outflow)
  for (long p = 0; p < np; ++p) {
    if (cell[p] < 0) continue;
    double E[3], vm[3];
    gather_one(g, Ev, cell[p], off + 3 * p, E);
    cyclotronic(vel + 3 * p, E, B, qm, dt, vm);
    int idx[3];
    cell_coords(g, cell[p], idx);
    double xi0[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d; ++a) xi0[a] = (idx[a] + off[3 * p + a]) / g->n[a];
    double x0[3], j[3][3];
    map_x_jac(m, xi0, x0, j);
    double xt[3];
    for (int a = 0; a < 3; ++a) xt[a] = (a < d) ? x0[a] + dt * vm[a] : 0.0;
    double xi1[3];
    map_invert(m, xt, xi0, xi1);
    int wa = -1;
    int st = place(g, xi1, &cell[p], off + 3 * p, &wa);
    if (st == 1) {
      cell[p] = -1;
      absorbed++;
    } else if (st == 2) {
      cell[p] = -2;
      outflow++;
    }
  }
  if (counts) {
    counts[0] = absorbed;
    counts[1] = outflow;
  }
  return 0;
}

int or_push(const or_map* m, const or_grid* g, double qm, double dt, const double* B, long np,
            int32_t* cell, double* off, double* vel, const double* Ev, long* counts) {
  int d = g->dim;
  long absorbed = 0, outflow = 0;
#pragma omp parallel for schedule(static) reduction(+ : absorbed, outflow)
  for (long p = 0; p < np; ++p) {
    if (cell[p] < 0) continue;
    double E[3];
    gather_one(g, Ev, cell[p], off + 3 * p, E);
    boris(vel + 3 * p, E, B, qm, dt);
    int idx[3];
    cell_coords(g, cell[p], idx);
    double xi0[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d; ++a) xi0[a] = (idx[a] + off[3 * p + a]) / g->n[a];
    double x0[3], j[3][3];
    map_x_jac(m, xi0, x0, j);
    double xt[3];
    for (int a = 0; a < 3; ++a) xt[a] = (a < d) ? x0[a] + dt * vel[3 * p + a] : 0.0;
    double xi1[3];
    map_invert(m, xt, xi0, xi1);
    int wa = -1;
    int st = place(g, xi1, &cell[p], off + 3 * p, &wa);
    if (st == 1) {
      cell[p] = -1;
      absorbed++;
    } else if (st == 2) {
      cell[p] = -2;
      outflow++;
    }
  }
  if (counts) {
    counts[0] = absorbed;
    counts[1] = outflow;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Predictor-corrector hybrid position update (Sec. "Particle mover",        */
/* Eqs. hybridx, step2, step3, step4).  The logical position moves with      */
/* d xi^i / dt = k^ij v^j, k = (dx/dxi)^{-1}:                                */
/*   predictor  xi' = xi^n + (dt/2) k(xi^n) v^{n+1/2},                       */
/*   corrector  xi^{n+1} = xi^n + dt k(xi') v^{n+1/2}.                       */
/* k is known at the vertices (the map's inverse Jacobian there) and carried */
/* to a position by the CIC vertex weights of Eq. Wvp with b1, Eq. step3 --  */
/* at xi^n as well as at xi'.  kmode 1 evaluates k from the map at the       */
/* position itself instead (no interpolation); it exists to pin the time     */
/* discretisation separately from the interpolation.                        */
/* ------------------------------------------------------------------------ */

static void k_exact(const or_map* m, int d, const double* xi, double k[3][3]) {
  double x[3], j[3][3];
  map_x_jac(m, xi, x, j);
  inv_d(d, j, k);
}

/* k at logical point xi.  Interpolation (kmode 0): the cell holding xi, the
   2^d vertices of that cell weighted by prod_a (1 - f_a or f_a).  On a
   periodic axis xi is taken modulo 1; on a bounded axis it is clamped into
   [0, 1] (the predictor point of a particle about to leave). */
static void k_at(const or_map* m, const or_grid* g, int kmode, const double* xi_in, double k[3][3]) {
  int d = g->dim;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) k[a][b] = 0.0;
  if (kmode == 1) {
    double xi[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d; ++a) xi[a] = xi_in[a];
    k_exact(m, d, xi, k);
    return;
  }
  int idx[3] = {0, 0, 0};
  double f[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < d; ++a) {
    double u = xi_in[a] * g->n[a];
    if (g->bc_lo[a] == OR_PERIODIC) {
      u -= g->n[a] * floor(u / g->n[a]);
    } else {
      if (u < 0.0) u = 0.0;
      if (u > g->n[a]) u = g->n[a];
    }
    int i = (int)floor(u);
    if (i >= g->n[a]) i = g->n[a] - 1;
    if (i < 0) i = 0;
    idx[a] = i;
    f[a] = u - i;
  }
  int nk = (d == 3) ? 2 : 1;
  for (int cz = 0; cz < nk; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        int cc[3] = {cx, cy, cz};
        double w = 1.0, xv[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < d; ++a) {
          w *= cc[a] ? f[a] : 1.0 - f[a];
          xv[a] = (double)(idx[a] + cc[a]) / g->n[a]; /* vertex position */
        }
        double kv[3][3];
        k_exact(m, d, xv, kv);
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < d; ++b) k[a][b] += w * kv[a][b];
      }
}

/* One mover pass with the predictor-corrector position update; gather,
   Boris and boundaries as in or_push. */
int or_push_pc(const or_map* m, const or_grid* g, double qm, double dt, const double* B, long np,
               int32_t* cell, double* off, double* vel, const double* Ev, int kmode, long* counts) {
  int d = g->dim;
  long absorbed = 0, outflow = 0;
#pragma omp parallel for schedule(static) reduction(+ : absorbed, outflow)
  for (long p = 0; p < np; ++p) {
    if (cell[p] < 0) continue;
    double E[3];
    gather_one(g, Ev, cell[p], off + 3 * p, E);
    boris(vel + 3 * p, E, B, qm, dt);
    const double* v = vel + 3 * p;
    int idx[3];
    cell_coords(g, cell[p], idx);
    double xi0[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d; ++a) xi0[a] = (idx[a] + off[3 * p + a]) / g->n[a];
    double k0[3][3], k1[3][3];
    k_at(m, g, kmode, xi0, k0);
    double xip[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d; ++a) {
      double s = 0.0;
      for (int b = 0; b < d; ++b) s += k0[a][b] * v[b];
      xip[a] = xi0[a] + 0.5 * dt * s;
    }
    k_at(m, g, kmode, xip, k1);
    double xi1[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d; ++a) {
      double s = 0.0;
      for (int b = 0; b < d; ++b) s += k1[a][b] * v[b];
      xi1[a] = xi0[a] + dt * s;
    }
    int wa = -1;
    int st = place(g, xi1, &cell[p], off + 3 * p, &wa);
    if (st == 1) {
      cell[p] = -1;
      absorbed++;
    } else if (st == 2) {
      cell[p] = -2;
      outflow++;
    }
  }
  if (counts) {
    counts[0] = absorbed;
    counts[1] = outflow;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter-based RNG.      */
/* ------------------------------------------------------------------------ */

void or_philox4x32_10(const uint32_t* ctr_in, const uint32_t* key_in, uint32_t* out) {
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k[2] = {key_in[0], key_in[1]};
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)M0 * c[0];
    uint64_t p1 = (uint64_t)M1 * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    uint32_t n3 = lo0;
    c[0] = n0;
    c[1] = n1;
    c[2] = n2;
    c[3] = n3;
    k[0] += W0;
    k[1] += W1;
  }
  out[0] = c[0];
  out[1] = c[1];
  out[2] = c[2];
  out[3] = c[3];
}

/* Number of OpenMP threads the oracle's parallel loops use. */
int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Injection of a Maxwellian at rest through the upper face of axis 0 (the   */
/* outer wall), Sec. III: per step lambda = n0 v_th / sqrt(2 pi) * A dt / w   */
/* particles on average (one-sided Maxwellian flux through a face of area A), */
/* count = floor(lambda) + Bernoulli(frac lambda).  Each particle: uniform    */
/* tangential logical position, inward normal speed v_th sqrt(-2 ln u)        */
/* (flux-weighted half-Maxwellian), tangential components N(0, v_th^2) by     */
/* Box-Muller, then a free flight over a uniform fraction of the step from    */
/* the face.  Random numbers: Philox4x32-10, key (seed_lo, seed_hi), counter  */
/* (step, k, species, purpose); u = (r + 1/2) 2^-32.                          */
/* ------------------------------------------------------------------------ */

static double u01(uint32_t r) { return ((double)r + 0.5) * (1.0 / 4294967296.0); }

double or_face_area(const or_map* m) {
  if (m->kind == OR_POLAR_LOG) return 2.0 * OR_PI * m->r_out;
  double A = 1.0;
  for (int b = 1; b < m->dim; ++b) A *= m->L[b];
  return A;
}

/* Inward flux of a Maxwellian of thermal speed vth drifting with speed
   u = s vth along the inward normal: n0 vth (phi(s) + s Phi(s)), phi and Phi
   the standard normal density and distribution (s = 0: n0 vth / sqrt(2 pi)). */
double or_drift_flux(double n0, double vth, double s) {
  return n0 * vth * (exp(-0.5 * s * s) / sqrt(2.0 * OR_PI) + s * 0.5 * (1.0 + erf(s / sqrt(2.0))));
}

/* Inward normal speed of one injected particle (units of vth), distributed
   as w exp(-(w - s)^2 / 2) on w > 0 (the flux-weighted drifting Maxwellian).
   s = 0: w = sqrt(-2 ln U).  s > 0: rejection from the normal N(s + delta, 1),
   delta = 1 / mode = 2 / (s + sqrt(s^2 + 4)); the ratio of target to proposal
   is w exp((s - mu) w + const), so a proposal w > 0 is kept with probability
   delta w exp(1 - delta w).  Attempt t uses the Philox block of counter
   (step, k, species, 3 + t); 64 attempts at most (the last proposal is kept). */
static double inject_normal_speed(double s, const uint32_t* key, uint32_t step, uint32_t k, uint32_t species,
                                  double u_rayleigh) {
  if (s <= 0.0) return sqrt(-2.0 * log(u_rayleigh));
  double delta = 2.0 / (s + sqrt(s * s + 4.0)), mu = s + delta, w = mu;
  for (uint32_t t = 0; t < 64; ++t) {
    uint32_t c[4] = {step, k, species, 3u + t}, r[4];
    or_philox4x32_10(c, key, r);
    w = mu + sqrt(-2.0 * log(u01(r[0]))) * cos(2.0 * OR_PI * u01(r[1]));
    if (w > 0.0 && u01(r[2]) < delta * w * exp(1.0 - delta * w)) return w;
  }
  return w > 0.0 ? w : mu;
}

long or_inject(const or_map* m, const or_grid* g, double n0, double vth, double drift, double w, double dt,
               uint32_t seed_lo, uint32_t seed_hi, uint32_t step, uint32_t species, long cap,
               int32_t* cell, double* off, double* vel, long* kidx, long* drawn) {
  int d = g->dim;
  const double s_drift = drift / vth;
  double lam = or_drift_flux(n0, vth, s_drift) * or_face_area(m) * dt / w;
  uint32_t key[2] = {seed_lo, seed_hi};
  uint32_t c0[4] = {step, 0xFFFFFFFFu, species, 2u}, r[4];
  or_philox4x32_10(c0, key, r);
  long count = (long)floor(lam) + (u01(r[0]) < lam - floor(lam) ? 1 : 0);
  if (drawn) *drawn = count;
  long out = 0;
  for (long k = 0; k < count && out < cap; ++k) {
    uint32_t ca[4] = {step, (uint32_t)k, species, 0u}, cb[4] = {step, (uint32_t)k, species, 1u};
    uint32_t ra[4], rb[4];
    or_philox4x32_10(ca, key, ra);
    or_philox4x32_10(cb, key, rb);
    double xi_f[3] = {1.0, u01(ra[0]), (d == 3) ? u01(rb[1]) : 0.0};
    double vn = vth * inject_normal_speed(s_drift, key, step, (uint32_t)k, species, u01(ra[1]));
    double rho = sqrt(-2.0 * log(u01(ra[2])));
    double t1 = vth * rho * cos(2.0 * OR_PI * u01(ra[3]));
    double t2 = vth * rho * sin(2.0 * OR_PI * u01(ra[3]));
    double frac = u01(rb[0]);
    double xf[3], j[3][3];
    map_x_jac(m, xi_f, xf, j);
    /* orthonormal frame of the (orthogonal) map at the face: columns of j */
    double e[3][3];
    for (int b = 0; b < 3; ++b) {
      double nrm = 0.0;
      for (int a = 0; a < 3; ++a) nrm += j[a][b] * j[a][b];
      nrm = sqrt(nrm);
      for (int a = 0; a < 3; ++a) e[b][a] = j[a][b] / nrm;
    }
    double v[3];
    for (int a = 0; a < 3; ++a) v[a] = -vn * e[0][a] + t1 * e[1][a];
    if (d == 2)
      v[2] += t2;
    else
      for (int a = 0; a < 3; ++a) v[a] += t2 * e[2][a];
    double xt[3];
    for (int a = 0; a < 3; ++a) xt[a] = (a < d) ? xf[a] + frac * dt * v[a] : 0.0;
    double xi[3];
    map_invert(m, xt, xi_f, xi);
    int wa = -1;
    int32_t c;
    double o[3];
    if (place(g, xi, &c, o, &wa) != 0) continue;
    cell[out] = c;
    for (int a = 0; a < 3; ++a) {
      off[3 * out + a] = o[a];
      vel[3 * out + a] = v[a];
    }
    if (kidx) kidx[out] = k;
    ++out;
  }
  return out;
}
