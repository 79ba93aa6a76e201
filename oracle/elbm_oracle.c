/*
 * elbm_oracle.c -- plain FP64 CPU oracle of the entropic lattice Boltzmann
 * method (ELBM) with the closed-form relaxation parameter of Zhao & Yong.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
 * CPU baseline of the benchmark, never by the product path.  It shares no
 * code with the HIP library.
 *
 * The code follows the paper's statement of the scheme in the paper's order:
 *   moments (conservation constraints after Eq. (3))
 *   -> entropic equilibrium (minimiser of Eq. (3) under those constraints)
 *   -> alpha_max (definition after Eq. (7)) -> alpha_* (Eq. (8))
 *   -> acceptance test H(f*(alpha_*)) <= H(f) -> otherwise Eq. (9)
 *   -> collision Eq. (1) (= Eq. (5a)) -> periodic streaming Eq. (5b).
 * Comparison solvers of the entropy balance Eq. (4): bisection with the stop
 * window used for the double shear flow, a bracketed Newton iteration, and
 * the modified secant iteration of the closing remark.  LBGK (alpha = 2 with
 * the polynomial equilibrium) is the special case named after Eq. (4).
 *
 * The paper states the scheme for the Boltzmann entropy of Eq. (3) and
 * remarks that the formula holds for any convex entropy; the oracle also
 * runs it with Burg's entropy H(f) = -sum_i W_i ln(f_i / W_i).
 *
 * Readings of points the paper leaves open (each one is listed with its
 * reason in the design notes of the repository):
 *   - lattice units, c_s^2 = 1/3, tensor-product weights W = (2/3,1/6,1/6)^D;
 *   - on the tensor-product lattices the equilibrium is written in its closed
 *     product form (derived below); on D3Q19, whose weights do not factorise,
 *     it is the minimiser of Eq. (3) found by Newton's method on the Lagrange
 *     multipliers (the same solver is exported for every lattice);
 *   - entropy differences between states with equal moments are evaluated
 *     as relative entropies with respect to f^eq (exact identity, below);
 *   - 0 ln 0 = 0; alpha_max = +inf when no i has f_i^eq < f_i;
 *   - when f = f^eq to rounding (D(f) <= 1e-26 rho, or alpha_max = +inf),
 *     alpha := alpha_* (the paper: alpha is then arbitrary);
 *   - Eq. (9)'s result is clamped to [1, alpha_*], where it lies exactly;
 *   - with Burg's entropy, which is infinite at a zero population, alpha_* =
 *     alpha_max < 2 makes both entropy differences of Eq. (9) infinite: their
 *     ratio is 1 in the limit, so Eq. (9) (and the modified secant) give
 *     alpha = 1.
 */
#include "elbm_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QMAX 27
#define GUARD_REL 1e-26

enum { ENT_BOLTZMANN = 0, ENT_BURG = 1 };

typedef struct {
  int D, Q;
  int product;          /* weights factorise per axis (D1Q3, D2Q9, D3Q27)  */
  int ent;              /* ENT_BOLTZMANN (Eq. (3)) or ENT_BURG              */
  int c[QMAX][3];
  double W[QMAX];
} lat_t;

/* Lattice codes: 1, 2, 3 for the tensor-product lattices D1Q3, D2Q9, D3Q27,
 * 19 for D3Q19.
 * Direction i <-> c_i on the tensor-product lattices: i = d(c_x) + 3 d(c_y)
 * + 9 d(c_z), d(0)=0, d(1)=1, d(-1)=2.  W_i = prod_a w(c_ia), w(0) = 4/6,
 * w(+-1) = 1/6, i.e. W_i = 4^{#zero components} / 6^D, formed with one
 * rounding.
 * D3Q19 keeps the D3Q27 directions with at most two nonzero components, in
 * the order of their D3Q27 index, with the standard weights 1/3 (rest),
 * 1/18 (|c|^2 = 1) and 1/36 (|c|^2 = 2). */
static int make_lattice(int code, lat_t *L) {
  L->ent = ENT_BOLTZMANN;
  if (code == 19) {
    L->D = 3;
    L->Q = 0;
    L->product = 0;
    for (int j = 0; j < 27; ++j) {
      int c[3], rem = j, nnz = 0;
      for (int a = 0; a < 3; ++a) {
        int d = rem % 3;
        rem /= 3;
        c[a] = (d == 0) ? 0 : (d == 1) ? 1 : -1;
        nnz += (c[a] != 0);
      }
      if (nnz == 3) continue;
      for (int a = 0; a < 3; ++a) L->c[L->Q][a] = c[a];
      L->W[L->Q] = (nnz == 0) ? 1.0 / 3.0 : (nnz == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
      L->Q++;
    }
    return 0;
  }
  int D = code;
  if (D < 1 || D > 3) return -1;
  L->D = D;
  L->product = 1;
  L->Q = (D == 1) ? 3 : (D == 2) ? 9 : 27;
  double den = (D == 1) ? 6.0 : (D == 2) ? 36.0 : 216.0;
  for (int i = 0; i < L->Q; ++i) {
    int rem = i, nzero = 0;
    for (int a = 0; a < 3; ++a) {
      int c = 0;
      if (a < D) {
        int d = rem % 3;
        rem /= 3;
        c = (d == 0) ? 0 : (d == 1) ? 1 : -1;
        if (c == 0) nzero++;
      }
      L->c[i][a] = c;
    }
    double num = 1.0;
    for (int k = 0; k < nzero; ++k) num *= 4.0;
    L->W[i] = num / den;
  }
  return 0;
}

/* Model code of the single-state functions: lattice code + 256 x entropy
 * (0: the Boltzmann entropy of Eq. (3), 1: Burg's entropy). */
static int make_model(int code, lat_t *L) {
  const int ent = code >> 8;
  if (code < 0 || ent > ENT_BURG || make_lattice(code & 255, L)) return -1;
  L->ent = ent;
  return 0;
}

/* u inside the domain of the entropic equilibrium: the interior of the
 * convex hull of the velocities (the mean of c under positive weights).
 * Tensor-product lattices: |u_a| < 1.  D3Q19 (no corner velocities): also
 * |u_x| + |u_y| + |u_z| < 2. */
static int u_admissible(const lat_t *L, const double *u) {
  double s = 0.0;
  for (int a = 0; a < L->D; ++a) {
    if (!(fabs(u[a]) < 1.0)) return 0;
    s += fabs(u[a]);
  }
  return L->product || s < 2.0;
}

/* ---- moments: rho = sum_i f_i, rho u = sum_i c_i f_i (after Eq. (3)) ---- */
static void moments(const lat_t *L, const double *f, double *rho, double *u) {
  double r = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < L->Q; ++i) {
    r += f[i];
    for (int a = 0; a < L->D; ++a) j[a] += L->c[i][a] * f[i];
  }
  *rho = r;
  for (int a = 0; a < 3; ++a) u[a] = (a < L->D) ? j[a] / r : 0.0;
}

/* ---- entropic equilibrium ------------------------------------------------
 * f^eq minimises H(f) = sum_i f_i ln(f_i/W_i) (Eq. (3)) subject to the mass
 * and momentum constraints.  Stationarity of the Lagrangian gives
 * f_i^eq = W_i exp(l0 + l.c_i); with tensor-product weights the sums over i
 * factorise per axis a, with z_a = exp(l_a):
 *   u_a = (z - 1/z) / (4 + z + 1/z)        ->  z_a = (2u_a + s_a)/(1 - u_a),
 *   s_a = sqrt(1 + 3 u_a^2),  normalisation (2/3 + (z+1/z)/6)^-1 = 2 - s_a,
 * hence f_i^eq = rho W_i prod_a (2 - s_a) z_a^{c_ia}, defined for |u_a| < 1. */
static void equilibrium_product(const lat_t *L, double rho, const double *u,
                                double *feq) {
  double A[3] = {1.0, 1.0, 1.0}, z[3] = {1.0, 1.0, 1.0};
  for (int a = 0; a < L->D; ++a) {
    double s = sqrt(1.0 + 3.0 * u[a] * u[a]);
    A[a] = 2.0 - s;
    z[a] = (2.0 * u[a] + s) / (1.0 - u[a]);
  }
  for (int i = 0; i < L->Q; ++i) {
    double v = rho * L->W[i];
    for (int a = 0; a < L->D; ++a) {
      double zc = (L->c[i][a] == 1) ? z[a] : (L->c[i][a] == -1) ? 1.0 / z[a] : 1.0;
      v *= A[a] * zc;
    }
    feq[i] = v;
  }
}

/* The same minimiser for any velocity set, without a closed form.  With
 * p_i(l) = W_i exp(l.c_i) / Z(l), Z(l) = sum_i W_i exp(l.c_i), the
 * constraints read m(l) := sum_i c_i p_i(l) = u, and m(l) - u is the gradient
 * of the convex function F(l) = ln Z(l) - l.u, whose Hessian is the
 * covariance sum_i c_i c_i^T p_i - m m^T.  Newton's method on F from l = 0,
 * with step halving while a long step fails to decrease F; it stops after a
 * step below 1e-12 (quadratic convergence leaves an error of order its
 * square).  Then f_i^eq = rho p_i(l).  Returns the iteration count, or -1 if
 * it did not converge (feq is then NaN). */
static void F_of(const lat_t *L, const double *u, const double *l, double *F,
                 double *g, double H[3][3]) {
  double Z = 0.0, m[3] = {0.0, 0.0, 0.0}, S[3][3] = {{0.0}};
  for (int i = 0; i < L->Q; ++i) {
    double lc = 0.0;
    for (int a = 0; a < L->D; ++a) lc += l[a] * L->c[i][a];
    double p = L->W[i] * exp(lc);
    Z += p;
    for (int a = 0; a < L->D; ++a) {
      m[a] += L->c[i][a] * p;
      for (int b = 0; b < L->D; ++b) S[a][b] += L->c[i][a] * L->c[i][b] * p;
    }
  }
  double lu = 0.0;
  for (int a = 0; a < L->D; ++a) lu += l[a] * u[a];
  *F = log(Z) - lu;
  if (g)
    for (int a = 0; a < L->D; ++a) {
      g[a] = m[a] / Z - u[a];
      for (int b = 0; b < L->D; ++b) H[a][b] = S[a][b] / Z - (m[a] / Z) * (m[b] / Z);
    }
}

/* Solve A x = r (n <= 3) by Gaussian elimination with partial pivoting. */
static int solve_small(int n, double A[3][3], double *r, double *x) {
  double M[3][4];
  for (int a = 0; a < n; ++a) {
    for (int b = 0; b < n; ++b) M[a][b] = A[a][b];
    M[a][n] = r[a];
  }
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int a = k + 1; a < n; ++a)
      if (fabs(M[a][k]) > fabs(M[piv][k])) piv = a;
    if (M[piv][k] == 0.0) return -1;
    for (int b = 0; b <= n; ++b) {
      double t = M[k][b];
      M[k][b] = M[piv][b];
      M[piv][b] = t;
    }
    for (int a = k + 1; a < n; ++a) {
      double f = M[a][k] / M[k][k];
      for (int b = k; b <= n; ++b) M[a][b] -= f * M[k][b];
    }
  }
  for (int a = n - 1; a >= 0; --a) {
    double v = M[a][n];
    for (int b = a + 1; b < n; ++b) v -= M[a][b] * x[b];
    x[a] = v / M[a][a];
  }
  return 0;
}

static int equilibrium_minimiser(const lat_t *L, double rho, const double *u,
                                 double *feq) {
  const int D = L->D;
  double l[3] = {0.0, 0.0, 0.0};
  int iters = -1;
  for (int it = 1; it <= 60; ++it) {
    double F, g[3], H[3][3], d[3], ng[3];
    F_of(L, u, l, &F, g, H);
    for (int a = 0; a < D; ++a) ng[a] = -g[a];
    if (solve_small(D, H, ng, d)) break;
    double dmax = 0.0, slope = 0.0;
    for (int a = 0; a < D; ++a) {
      if (fabs(d[a]) > dmax) dmax = fabs(d[a]);
      slope += g[a] * d[a];
    }
    double t = 1.0;
    if (dmax > 1e-6) {
      /* a long step: halve it until F decreases enough (Armijo) */
      for (int k = 0; k < 40; ++k) {
        double lt[3], Ft;
        for (int a = 0; a < D; ++a) lt[a] = l[a] + t * d[a];
        F_of(L, u, lt, &Ft, NULL, NULL);
        if (Ft <= F + 1e-4 * t * slope) break;
        t *= 0.5;
      }
    }
    for (int a = 0; a < D; ++a) l[a] += t * d[a];
    if (t * dmax <= 1e-12) {
      iters = it;
      break;
    }
  }
  if (iters < 0) {
    for (int i = 0; i < L->Q; ++i) feq[i] = NAN;
    return -1;
  }
  double Z = 0.0, p[QMAX];
  for (int i = 0; i < L->Q; ++i) {
    double lc = 0.0;
    for (int a = 0; a < D; ++a) lc += l[a] * L->c[i][a];
    p[i] = L->W[i] * exp(lc);
    Z += p[i];
  }
  for (int i = 0; i < L->Q; ++i) feq[i] = rho * (p[i] / Z);
  return iters;
}

/* Burg's entropy H(f) = -sum_i W_i ln(f_i / W_i): stationarity of the
 * Lagrangian gives W_i / f_i = m0 + m.c_i, i.e. f_i = W_i / (mu.a_i) with
 * a_i = (1, c_i) and mu = (m0, m).  mu maximises the concave dual
 *   g(mu) = sum_i W_i ln(mu.a_i) - mu.b,   b = (rho, rho u),
 * whose gradient sum_i W_i a_i / (mu.a_i) - b is the constraint residual
 * and whose Hessian is -sum_i W_i a_i a_i^T / (mu.a_i)^2.  Newton's method on
 * g from the rest state mu = (1/rho, 0), halving a step while it would make
 * some mu.a_i non-positive or fail to increase g (Armijo); it stops after a
 * step below 1e-12 (m0 is of order 1/rho).  Returns the iteration count, or
 * -1 (feq NaN) without convergence. */
static int burg_dual(const lat_t *L, const double *mu, const double *b, double *g,
                     double *grad, double H[4][4]) {
  const int n = L->D + 1;
  double v = 0.0, s[4] = {0.0, 0.0, 0.0, 0.0}, S[4][4] = {{0.0}};
  for (int i = 0; i < L->Q; ++i) {
    double a[4] = {1.0, L->c[i][0], L->c[i][1], L->c[i][2]};
    double d = 0.0;
    for (int k = 0; k < n; ++k) d += mu[k] * a[k];
    if (!(d > 0.0)) return -1;
    v += L->W[i] * log(d);
    for (int k = 0; k < n; ++k) {
      s[k] += L->W[i] * a[k] / d;
      for (int m = 0; m < n; ++m) S[k][m] += L->W[i] * a[k] * a[m] / (d * d);
    }
  }
  for (int k = 0; k < n; ++k) v -= mu[k] * b[k];
  *g = v;
  if (grad)
    for (int k = 0; k < n; ++k) {
      grad[k] = s[k] - b[k];
      for (int m = 0; m < n; ++m) H[k][m] = S[k][m];  /* -Hessian, positive definite */
    }
  return 0;
}

static int solve4(int n, double A[4][4], const double *r, double *x) {
  double M[4][5];
  for (int a = 0; a < n; ++a) {
    for (int b = 0; b < n; ++b) M[a][b] = A[a][b];
    M[a][n] = r[a];
  }
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int a = k + 1; a < n; ++a)
      if (fabs(M[a][k]) > fabs(M[piv][k])) piv = a;
    if (M[piv][k] == 0.0) return -1;
    for (int b = 0; b <= n; ++b) {
      double t = M[k][b];
      M[k][b] = M[piv][b];
      M[piv][b] = t;
    }
    for (int a = k + 1; a < n; ++a) {
      double f = M[a][k] / M[k][k];
      for (int b = k; b <= n; ++b) M[a][b] -= f * M[k][b];
    }
  }
  for (int a = n - 1; a >= 0; --a) {
    double v = M[a][n];
    for (int b = a + 1; b < n; ++b) v -= M[a][b] * x[b];
    x[a] = v / M[a][a];
  }
  return 0;
}

static int equilibrium_burg(const lat_t *L, double rho, const double *u, double *feq) {
  const int n = L->D + 1;
  double mu[4] = {1.0 / rho, 0.0, 0.0, 0.0}, b[4] = {rho, 0.0, 0.0, 0.0};
  for (int a = 0; a < L->D; ++a) b[a + 1] = rho * u[a];
  int iters = -1;
  for (int it = 1; it <= 80; ++it) {
    double g, grad[4], H[4][4], d[4];
    if (burg_dual(L, mu, b, &g, grad, H) || solve4(n, H, grad, d)) break;
    /* ascent direction d = (-Hessian)^-1 grad */
    double dmax = 0.0, slope = 0.0;
    for (int k = 0; k < n; ++k) {
      if (fabs(d[k]) > dmax) dmax = fabs(d[k]);
      slope += grad[k] * d[k];
    }
    double t = 1.0;
    for (int k = 0; k < 60; ++k) {
      double mt[4], gt;
      for (int m = 0; m < n; ++m) mt[m] = mu[m] + t * d[m];
      if (!burg_dual(L, mt, b, &gt, NULL, NULL) && (dmax <= 1e-6 || gt >= g + 1e-4 * t * slope))
        break;
      t *= 0.5;
    }
    for (int k = 0; k < n; ++k) mu[k] += t * d[k];
    if (t * dmax <= 1e-12) {
      iters = it;
      break;
    }
  }
  if (iters < 0) {
    for (int i = 0; i < L->Q; ++i) feq[i] = NAN;
    return -1;
  }
  for (int i = 0; i < L->Q; ++i) {
    double d = mu[0];
    for (int a = 0; a < L->D; ++a) d += mu[a + 1] * L->c[i][a];
    feq[i] = L->W[i] / d;
  }
  return iters;
}

/* f^eq: for the Boltzmann entropy by the closed product form where the
 * weights factorise, else by the minimiser; for Burg's entropy by its own
 * minimiser. */
static void equilibrium(const lat_t *L, double rho, const double *u, double *feq) {
  if (L->ent == ENT_BURG) (void)equilibrium_burg(L, rho, u, feq);
  else if (L->product) equilibrium_product(L, rho, u, feq);
  else (void)equilibrium_minimiser(L, rho, u, feq);
}

/* Polynomial (second-order) equilibrium of LBGK, the alpha = 2 special case
 * named after Eq. (4): W_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2). */
static void equilibrium_poly(const lat_t *L, double rho, const double *u,
                             double *feq) {
  double uu = 0.0;
  for (int a = 0; a < L->D; ++a) uu += u[a] * u[a];
  for (int i = 0; i < L->Q; ++i) {
    double cu = 0.0;
    for (int a = 0; a < L->D; ++a) cu += L->c[i][a] * u[a];
    feq[i] = L->W[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

/* ---- entropy --------------------------------------------------------------
 * Eq. (3) literally, with 0 ln 0 = 0; NaN for a negative population.  Burg:
 * -sum_i W_i ln(f_i / W_i), +inf at a zero population. */
static double entropy(const lat_t *L, const double *f) {
  double h = 0.0;
  for (int i = 0; i < L->Q; ++i) {
    if (f[i] < 0.0) return NAN;
    if (L->ent == ENT_BURG) {
      if (f[i] == 0.0) return INFINITY;
      h -= L->W[i] * log(f[i] / L->W[i]);
    } else if (f[i] > 0.0) {
      h += f[i] * log(f[i] / L->W[i]);
    }
  }
  return h;
}

/* Relative-entropy densities.  For an entropy H(f) = sum_i h_i(f_i) whose
 * equilibrium makes h_i'(f_i^eq) affine in (1, c_i), every g with the
 * moments of f^eq satisfies sum_i (g_i - f_i^eq) h_i'(f_i^eq) = 0, so
 *   H(g) - H(f^eq) = sum_i w_i psi(g_i / f_i^eq - 1)
 * exactly, without the cancellation of two O(rho) entropies:
 *   Boltzmann (Eq. (3)): w_i = f_i^eq, psi = phi, phi(y) = (1+y) ln(1+y) - y;
 *   Burg:                w_i = W_i,    psi = chi, chi(y) = y - ln(1+y).
 * phi(-1) = 1 is the 0 ln 0 = 0 limit (a population that is exactly zero);
 * chi(-1) = +inf.  At alpha = alpha_max the component that defines alpha_max
 * has f*_k = 0 exactly, but the rounded y_k = (1 - alpha_max) x_k can land an
 * ulp below -1; every y <= -1 met here is that rounding, so it is read as
 * f*_k = 0. */
static double phi(double y) {
  if (y <= -1.0) return 1.0;
  return (1.0 + y) * log1p(y) - y;
}

static double chi(double y) {
  if (y <= -1.0) return INFINITY;
  return y - log1p(y);
}

static double psi(const lat_t *L, double y) {
  return L->ent == ENT_BURG ? chi(y) : phi(y);
}

/* psi'(y): ln(1 + y) (Boltzmann), y / (1 + y) (Burg). */
static double dpsi(const lat_t *L, double y) {
  if (L->ent == ENT_BURG) return y <= -1.0 ? -INFINITY : y / (1.0 + y);
  return log1p(y < -1.0 ? -1.0 : y);
}

static double weight_of(const lat_t *L, const double *feq, int i) {
  return L->ent == ENT_BURG ? L->W[i] : feq[i];
}

/* x_i = f_i / f_i^eq - 1, formed as (f_i - f_i^eq) / f_i^eq. */
static void deviations(const lat_t *L, const double *f, const double *feq,
                       double *x) {
  for (int i = 0; i < L->Q; ++i) x[i] = (f[i] - feq[i]) / feq[i];
}

/* f*(alpha) = f + alpha (f^eq - f) = f^eq (1 + (1 - alpha) x), so
 *   G(alpha) := H(f*(alpha)) - H(f)
 *             = sum_i w_i [psi((1 - alpha) x_i) - psi(x_i)].            */
static double G_of(const lat_t *L, const double *feq, const double *x,
                   double alpha) {
  double g = 0.0;
  for (int i = 0; i < L->Q; ++i)
    g += weight_of(L, feq, i) * (psi(L, (1.0 - alpha) * x[i]) - psi(L, x[i]));
  return g;
}

/* G'(alpha) = -sum_i w_i x_i psi'((1 - alpha) x_i). */
static double dG_of(const lat_t *L, const double *feq, const double *x,
                    double alpha) {
  double g = 0.0;
  for (int i = 0; i < L->Q; ++i)
    g -= weight_of(L, feq, i) * x[i] * dpsi(L, (1.0 - alpha) * x[i]);
  return g;
}

/* H(f*(alpha)) - H(f^eq) = sum_i w_i psi((1 - alpha) x_i)  (Eq. (9) denominator) */
static double Hrel_of(const lat_t *L, const double *feq, const double *x,
                      double alpha) {
  double h = 0.0;
  for (int i = 0; i < L->Q; ++i) h += weight_of(L, feq, i) * psi(L, (1.0 - alpha) * x[i]);
  return h;
}

/* alpha_max = min over {i : f_i^eq < f_i} of f_i / (f_i - f_i^eq)
 * (definition after Eq. (7)); +inf for an empty set. */
static double alpha_max_of(const lat_t *L, const double *f, const double *feq) {
  double am = INFINITY;
  for (int i = 0; i < L->Q; ++i)
    if (feq[i] < f[i]) {
      double v = f[i] / (f[i] - feq[i]);
      if (v < am) am = v;
    }
  return am;
}

/* Bisection on [1, alpha_max] for the nontrivial root of Eq. (4), stopping at
 * the first midpoint with -tol <= G <= 0 (the criterion of the double-shear
 * comparison).  G(1) = -D <= 0; if G(alpha_max) <= 0 there is no root in the
 * admissible range and alpha_max is returned.  Returns the last point with
 * G <= 0 if the cap is reached. */
static double solve_bisect(const lat_t *L, const double *feq, const double *x,
                           double amax, double tol, int maxit, int *iters) {
  double lo = 1.0, hi = amax;
  *iters = 0;
  if (G_of(L, feq, x, hi) <= 0.0) return hi;
  for (int k = 1; k <= maxit; ++k) {
    double mid = 0.5 * (lo + hi);
    double g = G_of(L, feq, x, mid);
    *iters = k;
    if (g <= 0.0 && g >= -tol) return mid;
    if (g > 0.0) hi = mid;
    else lo = mid;
  }
  return lo;
}

/* Bracketed Newton iteration for the root of Eq. (4) on [1, alpha_max],
 * started at alpha_* (at the bracket midpoint when alpha_* = alpha_max, where
 * G' is unbounded).  A step that leaves the bracket is replaced by the
 * midpoint.  The iteration stops
 *   - when |G(a)| is at the rounding level of its own evaluation,
 *     eps sum_i w_i (|x_i| + |(1 - a) x_i|) (each term w_i phi(y) is formed
 *     from O(|y|) parts): a is then a root to the accuracy G can be known
 *     with, and further steps would only follow rounding noise; or
 *   - at a step (Newton or midpoint) below 1e-13 alpha.
 * A Newton step below that size that rounds onto (or past) the end of the
 * bracket is a converged step too, and stops there instead of restarting
 * bisection.
 *
 * G is convex with G(1) = -D <= 0 and G' > 0 on (1, alpha_max], so G < 0 on
 * [1, root) and G > 0 beyond it, and a Newton step from a point with G < 0
 * lands at or beyond the root.  Whether the root lies inside [1, alpha_max]
 * (G(alpha_max) > 0) is therefore only asked when a step leaves the bracket
 * while its upper end is still alpha_max: if G(alpha_max) <= 0 the root lies
 * beyond and alpha_max is returned.  The result is the root to the rounding
 * of G; it can sit on either side of it. */
static double solve_newton(const lat_t *L, const double *feq, const double *x,
                           double amax, double astar, int maxit, int *iters) {
  double lo = 1.0, hi = amax;
  int hi_positive = 0; /* G(hi) > 0 known */
  double sx = 0.0;     /* sum_i w_i |x_i| */
  for (int i = 0; i < L->Q; ++i) sx += weight_of(L, feq, i) * fabs(x[i]);
  double a = (astar < amax) ? astar : 0.5 * (lo + hi);
  *iters = 0;
  for (int k = 1; k <= maxit; ++k) {
    double g = G_of(L, feq, x, a);
    *iters = k;
    if (fabs(g) <= DBL_EPSILON * (1.0 + fabs(1.0 - a)) * sx) return a;
    if (g > 0.0) {
      hi = a;
      hi_positive = 1;
    } else {
      lo = a;
    }
    double an = a - g / dG_of(L, feq, x, a);
    if (!(an > lo && an < hi)) {
      /* a converged step that rounds onto (or just past) the bracket end */
      if (fabs(an - a) <= 1e-13 * a) return (an < lo) ? lo : (an > hi) ? hi : an;
      if (!hi_positive) {
        if (G_of(L, feq, x, hi) <= 0.0) return hi;
        hi_positive = 1;
      }
      an = 0.5 * (lo + hi);
    }
    if (fabs(an - a) <= 1e-13 * a) return an;
    a = an;
  }
  return a;
}

/* The per-site choice of alpha. */
static double choose_alpha(const lat_t *L, const orc_params *p, const double *f,
                           const double *feq, double rho, orc_site_info *info) {
  double x[QMAX] = {0.0};
  deviations(L, f, feq, x);
  double amax = alpha_max_of(L, f, feq);
  double astar = (amax < 2.0) ? amax : 2.0;        /* Eq. (8) */
  double Dv = Hrel_of(L, feq, x, 0.0);              /* H(f) - H(f^eq) */
  int guard = (Dv <= GUARD_REL * rho) || isinf(amax);
  /* Burg's entropy is infinite at the zero population of f*(alpha_max) */
  const int inf_star = (L->ent == ENT_BURG) && astar == amax;
  double Gs = guard ? 0.0 : inf_star ? INFINITY : G_of(L, feq, x, astar); /* H(f*(a_*)) - H(f) */
  double alpha = astar;
  int iters = 0;

  if (!guard) {
    if (p->mode == ORC_ALPHA_CLOSED) {
      if (Gs > 0.0) {
        /* Eq. (9); both differences infinite: their ratio's limit is 1 */
        double ratio = inf_star ? 1.0 : Gs / Hrel_of(L, feq, x, astar); /* den: H(f*(a_*)) - H(f^eq) */
        alpha = astar + ratio * (1.0 - astar);
        if (alpha < 1.0) alpha = 1.0;
        if (alpha > astar) alpha = astar;
        iters = 1;
      }
    } else if (p->mode == ORC_ALPHA_SECANT) {
      if (Gs > 0.0) {
        /* alpha^(k+1) = a_* + G(a_*) / (G(a_*) - G(alpha^(k))) (alpha^(k) - a_*),
         * alpha^(0) = 1 (G(1) = H(f^eq) - H(f)) so that the first iterate
         * is Eq. (9). */
        double a = 1.0;
        /* G(a_*) infinite: every iterate stays at alpha^(0) = 1 */
        for (int k = 0; k < (inf_star ? 0 : p->secant_iters); ++k) {
          double Ga = G_of(L, feq, x, a);
          double an = astar + Gs / (Gs - Ga) * (a - astar);
          iters = k + 1;
          if (an == a) break;
          a = an;
        }
        if (inf_star) iters = 1;
        if (a < 1.0) a = 1.0;
        if (a > astar) a = astar;
        alpha = a;
      }
    } else if (p->mode == ORC_ALPHA_BISECT) {
      alpha = solve_bisect(L, feq, x, amax, p->root_tol, p->root_max_iter, &iters);
    } else if (p->mode == ORC_ALPHA_NEWTON) {
      alpha = solve_newton(L, feq, x, amax, astar, p->root_max_iter, &iters);
    }
  }
  if (info) {
    info->alpha = alpha;
    info->alpha_max = amax;
    info->alpha_star = astar;
    info->G_star = Gs;
    info->D = Dv;
    info->guard = guard;
    info->accepted2 = (astar == 2.0) && (guard || Gs <= 0.0);
    info->iters = iters;
  }
  return alpha;
}

static int check_params(const orc_params *p, lat_t *L) {
  if (!p) return -1;
  if (make_lattice(p->lattice, L)) return -1;
  if (p->entropy != ENT_BOLTZMANN && p->entropy != ENT_BURG) return -1;
  L->ent = p->entropy;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return -1;
  if (L->D == 1 && (p->ny != 1 || p->nz != 1)) return -1;
  if (L->D == 2 && p->nz != 1) return -1;
  if (!(p->beta > 0.0 && p->beta < 1.0)) return -1;
  if (p->mode < ORC_ALPHA_CLOSED || p->mode > ORC_ALPHA_SECANT) return -1;
  if (p->mode == ORC_ALPHA_SECANT && p->secant_iters < 1) return -1;
  if ((p->mode == ORC_ALPHA_NEWTON || p->mode == ORC_ALPHA_BISECT) &&
      p->root_max_iter < 1)
    return -1;
  return 0;
}

/* One site: moments, equilibrium, alpha, then Eq. (1):
 *   f~_i = f_i + alpha beta (f_i^eq - f_i). */
static void collide(const lat_t *L, const orc_params *p, const double *f,
                    double *ft, orc_site_info *info) {
  double rho, u[3], feq[QMAX], alpha;
  moments(L, f, &rho, u);
  if (p->mode == ORC_ALPHA_BGK) {
    equilibrium_poly(L, rho, u, feq);
    alpha = 2.0;
    if (info) {
      double fe[QMAX];
      equilibrium(L, rho, u, fe);
      choose_alpha(L, p, f, fe, rho, info); /* diagnostics only */
      info->alpha = 2.0;
      info->iters = 0;
    }
  } else {
    equilibrium(L, rho, u, feq);
    alpha = choose_alpha(L, p, f, feq, rho, info);
  }
  for (int i = 0; i < L->Q; ++i) ft[i] = f[i] + alpha * p->beta * (feq[i] - f[i]);
  if (info) {
    info->rho = rho;
    for (int a = 0; a < 3; ++a) info->u[a] = u[a];
  }
}

/* ---- exported single-state functions ------------------------------------ */
int orc_lattice(int32_t lattice, int32_t *Q, int32_t *c, double *W) {
  lat_t L;
  if (make_model(lattice, &L)) return -1;
  if (Q) *Q = L.Q;
  for (int i = 0; i < L.Q; ++i) {
    if (c)
      for (int a = 0; a < 3; ++a) c[3 * i + a] = L.c[i][a];
    if (W) W[i] = L.W[i];
  }
  return 0;
}

int orc_equilibrium(int32_t lattice, double rho, const double *u, double *feq) {
  lat_t L;
  if (make_model(lattice, &L) || !(rho > 0.0) || !u_admissible(&L, u)) return -1;
  double v[QMAX];
  equilibrium(&L, rho, u, v);
  for (int i = 0; i < L.Q; ++i) {
    if (isnan(v[i])) return -1;
    feq[i] = v[i];
  }
  return 0;
}

int orc_equilibrium_minimiser(int32_t lattice, double rho, const double *u,
                              double *feq, int32_t *iters) {
  lat_t L;
  if (make_model(lattice, &L) || !(rho > 0.0) || !u_admissible(&L, u)) return -1;
  int it = L.ent == ENT_BURG ? equilibrium_burg(&L, rho, u, feq)
                             : equilibrium_minimiser(&L, rho, u, feq);
  if (iters) *iters = it;
  return it < 0 ? -1 : 0;
}

int orc_equilibrium_poly(int32_t lattice, double rho, const double *u, double *feq) {
  lat_t L;
  if (make_model(lattice, &L)) return -1;
  equilibrium_poly(&L, rho, u, feq);
  return 0;
}

int orc_moments_site(int32_t lattice, const double *f, double *rho, double *u) {
  lat_t L;
  if (make_model(lattice, &L)) return -1;
  moments(&L, f, rho, u);
  return 0;
}

double orc_entropy(int32_t lattice, const double *f) {
  lat_t L;
  if (make_model(lattice, &L)) return NAN;
  return entropy(&L, f);
}

double orc_entropy_rel(int32_t lattice, const double *g, const double *feq) {
  lat_t L;
  if (make_model(lattice, &L)) return NAN;
  double x[QMAX];
  deviations(&L, g, feq, x);
  return Hrel_of(&L, feq, x, 0.0);
}

double orc_alpha_max(int32_t lattice, const double *f, const double *feq) {
  lat_t L;
  if (make_model(lattice, &L)) return NAN;
  return alpha_max_of(&L, f, feq);
}

double orc_G(int32_t lattice, const double *f, double alpha) {
  lat_t L;
  if (make_model(lattice, &L)) return NAN;
  double rho, u[3], feq[QMAX], x[QMAX];
  moments(&L, f, &rho, u);
  equilibrium(&L, rho, u, feq);
  deviations(&L, f, feq, x);
  return G_of(&L, feq, x, alpha);
}

int orc_alpha(const orc_params *p, const double *f, orc_site_info *info) {
  lat_t L;
  if (check_params(p, &L) || !info) return -1;
  double ft[QMAX];
  collide(&L, p, f, ft, info);
  return 0;
}

int orc_collide_site(const orc_params *p, const double *f, double *ftilde,
                     orc_site_info *info) {
  lat_t L;
  if (check_params(p, &L)) return -1;
  collide(&L, p, f, ftilde, info);
  return 0;
}

/* ---- whole-box functions ------------------------------------------------- */
static int64_t nsites(const orc_params *p) {
  return (int64_t)p->nx * p->ny * p->nz;
}

int orc_init(const orc_params *p, const double *rho0, const double *u0,
             double *f) {
  lat_t L;
  if (check_params(p, &L)) return -1;
  int64_t N = nsites(p);
  for (int64_t s = 0; s < N; ++s) {
    double u[3] = {0.0, 0.0, 0.0}, feq[QMAX];
    if (!(rho0[s] > 0.0)) return -2;
    for (int a = 0; a < L.D; ++a) u[a] = u0[a * N + s];
    if (!u_admissible(&L, u)) return -2;
    equilibrium(&L, rho0[s], u, feq);
    if (isnan(feq[0])) return -2;
    for (int i = 0; i < L.Q; ++i) f[i * N + s] = feq[i];
  }
  return 0;
}

int orc_moments(const orc_params *p, const double *f, double *rho, double *u) {
  lat_t L;
  if (check_params(p, &L)) return -1;
  int64_t N = nsites(p);
  for (int64_t s = 0; s < N; ++s) {
    double fs[QMAX], r, v[3];
    for (int i = 0; i < L.Q; ++i) fs[i] = f[i * N + s];
    moments(&L, fs, &r, v);
    rho[s] = r;
    for (int a = 0; a < L.D; ++a) u[a * N + s] = v[a];
  }
  return 0;
}

static int wrap(int v, int n) { return (v < 0) ? v + n : (v >= n) ? v - n : v; }

/* One time step on the periodic box: collide every site (Eq. (1)), then
 * stream f_i(x + c_i, t+1) = f~_i(x, t) (Eq. (5b)). */
int orc_step(const orc_params *p, const double *f, double *fnext,
             double *alpha, orc_diag *diag) {
  lat_t L;
  if (check_params(p, &L) || f == fnext) return -1;
  const int nx = p->nx, ny = p->ny, nz = p->nz;
  const int64_t N = nsites(p);
  orc_site_info *info = NULL;
  double *hsite = NULL;
  int64_t *nneg = NULL;
  if (diag) {
    info = (orc_site_info *)malloc(sizeof(orc_site_info) * (size_t)N);
    hsite = (double *)malloc(sizeof(double) * (size_t)N);
    nneg = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    if (!info || !hsite || !nneg) {
      free(info); free(hsite); free(nneg);
      return -3;
    }
  }
  int nth = p->nthreads > 0 ? p->nthreads : 1;
  (void)nth;
#pragma omp parallel for schedule(static) num_threads(nth)
  for (int64_t s = 0; s < N; ++s) {
    double fs[QMAX], ft[QMAX];
    orc_site_info si;
    for (int i = 0; i < L.Q; ++i) fs[i] = f[i * N + s];
    collide(&L, p, fs, ft, (diag || alpha) ? &si : NULL);
    int x = (int)(s % nx), y = (int)((s / nx) % ny), z = (int)(s / ((int64_t)nx * ny));
    for (int i = 0; i < L.Q; ++i) {
      int xd = wrap(x + L.c[i][0], nx), yd = wrap(y + L.c[i][1], ny),
          zd = wrap(z + L.c[i][2], nz);
      fnext[i * N + xd + (int64_t)nx * (yd + (int64_t)ny * zd)] = ft[i];
    }
    if (alpha) alpha[s] = si.alpha;
    if (diag) {
      info[s] = si;
      hsite[s] = entropy(&L, fs);
      int64_t neg = 0;
      for (int i = 0; i < L.Q; ++i) neg += (ft[i] < 0.0);
      nneg[s] = neg;
    }
  }
  if (diag) {
    memset(diag, 0, sizeof(*diag));
    diag->n_sites = N;
    diag->alpha_min = INFINITY;
    diag->alpha_max = -INFINITY;
    for (int64_t s = 0; s < N; ++s) {
      const orc_site_info *si = &info[s];
      diag->n_accept2 += si->accepted2;
      diag->n_alphastar_lt2 += (si->alpha_star < 2.0);
      diag->n_alpha_lt2 += (si->alpha < 2.0);
      diag->n_guard += si->guard;
      diag->n_negative += nneg[s];
      diag->total_iters += si->iters;
      if (si->alpha < diag->alpha_min) diag->alpha_min = si->alpha;
      if (si->alpha > diag->alpha_max) diag->alpha_max = si->alpha;
      diag->sum_rho += si->rho;
      for (int a = 0; a < L.D; ++a) diag->sum_j[a] += si->rho * si->u[a];
      diag->sum_H += hsite[s];
    }
    free(info);
    free(hsite);
    free(nneg);
  }
  return 0;
}
