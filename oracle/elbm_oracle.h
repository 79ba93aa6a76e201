/*
 * elbm_oracle.h -- plain FP64 CPU oracle of the entropic lattice Boltzmann
 * step with the closed-form relaxation parameter (Zhao & Yong,
 * "Relaxation-rate formula for the entropic lattice Boltzmann method").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this library: only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no source with the HIP
 * library; the only thing the two agree on is the interface convention
 * below (direction order, SoA layout), which both write out independently.
 *
 * Conventions (the same ones the C-ABI library documents):
 *   - lattice units, delta_x = delta_t = 1, c_s^2 = 1/3;
 *   - lattice codes 1, 2, 3: the tensor-product lattices D1Q3, D2Q9, D3Q27,
 *     Q = 3^D, c_i in {-1,0,1}^D with the index
 *     i = d(c_x) + 3 d(c_y) + 9 d(c_z), d(0)=0, d(+1)=1, d(-1)=2, and
 *     weights W_i = prod_a w(c_ia), w(0)=2/3, w(+-1)=1/6
 *     (D1Q3, D2Q9: 4/9,1/9,1/36, D3Q27: 8/27,2/27,1/54,1/216);
 *   - lattice code 19: D3Q19, the D3Q27 directions with at most two nonzero
 *     components in the order of their D3Q27 index, W = 1/3 (rest),
 *     1/18 (|c|^2 = 1), 1/36 (|c|^2 = 2);
 *   - entropy: 0 the Boltzmann entropy of Eq. (3), 1 Burg's entropy
 *     H(f) = -sum_i W_i ln(f_i / W_i) (the paper's formula holds for any
 *     convex entropy); single-state functions take a model code, the lattice
 *     code + 256 x entropy;
 *   - populations are SoA: f[i*N + s], s = x + nx*(y + ny*z), x fastest;
 *     velocities are SoA: u[a*N + s].
 *
 * Everything is double precision, built with -ffp-contract=off and no
 * fast-math so that every operation rounds exactly once as written.
 * Functions return 0 on success and a negative number on invalid input.
 */
#ifndef ELBM_ORACLE_H
#define ELBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_ALPHA_CLOSED = 0, /* Eq. (8) + acceptance test + Eq. (9)              */
  ORC_ALPHA_NEWTON = 1, /* Newton root of the entropy balance Eq. (4)       */
  ORC_ALPHA_BISECT = 2, /* bisection root of Eq. (4), stop window as in E2  */
  ORC_ALPHA_BGK = 3,    /* alpha = 2 with the polynomial equilibrium (LBGK) */
  ORC_ALPHA_SECANT = 4  /* modified secant iteration of the closing remark  */
};

typedef struct {
  int32_t lattice;      /* lattice code: 1, 2, 3 or 19                        */
  int32_t nx, ny, nz;   /* periodic box; ny = 1 for D = 1, nz = 1 for D <= 2  */
  double beta;          /* Eq. (2), in (0,1)                                  */
  int32_t mode;         /* ORC_ALPHA_*                                        */
  int32_t secant_iters; /* iterations of the modified secant (>= 1)           */
  double root_tol;      /* bisection window -tol <= G <= 0 (paper: 1e-13)     */
  int32_t root_max_iter;/* cap on root-solver iterations                      */
  int32_t nthreads;     /* OpenMP threads for the site loop (1 = serial)      */
  int32_t entropy;      /* 0 Boltzmann (Eq. (3)), 1 Burg                      */
} orc_params;

/* Per-site record of how alpha was chosen. */
typedef struct {
  double rho, u[3];
  double alpha;
  double alpha_max;     /* +inf when no i has f_i^eq < f_i                   */
  double alpha_star;    /* Eq. (8)                                           */
  double G_star;        /* H(f*(alpha_*)) - H(f)                             */
  double D;             /* H(f) - H(f^eq) >= 0                               */
  int32_t accepted2;    /* alpha_* = 2 and H(f*(2)) <= H(f)                  */
  int32_t guard;        /* f^eq = f to rounding: alpha := alpha_*            */
  int32_t iters;        /* root-solver / secant iterations used              */
} orc_site_info;

/* Domain diagnostics of one step (pre-collision state f(x,t)). */
typedef struct {
  int64_t n_sites;
  int64_t n_accept2;      /* sites with H(f*(2)) <= H(f)  (Fig. 5 count)     */
  int64_t n_alphastar_lt2;/* sites with alpha_max < 2                        */
  int64_t n_alpha_lt2;    /* sites with alpha < 2                            */
  int64_t n_guard;        /* sites treated as f = f^eq                        */
  int64_t n_negative;     /* post-collision populations < 0                  */
  int64_t total_iters;    /* summed root-solver iterations                   */
  double alpha_min, alpha_max;
  double sum_rho, sum_j[3];
  double sum_H;           /* sum_x H(f(x,t)), Eq. (3) summed as in Eq. (6)   */
} orc_diag;

/* ---- lattice and single-state functions -------------------------------- */
/* The first argument is a model code (lattice code + 256 x entropy); u has
 * 3 entries (unused ones 0). */
int orc_lattice(int32_t lattice, int32_t *Q, int32_t *c /* Q*3 */, double *W);
/* f^eq: the closed product form (codes 1-3) or the minimiser (code 19);
 * -1 outside the domain (rho <= 0, u outside the velocities' hull). */
int orc_equilibrium(int32_t lattice, double rho, const double *u, double *feq);
/* f^eq by Newton's method on the Lagrange multipliers, for any lattice and
 * either entropy; *iters = Newton iterations. */
int orc_equilibrium_minimiser(int32_t lattice, double rho, const double *u,
                              double *feq, int32_t *iters);
int orc_equilibrium_poly(int32_t lattice, double rho, const double *u, double *feq);
int orc_moments_site(int32_t lattice, const double *f, double *rho, double *u);
double orc_entropy(int32_t lattice, const double *f);                /* Eq. (3) */
double orc_entropy_rel(int32_t lattice, const double *g, const double *feq);
double orc_alpha_max(int32_t lattice, const double *f, const double *feq);
double orc_G(int32_t lattice, const double *f, double alpha);        /* H(f*)-H(f) */
int orc_alpha(const orc_params *p, const double *f, orc_site_info *info);
int orc_collide_site(const orc_params *p, const double *f, double *ftilde,
                     orc_site_info *info);

/* ---- whole-box functions (periodic) ------------------------------------ */
int orc_init(const orc_params *p, const double *rho0, const double *u0,
             double *f);
int orc_moments(const orc_params *p, const double *f, double *rho, double *u);
int orc_step(const orc_params *p, const double *f, double *fnext,
             double *alpha /* N or NULL */, orc_diag *diag /* or NULL */);

#ifdef __cplusplus
}
#endif
#endif
