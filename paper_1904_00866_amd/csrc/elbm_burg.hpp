// elbm_burg.hpp -- the equilibrium of Burg's entropy
// H(f) = -sum_i W_i ln(f_i / W_i) on a lattice L (Lattice<D> or LatticeQ19):
// f^eq_i = W_i / d_i with d_i = mu[0] + sum_a c_ia mu[a + 1], where the D + 1
// multipliers mu solve the mass and momentum constraints (stationarity of
// the Lagrangian makes h'(f^eq_i) = -W_i / f^eq_i affine in (1, c_i)).
#pragma once

#include "elbm_q19.hpp"
#include "elbm_site.hpp"

namespace elbm {

// Direction index of the digits (dx, dy, dz) on lattice L, or -1 if L has
// no such direction.
template <class L>
struct Dirs;
template <int D>
struct Dirs<Lattice<D>> {
  static constexpr int index(int dx, int dy, int dz) {
    return ((D < 2 && dy != 0) || (D < 3 && dz != 0)) ? -1 : dx + 3 * dy + 9 * dz;
  }
};
template <>
struct Dirs<LatticeQ19> {
  static constexpr int index(int dx, int dy, int dz) {
    return (dx != 0 && dy != 0 && dz != 0)
               ? -1
               : (dx + 3 * dy + 9 * dz) - 2 * ((dx + 3 * dy + 9 * dz) >= 13) -
                     2 * ((dx + 3 * dy + 9 * dz) >= 18) - 2 * ((dx + 3 * dy + 9 * dz) >= 22);
  }
};

// Index of the direction -c_i (digits 1 and 2 swapped).
template <class L>
constexpr int opposite(int i) {
  return Dirs<L>::index((3 - L::dg(i, 0)) % 3, (3 - L::dg(i, 1)) % 3, (3 - L::dg(i, 2)) % 3);
}

template <class L>
__device__ __forceinline__ double burg_den(const double (&mu)[4], int i) {
  double v = mu[0];
#pragma unroll
  for (int a = 0; a < L::Dim; ++a) {
    const int c = L::c(i, a);
    if (c > 0) v += mu[a + 1];
    else if (c < 0) v -= mu[a + 1];
  }
  return v;
}

// Solve S z = r for a symmetric positive definite S of order N <= 4 (only
// S[k][m], k <= m, is read) by an LDL^T factorisation.
template <int N>
__device__ __forceinline__ void ldl_solve(const double (&S)[4][4], const double (&r)[4],
                                          double (&z)[4]) {
  double Lm[4][4], Dg[4], iD[4];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double dj = S[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) dj -= Lm[j][k] * Lm[j][k] * Dg[k];
    Dg[j] = dj;
    iD[j] = rcp_n<double>(dj);
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      double v = S[j][i];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= Lm[i][k] * Lm[j][k] * Dg[k];
      Lm[i][j] = v * iD[j];
    }
  }
  double y[4];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double v = r[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= Lm[i][k] * y[k];
    y[i] = v;
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    double v = y[i] * iD[i];
#pragma unroll
    for (int k = i + 1; k < N; ++k) v -= Lm[k][i] * z[k];
    z[i] = v;
  }
}

// Burg equilibrium: mu maximises the concave dual
//   g(mu) = sum_i W_i ln(d_i) - mu.b,   b = (rho, rho u),
// whose gradient F(mu) = sum_i W_i a_i / d_i - b (a_i = (1, c_i)) is the
// constraint residual and whose Hessian is -S, S = sum_i W_i a_i a_i^T / d_i^2.
// Newton's method mu <- mu + t S^-1 F from the third-order solution
// mu = ((1 + 3 u.u) / rho, -3 u (1 - 3 u.u) / rho) (expanding the constraints
// with the lattices' isotropic moments up to fourth order), its velocity part
// scaled down where that would leave some d_i below mu_0 / 2 (the constraint
// equations have other roots, with negative populations, outside d > 0).
// t is halved while a step would make some d_i non-positive or, for a step
// above 5 % of mu_0, fail to increase g (Armijo); a step whose (D+1) max|z|
// is below min_i d_i keeps every d_i positive, and small steps near the
// solution take t = 1 with neither check.  Stops after a step below 1e-9 mu_0 (quadratic convergence
// leaves an error of order its square), at most 32 iterations.
template <class L>
__device__ __forceinline__ double burg_dual(const double (&mu)[4], double rho, const double (&u)[3]) {
  double v = -mu[0] * rho;
#pragma unroll
  for (int a = 0; a < L::Dim; ++a) v -= mu[a + 1] * rho * u[a];
#pragma unroll
  for (int i = 0; i < L::Q; ++i) v += L::W(i) * log(burg_den<L>(mu, i));
  return v;
}

template <class L>
__device__ __forceinline__ void burg_multipliers(double rho, double irho, const double (&u)[3],
                                                 double (&mu)[4]) {
  constexpr int D = L::Dim, N = D + 1, Q = L::Q;
  double uu = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) uu += u[a] * u[a];
  mu[0] = (1.0 + 3.0 * uu) * irho;
  const double sv = -3.0 * (1.0 - 3.0 * uu) * irho;
#pragma unroll
  for (int a = 0; a < 3; ++a) mu[a + 1] = a < D ? sv * u[a] : 0.0;
  double dmin = INFINITY;
#pragma unroll
  for (int i = 0; i < Q; ++i) dmin = fmin(dmin, burg_den<L>(mu, i));
  if (dmin < 0.5 * mu[0]) {
    const double sc = 0.5 * mu[0] / (mu[0] - dmin);
#pragma unroll
    for (int a = 1; a < 4; ++a) mu[a] *= sc;
  }
  bool done = false;
  for (int it = 0; it < 32; ++it) {
    if (!done) {
      double F[4] = {0.0, 0.0, 0.0, 0.0}, Sm[4][4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int m = 0; m < 4; ++m) Sm[k][m] = 0.0;
      // Directions in pairs (c, -c) with W_-c = W_c: d_+- = mu_0 +- v,
      // v = sum_a c_a mu_a; one reciprocal of d_+ d_- gives both 1/d_+-, and
      // the pair adds W (r_+ + r_-) a a^T-even and W (r_+ - r_-) odd terms.
      double dlo = INFINITY;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int io = opposite<L>(i);
        if (io < i) continue;  // the pair was taken at io
        double v = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const int c = L::c(i, a);
          if (c > 0) v += mu[a + 1];
          else if (c < 0) v -= mu[a + 1];
        }
        const double W = L::W(i);
        if (io == i) {  // the rest direction: a = (1, 0, ...)
          const double r = rcp_n<double>(mu[0]);
          dlo = fmin(dlo, mu[0]);
          F[0] += W * r;
          Sm[0][0] += W * r * r;
          continue;
        }
        const double dp = mu[0] + v, dm = mu[0] - v;
        dlo = fmin(dlo, fmin(dp, dm));
        const double rp2 = rcp_n<double>(dp * dm);
        const double rp = dm * rp2, rm = dp * rp2;
        const double ev = W * (rp + rm), od = W * (rp - rm);
        const double ev2 = W * fma(rp, rp, rm * rm), od2 = W * ((rp + rm) * (rp - rm));
        F[0] += ev;
        Sm[0][0] += ev2;
#pragma unroll
        for (int k = 1; k < N; ++k) {
          const int ck = L::c(i, k - 1);
          if (ck == 0) continue;
          F[k] += ck > 0 ? od : -od;
          Sm[0][k] += ck > 0 ? od2 : -od2;
#pragma unroll
          for (int m = k; m < N; ++m) {
            const int cm = L::c(i, m - 1);
            if (cm == 0) continue;
            Sm[k][m] += ck * cm > 0 ? ev2 : -ev2;
          }
        }
      }
      F[0] -= rho;
#pragma unroll
      for (int a = 0; a < D; ++a) F[a + 1] -= rho * u[a];
      double z[4];
      ldl_solve<N>(Sm, F, z);
      double zmax = 0.0, slope = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        zmax = fmax(zmax, fabs(z[k]));
        slope += F[k] * z[k];
      }
      const bool big = zmax > 0.05 * mu[0];
      const double g0 = big ? burg_dual<L>(mu, rho, u) : 0.0;
      double t = 1.0;
      // |change of d_i| <= (D + 1) max|z|: below min d_i no d_i can turn
      const bool safe = !big && double(N) * zmax < dlo;
      for (int h = 0; h < (safe ? 0 : 12); ++h) {
        double mt[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) mt[k] = k < N ? mu[k] + t * z[k] : 0.0;
        bool ok = true;
#pragma unroll
        for (int i = 0; i < Q; ++i) ok = ok && burg_den<L>(mt, i) > 0.0;
        if (ok && big) ok = burg_dual<L>(mt, rho, u) >= g0 + 1e-4 * t * slope;
        if (ok) break;
        t *= 0.5;
      }
#pragma unroll
      for (int k = 0; k < N; ++k) mu[k] += t * z[k];
      done = !(t * zmax > 1e-9 * mu[0]);
    }
    if (__all(done)) break;
  }
}

}  // namespace elbm
