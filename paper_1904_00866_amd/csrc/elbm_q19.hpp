// elbm_q19.hpp -- the D3Q19 lattice and its entropic equilibrium (used by
// the D3Q19 step kernel and the auxiliary kernels).
#pragma once

#include "elbm_site.hpp"

namespace elbm {

// D3Q19: the D3Q27 directions with at most two nonzero components (the
// eight corners c in {+-1}^3 dropped), in the order of their D3Q27 index,
// with weights 1/3 (rest), 1/18 (|c|^2 = 1) and 1/36 (|c|^2 = 2); c_s^2 = 1/3.
// The weights do not factorise per axis.
struct LatticeQ19 {
  static constexpr int Dim = 3;
  static constexpr int Q = 19;
  // D3Q27 index of direction i (skips 13, 14, 16, 17, 22, 23, 25, 26); an
  // arithmetic form, so that a run-time i needs no table
  __host__ __device__ static constexpr int q27(int i) {
    return i + 2 * (i >= 13) + 2 * (i >= 14) + 2 * (i >= 18);
  }
  __host__ __device__ static constexpr int dg(int i, int a) { return digit(q27(i), a); }
  __host__ __device__ static constexpr int c(int i, int a) { return cval(dg(i, a)); }
  __host__ __device__ static constexpr int nnz(int i) {
    return (dg(i, 0) != 0) + (dg(i, 1) != 0) + (dg(i, 2) != 0);
  }
  __host__ __device__ static constexpr double W(int i) {
    return nnz(i) == 0 ? 1.0 / 3.0 : nnz(i) == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
  }
  __host__ __device__ static constexpr double invW(int i) {
    return nnz(i) == 0 ? 3.0 : nnz(i) == 1 ? 18.0 : 36.0;
  }
};

// D3Q19 equilibrium.  Stationarity again gives f_i^eq = rho W_i exp(l.c_i) / Z
// with Z(l) = sum_i W_i exp(l.c_i), but without the per-axis factorisation
// the multipliers l solve the momentum constraint m(l) = u,
// m(l) = sum_i c_i W_i exp(l.c_i) / Z, by Newton's method.  With
// ch_a = cosh l_a, sh_a = sinh l_a and the D3Q19 weights the sums are short:
//   9 Z = 3 + T + S2,           T = sum_a ch_a,  S2 = sum_{a<b} ch_a ch_b,
//   9 dZ/dl_a = sh_a P_a,       P_a = 1 + T - ch_a,
//   9 d2Z/dl_a^2 = ch_a P_a,    9 d2Z/dl_a dl_b = sh_a sh_b  (a != b),
// m_a = sh_a P_a / (9 Z), and the Jacobian of m is the covariance
// Z''/Z - m m^T (symmetric positive definite).  The iteration runs on
// X_a = exp(l_a) (Newton's method in X_a: X_a <- X_a (1 + d_a) with d the
// Newton step in l), from the D1Q3 solution of each axis,
// X_a = (2 u_a + s_a) / (1 - u_a), exact when the other components vanish;
// it stops after a step below 1e-9 (FP64) or 3e-4 (FP32), leaving an error
// of the order of that step's square.  Steps are clamped to [-1/2, 1] so
// that X stays positive far from the solution.  In FP64, once a first step
// was small (at most kChordMax), the later steps reuse its inverse Jacobian
// (chord steps: no new Jacobian, adjugate or determinant).  The Jacobian
// has moved by O(|d_1|) since, so a chord step leaves an error of about
// |d_1| times its own size; the iteration stops once that product is at
// the rounding level of FP64 (2^-53), which at the usual velocities
// (|d_1| ~ 1e-6 when all three components are nonzero) is the second step.
template <class R>
struct EquilibriumQ19 {
  R X[3], Y[3];  // exp(l_a), exp(-l_a)
  R Z9;          // 9 Z(l) at the final X
  static constexpr int kMaxIter = 12;
  static constexpr double kChordMax = 1e-4;

  __device__ __forceinline__ void sums(R (&ch)[3], R (&sh)[3], R& T, R& S2) const {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ch[a] = R(0.5) * (X[a] + Y[a]);
      sh[a] = R(0.5) * (X[a] - Y[a]);
    }
    T = ch[0] + ch[1] + ch[2];
    S2 = fma(ch[0], ch[1] + ch[2], ch[1] * ch[2]);
  }

  __device__ __forceinline__ void build(const R u[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const R s = sqrt_n<R>(fma(R(3) * u[a], u[a], R(1)));
      const R nu = fma(R(2), u[a], s), de = R(1) - u[a];
      const R r = rcp_n<R>(nu * de);
      X[a] = nu * (nu * r);
      Y[a] = de * (de * r);
    }
    const R tol = sizeof(R) == 8 ? R(1e-9) : R(3e-4);
    constexpr bool kChord = sizeof(R) == 8;
    bool done = false;
    // the last Jacobian's adjugate and -1/det, and the first step's size
    R A00 = R(0), A11 = R(0), A22 = R(0), A01 = R(0), A02 = R(0), A12 = R(0), idet = R(0);
    R d1 = R(1);
    for (int it = 0; it < kMaxIter; ++it) {
      if (!done) {
        R ch[3], sh[3], T, S2;
        sums(ch, sh, T, S2);
        const R iZ = rcp_n<R>(R(3) + T + S2);
        R m[3], g[3], P[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          P[a] = R(1) + T - ch[a];
          m[a] = sh[a] * P[a] * iZ;
          g[a] = m[a] - u[a];
        }
        const bool chord = kChord && it > 0 && d1 <= R(kChordMax);
        if (!chord) {
          const R H00 = fma(ch[0] * P[0], iZ, -m[0] * m[0]);
          const R H11 = fma(ch[1] * P[1], iZ, -m[1] * m[1]);
          const R H22 = fma(ch[2] * P[2], iZ, -m[2] * m[2]);
          const R H01 = fma(sh[0] * sh[1], iZ, -m[0] * m[1]);
          const R H02 = fma(sh[0] * sh[2], iZ, -m[0] * m[2]);
          const R H12 = fma(sh[1] * sh[2], iZ, -m[1] * m[2]);
          // d = -H^-1 g by the adjugate of the symmetric 3 x 3 matrix
          A00 = fma(H11, H22, -H12 * H12);
          A11 = fma(H00, H22, -H02 * H02);
          A22 = fma(H00, H11, -H01 * H01);
          A01 = fma(H02, H12, -H01 * H22);
          A02 = fma(H01, H12, -H02 * H11);
          A12 = fma(H01, H02, -H00 * H12);
          idet = -rcp_n<R>(fma(H00, A00, fma(H01, A01, H02 * A02)));
        }
        R d[3];
        d[0] = fma(A00, g[0], fma(A01, g[1], A02 * g[2])) * idet;
        d[1] = fma(A01, g[0], fma(A11, g[1], A12 * g[2])) * idet;
        d[2] = fma(A02, g[0], fma(A12, g[1], A22 * g[2])) * idet;
        R dmax = R(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          d[a] = fmin(fmax(d[a], R(-0.5)), R(1));
          dmax = fmax(dmax, fabs(d[a]));
          X[a] = fma(X[a], d[a], X[a]);
          Y[a] = rcp_n<R>(X[a]);
        }
        if (it == 0) d1 = dmax;
        done = chord ? !(dmax * d1 > R(0x1p-53)) : !(dmax > tol);
      }
      if (__all(done)) break;
    }
    R ch[3], sh[3], T, S2;
    sums(ch, sh, T, S2);
    Z9 = R(3) + T + S2;
  }
};

}  // namespace elbm
