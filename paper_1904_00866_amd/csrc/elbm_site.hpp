// elbm_site.hpp -- per-site arithmetic of the entropic lattice Boltzmann step
// for gfx950: lattice constants, population storage codecs, the entropic
// equilibrium, the relaxation parameter alpha and the collision.
//
// Method: Zhao & Yong, "Relaxation-rate formula for the entropic lattice
// Boltzmann method".  Per site:
//   rho, rho u                      conservation constraints after Eq. (3)
//   f^eq = argmin H, H = sum f ln(f/W)   Eq. (3) and the constraints
//   alpha_max, alpha_*              definition after Eq. (7), Eq. (8)
//   alpha = alpha_* if H(f*(alpha_*)) <= H(f), else Eq. (9)
//   f~ = f + alpha beta (f^eq - f)  Eq. (1) / Eq. (5a)
// Comparators: Eq. (4) by bracketed Newton or by bisection (the stop window of
// the double-shear comparison), the modified secant iteration of the closing
// remark, and LBGK (alpha = 2, polynomial equilibrium; named after Eq. (4)).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace elbm {

// ---------------------------------------------------------------- lattice --
// Directions are the tensor product of {0, +1, -1} per axis:
//   i = d(c_x) + 3 d(c_y) + 9 d(c_z),  d(0) = 0, d(+1) = 1, d(-1) = 2.
// The weights factorise, W_i = prod_a w(c_ia), w(0) = 2/3, w(+-1) = 1/6,
// and c_s^2 = 1/3 (lattice units).
__host__ __device__ constexpr int ipow3(int d) { return d == 0 ? 1 : 3 * ipow3(d - 1); }
__host__ __device__ constexpr int digit(int i, int a) {
  return (a == 0 ? i : a == 1 ? i / 3 : i / 9) % 3;
}
__host__ __device__ constexpr int cval(int dg) { return dg == 0 ? 0 : (dg == 1 ? 1 : -1); }

template <int D>
struct Lattice {
  static constexpr int Dim = D;
  static constexpr int Q = ipow3(D);
  __host__ __device__ static constexpr int c(int i, int a) { return a < D ? cval(digit(i, a)) : 0; }
  __host__ __device__ static constexpr int dg(int i, int a) { return a < D ? digit(i, a) : 0; }
  // W_i = 4^(number of zero components) / 6^D; exact as a quotient of
  // small integers and its reciprocal 6^D / 4^k is exact in binary.
  __host__ __device__ static constexpr int nzero(int i) {
    return (D > 0 && digit(i, 0) == 0) + (D > 1 && digit(i, 1) == 0) + (D > 2 && digit(i, 2) == 0);
  }
  __host__ __device__ static constexpr double den() { return D == 1 ? 6.0 : D == 2 ? 36.0 : 216.0; }
  __host__ __device__ static constexpr double num(int i) {
    return nzero(i) == 0 ? 1.0 : nzero(i) == 1 ? 4.0 : nzero(i) == 2 ? 16.0 : 64.0;
  }
  __host__ __device__ static constexpr double W(int i) { return num(i) / den(); }
  __host__ __device__ static constexpr double invW(int i) { return den() / num(i); }
};

// ---------------------------------------------------------------- storage --
// Populations live in SoA planes of one of four element types.  The
// deviation formats hold s_i = f_i / W_i - rho_ref, so that the stored
// number is O(|u| + |x|) whatever the weight; decode f_i = W_i (rho_ref + s_i).
struct StoreF64 {
  using T = double;
  static constexpr bool dev = false;
};
struct StoreF32 {
  using T = float;
  static constexpr bool dev = false;
};
struct StoreF32Dev {
  using T = float;
  static constexpr bool dev = true;
};
struct StoreF16Dev {
  using T = _Float16;
  static constexpr bool dev = true;
};

// What a site keeps of each loaded population between its passes: the
// stored value, except for FP16 deviations, which are kept converted to FP32
// (exactly), so that each pass needs one widening instead of two.
template <class S>
struct Kept {
  using type = typename S::T;
};
template <>
struct Kept<StoreF16Dev> {
  using type = float;
};

template <class S, class R>
struct Codec {
  static constexpr bool kF16 = S::dev && sizeof(typename S::T) == 2;
  // decoded population f = W (rho_ref + s) (deviation formats), formed as
  // W s + W rho_ref with one rounding; or the stored value
  __device__ static __forceinline__ R dec(typename S::T v, R W, R rho_ref) {
    if constexpr (S::dev) return fma(W, (R)v, W * rho_ref);
    else return (R)v;
  }
  __device__ static __forceinline__ typename Kept<S>::type keep(typename S::T v) {
    if constexpr (kF16) return (float)v;
    else return v;
  }
  // decode of a kept value already widened to R (the same arithmetic as dec)
  __device__ static __forceinline__ R dec_wide(R v, R W, R rho_ref) {
    if constexpr (S::dev) return fma(W, v, W * rho_ref);
    else return v;
  }
  // FP16 is formed from the FP32 value by two conversion instructions (there
  // is none from FP64 to FP16): round to nearest even twice, which differs
  // from a single rounding only for FP64 values within half an FP32 ulp of
  // an FP16 midpoint.  The FP32 value is hidden from the optimiser: allowed
  // to contract the two roundings, it merges them into one FP64 -> FP16
  // rounding carried out in integer arithmetic, about 40 instructions per
  // population.
  __device__ static __forceinline__ typename S::T enc(R f, R invW, R rho_ref) {
    using T = typename S::T;
    if constexpr (S::dev) {
      const R sdev = f * invW - rho_ref;
      if constexpr (sizeof(T) == 2) {
        float h = (float)sdev;
        asm volatile("" : "+v"(h));
        return (T)h;
      } else {
        return (T)sdev;
      }
    } else {
      return (T)f;
    }
  }
};

// -------------------------------------------------------------- precision --
template <class R>
struct Prec;
// guard: f = f^eq to rounding when H(f) - H(f^eq) <= guard * rho.
template <>
struct Prec<double> {
  static constexpr double guard = 1e-26;
  __device__ static __forceinline__ double log1p_(double y) { return ::log1p(y); }
  __device__ static __forceinline__ double sqrt_(double y) { return ::sqrt(y); }
};
template <>
struct Prec<float> {
  static constexpr float guard = 1e-30f;
  __device__ static __forceinline__ float log1p_(float y) { return ::log1pf(y); }
  __device__ static __forceinline__ float sqrt_(float y) { return ::sqrtf(y); }
};

// ------------------------------------------------ reciprocal, square root --
// For arguments in the normal range (the site arithmetic never sees zeros,
// infinities or subnormals here: rho > 0, 1 <= 1 + 3 u^2 < 4, and the
// equilibrium's denominators lie in (0, 54) for |u| < 1), the hardware
// estimates refined by Newton's iteration for 1/y (e = 1 - y r,
// r <- r + r e, quadratic convergence) and Goldschmidt's iteration for
// sqrt(y) (g ~ sqrt(y), h ~ 1/(2 sqrt(y)), then residual corrections) give
// the result to about one unit in the last place without the scaling and
// special-case handling of the library routines.
template <class R>
__device__ __forceinline__ R rcp_n(R y) {
  if constexpr (std::is_same<R, double>::value) {
    R r = __builtin_amdgcn_rcp(y);
    R e = fma(-y, r, 1.0);
    r = fma(r, e, r);
    e = fma(-y, r, 1.0);
    return fma(r, e, r);
  } else {
    return R(1) / y;
  }
}
template <class R>
__device__ __forceinline__ R sqrt_n(R y) {
  if constexpr (std::is_same<R, double>::value) {
    const R r = __builtin_amdgcn_rsq(y);
    R g = y * r, h = 0.5 * r;
    const R e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    R d = fma(-g, g, y);
    g = fma(d, h, g);
    d = fma(-g, g, y);
    return fma(d, h, g);
  } else {
    return Prec<R>::sqrt_(y);
  }
}

// ------------------------------------------------------------ equilibrium --
// The minimiser of H under mass and momentum is f_i^eq = W_i exp(l0 + l.c_i).
// With tensor-product weights it factorises per axis a:
//   s_a = sqrt(1 + 3 u_a^2), A_a = 2 - s_a, z_a = (2 u_a + s_a) / (1 - u_a),
//   f_i^eq = rho prod_a w(c_ia) A_a z_a^(c_ia),        |u_a| < 1.
// E[a][d] holds the unweighted factor A_a z_a^c for digit d of c and IE[a][d]
// its reciprocal; with nu = 2 u + s, de = 1 - u and r = 1 / (A nu de) all six
// follow from one reciprocal:
//   A z = (A nu)^2 r,  A / z = (A de)^2 r,  1/A = nu de r,
//   1/(A z) = de^2 r,  z / A = nu^2 r.
// The weights w(0) = 2/3, w(+-1) = 1/6 are applied by the users (weight()).
template <class R, int D>
struct Equilibrium {
  R E[3][3];
  R IE[3][3];

  __host__ __device__ static constexpr double weight(int d) { return d == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }

  __device__ __forceinline__ void build(const R u[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a < D) {
        const R ua = u[a];
        const R s = sqrt_n<R>(fma(R(3) * ua, ua, R(1)));
        const R A = R(2) - s;
        const R nu = fma(R(2), ua, s);
        const R de = R(1) - ua;
        const R P = A * nu, M = A * de, Z = nu * de;
        const R r = rcp_n<R>(A * Z);
        E[a][0] = A;
        E[a][1] = P * (P * r);
        E[a][2] = M * (M * r);
        IE[a][0] = Z * r;
        IE[a][1] = de * (de * r);
        IE[a][2] = nu * (nu * r);
      } else {
        // absent axes are never read (e() and ie() return 1 for them)
        E[a][0] = E[a][1] = E[a][2] = R(1);
        IE[a][0] = IE[a][1] = IE[a][2] = R(1);
      }
    }
  }
  // weighted factors w(d) E and their reciprocals
  __device__ __forceinline__ R e(int a, int d) const {
    return a < D ? R(weight(d)) * E[a][d] : R(1);
  }
  __device__ __forceinline__ R ie(int a, int d) const {
    return a < D ? IE[a][d] * R(1.0 / weight(d)) : R(1);
  }
};

// ---------------------------------------------------------- entropy sums --
// phi(y) = (1+y) ln(1+y) - y.  Because ln(f^eq_i/W_i) is affine in (1, c_i),
// any g with the moments of f^eq has H(g) - H(f^eq) = sum_i f^eq_i phi(g_i/f^eq_i - 1).
// With x_i = f_i/f^eq_i - 1 and f*(alpha) = f^eq (1 + (1 - alpha) x):
//   D      = H(f) - H(f^eq)          = sum f^eq phi(x)
//   G(a)   = H(f*(a)) - H(f)         = sum f^eq [phi((1-a)x) - phi(x)]
//   D*(a)  = H(f*(a)) - H(f^eq)      = sum f^eq phi((1-a)x)   (Eq. (9) denominator)
// At alpha_* = 2 the Maclaurin series of ln(1 +- x) give, with
//   E(x) = sum_k x^(2k) / (2k (2k-1)),  O(x) = sum_k x^(2k+1) / ((2k+1) 2k),
//   phi(x) = E - O, phi(-x) = E + O, G(2) = 2 sum f^eq O: no cancellation.
template <class R>
__device__ __forceinline__ R phi_log(R y) {
  // y <= -1 only arises as the rounding of (1 - alpha_max) x_k = -1, i.e. a
  // population driven exactly to zero: the 0 ln 0 = 0 limit is phi = 1.
  if (y <= R(-1)) return R(1);
  return (R(1) + y) * Prec<R>::log1p_(y) - y;
}

template <class R>
__device__ __forceinline__ R dlog_clamped(R y) {
  return Prec<R>::log1p_(y < R(-1) ? R(-1) : y);
}

// Truncated series, K terms each, in t = x^2:
//   E(x) = sum_k c_k t^k, c_k = 1/(2k (2k-1));  O(x) = x sum_k d_k t^k,
//   d_k = 1/((2k+1) 2k).
// SeriesK holds E / c_K and O / d_K as monic polynomials: each Horner step
// then takes one constant, and the constants sit in scalar registers (an
// FP64 VALU operation can read one scalar operand but no 64-bit literal, so
// a constant not held in a scalar register costs vector moves at every use).
// Multiply the sums by series_scale() afterwards.
template <class R>
__device__ __forceinline__ R in_sgpr(R v) {
  asm volatile("" : "+s"(v));
  return v;
}

template <class R, int K>
struct SeriesK {
  R e[K > 1 ? K - 1 : 1], o[K > 1 ? K - 1 : 1];  // e[k-1], o[k-1] for k = 1 .. K-1
  __device__ __forceinline__ SeriesK() {
#pragma unroll
    for (int k = 1; k < K; ++k) {
      e[k - 1] = in_sgpr(R((1.0 / ((2.0 * k) * (2.0 * k - 1.0))) /
                           (1.0 / ((2.0 * K) * (2.0 * K - 1.0)))));
      o[k - 1] = in_sgpr(R((1.0 / ((2.0 * k + 1.0) * (2.0 * k))) /
                           (1.0 / ((2.0 * K + 1.0) * (2.0 * K)))));
    }
  }
  // sE += f E(x), sO += f O(x), the K-term sums scaled by 1/c_K, 1/d_K, with
  // f x^2 formed once for both: one multiplication fewer per direction.
  __device__ __forceinline__ void accum(R x, R f, R& sE, R& sO) const {
    const R t = x * x;
    R pe = R(1), po = R(1);
    if constexpr (K >= 2) {
      pe = t + e[K - 2];
      po = t + o[K - 2];
    }
#pragma unroll
    for (int k = K - 2; k >= 1; --k) {
      pe = fma(pe, t, e[k - 1]);
      po = fma(po, t, o[k - 1]);
    }
    const R w = f * t;
    sE = fma(w, pe, sE);
    sO = fma(w * x, po, sO);
  }
};

// (c_K, d_K): the factors that restore the sums of SeriesK.
template <class R, int K>
__device__ __forceinline__ void series_scale(R& cE, R& cO) {
  cE = R(1.0 / ((2.0 * K) * (2.0 * K - 1.0)));
  cO = R(1.0 / ((2.0 * K + 1.0) * (2.0 * K)));
}

}  // namespace elbm
