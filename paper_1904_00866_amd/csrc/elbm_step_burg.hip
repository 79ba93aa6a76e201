// elbm_step_burg.hip -- the fused pull-stream + collide step with Burg's
// entropy H(f) = -sum_i W_i ln(f_i / W_i) in place of the Boltzmann entropy
// of Eq. (3).
//
// The paper remarks that the closed-form alpha (Eq. (9)) needs only a convex
// entropy; this kernel runs the same scheme (pull, moments, equilibrium,
// alpha_max, Eq. (8), acceptance test, Eq. (9), Eq. (1), store) with Burg's
// entropy, on every lattice (D1Q3, D2Q9, D3Q27, D3Q19):
//   - equilibrium: stationarity gives W_i / f^eq_i = m0 + m.c_i, so
//     f^eq_i = W_i / d_i with d_i = mu . (1, c_i); the D + 1 multipliers mu
//     solve the mass and momentum constraints, found per site by Newton's
//     method (elbm_burg.hpp);
//   - x_i = g_i / f^eq_i - 1 = g_i d_i / W_i - 1 needs no reciprocal;
//   - entropy differences between states with the moments of f^eq are the
//     exact relative form H(g) - H(f^eq) = sum_i W_i chi(g_i / f^eq_i - 1),
//     chi(y) = y - ln(1 + y) (h'(f^eq) = -W / f^eq is affine in (1, c_i));
//     at alpha_* = 2 the even / odd split E = sum W sum_k x^2k / 2k,
//     O = sum W sum_k x^(2k+1) / (2k+1) gives D = E - O, D* = E + O,
//     G(2) = 2 O without cancellation;
//   - Burg's entropy is infinite at a zero population, so with
//     alpha_* = alpha_max (< 2) both differences of Eq. (9) are infinite and
//     their ratio tends to 1: alpha = 1 (closed form and modified secant).
// FP64 site arithmetic; FP64 or FP32 storage.
#include "elbm_burg.hpp"
#include "elbm_q19.hpp"
#include "elbm_step_impl.hpp"

namespace elbm {
namespace {

// Pull of the Q populations when the wavefront's 64 sites lie in one x-row
// (one descriptor per source row (c_y, c_z); see load_site_row).
template <class L, class T>
__device__ __forceinline__ void load_row_l(const SimDesc& d, const T* src, uint32_t s,
                                           T (&raw)[L::Q]) {
  constexpr int D = L::Dim, Q = L::Q;
  const uint32_t nx = (uint32_t)d.nx, ny = (uint32_t)d.ny, nz = (uint32_t)d.nz;
  const uint32_t row = __builtin_amdgcn_readfirstlane(D == 1 ? 0u : qdiv(s, d.inv_nx));
  const uint32_t x = s - row * nx;
  uint32_t ys[3] = {0u, 0u, 0u}, zs[3] = {0u, 0u, 0u};
  if constexpr (D > 1) {
    const uint32_t z = D == 3 ? __builtin_amdgcn_readfirstlane(qdiv(row, d.inv_ny)) : 0u;
    const uint32_t y = row - z * ny;
    ys[0] = y * nx;
    ys[1] = (y == 0 ? ny - 1 : y - 1) * nx;
    ys[2] = (y == ny - 1 ? 0 : y + 1) * nx;
    const uint32_t nxy = nx * ny;
    zs[0] = z * nxy;
    zs[1] = (z == 0 ? nz - 1 : z - 1) * nxy;
    zs[2] = (z == nz - 1 ? 0 : z + 1) * nxy;
  }
  constexpr uint32_t es = sizeof(T);
  uint32_t xo[3];
  const uint32_t xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  xo[0] = (uint32_t)pidx<Q>(x, 0) * es;
  xo[1] = (uint32_t)pidx<Q>(xm, 0) * es;
  xo[2] = (uint32_t)pidx<Q>(xp, 0) * es;
  const gaddr base = buffer_base(src);
  const uint32_t rowbytes = nx * (uint32_t)Q * es;
#pragma unroll
  for (int dz = 0; dz < (D > 2 ? 3 : 1); ++dz)
#pragma unroll
    for (int dy = 0; dy < (D > 1 ? 3 : 1); ++dy) {
      const __amdgpu_buffer_rsrc_t r = rsrc(base + (uint64_t)(zs[dz] + ys[dy]) * Q * es, rowbytes);
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int i = Dirs<L>::index(dx, dy, dz);
        if (i < 0) continue;
        raw[i] = ld_buf<T>(r, xo[dx], (uint32_t)i * kLane * es);
      }
    }
}

// Pull of the Q populations of site s (s < N), any box.
template <class L, class T>
__device__ __forceinline__ void load_l(const SimDesc& d, const T* src, uint32_t s, T (&raw)[L::Q]) {
  const Where w = locate<L::Dim>(d, s);
  const gaddr base = buffer_base(src);
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const uint32_t sp = w.zs[L::dg(i, 2)] + w.ys[L::dg(i, 1)] + w.xs[L::dg(i, 0)];
    raw[i] = *(const gptr<T>)(base + pidx<L::Q>(sp, i) * sizeof(T));
  }
}

template <class L, class S>
struct SiteBurg {
  using T = typename S::T;
  using R = double;
  using Real = double;
  static constexpr int Q = L::Q;
  static constexpr int kDim = L::Dim;
  T raw[Q];
  R rho, irho, rho_ref;
  R u[3];
  R mu[4];  // f^eq_i = W_i / d_i, d_i = mu[0] + sum_a c_ia mu[a + 1]
  R x[Q];   // x_i = g_i / f^eq_i - 1

  __device__ __forceinline__ R g(int i) const {
    return Codec<S, R>::dec_wide(widen<R>(raw[i]), R(L::W(i)), rho_ref);
  }
  __device__ __forceinline__ R den(int i) const { return burg_den<L>(mu, i); }
  // H(f^eq) / rho = sum_i W_i ln(d_i) / rho
  __device__ __forceinline__ double heq_per_rho() const {
    double h = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) h += L::W(i) * log(den(i));
    return h * irho;
  }
};

template <class L, class S>
__device__ __forceinline__ void prepare_burg(SiteBurg<L, S>& v, const SimDesc& d, double (&j)[3]) {
  constexpr int Q = L::Q;
  v.rho_ref = d.rho_ref;
  double rho = 0.0;
  j[0] = j[1] = j[2] = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double gi = v.g(i);
    rho = i == 0 ? gi : rho + gi;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int c = L::c(i, a);
      if (c > 0) j[a] += gi;
      else if (c < 0) j[a] -= gi;
    }
  }
  v.rho = rho;
  v.irho = rcp_n<double>(rho);
#pragma unroll
  for (int a = 0; a < 3; ++a) v.u[a] = j[a] * v.irho;
  burg_multipliers<L>(v.rho, v.irho, v.u, v.mu);
#pragma unroll
  for (int i = 0; i < Q; ++i) v.x[i] = fma(v.g(i) * L::invW(i), v.den(i), -1.0);
}

// chi(y) = y - ln(1 + y) and chi'(y) = y / (1 + y); y <= -1 only arises as the
// rounding of a population driven exactly to zero (infinite entropy).
__device__ __forceinline__ double chi(double y) {
  return y <= -1.0 ? double(INFINITY) : y - log1p(y);
}
__device__ __forceinline__ double dchi(double y) {
  return y <= -1.0 ? -double(INFINITY) : y / (1.0 + y);
}

// chi(y) = sum_{n>=2} (-1)^n y^n / n for |y| <= kChiYmax, through y^11 / 11
// by Horner's rule: the first omitted term is below 2 y^10 / 12 < 2^-54 of
// the sum, which is about y^2 / 2 (no cancellation between y and ln(1 + y)).
constexpr double kChiYmax = 0.025;
__device__ __forceinline__ double chi_series(double y) {
  double p = -1.0 / 11.0;
#pragma unroll
  for (int n = 10; n >= 2; --n) p = fma(p, y, (n % 2 ? -1.0 : 1.0) / n);
  return y * y * p;
}

// S(a) = sum_i W_i chi((1 - a) x_i) = H(f*(a)) - H(f^eq): by the series
// where every lane of the wavefront has |(1 - a) x_i| <= kChiYmax, else by
// the library log1p.
template <class L, class S>
__device__ __forceinline__ double S_chi(const SiteBurg<L, S>& v, double a, double xabs) {
  double s = 0.0;
  if (__all(fabs(1.0 - a) * xabs <= kChiYmax)) {
#pragma unroll
    for (int i = 0; i < L::Q; ++i) s = fma(L::W(i), chi_series((1.0 - a) * v.x[i]), s);
  } else {
#pragma unroll
    for (int i = 0; i < L::Q; ++i) s += L::W(i) * chi((1.0 - a) * v.x[i]);
  }
  return s;
}

// Series tier: max|x_i| <= kThrB keeps the alpha error of the K-term sums
// below 2^-53 (truncation moves alpha by about 4 x^(2K+1) / (2K+3)).
constexpr int kKB = 4;
constexpr double kThrB = 0.018;

template <int MODE, class L, class S>
__device__ __forceinline__ AlphaOut<double> choose_alpha_burg(SiteBurg<L, S>& v, const SimDesc& d) {
  constexpr int Q = L::Q;
  AlphaOut<double> o;
  o.deferred = false;
  double xmax = -1.0, xabs = 0.0, sE = 0.0, sO = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double xi = v.x[i], t = xi * xi;
    xmax = fmax(xmax, xi);
    xabs = fmax(xabs, fabs(xi));
    // E_K(x) = sum_{k<=K} x^2k / 2k, O_K(x) = x sum_{k<=K} x^2k / (2k + 1)
    double pe = 1.0 / (2.0 * kKB), po = 1.0 / (2.0 * kKB + 1.0);
#pragma unroll
    for (int k = kKB - 1; k >= 1; --k) {
      pe = fma(pe, t, 1.0 / (2.0 * k));
      po = fma(po, t, 1.0 / (2.0 * k + 1.0));
    }
    sE = fma(L::W(i) * t, pe, sE);
    sO = fma(L::W(i) * t * xi, po, sO);
  }
  const bool rare = !(xabs <= kThrB);
  const bool has_pos = xmax > 0.0;
  const double amax = has_pos ? 1.0 + 1.0 / xmax : double(INFINITY);
  const bool star2 = !(xmax >= 1.0);  // alpha_max > 2
  const double astar = star2 ? 2.0 : amax;
  double Dv = sE - sO, Ds = sE + sO, Gs = 2.0 * sO;
  if (__any(rare)) {
    if (rare) {
      double sD = 0.0, sS = 0.0;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        sD += L::W(i) * chi(v.x[i]);
        if (star2) sS += L::W(i) * chi((1.0 - astar) * v.x[i]);
      }
      Dv = sD;
      Ds = star2 ? sS : double(INFINITY);
      Gs = star2 ? sS - sD : double(INFINITY);
    }
  }
  const bool guard = !has_pos || !(Dv > 1e-26 * v.rho);
  o.D = Dv;
  o.guard = guard;
  o.astar_lt2 = !star2;
  o.fallback = rare;
  o.accepted2 = star2 && (guard || Gs <= 0.0);
  double alpha = astar;
  int iters = 0;
  if (!guard) {
    if constexpr (MODE == kClosed) {
      if (Gs > 0.0) {
        // Eq. (9); with alpha_* = alpha_max both differences are infinite
        // and their ratio is 1 in the limit
        alpha = star2 ? astar + Gs / Ds * (1.0 - astar) : 1.0;
        alpha = fmin(fmax(alpha, 1.0), astar);
        iters = 1;
      }
    } else if constexpr (MODE == kSecant) {
      if (Gs > 0.0) {
        double a = 1.0;
        if (star2) {
          for (int k = 0; k < d.secant_iters; ++k) {
            const double Ga = S_chi(v, a, xabs) - Dv;
            const double an = astar + Gs / (Gs - Ga) * (a - astar);
            iters = k + 1;
            if (an == a) break;
            a = an;
          }
        } else {
          iters = 1;  // G(alpha_*) infinite: every iterate stays at 1
        }
        alpha = fmin(fmax(a, 1.0), astar);
      }
    } else if constexpr (MODE == kBisect) {
      // G(alpha_max) = +inf (zero population): the root lies inside
      double lo = 1.0, hi = amax;
      const double tol = d.root_tol;
      alpha = -1.0;
      for (int k = 1; k <= d.root_max_iter; ++k) {
        const double mid = 0.5 * (lo + hi);
        const double gm = S_chi(v, mid, xabs) - Dv;
        iters = k;
        if (gm <= 0.0 && gm >= -tol) {
          alpha = mid;
          break;
        }
        if (gm > 0.0) hi = mid;
        else lo = mid;
      }
      if (alpha < 0.0) alpha = lo;
    } else if constexpr (MODE == kNewton) {
      // stops when |G(a)| is at the rounding level of its evaluation,
      // eps sum_i W_i (|x_i| + |(1 - a) x_i|), or at a step below 1e-13 a
      double lo = 1.0, hi = amax;
      double a = (astar < amax) ? astar : 0.5 * (lo + hi);
      double sA = 0.0;
#pragma unroll
      for (int i = 0; i < Q; ++i) sA += L::W(i) * fabs(v.x[i]);
      for (int k = 1; k <= d.root_max_iter; ++k) {
        // S and S' = -sum_i W_i x_i chi'(y_i), chi'(y) = y / (1 + y): the
        // series and the refined reciprocal where every lane has
        // |y_i| <= kChiYmax, else the library forms
        double Sv = 0.0, dS = 0.0;
        if (__all(fabs(1.0 - a) * xabs <= kChiYmax)) {
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            const double y = (1.0 - a) * v.x[i];
            Sv = fma(L::W(i), chi_series(y), Sv);
            dS = fma(-L::W(i) * v.x[i], y * rcp_n<double>(1.0 + y), dS);
          }
        } else {
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            const double y = (1.0 - a) * v.x[i];
            Sv += L::W(i) * chi(y);
            dS -= L::W(i) * v.x[i] * dchi(y);
          }
        }
        const double gv = Sv - Dv;
        iters = k;
        if (fabs(gv) <= 2.220446049250313e-16 * (1.0 + fabs(1.0 - a)) * sA) break;
        if (gv > 0.0) hi = a;
        else lo = a;
        double an = a - gv / dS;
        if (!(an > lo && an < hi)) {
          // a converged step that rounds onto the end of the bracket stops
          // there; a longer one is replaced by the midpoint (G(alpha_max) is
          // infinite, so the root always lies inside)
          if (fabs(an - a) <= 1e-13 * a) {
            a = fmin(fmax(an, lo), hi);
            break;
          }
          an = 0.5 * (lo + hi);
        }
        if (fabs(an - a) <= 1e-13 * a) {
          a = an;
          break;
        }
        a = an;
      }
      alpha = a;
    }
  }
  o.alpha = alpha;
  o.iters = iters;
  return o;
}

template <class L, class S, int MODE, bool SUMS>
__device__ __forceinline__ uint32_t update_burg(const SimDesc& d, typename S::T* __restrict__ dst,
                                                uint32_t s, bool live, const typename S::T (&raw)[L::Q],
                                                Acc& acc, int diag) {
  constexpr int Q = L::Q;
  using T = typename S::T;
  constexpr uint32_t es = sizeof(T);
  SiteBurg<L, S> v;
#pragma unroll
  for (int i = 0; i < Q; ++i) v.raw[i] = raw[i];
  double j[3];
  prepare_burg(v, d, j);
  const AlphaOut<double> ao = choose_alpha_burg<MODE>(v, d);
  const double ab = ao.alpha * d.beta;
  double ftmin = INFINITY;
  const uint32_t lo = (s & 63u) * es;
  const gaddr blk = block_base<Q>(dst, s);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double gi = v.g(i);
    const double fe = L::W(i) * rcp_n<double>(v.den(i));
    const double ft = fma(ab, fe - gi, gi);
    ftmin = fmin(ftmin, ft);
    st_nt<T>(blk + i * kLane * es, kLane * es, lo, Codec<S, double>::enc(ft, L::invW(i), v.rho_ref));
  }
  return record_site<SUMS>(d, s, live, v, ao, ftmin, j, acc, diag);
}

// The step kernel: the workgroup, tile and XCD-aware order of k_step.
template <class L, class S, int MODE, bool SUMS>
__global__ void __launch_bounds__(kBlock) k_step_burg(const BatchArgs args) {
  using T = typename S::T;
  constexpr int Q = L::Q;
  constexpr int ELBM_TILES = tiles_per_block(sizeof(T), Q);
  const int b = blockIdx.x;
  int si = 0;
  for (int k = 1; k < args.n; ++k)
    if (b >= args.d[k].block_begin) si = k;
  const SimDesc& d = args.d[si];
  const T* __restrict__ src = static_cast<const T*>(d.src);
  T* __restrict__ dst = static_cast<T*>(d.dst);
  const int diag = d.diag;
  const uint32_t N = (uint32_t)d.nx * (uint32_t)d.ny * (uint32_t)d.nz;
  const uint32_t lb = (uint32_t)(b - d.block_begin);
  const uint32_t chunk = (uint32_t)d.nblocks >> 3;
  const uint32_t unit = (lb & 7u) * chunk + (lb >> 3);
  Acc acc;
  acc.init();
  if (unit * ELBM_TILES * kBlock < N) {
#pragma unroll 1
    for (int k = 0; k < ELBM_TILES; ++k) {
      const uint32_t s = (unit * ELBM_TILES + k) * kBlock + threadIdx.x;
      uint32_t flags = 0;
      if (k == 0 || (unit * ELBM_TILES + k) * kBlock < N) {
        T raw[Q];
        const uint32_t sl = s < N ? s : 0u;
        if (d.nx % 64 == 0)
          load_row_l<L>(d, src, sl, raw);
        else
          load_l<L>(d, src, sl, raw);
        flags = update_burg<L, S, MODE, SUMS>(d, dst, s, s < N, raw, acc, diag);
      }
      if (diag & kDiagCounts) acc.count_flags(flags);
    }
  } else if (!(diag & kDiagCounts)) {
    return;  // padding workgroup
  }
  // iterations are recorded for the secant and the root solvers, as in k_step
  if (diag & kDiagCounts) store_records<MODE != kClosed>(acc, d, (int)lb);
}

template <class L, class S, int MODE>
hipError_t launch_burg(const BatchArgs& a, int grid, hipStream_t st) {
  bool sums = false;
  for (int k = 0; k < a.n; ++k) sums = sums || (a.d[k].diag & kDiagSums);
  if (sums)
    k_step_burg<L, S, MODE, true><<<grid, kBlock, 0, st>>>(a);
  else
    k_step_burg<L, S, MODE, false><<<grid, kBlock, 0, st>>>(a);
  return hipGetLastError();
}

template <class L>
StepLauncher burg_for(int storage, int mode) {
#define ELBM_MODES(S)                                 \
  switch (mode) {                                     \
    case kClosed: return &launch_burg<L, S, kClosed>; \
    case kNewton: return &launch_burg<L, S, kNewton>; \
    case kBisect: return &launch_burg<L, S, kBisect>; \
    case kSecant: return &launch_burg<L, S, kSecant>; \
    default: return nullptr;                          \
  }
  switch (storage) {
    case kStoreF64: ELBM_MODES(StoreF64)
    case kStoreF32: ELBM_MODES(StoreF32)
    default: return nullptr;
  }
#undef ELBM_MODES
}

}  // namespace

StepLauncher step_launcher_burg(int lattice, int storage, int mode, int fp64) {
  if (fp64 != kArithF64) return nullptr;
  switch (lattice) {
    case 1: return burg_for<Lattice<1>>(storage, mode);
    case 2: return burg_for<Lattice<2>>(storage, mode);
    case 3: return burg_for<Lattice<3>>(storage, mode);
    case 19: return burg_for<LatticeQ19>(storage, mode);
    default: return nullptr;
  }
}

}  // namespace elbm
