// elbm_step_impl.hpp -- the fused pull-stream + collide kernel.
//
// One launch = one time step for up to kMaxBatch simulations.  Each
// simulation owns a contiguous range of workgroups, one per tile of kBlock
// consecutive sites (x fastest).  Per site (thread):
//   pull   g_i = src_i(x - c_i)                        Eq. (5b)
//   rho, u                                             constraints after Eq. (3)
//   f^eq, x_i = g_i / f^eq_i - 1                       minimiser of Eq. (3)
//   alpha (closed form / Newton / bisection / secant)  Eqs. (4), (8), (9)
//   dst_i(x) = g_i + alpha beta (f^eq_i - g_i)         Eq. (1)
// so that dst, pulled at the next step, is f(x, t+1).  Every value of src is
// read exactly once per step, every value of dst written once: 2 Q b bytes
// per site update for b-byte storage.
#pragma once

#include "elbm_internal.hpp"
#include "elbm_site.hpp"

namespace elbm {

template <class R>
struct AlphaOut {
  R alpha, D;
  int accepted2, astar_lt2, guard, fallback, iters;
};

// Keeps a value in registers but hides it from the optimiser, so that
// quantities derived from it are recomputed where they are used instead of
// being kept live (register pressure decides the occupancy of this kernel).
template <class R>
__device__ __forceinline__ R opaque(R v) {
  asm volatile("" : "+v"(v));
  return v;
}

// One site's loaded populations and its equilibrium factors.  x_i and
// f^eq_i are recomputed from them in each pass instead of being stored.
template <int D, class S, class R>
struct SiteView {
  using L = Lattice<D>;
  static constexpr int Q = L::Q;
  typename S::T raw[Q];
  R rho, irho, rho_ref;
  Equilibrium<R, D> eq;

  // The loaded value passes through opaque() so that its conversion is
  // redone in each pass rather than Q converted values being kept live.
  __device__ __forceinline__ R g(int i) const {
    return Codec<S, R>::dec(opaque(raw[i]), R(L::W(i)), rho_ref);
  }
  // f^eq_i = rho prod_a e[a][d_a(i)]
  __device__ __forceinline__ R fe(int i, R r) const {
    return r * (eq.e[0][L::dg(i, 0)] * eq.e[1][L::dg(i, 1)]) * eq.e[2][L::dg(i, 2)];
  }
  // x_i = g_i / f^eq_i - 1, with 1/f^eq_i = (1/rho) prod_a ie[a][d_a(i)]
  __device__ __forceinline__ R x(int i, R ir) const {
    const R ri = ir * (eq.ie[0][L::dg(i, 0)] * eq.ie[1][L::dg(i, 1)]) * eq.ie[2][L::dg(i, 2)];
    return fma(g(i), ri, R(-1));
  }
};

// S(a) = sum_i f^eq_i phi((1 - a) x_i); G(a) = H(f*(a)) - H(f) = S(a) - D.
template <int D, class S, class R>
__device__ __forceinline__ R S_log(const SiteView<D, S, R>& v, R a) {
  const R r = opaque(v.rho), ir = opaque(v.irho);
  R s = R(0);
#pragma unroll
  for (int i = 0; i < SiteView<D, S, R>::Q; ++i) s += v.fe(i, r) * phi_log<R>((R(1) - a) * v.x(i, ir));
  return s;
}

// S(a) and S'(a) = G'(a) = -sum_i f^eq_i x_i ln(1 + (1 - a) x_i).
template <int D, class S, class R>
__device__ __forceinline__ void S_dS_log(const SiteView<D, S, R>& v, R a, R& Sv, R& dS) {
  const R r = opaque(v.rho), ir = opaque(v.irho);
  Sv = R(0);
  dS = R(0);
#pragma unroll
  for (int i = 0; i < SiteView<D, S, R>::Q; ++i) {
    const R xi = v.x(i, ir), fi = v.fe(i, r);
    const R y = (R(1) - a) * xi;
    const R l = dlog_clamped<R>(y);
    Sv += fi * ((y <= R(-1)) ? R(1) : (R(1) + y) * l - y);
    dS -= fi * xi * l;
  }
}

template <int K, int D, class S, class R>
__device__ __forceinline__ void series_sums(const SiteView<D, S, R>& v, R& sE, R& sO) {
  const R r = opaque(v.rho), ir = opaque(v.irho);
  sE = R(0);
  sO = R(0);
#pragma unroll
  for (int i = 0; i < SiteView<D, S, R>::Q; ++i) {
    R E, O;
    series_EO<R, K>(v.x(i, ir), E, O);
    const R fi = v.fe(i, r);
    sE += fi * E;
    sO += fi * O;
  }
}

// The choice of alpha at one site.
template <int MODE, int D, class S, class R>
__device__ __forceinline__ AlphaOut<R> choose_alpha(const SiteView<D, S, R>& v, const SimDesc& d) {
  constexpr int Q = SiteView<D, S, R>::Q;
  AlphaOut<R> o;
  o.fallback = 0;
  R xmax, xabs;
  {
    const R ir = v.irho;
    const R x0 = v.x(0, ir);
    xmax = x0;
    xabs = fabs(x0);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const R xi = v.x(i, ir);
      xmax = fmax(xmax, xi);
      xabs = fmax(xabs, fabs(xi));
    }
  }
  // alpha_max = min over {f^eq_i < f_i} of f_i/(f_i - f^eq_i) = 1 + 1/max_i x_i
  // (definition after Eq. (7)); alpha_* = min(2, alpha_max) (Eq. (8)), and
  // alpha_* = 2 exactly when max_i x_i <= 1.
  const bool has_pos = xmax > R(0);
  const R amax = has_pos ? R(1) + R(1) / xmax : R(INFINITY);
  const bool star2 = !(xmax > R(1));
  const R astar = star2 ? R(2) : amax;

  // D = H(f) - H(f^eq), Gs = H(f*(a_*)) - H(f), Ds = H(f*(a_*)) - H(f^eq)
  R Dv, Gs, Ds;
  if (star2 && xabs <= Prec<R>::thr3) {
    // series branch; its length is uniform across the wavefront
    const bool need2 = __any(xabs > Prec<R>::thr1);
    const bool need3 = __any(xabs > Prec<R>::thr2);
    R sE, sO;
    if (need3) series_sums<Prec<R>::K3>(v, sE, sO);
    else if (need2) series_sums<Prec<R>::K2>(v, sE, sO);
    else series_sums<Prec<R>::K1>(v, sE, sO);
    Dv = sE - sO;
    Ds = sE + sO;
    Gs = R(2) * sO;
  } else {
    o.fallback = 1;
    const R r = opaque(v.rho), ir = opaque(v.irho);
    R sD = R(0), sS = R(0), sG = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R xi = v.x(i, ir), fi = v.fe(i, r);
      const R px = phi_log<R>(xi);
      const R py = phi_log<R>((R(1) - astar) * xi);
      sD += fi * px;
      sS += fi * py;
      sG += fi * (py - px);
    }
    Dv = sD;
    Ds = sS;
    Gs = sG;
  }
  // f = f^eq to rounding: the paper leaves alpha free there; take alpha_*.
  const bool guard = !has_pos || !(Dv > Prec<R>::guard * v.rho);
  o.D = Dv;
  o.guard = guard;
  o.astar_lt2 = !star2;
  o.accepted2 = star2 && (guard || Gs <= R(0));

  R alpha = astar;
  int iters = 0;
  if (!guard) {
    if constexpr (MODE == kClosed) {
      if (Gs > R(0)) {
        // Eq. (9)
        alpha = astar + Gs / Ds * (R(1) - astar);
        alpha = fmin(fmax(alpha, R(1)), astar);
        iters = 1;
      }
    } else if constexpr (MODE == kSecant) {
      if (Gs > R(0)) {
        // alpha^(k+1) = a_* + G(a_*) / (G(a_*) - G(alpha^(k))) (alpha^(k) - a_*),
        // alpha^(0) = 1, so the first iterate is Eq. (9).
        R a = R(1);
        for (int k = 0; k < d.secant_iters; ++k) {
          const R Ga = S_log(v, a) - Dv;
          const R an = astar + Gs / (Gs - Ga) * (a - astar);
          iters = k + 1;
          if (an == a) break;
          a = an;
        }
        alpha = fmin(fmax(a, R(1)), astar);
      }
    } else if constexpr (MODE == kBisect) {
      // Eq. (4) on [1, alpha_max]; first midpoint with -tol <= G <= 0.
      if (S_log(v, amax) - Dv <= R(0)) {
        alpha = amax;
      } else {
        R lo = R(1), hi = amax;
        const R tol = (R)d.root_tol;
        alpha = R(-1);
        for (int k = 1; k <= d.root_max_iter; ++k) {
          const R mid = R(0.5) * (lo + hi);
          const R gm = S_log(v, mid) - Dv;
          iters = k;
          if (gm <= R(0) && gm >= -tol) {
            alpha = mid;
            break;
          }
          if (gm > R(0)) hi = mid;
          else lo = mid;
        }
        if (alpha < R(0)) alpha = lo;
      }
    } else if constexpr (MODE == kNewton) {
      // Eq. (4) by Newton from alpha_* inside the bracket [1, alpha_max].
      if (S_log(v, amax) - Dv <= R(0)) {
        alpha = amax;
      } else {
        R lo = R(1), hi = amax;
        R a = (astar < amax) ? astar : R(0.5) * (lo + hi);
        for (int k = 1; k <= d.root_max_iter; ++k) {
          R Sv, dS;
          S_dS_log(v, a, Sv, dS);
          const R gv = Sv - Dv;
          iters = k;
          if (gv == R(0)) break;
          if (gv > R(0)) hi = a;
          else lo = a;
          R an = a - gv / dS;
          if (!(an > lo && an < hi)) an = R(0.5) * (lo + hi);
          if (fabs(an - a) <= R(1e-15) * a) {
            a = an;
            break;
          }
          a = an;
        }
        alpha = a;
      }
    }
  }
  o.alpha = alpha;
  o.iters = iters;
  return o;
}

struct Acc {
  int c[8];
  double amin, amax, rho, j[3], H;
  __device__ void init() {
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = 0;
    amin = INFINITY;
    amax = -INFINITY;
    rho = j[0] = j[1] = j[2] = H = 0.0;
  }
};

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ int wsumi(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wmin(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Wavefront reductions, then a fixed-order sum over the block's wavefronts:
// the record is a deterministic function of the block's sites.
__device__ void store_partial(const Acc& a, void* partials, int slot) {
  __shared__ int sc[kBlock / 64][8];
  __shared__ double sd[kBlock / 64][8];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int c[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) c[k] = wsumi(a.c[k]);
  const double v0 = wmin(a.amin), v1 = wmax(a.amax), v2 = wsum(a.rho), v3 = wsum(a.j[0]),
               v4 = wsum(a.j[1]), v5 = wsum(a.j[2]), v6 = wsum(a.H);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 8; ++k) sc[w][k] = c[k];
    sd[w][0] = v0; sd[w][1] = v1; sd[w][2] = v2; sd[w][3] = v3;
    sd[w][4] = v4; sd[w][5] = v5; sd[w][6] = v6; sd[w][7] = 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Partial p;
    for (int k = 0; k < 8; ++k) {
      int64_t s = 0;
      for (int q = 0; q < kBlock / 64; ++q) s += sc[q][k];
      p.cnt[k] = s;
    }
    p.amin = sd[0][0]; p.amax = sd[0][1];
    p.rho = sd[0][2]; p.jx = sd[0][3]; p.jy = sd[0][4]; p.jz = sd[0][5]; p.H = sd[0][6];
    for (int q = 1; q < kBlock / 64; ++q) {
      p.amin = fmin(p.amin, sd[q][0]);
      p.amax = fmax(p.amax, sd[q][1]);
      p.rho += sd[q][2]; p.jx += sd[q][3]; p.jy += sd[q][4]; p.jz += sd[q][5]; p.H += sd[q][6];
    }
    p.pad = 0.0;
    reinterpret_cast<Partial*>(partials)[slot] = p;
  }
}

// Quotient of s < 2^31 by n < 2^20 through one FP64 multiply: (s + 1/2)/n is
// at least 1/(2n) away from an integer, far more than the rounding error.
__device__ __forceinline__ uint32_t qdiv(uint32_t s, double inv_n) {
  return (uint32_t)(((double)s + 0.5) * inv_n);
}

// Byte-offset load/store from a uniform plane base: the offset stays a
// 32-bit unsigned VGPR so the address is SGPR base + VGPR offset.
template <class T>
__device__ __forceinline__ T ld(const T* base, uint32_t boff) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + boff);
}
template <class T>
__device__ __forceinline__ void st_nt(T* base, uint32_t boff, T v) {
  __builtin_nontemporal_store(v, reinterpret_cast<T*>(reinterpret_cast<char*>(base) + boff));
}

template <int D, class S, int MODE, class R>
__device__ __forceinline__ void site_update(const SimDesc& d, const typename S::T* __restrict__ src,
                                            typename S::T* __restrict__ dst, uint32_t s,
                                            Acc& acc, int diag) {
  using L = Lattice<D>;
  constexpr int Q = L::Q;
  using T = typename S::T;
  constexpr uint32_t es = sizeof(T);
  const uint32_t nx = (uint32_t)d.nx, ny = (uint32_t)d.ny, nz = (uint32_t)d.nz;
  uint32_t x, y, z;
  if constexpr (D == 1) {
    x = s; y = 0; z = 0;
  } else {
    const uint32_t row = qdiv(s, 1.0 / (double)d.nx);
    x = s - row * nx;
    z = (D == 3) ? qdiv(row, 1.0 / (double)d.ny) : 0u;
    y = row - z * ny;
  }
  // source coordinates for digit 0 (c = 0), 1 (c = +1: pull from -1), 2 (c = -1)
  const uint32_t xs[3] = {x, x == 0 ? nx - 1 : x - 1, x == nx - 1 ? 0 : x + 1};
  const uint32_t ys[3] = {y * nx, (y == 0 ? ny - 1 : y - 1) * nx, (y == ny - 1 ? 0 : y + 1) * nx};
  const uint32_t nxy = nx * ny;
  const uint32_t zs[3] = {z * nxy, (z == 0 ? nz - 1 : z - 1) * nxy, (z == nz - 1 ? 0 : z + 1) * nxy};

  SiteView<D, S, R> v;
  const int64_t pitch = d.pitch;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const uint32_t off = zs[L::dg(i, 2)] + ys[L::dg(i, 1)] + xs[L::dg(i, 0)];
    v.raw[i] = ld(src + (int64_t)i * pitch, off * es);
  }
  v.rho_ref = (R)d.rho_ref;

  // moments
  R rho = R(0), j[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R gi = v.g(i);
    rho += gi;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      if (L::c(i, a) == 1) j[a] += gi;
      if (L::c(i, a) == -1) j[a] -= gi;
    }
  }
  const R irho = R(1) / rho;
  R u[3] = {j[0] * irho, j[1] * irho, j[2] * irho};
  v.rho = rho;
  v.irho = irho;
  const R beta = (R)d.beta;
  const uint32_t so = s * es;  // own site: dst_i(x) is written here
  R alpha = R(2);

  if constexpr (MODE == kBGK) {
    // LBGK: alpha = 2 with the second-order polynomial equilibrium.
    const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const R tb = R(2) * beta;
    int neg = 0, nonfin = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R cu = R(L::c(i, 0)) * u[0] + R(L::c(i, 1)) * u[1] + R(L::c(i, 2)) * u[2];
      const R fe = R(L::W(i)) * rho * (R(1) + R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu);
      const R gi = v.g(i);
      const R ft = gi + tb * (fe - gi);
      if (diag & kDiagCounts) {
        neg += ft < R(0);
        nonfin += !isfinite(ft);
      }
      st_nt(dst + (int64_t)i * pitch, so, Codec<S, R>::enc(ft, R(L::invW(i)), v.rho_ref));
    }
    if (diag & kDiagCounts) {
      acc.c[5] += neg;
      acc.c[6] += nonfin;
    }
  } else {
    v.eq.build(u);
    const AlphaOut<R> ao = choose_alpha<MODE>(v, d);
    alpha = ao.alpha;
    // Eq. (1): f~_i = f_i + alpha beta (f^eq_i - f_i)
    const R ab = alpha * beta;
    const R r = opaque(v.rho);
    int neg = 0, nonfin = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R gi = v.g(i);
      const R ft = fma(ab, v.fe(i, r) - gi, gi);
      if (diag & kDiagCounts) {
        neg += ft < R(0);
        nonfin += !isfinite(ft);
      }
      st_nt(dst + (int64_t)i * pitch, so, Codec<S, R>::enc(ft, R(L::invW(i)), v.rho_ref));
    }
    if (diag & kDiagCounts) {
      acc.c[0] += ao.accepted2;
      acc.c[1] += ao.astar_lt2;
      acc.c[2] += alpha < R(2);
      acc.c[3] += ao.guard;
      acc.c[4] += ao.fallback;
      acc.c[5] += neg;
      acc.c[6] += nonfin;
      acc.c[7] += ao.iters;
      if (diag & kDiagEntropy) {
        // H(f) = H(f^eq) + D, H(f^eq) = rho [ln rho + sum_a (ln A_a + u_a ln z_a)]
        double h = log((double)rho);
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const double ua = (double)u[a];
          const double sa = sqrt(1.0 + 3.0 * ua * ua);
          h += log(2.0 - sa) + ua * log((2.0 * ua + sa) / (1.0 - ua));
        }
        acc.H += (double)rho * h + (double)ao.D;
      }
    }
  }
  if (diag & kDiagAlpha) d.alpha[s] = (double)alpha;
  if (diag & kDiagCounts) {
    acc.amin = fmin(acc.amin, (double)alpha);
    acc.amax = fmax(acc.amax, (double)alpha);
    acc.rho += (double)rho;
#pragma unroll
    for (int a = 0; a < D; ++a) acc.j[a] += (double)j[a];
  }
}

// One workgroup = one tile of kBlock consecutive sites.  Workgroups are
// issued round-robin over the 8 XCDs (workgroup b runs on XCD b mod 8), so
// the tile order is permuted to give each XCD one contiguous eighth of the
// box: neighbouring tiles, which share the cache lines at their x-edges,
// then run on the same XCD and L2.  Each simulation's workgroup count is a
// multiple of 8 and starts at a multiple of 8.
template <int D, class S, int MODE, class R>
__global__ void __launch_bounds__(kBlock) k_step(const BatchArgs args) {
  using T = typename S::T;
  const int b = blockIdx.x;
  int si = 0;
  for (int k = 1; k < args.n; ++k)
    if (b >= args.d[k].block_begin) si = k;
  const SimDesc& d = args.d[si];
  const T* __restrict__ src = static_cast<const T*>(d.src);
  T* __restrict__ dst = static_cast<T*>(d.dst);
  const uint32_t lb = (uint32_t)(b - d.block_begin);
  const uint32_t chunk = (uint32_t)d.nblocks >> 3;
  const uint32_t tile = (lb & 7u) * chunk + (lb >> 3);
  const int diag = d.diag;
  const uint32_t N = (uint32_t)d.nx * (uint32_t)d.ny * (uint32_t)d.nz;
  const uint32_t s = tile * kBlock + threadIdx.x;
  Acc acc;
  acc.init();
  if (s < N) site_update<D, S, MODE, R>(d, src, dst, s, acc, diag);
  if (diag & kDiagCounts) store_partial(acc, d.partials, (int)lb);
}

template <int D, class S, int MODE, class R>
hipError_t launch_step(const BatchArgs& a, int grid, hipStream_t st) {
  k_step<D, S, MODE, R><<<grid, kBlock, 0, st>>>(a);
  return hipGetLastError();
}

template <int D>
StepLauncher step_launcher_for(int storage, int mode, int fp64) {
#define ELBM_MODES(S, R)                                      \
  switch (mode) {                                             \
    case kClosed: return &launch_step<D, S, kClosed, R>;      \
    case kNewton: return &launch_step<D, S, kNewton, R>;      \
    case kBisect: return &launch_step<D, S, kBisect, R>;      \
    case kBGK: return &launch_step<D, S, kBGK, R>;            \
    case kSecant: return &launch_step<D, S, kSecant, R>;      \
    default: return nullptr;                                  \
  }
  if (fp64) {
    switch (storage) {
      case kStoreF64: ELBM_MODES(StoreF64, double)
      case kStoreF32: ELBM_MODES(StoreF32, double)
      case kStoreF32Dev: ELBM_MODES(StoreF32Dev, double)
      case kStoreF16Dev: ELBM_MODES(StoreF16Dev, double)
      default: return nullptr;
    }
  }
#undef ELBM_MODES
  if (mode != kClosed) return nullptr;
  switch (storage) {
    case kStoreF32: return &launch_step<D, StoreF32, kClosed, float>;
    case kStoreF32Dev: return &launch_step<D, StoreF32Dev, kClosed, float>;
    case kStoreF16Dev: return &launch_step<D, StoreF16Dev, kClosed, float>;
    default: return nullptr;
  }
}

}  // namespace elbm
