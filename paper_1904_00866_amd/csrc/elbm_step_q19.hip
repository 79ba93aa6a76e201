// elbm_step_q19.hip -- the fused pull-stream + collide kernel on the D3Q19
// lattice.
//
// Same step as on the tensor-product lattices (pull, moments, equilibrium,
// alpha, Eq. (1), store; one launch per time step for up to kMaxBatch
// simulations, 2 Q b bytes per site update), with two differences:
//   - the equilibrium is the minimiser of Eq. (3) under the moment
//     constraints found per site by Newton's method on the Lagrange
//     multipliers (EquilibriumQ19): the D3Q19 weights do not factorise, so
//     there is no closed product form;
//   - f^eq_i is still a product of per-axis factors exp(l_a c_ia) times a
//     weight that depends on the number of nonzero components of c_i, so the
//     site keeps two 3 x 3 tables over (c_x, c_y) -- one for c_z = 0, one
//     for c_z != 0 -- and the two z-axis factors; 1/f^eq_i comes from the
//     opposite direction's f^eq.
// The choice of alpha (tiers, modes, diagnostics) is the lattice-independent
// code of the tensor-product kernel.
#include "elbm_q19.hpp"
#include "elbm_step_impl.hpp"

namespace elbm {
namespace {

using L19 = LatticeQ19;

// D3Q19 direction of the D3Q27 index j (j not a corner).
__host__ __device__ constexpr int q19_of(int j) {
  return j - 2 * (j >= 13) - 2 * (j >= 18) - 2 * (j >= 22);
}
static_assert(q19_of(L19::q27(13)) == 13 && q19_of(L19::q27(18)) == 18 &&
                  q19_of(L19::q27(14)) == 14 && q19_of(L19::q27(12)) == 12,
              "D3Q19 index maps");

// 9 W for n nonzero components (3, 1/2, 1/4) and its reciprocal
__host__ __device__ constexpr double w9(int n) { return n == 0 ? 3.0 : n == 1 ? 0.5 : 0.25; }
__host__ __device__ constexpr double iw9(int n) { return n == 0 ? 1.0 / 3.0 : n == 1 ? 2.0 : 4.0; }

// Opposite digit: c -> -c swaps the digits 1 and 2.
__host__ __device__ constexpr int opp(int d) { return d == 0 ? 0 : 3 - d; }

template <class S, class R>
struct SiteQ19 {
  using L = L19;
  using T = typename S::T;
  using Real = R;
  static constexpr int Q = 19;
  static constexpr int kDim = 3;
  static constexpr bool kZFactor = false;
  // FP16 deviation storage with FP64 arithmetic: the closed form's common
  // tier takes its first-term sums from the deviations (sums_k1)
  static constexpr bool kSumsK1 =
      sizeof(T) == 2 && S::dev && std::is_same<R, double>::value;
  using Arith = R;
  typename Kept<S>::type raw[Q];  // the loaded populations as kept (Kept<S>)
  R rho, irho, rho_ref;
  R rhoA;   // rho, for the first-term tier's guard
  R dd[Q];  // s_i - s^eq_i as sums_k1 formed them, for the collision
  R u[3];
  // f^eq_i = F0[dx][dy] (c_z = 0) or F1[dx][dy] e2[dz] (c_z != 0); the
  // corner entries of F1 (no such direction) are zero.  Since
  // f^eq_i f^eq_{-i} = (rho W_i / Z)^2, the reciprocal is
  // 1/f^eq_i = kap[n] f^eq_{-i}, kap[n] = (Z / (rho W_i))^2 for n nonzero
  // components of c_i: no table of reciprocals is kept.
  R F0[3][3], F1[3][3];
  R e2[3];
  R kap[3];
  R Z9, X[3];  // for H(f^eq) (diagnostic sums)
  const T* src;
  uint32_t site;
  const SimDesc* desc;
  Where w;

  __device__ __forceinline__ R g(int i) const {
    return Codec<S, R>::dec_wide(widen<R>(raw[i]), R(L::W(i)), rho_ref);
  }
  struct Pass {
    R e2[3];
  };
  __device__ __forceinline__ Pass pass_opaque() const {
    Pass p;
#pragma unroll
    for (int k = 0; k < 3; ++k) p.e2[k] = opaque(e2[k]);
    return p;
  }
  __device__ __forceinline__ Pass pass() const {
    if constexpr (sizeof(T) == 8) return pass_opaque();
    Pass p;
#pragma unroll
    for (int k = 0; k < 3; ++k) p.e2[k] = e2[k];
    return p;
  }
  // f^eq of the direction with digits (dx, dy, dz)
  __device__ __forceinline__ R fd(int dx, int dy, int dz, const Pass& p) const {
    return dz == 0 ? F0[dx][dy] : F1[dx][dy] * p.e2[dz];
  }
  __device__ __forceinline__ R fe(int i, const Pass& p) const {
    return fd(L::dg(i, 0), L::dg(i, 1), L::dg(i, 2), p);
  }
  __device__ __forceinline__ R x(int i, const Pass& p) const {
    const R rf = fd(opp(L::dg(i, 0)), opp(L::dg(i, 1)), opp(L::dg(i, 2)), p) * kap[L::nnz(i)];
    return fma(g(i), rf, R(-1));
  }
  // The closed form's common tier on 2-byte deviation storage: the sums to
  // their first terms, E = sum_i f^eq_i x_i^2 / 2 and O = sum_i f^eq_i x_i^3 / 6,
  // and max_i |x_i|.  With the stored deviations s_i = f_i / W_i - rho_ref and
  // d_i = s_i - s^eq_i, f^eq_i x_i = f_i - f^eq_i = W_i d_i and
  // x_i = d_i W_i / f^eq_i = d_i (W_i kap[n]) f^eq_{-i}, so E and O are sums
  // of d_i x_i and d_i x_i^2 per weight class (n nonzero components),
  // weighted once at the end.
  __device__ __forceinline__ void sums_k1(const Pass& p, R& sE, R& sO, R& xabs) {
    static_assert(kSumsK1, "first-term sums on 2-byte deviation storage");
    R kw[3], e[3], o[3], xm = R(0);
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      kw[n] = R(n == 0 ? 1.0 / 3.0 : n == 1 ? 1.0 / 18.0 : 1.0 / 36.0) * kap[n];
      e[n] = o[n] = R(0);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int n = L::nnz(i);
      const R seq = fma(fe(i, p), R(L::invW(i)), -rho_ref);
      const R di = widen<R>(raw[i]) - seq;
      dd[i] = di;
      const R xi = di * (fd(opp(L::dg(i, 0)), opp(L::dg(i, 1)), opp(L::dg(i, 2)), p) * kw[n]);
      const R t = di * xi;
      e[n] += t;
      o[n] = fma(t, xi, o[n]);
      xm = fmax(xm, fabs(xi));
    }
    R E = R(0), O = R(0);
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const R w = R(n == 0 ? 1.0 / 3.0 : n == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
      E = fma(w, e[n], E);
      O = fma(w, o[n], O);
    }
    sE = R(0.5) * E;
    sO = O * R(1.0 / 6.0);
    xabs = xm;
  }

  __device__ __forceinline__ void fold(const EquilibriumQ19<R>& eq) {
    const R cF = rho * rcp_n<R>(eq.Z9), cG = eq.Z9 * irho;
    const R e0[3] = {R(1), eq.X[0], eq.Y[0]}, e1[3] = {R(1), eq.X[1], eq.Y[1]};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const int n = (a != 0) + (b != 0);
        F0[a][b] = (cF * R(w9(n))) * (e0[a] * e1[b]);
        F1[a][b] = n < 2 ? (cF * R(w9(n + 1))) * (e0[a] * e1[b]) : R(0);
      }
    e2[0] = R(1);
    e2[1] = eq.X[2];
    e2[2] = eq.Y[2];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const R k = cG * R(iw9(n));
      kap[n] = k * k;
    }
    Z9 = eq.Z9;
#pragma unroll
    for (int a = 0; a < 3; ++a) X[a] = eq.X[a];
  }

  // H(f^eq) / rho = ln rho - ln Z + l.u
  __device__ __forceinline__ double heq_per_rho() const {
    double h = log((double)rho) - log((double)Z9 / 9.0);
#pragma unroll
    for (int a = 0; a < 3; ++a) h += (double)u[a] * log((double)X[a]);
    return h;
  }

  // run-time (wavefront-uniform) i: the population is re-read from the
  // source buffer, as on the tensor-product lattices
  __device__ __forceinline__ R fsel(int dx, int dy, int dz) const {
    return dz == 0 ? sel9(F0, dx, dy) : sel9(F1, dx, dy) * sel3(e2, dz);
  }
  __device__ __forceinline__ void xfe(int i, R& xi, R& fi, R* gout = nullptr) const {
    const int j = L::q27(i);
    const int dx = j % 3, dy = (j / 3) % 3, dz = j / 9;
    const int n = (dx != 0) + (dy != 0) + (dz != 0);
    const R W = n == 0 ? R(1.0 / 3.0) : n == 1 ? R(1.0 / 18.0) : R(1.0 / 36.0);
    const uint32_t sp = sel3(w.zs, dz) + sel3(w.ys, dy) + sel3(w.xs, dx);
    const T gv = *(const gptr<T>)((gaddr)(uintptr_t)src + pidx<Q>(sp, i) * sizeof(T));
    const R gi = Codec<S, R>::dec(gv, W, rho_ref);
    fi = fsel(dx, dy, dz);
    const R rf = fsel(opp(dx), opp(dy), opp(dz)) * sel3(kap, n);
    xi = fma(gi, rf, R(-1));
    if (gout) *gout = gi;
  }
};

// Pull of the 19 populations when the wavefront's 64 sites lie in one x-row
// (nx a multiple of 64): one descriptor per source row (c_y, c_z), the three
// x positions as per-lane offsets (see load_site_row).
template <class T>
__device__ __forceinline__ void load_row_q19(const SimDesc& d, const T* src, uint32_t s,
                                             T (&raw)[19]) {
  const uint32_t nx = (uint32_t)d.nx, ny = (uint32_t)d.ny, nz = (uint32_t)d.nz;
  const uint32_t row = __builtin_amdgcn_readfirstlane(qdiv(s, d.inv_nx));
  const uint32_t x = s - row * nx;
  const uint32_t z = __builtin_amdgcn_readfirstlane(qdiv(row, d.inv_ny));
  const uint32_t y = row - z * ny;
  uint32_t ys[3], zs[3];
  ys[0] = y * nx;
  ys[1] = (y == 0 ? ny - 1 : y - 1) * nx;
  ys[2] = (y == ny - 1 ? 0 : y + 1) * nx;
  const uint32_t nxy = nx * ny;
  zs[0] = z * nxy;
  zs[1] = (z == 0 ? nz - 1 : z - 1) * nxy;
  zs[2] = (z == nz - 1 ? 0 : z + 1) * nxy;
  constexpr uint32_t es = sizeof(T);
  constexpr int Q = 19;
  uint32_t xo[3];
  const uint32_t xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  xo[0] = (uint32_t)pidx<Q>(x, 0) * es;
  xo[1] = (uint32_t)pidx<Q>(xm, 0) * es;
  xo[2] = (uint32_t)pidx<Q>(xp, 0) * es;
  const gaddr base = buffer_base(src);
  const uint32_t rowbytes = nx * (uint32_t)Q * es;
#pragma unroll
  for (int dz = 0; dz < 3; ++dz)
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const __amdgpu_buffer_rsrc_t r = rsrc(base + (uint64_t)(zs[dz] + ys[dy]) * Q * es, rowbytes);
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        if (dx != 0 && dy != 0 && dz != 0) continue;  // corner: not a D3Q19 direction
        const int i = q19_of(dx + 3 * dy + 9 * dz);
        raw[i] = ld_buf<T>(r, xo[dx], (uint32_t)i * kLane * es);
      }
    }
}

// Pull of the 19 populations of site s (s < N): raw_i = src_i(x - c_i).
template <class T>
__device__ __forceinline__ void load_q19(const SimDesc& d, const T* src, uint32_t s,
                                         T (&raw)[19]) {
  const Where w = locate<3>(d, s);
  const gaddr base = buffer_base(src);
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const uint32_t sp = w.zs[L19::dg(i, 2)] + w.ys[L19::dg(i, 1)] + w.xs[L19::dg(i, 0)];
    raw[i] = *(const gptr<T>)(base + pidx<19>(sp, i) * sizeof(T));
  }
}

// First direction with a nonzero component a.
__host__ __device__ constexpr int first_nz(int a) {
  int i = 0;
  while (L19::c(i, a) == 0) ++i;
  return i;
}

// rho and rho u; each sum starts from its first term.
template <class S, class R>
__device__ __forceinline__ void moments_q19(const SiteQ19<S, R>& v, R& rho, R (&j)[3]) {
  j[0] = j[1] = j[2] = R(0);
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const R gi = v.g(i);
    rho = i == 0 ? gi : rho + gi;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int c = L19::c(i, a);
      if (c != 0)
        j[a] = i == first_nz(a) ? (c > 0 ? gi : -gi) : (c > 0 ? j[a] + gi : j[a] - gi);
    }
  }
}

template <class S, class R>
__device__ __forceinline__ void prepare_q19(SiteQ19<S, R>& v, const SimDesc& d,
                                            const typename S::T* src, uint32_t sl, R& rho,
                                            R (&j)[3], bool equilibrium) {
  v.src = src;
  v.site = sl;
  v.desc = &d;
  v.rho_ref = (R)d.rho_ref;
  moments_q19(v, rho, j);
  const R irho = rcp_n<R>(rho);
  v.rho = rho;
  v.rhoA = rho;
  v.irho = irho;
#pragma unroll
  for (int a = 0; a < 3; ++a) v.u[a] = j[a] * irho;
  if (equilibrium) {
    EquilibriumQ19<R> eq;
    eq.build(v.u);
    v.fold(eq);
  }
}

// One site: moments, equilibrium, alpha, Eq. (1), store (see site_update).
template <class S, int MODE, class R, bool SUMS, int PHASE = kPhaseAll>
__device__ __forceinline__ SiteOut update_q19(const SimDesc& d, const typename S::T* __restrict__ src,
                                              typename S::T* __restrict__ dst, uint32_t s, bool live,
                                              const typename S::T (&raw)[19], Acc& acc, int diag) {
  constexpr int Q = 19;
  using T = typename S::T;
  constexpr uint32_t es = sizeof(T);
  const uint32_t sl = live ? s : 0u;
  SiteQ19<S, R> v;
#pragma unroll
  for (int i = 0; i < Q; ++i) v.raw[i] = Codec<S, R>::keep(raw[i]);
  R rho, j[3];
  prepare_q19(v, d, src, sl, rho, j, MODE != kBGK);
  const R beta = (R)d.beta;
  const uint32_t lo = (s & 63u) * es;
  const gaddr blk = block_base<Q>(dst, s);

  if constexpr (MODE == kBGK) {
    // LBGK: alpha = 2 with the second-order polynomial equilibrium.
    const R* u = v.u;
    const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const R tb = R(2) * beta;
    R ftmin = R(INFINITY);
    uint32_t flags = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R cu = R(L19::c(i, 0)) * u[0] + R(L19::c(i, 1)) * u[1] + R(L19::c(i, 2)) * u[2];
      const R fe = R(L19::W(i)) * rho * (R(1) + R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu);
      const R gi = v.g(i);
      const R ft = gi + tb * (fe - gi);
      ftmin = fmin(ftmin, ft);
      st_nt<T>(blk + i * kLane * es, kLane * es, lo, Codec<S, R>::enc(ft, R(L19::invW(i)), v.rho_ref));
    }
    if (diag & kDiagCounts) {
      if (live)
        flags = flag(kCntNeg, ftmin < R(0)) |
                flag(kCntNonfinite, !isfinite(rho * u[0] * u[1] * u[2] + rho));
    }
    if (diag & kDiagAlpha) d.alpha[s] = 2.0;
    if (live && (diag & kDiagCounts)) {
      acc.amin = fminf(acc.amin, 2.0f);
      acc.amax = fmaxf(acc.amax, 2.0f);
      if (SUMS && (diag & kDiagSums)) {
        acc.rho += (double)rho;
#pragma unroll
        for (int a = 0; a < 3; ++a) acc.j[a] += (double)j[a];
      }
    }
    return SiteOut{false, flags};
  } else {
    const AlphaOut<R> ao = choose_alpha<MODE, PHASE>(v, d);
    if (PHASE == kPhaseCommon && ao.deferred) return SiteOut{true, 0u};
    const R ab = ao.alpha * beta;
    const auto P = v.pass();
    R ftmin = R(INFINITY);
    // the common phase of the closed form on 2-byte deviation storage takes
    // s_i - s^eq_i from its sums (sums_k1): s~_i = s_i - alpha beta d_i
    constexpr bool kDD = SiteQ19<S, R>::kSumsK1 && MODE == kClosed && PHASE == kPhaseCommon;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if constexpr (kDD) {
        float h = float(fma(-ab, v.dd[i], widen<R>(v.raw[i])));
        asm volatile("" : "+v"(h));  // two roundings, as Codec::enc takes them
        st_nt<T>(blk + i * kLane * es, kLane * es, lo, T(h));
      } else {
        const R gi = v.g(i);
        const R ft = fma(ab, v.fe(i, P) - gi, gi);
        // common and middle tiers: |x_i| <= 0.025, no negative population
        if constexpr (PHASE != kPhaseCommon) ftmin = fmin(ftmin, ft);
        st_nt<T>(blk + i * kLane * es, kLane * es, lo, Codec<S, R>::enc(ft, R(L19::invW(i)), v.rho_ref));
      }
    }
    return SiteOut{false, record_site<SUMS>(d, s, live, v, ao, ftmin, j, acc, diag)};
  }
}

// A lane deferred by the common phase (see site_update_rare).
template <class S, int MODE, class R, bool SUMS>
__device__ __forceinline__ uint32_t update_rare_q19(const SimDesc& d,
                                                    const typename S::T* __restrict__ src,
                                                    typename S::T* __restrict__ dst, uint32_t s,
                                                    bool live, Acc& acc, int diag) {
  constexpr int Q = 19;
  using T = typename S::T;
  constexpr uint32_t es = sizeof(T);
  const uint32_t sl = live ? s : 0u;
  SiteQ19<S, R> v;
  if constexpr (Codec<S, R>::kF16) {
    T raw[Q];
    load_q19(d, src, sl, raw);
#pragma unroll
    for (int i = 0; i < Q; ++i) v.raw[i] = Codec<S, R>::keep(raw[i]);
  } else {
    load_q19(d, src, sl, v.raw);
  }
  R rho, j[3];
  prepare_q19(v, d, src, sl, rho, j, true);
  const AlphaOut<R> ao = choose_alpha<MODE, kPhaseRare>(v, d);
  const R ab = ao.alpha * (R)d.beta;
  R ftmin = R(INFINITY);
  const uint32_t lo = (s & 63u) * es;
  const gaddr blk = block_base<Q>(dst, s);
#pragma unroll 1
  for (int i = 0; i < Q; ++i) {
    R xi, fi, gi;
    v.xfe(i, xi, fi, &gi);
    const R ft = fma(ab, fi - gi, gi);
    ftmin = fmin(ftmin, ft);
    const int jj = L19::q27(i);
    const int n = (jj % 3 != 0) + ((jj / 3) % 3 != 0) + (jj / 9 != 0);
    const R invW = n == 0 ? R(3) : n == 1 ? R(18) : R(36);
    st_nt<T>(blk + (uint64_t)i * kLane * es, kLane * es, lo, Codec<S, R>::enc(ft, invW, v.rho_ref));
  }
  return record_site<SUMS>(d, s, live, v, ao, ftmin, j, acc, diag);
}

// The step kernel: the workgroup, tile and XCD-aware order of k_step.
template <class S, int MODE, class R, bool SUMS>
__global__ void __launch_bounds__(kBlock, (step_waves<S, MODE>())) k_step_q19(const BatchArgs args) {
  using T = typename S::T;
  constexpr int Q = 19;
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
    T raw[ELBM_TILES][Q];
#if ELBM_LOAD_PRIO
    __builtin_amdgcn_s_setprio(ELBM_LOAD_PRIO);
#endif
#pragma unroll
    for (int k = 0; k < ELBM_TILES; ++k) {
      const uint32_t s = (unit * ELBM_TILES + k) * kBlock + threadIdx.x;
      if (d.nx % 64 == 0)
        load_row_q19(d, src, s < N ? s : 0u, raw[k]);
      else
        load_q19(d, src, s < N ? s : 0u, raw[k]);
    }
#if ELBM_LOAD_PRIO
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_setprio(0);
#endif
    uint32_t flags = 0;
    if constexpr (MODE == kClosed) {
      constexpr uint32_t kCommonFlags =
          (1u << kCntAccept2) | (1u << kCntAlphaLt2) | (1u << kCntGuard);
      bool deferred[ELBM_TILES];
#pragma unroll
      for (int k = 0; k < ELBM_TILES; ++k) {
        const uint32_t s = (unit * ELBM_TILES + k) * kBlock + threadIdx.x;
        deferred[k] = false;
        if (k == 0 || (unit * ELBM_TILES + k) * kBlock < N) {
          const SiteOut o =
              update_q19<S, MODE, R, SUMS, kPhaseCommon>(d, src, dst, s, s < N, raw[k], acc, diag);
          deferred[k] = o.deferred;
          flags = o.flags;
        }
        if (diag & kDiagCounts) acc.count_flags<kCommonFlags>(flags);
        flags = 0;
      }
#pragma unroll
      for (int k = 0; k < ELBM_TILES; ++k) {
        if (__any(deferred[k])) {
          uint32_t f = 0;
          if (deferred[k]) {
            const uint32_t s = (unit * ELBM_TILES + k) * kBlock + threadIdx.x;
            f = update_rare_q19<S, MODE, R, SUMS>(d, src, dst, s, s < N, acc, diag);
          }
          if (diag & kDiagCounts) acc.count_flags(f);
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < ELBM_TILES; ++k) {
        const uint32_t s = (unit * ELBM_TILES + k) * kBlock + threadIdx.x;
        if (k == 0 || (unit * ELBM_TILES + k) * kBlock < N)
          flags = update_q19<S, MODE, R, SUMS>(d, src, dst, s, s < N, raw[k], acc, diag).flags;
        if (diag & kDiagCounts) acc.count_flags(flags);
        flags = 0;
      }
    }
  } else if (!(diag & kDiagCounts)) {
    return;  // padding workgroup
  }
  if (diag & kDiagCounts)
    store_records<MODE == kNewton || MODE == kBisect || MODE == kSecant>(acc, d, (int)lb);
}

template <class S, int MODE, class R>
hipError_t launch_q19(const BatchArgs& a, int grid, hipStream_t st) {
  bool sums = false;
  for (int k = 0; k < a.n; ++k) sums = sums || (a.d[k].diag & kDiagSums);
  if (sums)
    k_step_q19<S, MODE, R, true><<<grid, kBlock, 0, st>>>(a);
  else
    k_step_q19<S, MODE, R, false><<<grid, kBlock, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace

StepLauncher step_launcher_q19(int storage, int mode, int fp64) {
#define ELBM_MODES(S, R)                                 \
  switch (mode) {                                        \
    case kClosed: return &launch_q19<S, kClosed, R>;     \
    case kNewton: return &launch_q19<S, kNewton, R>;     \
    case kBisect: return &launch_q19<S, kBisect, R>;     \
    case kBGK: return &launch_q19<S, kBGK, R>;           \
    case kSecant: return &launch_q19<S, kSecant, R>;     \
    default: return nullptr;                             \
  }
  if (fp64 == kArithF64) {
    switch (storage) {
      case kStoreF64: ELBM_MODES(StoreF64, double)
      case kStoreF32: ELBM_MODES(StoreF32, double)
      case kStoreF32Dev: ELBM_MODES(StoreF32Dev, double)
      case kStoreF16Dev: ELBM_MODES(StoreF16Dev, double)
      default: return nullptr;
    }
  }
#undef ELBM_MODES
  if (mode != kClosed || fp64 != kArithF32) return nullptr;
  switch (storage) {
    case kStoreF32: return &launch_q19<StoreF32, kClosed, float>;
    case kStoreF32Dev: return &launch_q19<StoreF32Dev, kClosed, float>;
    case kStoreF16Dev: return &launch_q19<StoreF16Dev, kClosed, float>;
    default: return nullptr;
  }
}

}  // namespace elbm
