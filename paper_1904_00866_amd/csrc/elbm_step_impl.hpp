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
//
// Register budget.  The populations stay in registers in their storage type;
// x_i and f^eq_i are recomputed from per-axis factors wherever they are
// needed instead of being kept (Q doubles each).  The common case -- alpha_* =
// 2 and max_i |x_i| small -- is one unrolled pass with a short series.  Rare
// cases (a longer series, the log1p forms, the root solvers) run as
// non-unrolled loops over the directions so they add little register
// pressure to the common path.
#pragma once

#include <type_traits>

#include "elbm_internal.hpp"
#include "elbm_site.hpp"


namespace elbm {

// Keeps a value in registers but hides it from the optimiser, so that
// quantities derived from it are recomputed where they are used instead of
// being kept live (register pressure decides the occupancy of this kernel).
template <class R>
__device__ __forceinline__ R opaque(R v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Wave priority while a wave issues its loads.  A wave that starts raises
// its priority until its Q loads are issued, so the instruction arbiter
// issues them ahead of the arithmetic of the waves already computing: the
// loads of the next tiles then overlap that arithmetic instead of waiting
// behind it (512^3 D3Q27 closed form: 5.26 -> 5.07 ms per step).
#ifndef ELBM_LOAD_PRIO
#define ELBM_LOAD_PRIO 2
#endif
// Scheduling fence every ELBM_SCHED_GROUP directions of an unrolled pass
// (0: none): keeps the scheduler from hoisting the loads and conversions of
// many directions at once, which would hold their registers live.
#ifndef ELBM_SCHED_GROUP
#define ELBM_SCHED_GROUP 0
#endif
// Scheduling fence after each group of directions of a Newton pass (0:
// none): bounds how many directions' logarithms the scheduler interleaves,
// and with it the registers they hold.
#ifndef ELBM_NEWTON_FENCE
#define ELBM_NEWTON_FENCE 1
#endif
#ifndef ELBM_NEWTON_OPAQUE
#define ELBM_NEWTON_OPAQUE 1
#endif
__device__ __forceinline__ void sched_group(int i) {
  if (ELBM_SCHED_GROUP > 0 && i % (ELBM_SCHED_GROUP > 0 ? ELBM_SCHED_GROUP : 1) ==
                                  (ELBM_SCHED_GROUP > 0 ? ELBM_SCHED_GROUP : 1) - 1)
    __builtin_amdgcn_sched_barrier(0);
}

// The stored population widened to the arithmetic type.  FP32 -> FP64 goes
// through a volatile asm conversion: the compiler can neither merge the
// conversions of different passes (which would keep Q doubles live) nor needs
// to copy the source register first, as an opaque() barrier would.
template <class R, class T>
__device__ __forceinline__ auto widen(T v) {
  if constexpr (std::is_same<T, float>::value && std::is_same<R, double>::value) {
    double d;
    asm volatile("v_cvt_f64_f32 %0, %1" : "=v"(d) : "v"(v));
    return d;
  } else if constexpr (std::is_same<T, _Float16>::value && std::is_same<R, double>::value) {
    const float f = (float)v;
    double d;
    asm volatile("v_cvt_f64_f32 %0, %1" : "=v"(d) : "v"(f));
    return d;
  } else if constexpr (std::is_same<T, _Float16>::value) {
    return (float)v;
  } else {
    return v;
  }
}

template <class R>
__device__ __forceinline__ R sel3(const R (&a)[3], int d) {
  return d == 0 ? a[0] : (d == 1 ? a[1] : a[2]);
}
template <class R>
__device__ __forceinline__ R sel9(const R (&a)[3][3], int dx, int dy) {
  return sel3(a[0], dy) * R(dx == 0) + sel3(a[1], dy) * R(dx == 1) + sel3(a[2], dy) * R(dx == 2);
}

// Series lengths of the three tiers and their validity bounds on
// max_i |x_i|: truncating E and O after K terms changes alpha by about
// 2 x^(2K+1)/((2K+3)(2K+2)), kept below 2^-53 (FP64) or 2^-24 (FP32).
//   common tier: K terms, one unrolled pass fused with the x range;
//   middle tier: KM terms, one more unrolled pass for wavefronts that need it;
//   rare tier:   KL terms (or the log1p forms beyond thrL, or when
//                alpha_* < 2), a rolled loop for the lanes that need it.
template <class R>
struct Base;
#ifndef ELBM_BASE_K
#define ELBM_BASE_K 3
#endif
template <>
struct Base<double> {
  static constexpr int K = ELBM_BASE_K;
  // 2^-53 bound of the common tier for K = 2, 3, 4
  static constexpr double thr = K <= 2 ? 1.15e-3 : (K == 3 ? 8.5e-3 : 0.025);
  static constexpr int KM = 4;
  static constexpr double thrM = 0.025;
  static constexpr int KL = 14;
  static constexpr double thrL = 0.30;
};
template <>
struct Base<float> {
  static constexpr int K = 2;
  static constexpr float thr = 0.06f;
  static constexpr int KM = 4;
  static constexpr float thrM = 0.24f;
  static constexpr int KL = 7;
  static constexpr float thrL = 0.30f;
};

// Addressing.  Bases are uniform (scalar registers) and a lane's byte
// offset a 32-bit vector register, so loads and stores take the
// scalar-base + vector-offset form.  The buffer base is passed through
// in_sgpr() once per tile and the per-direction bases are formed with
// scalar adds; the explicit global address space keeps the accesses global
// rather than generic.
using gaddr = uint64_t;
template <class T>
using gptr = __attribute__((address_space(1))) T*;

template <class T>
__device__ __forceinline__ gaddr buffer_base(const T* buf) {
  return in_sgpr((gaddr)(uintptr_t)buf);
}
// Load of one population as a raw buffer load from a range of `bytes`
// bytes at `base` (scalar descriptor, vector byte offset); an offset past
// the range reads 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(gaddr base, uint32_t bytes) {
  // word 3: 32-bit data format, the raw-buffer setting of this architecture
  return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(base), (short)0, (int)bytes,
                                           0x00020000);
}
// soff: a uniform byte offset added to the base (scalar operand)
template <class T>
__device__ __forceinline__ T ld_buf(__amdgpu_buffer_rsrc_t r, uint32_t boff, uint32_t soff) {
  if constexpr (sizeof(T) == 8) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, boff, soff, 0));
  } else if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, boff, soff, 0));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, boff, soff, 0));
  }
}

// A loaded population as the loaders hand it to the site update: 2-byte
// values are held zero-extended, one per 32-bit register.  Kept as 16-bit
// values, they are packed two to a register as soon as they arrive, so the
// wavefront waits for each group of loads before it issues the next and the
// loads of several tiles are no longer in flight together.
template <class T>
using Slot = typename std::conditional<sizeof(T) == 2, uint32_t, T>::type;
template <class T>
__device__ __forceinline__ Slot<T> ld_slot(__amdgpu_buffer_rsrc_t r, uint32_t boff, uint32_t soff) {
  if constexpr (sizeof(T) == 2) return uint32_t(__builtin_amdgcn_raw_buffer_load_b16(r, boff, soff, 0));
  else return ld_buf<T>(r, boff, soff);
}
template <class T>
__device__ __forceinline__ T from_slot(Slot<T> v) {
  if constexpr (sizeof(T) == 2) return __builtin_bit_cast(T, uint16_t(v));
  else return v;
}

// Non-temporal store of one population into a range of `bytes` bytes at
// `base`, as a raw buffer store: the descriptor is formed in scalar
// registers and the lane's byte offset is the only vector operand, so a
// store costs no vector address arithmetic.  An offset at or past `bytes`
// is discarded by the hardware range check.
template <class T>
__device__ __forceinline__ void st_nt(gaddr base, uint32_t bytes, uint32_t boff, T v) {
  const __amdgpu_buffer_rsrc_t r = rsrc(base, bytes);
  constexpr int kNT = 2;  // cache policy: non-temporal
  if constexpr (sizeof(T) == 8) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, boff, 0, kNT);
  } else if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, boff, 0, kNT);
  } else {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, boff, 0, kNT);
  }
}

// Byte address of the block that holds the wavefront's 64 sites in `buf`
// (the sites of a wavefront are 64 consecutive, 64-aligned indices, so the
// block is uniform).
template <int Q, class T>
__device__ __forceinline__ gaddr block_base(const T* buf, uint32_t s) {
  const uint32_t blk = __builtin_amdgcn_readfirstlane(s >> 6);
  return buffer_base(buf) + (uint64_t)blk * ((uint64_t)Q * kLane * sizeof(T));
}

// Quotient of s < 2^31 by n < 2^20 through one FP64 multiply: (s + 1/2)/n is
// at least 1/(2n) away from an integer, far more than the rounding error.
__device__ __forceinline__ uint32_t qdiv(uint32_t s, double inv_n) {
  return (uint32_t)(((double)s + 0.5) * inv_n);
}

// Source coordinates of one site for digit 0 (c = 0), 1 (c = +1: pull from
// -1) and 2 (c = -1), as element offsets: x, y * nx, z * nx * ny.
struct Where {
  uint32_t xs[3], ys[3], zs[3];
};

template <int D>
__device__ __forceinline__ Where locate(const SimDesc& d, uint32_t s) {
  const uint32_t nx = (uint32_t)d.nx, ny = (uint32_t)d.ny, nz = (uint32_t)d.nz;
  uint32_t x, y, z;
  if constexpr (D == 1) {
    x = s;
    y = 0;
    z = 0;
  } else {
    const uint32_t row = qdiv(s, d.inv_nx);
    x = s - row * nx;
    z = (D == 3) ? qdiv(row, d.inv_ny) : 0u;
    y = row - z * ny;
  }
  Where w;
  w.xs[0] = x;
  w.xs[1] = x == 0 ? nx - 1 : x - 1;
  w.xs[2] = x == nx - 1 ? 0 : x + 1;
  w.ys[0] = y * nx;
  w.ys[1] = (y == 0 ? ny - 1 : y - 1) * nx;
  w.ys[2] = (y == ny - 1 ? 0 : y + 1) * nx;
  const uint32_t nxy = nx * ny;
  w.zs[0] = z * nxy;
  w.zs[1] = (z == 0 ? nz - 1 : z - 1) * nxy;
  w.zs[2] = (z == nz - 1 ? 0 : z + 1) * nxy;
  return w;
}

// One site's loaded populations, density and equilibrium factors.
template <int D, class S, class R>
struct Site {
  using L = Lattice<D>;
  using T = typename S::T;
  using Real = R;
  static constexpr int Q = L::Q;
  static constexpr int kDim = D;
  // f^eq_i = f01[dx][dy] e2[dz]: the common tier sums over c_z per (c_x, c_y)
  static constexpr bool kZFactor = (D == 3);
  static constexpr bool kSumsK1 = false;
  typename Kept<S>::type raw[Q];  // the loaded populations as kept (Kept<S>)
  R rho, irho, rho_ref;
  R u[3];
  // With e[a][d] = w(c) A_a z_a^c (digit d of c) and ie[a][d] = 1/e[a][d]
  // of the equilibrium's per-axis factors, the site keeps only
  R f01[3][3]; // rho e[0][dx] e[1][dy]:  f^eq_i = f01[dx][dy] e2[dz]
  R r01[3][3]; // ie[0][dx] ie[1][dy] / rho: 1/f^eq_i = r01[dx][dy] ie2[dz]
  R e2[3], ie2[3];  // e[2][dz], ie[2][dz]
  // where the populations came from, for the loops of the rare paths
  const T* src;
  uint32_t site;
  const SimDesc* desc;
  Where w;  // filled by locate_rare() before a rare-path loop

  // -- unrolled accessors (compile-time i) --------------------------------
  // The stored value is widened in each pass (cvt_fresh) rather than Q
  // widened values being kept live across passes.
  __device__ __forceinline__ R g(int i) const {
    return Codec<S, R>::dec_wide(widen<R>(raw[i]), R(L::W(i)), rho_ref);
  }
  // The z-axis factors a pass uses.  f^eq_i and 1/f^eq_i (one product
  // each) are recomputed per pass, not kept; passes that could share such
  // products (the middle tier with either of the others) take opaque copies
  // (pass_opaque) so that the compiler does not keep Q products live across
  // them.
  struct Pass {
    R e2[3], ie2[3];
  };
  __device__ __forceinline__ Pass pass_opaque() const {
    Pass p;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      p.e2[k] = opaque(e2[k]);
      p.ie2[k] = opaque(ie2[k]);
    }
    return p;
  }
  __device__ __forceinline__ Pass pass() const {
    // with FP64 storage every pass takes opaque copies (the register file
    // has no room for shared products next to Q FP64 populations)
    if constexpr (sizeof(T) == 8) return pass_opaque();
    Pass p;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      p.e2[k] = e2[k];
      p.ie2[k] = ie2[k];
    }
    return p;
  }

  __device__ __forceinline__ R fe(int i, const Pass& p) const {
    const R q = f01[L::dg(i, 0)][L::dg(i, 1)];
    return D > 2 ? q * p.e2[L::dg(i, 2)] : q;
  }
  __device__ __forceinline__ R x(int i, const Pass& p) const {
    const R q = r01[L::dg(i, 0)][L::dg(i, 1)];
    return fma(g(i), D > 2 ? q * p.ie2[L::dg(i, 2)] : q, R(-1));
  }
  // The x- and y-axis factors are folded with rho into f01 / r01 and not
  // kept, which saves 12 doubles of registers over the whole update.
  __device__ __forceinline__ void fold(const Equilibrium<R, D>& eq) {
    using EQ = Equilibrium<R, D>;
    // rho and the weights enter the x- and y-axis factors once each
    const R rw0 = rho * R(EQ::weight(0)), rw1 = rho * R(EQ::weight(1));
    const R iw0 = irho * R(1.0 / EQ::weight(0)), iw1 = irho * R(1.0 / EQ::weight(1));
    R x0[3], y0[3], ix0[3], iy0[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      x0[d] = (d == 0 ? rw0 : rw1) * eq.E[0][d];
      ix0[d] = (d == 0 ? iw0 : iw1) * eq.IE[0][d];
      y0[d] = D > 1 ? R(EQ::weight(d)) * eq.E[1][d] : R(1);
      iy0[d] = D > 1 ? eq.IE[1][d] * R(1.0 / EQ::weight(d)) : R(1);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        f01[a][b] = x0[a] * y0[b];
        r01[a][b] = ix0[a] * iy0[b];
      }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      e2[k] = eq.e(2, k);
      ie2[k] = eq.ie(2, k);
    }
  }

  // H(f^eq) / rho = ln rho + sum_a (ln A_a + u_a ln z_a)
  __device__ __forceinline__ double heq_per_rho() const {
    double h = log((double)rho);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double ua = (double)u[a];
      const double sa = sqrt(1.0 + 3.0 * ua * ua);
      h += log(2.0 - sa) + ua * log((2.0 * ua + sa) / (1.0 - ua));
    }
    return h;
  }

  // -- loop accessors (run-time, wavefront-uniform i) -----------------------
  // Register arrays are never indexed at run time (that would move them to
  // scratch memory); the population is re-read from the source buffer,
  // whose lines this wavefront has just brought into the caches.
  __device__ __forceinline__ void xfe(int i, R& xi, R& fi, R* gout = nullptr) const {
    const int dx = i % 3, dy = D > 1 ? (i / 3) % 3 : 0, dz = D > 2 ? i / 9 : 0;
    const int nz0 = (dx == 0) + (D > 1 && dy == 0) + (D > 2 && dz == 0);
    const R W = R(nz0 == 0 ? 1.0 : nz0 == 1 ? 4.0 : nz0 == 2 ? 16.0 : 64.0) / R(L::den());
    const uint32_t sp = sel3(w.zs, dz) + sel3(w.ys, dy) + sel3(w.xs, dx);
    const T gv = *(const gptr<T>)((gaddr)(uintptr_t)src + pidx<Q>(sp, i) * sizeof(T));
    const R gi = Codec<S, R>::dec(gv, W, rho_ref);
    fi = sel9(f01, dx, dy) * sel3(e2, dz);
    const R ri = sel9(r01, dx, dy) * sel3(ie2, dz);
    xi = fma(gi, ri, R(-1));
    if (gout) *gout = gi;
  }
};

// --------------------------------------------------- deviation arithmetic --
// The site of the mixed arithmetic policy.  Its FP32 arithmetic acts on the
// deviations s_i = f_i / W_i - rho_ref, which are O(|u| + |x|), so that each
// rounding is relative to a deviation rather than to f_i ~ W_i rho (FP32
// arithmetic on f_i itself drifts: the equilibrium's rounding, a smooth
// function of u, adds up over the steps).  With sum_i W_i = 1 and
// sum_i W_i c_i = 0:
//   rho = rho_ref + dr, dr = sum_i W_i s_i;  rho u = sum_i W_i c_i s_i.
// The equilibrium's per-axis factors A_a z_a^c are written 1 + dl_a(c).  With
// s_a = sqrt(1 + 3u^2) and q = s_a - 1 = 3u^2 / (1 + s_a) (no cancellation)
// they are A = 1 - q and A z^(+-1) = 2 s_a - 1 +- 3u (expand
// (1 - q)(1 + 2u + q) - (1 - u) and use q^2 + 2q = 3u^2):
//   dl(0) = -q,   dl(+-1) = 2q +- 3u,
// one rounding each, so that sum_c w(c) dl(c) = 0 and sum_c w(c) c dl(c) = u
// hold up to those roundings.  Then f^eq_i / W_i = rho (1 + Dl_i) with
// Dl_i = prod_a (1 + dl_a) - 1 expanded pairwise, s^eq_i = dr + rho Dl_i,
// and the entropy differences and alpha are evaluated in FP64 from
//   x_i = f_i / f^eq_i - 1 = (s_i - s^eq_i) / (rho_ref + s^eq_i),
//   f^eq_i = W_i (rho_ref + s^eq_i);
// the collision (Eq. (1)) is s~_i = s_i + alpha beta (s^eq_i - s_i).
// The site arithmetic A of the deviation form: FP32 (the mixed policy) or
// FP64 (the closed form's common tier on FP16 deviation storage with FP64
// site arithmetic).  Its reciprocals and square roots: the hardware
// estimates, refined by one Newton step where noted (FP32), or the
// refined estimates of rcp_n / sqrt_n (FP64).
template <class A>
__device__ __forceinline__ A rcp_a(A y) {
  if constexpr (std::is_same<A, float>::value) {
    const float r0 = __builtin_amdgcn_rcpf(y);
    return fmaf(r0, fmaf(-y, r0, 1.0f), r0);
  } else {
    return rcp_n<A>(y);
  }
}
template <class A>
__device__ __forceinline__ A rcp_hw(A y) {  // FP32: the estimate alone (1 ulp)
  if constexpr (std::is_same<A, float>::value) return __builtin_amdgcn_rcpf(y);
  else return rcp_n<A>(y);
}
template <class A>
__device__ __forceinline__ A sqrt_hw(A y) {  // FP32: the estimate alone (1 ulp)
  if constexpr (std::is_same<A, float>::value) return __builtin_amdgcn_sqrtf(y);
  else return sqrt_n<A>(y);
}

template <int D, class S, class A = float>
struct SiteDevT {
  using L = Lattice<D>;
  using T = typename S::T;
  using Real = double;  // arithmetic of the alpha evaluation
  using Arith = A;      // arithmetic of the deviations
  static constexpr int Q = L::Q;
  static constexpr int kDim = D;
  static constexpr bool kZFactor = false;  // f^eq_i comes from s^eq_i
  static constexpr bool kSumsK1 = true;     // sums_k1() below
  // the collision takes s_i - s^eq_i as sums_k1 formed them where that costs
  // fewer registers than the factors s^eq_i is recomputed from
  static constexpr bool kKeepD = std::is_same<A, float>::value || Q <= 9;
  typename Kept<S>::type raw[Q];
  A r, dr, rhoA;  // rho_ref, rho - rho_ref, rho (in the arithmetic A)
  double rho, u[3];    // rho and u widened (alpha's guard, diagnostics)
  // s^eq_i = dr + rho Dl_i with Dl_i = (1 + a)(1 + dl_z(dz)) - 1,
  // a = (1 + dl_x(dx)) (1 + dl_y(dy)) - 1, formed as one multiply-add
  // s^eq_i = seqA + seqB dl_z(dz) from seqA = dr + rho a and seqB = rho (1 + a)
  A seqA[3][3], seqB[3][3];
  A dlz[3];        // dl_z(dz)
  // 1 / (rho_ref + s^eq_i) = W_i / f^eq_i = rxy[dx][dy] rlz[dz]: with
  // rho_ref + s^eq_i = rho prod_a (1 + dl_a), the reciprocals of the nine
  // per-axis factors (and 1/rho) give it with one product per direction
  A rxy[3][3];     // 1 / (rho (1 + dl_x(dx)) (1 + dl_y(dy)))
  A rlz[3];        // 1 / (1 + dl_z(dz))
  A dd[Q];         // s_i - s^eq_i as sums_k1 formed them (kKeepD)
  const T* src;
  uint32_t site;
  const SimDesc* desc;
  Where w;  // filled by locate() before a rare-path loop

  // s_i from the kept value (FP32 storage holds f_i: one rounding)
  __device__ __forceinline__ A s(int i) const {
    if constexpr (S::dev) return A(raw[i]);
    else return fma(A(raw[i]), A(L::invW(i)), -r);
  }
  struct Pass {
    A dlz[3], rlz[3];
  };
  __device__ __forceinline__ Pass pass() const {
    Pass p;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      p.dlz[k] = dlz[k];
      p.rlz[k] = rlz[k];
    }
    return p;
  }
  // copies hidden from the optimiser, so that the s^eq_i of different
  // passes are not kept live between them
  __device__ __forceinline__ Pass pass_opaque() const {
    Pass p;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      p.dlz[k] = opaque(dlz[k]);
      p.rlz[k] = opaque(rlz[k]);
    }
    return p;
  }
  __device__ __forceinline__ A seq(int i, const Pass& p) const {
    const A Av = seqA[L::dg(i, 0)][L::dg(i, 1)];
    return D > 2 ? fma(seqB[L::dg(i, 0)][L::dg(i, 1)], p.dlz[L::dg(i, 2)], Av) : Av;
  }
  __device__ __forceinline__ double fe(int i, const Pass& p) const {
    return double(A(L::W(i)) * (r + seq(i, p)));
  }
  // x_i = (s_i - s^eq_i) / (rho_ref + s^eq_i) to the arithmetic's relative
  // accuracy (a few roundings of the reciprocal factors): its absolute error
  // is that of s_i - s^eq_i, O(|u|) times the rounding
  __device__ __forceinline__ A rfac(int i, const Pass& p) const {
    const A R = rxy[L::dg(i, 0)][L::dg(i, 1)];
    return D > 2 ? R * p.rlz[L::dg(i, 2)] : R;
  }
  __device__ __forceinline__ double x(int i, const Pass& p) const {
    return double((s(i) - seq(i, p)) * rfac(i, p));
  }
  // The common-tier sums to their first terms, E = sum_i f^eq_i x_i^2 / 2
  // and O = sum_i f^eq_i x_i^3 / 6, and max_i |x_i|, for results stored in
  // 2 bytes (the closed form's one-term tier).  In FP32 the rounding moves
  // alpha by about 2^-24 max|x_i|, far below what 11 stored bits resolve.
  // With d_i = s_i - s^eq_i, f^eq_i x_i = W_i d_i, so E and O are W-weighted
  // sums of d_i x_i and d_i x_i^2, summed per weight class (W_i = 4^z / 6^D,
  // z the number of zero components of c_i) and weighted once at the end.
  __device__ __forceinline__ void sums_k1(const Pass& p, A& sE, A& sO, A& xabs) {
    A e[D + 1], o[D + 1], xm = A(0);
#pragma unroll
    for (int z = 0; z <= D; ++z) e[z] = o[z] = A(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const A di = s(i) - seq(i, p);
      if constexpr (kKeepD) dd[i] = di;
      const A xi = di * rfac(i, p);
      const A t = di * xi;
      const int z = L::nzero(i);
      e[z] += t;
      o[z] = fma(t, xi, o[z]);
      xm = fmax(xm, fabs(xi));
      sched_group(i);
    }
    A E = A(0), O = A(0);
#pragma unroll
    for (int z = 0; z <= D; ++z) {
      const A wz = A(double(1 << (2 * z)) / L::den());
      E = fma(wz, e[z], E);
      O = fma(wz, o[z], O);
    }
    sE = A(0.5) * E;
    sO = O * A(1.0 / 6.0);
    xabs = xm;
  }
  // s_i - s^eq_i for the collision
  __device__ __forceinline__ A dev(int i, const Pass& p) const {
    if constexpr (kKeepD) return dd[i];
    else return s(i) - seq(i, p);
  }
  // the stored value of s~_i.  FP32 storage holds f~_i = W_i (rho_ref + s~_i),
  // rounded once from W_i = wh + wl (wl: the residual of W_i's FP32
  // rounding): with the FP32 weight alone every step would scale f_i by
  // float(W_i) / W_i, a bias that adds up (the read divides by 1 / W_i, which
  // is exact).  An FP64 deviation goes to FP16 through FP32 (two roundings
  // to nearest even; gfx950 has no FP64 -> FP16 conversion, and allowed to
  // merge the two the compiler would expand one into integer arithmetic).
  __host__ __device__ static constexpr float w_lo(double W) { return float(W - double(float(W))); }
  __device__ __forceinline__ static T enc_f(float wh, float wl, float rr, float sn) {
    return T(fmaf(wh, rr, fmaf(wh, sn, wl * (rr + sn))));
  }
  __device__ __forceinline__ T enc(int i, A sn) const {
    if constexpr (std::is_same<A, double>::value) {
      static_assert(S::dev, "FP64 deviation arithmetic is built for deviation storage");
      float h = float(sn);
      asm volatile("" : "+v"(h));
      return T(h);
    } else if constexpr (S::dev) {
      return T(sn);
    } else {
      return enc_f(float(L::W(i)), w_lo(L::W(i)), r, sn);
    }
  }

  // H(f^eq) / rho, as for the FP64 site
  __device__ __forceinline__ double heq_per_rho() const {
    double h = log(rho);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double ua = u[a];
      const double sa = sqrt(1.0 + 3.0 * ua * ua);
      h += log(2.0 - sa) + ua * log((2.0 * ua + sa) / (1.0 - ua));
    }
    return h;
  }

  // -- loop accessors (run-time, wavefront-uniform i) -----------------------
  // The population is re-read from the source buffer (see Site::xfe).
  // W_i = num / den with num = 4^(number of zero components of c_i); both
  // quotients round as float(L::W(i)) and float(L::invW(i)) do (den / num is
  // exact)
  __device__ __forceinline__ static float weight_num(int i) {
    const int dx = i % 3, dy = D > 1 ? (i / 3) % 3 : 0, dz = D > 2 ? i / 9 : 0;
    const int nz0 = (dx == 0) + (D > 1 && dy == 0) + (D > 2 && dz == 0);
    return nz0 == 0 ? 1.0f : nz0 == 1 ? 4.0f : nz0 == 2 ? 16.0f : 64.0f;
  }
  __device__ __forceinline__ static float weight_of(int i) { return weight_num(i) / float(L::den()); }
  // w_lo of the weight weight_of(i) rounds (the four weights of the lattice)
  __device__ __forceinline__ static float weight_lo(int i) {
    const float n = weight_num(i);
    return n == 1.0f ? w_lo(1.0 / L::den()) : n == 4.0f ? w_lo(4.0 / L::den())
         : n == 16.0f ? w_lo(16.0 / L::den()) : w_lo(64.0 / L::den());
  }
  __device__ __forceinline__ static float invweight_of(int i) { return float(L::den()) / weight_num(i); }
  __device__ __forceinline__ void sq(int i, float& si, float& seqi) const {
    const int dx = i % 3, dy = D > 1 ? (i / 3) % 3 : 0, dz = D > 2 ? i / 9 : 0;
    const uint32_t sp = sel3(w.zs, dz) + sel3(w.ys, dy) + sel3(w.xs, dx);
    const T gv = *(const gptr<T>)((gaddr)(uintptr_t)src + pidx<Q>(sp, i) * sizeof(T));
    if constexpr (S::dev) si = float(gv);
    else si = fmaf(float(gv), invweight_of(i), -r);
    // the selections multiply by 0 and 1 and add zeros: exact
    const float sa = sel9(seqA, dx, dy);
    seqi = D > 2 ? fmaf(sel9(seqB, dx, dy), sel3(dlz, dz), sa) : sa;
  }
  __device__ __forceinline__ void xfe(int i, double& xi, double& fi, double* = nullptr) const {
    float si, seqi;
    sq(i, si, seqi);
    xi = double((si - seqi) * __builtin_amdgcn_rcpf(r + seqi));
    fi = double(weight_of(i) * (r + seqi));
  }
};
template <int D, class S>
using SiteDev = SiteDevT<D, S, float>;

// S(a) = sum_i f^eq_i phi((1 - a) x_i); G(a) = H(f*(a)) - H(f) = S(a) - D.
template <class V, class R>
__device__ __forceinline__ R S_log(const V& v, R a) {
  R s = R(0);
#pragma unroll 1
  for (int i = 0; i < V::Q; ++i) {
    R xi, fi;
    v.xfe(i, xi, fi);
    s += fi * phi_log<R>((R(1) - a) * xi);
  }
  return s;
}

// S(a) and S'(a) = G'(a) = -sum_i f^eq_i x_i ln(1 + (1 - a) x_i).
// With sA, also sum_i f^eq_i |x_i|.
template <class V, class R>
__device__ __forceinline__ void S_dS_log(const V& v, R a, R& Sv, R& dS, R* sA = nullptr) {
  Sv = R(0);
  dS = R(0);
  R sa = R(0);
#pragma unroll 1
  for (int i = 0; i < V::Q; ++i) {
    R xi, fi;
    v.xfe(i, xi, fi);
    const R y = (R(1) - a) * xi;
    const R l = dlog_clamped<R>(y);
    Sv += fi * ((y <= R(-1)) ? R(1) : (R(1) + y) * l - y);
    dS -= fi * xi * l;
    sa = fma(fi, fabs(xi), sa);
  }
  if (sA) *sA = sa;
}

constexpr double kEpsF64 = 2.220446049250313e-16;  // 2^-52

// ln(1 + y) for the root solvers' passes, in two tiers, without the range
// reduction and double-double steps of the library routine (about 140
// instructions in FP64).
//
// Log1pM, |y| <= 0.025: the Maclaurin series y - y^2/2 + y^3/3 - ...
// through y^10 / 10 by Horner's rule; the first omitted term is below
// 0.025^10 / 11 < 2^-54 of the sum.
struct Log1pM {
  static constexpr double ymax = 0.025;
  double c[9];  // c[k] = (-1)^(k+1) / (k + 2): the coefficients of y^2 .. y^10
  __device__ __forceinline__ Log1pM() {
#pragma unroll
    for (int k = 0; k < 9; ++k) c[k] = in_sgpr((k % 2 ? 1.0 : -1.0) / (k + 2.0));
  }
  __device__ __forceinline__ double operator()(double y) const {
    double p = c[8];
#pragma unroll
    for (int k = 7; k >= 0; --k) p = fma(p, y, c[k]);
    return fma(y * y, p, y);  // y + y^2 (-1/2 + y/3 - ...)
  }
};

// Log1pK<10>, |y| <= 0.29: ln(1 + y) = 2 artanh(s) = 2 s (1 + s^2/3 +
// s^4/5 + ...) with s = y / (2 + y), truncated after K terms; the first
// omitted term, s^(2K) / (2K + 1) <= (ymax / (2 - ymax))^(2K) / (2K + 1), is
// below 2^-54 of the sum.  s carries about two roundings (the reciprocal is
// the refined hardware estimate), so the result is good to about two units
// in the last place.
template <int K>
struct Log1pK {
  static constexpr double ymax = 0.29;
  static_assert(K == 10, "one tier: K = 10 (|y| <= 0.29)");
  double c[K - 1];  // c[k] = 1 / (2k + 3): the coefficients of s^2 .. s^(2K-2)
  __device__ __forceinline__ Log1pK() {
#pragma unroll
    for (int k = 0; k < K - 1; ++k) c[k] = in_sgpr(1.0 / (2.0 * k + 3.0));
  }
  __device__ __forceinline__ double operator()(double y) const {
    const double s = y * rcp_n<double>(2.0 + y);
    const double t = s * s;
    double q = c[K - 2];
#pragma unroll
    for (int k = K - 3; k >= 0; --k) q = fma(q, t, c[k]);
    const double s2 = s + s;
    return fma(s2 * t, q, s2);  // 2s + 2s (s^2/3 + s^4/5 + ...)
  }
};

// S(a) and S'(a) as S_dS_log, but as one unrolled pass over the populations
// the site holds in registers, with ln(1 + y) from LN (Log1pM or
// Log1pK<10>): valid while every |(1 - a) x_i| <= LN::ymax (the caller
// checks this for the whole wavefront); also sA = sum_i f^eq_i |x_i|.  For D3Q27 (f^eq_i = f01[dx][dy] e2[dz]) the sums over
// c_z are formed with e2 and multiplied by f01 once per (c_x, c_y).
template <class LN, class V, class R>
__device__ __forceinline__ void S_dS_series(const V& v, R a, R& Sv, R& dS, R& sA) {
  constexpr int Q = V::Q;
  const LN ln1p;
#if ELBM_NEWTON_OPAQUE
  const auto P = v.pass_opaque();
#else
  const auto P = v.pass();
#endif
  const R c = R(1) - a;
  Sv = R(0);
  dS = R(0);
  sA = R(0);
  if constexpr (V::kZFactor) {
#pragma unroll
    for (int dxy = 0; dxy < 9; ++dxy) {
      R iS = R(0), iD = R(0), iA = R(0);
#pragma unroll
      for (int dz = 0; dz < 3; ++dz) {
        const R xi = v.x(dxy + 9 * dz, P);
        const R y = c * xi;
        const R l = ln1p(y);
        iS = fma(P.e2[dz], fma(R(1) + y, l, -y), iS);
        iD = fma(P.e2[dz] * xi, l, iD);
        iA = fma(P.e2[dz], fabs(xi), iA);
      }
      Sv = fma(v.f01[dxy % 3][dxy / 3], iS, Sv);
      dS = fma(-v.f01[dxy % 3][dxy / 3], iD, dS);
      sA = fma(v.f01[dxy % 3][dxy / 3], iA, sA);
#if ELBM_NEWTON_FENCE
      __builtin_amdgcn_sched_barrier(0);
#endif
    }
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R xi = v.x(i, P);
      const R fi = v.fe(i, P);
      const R y = c * xi;
      const R l = ln1p(y);
      Sv = fma(fi, fma(R(1) + y, l, -y), Sv);
      dS = fma(-fi * xi, l, dS);
      sA = fma(fi, fabs(xi), sA);
#if ELBM_NEWTON_FENCE
      if (i % 3 == 2) __builtin_amdgcn_sched_barrier(0);
#endif
    }
  }
}

// S(a), S'(a) for one Newton iteration: the unrolled register passes when
// every active lane's |(1 - a) x_i| fits a series tier (xabs = max_i |x_i|
// of the lane), else the rolled pass with the library logarithm.
template <class V, class R>
__device__ __forceinline__ void S_dS_newton(V& v, const SimDesc& d, R a, R xabs, R& Sv, R& dS,
                                            R& sA) {
  if constexpr (std::is_same<R, double>::value) {
    const R yb = fabs(R(1) - a) * xabs;
    if (__all(yb <= R(Log1pM::ymax))) {
      S_dS_series<Log1pM>(v, a, Sv, dS, sA);
      return;
    }
    if (__all(yb <= R(Log1pK<10>::ymax))) {
      S_dS_series<Log1pK<10>>(v, a, Sv, dS, sA);
      return;
    }
  }
  // the rolled pass re-reads the populations: their source offsets are
  // formed here, not kept live through the register passes
  v.w = locate<V::kDim>(d, v.site);
  S_dS_log(v, a, Sv, dS, &sA);
}

// The rare path of one lane: the long series when alpha_* = 2 and
// max|x| <= thrL, else the log1p forms.
template <class V, class R>
__device__ __forceinline__ void rare_sums(const V& v, R astar, bool star2, R xabs, R& Dv, R& Ds,
                          R& Gs) {
  constexpr int Q = V::Q;
  if (star2 && xabs <= Base<R>::thrL) {
    R sE = R(0), sO = R(0);
    const SeriesK<R, Base<R>::KL> ser;
#pragma unroll 1
    for (int i = 0; i < Q; ++i) {
      R xi, fi;
      v.xfe(i, xi, fi);
      ser.accum(xi, fi, sE, sO);
    }
    R cE, cO;
    series_scale<R, Base<R>::KL>(cE, cO);
    sE *= cE;
    sO *= cO;
    Dv = sE - sO;
    Ds = sE + sO;
    Gs = R(2) * sO;
    return;
  }
  R sD = R(0), sS = R(0), sG = R(0);
#pragma unroll 1
  for (int i = 0; i < Q; ++i) {
    R xi, fi;
    v.xfe(i, xi, fi);
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

template <class R>
struct AlphaOut {
  R alpha, D;
  bool accepted2, astar_lt2, guard, fallback, deferred;
  int iters;
};

// Phases of the closed form.  kPhaseAll evaluates every tier in one call.
// kPhaseCommon evaluates the short-series tiers and defers the lanes that
// need the rare tier (alpha_* < 2, or max|x_i| beyond the middle tier);
// kPhaseRare then handles only those lanes, after the common phase's values
// have died, so the long series and the logarithms do not raise the
// register peak of the common path.
enum { kPhaseAll = 0, kPhaseCommon = 1, kPhaseRare = 2 };

// The choice of alpha at one site (all lanes of the wavefront call it).
// V: the site type (lattice, storage, arithmetic).
template <int MODE, int PHASE, class V>
__device__ __forceinline__ AlphaOut<typename V::Real> choose_alpha(V& v, const SimDesc& d) {
  using R = typename V::Real;
  constexpr int D = V::kDim;
  constexpr int Q = V::Q;
  AlphaOut<R> o;
  o.deferred = false;
  // The root solvers need alpha_max on every lane; the closed form and the
  // secant need it only where alpha_* < 2, which the tiers below detect.
  constexpr bool kXmax = (MODE == kNewton || MODE == kBisect);
  // The closed form on 2-byte storage takes the first-term sums (and, on the
  // mixed site, forms them in FP32: sums_k1).  The root solvers keep the full
  // tiers: their root moves with D itself, by about x^2 / 12 under the
  // one-term truncation, while Eq. (9) depends on the ratio O / (E + O),
  // in which the truncations of E and O largely cancel.
  constexpr bool kS16 =
      sizeof(typename V::T) == 2 && std::is_same<R, double>::value && MODE == kClosed;
  constexpr bool kK1 = kS16 && V::kSumsK1 && !kXmax;
  if constexpr (kK1 && MODE == kClosed && PHASE == kPhaseCommon) {
    // The common phase of the closed form on them, in the deviation site's
    // arithmetic A: alpha_* = 2 (max|x_i| <= 0.025 < 1), D = E - O,
    // G(2) = 2 O, D*(2) = E + O, and Eq. (9) gives alpha = 2 - 2 O / (E + O)
    // where G(2) > 0.  The quotient (below |x| / 3) carries A's rounding;
    // 2 minus it is formed in FP64.
    using A = typename V::Arith;
    A E, O, xm;
    v.sums_k1(v.pass(), E, O, xm);
    o.iters = 0;
    o.astar_lt2 = o.fallback = false;
    if (!(xm <= A(Base<R>::thrM))) {
      o.deferred = true;
      o.alpha = R(2);
      o.D = R(0);
      o.accepted2 = o.guard = false;
      return o;
    }
    const A Dv = E - O;
    o.D = R(Dv);
    o.guard = !(Dv > A(Prec<R>::guard) * v.rhoA);
    o.accepted2 = o.guard || !(O > A(0));
    o.alpha = R(2);
    if (!o.accepted2) {
      const A r = rcp_a(E + O);
      o.alpha = R(2) - R(fmin(A(2) * O * r, A(1)));  // clamped to [1, 2]
      o.iters = 1;
    }
    return o;
  }
  // The rolled passes (rare tier, root solvers) re-read the populations
  // from the source buffer; their source offsets (v.w) are formed just
  // before each such pass rather than kept live through the whole update.
  // Common tier: x_i, max|x_i| and the KC-term series sums in one pass.
  // With 2-byte storage the stored result carries 11 bits: for the closed
  // form one term (E = sum f^eq x^2 / 2, O = sum f^eq x^3 / 6) up to
  // max|x_i| <= thrM = 0.025 leaves out x^4/12 of E and x^5/20 of O, which
  // moves 2 - alpha (<= 2|x|/3) by at most 0.47 x^2 of itself, alpha by at
  // most 5e-6 and f~_i = f^eq_i (1 + (1 - alpha beta) x_i) by at most
  // 1.3e-7 f^eq_i: about 2 % of half a unit of an FP16 deviation s_i of the
  // size of x_i.  Otherwise the tiers keep alpha to 2^-53.
  constexpr int KC = kS16 ? 1 : Base<R>::K;
  const R thrC = kS16 ? Base<R>::thrM : Base<R>::thr;
  R xmax = R(-1), xabs = R(0), sE = R(0), sO = R(0);
  if constexpr (PHASE != kPhaseRare && kK1) {
    typename V::Arith E, O, xm;
    v.sums_k1(v.pass(), E, O, xm);
    sE = E;
    sO = O;
    xabs = xm;
  } else if constexpr (PHASE != kPhaseRare) {
  const SeriesK<R, KC> ser;
  const auto P = v.pass();
  if constexpr (V::kZFactor) {
    // f^eq_i = f01[dx][dy] e2[dz]: the sums over dz are formed with e2
    // alone and multiplied by f01 once per (dx, dy)
#pragma unroll
    for (int dxy = 0; dxy < 9; ++dxy) {
      R iE = R(0), iO = R(0);
#pragma unroll
      for (int dz = 0; dz < 3; ++dz) {
        const int i = dxy + 9 * dz;
        const R xi = v.x(i, P);
        if (kXmax) xmax = fmax(xmax, xi);
        xabs = fmax(xabs, fabs(xi));
        ser.accum(xi, P.e2[dz], iE, iO);
      }
      sE = fma(v.f01[dxy % 3][dxy / 3], iE, sE);
      sO = fma(v.f01[dxy % 3][dxy / 3], iO, sO);
      sched_group(dxy);
    }
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R xi = v.x(i, P);
      if (kXmax) xmax = fmax(xmax, xi);
      xabs = fmax(xabs, fabs(xi));
      ser.accum(xi, v.fe(i, P), sE, sO);
      sched_group(i);
    }
  }
  }
  if constexpr (PHASE != kPhaseRare) {
    if constexpr (!kK1) {
      R cE, cO;
      series_scale<R, KC>(cE, cO);
      sE *= cE;
      sO *= cO;
    }
  } else {
    // only deferred lanes are active: max|x_i| again, by the loop accessors
    v.w = locate<D>(d, v.site);
#pragma unroll 1
    for (int i = 0; i < Q; ++i) {
      R xi, fi;
      v.xfe(i, xi, fi);
      xabs = fmax(xabs, fabs(xi));
    }
  }
  // D = H(f) - H(f^eq), Gs = H(f*(a_*)) - H(f), Ds = H(f*(a_*)) - H(f^eq); at
  // alpha_* = 2: D = E - O, Ds = E + O, Gs = 2 O.
  R Dv = sE - sO, Ds = sE + sO, Gs = R(2) * sO;
  // max|x| <= thrM < 1 implies max x <= 1, i.e. alpha_* = 2.  A lane in the
  // rare phase was deferred by the common phase and stays rare: max|x_i|
  // formed again by the loop accessors may round differently and must not
  // send it back to a tier whose sums it has not formed.
  const bool common = PHASE != kPhaseRare && xabs <= thrC;
  const bool mid = PHASE != kPhaseRare && !common && xabs <= Base<R>::thrM;
  const bool rare = PHASE == kPhaseRare || !(xabs <= Base<R>::thrM);
  if constexpr (PHASE == kPhaseCommon) {
    if (rare) {
      o.deferred = true;
      o.alpha = R(2);
      o.D = R(0);
      o.accepted2 = o.astar_lt2 = o.guard = o.fallback = false;
      o.iters = 0;
    }
  }
  if (PHASE != kPhaseRare && __any(mid)) {
    R mE = R(0), mO = R(0);
    const SeriesK<R, Base<R>::KM> ser;
    const auto P = v.pass_opaque();
#pragma unroll
    for (int i = 0; i < Q; ++i) ser.accum(v.x(i, P), v.fe(i, P), mE, mO);
    R cE, cO;
    series_scale<R, Base<R>::KM>(cE, cO);
    mE *= cE;
    mO *= cO;
    if (mid) {
      Dv = mE - mO;
      Ds = mE + mO;
      Gs = R(2) * mO;
    }
  }
  if constexpr (PHASE == kPhaseCommon) {
    if (rare) return o;
  }
  if (PHASE == kPhaseAll && __any(rare)) v.w = locate<D>(d, v.site);
  if (rare && !kXmax) {
    xmax = R(-1);
#pragma unroll 1
    for (int i = 0; i < Q; ++i) {
      R xi, fi;
      v.xfe(i, xi, fi);
      xmax = fmax(xmax, xi);
    }
  }
  // alpha_max = min over {f^eq_i < f_i} of f_i/(f_i - f^eq_i) = 1 + 1/max_i x_i
  // (definition after Eq. (7)); alpha_* = min(2, alpha_max) (Eq. (8)), and
  // alpha_* = 2 exactly when max_i x_i <= 1.  Outside the rare tier (and the
  // root solvers) xmax is not formed and alpha_* = 2.
  const bool has_pos = (rare || kXmax) ? xmax > R(0) : true;
  const R amax = has_pos ? R(1) + R(1) / xmax : R(INFINITY);
  const bool star2 = (rare || kXmax) ? !(xmax > R(1)) : true;
  const R astar = star2 ? R(2) : amax;
  o.fallback = rare;
  if (__any(rare)) {
    if (rare) rare_sums(v, astar, star2, xabs, Dv, Ds, Gs);
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
        // alpha^(0) = 1, so the first iterate is Eq. (9): G(1) = -D needs no
        // pass.  Later iterates take G from the populations held in
        // registers: where every active lane is on the common tier and two
        // or more evaluations follow, from one pass forming the power sums
        // M_n = sum_i f^eq_i x_i^n, n = 2 .. 2K + 1, which give
        // S(a) = sum_n (-1)^n (1 - a)^n M_n / (n (n - 1)) truncated where
        // the tier truncates E and O (the iterates lie in [1, 2], so
        // |(1 - a) x_i| <= |x_i|); otherwise from Newton's passes (series
        // where every lane's |(1 - a) x_i| allows it, else log1p).
        constexpr int KS = Base<R>::K, NP = 2 * KS + 2;
        const bool poly = PHASE != kPhaseRare && d.secant_iters > 2 && __all(common);
        R M[NP];
#pragma unroll
        for (int n = 0; n < NP; ++n) M[n] = R(0);
        if (poly) {
          const auto P = v.pass_opaque();
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            const R xi = v.x(i, P);
            R w = v.fe(i, P) * xi * xi;
#pragma unroll
            for (int n = 2; n < NP; ++n) {
              M[n] += w;
              if (n + 1 < NP) w *= xi;
            }
            sched_group(i);
          }
        }
        R a = R(1);
        for (int k = 0; k < d.secant_iters; ++k) {
          R Ga = -Dv;
          if (k > 0) {
            R Sv = R(0);
            if (poly) {
              const R b = R(1) - a;
              R bn = b * b;
#pragma unroll
              for (int n = 2; n < NP; ++n) {
                Sv = fma(R((n % 2 ? -1.0 : 1.0) / (double(n) * (n - 1))) * bn, M[n], Sv);
                bn *= b;
              }
            } else {
              R dS, sA;
              S_dS_newton(v, d, a, xabs, Sv, dS, sA);
            }
            Ga = Sv - Dv;
          }
          const R an = astar + Gs / (Gs - Ga) * (a - astar);
          iters = k + 1;
          if (an == a) break;
          a = an;
        }
        alpha = fmin(fmax(a, R(1)), astar);
      }
    } else if constexpr (MODE == kBisect) {
      // Eq. (4) on [1, alpha_max]; first midpoint with -tol <= G <= 0.  G is
      // taken as in Newton's passes (series on the register-held
      // populations where every lane allows it, else the log1p pass).  Pass
      // 0 asks whether G(alpha_max) <= 0 (then alpha = alpha_max); one call
      // site, so that the pass is inlined once.
      R lo = R(1), hi = amax;
      const R tol = (R)d.root_tol;
      alpha = R(-1);
      for (int k = 0; k <= d.root_max_iter; ++k) {
        const R a = k == 0 ? amax : R(0.5) * (lo + hi);
        R Sv, dS, sA;
        S_dS_newton(v, d, a, xabs, Sv, dS, sA);
        const R g = Sv - Dv;
        if (k == 0) {
          if (g <= R(0)) {
            alpha = amax;
            break;
          }
          continue;
        }
        iters = k;
        if (g <= R(0) && g >= -tol) {
          alpha = a;
          break;
        }
        if (g > R(0)) hi = a;
        else lo = a;
      }
      if (alpha < R(0)) alpha = lo;
    } else if constexpr (MODE == kNewton) {
      // Eq. (4) by Newton from alpha_* inside the bracket [1, alpha_max]
      // (from its midpoint when alpha_* = alpha_max, where G' is unbounded).
      // G is convex, G(1) <= 0 and G' > 0 beyond 1, so a step from a point
      // with G < 0 lands at or beyond the root; whether the root lies inside
      // the bracket (G(alpha_max) > 0) is asked only when a step leaves it
      // while its upper end is still alpha_max.  A step leaving the bracket
      // is replaced by the midpoint.  The iteration stops when |G(a)| is at
      // the rounding level of its evaluation, eps sum_i f^eq_i (|x_i| +
      // |(1 - a) x_i|) (each term is formed from O(|y|) parts), or at a step
      // below 1e-13 alpha (the rounding of G near the root moves alpha by
      // about that much); a converged Newton step that rounds onto the end
      // of the bracket stops there.
      R lo = R(1), hi = amax;
      bool hi_pos = false;  // G(hi) > 0 known
      R a = (astar < amax) ? astar : R(0.5) * (lo + hi);
      alpha = R(-1);
      for (int k = 1; k <= d.root_max_iter; ++k) {
        R Sv, dS, sA;
        S_dS_newton(v, d, a, xabs, Sv, dS, sA);
        const R gv = Sv - Dv;
        iters = k;
        if (fabs(gv) <= R(kEpsF64) * (R(1) + fabs(R(1) - a)) * sA) {
          alpha = a;
          break;
        }
        if (gv > R(0)) {
          hi = a;
          hi_pos = true;
        } else {
          lo = a;
        }
        R an = a - gv / dS;
        if (!(an > lo && an < hi)) {
          if (fabs(an - a) <= R(1e-13) * a) {
            alpha = fmin(fmax(an, lo), hi);
            break;
          }
          if (!hi_pos) {
            v.w = locate<D>(d, v.site);
            if (S_log(v, hi) - Dv <= R(0)) {
              alpha = hi;
              break;
            }
            hi_pos = true;
          }
          an = R(0.5) * (lo + hi);
        }
        if (fabs(an - a) <= R(1e-13) * a) {
          alpha = an;
          break;
        }
        a = an;
      }
      if (alpha < R(0)) alpha = a;
    }
  }
  o.alpha = alpha;
  o.iters = iters;
  return o;
}

// Per-thread diagnostics of the sites a thread updated.
struct Acc {
  uint32_t c[kNumCounts];  // wavefront totals (uniform), from ballots
  int iters;               // per lane (root-solver modes)
  float amin, amax;        // per lane
  double rho, j[3], H;     // per lane (ELBM_DIAG_SUMS)
  __device__ void init() {
#pragma unroll
    for (int k = 0; k < kNumCounts; ++k) c[k] = 0;
    iters = 0;
    amin = INFINITY;
    amax = 0.0f;  // alpha >= 1: +0 is below every value (see wmax_nonneg)
    rho = j[0] = j[1] = j[2] = H = 0.0;
  }
  // wavefront counts of the count predicates; all lanes must be active
  // (MASK: the bits that can be set; the others are not counted)
  template <uint32_t MASK = (1u << kCntIters) - 1u>
  __device__ __forceinline__ void count_flags(uint32_t flags) {
#pragma unroll
    for (int k = 0; k < kCntIters; ++k)
      if (MASK & (1u << k)) c[k] += (uint32_t)__popcll(__ballot((flags >> k) & 1u));
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
// Wavefront min / max by data-parallel-primitive moves (one VALU operation
// per step instead of an LDS permute and its lane arithmetic): lane pairs
// and quads (quad_perm [1,0,3,2], [2,3,0,1]), half rows and rows of 16 lanes
// (row_half_mirror, row_mirror; every lane then holds its row's result), row
// 0 into row 1 and row 2 into row 3 (row_bcast:15 on rows 1 and 3), rows 0-1
// into rows 2-3 (row_bcast:31 on rows 2 and 3); lane 63 holds the
// wavefront's result.  All lanes must be active.  The values reduced are
// non-negative floats (alpha, +inf in the minimum and +0 in the maximum for
// a lane without sites), whose bit patterns order as unsigned integers: the
// steps are integer min / max, exact and free of the NaN quieting that
// float min / max apply to their operands.
// The moved value of a lane outside the row mask is the operation's
// identity ID, so that the move folds into the min / max instruction.
template <int CTRL, int ROW_MASK, uint32_t ID>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)ID, (int)v, CTRL, ROW_MASK, 0xf, false);
}
template <uint32_t ID, class OP>
__device__ __forceinline__ uint32_t wreduce_dpp(uint32_t v, OP op) {
  v = op(v, dpp_u32<0xB1, 0xf, ID>(v));   // quad_perm [1,0,3,2]
  v = op(v, dpp_u32<0x4E, 0xf, ID>(v));   // quad_perm [2,3,0,1]
  v = op(v, dpp_u32<0x141, 0xf, ID>(v));  // row_half_mirror
  v = op(v, dpp_u32<0x140, 0xf, ID>(v));  // row_mirror
  v = op(v, dpp_u32<0x142, 0xA, ID>(v));  // row_bcast:15 into rows 1, 3
  v = op(v, dpp_u32<0x143, 0xC, ID>(v));  // row_bcast:31 into rows 2, 3
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ float wmin_nonneg(float v) {
  return __builtin_bit_cast(float, wreduce_dpp<0xffffffffu>(
                                        __builtin_bit_cast(uint32_t, v),
                                        [](uint32_t a, uint32_t b) { return a < b ? a : b; }));
}
__device__ __forceinline__ float wmax_nonneg(float v) {
  return __builtin_bit_cast(float, wreduce_dpp<0u>(
                                        __builtin_bit_cast(uint32_t, v),
                                        [](uint32_t a, uint32_t b) { return a > b ? a : b; }));
}

// Wavefront reductions, then a fixed-order combination over the block's
// wavefronts: each record is a deterministic function of the block's sites.
template <bool ITERS>
__device__ void store_records(const Acc& a, const SimDesc& d, int slot) {
  constexpr int NW = kBlock / 64;
  __shared__ uint32_t sc[NW][kNumCounts];
  __shared__ float sa[NW][2];
  __shared__ double ss[NW][5];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const bool sums = (d.diag & kDiagSums) != 0;
  uint32_t it = 0;
  if constexpr (ITERS) it = (uint32_t)wsumi(a.iters);
  const float mn = wmin_nonneg(a.amin), mx = wmax_nonneg(a.amax);
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (sums) {
    v[0] = wsum(a.rho);
    v[1] = wsum(a.j[0]);
    v[2] = wsum(a.j[1]);
    v[3] = wsum(a.j[2]);
    v[4] = wsum(a.H);
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < kNumCounts; ++k) sc[w][k] = a.c[k];
    if (ITERS) sc[w][kCntIters] = it;
    sa[w][0] = mn;
    sa[w][1] = mx;
#pragma unroll
    for (int k = 0; k < 5; ++k) ss[w][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    CountRec r;
    for (int k = 0; k < kNumCounts; ++k) {
      uint32_t s = 0;
      for (int q = 0; q < NW; ++q) s += sc[q][k];
      r.cnt[k] = s;
    }
    r.amin = sa[0][0];
    r.amax = sa[0][1];
    for (int q = 1; q < NW; ++q) {
      r.amin = fminf(r.amin, sa[q][0]);
      r.amax = fmaxf(r.amax, sa[q][1]);
    }
    r.pad[0] = r.pad[1] = 0;
    reinterpret_cast<CountRec*>(d.counts)[slot] = r;
    if (sums) {
      SumRec q;
      q.rho = ss[0][0];
      q.j[0] = ss[0][1];
      q.j[1] = ss[0][2];
      q.j[2] = ss[0][3];
      q.H = ss[0][4];
      for (int k = 1; k < NW; ++k) {
        q.rho += ss[k][0];
        q.j[0] += ss[k][1];
        q.j[1] += ss[k][2];
        q.j[2] += ss[k][3];
        q.H += ss[k][4];
      }
      q.pad[0] = q.pad[1] = q.pad[2] = 0.0;
      reinterpret_cast<SumRec*>(d.sums)[slot] = q;
    }
  }
}

// The same when the 64 sites of the wavefront lie in one x-row (nx a
// multiple of 64): the source row of each (c_y, c_z) is then uniform and
// goes into the scalar base address, and only the three x positions
// (x, x - 1, x + 1 with periodic wrap) are per-lane offsets.
template <int D, class T>
__device__ __forceinline__ void load_site_row(const SimDesc& d, const T* src, uint32_t s,
                                              Slot<T> (&raw)[Lattice<D>::Q]) {
  using L = Lattice<D>;
  const uint32_t nx = (uint32_t)d.nx, ny = (uint32_t)d.ny, nz = (uint32_t)d.nz;
  // row index of the wavefront (uniform), x per lane
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
  // A row of nx sites (nx a multiple of 64) is nx/64 whole blocks, i.e.
  // nx Q contiguous elements starting at element (row start) Q.  Within the
  // row, the source x of each lane sits at ((x / 64) Q) 64 + x % 64 plus the
  // direction's 64 i.
  constexpr uint32_t es = sizeof(T);
  constexpr int Q = L::Q;
  uint32_t xo[3];
  const uint32_t xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  xo[0] = (uint32_t)pidx<Q>(x, 0) * es;
  xo[1] = (uint32_t)pidx<Q>(xm, 0) * es;
  xo[2] = (uint32_t)pidx<Q>(xp, 0) * es;
  const gaddr base = buffer_base(src);
  const uint32_t rowbytes = nx * (uint32_t)Q * es;
  // one descriptor per source row (c_y, c_z); direction i's run within the
  // row's blocks is the scalar offset 64 i elements (every address stays
  // inside the row)
#pragma unroll
  for (int dz = 0; dz < (D > 2 ? 3 : 1); ++dz)
#pragma unroll
    for (int dy = 0; dy < (D > 1 ? 3 : 1); ++dy) {
      const __amdgpu_buffer_rsrc_t r =
          rsrc(base + (uint64_t)(zs[dz] + ys[dy]) * Q * es, rowbytes);
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int i = dx + 3 * dy + 9 * dz;
        raw[i] = ld_slot<T>(r, xo[dx], (uint32_t)i * kLane * es);
      }
    }
}

// The loads of a group of TILES tiles that lie in one x-row (nx a multiple of
// TILES kBlock: the group is TILES kBlock consecutive sites of one row, tile
// k's sites are tile 0's plus k kBlock, and their elements sit
// k kBlock Q further on).  The per-lane offsets of tile 0 serve every tile,
// with the tile's shift in the scalar offset; only tile 0's x - 1 and the
// last tile's x + 1 can wrap around the row, and those two take offsets of
// their own.  Every vector offset is a non-negative position inside the row.
template <int D, int TILES, class T>
__device__ __forceinline__ void load_group_row(const SimDesc& d, const T* src, uint32_t s0,
                                               Slot<T> (&raw)[TILES][Lattice<D>::Q]) {
  using L = Lattice<D>;
  constexpr int Q = L::Q;
  constexpr uint32_t es = sizeof(T);
  const uint32_t nx = (uint32_t)d.nx, ny = (uint32_t)d.ny, nz = (uint32_t)d.nz;
  const uint32_t row = __builtin_amdgcn_readfirstlane(D == 1 ? 0u : qdiv(s0, d.inv_nx));
  const uint32_t x = s0 - row * nx;  // tile 0's x
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
  constexpr uint32_t step = (uint32_t)kBlock * Q * es;  // bytes from one tile to the next
  const auto off = [](uint32_t xx) { return (uint32_t)pidx<Q>(xx, 0) * es; };
  const uint32_t o0 = off(x);
  const uint32_t om0 = off(x == 0 ? nx - 1 : x - 1);   // tile 0, x - 1 (wrapped)
  const uint32_t om1 = off(x + kBlock - 1);             // tile 1, x - 1
  const uint32_t op = off(x + 1);                       // x + 1 of the tiles before the last
  const uint32_t xl = x + (TILES - 1) * kBlock;         // the last tile's x
  const uint32_t opl = xl == nx - 1 ? 0u : op + (TILES - 1) * step;  // its x + 1 (wrapped)
  const gaddr base = buffer_base(src);
  const uint32_t rowbytes = nx * (uint32_t)Q * es;
  constexpr int NR = (D > 2 ? 3 : 1) * (D > 1 ? 3 : 1);  // source rows (c_y, c_z)
  __amdgpu_buffer_rsrc_t r[NR];
#pragma unroll
  for (int n = 0; n < NR; ++n)
    r[n] = rsrc(base + (uint64_t)(zs[n / 3] + ys[n % 3]) * Q * es, rowbytes);
  // tile by tile, so that a tile's loads complete before the next tile's
  // (a scheduling barrier per tile keeps the compiler from regrouping them
  // by source row)
#pragma unroll
  for (int k = 0; k < TILES; ++k) {
    if (k > 0) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int n = 0; n < NR; ++n) {
      const int i0 = 3 * n;  // i = dx + 3 dy + 9 dz with n = dy + 3 dz
      const uint32_t so = (uint32_t)i0 * kLane * es;
      // c_x = 0, +1 (source x - 1), -1 (source x + 1)
      raw[k][i0] = ld_slot<T>(r[n], o0, so + k * step);
      raw[k][i0 + 1] = k == 0 ? ld_slot<T>(r[n], om0, so + kLane * es)
                              : ld_slot<T>(r[n], om1, so + kLane * es + (k - 1) * step);
      raw[k][i0 + 2] = k == TILES - 1 ? ld_slot<T>(r[n], opl, so + 2 * kLane * es)
                                      : ld_slot<T>(r[n], op, so + 2 * kLane * es + k * step);
    }
  }
}

// Pull the Q populations of site s (s < N): raw_i = src_i(x - c_i).
template <int D, class T>
__device__ __forceinline__ void load_site(const SimDesc& d, const T* src, uint32_t s,
                                          Slot<T> (&raw)[Lattice<D>::Q]) {
  using L = Lattice<D>;
  const Where w = locate<D>(d, s);
  const gaddr base = buffer_base(src);
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const uint32_t sp = w.zs[L::dg(i, 2)] + w.ys[L::dg(i, 1)] + w.xs[L::dg(i, 0)];
    using U = typename std::conditional<sizeof(T) == 2, uint16_t, T>::type;
    raw[i] = Slot<T>(*(const gptr<U>)(base + pidx<L::Q>(sp, i) * sizeof(T)));
  }
}

// rho and rho u of a site, summed per x-row of directions first: for each
// (c_y, c_z) the three directions c_x = 0, +1, -1 give a row sum and an
// x-momentum term.
template <int D, class R, class G>
__device__ __forceinline__ void moments_of(const G& g, R& rho, R (&j)[3]) {
  constexpr int NY = D > 1 ? 3 : 1, NZ = D > 2 ? 3 : 1;
  R rs[3][3], rx[3][3];
#pragma unroll
  for (int dz = 0; dz < NZ; ++dz)
#pragma unroll
    for (int dy = 0; dy < NY; ++dy) {
      const int i0 = 9 * dz + 3 * dy;
      const R g0 = g(i0), gp = g(i0 + 1), gm = g(i0 + 2);
      rs[dy][dz] = g0 + (gp + gm);
      rx[dy][dz] = gp - gm;
    }
  // sums start from their first term (adding to a zero is not free in IEEE
  // arithmetic)
  R cz[3];
  j[0] = rx[0][0];
#pragma unroll
  for (int dz = 0; dz < NZ; ++dz) {
    cz[dz] = rs[0][dz];
#pragma unroll
    for (int dy = 1; dy < NY; ++dy) cz[dz] += rs[dy][dz];
#pragma unroll
    for (int dy = 0; dy < NY; ++dy)
      if (dy + dz > 0) j[0] += rx[dy][dz];
  }
  rho = cz[0];
#pragma unroll
  for (int dz = 1; dz < NZ; ++dz) rho += cz[dz];
  j[1] = R(0);
  j[2] = R(0);
  if constexpr (D > 1) {
    j[1] = rs[1][0] - rs[2][0];
#pragma unroll
    for (int dz = 1; dz < NZ; ++dz) j[1] += rs[1][dz] - rs[2][dz];
  }
  if constexpr (D > 2) j[2] = cz[1] - cz[2];
}
// rho - rho_ref and rho u from the deviations s_i, in FP32.  With
// W_i = 4^z(i) / 6^D (z: the number of zero components of c_i), the sums
// sum_i W_i s_i and sum_i W_i c_i s_i are 6^-D times sums of 4^z(i) s_i,
// whose factors 4 are exact.  They are formed axis by axis: per source row
// (c_y, c_z), a = 4 s_0 + (s_+ + s_-) and b = s_+ - s_-; over c_y the same
// on the rows' a and b, with a_+ - a_- for the y momentum; then over c_z.
// 6^-D is applied once, in two FP32 parts: its FP32 rounding alone would
// scale every moment by the same wrong factor at every step, a bias that
// the collision hands on to the state.
template <int D, class A, class G>
__device__ __forceinline__ void moments_w4(const G& s, A& dr, A (&j)[3]) {
  constexpr int NY = D > 1 ? 3 : 1, NZ = D > 2 ? 3 : 1;
  A ax[3][3], bx[3][3];  // [c_y][c_z]
#pragma unroll
  for (int dz = 0; dz < NZ; ++dz)
#pragma unroll
    for (int dy = 0; dy < NY; ++dy) {
      const int i0 = 9 * dz + 3 * dy;
      const A s0 = s(i0), sp = s(i0 + 1), sm = s(i0 + 2);
      ax[dy][dz] = fma(A(4), s0, sp + sm);
      bx[dy][dz] = sp - sm;
    }
  A ay[3], by[3], cy[3];  // [c_z]
#pragma unroll
  for (int dz = 0; dz < NZ; ++dz) {
    if constexpr (D > 1) {
      ay[dz] = fma(A(4), ax[0][dz], ax[1][dz] + ax[2][dz]);
      by[dz] = fma(A(4), bx[0][dz], bx[1][dz] + bx[2][dz]);
      cy[dz] = ax[1][dz] - ax[2][dz];
    } else {
      ay[dz] = ax[0][dz];
      by[dz] = bx[0][dz];
      cy[dz] = A(0);
    }
  }
  A S, J[3];
  if constexpr (D > 2) {
    S = fma(A(4), ay[0], ay[1] + ay[2]);
    J[0] = fma(A(4), by[0], by[1] + by[2]);
    J[1] = fma(A(4), cy[0], cy[1] + cy[2]);
    J[2] = ay[1] - ay[2];
  } else {
    S = ay[0];
    J[0] = by[0];
    J[1] = cy[0];
    J[2] = A(0);
  }
  constexpr double c = 1.0 / Lattice<D>::den();
  if constexpr (std::is_same<A, float>::value) {
    constexpr float ch = float(c), cl = float(c - double(float(c)));
    dr = fmaf(ch, S, cl * S);
#pragma unroll
    for (int a = 0; a < 3; ++a) j[a] = a < D ? fmaf(ch, J[a], cl * J[a]) : 0.0f;
  } else {
    dr = A(c) * S;
#pragma unroll
    for (int a = 0; a < 3; ++a) j[a] = a < D ? A(c) * J[a] : A(0);
  }
}

template <int D, class S, class R>
__device__ __forceinline__ void site_moments(const Site<D, S, R>& v, R& rho, R (&j)[3]) {
  moments_of<D>([&](int i) { return v.g(i); }, rho, j);
}

// Loads (or takes) the site's populations, forms rho, u and, for the
// entropic modes, the equilibrium factors.
template <int D, class S, class R>
__device__ __forceinline__ void site_prepare(Site<D, S, R>& v, const SimDesc& d,
                                             const typename S::T* src, uint32_t sl, R& rho,
                                             R (&j)[3], bool equilibrium) {
  v.src = src;
  v.site = sl;
  v.desc = &d;
  v.rho_ref = (R)d.rho_ref;
  site_moments(v, rho, j);
  const R irho = rcp_n<R>(rho);
  v.rho = rho;
  v.irho = irho;
#pragma unroll
  for (int a = 0; a < 3; ++a) v.u[a] = j[a] * irho;
  if (equilibrium) {
    Equilibrium<R, D> eq;
    eq.build(v.u);
    v.fold(eq);
  }
}

// Arithmetic policies: R = double (all FP64) or float (all FP32) is the
// site arithmetic itself; Mixed runs FP32 arithmetic on the deviations
// (SiteDev) and evaluates the entropy differences and alpha in FP64.
struct Mixed {};
template <class P>
constexpr bool kIsMixed = std::is_same<P, Mixed>::value;

// The preparation of the deviation site (SiteDevT): moments of the
// deviations and the per-axis deviations dl of the equilibrium factors, in
// the site's arithmetic A.
template <int D, class S, class A>
__device__ __forceinline__ void site_prepare_dev(SiteDevT<D, S, A>& v, const SimDesc& d,
                                                 const typename S::T* src, uint32_t sl,
                                                 double (&j)[3]) {
  v.src = src;
  v.site = sl;
  v.desc = &d;
  v.r = A(d.rho_ref);
  A dr, jA[3];
  moments_w4<D>([&](int i) { return v.s(i); }, dr, jA);
  const A rho = v.r + dr;
  // FP32: the hardware reciprocal refined by one Newton step and the
  // hardware square root (1 ulp) instead of the correctly rounded library
  // division and square root; FP64: refined estimates
  const A irho = rcp_a(rho);
  A dl[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a < D) {
      const A ua = jA[a] * irho, t = A(3) * ua * ua;
      const A q = t * rcp_hw(A(1) + sqrt_hw(A(1) + t));
      dl[a][0] = -q;
      dl[a][1] = fma(A(3), ua, A(2) * q);
      dl[a][2] = fma(A(-3), ua, A(2) * q);
      v.u[a] = ua;
    } else {
      dl[a][0] = dl[a][1] = dl[a][2] = A(0);
      v.u[a] = 0.0;
    }
  }
  // 1 / (1 + dl_a(c)) from one reciprocal: with F_c = 1 + dl_a(c), the
  // cofactor C_c (product of the other two factors of the axis) and
  // P_a = F_0 F_+ F_- = F_c C_c, 1 / F_c = C_c / P_a.  The x and y axes share
  // one reciprocal, 1 / (rho P_x P_y), times 1/rho's; z has its own.  Each
  // quotient carries a few roundings of the arithmetic (the FP32 hardware
  // reciprocal is good to 1 ulp).
  A F[3][3], C[3][3], P[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a < D) {
#pragma unroll
      for (int c = 0; c < 3; ++c) F[a][c] = A(1) + dl[a][c];
      C[a][0] = F[a][1] * F[a][2];
      C[a][1] = F[a][0] * F[a][2];
      C[a][2] = F[a][0] * F[a][1];
      P[a] = F[a][0] * C[a][0];
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) F[a][c] = C[a][c] = A(1);
      P[a] = A(1);
    }
  }
  const A Rxy = irho * rcp_hw(D > 1 ? P[0] * P[1] : P[0]);
  // s^eq_i = dr + rho (F_x F_y F_z - 1), expanded so that no term cancels:
  // seqA = dr + rho (F_x F_y - 1) = (dr + rho dl_x) + (rho dl_y) F_x and
  // seqB = rho F_x F_y, then s^eq_i = seqA + seqB dl_z
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const A Rx = Rxy * C[0][a];
    const A Ax = fma(rho, dl[0][a], dr);
    const A RFx = rho * F[0][a];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      v.seqA[a][b] = D > 1 ? fma(rho * dl[1][b], F[0][a], Ax) : Ax;
      v.seqB[a][b] = D > 1 ? RFx * F[1][b] : RFx;
      v.rxy[a][b] = D > 1 ? Rx * C[1][b] : Rx;
    }
  }
  const A Rz = D > 2 ? rcp_hw(P[2]) : A(1);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v.dlz[k] = dl[2][k];
    v.rlz[k] = Rz * C[2][k];
  }
  v.dr = dr;
  v.rhoA = rho;
  v.rho = rho;
#pragma unroll
  for (int a = 0; a < 3; ++a) j[a] = jA[a];
}

// Count predicates of one site as bits kCnt*: they are turned into
// wavefront counts by ballots where all lanes of the wavefront are active.
__device__ __forceinline__ uint32_t flag(int k, bool p) { return p ? (1u << k) : 0u; }

struct SiteOut {
  bool deferred;   // left to the rare phase (closed form)
  uint32_t flags;  // count predicates (bits kCnt*)
};

// Diagnostics of one updated site of an entropic mode: per-lane values
// here, count predicates returned.
// Whether rho, u and alpha of a site are all finite (one product carries a
// NaN or infinity of any factor; the trailing + rho catches a zero product).
// The mixed site's values are FP32 numbers and are tested in FP32.
template <class V, class R>
__device__ __forceinline__ bool site_finite(const V& v, R alpha) {
  return isfinite(v.rho * alpha * v.u[0] * v.u[1] * v.u[2] + v.rho);
}
template <int D, class S>
__device__ __forceinline__ bool site_finite(const SiteDev<D, S>& v, double alpha) {
  return isfinite(v.rhoA * float(alpha) * float(v.u[0]) * float(v.u[1]) * float(v.u[2]) +
                  v.rhoA);
}

template <bool SUMS, class V, class R>
__device__ __forceinline__ uint32_t record_site(const SimDesc& d, uint32_t s, bool live,
                                            const V& v, const AlphaOut<R>& ao,
                                            R ftmin, const R (&j)[3], Acc& acc, int diag) {
  constexpr int D = V::kDim;
  const R alpha = ao.alpha, rho = v.rho;
  uint32_t flags = 0;
  if (diag & kDiagCounts) {
    if (live)
      flags = flag(kCntAccept2, ao.accepted2) | flag(kCntAstarLt2, ao.astar_lt2) |
              flag(kCntAlphaLt2, alpha < R(2)) | flag(kCntGuard, ao.guard) |
              flag(kCntFallback, ao.fallback) | flag(kCntNeg, ftmin < R(0)) |
              flag(kCntNonfinite, !site_finite(v, alpha));
    if (live) acc.iters += ao.iters;
    if (SUMS && live && (diag & kDiagSums)) {
      // H(f) = H(f^eq) + D
      acc.H += (double)rho * v.heq_per_rho() + (double)ao.D;
    }
  }
  if (diag & kDiagAlpha) d.alpha[s] = (double)alpha;
  if (live && (diag & kDiagCounts)) {
    acc.amin = fminf(acc.amin, (float)alpha);
    acc.amax = fmaxf(acc.amax, (float)alpha);
    if (SUMS && (diag & kDiagSums)) {
      acc.rho += (double)rho;
#pragma unroll
      for (int a = 0; a < D; ++a) acc.j[a] += (double)j[a];
    }
  }
  return flags;
}

// The site update on the deviations (SiteDevT) in the arithmetic A: FP32
// (the mixed policy, every mode; the entropy differences and alpha in
// FP64), or FP64 (the closed form's common phase on FP16 deviation storage).
template <int D, class S, class A, int MODE, bool SUMS, int PHASE>
__device__ __forceinline__ SiteOut site_update_dev(const SimDesc& d,
                                                const typename S::T* __restrict__ src,
                                                typename S::T* __restrict__ dst, uint32_t s,
                                                bool live,
                                                const Slot<typename S::T> (&raw)[Lattice<D>::Q],
                                                Acc& acc, int diag) {
  using L = Lattice<D>;
  constexpr int Q = L::Q;
  using T = typename S::T;
  constexpr uint32_t es = sizeof(T);
  const uint32_t sl = live ? s : 0u;
  SiteDevT<D, S, A> v;
#pragma unroll
  for (int i = 0; i < Q; ++i) v.raw[i] = Codec<S, double>::keep(from_slot<typename S::T>(raw[i]));
  double j[3];
  site_prepare_dev(v, d, src, sl, j);
  const AlphaOut<double> ao = choose_alpha<MODE, PHASE>(v, d);
  if (PHASE == kPhaseCommon && ao.deferred) return SiteOut{true, 0u};
  const A ab = A(ao.alpha * d.beta);
  const auto P = v.pass_opaque();
  A tmin = A(INFINITY);  // min of f~_i / W_i: its sign is that of f~_i
  const uint32_t lo = (s & 63u) * es;
  const gaddr blk = block_base<Q>(dst, s);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const A si = v.s(i);
    // the common phase of the closed form on 2-byte storage takes the
    // deviations s_i - s^eq_i from its sums (sums_k1)
    constexpr bool kDD = sizeof(T) == 2 && MODE == kClosed && PHASE == kPhaseCommon;
    const A sn = kDD ? fma(-ab, v.dev(i, P), si) : fma(ab, v.seq(i, P) - si, si);
    if constexpr (PHASE != kPhaseCommon) tmin = fmin(tmin, v.r + sn);
    st_nt<T>(blk + i * kLane * es, kLane * es, lo, v.enc(i, sn));
    sched_group(i);
  }
  return SiteOut{false, record_site<SUMS>(d, s, live, v, ao, double(tmin), j, acc, diag)};
}

// The site update in FP64 or FP32 site arithmetic (R), every alpha mode.
template <int D, class S, int MODE, class R, bool SUMS, int PHASE>
__device__ __forceinline__ SiteOut site_update_fp(const SimDesc& d,
                                               const typename S::T* __restrict__ src,
                                               typename S::T* __restrict__ dst, uint32_t s,
                                               bool live, const Slot<typename S::T> (&raw)[Lattice<D>::Q],
                                               Acc& acc, int diag) {
  using L = Lattice<D>;
  constexpr int Q = L::Q;
  using T = typename S::T;
  constexpr uint32_t es = sizeof(T);
  const uint32_t sl = live ? s : 0u;  // the site whose values were loaded

  Site<D, S, R> v;
#pragma unroll
  for (int i = 0; i < Q; ++i) v.raw[i] = Codec<S, R>::keep(from_slot<typename S::T>(raw[i]));
  R rho, j[3];
  site_prepare(v, d, src, sl, rho, j, MODE != kBGK);
  const R beta = (R)d.beta;

  if constexpr (MODE == kBGK) {
    // LBGK: alpha = 2 with the second-order polynomial equilibrium.
    const R* u = v.u;
    const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const R tb = R(2) * beta;
    R ftmin = R(INFINITY);
    uint32_t flags = 0;
    const uint32_t lo = (s & 63u) * es;
    const gaddr blk = block_base<Q>(dst, s);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R cu = R(L::c(i, 0)) * u[0] + R(L::c(i, 1)) * u[1] + R(L::c(i, 2)) * u[2];
      const R fe = R(L::W(i)) * rho * (R(1) + R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu);
      const R gi = v.g(i);
      const R ft = gi + tb * (fe - gi);
      ftmin = fmin(ftmin, ft);
      st_nt<T>(blk + i * kLane * es, kLane * es, lo, Codec<S, R>::enc(ft, R(L::invW(i)), v.rho_ref));
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
        for (int a = 0; a < D; ++a) acc.j[a] += (double)j[a];
      }
    }
    return SiteOut{false, flags};
  } else {
    const AlphaOut<R> ao = choose_alpha<MODE, PHASE>(v, d);
    if (PHASE == kPhaseCommon && ao.deferred) return SiteOut{true, 0u};
    // Eq. (1): f~_i = f_i + alpha beta (f^eq_i - f_i), in the site
    // arithmetic's precision; the result is rounded once, into the storage
    // format.
    const R ab = ao.alpha * beta;
    const auto P = v.pass();
    R ftmin = R(INFINITY);
    const uint32_t lo = (s & 63u) * es;
    const gaddr blk = block_base<Q>(dst, s);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R gi = v.g(i);
      const R ft = fma(ab, v.fe(i, P) - gi, gi);
      // In the common and middle tiers |x_i| <= 0.025 and 0 < alpha beta < 2,
      // so f~_i = f^eq_i (1 + (1 - alpha beta) x_i) > 0.975 f^eq_i: no
      // negative population to look for.
      if constexpr (PHASE != kPhaseCommon) ftmin = fmin(ftmin, ft);
      st_nt<T>(blk + i * kLane * es, kLane * es, lo, Codec<S, R>::enc(ft, R(L::invW(i)), v.rho_ref));
      sched_group(i);
    }
    return SiteOut{false, record_site<SUMS>(d, s, live, v, ao, ftmin, j, acc, diag)};
  }
}

// One site from its pulled populations: moments, equilibrium, alpha,
// collision, store of dst_i(x) at the site's own index.  `live` is false for
// the padding lanes of the last tile: they compute on the values of site 0
// (so that wavefront-wide votes see ordinary numbers) and store into the
// padding blocks past N, which every buffer has up to the next whole tile
// and which no step reads.
//
// PHASE (closed form): kPhaseCommon leaves the lanes that need the rare
// tier untouched and returns true for them; site_update_rare completes them.
// AP: the arithmetic policy (double, float or Mixed).
template <int D, class S, int MODE, class AP, bool SUMS, int PHASE = kPhaseAll>
__device__ __forceinline__ SiteOut site_update(const SimDesc& d, const typename S::T* __restrict__ src,
                                            typename S::T* __restrict__ dst, uint32_t s,
                                            bool live, const Slot<typename S::T> (&raw)[Lattice<D>::Q],
                                            Acc& acc, int diag) {
  // the closed form's common phase on FP16 deviations with FP64 site
  // arithmetic, up to nine directions: the deviation site in FP64 (its rare
  // phase: the FP64 site).  With 27 directions its FP64 state does not fit
  // the registers of three waves per SIMD, and the FP64 site is faster.
  constexpr bool kDev64 = std::is_same<AP, double>::value && Codec<S, double>::kF16 &&
                          MODE == kClosed && PHASE == kPhaseCommon && Lattice<D>::Q <= 9;
  if constexpr (kIsMixed<AP>)
    return site_update_dev<D, S, float, MODE, SUMS, PHASE>(d, src, dst, s, live, raw, acc, diag);
  else if constexpr (kDev64)
    return site_update_dev<D, S, double, MODE, SUMS, PHASE>(d, src, dst, s, live, raw, acc, diag);
  else
    return site_update_fp<D, S, MODE, AP, SUMS, PHASE>(d, src, dst, s, live, raw, acc, diag);
}

// The rare path of the mixed policy (SiteDev).
template <int D, class S, int MODE, bool SUMS>
__device__ __forceinline__ uint32_t site_update_rare_dev(const SimDesc& d, const typename S::T* __restrict__ src,
    typename S::T* __restrict__ dst, uint32_t s, bool live, Acc& acc, int diag) {
  using L = Lattice<D>;
  constexpr int Q = L::Q;
  using T = typename S::T;
  constexpr uint32_t es = sizeof(T);
  const uint32_t sl = live ? s : 0u;
  SiteDev<D, S> v;
  if constexpr (Codec<S, double>::kF16) {
    Slot<T> raw[Q];
    load_site<D>(d, src, sl, raw);
#pragma unroll
    for (int i = 0; i < Q; ++i) v.raw[i] = Codec<S, double>::keep(from_slot<T>(raw[i]));
  } else {
    load_site<D>(d, src, sl, v.raw);
  }
  double j[3];
  site_prepare_dev(v, d, src, sl, j);
  const AlphaOut<double> ao = choose_alpha<MODE, kPhaseRare>(v, d);
  const float ab = float(ao.alpha * d.beta);
  float tmin = INFINITY;
  const uint32_t lo = (s & 63u) * es;
  const gaddr blk = block_base<Q>(dst, s);
#pragma unroll 1
  for (int i = 0; i < Q; ++i) {
    float si, seqi;
    v.sq(i, si, seqi);
    const float sn = fmaf(ab, seqi - si, si);
    tmin = fminf(tmin, v.r + sn);
    T out;
    if constexpr (S::dev)
      out = T(sn);
    else
      out = SiteDev<D, S>::enc_f(SiteDev<D, S>::weight_of(i), SiteDev<D, S>::weight_lo(i), v.r, sn);
    st_nt<T>(blk + (uint64_t)i * kLane * es, kLane * es, lo, out);
  }
  return record_site<SUMS>(d, s, live, v, ao, double(tmin), j, acc, diag);
}

// The rare path in FP64 or FP32 site arithmetic (R).
template <int D, class S, int MODE, class R, bool SUMS>
__device__ __forceinline__ uint32_t site_update_rare_fp(const SimDesc& d, const typename S::T* __restrict__ src,
    typename S::T* __restrict__ dst, uint32_t s, bool live, Acc& acc, int diag) {
  using L = Lattice<D>;
  constexpr int Q = L::Q;
  using T = typename S::T;
  constexpr uint32_t es = sizeof(T);
  const uint32_t sl = live ? s : 0u;
  Site<D, S, R> v;
  if constexpr (Codec<S, R>::kF16) {
    Slot<T> raw[Q];
    load_site<D>(d, src, sl, raw);
#pragma unroll
    for (int i = 0; i < Q; ++i) v.raw[i] = Codec<S, R>::keep(from_slot<T>(raw[i]));
  } else {
    load_site<D>(d, src, sl, v.raw);
  }
  R rho, j[3];
  site_prepare(v, d, src, sl, rho, j, true);
  const AlphaOut<R> ao = choose_alpha<MODE, kPhaseRare>(v, d);
  const uint32_t lo = (s & 63u) * es;
  const gaddr blk = block_base<Q>(dst, s);
  const R ab = ao.alpha * (R)d.beta;
  R ftmin = R(INFINITY);
#pragma unroll 1
  for (int i = 0; i < Q; ++i) {
    R xi, fi, gi;
    v.xfe(i, xi, fi, &gi);
    const R ft = fma(ab, fi - gi, gi);
    ftmin = fmin(ftmin, ft);
    const int nz0 = (i % 3 == 0) + (D > 1 && (i / 3) % 3 == 0) + (D > 2 && i / 9 == 0);
    const R invW = R(L::den()) / R(nz0 == 0 ? 1.0 : nz0 == 1 ? 4.0 : nz0 == 2 ? 16.0 : 64.0);
    st_nt<T>(blk + (uint64_t)i * kLane * es, kLane * es, lo, Codec<S, R>::enc(ft, invW, v.rho_ref));
  }
  return record_site<SUMS>(d, s, live, v, ao, ftmin, j, acc, diag);
}

// A lane deferred by the common phase: the populations are reloaded (from
// the caches, which this wavefront has just filled), the moments and the
// equilibrium recomputed by the same arithmetic, alpha taken from the rare
// tier, and the collision run as a rolled loop that re-reads each
// population, so no per-direction array stays live across the logarithms.
template <int D, class S, int MODE, class AP, bool SUMS>
__device__ __forceinline__ uint32_t site_update_rare(const SimDesc& d,
                                                 const typename S::T* __restrict__ src,
                                                 typename S::T* __restrict__ dst, uint32_t s,
                                                 bool live, Acc& acc, int diag) {
  if constexpr (kIsMixed<AP>)
    return site_update_rare_dev<D, S, MODE, SUMS>(d, src, dst, s, live, acc, diag);
  else
    return site_update_rare_fp<D, S, MODE, AP, SUMS>(d, src, dst, s, live, acc, diag);
}

// One workgroup per ELBM_TILES tiles of kBlock consecutive sites; the loads
// of all its tiles are issued before the first tile's arithmetic, so that
// the later tiles' memory latency overlaps it.
//
// XCD-aware order: workgroups are issued round-robin over the 8 XCDs
// (workgroup b runs on XCD b mod 8), so the tile order is permuted to give
// each XCD one contiguous eighth of the box: neighbouring tiles, which share
// the cache lines at their x-edges, then run on the same XCD and L2.  Each
// simulation's workgroup count is a multiple of 8 and starts at a multiple
// of 8.
// The root solvers and FP64 storage keep the registers they need (Newton,
// the secant and bisection with 2- and 4-byte storage: three waves per
// SIMD; their passes over the register-held populations fit without
// spilling outside the diagnostics-sums variants).
#ifndef ELBM_NEWTON_WAVES
#define ELBM_NEWTON_WAVES 3
#endif
#ifndef ELBM_CLOSED_WAVES
#define ELBM_CLOSED_WAVES 4
#endif
// Waves per SIMD the step kernel is compiled for.  Closed form and LBGK on
// 4-byte storage: four (at most 128 VGPRs; the common path has no spills).
// Closed form on 2-byte storage: three (its common path holds about 140
// VGPRs: the decoded deviations and the per-axis factors of both the
// equilibrium and its reciprocal; four waves spill in the common path and
// run 5.02 ms against 3.86 ms at 512^3 with mixed arithmetic).
template <class S, int MODE>
constexpr int step_waves() {
  if (sizeof(typename S::T) == 2 && MODE == kClosed) return 3;
  if (sizeof(typename S::T) <= 4 && (MODE == kClosed || MODE == kBGK)) return ELBM_CLOSED_WAVES;
  if (sizeof(typename S::T) <= 4 && (MODE == kNewton || MODE == kSecant || MODE == kBisect))
    return ELBM_NEWTON_WAVES;
  return 1;
}

template <int D, class S, int MODE, class R, bool SUMS>
__global__ void __launch_bounds__(kBlock, (step_waves<S, MODE>())) k_step(const BatchArgs args) {
  using T = typename S::T;
  constexpr int Q = Lattice<D>::Q;
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
  const uint32_t unit = (lb & 7u) * chunk + (lb >> 3);  // this workgroup's tile group
  Acc acc;
  acc.init();
  if (unit * ELBM_TILES * kBlock < N) {
    Slot<T> raw[ELBM_TILES][Q];
#if ELBM_LOAD_PRIO
    __builtin_amdgcn_s_setprio(ELBM_LOAD_PRIO);
#endif
    // the loads of every tile issued back to back, on one path (a branch per
    // tile would put control-flow joins between them, at which the
    // compiler's wait counting turns conservative)
    const uint32_t s0 = unit * ELBM_TILES * kBlock + threadIdx.x;
    if (ELBM_TILES > 1 && d.nx % (ELBM_TILES * kBlock) == 0) {
      // (then N is a multiple of the group: every site is live)
      load_group_row<D, ELBM_TILES>(d, src, s0, raw);
    } else if (d.nx % 64 == 0) {
#pragma unroll
      for (int k = 0; k < ELBM_TILES; ++k) {
        const uint32_t s = s0 + k * kBlock;
        load_site_row<D>(d, src, s < N ? s : 0u, raw[k]);
      }
    } else {
#pragma unroll
      for (int k = 0; k < ELBM_TILES; ++k) {
        const uint32_t s = s0 + k * kBlock;
        load_site<D>(d, src, s < N ? s : 0u, raw[k]);
      }
    }
#if ELBM_LOAD_PRIO
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_setprio(0);
#endif
    uint32_t flags = 0;
    if constexpr (MODE == kClosed) {
      // A lane the common phase completes has alpha_* = 2, no negative
      // population (|x_i| <= 0.025) and finite values (a non-finite max|x_i|
      // fails the tier tests and is deferred): only these counts can be set.
      constexpr uint32_t kCommonFlags =
          (1u << kCntAccept2) | (1u << kCntAlphaLt2) | (1u << kCntGuard);
      // the closed form in two phases: the rare tier after the common one
      bool deferred[ELBM_TILES];
#pragma unroll
      for (int k = 0; k < ELBM_TILES; ++k) {
        const uint32_t s = (unit * ELBM_TILES + k) * kBlock + threadIdx.x;
        deferred[k] = false;
        if (k == 0 || (unit * ELBM_TILES + k) * kBlock < N) {
          const SiteOut o = site_update<D, S, MODE, R, SUMS, kPhaseCommon>(d, src, dst, s, s < N,
                                                                           raw[k], acc, diag);
          deferred[k] = o.deferred;
          flags = o.flags;
        }
        if (ELBM_TILES > 1 && (diag & kDiagCounts)) {
          acc.count_flags<kCommonFlags>(flags);
          flags = 0;
        }
      }
      if (ELBM_TILES == 1 && (diag & kDiagCounts)) acc.count_flags<kCommonFlags>(flags);
      flags = 0;
#pragma unroll
      for (int k = 0; k < ELBM_TILES; ++k) {
        if (__any(deferred[k])) {
          uint32_t f = 0;
          if (deferred[k]) {
            const uint32_t s = (unit * ELBM_TILES + k) * kBlock + threadIdx.x;
            f = site_update_rare<D, S, MODE, R, SUMS>(d, src, dst, s, s < N, acc, diag);
          }
          if (diag & kDiagCounts) acc.count_flags(f);
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < ELBM_TILES; ++k) {
        const uint32_t s = (unit * ELBM_TILES + k) * kBlock + threadIdx.x;
        if (k == 0 || (unit * ELBM_TILES + k) * kBlock < N)
          flags = site_update<D, S, MODE, R, SUMS>(d, src, dst, s, s < N, raw[k], acc, diag).flags;
        if (ELBM_TILES > 1 && (diag & kDiagCounts)) {
          acc.count_flags(flags);
          flags = 0;
        }
      }
      if (ELBM_TILES == 1 && (diag & kDiagCounts)) acc.count_flags(flags);
    }
  } else if (!(diag & kDiagCounts)) {
    return;  // padding workgroup
  }
  if (diag & kDiagCounts)
    store_records<MODE == kNewton || MODE == kBisect || MODE == kSecant>(acc, d, (int)lb);
}

// The sums of ELBM_DIAG_SUMS (which need logarithms per site) are compiled
// into a kernel of their own, used when a simulation of the batch asks for
// them, so that the other kernels do not carry their registers.
template <int D, class S, int MODE, class R>
hipError_t launch_step(const BatchArgs& a, int grid, hipStream_t st) {
  bool sums = false;
  for (int k = 0; k < a.n; ++k) sums = sums || (a.d[k].diag & kDiagSums);
  if (sums)
    k_step<D, S, MODE, R, true><<<grid, kBlock, 0, st>>>(a);
  else
    k_step<D, S, MODE, R, false><<<grid, kBlock, 0, st>>>(a);
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
  if (mode != kClosed) return nullptr;
  if (fp64 == kArithMixed) {
    switch (storage) {
      case kStoreF32: return &launch_step<D, StoreF32, kClosed, Mixed>;
      case kStoreF32Dev: return &launch_step<D, StoreF32Dev, kClosed, Mixed>;
      case kStoreF16Dev: return &launch_step<D, StoreF16Dev, kClosed, Mixed>;
      default: return nullptr;
    }
  }
  if (fp64 != kArithF32) return nullptr;
  switch (storage) {
    case kStoreF32: return &launch_step<D, StoreF32, kClosed, float>;
    case kStoreF32Dev: return &launch_step<D, StoreF32Dev, kClosed, float>;
    case kStoreF16Dev: return &launch_step<D, StoreF16Dev, kClosed, float>;
    default: return nullptr;
  }
}

}  // namespace elbm
