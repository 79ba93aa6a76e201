// elbm_aux.hip -- auxiliary kernels of the ELBM library: validation and
// placement of initial states, gathers of f(x,t), moments, and the
// fixed-order reduction of the per-workgroup diagnostics records.
//
// Pull convention: the buffer read by the next step holds P_i(y) with
// P_i(x - c_i) = f_i(x, t), i.e. the post-collision values of the previous
// step before streaming (Eq. (5b) is carried out by the reader).
#include "elbm_internal.hpp"
#include "elbm_burg.hpp"
#include "elbm_q19.hpp"
#include "elbm_site.hpp"

namespace elbm {

namespace {

struct Coord {
  int64_t x, y, z;
};

__device__ __forceinline__ Coord coord_of(const BoxDesc& b, int64_t s) {
  Coord c;
  c.x = s % b.nx;
  const int64_t r = s / b.nx;
  c.y = r % b.ny;
  c.z = r / b.ny;
  return c;
}

__device__ __forceinline__ int64_t wrapi(int64_t v, int64_t n) {
  return v < 0 ? v + n : (v >= n ? v - n : v);
}

// site index of x - c_i
template <class L>
__device__ __forceinline__ int64_t upstream(const BoxDesc& b, const Coord& c, int i) {
  const int64_t x = wrapi(c.x - L::c(i, 0), b.nx);
  const int64_t y = wrapi(c.y - L::c(i, 1), b.ny);
  const int64_t z = wrapi(c.z - L::c(i, 2), b.nz);
  return x + b.nx * (y + b.ny * z);
}

// rho0 > 0 and u0 inside the hull of the velocities: |u_a| < 1, and on
// D3Q19 (no corner velocities, hull2 set) also |u_x| + |u_y| + |u_z| < 2.
__global__ void k_validate(int64_t N, int D, int hull2, const double* __restrict__ rho0,
                           const double* __restrict__ u0, unsigned long long* bad) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int ok = 1;
  if (s < N) {
    ok = rho0[s] > 0.0 && isfinite(rho0[s]);
    double l1 = 0.0;
    for (int a = 0; a < D; ++a) {
      ok = ok && fabs(u0[a * N + s]) < 1.0;
      l1 += fabs(u0[a * N + s]);
    }
    if (hull2) ok = ok && l1 < 2.0;
  }
  const unsigned long long nb = __ballot(!ok);
  if ((threadIdx.x & 63) == 0 && nb) atomicAdd(bad, (unsigned long long)__popcll(nb));
}

template <class L, class S>
__global__ void k_scatter(const BoxDesc b, typename S::T* __restrict__ buf,
                          const double* __restrict__ rho0, const double* __restrict__ u0,
                          const double* __restrict__ f, int which) {
  constexpr int D = L::Dim;
  constexpr int Q = L::Q;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.N) return;
  const Coord c = coord_of(b, s);
  double fv[Q];
  if (which == 0) {
    double u[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < D; ++a) u[a] = u0[a * b.N + s];
    if (b.entropy == 1) {
      // Burg's entropy: f^eq_i = W_i / d_i (elbm_burg.hpp)
      double mu[4];
      burg_multipliers<L>(rho0[s], 1.0 / rho0[s], u, mu);
#pragma unroll
      for (int i = 0; i < Q; ++i) fv[i] = L::W(i) / burg_den<L>(mu, i);
    } else if constexpr (Q == 19) {
      // f^eq_i = rho W_i prod_a X_a^c_ia / Z  (EquilibriumQ19)
      EquilibriumQ19<double> eq;
      eq.build(u);
      const double cF = rho0[s] / eq.Z9;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        double p = cF * (9.0 * L::W(i));
#pragma unroll
        for (int a = 0; a < 3; ++a)
          p *= L::dg(i, a) == 0 ? 1.0 : (L::dg(i, a) == 1 ? eq.X[a] : eq.Y[a]);
        fv[i] = p;
      }
    } else {
      Equilibrium<double, D> eq;
      eq.build(u);
#pragma unroll
      for (int i = 0; i < Q; ++i)
        fv[i] = rho0[s] * (eq.e(0, L::dg(i, 0)) * eq.e(1, L::dg(i, 1))) * eq.e(2, L::dg(i, 2));
    }
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) fv[i] = f[i * b.N + s];
  }
#pragma unroll
  for (int i = 0; i < Q; ++i)
    buf[pidx<Q>(upstream<L>(b, c, i), i)] =
        Codec<S, double>::enc(fv[i], L::invW(i), b.rho_ref);
}

template <class L, class S>
__global__ void k_gather(const BoxDesc b, const typename S::T* __restrict__ buf,
                         const int64_t* __restrict__ sites, int64_t n, int which,
                         double* __restrict__ out) {
  constexpr int Q = L::Q;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t s = sites ? sites[k] : k;
  if (s < 0 || s >= b.N) {
    for (int i = 0; i < Q; ++i) out[i * n + k] = NAN;
    return;
  }
  const Coord c = coord_of(b, s);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int64_t src = which == 0 ? upstream<L>(b, c, i) : s;
    out[i * n + k] = Codec<S, double>::dec(buf[pidx<Q>(src, i)], L::W(i), b.rho_ref);
  }
}

template <class L, class S>
__global__ void k_moments(const BoxDesc b, const typename S::T* __restrict__ buf,
                          double* __restrict__ rho, double* __restrict__ u) {
  constexpr int D = L::Dim;
  constexpr int Q = L::Q;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.N) return;
  const Coord c = coord_of(b, s);
  double r = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double g = Codec<S, double>::dec(buf[pidx<Q>(upstream<L>(b, c, i), i)], L::W(i), b.rho_ref);
    r += g;
    for (int a = 0; a < D; ++a) j[a] += L::c(i, a) * g;
  }
  rho[s] = r;
  for (int a = 0; a < D; ++a) u[a * b.N + s] = j[a] / r;
}

// Fixed-order reduction of the per-workgroup records: thread t folds records
// t, t + kBlock, ... in order, then a fixed tree combines the threads.
__global__ void k_reduce(const CountRec* __restrict__ cr, const SumRec* __restrict__ sr, int n,
                         Reduced* __restrict__ out) {
  __shared__ double sd[kBlock][5];
  __shared__ float sa[kBlock][2];
  __shared__ unsigned long long sc[kBlock][kNumCounts];
  const int t = threadIdx.x;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  float mn = INFINITY, mx = -INFINITY;
  unsigned long long c[kNumCounts];
  for (int m = 0; m < kNumCounts; ++m) c[m] = 0;
  for (int k = t; k < n; k += kBlock) {
    const CountRec& q = cr[k];
    for (int m = 0; m < kNumCounts; ++m) c[m] += q.cnt[m];
    mn = fminf(mn, q.amin);
    mx = fmaxf(mx, q.amax);
    if (sr) {
      const SumRec& w = sr[k];
      v[0] += w.rho; v[1] += w.j[0]; v[2] += w.j[1]; v[3] += w.j[2]; v[4] += w.H;
    }
  }
  for (int m = 0; m < 5; ++m) sd[t][m] = v[m];
  sa[t][0] = mn;
  sa[t][1] = mx;
  for (int m = 0; m < kNumCounts; ++m) sc[t][m] = c[m];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (t < w) {
      for (int m = 0; m < 5; ++m) sd[t][m] += sd[t + w][m];
      sa[t][0] = fminf(sa[t][0], sa[t + w][0]);
      sa[t][1] = fmaxf(sa[t][1], sa[t + w][1]);
      for (int m = 0; m < kNumCounts; ++m) sc[t][m] += sc[t + w][m];
    }
    __syncthreads();
  }
  if (t == 0) {
    for (int m = 0; m < kNumCounts; ++m) out->cnt[m] = (int64_t)sc[0][m];
    out->amin = sa[0][0];
    out->amax = sa[0][1];
    out->rho = sd[0][0];
    out->j[0] = sd[0][1]; out->j[1] = sd[0][2]; out->j[2] = sd[0][3];
    out->H = sd[0][4];
  }
}

__global__ void k_copy_f64(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) b[s] = a[s];
}

inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// lattice: 1, 2, 3 (D1Q3, D2Q9, D3Q27) or 19 (D3Q19)
template <template <class, class> class Fn, class... A>
hipError_t dispatch(int lattice, int storage, A&&... a) {
#define ELBM_ST(LL)                                                            \
  switch (storage) {                                                           \
    case kStoreF64: return Fn<LL, StoreF64>::run(a...);                        \
    case kStoreF32: return Fn<LL, StoreF32>::run(a...);                        \
    case kStoreF32Dev: return Fn<LL, StoreF32Dev>::run(a...);                  \
    case kStoreF16Dev: return Fn<LL, StoreF16Dev>::run(a...);                  \
    default: return hipErrorInvalidValue;                                      \
  }
  switch (lattice) {
    case 1: ELBM_ST(Lattice<1>)
    case 2: ELBM_ST(Lattice<2>)
    case 3: ELBM_ST(Lattice<3>)
    case 19: ELBM_ST(LatticeQ19)
    default: return hipErrorInvalidValue;
  }
#undef ELBM_ST
}

template <class L, class S>
struct ScatterFn {
  static hipError_t run(const BoxDesc& b, void* buf, const double* rho0, const double* u0,
                        const double* f, int which, hipStream_t st) {
    if (b.N == 0) return hipSuccess;
    k_scatter<L, S><<<grid_for(b.N, 256), 256, 0, st>>>(b, static_cast<typename S::T*>(buf),
                                                       rho0, u0, f, which);
    return hipGetLastError();
  }
};

template <class L, class S>
struct GatherFn {
  static hipError_t run(const BoxDesc& b, const void* buf, const int64_t* sites, int64_t n,
                        int which, double* out, hipStream_t st) {
    if (n == 0) return hipSuccess;
    k_gather<L, S><<<grid_for(n, 256), 256, 0, st>>>(b, static_cast<const typename S::T*>(buf),
                                                    sites, n, which, out);
    return hipGetLastError();
  }
};

template <class L, class S>
struct MomentsFn {
  static hipError_t run(const BoxDesc& b, const void* buf, double* rho, double* u,
                        hipStream_t st) {
    if (b.N == 0) return hipSuccess;
    k_moments<L, S><<<grid_for(b.N, 256), 256, 0, st>>>(b, static_cast<const typename S::T*>(buf),
                                                       rho, u);
    return hipGetLastError();
  }
};

}  // namespace

hipError_t launch_validate_init(const BoxDesc& b, const double* rho0, const double* u0,
                                unsigned long long* bad, hipStream_t st) {
  if (b.N == 0) return hipSuccess;
  k_validate<<<grid_for(b.N, 256), 256, 0, st>>>(b.N, b.D, b.lattice == 19, rho0, u0, bad);
  return hipGetLastError();
}

hipError_t launch_scatter(const BoxDesc& b, void* buf, const double* rho0, const double* u0,
                          const double* f, int which, hipStream_t st) {
  return dispatch<ScatterFn>(b.lattice, b.storage, b, buf, rho0, u0, f, which, st);
}

hipError_t launch_gather(const BoxDesc& b, const void* buf, const int64_t* sites, int64_t n,
                         int which, double* out, hipStream_t st) {
  return dispatch<GatherFn>(b.lattice, b.storage, b, buf, sites, n, which, out, st);
}

hipError_t launch_moments(const BoxDesc& b, const void* buf, double* rho, double* u,
                          hipStream_t st) {
  return dispatch<MomentsFn>(b.lattice, b.storage, b, buf, rho, u, st);
}

hipError_t launch_reduce(const void* counts, const void* sums, int nblocks, Reduced* out,
                         hipStream_t st) {
  k_reduce<<<1, kBlock, 0, st>>>(static_cast<const CountRec*>(counts),
                                 static_cast<const SumRec*>(sums), nblocks, out);
  return hipGetLastError();
}

hipError_t launch_copy_f64(const double* src, double* dst, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  k_copy_f64<<<grid_for(n, 256), 256, 0, st>>>(src, dst, n);
  return hipGetLastError();
}

StepLauncher step_launcher(int lattice, int storage, int mode, int fp64, int entropy) {
  if (entropy == 1) return step_launcher_burg(lattice, storage, mode, fp64);
  if (entropy != 0) return nullptr;
  switch (lattice) {
    case 1: return step_launcher_d1(storage, mode, fp64);
    case 2: return step_launcher_d2(storage, mode, fp64);
    case 3: return step_launcher_d3(storage, mode, fp64);
    case 19: return step_launcher_q19(storage, mode, fp64);
    default: return nullptr;
  }
}

}  // namespace elbm
