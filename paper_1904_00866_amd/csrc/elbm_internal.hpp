// elbm_internal.hpp -- types shared by the kernels and the host runtime of
// the ELBM library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace elbm {

constexpr int kBlock = 256;        // threads per workgroup of the step kernel

// Tiles of kBlock sites per step workgroup, whose loads a wavefront issues
// before the first tile's arithmetic.  Lattices with 19 or 27 directions:
// one; they run four waves per SIMD, which hide the memory latency better
// than a second tile's loads issued ahead within one wave.  Lattices with 3
// or 9 directions have few loads per site, so more tiles put more bytes in
// flight per wave (ELBM_TILES_SMALLQ; 2- and 4-byte storage only).
#ifndef ELBM_TILES_NARROW
#define ELBM_TILES_NARROW 1
#endif
#ifndef ELBM_TILES_SMALLQ
#define ELBM_TILES_SMALLQ 4
#endif
constexpr int tiles_per_block(int elem_bytes, int Q) {
  return elem_bytes < 8 ? (Q <= 9 ? ELBM_TILES_SMALLQ : ELBM_TILES_NARROW) : 1;
}
constexpr int kMaxBatch = 16;      // simulations per batched launch
constexpr int kCountBytes = 48;    // per-workgroup counts record
constexpr int kSumBytes = 64;      // per-workgroup sums record

// Diagnostics bits (same values as ELBM_DIAG_* of the public header).
constexpr int kDiagAlpha = 1, kDiagCounts = 2, kDiagSums = 4;

// Storage codes (same values as ELBM_STORE_*).
constexpr int kStoreF64 = 0, kStoreF32 = 1, kStoreF32Dev = 2, kStoreF16Dev = 3;
// Site arithmetic codes (same values as ELBM_ARITH_*).
constexpr int kArithF32 = 0, kArithF64 = 1, kArithMixed = 2;

// Alpha modes (same values as ELBM_ALPHA_*).
constexpr int kClosed = 0, kNewton = 1, kBisect = 2, kBGK = 3, kSecant = 4;

// Population layout of a buffer: blocks of kLane = 64 consecutive sites
// (one wavefront's sites), each block holding its Q directions one after
// another as kLane values:
//   element (i, s) is at ((s / 64) Q + i) 64 + s % 64.
// A wavefront then reads and writes Q contiguous runs inside one block of
// 64 Q elements instead of Q runs spread over Q separate planes, which the
// memory system serves markedly faster.  A buffer holds the padded site
// range (whole workgroup tiles), so the idle lanes of the last tile write
// into blocks that no step reads.
constexpr int kLane = 64;
template <int Q>
__host__ __device__ __forceinline__ uint64_t pidx(uint64_t s, int i) {
  return ((s >> 6) * (uint64_t)Q + (uint64_t)i) * (uint64_t)kLane + (s & 63u);
}

// One simulation as the step kernel sees it.  The step kernel reads `src`
// (post-collision values of the previous step; pulling src_i(x - c_i)
// gives f_i(x, t)) and writes `dst` at each site.
struct SimDesc {
  const void* src;
  void* dst;
  double* alpha;    // alpha(x) of this step, or nullptr
  void* counts;     // nblocks CountRec records, or nullptr
  void* sums;       // nblocks SumRec records, or nullptr
  int64_t padded;   // sites in the buffers (a multiple of the tile size)
  double beta, rho_ref, root_tol;
  double inv_nx, inv_ny;     // 1/nx, 1/ny for the site-coordinate quotients
  int32_t nx, ny, nz, rows;  // rows = ny * nz x-rows of nx sites
  int32_t nblocks;           // workgroups given to this simulation
  int32_t block_begin;       // first workgroup of this simulation
  int32_t root_max_iter, secant_iters;
  int32_t diag;              // kDiag* bits for this step
  int32_t pad_;
};

struct BatchArgs {
  SimDesc d[kMaxBatch];
  int32_t n;
};

// Per-workgroup diagnostics records.  Counts are per site: accepted alpha = 2,
// alpha_max < 2, alpha < 2, guard, long-series/log1p path, a negative output
// population, a non-finite rho/u/alpha; then root-solver iterations.
enum { kCntAccept2 = 0, kCntAstarLt2, kCntAlphaLt2, kCntGuard, kCntFallback, kCntNeg,
       kCntNonfinite, kCntIters, kNumCounts };
struct CountRec {
  uint32_t cnt[kNumCounts];
  float amin, amax;
  uint32_t pad[2];
};
static_assert(sizeof(CountRec) == kCountBytes, "count record size");
struct SumRec {
  double rho, j[3], H, pad[3];
};
static_assert(sizeof(SumRec) == kSumBytes, "sum record size");

// Reduced diagnostics (layout of elbm_stats_t after its `step` field).
struct Reduced {
  int64_t n_sites;
  int64_t cnt[8];
  double amin, amax, rho, j[3], H;
};

// Launchers (defined in the kernel translation units).  Each returns the
// hipError_t of its launch.
using StepLauncher = hipError_t (*)(const BatchArgs&, int grid, hipStream_t);
// lattice: 1, 2, 3 (D1Q3, D2Q9, D3Q27) or 19 (D3Q19); entropy: 0 Boltzmann, 1 Burg
StepLauncher step_launcher(int lattice, int storage, int mode, int fp64, int entropy);
StepLauncher step_launcher_d1(int storage, int mode, int fp64);
StepLauncher step_launcher_d2(int storage, int mode, int fp64);
StepLauncher step_launcher_d3(int storage, int mode, int fp64);
StepLauncher step_launcher_q19(int storage, int mode, int fp64);
StepLauncher step_launcher_burg(int lattice, int storage, int mode, int fp64);

// Auxiliary kernels: a population buffer `buf` in the layout of pidx().
struct BoxDesc {
  int lattice, D, storage;
  int entropy;  // 0 Boltzmann, 1 Burg (the equilibrium that init places)
  int32_t nx, ny, nz;
  int64_t N, padded;
  double rho_ref;
};
hipError_t launch_validate_init(const BoxDesc& b, const double* rho0, const double* u0,
                                unsigned long long* bad, hipStream_t st);
// which = 0: write f^eq(rho0, u0) in pull convention; 1: write given f(x,t)
hipError_t launch_scatter(const BoxDesc& b, void* buf, const double* rho0, const double* u0,
                          const double* f, int which, hipStream_t st);
// which = 0: pre-collision f(x,t) (pull); 1: stored value at x
hipError_t launch_gather(const BoxDesc& b, const void* buf, const int64_t* sites, int64_t n,
                         int which, double* out, hipStream_t st);
hipError_t launch_moments(const BoxDesc& b, const void* buf, double* rho, double* u,
                          hipStream_t st);
hipError_t launch_reduce(const void* counts, const void* sums, int nblocks, Reduced* out,
                         hipStream_t st);
hipError_t launch_copy_f64(const double* src, double* dst, int64_t n, hipStream_t st);

}  // namespace elbm
