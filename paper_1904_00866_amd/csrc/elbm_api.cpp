// elbm_api.cpp -- host runtime of the ELBM library: configuration checks,
// placement of the state in the caller's device buffer, launch set-up,
// stream handling and error reporting behind the C ABI of include/elbm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/elbm.h"
#include "elbm_internal.hpp"

using namespace elbm;

static_assert(kStoreF64 == ELBM_STORE_F64 && kStoreF32 == ELBM_STORE_F32 &&
                  kStoreF32Dev == ELBM_STORE_F32_DEV && kStoreF16Dev == ELBM_STORE_F16_DEV,
              "storage codes");
static_assert(kArithF32 == ELBM_ARITH_FP32 && kArithF64 == ELBM_ARITH_FP64 &&
                  kArithMixed == ELBM_ARITH_MIXED,
              "arithmetic codes");

namespace {

thread_local std::string g_err;

elbm_status fail(elbm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

elbm_status hip_fail(hipError_t e, const char* what) {
  return fail(ELBM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
constexpr int64_t kMaxDim = (1 << 20) - 1;  // site-coordinate arithmetic limit
constexpr int64_t kMaxSites = (int64_t(1) << 31) - 1;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ---- the diagnostics scratch of elbm_step_noalloc ---------------------------
// A file-scope device array that holds the per-workgroup diagnostics records
// (counts, then sums) of the steps elbm_step_noalloc runs, so that it needs
// no workspace from the caller.  Every GPU the library runs on holds its own
// copy (kScratchBytes) until the process ends.  In host code `scratch` names
// a host-side stand-in, not device memory: kernels get the device's own
// address, looked up once per device with that device current.
constexpr int kScratchBlocks = 65536;  // workgroup records: up to 2^24 sites
constexpr size_t kScratchCountBytes = size_t(kScratchBlocks) * kCountBytes;
constexpr size_t kScratchBytes = kScratchCountBytes + size_t(kScratchBlocks) * kSumBytes;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
void* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];

// The address of `scratch` on device dev, which must be the current device;
// looked up on the first call for that device and kept.
hipError_t scratch_on(int dev, void** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::call_once(g_scratch_once[dev], [dev] {
    void* p = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? p : nullptr;
  });
  *out = g_scratch_ptr[dev];
  return g_scratch_err[dev];
}

// step and n_sites of a device elbm_stats_t (the rest comes from k_reduce)
__global__ void k_stats_header(elbm_stats_t* out, int64_t step, int64_t n_sites) {
  out->step = step;
  out->n_sites = n_sites;
}
static_assert(offsetof(elbm_stats_t, n_sites) == 8 && offsetof(elbm_stats_t, sum_H) ==
                  8 + offsetof(Reduced, H) && sizeof(elbm_stats_t) == 8 + sizeof(Reduced),
              "Reduced is elbm_stats_t after its step field");

int elem_size(int storage) {
  switch (storage) {
    case ELBM_STORE_F64: return 8;
    case ELBM_STORE_F32: return 4;
    case ELBM_STORE_F32_DEV: return 4;
    case ELBM_STORE_F16_DEV: return 2;
    default: return 0;
  }
}

struct Layout {
  int lattice, D, Q, esize;
  int64_t N, padded;
  int nblocks;
  size_t off_buf[2], off_alpha, off_counts, off_sums, off_misc, total;
};

elbm_status check_config(const elbm_config* c, Layout* L) {
  if (!c) return fail(ELBM_EINVAL, "config is NULL");
  if ((c->lattice < ELBM_D1Q3 || c->lattice > ELBM_D3Q27) && c->lattice != ELBM_D3Q19)
    return fail(ELBM_EINVAL, "unknown lattice %d", c->lattice);
  const int D = c->lattice == ELBM_D3Q19 ? 3 : c->lattice;
  if (c->nx < 1 || c->ny < 1 || c->nz < 1)
    return fail(ELBM_EINVAL, "box %d x %d x %d: every extent must be >= 1", c->nx, c->ny, c->nz);
  if (c->nx > kMaxDim || c->ny > kMaxDim || c->nz > kMaxDim)
    return fail(ELBM_EINVAL, "box extent above %lld", (long long)kMaxDim);
  if (D == 1 && (c->ny != 1 || c->nz != 1)) return fail(ELBM_EINVAL, "D1Q3 needs ny = nz = 1");
  if (D == 2 && c->nz != 1) return fail(ELBM_EINVAL, "D2Q9 needs nz = 1");
  const int64_t N = int64_t(c->nx) * c->ny * c->nz;
  if (N > kMaxSites) return fail(ELBM_EINVAL, "%lld sites exceed %lld", (long long)N, (long long)kMaxSites);
  if (!(c->beta > 0.0 && c->beta < 1.0))
    return fail(ELBM_EINVAL, "beta = %g outside (0, 1) (Eq. (2))", c->beta);
  if (c->alpha_mode < ELBM_ALPHA_CLOSED || c->alpha_mode > ELBM_ALPHA_SECANT)
    return fail(ELBM_EINVAL, "unknown alpha mode %d", c->alpha_mode);
  const int es = elem_size(c->storage);
  if (!es) return fail(ELBM_EINVAL, "unknown storage %d", c->storage);
  if (c->alpha_fp64 != ELBM_ARITH_FP32 && c->alpha_fp64 != ELBM_ARITH_FP64 &&
      c->alpha_fp64 != ELBM_ARITH_MIXED)
    return fail(ELBM_EINVAL, "alpha_fp64 must be ELBM_ARITH_FP32, _FP64 or _MIXED");
  if (c->alpha_fp64 != ELBM_ARITH_FP64 && c->storage == ELBM_STORE_F64)
    return fail(ELBM_EUNSUPPORTED, "FP64 storage needs FP64 arithmetic");
  if (c->alpha_fp64 != ELBM_ARITH_FP64 && c->alpha_mode != ELBM_ALPHA_CLOSED)
    return fail(ELBM_EUNSUPPORTED, "FP32 and mixed arithmetic are built for the closed-form alpha only");
  if ((c->storage == ELBM_STORE_F32_DEV || c->storage == ELBM_STORE_F16_DEV) &&
      !(c->rho_ref > 0.0 && std::isfinite(c->rho_ref)))
    return fail(ELBM_EINVAL, "rho_ref must be > 0 for deviation storage");
  if (c->alpha_mode == ELBM_ALPHA_SECANT && c->secant_iters < 1)
    return fail(ELBM_EINVAL, "secant_iters must be >= 1");
  if ((c->alpha_mode == ELBM_ALPHA_NEWTON || c->alpha_mode == ELBM_ALPHA_BISECT) &&
      c->root_max_iter < 1)
    return fail(ELBM_EINVAL, "root_max_iter must be >= 1");
  if (c->alpha_mode == ELBM_ALPHA_BISECT && !(c->root_tol >= 0.0))
    return fail(ELBM_EINVAL, "root_tol must be >= 0");
  if (c->diag & ~7u) return fail(ELBM_EINVAL, "unknown diagnostics bits 0x%x", c->diag);
  if ((c->diag & ELBM_DIAG_SUMS) && !(c->diag & ELBM_DIAG_COUNTS))
    return fail(ELBM_EINVAL, "ELBM_DIAG_SUMS needs ELBM_DIAG_COUNTS");
  if (c->reserved != 0) return fail(ELBM_EINVAL, "reserved must be 0");
  if (c->entropy != ELBM_ENTROPY_BOLTZMANN && c->entropy != ELBM_ENTROPY_BURG)
    return fail(ELBM_EINVAL, "unknown entropy %d", c->entropy);
  if (c->entropy == ELBM_ENTROPY_BURG && c->alpha_mode == ELBM_ALPHA_BGK)
    return fail(ELBM_EUNSUPPORTED, "LBGK uses no entropy function: use ELBM_ENTROPY_BOLTZMANN");
  if (!step_launcher(c->lattice, c->storage, c->alpha_mode, c->alpha_fp64, c->entropy))
    return fail(ELBM_EUNSUPPORTED, "no kernel for this lattice/storage/mode/precision/entropy");

  L->lattice = c->lattice;
  L->D = D;
  L->Q = c->lattice == ELBM_D3Q19 ? 19 : D == 1 ? 3 : D == 2 ? 9 : 27;
  L->esize = es;
  L->N = N;
  // One workgroup per tiles_per_block() tiles of kBlock sites, rounded up to a
  // multiple of 8 (the kernel's XCD-aware tile order needs it).  The count
  // depends only on the box, so per-workgroup diagnostics sum in the same
  // order wherever and however the simulation is stepped.
  const int64_t tpb = tiles_per_block(es, L->Q);
  const int64_t ntiles = (N + kBlock - 1) / kBlock;
  const int64_t units = (ntiles + tpb - 1) / tpb;
  L->nblocks = int((units + 7) / 8 * 8);
  // Each buffer holds the padded site range (whole tiles of every
  // workgroup) in the blocked layout of pidx(): padded * Q elements.  Every
  // address is formed in 64 bits or relative to a row of at most
  // 2^20 Q elements, so no further size limit applies.
  const int64_t padded = L->nblocks * tpb * kBlock;
  L->padded = padded;
  size_t off = 0;
  const size_t bufbytes = align_up(size_t(L->Q) * size_t(padded) * es, kAlign);
  L->off_buf[0] = off;
  off += bufbytes;
  L->off_buf[1] = off;
  off += bufbytes;
  L->off_alpha = off;
  if (c->diag & ELBM_DIAG_ALPHA) off += align_up(size_t(padded) * 8, kAlign);
  L->off_counts = off;
  if (c->diag & ELBM_DIAG_COUNTS) off += align_up(size_t(L->nblocks) * kCountBytes, kAlign);
  L->off_sums = off;
  if (c->diag & ELBM_DIAG_SUMS) off += align_up(size_t(L->nblocks) * kSumBytes, kAlign);
  L->off_misc = off;
  off += align_up(sizeof(Reduced) + 64, kAlign);
  L->total = off;
  return ELBM_OK;
}

// Makes the handle's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) {
      ok = false;
      return;
    }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

struct elbm_sim {
  elbm_config cfg;
  Layout L;
  char* base;
  void* buf[2];
  int cur;  // buffer holding the state that the next step reads
  double* alpha;
  void* counts;
  void* sums;
  Reduced* reduced;
  unsigned long long* counter;
  hipStream_t stream;
  int device;
  int64_t t;
  bool have_alpha, have_stats;
  StepLauncher launch;
};

namespace {

BoxDesc box_of(const elbm_sim* s) {
  BoxDesc b;
  b.lattice = s->L.lattice;
  b.D = s->L.D;
  b.entropy = s->cfg.entropy;
  b.storage = s->cfg.storage;
  b.nx = s->cfg.nx;
  b.ny = s->cfg.ny;
  b.nz = s->cfg.nz;
  b.N = s->L.N;
  b.padded = s->L.padded;
  b.rho_ref = s->cfg.rho_ref;
  return b;
}

SimDesc desc_of(const elbm_sim* s, int block_begin) {
  SimDesc d;
  std::memset(&d, 0, sizeof d);
  d.src = s->buf[s->cur];
  d.dst = s->buf[1 - s->cur];
  d.alpha = (s->cfg.diag & ELBM_DIAG_ALPHA) ? s->alpha : nullptr;
  d.counts = (s->cfg.diag & ELBM_DIAG_COUNTS) ? s->counts : nullptr;
  d.sums = (s->cfg.diag & ELBM_DIAG_SUMS) ? s->sums : nullptr;
  d.padded = s->L.padded;
  d.beta = s->cfg.beta;
  d.rho_ref = s->cfg.rho_ref;
  d.root_tol = s->cfg.root_tol;
  d.inv_nx = 1.0 / double(s->cfg.nx);
  d.inv_ny = 1.0 / double(s->cfg.ny);
  d.nx = s->cfg.nx;
  d.ny = s->cfg.ny;
  d.nz = s->cfg.nz;
  d.rows = s->cfg.ny * s->cfg.nz;
  d.nblocks = s->L.nblocks;
  d.block_begin = block_begin;
  d.root_max_iter = s->cfg.root_max_iter;
  d.secant_iters = s->cfg.secant_iters;
  d.diag = int(s->cfg.diag);
  return d;
}

void after_step(elbm_sim* s) {
  s->cur = 1 - s->cur;
  s->t += 1;
  if (s->cfg.diag & ELBM_DIAG_ALPHA) s->have_alpha = true;
  if (s->cfg.diag & ELBM_DIAG_COUNTS) s->have_stats = true;
}

elbm_status check_sim(const elbm_sim* s) {
  if (!s) return fail(ELBM_EINVAL, "simulation handle is NULL");
  return ELBM_OK;
}

}  // namespace

extern "C" {

elbm_status elbm_config_default(elbm_config* c, int32_t lattice, int32_t nx, int32_t ny,
                                int32_t nz) {
  if (!c) return fail(ELBM_EINVAL, "config is NULL");
  std::memset(c, 0, sizeof *c);
  c->lattice = lattice;
  c->nx = nx;
  c->ny = ny;
  c->nz = nz;
  c->beta = 0.95;
  c->alpha_mode = ELBM_ALPHA_CLOSED;
  c->storage = ELBM_STORE_F32;
  c->alpha_fp64 = 1;
  c->secant_iters = 3;
  c->rho_ref = 1.0;
  c->root_tol = 1e-13;
  c->root_max_iter = 200;
  c->diag = 0;
  return ELBM_OK;
}

size_t elbm_state_bytes(const elbm_config* cfg) {
  Layout L;
  if (check_config(cfg, &L) != ELBM_OK) return 0;
  return L.total;
}

}  // extern "C"

namespace elbm {

// elbm_init without the device-side validation of rho0/u0 (and so without
// its synchronisation): for callers that validated the fields on the host.
elbm_status init_sim(const elbm_config* cfg, const double* rho0, const double* u0,
                     void* dev_state, size_t bytes, void* hip_stream, elbm_sim** out,
                     bool validate);

// A simulation over dev_state that continues from a checkpoint held in
// host memory (pinned, ckpt_bytes == elbm_checkpoint_bytes) at time t: the
// copy is enqueued on hip_stream, so the host buffer must stay valid until
// the stream has passed it.  Used by the server to resume a preempted request.
elbm_status resume_sim(const elbm_config* cfg, void* dev_state, size_t bytes, void* hip_stream,
                       const void* host_ckpt, size_t ckpt_bytes, int64_t t, elbm_sim** out);

// The current populations (a checkpoint) copied to host memory on the
// simulation's stream, behind the work already enqueued; *t receives t.
elbm_status checkpoint_to_host(elbm_sim* sim, void* host_dst, size_t bytes, int64_t* t);

// Free a handle whose stream work the caller knows to be complete (no sync).
void release_sim(elbm_sim* sim) { delete sim; }

// Set the calling thread's error message.
elbm_status set_error(elbm_status st, const char* msg) { return fail(st, "%s", msg); }

}  // namespace elbm

extern "C" elbm_status elbm_init(const elbm_config* cfg, const double* rho0, const double* u0,
                                 void* dev_state, size_t bytes, void* hip_stream,
                                 elbm_sim** out) {
  return elbm::init_sim(cfg, rho0, u0, dev_state, bytes, hip_stream, out, true);
}

namespace {
// A handle over dev_state for a checked configuration (no device work).
elbm_sim* new_handle(const elbm_config* cfg, const Layout& L, void* dev_state, void* hip_stream,
                     int dev) {
  elbm_sim* s = new (std::nothrow) elbm_sim;
  if (!s) return nullptr;
  s->cfg = *cfg;
  s->L = L;
  s->base = static_cast<char*>(dev_state);
  s->buf[0] = s->base + L.off_buf[0];
  s->buf[1] = s->base + L.off_buf[1];
  s->cur = 0;
  s->alpha = reinterpret_cast<double*>(s->base + L.off_alpha);
  s->counts = s->base + L.off_counts;
  s->sums = s->base + L.off_sums;
  s->reduced = reinterpret_cast<Reduced*>(s->base + L.off_misc);
  s->counter = reinterpret_cast<unsigned long long*>(s->base + L.off_misc + sizeof(Reduced));
  s->stream = static_cast<hipStream_t>(hip_stream);
  s->device = dev;
  s->t = 0;
  s->have_alpha = s->have_stats = false;
  s->launch = step_launcher(cfg->lattice, cfg->storage, cfg->alpha_mode, cfg->alpha_fp64,
                            cfg->entropy);
  return s;
}
}  // namespace

elbm_status elbm::init_sim(const elbm_config* cfg, const double* rho0, const double* u0,
                           void* dev_state, size_t bytes, void* hip_stream, elbm_sim** out,
                           bool validate) {
  if (!out) return fail(ELBM_EINVAL, "out is NULL");
  *out = nullptr;
  Layout L;
  elbm_status st = check_config(cfg, &L);
  if (st != ELBM_OK) return st;
  if (!dev_state) return fail(ELBM_EINVAL, "dev_state is NULL");
  if (reinterpret_cast<uintptr_t>(dev_state) % kAlign)
    return fail(ELBM_EINVAL, "dev_state must be %zu-byte aligned", kAlign);
  if (bytes < L.total)
    return fail(ELBM_ENOMEM, "state buffer of %zu bytes, %zu needed", bytes, L.total);
  if (!rho0 || !u0) return fail(ELBM_EINVAL, "rho0 / u0 is NULL");

  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  {
    // set-up of the no-allocation step's scratch on this device (a failed
    // lookup is reported by elbm_step_noalloc, which is its only user)
    void* p;
    (void)scratch_on(dev, &p);
  }
  elbm_sim* s = new_handle(cfg, L, dev_state, hip_stream, dev);
  if (!s) return fail(ELBM_EINVAL, "out of host memory");

  const BoxDesc b = box_of(s);
  unsigned long long nbad = 0;
  if (validate &&
      ((e = hipMemsetAsync(s->counter, 0, sizeof(unsigned long long), s->stream)) != hipSuccess ||
      (e = launch_validate_init(b, rho0, u0, s->counter, s->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(&nbad, s->counter, sizeof nbad, hipMemcpyDeviceToHost, s->stream)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(s->stream)) != hipSuccess)) {
    delete s;
    return hip_fail(e, "elbm_init validation");
  }
  if (nbad) {
    delete s;
    return fail(ELBM_EINVAL,
                "%llu sites with rho0 <= 0 or u0 outside the hull of the velocities "
                "(|u0_a| >= 1, or on D3Q19 |u0_x| + |u0_y| + |u0_z| >= 2): outside the "
                "entropic equilibrium's domain",
                nbad);
  }
  // Zero both buffers' padding once so that every byte of the state is
  // defined, then place f^eq(rho0, u0) in pull convention.
  if ((e = hipMemsetAsync(s->base, 0, L.off_alpha, s->stream)) != hipSuccess ||
      (e = launch_scatter(b, s->buf[0], rho0, u0, nullptr, 0, s->stream)) != hipSuccess) {
    delete s;
    return hip_fail(e, "elbm_init");
  }
  *out = s;
  return ELBM_OK;
}

elbm_status elbm::resume_sim(const elbm_config* cfg, void* dev_state, size_t bytes,
                             void* hip_stream, const void* host_ckpt, size_t ckpt_bytes,
                             int64_t t, elbm_sim** out) {
  if (!out) return fail(ELBM_EINVAL, "out is NULL");
  *out = nullptr;
  Layout L;
  elbm_status st = check_config(cfg, &L);
  if (st != ELBM_OK) return st;
  if (!dev_state || reinterpret_cast<uintptr_t>(dev_state) % kAlign)
    return fail(ELBM_EINVAL, "dev_state is NULL or not %zu-byte aligned", kAlign);
  if (bytes < L.total)
    return fail(ELBM_ENOMEM, "state buffer of %zu bytes, %zu needed", bytes, L.total);
  if (!host_ckpt || t < 0) return fail(ELBM_EINVAL, "checkpoint is NULL or t < 0");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  elbm_sim* s = new_handle(cfg, L, dev_state, hip_stream, dev);
  if (!s) return fail(ELBM_EINVAL, "out of host memory");
  const size_t n = elbm_checkpoint_bytes(s);
  if (ckpt_bytes != n) {
    delete s;
    return fail(ELBM_EINVAL, "checkpoint of %zu bytes, this simulation's is %zu", ckpt_bytes, n);
  }
  // every byte of the state defined, as after elbm_init; then the populations
  if ((e = hipMemsetAsync(s->base, 0, L.off_alpha, s->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(s->buf[0], host_ckpt, n, hipMemcpyHostToDevice, s->stream)) !=
          hipSuccess) {
    delete s;
    return hip_fail(e, "resume");
  }
  s->t = t;
  *out = s;
  return ELBM_OK;
}

elbm_status elbm::checkpoint_to_host(elbm_sim* s, void* host_dst, size_t bytes, int64_t* t) {
  elbm_status st = check_sim(s);
  if (st != ELBM_OK) return st;
  const size_t n = elbm_checkpoint_bytes(s);
  if (!host_dst || !t) return fail(ELBM_EINVAL, "dst / t is NULL");
  if (bytes < n) return fail(ELBM_ENOMEM, "checkpoint buffer of %zu bytes, %zu needed", bytes, n);
  DeviceGuard g(s->device);
  if (!g.ok) return fail(ELBM_EDEVICE, "cannot select the simulation's device");
  const hipError_t e =
      hipMemcpyAsync(host_dst, s->buf[s->cur], n, hipMemcpyDeviceToHost, s->stream);
  if (e != hipSuccess) return hip_fail(e, "checkpoint to host");
  *t = s->t;
  return ELBM_OK;
}

extern "C" {

elbm_status elbm_set_populations(elbm_sim* s, const double* f) {
  elbm_status st = check_sim(s);
  if (st != ELBM_OK) return st;
  if (!f) return fail(ELBM_EINVAL, "f is NULL");
  DeviceGuard g(s->device);
  if (!g.ok) return fail(ELBM_EDEVICE, "cannot select the simulation's device");
  hipError_t e = launch_scatter(box_of(s), s->buf[s->cur], nullptr, nullptr, f, 1, s->stream);
  if (e != hipSuccess) return hip_fail(e, "elbm_set_populations");
  s->have_alpha = s->have_stats = false;
  return ELBM_OK;
}

elbm_status elbm_step(elbm_sim* s, int64_t nsteps) {
  elbm_status st = check_sim(s);
  if (st != ELBM_OK) return st;
  if (nsteps < 0) return fail(ELBM_EINVAL, "nsteps < 0");
  DeviceGuard g(s->device);
  if (!g.ok) return fail(ELBM_EDEVICE, "cannot select the simulation's device");
  BatchArgs a;
  a.n = 1;
  for (int64_t k = 0; k < nsteps; ++k) {
    a.d[0] = desc_of(s, 0);
    hipError_t e = s->launch(a, s->L.nblocks, s->stream);
    if (e != hipSuccess) return hip_fail(e, "step kernel launch");
    after_step(s);
  }
  return ELBM_OK;
}

elbm_status elbm_step_batch(elbm_sim* const* sims, const int64_t* nsteps, int32_t n) {
  if (n < 0 || (n > 0 && (!sims || !nsteps))) return fail(ELBM_EINVAL, "bad batch arguments");
  if (n == 0) return ELBM_OK;
  const elbm_sim* s0 = sims[0];
  int64_t kmax = 0;
  for (int32_t k = 0; k < n; ++k) {
    const elbm_sim* s = sims[k];
    if (!s) return fail(ELBM_EINVAL, "batch entry %d is NULL", k);
    if (nsteps[k] < 0) return fail(ELBM_EINVAL, "batch entry %d: nsteps < 0", k);
    if (s->L.lattice != s0->L.lattice || s->cfg.storage != s0->cfg.storage ||
        s->cfg.alpha_mode != s0->cfg.alpha_mode || s->cfg.alpha_fp64 != s0->cfg.alpha_fp64 ||
        s->cfg.entropy != s0->cfg.entropy)
      return fail(ELBM_EINVAL, "batch entry %d: lattice/storage/mode/precision/entropy differ", k);
    if (s->stream != s0->stream || s->device != s0->device)
      return fail(ELBM_EINVAL, "batch entry %d: different stream or device", k);
    for (int32_t m = 0; m < k; ++m)
      if (sims[m] == s) return fail(ELBM_EINVAL, "batch entry %d repeats entry %d", k, m);
    if (nsteps[k] > kmax) kmax = nsteps[k];
  }
  DeviceGuard g(s0->device);
  if (!g.ok) return fail(ELBM_EDEVICE, "cannot select the simulations' device");
  std::vector<elbm_sim*> active;
  active.reserve(size_t(n));
  for (int64_t step = 0; step < kmax; ++step) {
    active.clear();
    for (int32_t k = 0; k < n; ++k)
      if (nsteps[k] > step) active.push_back(sims[k]);
    for (size_t c0 = 0; c0 < active.size(); c0 += kMaxBatch) {
      BatchArgs a;
      a.n = 0;
      int blocks = 0;
      const size_t c1 = std::min(active.size(), c0 + size_t(kMaxBatch));
      for (size_t k = c0; k < c1; ++k) {
        a.d[a.n++] = desc_of(active[k], blocks);
        blocks += active[k]->L.nblocks;
      }
      hipError_t e = s0->launch(a, blocks, s0->stream);
      if (e != hipSuccess) return hip_fail(e, "batched step kernel launch");
      for (size_t k = c0; k < c1; ++k) after_step(active[k]);
    }
  }
  return ELBM_OK;
}

elbm_status elbm_step_noalloc(elbm_sim* s, int64_t nsteps, uint32_t diag,
                              elbm_stats_t* dev_stats) {
  elbm_status st = check_sim(s);
  if (st != ELBM_OK) return st;
  if (nsteps < 1) return fail(ELBM_EINVAL, "nsteps < 1");
  if (!dev_stats) return fail(ELBM_EINVAL, "dev_stats is NULL");
  if (!(diag & ELBM_DIAG_COUNTS) || (diag & ~(uint32_t)(ELBM_DIAG_COUNTS | ELBM_DIAG_SUMS)))
    return fail(ELBM_EINVAL, "diag must be ELBM_DIAG_COUNTS, optionally with ELBM_DIAG_SUMS");
  if (s->L.nblocks > kScratchBlocks)
    return fail(ELBM_EINVAL,
                "%lld sites need %d workgroup records; the static scratch holds %d "
                "(at most %lld sites)",
                (long long)s->L.N, s->L.nblocks, kScratchBlocks,
                (long long)kScratchBlocks * kBlock * tiles_per_block(s->L.esize, s->L.Q));
  DeviceGuard g(s->device);
  if (!g.ok) return fail(ELBM_EDEVICE, "cannot select the simulation's device");
  void* p = nullptr;
  hipError_t e = scratch_on(s->device, &p);
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  char* counts = static_cast<char*>(p);
  char* sums = (diag & ELBM_DIAG_SUMS) ? counts + kScratchCountBytes : nullptr;
  BatchArgs a;
  a.n = 1;
  for (int64_t k = 0; k < nsteps; ++k) {
    a.d[0] = desc_of(s, 0);
    a.d[0].counts = counts;
    a.d[0].sums = sums;
    a.d[0].diag = int((s->cfg.diag & ELBM_DIAG_ALPHA) | diag);
    if ((e = s->launch(a, s->L.nblocks, s->stream)) != hipSuccess)
      return hip_fail(e, "step kernel launch");
    after_step(s);
  }
  // the handle's own records were not written by these steps
  s->have_stats = false;
  if ((e = launch_reduce(counts, sums, s->L.nblocks,
                         reinterpret_cast<Reduced*>(reinterpret_cast<char*>(dev_stats) + 8),
                         s->stream)) != hipSuccess)
    return hip_fail(e, "diagnostics reduction");
  k_stats_header<<<1, 1, 0, s->stream>>>(dev_stats, s->t, s->L.N);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "diagnostics header");
  return ELBM_OK;
}

elbm_status elbm_moments(elbm_sim* s, double* rho, double* u) {
  elbm_status st = check_sim(s);
  if (st != ELBM_OK) return st;
  if (!rho || !u) return fail(ELBM_EINVAL, "rho / u is NULL");
  DeviceGuard g(s->device);
  if (!g.ok) return fail(ELBM_EDEVICE, "cannot select the simulation's device");
  hipError_t e = launch_moments(box_of(s), s->buf[s->cur], rho, u, s->stream);
  return e == hipSuccess ? ELBM_OK : hip_fail(e, "elbm_moments");
}

elbm_status elbm_populations(elbm_sim* s, double* f) {
  elbm_status st = check_sim(s);
  if (st != ELBM_OK) return st;
  if (!f) return fail(ELBM_EINVAL, "f is NULL");
  DeviceGuard g(s->device);
  if (!g.ok) return fail(ELBM_EDEVICE, "cannot select the simulation's device");
  hipError_t e = launch_gather(box_of(s), s->buf[s->cur], nullptr, s->L.N, 0, f, s->stream);
  return e == hipSuccess ? ELBM_OK : hip_fail(e, "elbm_populations");
}

elbm_status elbm_gather(elbm_sim* s, const int64_t* sites, int64_t n, int32_t which,
                        double* out) {
  elbm_status st = check_sim(s);
  if (st != ELBM_OK) return st;
  if (n < 0 || (n > 0 && (!sites || !out))) return fail(ELBM_EINVAL, "bad gather arguments");
  if (which != 0 && which != 1) return fail(ELBM_EINVAL, "which must be 0 or 1");
  if (which == 1 && s->t == 0) return fail(ELBM_ESTATE, "no step has been taken yet");
  DeviceGuard g(s->device);
  if (!g.ok) return fail(ELBM_EDEVICE, "cannot select the simulation's device");
  hipError_t e = launch_gather(box_of(s), s->buf[s->cur], sites, n, which, out, s->stream);
  return e == hipSuccess ? ELBM_OK : hip_fail(e, "elbm_gather");
}

elbm_status elbm_alpha_field(elbm_sim* s, double* alpha) {
  elbm_status st = check_sim(s);
  if (st != ELBM_OK) return st;
  if (!alpha) return fail(ELBM_EINVAL, "alpha is NULL");
  if (!(s->cfg.diag & ELBM_DIAG_ALPHA)) return fail(ELBM_ESTATE, "ELBM_DIAG_ALPHA is off");
  if (!s->have_alpha) return fail(ELBM_ESTATE, "no step has recorded alpha yet");
  DeviceGuard g(s->device);
  if (!g.ok) return fail(ELBM_EDEVICE, "cannot select the simulation's device");
  hipError_t e = launch_copy_f64(s->alpha, alpha, s->L.N, s->stream);
  return e == hipSuccess ? ELBM_OK : hip_fail(e, "elbm_alpha_field");
}

elbm_status elbm_stats(elbm_sim* s, elbm_stats_t* out) {
  elbm_status st = check_sim(s);
  if (st != ELBM_OK) return st;
  if (!out) return fail(ELBM_EINVAL, "stats is NULL");
  if (!(s->cfg.diag & ELBM_DIAG_COUNTS)) return fail(ELBM_ESTATE, "ELBM_DIAG_COUNTS is off");
  if (!s->have_stats) return fail(ELBM_ESTATE, "no step has recorded diagnostics yet");
  DeviceGuard g(s->device);
  if (!g.ok) return fail(ELBM_EDEVICE, "cannot select the simulation's device");
  Reduced r;
  hipError_t e;
  const void* sums = (s->cfg.diag & ELBM_DIAG_SUMS) ? s->sums : nullptr;
  if ((e = launch_reduce(s->counts, sums, s->L.nblocks, s->reduced, s->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(&r, s->reduced, sizeof r, hipMemcpyDeviceToHost, s->stream)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(s->stream)) != hipSuccess)
    return hip_fail(e, "elbm_stats");
  out->step = s->t;
  out->n_sites = s->L.N;
  out->n_accept2 = r.cnt[0];
  out->n_alphastar_lt2 = r.cnt[1];
  out->n_alpha_lt2 = r.cnt[2];
  out->n_guard = r.cnt[3];
  out->n_fallback = r.cnt[4];
  out->n_negative = r.cnt[5];
  out->n_nonfinite = r.cnt[6];
  out->total_iters = r.cnt[7];
  out->alpha_min = r.amin;
  out->alpha_max = r.amax;
  out->sum_rho = r.rho;
  out->sum_j[0] = r.j[0];
  out->sum_j[1] = r.j[1];
  out->sum_j[2] = r.j[2];
  out->sum_H = r.H;
  return ELBM_OK;
}

int64_t elbm_time(const elbm_sim* s) { return s ? s->t : -1; }

elbm_status elbm_destroy(elbm_sim* s) {
  if (!s) return ELBM_OK;
  elbm_status st = ELBM_OK;
  {
    DeviceGuard g(s->device);
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) st = hip_fail(e, "elbm_destroy");
  }
  delete s;
  return st;
}

size_t elbm_checkpoint_bytes(const elbm_sim* s) {
  if (!s) {
    fail(ELBM_EINVAL, "simulation handle is NULL");
    return 0;
  }
  return size_t(s->L.Q) * size_t(s->L.padded) * size_t(s->L.esize);
}

elbm_status elbm_export(elbm_sim* s, void* dst, size_t bytes, int64_t* t) {
  elbm_status st = check_sim(s);
  if (st != ELBM_OK) return st;
  const size_t n = elbm_checkpoint_bytes(s);
  if (!dst || !t) return fail(ELBM_EINVAL, "dst / t is NULL");
  if (bytes < n) return fail(ELBM_ENOMEM, "checkpoint buffer of %zu bytes, %zu needed", bytes, n);
  DeviceGuard g(s->device);
  if (!g.ok) return fail(ELBM_EDEVICE, "cannot select the simulation's device");
  const hipError_t e = hipMemcpyAsync(dst, s->buf[s->cur], n, hipMemcpyDeviceToDevice, s->stream);
  if (e != hipSuccess) return hip_fail(e, "elbm_export");
  *t = s->t;
  return ELBM_OK;
}

elbm_status elbm_import(elbm_sim* s, const void* src, size_t bytes, int64_t t) {
  elbm_status st = check_sim(s);
  if (st != ELBM_OK) return st;
  const size_t n = elbm_checkpoint_bytes(s);
  if (!src) return fail(ELBM_EINVAL, "src is NULL");
  if (bytes != n)
    return fail(ELBM_EINVAL, "checkpoint of %zu bytes, this simulation's is %zu", bytes, n);
  if (t < 0) return fail(ELBM_EINVAL, "t < 0");
  DeviceGuard g(s->device);
  if (!g.ok) return fail(ELBM_EDEVICE, "cannot select the simulation's device");
  const hipError_t e = hipMemcpyAsync(s->buf[s->cur], src, n, hipMemcpyDeviceToDevice, s->stream);
  if (e != hipSuccess) return hip_fail(e, "elbm_import");
  s->t = t;
  s->have_alpha = s->have_stats = false;
  return ELBM_OK;
}

const char* elbm_last_error(void) { return g_err.c_str(); }

}  // extern "C"
