// elbm_serve.cpp -- continuous-batching server of the ELBM library
// (elbm_server_* in include/elbm.h).
//
// One scheduler thread per server.  Each iteration it
//   1. retires rounds whose event has completed (blocking on the oldest when
//      two are in flight): finished requests get their completion time, and
//      the pool blocks of finished, not kept, simulations and of consumed
//      staging copies return to the free list;
//   2. with preemption enabled (preempt_rounds > 0), moves long-resident
//      requests out to pinned host memory when that makes room for the
//      request at the head of the queue (preempt());
//   3. admits queued requests first come, first served while a slot is free
//      and the pool has room for state + staging copy of the initial fields:
//      pinned host copy -> staging block -> f^eq(rho0, u0) in the state; a
//      preempted request needs only its state block and continues from its
//      checkpoint;
//   4. launches one round: up to round_steps steps of every resident
//      simulation, one batched launch per step for each group of residents
//      that share a kernel (lattice, storage, alpha mode, arithmetic), then
//      the final moments of the requests that finish, then an event.
// With two rounds in flight the host work of 1-3 overlaps the GPU.  All
// device work runs on one stream, in order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/elbm.h"
#include "elbm_internal.hpp"

namespace elbm {
elbm_status init_sim(const elbm_config* cfg, const double* rho0, const double* u0,
                     void* dev_state, size_t bytes, void* hip_stream, elbm_sim** out,
                     bool validate);
void release_sim(elbm_sim* sim);
elbm_status set_error(elbm_status st, const char* msg);
elbm_status resume_sim(const elbm_config* cfg, void* dev_state, size_t bytes, void* hip_stream,
                       const void* host_ckpt, size_t ckpt_bytes, int64_t t, elbm_sim** out);
elbm_status checkpoint_to_host(elbm_sim* sim, void* host_dst, size_t bytes, int64_t* t);
}  // namespace elbm

using elbm::set_error;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kPinnedCacheBytes = size_t(1) << 30;  // pinned copies kept for reuse

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Dimension of a lattice code (ELBM_D1Q3 = 1, ELBM_D2Q9 = 2, ELBM_D3Q27 = 3,
// ELBM_D3Q19 = 19); the config check rejects other codes.
int lattice_dim(int32_t lattice) { return lattice == ELBM_D3Q19 ? 3 : lattice; }

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit sub-allocator over [0, size) in kAlign units, coalescing frees.
class Pool {
 public:
  explicit Pool(size_t size) {
    if (size) free_[0] = size;
  }
  bool alloc(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n, start = it->first + n;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    return false;
  }
  void release(size_t off, size_t n) {
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;  // offset -> length
};

struct Pinned {
  double* p = nullptr;
  size_t bytes = 0;
};

struct Req {
  int64_t id = 0;
  elbm_config cfg{};
  int64_t N = 0, nsteps = 0, done = 0;
  double* out_rho = nullptr;
  double* out_u = nullptr;
  bool keep = false;
  int state = ELBM_REQ_QUEUED;
  double t_submit = 0, t_admit = 0, t_done = 0;
  size_t state_bytes = 0, stage_bytes = 0;
  size_t off = 0;  // state block in the pool
  Pinned host;     // rho0 then u0, until staged
  elbm_sim* sim = nullptr;
  bool admitted = false;     // admitted at least once
  int64_t rounds = 0;        // rounds launched since the last admission
  int32_t preemptions = 0;
  Pinned ckpt;               // populations while preempted, until resumed
  size_t ckpt_bytes = 0;
  int64_t ckpt_t = 0;
  bool cancel = false;       // elbm_server_cancel, applied between rounds
};

// Work enqueued on the stream, and what to do once the GPU has passed it.
struct Round {
  hipEvent_t ev = nullptr;
  std::vector<Req*> finished;
  std::vector<std::pair<size_t, size_t>> staging;  // pool blocks to free
  std::vector<Pinned> pinned;                      // host copies to recycle
  int64_t updates = 0;
};

}  // namespace

struct elbm_server {
  elbm_server_config cfg{};
  hipStream_t stream = nullptr;
  int device = 0;
  char* base = nullptr;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req*> queue;
  std::unordered_map<int64_t, std::unique_ptr<Req>> reqs;
  std::vector<Req*> active;
  std::unique_ptr<Pool> pool;
  std::deque<Round> rounds;  // in flight, oldest first
  Round pending;             // admissions since the last round
  std::vector<hipEvent_t> spare_events;
  std::vector<Pinned> pinned_cache;
  size_t pinned_cached = 0;
  std::thread worker;
  bool stop = false;
  bool broken = false;
  std::string error;
  uint64_t kick = 0;  // bumped by submit, release, cancel and destroy
  bool cancels = false;  // some request carries a cancel flag
  int64_t next_id = 1;
  elbm_server_stats stats{};
  double t0 = 0;
};

namespace {

// Pinned host buffers: reuse before allocating, since freeing pinned memory
// may synchronise the device.
Pinned take_pinned(elbm_server* s, size_t bytes) {
  std::lock_guard<std::mutex> lk(s->mu);
  size_t best = SIZE_MAX;
  for (size_t k = 0; k < s->pinned_cache.size(); ++k)
    if (s->pinned_cache[k].bytes >= bytes &&
        (best == SIZE_MAX || s->pinned_cache[k].bytes < s->pinned_cache[best].bytes))
      best = k;
  if (best == SIZE_MAX) return Pinned{};
  Pinned p = s->pinned_cache[best];
  s->pinned_cache.erase(s->pinned_cache.begin() + best);
  s->pinned_cached -= p.bytes;
  return p;
}

// caller holds the lock
void recycle_pinned(elbm_server* s, Pinned p) {
  if (!p.p) return;
  if (s->pinned_cached + p.bytes <= kPinnedCacheBytes) {
    s->pinned_cache.push_back(p);
    s->pinned_cached += p.bytes;
  } else {
    (void)hipHostFree(p.p);
  }
}

bool group_less(const Req* a, const Req* b) {
  return std::make_tuple(a->cfg.lattice, a->cfg.storage, a->cfg.alpha_mode, a->cfg.alpha_fp64,
                         a->cfg.entropy) <
         std::make_tuple(b->cfg.lattice, b->cfg.storage, b->cfg.alpha_mode, b->cfg.alpha_fp64,
                         b->cfg.entropy);
}

bool same_group(const Req* a, const Req* b) { return !group_less(a, b) && !group_less(b, a); }

void fail_req(elbm_server* s, Req* r) {
  r->state = ELBM_REQ_FAILED;
  r->t_done = now_s() - s->t0;
  s->stats.failed++;
}

void mark_broken(elbm_server* s, const std::string& why) {
  if (!s->broken) s->error = why;
  s->broken = true;
}

hipEvent_t take_event(elbm_server* s) {
  if (!s->spare_events.empty()) {
    hipEvent_t e = s->spare_events.back();
    s->spare_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

// Admission, first come first served.  Pool blocks are taken with the lock
// held; the copies and launches run with it released (a launch can block
// while the device queue is full, and submitters must not wait on that).
void admit(elbm_server* s, std::unique_lock<std::mutex>& lk) {
  struct Adm {
    Req* r;
    size_t soff;
  };
  std::vector<Adm> take;
  size_t slots = s->active.size();
  while (!s->broken && !s->queue.empty() && (int)slots < s->cfg.max_active) {
    Req* r = s->queue.front();
    size_t off = 0, soff = 0;
    if (!s->pool->alloc(r->state_bytes, &off)) break;
    if (!r->ckpt.p && !s->pool->alloc(r->stage_bytes, &soff)) {
      s->pool->release(off, r->state_bytes);
      break;
    }
    s->queue.pop_front();
    r->off = off;
    take.push_back({r, soff});
    ++slots;
  }
  if (take.empty()) return;
  std::vector<elbm_status> st(take.size(), ELBM_EDEVICE);
  bool any_failed = false;
  lk.unlock();
  for (size_t k = 0; k < take.size(); ++k) {
    Req* r = take[k].r;
    if (r->ckpt.p) {
      st[k] = elbm::resume_sim(&r->cfg, s->base + r->off, r->state_bytes, s->stream, r->ckpt.p,
                               r->ckpt_bytes, r->ckpt_t, &r->sim);
    } else {
      double* stage = reinterpret_cast<double*>(s->base + take[k].soff);
      const size_t nbytes = size_t(r->N) * (1 + lattice_dim(r->cfg.lattice)) * sizeof(double);
      if (hipMemcpyAsync(stage, r->host.p, nbytes, hipMemcpyHostToDevice, s->stream) ==
          hipSuccess)
        st[k] = elbm::init_sim(&r->cfg, stage, stage + r->N, s->base + r->off, r->state_bytes,
                               s->stream, &r->sim, false);
    }
    any_failed |= st[k] != ELBM_OK;
  }
  // nothing of a failed admission may still be in use on the stream
  if (any_failed) (void)hipStreamSynchronize(s->stream);
  lk.lock();
  const double t = now_s() - s->t0;
  for (size_t k = 0; k < take.size(); ++k) {
    Req* r = take[k].r;
    const bool resumed = r->ckpt.p != nullptr;
    if (st[k] != ELBM_OK) {
      s->pool->release(r->off, r->state_bytes);
      if (resumed) {
        recycle_pinned(s, r->ckpt);
        r->ckpt = Pinned{};
      } else {
        s->pool->release(take[k].soff, r->stage_bytes);
        recycle_pinned(s, r->host);
        r->host = Pinned{};
      }
      fail_req(s, r);
      continue;
    }
    r->state = ELBM_REQ_RUNNING;
    if (!r->admitted) r->t_admit = t;
    r->admitted = true;
    r->rounds = 0;
    s->active.push_back(r);
    if (resumed) {
      // the host checkpoint is read by the copy just enqueued
      s->pending.pinned.push_back(r->ckpt);
      r->ckpt = Pinned{};
    } else {
      s->pending.staging.push_back({take[k].soff, r->stage_bytes});
      s->pending.pinned.push_back(r->host);
      r->host = Pinned{};
    }
  }
  s->stats.max_resident = std::max<int64_t>(s->stats.max_resident, (int64_t)s->active.size());
}

// Enqueue one round over the resident simulations.  Only this thread touches
// the resident simulations, so the launches run with the lock released.
void launch_round(elbm_server* s, std::unique_lock<std::mutex>& lk) {
  Round rd = std::move(s->pending);
  s->pending = Round{};
  std::vector<Req*> act = s->active;
  std::vector<int64_t> todo(act.size());
  for (size_t k = 0; k < act.size(); ++k)
    todo[k] = std::min<int64_t>(act[k]->nsteps - act[k]->done, s->cfg.round_steps);
  lk.unlock();
  std::vector<size_t> order(act.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t a, size_t b) { return group_less(act[a], act[b]); });
  std::string err;
  int64_t launches = 0;
  std::vector<elbm_sim*> sims;
  std::vector<int64_t> steps;
  for (size_t g0 = 0, g1; g0 < order.size() && err.empty(); g0 = g1) {
    g1 = g0 + 1;
    while (g1 < order.size() && same_group(act[order[g0]], act[order[g1]])) ++g1;
    sims.clear();
    steps.clear();
    for (size_t k = g0; k < g1; ++k) {
      sims.push_back(act[order[k]]->sim);
      steps.push_back(todo[order[k]]);
      rd.updates += todo[order[k]] * act[order[k]]->N;
    }
    if (elbm_step_batch(sims.data(), steps.data(), (int32_t)sims.size()) != ELBM_OK) {
      err = std::string("step launch: ") + elbm_last_error();
      break;
    }
    // one launch per step and per kMaxBatch simulations still stepping
    std::sort(steps.begin(), steps.end());
    int64_t prev = 0;
    for (size_t k = 0; k < steps.size(); ++k) {
      const int64_t left = int64_t(steps.size() - k);
      launches += (steps[k] - prev) * ((left + elbm::kMaxBatch - 1) / elbm::kMaxBatch);
      prev = steps[k];
    }
  }
  std::vector<char> fin(act.size(), 0);
  for (size_t k = 0; k < act.size() && err.empty(); ++k) {
    Req* r = act[k];
    if (r->done + todo[k] < r->nsteps) continue;
    fin[k] = 1;
    if (r->out_rho && elbm_moments(r->sim, r->out_rho, r->out_u) != ELBM_OK)
      err = std::string("moments: ") + elbm_last_error();
  }
  hipEvent_t ev = nullptr;
  if (err.empty()) {
    ev = take_event(s);
    if (!ev || hipEventRecord(ev, s->stream) != hipSuccess) {
      err = "hipEventRecord failed";
      if (ev) s->spare_events.push_back(ev);
      ev = nullptr;
    }
  }
  lk.lock();
  s->stats.launches += launches;
  s->stats.rounds++;
  if (!err.empty()) {
    mark_broken(s, err);
    s->pending = std::move(rd);  // freed once the stream has been drained
    return;
  }
  std::vector<Req*> still;
  for (size_t k = 0; k < act.size(); ++k) {
    act[k]->done += todo[k];
    act[k]->rounds++;
    if (fin[k])
      rd.finished.push_back(act[k]);
    else
      still.push_back(act[k]);
  }
  s->active.swap(still);
  rd.ev = ev;
  s->rounds.push_back(std::move(rd));
}

// Retire the oldest round, waiting for the GPU with the lock released.
void retire_oldest(elbm_server* s, std::unique_lock<std::mutex>& lk) {
  hipEvent_t ev = s->rounds.front().ev;
  lk.unlock();
  hipError_t e = ev ? hipEventSynchronize(ev) : hipStreamSynchronize(s->stream);
  lk.lock();
  if (e != hipSuccess) mark_broken(s, std::string("device error: ") + hipGetErrorString(e));
  Round rd = std::move(s->rounds.front());
  s->rounds.pop_front();
  const double t = now_s() - s->t0;
  const bool ok = e == hipSuccess && !s->broken;
  for (Req* r : rd.finished) {
    if (ok) {
      r->state = ELBM_REQ_DONE;
      r->t_done = t;
      s->stats.completed++;
      s->stats.t_last_done = t;
    } else {
      fail_req(s, r);
    }
    if (!r->keep || !ok) {
      elbm::release_sim(r->sim);
      r->sim = nullptr;
      s->pool->release(r->off, r->state_bytes);
    }
  }
  if (ok) s->stats.site_updates += rd.updates;
  for (auto& b : rd.staging) s->pool->release(b.first, b.second);
  for (auto& p : rd.pinned) recycle_pinned(s, p);
  if (rd.ev) s->spare_events.push_back(rd.ev);
  s->cv.notify_all();
}

// Preemption (preempt_rounds > 0; see elbm_server_config).  A resident is
// preempted only for a queue head with less than half its remaining work
// (steps x sites), so that long arrivals never evict and residents do not
// rotate under overload.  A victim's
// populations are copied to pinned host memory by a copy enqueued behind its
// last step; since every later use of its pool block (another request's
// staging or state) is enqueued after that copy on the same stream, the block
// returns to the free list at once.  Victims are chosen only if freeing their
// blocks (tried on a copy of the free list) lets the head of the queue in.
void preempt(elbm_server* s, std::unique_lock<std::mutex>& lk) {
  if (s->cfg.preempt_rounds <= 0 || s->broken || s->queue.empty()) return;
  const Req* head = s->queue.front();
  const size_t head_stage = head->ckpt.p ? 0 : head->stage_bytes;
  auto fits = [&](Pool pool, size_t resident) {  // on a copy of the free list
    size_t off = 0;
    return resident < size_t(s->cfg.max_active) && pool.alloc(head->state_bytes, &off) &&
           (head_stage == 0 || pool.alloc(head_stage, &off));
  };
  if (fits(*s->pool, s->active.size())) return;
  // only for a head with much less work left than the victim (shortest
  // remaining work first, with a factor 2 against needless swaps)
  const int64_t head_work = (head->nsteps - head->done) * head->N;
  std::vector<Req*> cand;
  for (Req* r : s->active)
    if (r->rounds >= s->cfg.preempt_rounds && r->nsteps - r->done > s->cfg.round_steps &&
        (r->nsteps - r->done) * r->N > 2 * head_work)
      cand.push_back(r);
  std::stable_sort(cand.begin(), cand.end(), [](const Req* a, const Req* b) {
    return (a->nsteps - a->done) * a->N > (b->nsteps - b->done) * b->N;
  });
  Pool trial = *s->pool;
  size_t nv = 0;
  bool room = false;
  while (nv < cand.size() && !room) {
    trial.release(cand[nv]->off, cand[nv]->state_bytes);
    ++nv;
    room = fits(trial, s->active.size() - nv);
  }
  if (!room) return;
  cand.resize(nv);
  std::vector<Req*> still;
  for (Req* r : s->active)
    if (std::find(cand.begin(), cand.end(), r) == cand.end()) still.push_back(r);
  s->active.swap(still);
  // the copies run with the lock released (see admit)
  std::vector<Pinned> buf(nv);
  std::vector<size_t> nb(nv, 0);
  std::vector<int64_t> tk(nv, 0);
  std::vector<elbm_status> st(nv, ELBM_EDEVICE);
  lk.unlock();
  for (size_t k = 0; k < nv; ++k) {
    const size_t n = nb[k] = elbm_checkpoint_bytes(cand[k]->sim);
    buf[k] = take_pinned(s, n);
    if (!buf[k].p) {
      void* q = nullptr;
      if (hipHostMalloc(&q, n, hipHostMallocDefault) == hipSuccess) {
        buf[k].p = static_cast<double*>(q);
        buf[k].bytes = n;
      }
    }
    st[k] = buf[k].p ? elbm::checkpoint_to_host(cand[k]->sim, buf[k].p, n, &tk[k]) : ELBM_ENOMEM;
  }
  lk.lock();
  for (size_t k = 0; k < nv; ++k) {
    Req* r = cand[k];
    if (st[k] == ELBM_ENOMEM) {
      // no host memory for the checkpoint: nothing was enqueued, the victim
      // stays resident and the head waits as without preemption
      recycle_pinned(s, buf[k]);
      s->active.push_back(r);
      continue;
    }
    if (st[k] != ELBM_OK) {
      // the server stops here: the victim is failed with the residents
      mark_broken(s, std::string("preemption: ") + elbm_last_error());
      if (buf[k].p) r->ckpt = buf[k];  // freed by elbm_server_destroy after the stream
      s->active.push_back(r);
      continue;
    }
    s->pool->release(r->off, r->state_bytes);
    elbm::release_sim(r->sim);
    r->sim = nullptr;
    r->ckpt = buf[k];
    r->ckpt_bytes = nb[k];
    r->ckpt_t = tk[k];
    r->state = ELBM_REQ_QUEUED;
    r->rounds = 0;
    r->preemptions++;
    s->stats.preemptions++;
    s->queue.push_back(r);
  }
}

// Cancellations (elbm_server_cancel), applied by the scheduler thread
// between rounds with the lock held, so that no launch is being enqueued for
// the simulations it releases.  A queued request drops its host copies; its
// checkpoint, if it was preempted, may still be the destination of the copy
// that preempted it, so it is recycled only once the stream has passed the
// next round.  A resident request gives back its simulation and pool block
// at once: every later use of the block is enqueued behind its last step on
// the same stream.  A request whose last round is already enqueued is no
// longer resident and completes.
void apply_cancels(elbm_server* s) {
  if (!s->cancels) return;
  s->cancels = false;
  const double t = now_s() - s->t0;
  auto cancelled = [&](Req* r) {
    r->state = ELBM_REQ_CANCELLED;
    r->t_done = t;
    s->stats.cancelled++;
  };
  for (auto it = s->queue.begin(); it != s->queue.end();) {
    Req* r = *it;
    if (!r->cancel) {
      ++it;
      continue;
    }
    recycle_pinned(s, r->host);
    r->host = Pinned{};
    if (r->ckpt.p) s->pending.pinned.push_back(r->ckpt);
    r->ckpt = Pinned{};
    cancelled(r);
    it = s->queue.erase(it);
  }
  std::vector<Req*> still;
  for (Req* r : s->active) {
    if (!r->cancel) {
      still.push_back(r);
      continue;
    }
    elbm::release_sim(r->sim);
    r->sim = nullptr;
    s->pool->release(r->off, r->state_bytes);
    cancelled(r);
  }
  s->active.swap(still);
  s->cv.notify_all();
}

void worker_main(elbm_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  uint64_t seen = s->kick;
  for (;;) {
    while (!s->rounds.empty() &&
           (s->rounds.size() >= 2 || !s->rounds.front().ev ||
            hipEventQuery(s->rounds.front().ev) == hipSuccess))
      retire_oldest(s, lk);
    if (s->broken) {
      // after a device error the stream is not trusted: fail what is left
      while (!s->rounds.empty()) retire_oldest(s, lk);
      if (!s->pending.staging.empty() || !s->pending.pinned.empty()) {
        lk.unlock();
        (void)hipStreamSynchronize(s->stream);
        lk.lock();
        for (auto& b : s->pending.staging) s->pool->release(b.first, b.second);
        for (auto& p : s->pending.pinned) recycle_pinned(s, p);
        s->pending = Round{};
      }
      for (Req* r : s->active) {
        elbm::release_sim(r->sim);
        r->sim = nullptr;
        s->pool->release(r->off, r->state_bytes);
        fail_req(s, r);
      }
      s->active.clear();
      for (Req* r : s->queue) fail_req(s, r);
      s->queue.clear();
      s->cv.notify_all();
      if (s->stop) break;
      s->cv.wait(lk, [&] { return s->stop || s->kick != seen; });
      seen = s->kick;
      continue;
    }
    apply_cancels(s);
    preempt(s, lk);
    if (s->broken) continue;
    admit(s, lk);
    if (s->broken) continue;
    if (!s->active.empty()) {
      launch_round(s, lk);
      continue;
    }
    if (!s->rounds.empty()) {
      retire_oldest(s, lk);
      continue;
    }
    // nothing resident and nothing in flight
    if (!s->pending.staging.empty() || !s->pending.pinned.empty()) {
      s->rounds.push_back(std::move(s->pending));  // no event: retired by a stream sync
      s->pending = Round{};
      continue;
    }
    if (s->stop) {
      // what is still queued cannot be admitted while kept states hold the pool
      for (Req* r : s->queue) fail_req(s, r);
      s->queue.clear();
      s->cv.notify_all();
      break;
    }
    if (s->kick == seen) s->cv.wait(lk, [&] { return s->stop || s->kick != seen; });
    seen = s->kick;
  }
}

Req* find_req(elbm_server* s, int64_t id) {
  auto it = s->reqs.find(id);
  return it == s->reqs.end() ? nullptr : it->second.get();
}

}  // namespace

extern "C" {

elbm_status elbm_server_create(const elbm_server_config* cfg, elbm_server** out) {
  if (!cfg || !out) return set_error(ELBM_EINVAL, "config / out is NULL");
  *out = nullptr;
  if (!cfg->pool || cfg->pool_bytes < kAlign)
    return set_error(ELBM_EINVAL, "server pool is NULL or smaller than 256 bytes");
  if (reinterpret_cast<uintptr_t>(cfg->pool) % kAlign)
    return set_error(ELBM_EINVAL, "server pool must be 256-byte aligned");
  if (cfg->max_active < 1 || cfg->round_steps < 1)
    return set_error(ELBM_EINVAL, "max_active and round_steps must be >= 1");
  if (cfg->preempt_rounds < 0 || cfg->reserved != 0)
    return set_error(ELBM_EINVAL, "preempt_rounds < 0 or reserved != 0");
  auto* s = new (std::nothrow) elbm_server;
  if (!s) return set_error(ELBM_EINVAL, "out of host memory");
  s->cfg = *cfg;
  s->cfg.pool_bytes = cfg->pool_bytes / kAlign * kAlign;
  s->stream = static_cast<hipStream_t>(cfg->hip_stream);
  s->base = static_cast<char*>(cfg->pool);
  s->pool.reset(new Pool(s->cfg.pool_bytes));
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return set_error(ELBM_EDEVICE, "hipGetDevice failed");
  }
  s->t0 = now_s();
  try {
    s->worker = std::thread(worker_main, s);
  } catch (...) {
    delete s;
    return set_error(ELBM_EDEVICE, "cannot start the scheduler thread");
  }
  *out = s;
  return ELBM_OK;
}

elbm_status elbm_server_submit(elbm_server* s, const elbm_request* q, int64_t* id) {
  const double t = now_s();
  if (!s || !q || !id) return set_error(ELBM_EINVAL, "server / request / id is NULL");
  if (q->nsteps < 0 || q->reserved != 0)
    return set_error(ELBM_EINVAL, "nsteps < 0 or reserved != 0");
  if (!q->rho0 || !q->u0) return set_error(ELBM_EINVAL, "rho0 / u0 is NULL");
  if ((q->out_rho == nullptr) != (q->out_u == nullptr))
    return set_error(ELBM_EINVAL, "out_rho and out_u must both be given or both be NULL");
  const size_t sb = elbm_state_bytes(&q->cfg);
  if (!sb) return ELBM_EINVAL;  // elbm_state_bytes has set the message
  const int D = lattice_dim(q->cfg.lattice);
  const int64_t N = int64_t(q->cfg.nx) * q->cfg.ny * q->cfg.nz;
  for (int64_t k = 0; k < N; ++k)
    if (!(q->rho0[k] > 0.0) || !std::isfinite(q->rho0[k]))
      return set_error(ELBM_EINVAL, "rho0 <= 0 or not finite");
  for (int64_t k = 0; k < int64_t(D) * N; ++k)
    if (!(std::fabs(q->u0[k]) < 1.0)) return set_error(ELBM_EINVAL, "|u0| >= 1 or not finite");
  if (q->cfg.lattice == ELBM_D3Q19)
    for (int64_t k = 0; k < N; ++k)
      if (!(std::fabs(q->u0[k]) + std::fabs(q->u0[N + k]) + std::fabs(q->u0[2 * N + k]) < 2.0))
        return set_error(ELBM_EINVAL, "|u0_x| + |u0_y| + |u0_z| >= 2 on D3Q19");
  auto r = std::make_unique<Req>();
  r->cfg = q->cfg;
  r->N = N;
  r->nsteps = q->nsteps;
  r->out_rho = q->out_rho;
  r->out_u = q->out_u;
  r->keep = q->keep_state != 0;
  r->state_bytes = align_up(sb);
  const size_t host_bytes = size_t(N) * (1 + D) * sizeof(double);
  r->stage_bytes = align_up(host_bytes);
  if (r->state_bytes + r->stage_bytes > s->cfg.pool_bytes)
    return set_error(ELBM_ENOMEM, "request footprint (state + staging) exceeds the server pool");
  r->host = take_pinned(s, host_bytes);
  if (!r->host.p) {
    void* p = nullptr;
    if (hipHostMalloc(&p, host_bytes, hipHostMallocDefault) != hipSuccess)
      return set_error(ELBM_EDEVICE, "hipHostMalloc of the staging copy failed");
    r->host.p = static_cast<double*>(p);
    r->host.bytes = host_bytes;
  }
  std::memcpy(r->host.p, q->rho0, size_t(N) * sizeof(double));
  std::memcpy(r->host.p + N, q->u0, size_t(D) * N * sizeof(double));
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop || s->broken) {
    recycle_pinned(s, r->host);
    return set_error(ELBM_ESTATE, s->broken ? "server hit a device error" : "server is stopping");
  }
  r->id = s->next_id++;
  r->t_submit = t - s->t0;
  if (s->stats.submitted == 0) s->stats.t_first_submit = r->t_submit;
  s->stats.submitted++;
  *id = r->id;
  s->queue.push_back(r.get());
  s->reqs.emplace(r->id, std::move(r));
  s->kick++;
  s->cv.notify_all();
  return ELBM_OK;
}

elbm_status elbm_server_poll(elbm_server* s, int64_t id, elbm_request_info* info) {
  if (!s || !info) return set_error(ELBM_EINVAL, "server / info is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  const Req* r = find_req(s, id);
  if (!r) return set_error(ELBM_EINVAL, "unknown request id");
  std::memset(info, 0, sizeof *info);
  info->state = r->state;
  info->preemptions = r->preemptions;
  info->steps_done = r->done;  // steps enqueued so far
  info->t_submit = r->t_submit;
  info->t_admit = r->t_admit;
  info->t_done = r->t_done;
  info->footprint = r->state_bytes + r->stage_bytes;
  return ELBM_OK;
}

elbm_status elbm_server_wait(elbm_server* s, int64_t id, double timeout_s) {
  if (!s) return set_error(ELBM_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  const Req* r = find_req(s, id);
  if (!r) return set_error(ELBM_EINVAL, "unknown request id");
  auto done = [r] {
    return r->state == ELBM_REQ_DONE || r->state == ELBM_REQ_FAILED ||
           r->state == ELBM_REQ_CANCELLED;
  };
  if (timeout_s < 0) {
    s->cv.wait(lk, done);
  } else if (!s->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
    return set_error(ELBM_ESTATE, "timed out waiting for the request");
  }
  if (r->state == ELBM_REQ_DONE) return ELBM_OK;
  if (r->state == ELBM_REQ_CANCELLED) return set_error(ELBM_ESTATE, "request was cancelled");
  return set_error(ELBM_EDEVICE, s->error.empty() ? "request failed" : s->error.c_str());
}

elbm_status elbm_server_cancel(elbm_server* s, int64_t id) {
  if (!s) return set_error(ELBM_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  Req* r = find_req(s, id);
  if (!r) return set_error(ELBM_EINVAL, "unknown request id");
  if (r->state != ELBM_REQ_QUEUED && r->state != ELBM_REQ_RUNNING)
    return set_error(ELBM_ESTATE, "request already finished");
  r->cancel = true;
  s->cancels = true;
  s->kick++;
  s->cv.notify_all();
  return ELBM_OK;
}

elbm_status elbm_server_sim(elbm_server* s, int64_t id, elbm_sim** sim) {
  if (!s || !sim) return set_error(ELBM_EINVAL, "server / sim is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  const Req* r = find_req(s, id);
  if (!r) return set_error(ELBM_EINVAL, "unknown request id");
  if (r->state != ELBM_REQ_DONE || !r->keep || !r->sim)
    return set_error(ELBM_ESTATE, "not a completed keep_state request");
  *sim = r->sim;
  return ELBM_OK;
}

elbm_status elbm_server_release(elbm_server* s, int64_t id) {
  if (!s) return set_error(ELBM_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  Req* r = find_req(s, id);
  if (!r) return set_error(ELBM_EINVAL, "unknown request id");
  if (r->state != ELBM_REQ_DONE || !r->keep || !r->sim)
    return set_error(ELBM_ESTATE, "not a completed keep_state request");
  elbm_sim* sim = r->sim;
  r->sim = nullptr;
  lk.unlock();
  // the caller's own work on the simulation runs on the server's stream
  const hipError_t e = hipStreamSynchronize(s->stream);
  lk.lock();
  elbm::release_sim(sim);
  s->pool->release(r->off, r->state_bytes);
  s->kick++;
  s->cv.notify_all();
  return e == hipSuccess ? ELBM_OK : set_error(ELBM_EDEVICE, "hipStreamSynchronize failed");
}

elbm_status elbm_server_get_stats(elbm_server* s, elbm_server_stats* out) {
  if (!s || !out) return set_error(ELBM_EINVAL, "server / stats is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  return ELBM_OK;
}

elbm_status elbm_server_destroy(elbm_server* s) {
  if (!s) return ELBM_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->kick++;
    s->cv.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  const hipError_t e = hipStreamSynchronize(s->stream);
  for (auto& kv : s->reqs) {
    Req* r = kv.second.get();
    if (r->sim) elbm::release_sim(r->sim);
    if (r->host.p) (void)hipHostFree(r->host.p);
    if (r->ckpt.p) (void)hipHostFree(r->ckpt.p);
  }
  for (auto& p : s->pinned_cache) (void)hipHostFree(p.p);
  for (hipEvent_t ev : s->spare_events) (void)hipEventDestroy(ev);
  const bool broken = s->broken;
  const std::string why = s->error;
  delete s;
  if (broken) return set_error(ELBM_EDEVICE, why.c_str());
  return e == hipSuccess ? ELBM_OK : set_error(ELBM_EDEVICE, "hipStreamSynchronize failed");
}

}  // extern "C"
