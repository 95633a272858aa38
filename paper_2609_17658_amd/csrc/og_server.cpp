// Serving: continuous batching of force-evaluation requests.
//
// Each request is one box (positions, masses, parameters, output buffers).
// A request is admitted when a stream slot is free and its tree's device
// footprint (og_tree_workspace_bound) fits in what is left of the HBM budget;
// the footprint is carved from one device arena (first fit), so admission
// never calls hipMalloc.  Admitted requests are built and walked on their own
// stream, so their kernels overlap on the device; the request queue is
// first-come first-served.  A request's completion is observed through an
// event; its slot is then free for the next request while its tree stays
// resident (and its memory reserved) until the caller releases the ticket.
//
// Inputs are ordered after the caller's stream: submit records an event on
// the request's params.stream, and the slot stream waits for it before the
// build, so positions still being written there are read only once written.
#include <hip/hip_runtime.h>

#include <chrono>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "og_forest.h"

using namespace og;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) with coalescing free list.
struct Arena {
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  void init(size_t n) {
    size = n;
    free_.clear();
    free_[0] = n;
  }
  bool alloc(size_t n, size_t &off) {
    n = (n + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        off = it->first;
        const size_t rest = it->second - n;
        free_.erase(it);
        if (rest) free_[off + n] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) & ~(size_t)255;
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
};

enum State { kPending = 0, kRunning = 1, kDone = 2, kFailed = 3 };

// An event shared between the request and any thread waiting on it outside
// the server's lock, so that a concurrent release cannot destroy it under
// the waiter: it is destroyed when the last holder lets go.
struct Event {
  hipEvent_t e = nullptr;
  ~Event() {
    if (e) (void)hipEventDestroy(e);
  }
};
using EventRef = std::shared_ptr<Event>;

EventRef make_event() {
  auto ev = std::make_shared<Event>();
  if (hipEventCreateWithFlags(&ev->e, hipEventDisableTiming) != hipSuccess) {
    ev->e = nullptr;
    return nullptr;
  }
  return ev;
}

struct Request {
  og_box box;
  size_t bytes = 0, off = 0;
  int slot = -1;
  bool has_mem = false;
  State state = kPending;
  int error = OG_OK;
  double t_arrive = 0, t_done = 0;
  og_tree *tree = nullptr;
  EventRef ready;  // recorded on the caller's stream at submit
  EventRef done;   // recorded on the slot stream after the walk
};

}  // namespace

struct og_server {
  std::mutex mu;
  size_t budget = 0, reserved = 0;
  void *mem = nullptr;
  Arena arena;
  std::vector<hipStream_t> streams;
  std::vector<int> slot_busy;
  std::deque<uint64_t> pending;
  std::unordered_map<uint64_t, Request> reqs;
  uint64_t next_ticket = 1;
  int in_flight = 0;
  size_t max_pending = 1u << 16;

  int admit_locked();
  int retire_locked();
};

int og_server::retire_locked() {
  for (auto &kv : reqs) {
    Request &r = kv.second;
    if (r.state != kRunning) continue;
    hipError_t e = hipEventQuery(r.done->e);
    if (e == hipErrorNotReady) continue;
    if (e != hipSuccess) {
      (void)hipGetLastError();
      r.error = OG_EDEVICE;
      r.state = kFailed;
    } else {
      r.state = kDone;
      const int st = og_tree_status(r.tree);
      if (st != OG_OK) {
        r.error = st;
        r.state = kFailed;
      }
    }
    r.t_done = now_s();
    slot_busy[r.slot] = 0;
    r.slot = -1;
    --in_flight;
  }
  return OG_OK;
}

int og_server::admit_locked() {
  while (!pending.empty()) {
    const uint64_t tk = pending.front();
    Request &r = reqs[tk];
    int slot = -1;
    for (size_t s = 0; s < streams.size(); ++s)
      if (!slot_busy[s]) {
        slot = (int)s;
        break;
      }
    if (slot < 0) return OG_OK;                      // wait for a slot
    if (reserved + r.bytes > budget) return OG_OK;   // wait for memory
    if (fault_fires(kFaultAlloc)) {                  // forced: this request fails, the rest go on
      pending.pop_front();
      r.error = fail(OG_ENOMEM, "forced failure of the admission (OG_FAULT_ALLOC)");
      r.state = kFailed;
      r.t_done = now_s();
      continue;
    }
    size_t off = 0;
    if (!arena.alloc(r.bytes, off)) return OG_OK;    // fragmented: wait for releases
    pending.pop_front();
    r.off = off;
    r.has_mem = true;
    r.slot = slot;
    reserved += (r.bytes + 255) & ~(size_t)255;
    og_params p = r.box.params;
    p.stream = streams[slot];
    p.workspace = static_cast<char *>(mem) + off;
    p.workspace_bytes = r.bytes;
    int rc = hipStreamWaitEvent(streams[slot], r.ready->e, 0) == hipSuccess ? OG_OK
                                                                           : hip_fail(hipGetLastError(), "hipStreamWaitEvent");
    if (rc == OG_OK) rc = og_tree_build(r.box.pos, r.box.mass, r.box.N, r.box.box, &p, &r.tree);
    if (rc == OG_OK) rc = og_tree_force(r.tree, nullptr, r.box.acc, r.box.pot);
    if (rc == OG_OK && hipEventRecord(r.done->e, streams[slot]) != hipSuccess) rc = OG_EDEVICE;
    if (rc != OG_OK) {
      // whatever was enqueued before the failure must finish before the
      // request's arena range can be handed to another request
      (void)hipStreamSynchronize(streams[slot]);
      (void)hipGetLastError();
      r.error = rc;
      r.state = kFailed;
      r.t_done = now_s();
      r.slot = -1;
      continue;
    }
    r.state = kRunning;
    slot_busy[slot] = 1;
    ++in_flight;
  }
  return OG_OK;
}

extern "C" {

int og_server_create(size_t hbm_budget_bytes, int32_t max_slots, og_server **out) {
  if (!out) return fail(OG_EINVAL, "out is NULL");
  if (hbm_budget_bytes < (1u << 20)) return fail(OG_EINVAL, "budget below 1 MiB");
  if (max_slots < 1 || max_slots > 64) return fail(OG_EINVAL, "max_slots outside 1..64");
  og_server *s = new (std::nothrow) og_server();
  if (!s) return fail(OG_ENOMEM, "host allocation");
  s->budget = hbm_budget_bytes;
  if (fault_fires(kFaultAlloc)) {
    delete s;
    return fail(OG_ENOMEM, "forced failure of the server arena (OG_FAULT_ALLOC)");
  }
  hipError_t e = hipMalloc(&s->mem, hbm_budget_bytes);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "hipMalloc(server arena)");
  }
  s->arena.init(hbm_budget_bytes);
  s->streams.resize(max_slots, nullptr);
  s->slot_busy.assign(max_slots, 0);
  for (int i = 0; i < max_slots; ++i) {
    e = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking);
    if (e != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipStreamDestroy(s->streams[j]);
      (void)hipFree(s->mem);
      delete s;
      return hip_fail(e, "hipStreamCreate");
    }
  }
  *out = s;
  return OG_OK;
}

int og_server_submit(og_server *s, const og_box *req, uint64_t *ticket) {
  const og::TraceRange trace_range("og_server_submit");
  if (!s || !req || !ticket) return fail(OG_EINVAL, "NULL argument");
  int rc = check_params(&req->params, req->N, req->box, false);
  if (rc) return rc;
  if (req->params.criterion == OG_OPEN_RELATIVE)
    return fail(OG_EUNSUPPORTED, "the relative criterion needs a_old, not available to served requests");
  if (!is_device_ptr(req->pos) || !is_device_ptr(req->mass) || !is_device_ptr(req->acc) ||
      (req->pot && !is_device_ptr(req->pot)))
    return fail(OG_EINVAL, "pos/mass/acc/pot must be device pointers");
  og_params p = req->params;
  p.workspace = nullptr;
  const size_t bytes = og_tree_workspace_bound(req->N, &p);
  if (bytes == 0) return fail(OG_EINVAL, "invalid request size");
  std::lock_guard<std::mutex> lk(s->mu);
  if (bytes > s->budget) return fail(OG_EBUSY, "request needs %zu bytes, budget is %zu", bytes, s->budget);
  if (s->pending.size() >= s->max_pending) return fail(OG_EBUSY, "pending queue full");
  const uint64_t tk = s->next_ticket++;
  Request &r = s->reqs[tk];
  r.box = *req;
  r.bytes = bytes;
  r.t_arrive = now_s();
  r.ready = make_event();
  r.done = make_event();
  if (!r.ready || !r.done) {
    s->reqs.erase(tk);
    return hip_fail(hipGetLastError(), "hipEventCreate");
  }
  if (hipEventRecord(r.ready->e, (hipStream_t)req->params.stream) != hipSuccess) {
    s->reqs.erase(tk);
    return hip_fail(hipGetLastError(), "hipEventRecord(caller stream)");
  }
  s->pending.push_back(tk);
  s->retire_locked();
  s->admit_locked();
  *ticket = tk;
  return OG_OK;
}

int og_server_progress(og_server *s) {
  if (!s) return fail(OG_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  s->retire_locked();
  return s->admit_locked();
}

int og_server_poll(og_server *s, uint64_t ticket, int32_t *done, double *t_arrive, double *t_done) {
  if (!s) return fail(OG_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  s->retire_locked();
  s->admit_locked();
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(OG_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  const Request &r = it->second;
  if (done) *done = (r.state == kDone || r.state == kFailed) ? 1 : 0;
  if (t_arrive) *t_arrive = r.t_arrive;
  if (t_done) *t_done = r.t_done;
  if (r.state == kFailed) return fail(r.error, "request failed");
  return OG_OK;
}

int og_server_wait(og_server *s, uint64_t ticket) {
  if (!s) return fail(OG_EINVAL, "server is NULL");
  while (true) {
    EventRef ev;  // held outside the lock: a concurrent release cannot destroy it
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->retire_locked();
      s->admit_locked();
      auto it = s->reqs.find(ticket);
      if (it == s->reqs.end()) return fail(OG_ENOTFOUND, "unknown ticket");
      const Request &r = it->second;
      if (r.state == kDone) return OG_OK;
      if (r.state == kFailed) return fail(r.error, "request failed");
      if (r.state == kRunning) ev = r.done;
      else if (s->in_flight > 0) {
        // pending: wait for any running request to finish
        for (auto &kv : s->reqs)
          if (kv.second.state == kRunning) {
            ev = kv.second.done;
            break;
          }
      }
    }
    if (ev) {
      hipError_t e = hipEventSynchronize(ev->e);
      if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    } else {
      // pending with nothing running: memory is held by done, unreleased requests
      return fail(OG_EBUSY, "request cannot be admitted until resident trees are released");
    }
  }
}

int og_server_release(og_server *s, uint64_t ticket) {
  if (!s) return fail(OG_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  s->retire_locked();
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(OG_ENOTFOUND, "unknown ticket");
  Request &r = it->second;
  if (r.state == kRunning) {
    (void)hipEventSynchronize(r.done->e);
    s->retire_locked();
  }
  if (r.state == kPending) {
    for (auto p = s->pending.begin(); p != s->pending.end(); ++p)
      if (*p == ticket) {
        s->pending.erase(p);
        break;
      }
  } else {
    if (r.tree) og::tree_free_nosync(r.tree);  // its work has completed
    if (r.has_mem) {
      s->arena.release(r.off, r.bytes);
      s->reserved -= (r.bytes + 255) & ~(size_t)255;
    }
  }
  s->reqs.erase(it);  // its events go with the last holder
  s->admit_locked();
  return OG_OK;
}

int og_server_stats(const og_server *cs, size_t *reserved, int32_t *in_flight, int32_t *pending) {
  if (!cs) return fail(OG_EINVAL, "server is NULL");
  og_server *s = const_cast<og_server *>(cs);
  std::lock_guard<std::mutex> lk(s->mu);
  if (reserved) *reserved = s->reserved;
  if (in_flight) *in_flight = s->in_flight;
  if (pending) *pending = (int32_t)s->pending.size();
  return OG_OK;
}

int og_server_destroy(og_server *s) {
  if (!s) return OG_OK;
  for (auto st : s->streams) (void)hipStreamSynchronize(st);
  for (auto &kv : s->reqs)
    if (kv.second.tree) og::tree_free_nosync(kv.second.tree);
  s->reqs.clear();
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  if (s->mem) (void)hipFree(s->mem);
  delete s;
  return OG_OK;
}

}  // extern "C"
