// Continuous-batching request server.
//
// The map and its pyramid stay resident; view and edit requests arrive
// from any client thread and one server thread turns them into GPU work:
//
//  * admission: requests are taken strictly in submission order; a view is
//    admitted when its hit buffer fits in the device pool (the in-flight
//    budget), otherwise it and everything behind it wait for releases;
//  * batching: admitted views are launched together as one render call on
//    one of several streams, so batches that arrive while others run
//    overlap on the device;
//  * edits: the map lives in two version buffers.  A view renders the
//    version holding exactly the edits submitted before it.  Edit k goes
//    into the buffer that does not hold the newest version -- once no batch
//    still reads it -- after that buffer has caught up by replaying edit
//    k - 1 (it holds every edit before that one), on a separate stream;
//    batches of later views wait for that stream's event.  The catch-up
//    replay runs as soon as no batch reads the older buffer, usually well
//    before edit k arrives, so edit k then costs only its own update.
//    Every edit is thus applied twice, once per buffer, and no map is ever
//    copied.  A view's result is the same alone and in any mix.
//  * batches run the render mode and options of the context; the split
//    pass of the hierarchical mode runs for batches of at most two views
//    (a lone large view's longest rays then finish in parallel, as in
//    tc_render_views) and is off for larger ones (there the second launch
//    costs more latency than the long walks it shortens);
//  * wake-up: submissions signal the server thread; it polls while work is
//    queued or on the device, keeps polling for a short while after the
//    last activity (so a request arriving soon after does not wait for a
//    thread wake-up), and only then sleeps until the next signal.
//
// Section 2 of the paper: edits are gameplay operations whose results must
// be visible without reloading; Section 7: its frames are submitted and
// awaited one at a time, with nothing overlapping.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "tc_context.h"

using tci::fail;
using tci::hip_fail;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

enum : int32_t { kQueued = 0, kInFlight = 1, kDone = 2 };

struct Request {
  uint64_t id = 0;
  bool is_edit = false;
  tc_view view{};
  std::vector<tc_edit> edits;
  std::vector<uint8_t> patch;
  uint64_t epoch = 0;       // views: edits before it; edits: its number
  size_t bytes = 0;
  size_t pool_off = 0;
  bool has_mem = false;
  int32_t state = kQueued;
  double t_submit = 0, t_launch = 0, t_done = 0;
  int64_t rays = 0;
};

// Batches of at most this many views run the split pass.
constexpr size_t kSplitMaxViews = 2;
// After the last activity the server thread keeps polling this long
// before it sleeps.
constexpr double kSpinSeconds = 200e-6;
// A batch starts beside one already on the device only when at least this
// many views wait: a lone view waits for the batch in flight instead, since
// two concurrent launches slow the one in flight by about what they save the
// newcomer (at low rates that was the served p99's excess over FIFO).
constexpr size_t kOverlapMinViews = 2;

// First-fit allocator over [0, size) with 256-byte granules.
class Pool {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    used_ = 0;
  }
  bool alloc(size_t n, size_t* off) {
    n = (n + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        size_t rest = it->second - n, o = it->first + n;
        free_.erase(it);
        if (rest) free_[o] = rest;
        used_ += n;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) & ~(size_t)255;
    used_ -= n;
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
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

// An uploaded edit list, kept until both version buffers hold it.
struct EditUpload {
  tci::EditPlan plan;
  tci::Slot slot;
  uint64_t epoch = 0;
  bool valid = false;
};

struct Batch {
  std::vector<uint64_t> ids;
  int version = 0;
  hipEvent_t done = nullptr;
  tci::Slot slot;
  bool busy = false;
  hipStream_t stream = nullptr;
  uint64_t edit_seen = 0;   // the edit_ev recording this stream last waited for
};

}  // namespace

struct tc_server {
  tc_context* ctx = nullptr;
  uint32_t flags = 0;
  size_t budget = 0;
  int32_t max_batch = 64;
  char* pool_dev = nullptr;
  Pool pool;
  // map versions: buffer pointers, the epoch each holds, batches reading it
  uint32_t* ver[2] = {nullptr, nullptr};
  uint64_t ver_epoch[2] = {0, 0};
  int ver_readers[2] = {0, 0};
  int current = 0;
  bool own_ver[2] = {false, false};
  hipStream_t edit_stream = nullptr;
  hipEvent_t edit_ev = nullptr;           // end of the newest edit
  uint64_t edit_gen = 0;                   // recordings of edit_ev so far
  std::deque<std::pair<uint64_t, hipEvent_t>> edits_in_flight;
  EditUpload uploads[2];                   // the newest edit and the one before
  uint64_t edits_applied = 0;
  std::vector<Batch> slots;
  // request state (guarded by mu)
  std::mutex mu;
  std::condition_variable cv_done;
  std::condition_variable cv_work;         // signalled on submission and stop
  std::unordered_map<uint64_t, Request> reqs;
  std::deque<uint64_t> incoming;
  uint64_t next_id = 1;
  uint64_t edits_submitted = 0;
  // owned by the server thread
  std::deque<uint64_t> fifo;
  std::vector<uint64_t> admitted;
  std::thread thread;
  std::atomic<bool> stop{false};
  std::atomic<int> error{0};
  std::string err;
  // statistics
  std::atomic<uint64_t> st_batches{0}, st_edits{0}, st_views{0}, st_rays{0};
  std::atomic<uint64_t> st_peak_bytes{0};
  double st_queue_s = 0, st_run_s = 0;    // sums over finished views (under mu)
};

namespace {

tci_map version_desc(const tc_server* s, int v) {
  tci_map d = s->ctx->desc;
  d.base = s->ver[v];
  return d;
}

void set_error(tc_server* s, hipError_t e, const char* what) {
  std::lock_guard<std::mutex> g(s->mu);
  if (!s->error.load()) {
    s->err = std::string(what) + ": " + hipGetErrorString(e);
    s->error.store(1);
  }
  s->cv_done.notify_all();
}

void complete(tc_server* s, const std::vector<uint64_t>& ids, double t) {
  std::lock_guard<std::mutex> g(s->mu);
  for (uint64_t id : ids) {
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) continue;
    Request& r = it->second;
    r.state = kDone;
    r.t_done = t;
    if (!r.is_edit) {
      s->st_views++;
      s->st_rays += (uint64_t)r.rays;
      s->st_queue_s += r.t_launch - r.t_submit;
      s->st_run_s += t - r.t_launch;
      if ((s->flags & TC_SERVER_AUTO_RELEASE) && r.has_mem) {
        s->pool.release(r.pool_off, r.bytes);
        r.has_mem = false;
      }
    }
  }
  s->cv_done.notify_all();
}

// Launch the admitted views as one batch; returns false if no stream slot
// is free, or if a batch is in flight and fewer than kOverlapMinViews views
// wait.
bool launch_batch(tc_server* s) {
  if (s->admitted.empty()) return true;
  Batch* b = nullptr;
  bool in_flight = false;
  for (Batch& c : s->slots) {
    if (c.busy) in_flight = true;
    else if (!b) b = &c;
  }
  if (!b) return false;
  if (in_flight && s->admitted.size() < kOverlapMinViews) return false;
  tc_context* ctx = s->ctx;
  std::vector<tc_view> views;
  std::vector<size_t> offs;
  const double t = now_s();
  {
    std::lock_guard<std::mutex> g(s->mu);
    for (uint64_t id : s->admitted) {
      Request& r = s->reqs[id];
      views.push_back(r.view);
      offs.push_back(r.pool_off);
      r.state = kInFlight;
      r.t_launch = t;
    }
  }
  // the split pass for small batches only (see the header); its queue is
  // the slot's device-only buffer
  tci::ViewPlan plan;
  const bool split = views.size() <= kSplitMaxViews;
  if (tci::plan_views(ctx, views.data(), (int32_t)views.size(), plan, split) != TC_OK) {
    set_error(s, hipErrorInvalidValue, "server: view validation");
    return true;
  }
  for (size_t i = 0; i < views.size(); ++i) plan.views[i].out_base = (int64_t)(offs[i] / 8);
  plan.qcap = std::min<uint32_t>(plan.qcap, b->slot.qcap);
  if (b->slot.cap < plan.off_queue) {
    if (b->slot.host) (void)hipHostFree(b->slot.host);
    if (b->slot.dev) (void)hipFree(b->slot.dev);
    b->slot.host = b->slot.dev = nullptr;
    size_t cap = std::max<size_t>(plan.off_queue, tci::kSlotBytes);
    hipError_t e = tci::host_alloc(ctx, &b->slot.host, cap);
    if (e == hipSuccess) e = tci::dev_alloc(ctx, &b->slot.dev, cap);
    if (e != hipSuccess) {
      set_error(s, e, "server: staging allocation");
      return true;
    }
    b->slot.cap = cap;
  }
  tci::write_views(plan, (char*)b->slot.host);
  const int v = s->current;
  // a stream waits for each recording of edit_ev once: its later work is
  // ordered after that wait anyway (a wait is a packet of its own on the
  // stream, a few microseconds on every request otherwise)
  hipError_t e = hipSuccess;
  if (b->edit_seen != s->edit_gen) {
    e = hipStreamWaitEvent(b->stream, s->edit_ev, 0);
    if (e == hipSuccess) b->edit_seen = s->edit_gen;
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->slot.dev, b->slot.host, plan.off_queue, hipMemcpyHostToDevice,
                       b->stream);
  if (e == hipSuccess)
    e = tci::enqueue_render(ctx, version_desc(s, v), (const char*)b->slot.dev, plan,
                            s->pool_dev, b->stream, nullptr, nullptr, true, b->slot.queue);
  if (e == hipSuccess) e = hipEventRecord(b->done, b->stream);
  if (e != hipSuccess) {
    set_error(s, e, "server: render launch");
    return true;
  }
  b->ids.swap(s->admitted);
  s->admitted.clear();
  b->version = v;
  b->busy = true;
  s->ver_readers[v]++;
  s->st_batches++;
  return true;
}

// Apply the edit request at the head of the queue, if the target version
// buffer is free.  Returns true if it was applied (or failed for good).
bool apply_edit(tc_server* s, uint64_t id) {
  const int tgt = 1 - s->current;
  if (s->ver_readers[tgt] > 0) return false;
  Request* r;
  {
    std::lock_guard<std::mutex> g(s->mu);
    r = &s->reqs[id];
    r->state = kInFlight;
  }
  const tci_map d = version_desc(s, tgt);
  // the target holds every edit but the newest applied one: replay it
  hipError_t e = hipSuccess;
  if (s->ver_epoch[tgt] != s->ver_epoch[s->current]) {
    const EditUpload& prev = s->uploads[(s->edits_applied - 1) & 1];
    if (!prev.valid || prev.epoch != s->ver_epoch[s->current]) {
      set_error(s, hipErrorInvalidValue, "server: edit log out of step");
      return true;
    }
    e = tci::enqueue_edits(d, s->ver[tgt], (const char*)prev.slot.dev, prev.plan,
                           s->edit_stream);
  }
  // upload the new edit list into the other log slot; its previous content
  // (the edit before the replayed one) is in both buffers already
  EditUpload& u = s->uploads[s->edits_applied & 1];
  size_t patch_bytes = r->patch.size();
  tci::plan_edits(d, r->edits.data(), (int32_t)r->edits.size(), patch_bytes, nullptr, u.plan);
  if (u.slot.pending) {
    // the host buffer is rewritten only after its last upload was consumed
    (void)hipEventSynchronize(u.slot.ev);
    u.slot.pending = false;
  }
  if (u.slot.cap < u.plan.total) {
    (void)hipStreamSynchronize(s->edit_stream);
    if (u.slot.host) (void)hipHostFree(u.slot.host);
    if (u.slot.dev) (void)hipFree(u.slot.dev);
    u.slot.host = u.slot.dev = nullptr;
    u.slot.cap = 0;
    size_t cap = std::max<size_t>(u.plan.total, tci::kSlotBytes);
    hipError_t ea = tci::host_alloc(s->ctx, &u.slot.host, cap);
    if (ea == hipSuccess) ea = tci::dev_alloc(s->ctx, &u.slot.dev, cap);
    if (ea != hipSuccess) {
      set_error(s, ea, "server: edit staging");
      return true;
    }
    u.slot.cap = cap;
  }
  tci::plan_edits(d, r->edits.data(), (int32_t)r->edits.size(), patch_bytes,
                  (char*)u.slot.host, u.plan);
  if (e == hipSuccess)
    e = hipMemcpyAsync(u.slot.dev, u.slot.host, u.plan.total, hipMemcpyHostToDevice,
                       s->edit_stream);
  if (e == hipSuccess) e = hipEventRecord(u.slot.ev, s->edit_stream);
  if (e == hipSuccess) u.slot.pending = true;
  if (e == hipSuccess)
    e = tci::enqueue_edits(d, s->ver[tgt], (const char*)u.slot.dev, u.plan, s->edit_stream);
  hipEvent_t ev = nullptr;
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(ev, s->edit_stream);
  if (e == hipSuccess) e = hipEventRecord(s->edit_ev, s->edit_stream);
  if (e == hipSuccess) s->edit_gen++;
  if (e != hipSuccess) {
    if (ev) (void)hipEventDestroy(ev);
    set_error(s, e, "server: edit launch");
    return true;
  }
  u.epoch = r->epoch;
  u.valid = true;
  s->edits_applied++;
  s->ver_epoch[tgt] = r->epoch;
  s->current = tgt;
  s->edits_in_flight.emplace_back(id, ev);
  s->st_edits++;
  return true;
}

// Bring the version buffer that is not current up to date in the background
// (replay the newest edit onto it, on the edit stream) as soon as no batch
// reads it, so that the next edit finds it ready: views waiting on that
// edit then wait for its own update only, not for the replay before it.
void catch_up(tc_server* s) {
  const int other = 1 - s->current;
  if (s->edits_applied == 0 || s->ver_epoch[other] == s->ver_epoch[s->current] ||
      s->ver_readers[other] > 0)
    return;
  const EditUpload& prev = s->uploads[(s->edits_applied - 1) & 1];
  if (!prev.valid || prev.epoch != s->ver_epoch[s->current]) return;  // apply_edit reports it
  const hipError_t e = tci::enqueue_edits(version_desc(s, other), s->ver[other],
                                          (const char*)prev.slot.dev, prev.plan, s->edit_stream);
  if (e != hipSuccess) {
    set_error(s, e, "server: edit replay");
    return;
  }
  s->ver_epoch[other] = s->ver_epoch[s->current];
}

void poll_completions(tc_server* s) {
  for (Batch& b : s->slots) {
    if (!b.busy) continue;
    hipError_t q = hipEventQuery(b.done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) {
      set_error(s, q, "server: batch");
      continue;
    }
    complete(s, b.ids, now_s());
    b.ids.clear();
    b.busy = false;
    s->ver_readers[b.version]--;
  }
  while (!s->edits_in_flight.empty()) {
    auto& f = s->edits_in_flight.front();
    hipError_t q = hipEventQuery(f.second);
    if (q == hipErrorNotReady) break;
    (void)hipEventDestroy(f.second);
    complete(s, {f.first}, now_s());
    s->edits_in_flight.pop_front();
  }
}

void server_loop(tc_server* s) {
  (void)hipSetDevice(s->ctx->device);
  double last_active = now_s();
  while (true) {
    {
      std::lock_guard<std::mutex> g(s->mu);
      while (!s->incoming.empty()) {
        s->fifo.push_back(s->incoming.front());
        s->incoming.pop_front();
      }
    }
    poll_completions(s);
    if (s->error.load()) break;
    // admit in order
    while (!s->fifo.empty()) {
      const uint64_t id = s->fifo.front();
      bool is_edit;
      size_t bytes;
      {
        std::lock_guard<std::mutex> g(s->mu);
        Request& r = s->reqs[id];
        is_edit = r.is_edit;
        bytes = r.bytes;
      }
      if (is_edit) {
        if (!s->admitted.empty() && !launch_batch(s)) break;
        if (!s->admitted.empty()) break;
        if (!apply_edit(s, id)) break;
        s->fifo.pop_front();
        continue;
      }
      size_t off;
      bool ok;
      {
        std::lock_guard<std::mutex> g(s->mu);
        ok = s->pool.alloc(bytes, &off);
        if (ok) {
          Request& r = s->reqs[id];
          r.pool_off = off;
          r.has_mem = true;
          uint64_t used = s->pool.used();
          if (used > s->st_peak_bytes.load()) s->st_peak_bytes.store(used);
        }
      }
      if (!ok) break;
      s->admitted.push_back(id);
      s->fifo.pop_front();
      if ((int32_t)s->admitted.size() >= s->max_batch && !launch_batch(s)) break;
    }
    if (!s->admitted.empty()) launch_batch(s);
    catch_up(s);
    bool idle;
    {
      std::lock_guard<std::mutex> g(s->mu);
      idle = s->fifo.empty() && s->incoming.empty() && s->admitted.empty();
    }
    bool busy = !s->edits_in_flight.empty();
    for (Batch& b : s->slots) busy |= b.busy;
    if (!idle || busy) {
      last_active = now_s();
      std::this_thread::yield();
    } else if (now_s() - last_active < kSpinSeconds) {
      // just went idle: keep polling the submission queue for a while
      if (s->stop.load()) break;
      std::this_thread::yield();
    } else {
      if (s->stop.load()) break;
      // sleep until a submission or stop (the timeout only bounds a missed
      // signal)
      std::unique_lock<std::mutex> g(s->mu);
      s->cv_work.wait_for(g, std::chrono::milliseconds(2),
                          [s] { return !s->incoming.empty() || s->stop.load(); });
    }
  }
  // drain the device before leaving
  for (Batch& b : s->slots)
    if (b.stream) (void)hipStreamSynchronize(b.stream);
  if (s->edit_stream) (void)hipStreamSynchronize(s->edit_stream);
  poll_completions(s);
  std::lock_guard<std::mutex> g(s->mu);
  s->cv_done.notify_all();
}

void server_free(tc_server* s) {
  if (!s) return;
  for (Batch& b : s->slots) {
    if (b.stream) (void)hipStreamDestroy(b.stream);
    if (b.done) (void)hipEventDestroy(b.done);
    if (b.slot.host) (void)hipHostFree(b.slot.host);
    if (b.slot.dev) (void)hipFree(b.slot.dev);
    if (b.slot.queue) (void)hipFree(b.slot.queue);
  }
  for (auto& f : s->edits_in_flight) (void)hipEventDestroy(f.second);
  for (EditUpload& u : s->uploads) {
    if (u.slot.host) (void)hipHostFree(u.slot.host);
    if (u.slot.dev) (void)hipFree(u.slot.dev);
    if (u.slot.ev) (void)hipEventDestroy(u.slot.ev);
  }
  if (s->edit_ev) (void)hipEventDestroy(s->edit_ev);
  if (s->edit_stream) (void)hipStreamDestroy(s->edit_stream);
  for (int v = 0; v < 2; ++v)
    if (s->own_ver[v] && s->ver[v]) (void)hipFree(s->ver[v]);
  if (s->pool_dev) (void)hipFree(s->pool_dev);
  delete s;
}

}  // namespace

extern "C" {

tc_status tc_server_start(tc_context* ctx, uint64_t budget_bytes, int32_t max_batch_views,
                          int32_t streams, uint32_t flags, tc_server** out) {
  if (!ctx) return TC_INVALID_ARG;
  if (!out) return fail(ctx, TC_INVALID_ARG, "tc_server_start: out is NULL");
  *out = nullptr;
  ctx->err.clear();
  if (!ctx->map) return fail(ctx, TC_NO_MAP, "tc_server_start: no map loaded");
  if (ctx->server) return fail(ctx, TC_INVALID_ARG, "tc_server_start: a server is running");
  if (ctx->render_mode == 5 || ctx->vox)
    return fail(ctx, TC_INVALID_ARG,
                "tc_server_start: the voxel occupancy pyramid is not kept per map version; "
                "set TC_OPT_VOXEL_SHAPE to 0 first");
  if (budget_bytes < 4096 || budget_bytes > ((uint64_t)1 << 40))
    return fail(ctx, TC_INVALID_ARG, "tc_server_start: bad budget");
  if (max_batch_views < 1 || max_batch_views > 4096 || streams < 1 || streams > 16)
    return fail(ctx, TC_INVALID_ARG, "tc_server_start: bad batch or stream count");
  if (flags & ~(uint32_t)TC_SERVER_AUTO_RELEASE)
    return fail(ctx, TC_INVALID_ARG, "tc_server_start: unknown flags");
  tc_status st = tci::set_device(ctx);
  if (st) return st;
  tc_server* s = new (std::nothrow) tc_server();
  if (!s) return fail(ctx, TC_OUT_OF_MEMORY, "tc_server_start: host allocation");
  s->ctx = ctx;
  s->flags = flags;
  s->budget = budget_bytes;
  s->max_batch = max_batch_views;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = tci::dev_alloc(ctx, (void**)&s->pool_dev, budget_bytes);
  s->pool.reset(budget_bytes);
  s->ver[0] = ctx->map;
  if (e == hipSuccess) e = tci::dev_alloc(ctx, (void**)&s->ver[1], ctx->map_words * 4);
  s->own_ver[1] = e == hipSuccess;
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->edit_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->edit_ev, hipEventDisableTiming);
  for (EditUpload& u : s->uploads)
    if (e == hipSuccess) e = hipEventCreateWithFlags(&u.slot.ev, hipEventDisableTiming);
  // both version buffers start as the loaded map
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->ver[1], s->ver[0], ctx->map_words * 4, hipMemcpyDeviceToDevice,
                       s->edit_stream);
  if (e == hipSuccess) e = hipEventRecord(s->edit_ev, s->edit_stream);
  if (e == hipSuccess) s->edit_gen++;
  // staging of every batch slot and of the edit log, allocated up front
  s->slots.resize(streams);
  for (Batch& b : s->slots) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
    if (e == hipSuccess) e = tci::host_alloc(ctx, &b.slot.host, tci::kSlotBytes);
    if (e == hipSuccess) e = tci::dev_alloc(ctx, &b.slot.dev, tci::kSlotBytes);
    if (e == hipSuccess) b.slot.cap = tci::kSlotBytes;
    if (e == hipSuccess)
      e = tci::dev_alloc(ctx, (void**)&b.slot.queue,
                         tci::kQueueEntry * (size_t)ctx->split_queue);
    if (e == hipSuccess) b.slot.qcap = (uint32_t)ctx->split_queue;
  }
  for (EditUpload& u : s->uploads) {
    if (e == hipSuccess) e = tci::host_alloc(ctx, &u.slot.host, tci::kSlotBytes);
    if (e == hipSuccess) e = tci::dev_alloc(ctx, &u.slot.dev, tci::kSlotBytes);
    if (e == hipSuccess) u.slot.cap = tci::kSlotBytes;
  }
  if (e != hipSuccess) {
    server_free(s);
    return hip_fail(ctx, e, "tc_server_start");
  }
  try {
    s->thread = std::thread(server_loop, s);
  } catch (...) {
    server_free(s);
    return fail(ctx, TC_OUT_OF_MEMORY, "tc_server_start: cannot start the thread");
  }
  ctx->server = s;
  *out = s;
  return TC_OK;
}

tc_status tc_server_submit_view(tc_server* s, const tc_view* view, uint64_t* id) {
  if (!s || !view || !id) return TC_INVALID_ARG;
  tc_context* ctx = s->ctx;
  tci::ViewPlan plan;
  Request r;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->error.load()) return fail(ctx, TC_DEVICE_ERROR, "%s", s->err.c_str());
    tc_status st = tci::plan_views(ctx, view, 1, plan);
    if (st) return st;
    r.bytes = (size_t)plan.rays * sizeof(tc_hit);
    if (((r.bytes + 255) & ~(size_t)255) > s->budget)
      return fail(ctx, TC_OVER_BUDGET, "tc_server_submit_view: view exceeds the budget");
    r.id = s->next_id++;
    r.view = *view;
    r.rays = plan.rays;
    r.epoch = s->edits_submitted;
    r.t_submit = now_s();
    *id = r.id;
    s->incoming.push_back(r.id);
    s->reqs.emplace(r.id, std::move(r));
  }
  s->cv_work.notify_one();
  return TC_OK;
}

tc_status tc_server_submit_edit(tc_server* s, const tc_edit* edits, int32_t n, uint64_t* id) {
  if (!s || !id) return TC_INVALID_ARG;
  tc_context* ctx = s->ctx;
  size_t patch_bytes = 0;
  std::lock_guard<std::mutex> g(s->mu);
  if (s->error.load()) return fail(ctx, TC_DEVICE_ERROR, "%s", s->err.c_str());
  tc_status st = tci::validate_edits(ctx, edits, n, &patch_bytes);
  if (st) return st;
  if (n < 1) return fail(ctx, TC_INVALID_ARG, "tc_server_submit_edit: no edits");
  Request r;
  r.is_edit = true;
  r.edits.assign(edits, edits + n);
  r.patch.resize(patch_bytes);
  size_t po = 0;
  for (tc_edit& e : r.edits) {
    if (e.kind != TC_EDIT_SET) continue;
    size_t m = (size_t)e.w * e.h;
    memcpy(r.patch.data() + po, e.floor_top, m);
    memcpy(r.patch.data() + po + m, e.slab_bottom, m);
    memcpy(r.patch.data() + po + 2 * m, e.slab_top, m);
    e.floor_top = r.patch.data() + po;
    e.slab_bottom = r.patch.data() + po + m;
    e.slab_top = r.patch.data() + po + 2 * m;
    po += 3 * m;
  }
  r.id = s->next_id++;
  r.epoch = ++s->edits_submitted;
  r.t_submit = now_s();
  *id = r.id;
  s->incoming.push_back(r.id);
  s->reqs.emplace(r.id, std::move(r));
  s->cv_work.notify_one();
  return TC_OK;
}

tc_status tc_server_poll(tc_server* s, uint64_t id, int32_t* state, double* latency_s) {
  if (!s || !state) return TC_INVALID_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(s->ctx, TC_INVALID_ARG, "tc_server_poll: unknown id");
  *state = it->second.state;
  if (latency_s)
    *latency_s = it->second.state == kDone ? it->second.t_done - it->second.t_submit : -1.0;
  if (s->error.load()) return fail(s->ctx, TC_DEVICE_ERROR, "%s", s->err.c_str());
  return TC_OK;
}

tc_status tc_server_poll_many(tc_server* s, const uint64_t* ids, int32_t n, int32_t* states,
                              double* latencies_s) {
  if (!s || n < 0 || (n > 0 && (!ids || !states))) return TC_INVALID_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  for (int32_t i = 0; i < n; ++i)
    if (s->reqs.find(ids[i]) == s->reqs.end())
      return fail(s->ctx, TC_INVALID_ARG, "tc_server_poll_many: unknown id at %d", i);
  for (int32_t i = 0; i < n; ++i) {
    const Request& r = s->reqs.find(ids[i])->second;
    states[i] = r.state;
    if (latencies_s) latencies_s[i] = r.state == kDone ? r.t_done - r.t_submit : -1.0;
  }
  if (s->error.load()) return fail(s->ctx, TC_DEVICE_ERROR, "%s", s->err.c_str());
  return TC_OK;
}

tc_status tc_server_wait(tc_server* s, uint64_t id, double timeout_s) {
  if (!s) return TC_INVALID_ARG;
  std::unique_lock<std::mutex> g(s->mu);
  auto deadline = std::chrono::steady_clock::now() +
                  std::chrono::microseconds((int64_t)(std::max(0.0, timeout_s) * 1e6));
  while (true) {
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(s->ctx, TC_INVALID_ARG, "tc_server_wait: unknown id");
    if (it->second.state == kDone) return TC_OK;
    if (s->error.load()) return fail(s->ctx, TC_DEVICE_ERROR, "%s", s->err.c_str());
    if (s->cv_done.wait_until(g, deadline) == std::cv_status::timeout) {
      it = s->reqs.find(id);
      if (it != s->reqs.end() && it->second.state == kDone) return TC_OK;
      return TC_TIMEOUT;
    }
  }
}

tc_status tc_server_result(tc_server* s, uint64_t id, const tc_hit** device_ptr,
                           int64_t* records) {
  if (!s || !device_ptr || !records) return TC_INVALID_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end() || it->second.is_edit)
    return fail(s->ctx, TC_INVALID_ARG, "tc_server_result: unknown view id");
  const Request& r = it->second;
  if (r.state != kDone || !r.has_mem)
    return fail(s->ctx, TC_INVALID_ARG, "tc_server_result: no result held");
  *device_ptr = (const tc_hit*)(s->pool_dev + r.pool_off);
  *records = r.rays;
  return TC_OK;
}

tc_status tc_server_read(tc_server* s, uint64_t id, tc_hit* host_dst, int64_t records) {
  if (!s || !host_dst) return TC_INVALID_ARG;
  const tc_hit* src = nullptr;
  int64_t n = 0;
  tc_status st = tc_server_result(s, id, &src, &n);
  if (st) return st;
  if (records != n) return fail(s->ctx, TC_INVALID_ARG, "tc_server_read: size mismatch");
  hipError_t e = hipSetDevice(s->ctx->device);
  if (e == hipSuccess) e = hipMemcpy(host_dst, src, (size_t)n * sizeof(tc_hit), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(s->ctx, e, "tc_server_read");
  return TC_OK;
}

tc_status tc_server_release(tc_server* s, uint64_t id) {
  if (!s) return TC_INVALID_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(s->ctx, TC_INVALID_ARG, "tc_server_release: unknown id");
  if (it->second.state != kDone)
    return fail(s->ctx, TC_INVALID_ARG, "tc_server_release: request not done");
  if (it->second.has_mem) s->pool.release(it->second.pool_off, it->second.bytes);
  s->reqs.erase(it);
  return TC_OK;
}

tc_status tc_server_get_stats(tc_server* s, tc_server_stats* out) {
  if (!s || !out) return TC_INVALID_ARG;
  out->batches = s->st_batches.load();
  out->edits = s->st_edits.load();
  out->views = s->st_views.load();
  out->rays = s->st_rays.load();
  out->peak_bytes = s->st_peak_bytes.load();
  std::lock_guard<std::mutex> g(s->mu);
  out->bytes_in_use = s->pool.used();
  out->queue_s = s->st_queue_s;
  out->run_s = s->st_run_s;
  return TC_OK;
}

tc_status tc_server_stop(tc_server* s) {
  if (!s) return TC_INVALID_ARG;
  tc_context* ctx = s->ctx;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop.store(true);
  }
  s->cv_work.notify_all();
  if (s->thread.joinable()) s->thread.join();
  tc_status st = TC_OK;
  (void)hipSetDevice(ctx->device);
  // the newest version becomes the context's map
  if (s->current != 0) {
    hipError_t e = hipMemcpy(ctx->map, s->ver[s->current], ctx->map_words * 4,
                             hipMemcpyDeviceToDevice);
    if (e != hipSuccess) st = hip_fail(ctx, e, "tc_server_stop");
  }
  if (s->error.load()) st = fail(ctx, TC_DEVICE_ERROR, "%s", s->err.c_str());
  ctx->server = nullptr;
  server_free(s);
  return st;
}

}  // extern "C"
