// Serving runtime: continuous batching of independent k-core requests on one device.
//
// kcore_submit copies a host graph and queues it. One dispatcher thread owns the device side: it
// keeps up to `max_inflight` batches in flight, each on its own stream with its own device and
// pinned buffers ("slots"). Whenever a slot is free it admits queued requests in arrival order
// while their device footprint fits the HBM budget and the batch limits, packs them into one
// segmented CSR, and launches: H2D copy, batched peel, D2H copy, then a host callback that wakes
// the dispatcher. Batches on different slots overlap on the device, so requests that arrive while
// others run are started as soon as a slot and budget free up; they do not wait for the device
// to drain. Coreness is exact and independent of which batch a request lands in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/kcore.h"
#include "kcore_internal.h"

namespace {

enum ReqState { RQ_QUEUED, RQ_RUNNING, RQ_DONE, RQ_CANCELED, RQ_FAILED };

struct Request {
  uint64_t ticket = 0;
  int64_t n = 0, m = 0;
  std::vector<int64_t> off;  // owned copies (copying servers)
  std::vector<int32_t> adj;
  const int64_t* offp = nullptr;  // what the dispatcher reads: the copies or the caller's arrays
  const int32_t* adjp = nullptr;
  std::vector<int32_t> core;
  int state = RQ_QUEUED;
  int err = 0;
  int64_t bytes = 0;
  kcore_request_stats st{};
};

struct Slot {
  hipStream_t stream = nullptr;
  bool busy = false;
  std::atomic<int> finished{0};
  int64_t v_cap = 0, e_cap = 0, g_cap = 0;
  int64_t *vptr_d = nullptr, *off_d = nullptr;
  int32_t *adj_d = nullptr, *core_d = nullptr;
  int64_t *vptr_h = nullptr, *off_h = nullptr;
  int32_t *adj_h = nullptr, *core_h = nullptr;
  std::vector<Request*> reqs;
  int64_t bytes = 0;
  int64_t batch_id = 0;
  int rc = 0;
  bool large = false;
};

int64_t footprint(int64_t n, int64_t m) { return 8 * (n + 1) + 4 * m + 16 * n + 64; }

// Requests at least this large run in batches of their own class, so that a large graph (peeled by
// one workgroup) never holds up the completion of a batch of small ones.
constexpr int64_t kLargeEntries = 1 << 21;
bool is_large(int64_t n, int64_t m) { return m >= kLargeEntries || n >= (1 << 16); }

// memcpy split over a few threads for large buffers (request intake and batch packing are the
// host-side cost of serving large graphs).
void par_copy(void* dst, const void* src, size_t bytes) {
  const size_t kMin = 8u << 20;
  if (bytes < kMin) {
    memcpy(dst, src, bytes);
    return;
  }
  unsigned t = std::thread::hardware_concurrency();
  t = t < 2 ? 2 : (t > 8 ? 8 : t);
  const size_t chunk = ((bytes + t - 1) / t + 63) & ~size_t(63);
  std::vector<std::thread> th;
  for (unsigned i = 1; i < t; ++i) {
    const size_t o = chunk * i;
    if (o >= bytes) break;
    const size_t len = o + chunk > bytes ? bytes - o : chunk;
    th.emplace_back([=] { memcpy(static_cast<char*>(dst) + o, static_cast<const char*>(src) + o, len); });
  }
  memcpy(dst, src, chunk < bytes ? chunk : bytes);
  for (auto& x : th) x.join();
}

}  // namespace

struct kcore_server {
  kcore_server_config cfg{};
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;       // dispatcher wake-ups
  std::condition_variable done_cv;  // request completions
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, Request*> all;
  std::vector<Slot*> slots;
  int64_t bytes_in_use = 0;
  uint64_t next_ticket = 1;
  int64_t next_batch = 1;
  bool stop = false;
  std::thread th;

  double now_us() const {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

void host_done(void* p) {
  auto* pr = static_cast<std::pair<kcore_server*, Slot*>*>(p);
  kcore_server* s = pr->first;
  Slot* sl = pr->second;
  delete pr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    sl->finished.store(1);
  }
  s->cv.notify_all();
}

int grow(Slot* sl, int64_t V, int64_t E, int64_t G) {
  if (V <= sl->v_cap && E <= sl->e_cap && G <= sl->g_cap) return 0;
  const int64_t v = std::max(V, sl->v_cap) * 5 / 4 + 1024;
  const int64_t e = std::max(E, sl->e_cap) * 5 / 4 + 4096;
  const int64_t g = std::max(G, sl->g_cap) * 5 / 4 + 64;
  hipFree(sl->vptr_d);
  hipFree(sl->off_d);
  hipFree(sl->adj_d);
  hipFree(sl->core_d);
  hipHostFree(sl->vptr_h);
  hipHostFree(sl->off_h);
  hipHostFree(sl->adj_h);
  hipHostFree(sl->core_h);
  sl->vptr_d = sl->off_d = sl->vptr_h = sl->off_h = nullptr;
  sl->adj_d = sl->core_d = sl->adj_h = sl->core_h = nullptr;
  sl->v_cap = sl->e_cap = sl->g_cap = 0;
  if (hipMalloc(&sl->vptr_d, 8 * (g + 1)) != hipSuccess || hipMalloc(&sl->off_d, 8 * (v + 1)) != hipSuccess ||
      hipMalloc(&sl->adj_d, 4 * e) != hipSuccess || hipMalloc(&sl->core_d, 4 * v) != hipSuccess ||
      hipHostMalloc((void**)&sl->vptr_h, 8 * (g + 1), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&sl->off_h, 8 * (v + 1), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&sl->adj_h, 4 * e, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&sl->core_h, 4 * v, hipHostMallocDefault) != hipSuccess)
    return KCORE_ENOMEM;
  sl->v_cap = v;
  sl->e_cap = e;
  sl->g_cap = g;
  return 0;
}

// Packs the slot's requests into its pinned buffers and enqueues copy-in, peel, copy-out and the
// completion callback on the slot's stream. Called by the dispatcher without the server lock.
int launch_slot(kcore_server* s, Slot* sl) {
  int64_t V = 0, E = 0;
  for (Request* r : sl->reqs) {
    V += r->n;
    E += r->m;
  }
  const int64_t G = (int64_t)sl->reqs.size();
  if (int rc = grow(sl, V, E, G)) return rc;
  int64_t vb = 0, eb = 0;
  sl->vptr_h[0] = 0;
  hipStream_t st = sl->stream;
  // Borrowed large requests are copied to the device straight from the caller's arrays (one DMA
  // each); everything else is packed into the slot's pinned buffer and copied in one piece.
  const bool direct = s->cfg.borrow_inputs && sl->large;
  for (int64_t g = 0; g < G; ++g) {
    Request* r = sl->reqs[g];
    for (int64_t i = 0; i < r->n; ++i) sl->off_h[vb + i] = eb + r->offp[i];
    // adjacency keeps the request's own (local) ids: the peel is launched in local-id mode
    if (r->m) {
      if (direct) {
        if (hipMemcpyAsync(sl->adj_d + eb, r->adjp, sizeof(int32_t) * (size_t)r->m, hipMemcpyHostToDevice,
                           st) != hipSuccess)
          return KCORE_EDEVICE;
      } else {
        par_copy(sl->adj_h + eb, r->adjp, sizeof(int32_t) * (size_t)r->m);
      }
    }
    vb += r->n;
    eb += r->m;
    sl->vptr_h[g + 1] = vb;
  }
  sl->off_h[V] = E;
  if (hipMemcpyAsync(sl->vptr_d, sl->vptr_h, 8 * (G + 1), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(sl->off_d, sl->off_h, 8 * (V + 1), hipMemcpyHostToDevice, st) != hipSuccess ||
      (!direct && E > 0 && hipMemcpyAsync(sl->adj_d, sl->adj_h, 4 * E, hipMemcpyHostToDevice, st) != hipSuccess))
    return KCORE_EDEVICE;
  int rc = kc::decompose_batched_local(sl->vptr_d, sl->off_d, sl->adj_d, (int32_t)G, V, sl->core_d, st);
  if (rc) return rc;
  if (hipMemcpyAsync(sl->core_h, sl->core_d, 4 * V, hipMemcpyDeviceToHost, st) != hipSuccess)
    return KCORE_EDEVICE;
  auto* pr = new std::pair<kcore_server*, Slot*>(s, sl);
  if (hipLaunchHostFunc(st, host_done, pr) != hipSuccess) {
    delete pr;
    return KCORE_EDEVICE;
  }
  return 0;
}

void finish_slot(kcore_server* s, Slot* sl) {
  // called with s->mu held
  const double t = s->now_us();
  int64_t vb = 0;
  for (Request* r : sl->reqs) {
    if (sl->rc == 0) {
      r->core.assign(sl->core_h + vb, sl->core_h + vb + r->n);
      r->state = RQ_DONE;
    } else {
      r->state = RQ_FAILED;
      r->err = sl->rc;
    }
    vb += r->n;
    r->st.done_us = t;
    std::vector<int64_t>().swap(r->off);
    std::vector<int32_t>().swap(r->adj);
    r->offp = nullptr;
    r->adjp = nullptr;
  }
  s->bytes_in_use -= sl->bytes;
  sl->bytes = 0;
  sl->reqs.clear();
  sl->busy = false;
  sl->finished.store(0);
}

void dispatcher(kcore_server* s) {
  hipSetDevice(s->cfg.device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool progressed = false;
    for (Slot* sl : s->slots)
      if (sl->busy && sl->finished.load()) {
        finish_slot(s, sl);
        progressed = true;
      }
    if (progressed) s->done_cv.notify_all();
    int busy = 0;
    Slot* free_slot = nullptr;
    for (Slot* sl : s->slots) {
      if (sl->busy) ++busy;
      else if (!free_slot) free_slot = sl;
    }
    if (s->stop && busy == 0) break;
    if (!s->stop && free_slot && !s->queue.empty()) {
      // Admit in arrival order, one size class per batch: the class of the oldest request, then
      // every queued request of that class while the budget and batch limits allow. Large
      // batches may not take the last free slot, so small requests always have one.
      int busy_large = 0;
      for (Slot* sl : s->slots)
        if (sl->busy && sl->large) ++busy_large;
      const bool large_ok = s->slots.size() == 1 || busy_large + 1 < (int)s->slots.size();
      const bool large = large_ok && is_large(s->queue.front()->n, s->queue.front()->m);
      int64_t V = 0, bytes = 0;
      std::vector<Request*> take;
      for (auto it = s->queue.begin(); it != s->queue.end();) {
        Request* r = *it;
        if (is_large(r->n, r->m) != large) {
          ++it;
          continue;
        }
        if ((int64_t)take.size() >= s->cfg.max_batch_graphs) break;
        if (!take.empty() && V + r->n > s->cfg.max_batch_vertices) break;
        if (s->bytes_in_use + bytes + r->bytes > s->cfg.hbm_budget_bytes) break;
        it = s->queue.erase(it);
        take.push_back(r);
        V += r->n;
        bytes += r->bytes;
      }
      free_slot->large = large;
      if (!take.empty()) {
        const double t = s->now_us();
        free_slot->busy = true;
        free_slot->reqs = take;
        free_slot->bytes = bytes;
        free_slot->batch_id = s->next_batch++;
        s->bytes_in_use += bytes;
        for (Request* r : take) {
          r->state = RQ_RUNNING;
          r->st.admit_us = t;
          r->st.batch_id = free_slot->batch_id;
          r->st.batch_graphs = (int32_t)take.size();
        }
        lk.unlock();
        const double tl = s->now_us();
        int rc = launch_slot(s, free_slot);
        lk.lock();
        for (Request* r : take) r->st.launch_us = tl;
        if (rc) {
          // the failure belongs to this batch only
          free_slot->rc = rc;
          finish_slot(s, free_slot);
          free_slot->rc = 0;
          s->done_cv.notify_all();
        }
        continue;
      }
    }
    s->cv.wait_for(lk, std::chrono::microseconds(200));
  }
}

}  // namespace

extern "C" {

kcore_server* kcore_server_create(const kcore_server_config* cfg) {
  kc::set_error("");
  kcore_server_config c{};
  if (cfg) c = *cfg;
  if (c.max_inflight < 0 || c.max_batch_graphs < 0 || c.max_batch_vertices < 0 || c.hbm_budget_bytes < 0 ||
      c.max_request_vertices < 0 || c.batch_wait_us < 0) {
    kc::set_error("negative server configuration field");
    return nullptr;
  }
  if (!c.max_inflight) c.max_inflight = 4;
  if (!c.max_batch_graphs) c.max_batch_graphs = 4096;
  if (!c.max_batch_vertices) c.max_batch_vertices = 1 << 24;
  if (!c.hbm_budget_bytes) c.hbm_budget_bytes = 8ll << 30;
  if (!c.batch_wait_us) c.batch_wait_us = 50;
  int ndev = 0;
  (void)hipGetLastError();  // an earlier, unrelated failure must not be reported as ours
  const hipError_t de = hipGetDeviceCount(&ndev);
  if (de != hipSuccess || c.device < 0 || c.device >= ndev) {
    char msg[160];
    snprintf(msg, sizeof msg, "no such HIP device (%d of %d: %s)", c.device, ndev, hipGetErrorString(de));
    kc::set_error(msg);
    return nullptr;
  }
  if (hipSetDevice(c.device) != hipSuccess) {
    kc::set_error("hipSetDevice failed");
    return nullptr;
  }
  auto* s = new kcore_server;
  s->cfg = c;
  s->t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < c.max_inflight; ++i) {
    Slot* sl = new Slot;
    if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess) {
      kc::set_error("stream creation failed");
      delete sl;
      for (Slot* o : s->slots) {
        hipStreamDestroy(o->stream);
        delete o;
      }
      delete s;
      return nullptr;
    }
    s->slots.push_back(sl);
  }
  s->th = std::thread(dispatcher, s);
  return s;
}

int kcore_submit(kcore_server* s, const int64_t* offsets_host, const int32_t* adj_host, int64_t n,
                 uint64_t* ticket_out) {
  if (!s || !ticket_out || n < 0 || (n > 0 && !offsets_host)) return KCORE_EINVAL;
  if (n > 0x7fffffffLL) return KCORE_ETOOBIG;
  const int64_t m = n > 0 ? offsets_host[n] : 0;
  if (m < 0 || (m > 0 && !adj_host) || (n > 0 && offsets_host[0] != 0)) return KCORE_EINVAL;
  if (s->cfg.max_request_vertices && n > s->cfg.max_request_vertices) return KCORE_ETOOBIG;
  const int64_t bytes = footprint(n, m);
  if (bytes > s->cfg.hbm_budget_bytes || n > s->cfg.max_batch_vertices) return KCORE_ETOOBIG;
  auto* r = new Request;
  r->n = n;
  r->m = m;
  r->bytes = bytes;
  if (s->cfg.borrow_inputs) {
    r->offp = offsets_host;
    r->adjp = adj_host;
  } else {
    r->off.assign(offsets_host, offsets_host + n + 1);
    if (m) {
      r->adj.resize((size_t)m);
      par_copy(r->adj.data(), adj_host, sizeof(int32_t) * (size_t)m);
    }
    r->offp = r->off.data();
    r->adjp = r->adj.data();
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    r->st.submit_us = s->now_us();
    if (n == 0) {
      r->state = RQ_DONE;
      r->st.admit_us = r->st.launch_us = r->st.done_us = r->st.submit_us;
    } else {
      s->queue.push_back(r);
    }
    s->all[r->ticket] = r;
    *ticket_out = r->ticket;
  }
  s->cv.notify_all();
  return KCORE_OK;
}

static int take_result(kcore_server* s, Request* r, int32_t* out, kcore_request_stats* st) {
  // called with s->mu held
  int rc = KCORE_OK;
  if (r->state == RQ_CANCELED) rc = KCORE_ECANCELED;
  else if (r->state == RQ_FAILED) rc = r->err ? r->err : KCORE_EDEVICE;
  else if (out && r->n) memcpy(out, r->core.data(), sizeof(int32_t) * r->n);
  if (st) *st = r->st;
  s->all.erase(r->ticket);
  delete r;
  return rc;
}

int kcore_poll(kcore_server* s, uint64_t ticket, int32_t* coreness_host_out, kcore_request_stats* st) {
  if (!s) return KCORE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return KCORE_ENOTFOUND;
  Request* r = it->second;
  if (r->state == RQ_QUEUED || r->state == RQ_RUNNING) return KCORE_PENDING;
  return take_result(s, r, coreness_host_out, st);
}

int kcore_wait(kcore_server* s, uint64_t ticket, int32_t* coreness_host_out, kcore_request_stats* st,
               double timeout_us) {
  if (!s) return KCORE_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  const auto deadline = std::chrono::steady_clock::now() +
                        std::chrono::microseconds((int64_t)(timeout_us > 0 ? timeout_us : 0));
  for (;;) {
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return KCORE_ENOTFOUND;
    Request* r = it->second;
    if (r->state != RQ_QUEUED && r->state != RQ_RUNNING) return take_result(s, r, coreness_host_out, st);
    if (timeout_us > 0 && std::chrono::steady_clock::now() >= deadline) return KCORE_PENDING;
    s->done_cv.wait_for(lk, std::chrono::microseconds(500));
  }
}

int kcore_cancel(kcore_server* s, uint64_t ticket) {
  if (!s) return KCORE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return KCORE_ENOTFOUND;
  Request* r = it->second;
  if (r->state != RQ_QUEUED) return r->state == RQ_RUNNING ? KCORE_PENDING : KCORE_OK;
  for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
    if (*q == r) {
      s->queue.erase(q);
      break;
    }
  r->state = RQ_CANCELED;
  r->st.done_us = s->now_us();
  s->done_cv.notify_all();
  return KCORE_OK;
}

double kcore_server_now_us(const kcore_server* s) { return s ? s->now_us() : 0.0; }

void kcore_server_destroy(kcore_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (Request* r : s->queue) {
      r->state = RQ_CANCELED;
      r->st.done_us = s->now_us();
    }
    s->queue.clear();
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  hipSetDevice(s->cfg.device);
  for (Slot* sl : s->slots) {
    hipStreamSynchronize(sl->stream);
    hipFree(sl->vptr_d);
    hipFree(sl->off_d);
    hipFree(sl->adj_d);
    hipFree(sl->core_d);
    hipHostFree(sl->vptr_h);
    hipHostFree(sl->off_h);
    hipHostFree(sl->adj_h);
    hipHostFree(sl->core_h);
    hipStreamDestroy(sl->stream);
    delete sl;
  }
  for (auto& kv : s->all) delete kv.second;
  delete s;
}

}  // extern "C"
