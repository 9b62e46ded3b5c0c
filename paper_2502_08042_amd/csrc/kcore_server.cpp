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
#include <cstdlib>
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
  bool solo = false;  // retried alone after its batch failed to launch
  int err = 0;
  int64_t bytes = 0;
  kcore_request_stats st{};
};

// request size classes (see size_class)
enum SizeClass { SC_SMALL = 0, SC_MEDIUM = 1, SC_LARGE = 2 };

struct Slot {
  hipStream_t stream = nullptr;
  bool busy = false;
  std::atomic<int> finished{0};
  bool draining = false;   // the completion thread is copying this batch's results out
  bool launching = false;  // the dispatcher is still enqueueing this batch (its requests are its)
  int64_t v_cap = 0, e_cap = 0, g_cap = 0, c_cap = 0;      // device buffers (elements)
  int64_t vh_cap = 0, eh_cap = 0, gh_cap = 0, ch_cap = 0;  // pinned staging buffers
  std::vector<void*> retired_dev, retired_host;             // outgrown, freed at destroy
  unsigned* status_h = nullptr;  // pinned: the batch's device failure bits
  int64_t *vptr_d = nullptr, *off_d = nullptr;
  int32_t *adj_d = nullptr, *core_d = nullptr;
  int64_t *vptr_h = nullptr, *off_h = nullptr;
  int32_t *adj_h = nullptr, *core_h = nullptr;
  std::vector<Request*> reqs;
  int64_t bytes = 0;
  int64_t batch_id = 0;
  int rc = 0;
  bool large = false;
  int cls = SC_SMALL;
};

int64_t footprint(int64_t n, int64_t m) { return 8 * (n + 1) + 4 * m + 16 * n + 64; }

// Size classes, each batched on its own so that a bigger graph never holds up the completion of a
// batch of smaller ones: large (at least large_n vertices or 32 large_n entries; every graph peeled
// by a team of workgroups), medium (more vertices than the batched peel holds in LDS: one
// workgroup with its state in global memory, several times slower per entry) and small.
int size_class(int64_t n, int64_t m, int64_t large_n, int64_t medium_n) {
  if (n >= large_n || m >= 32 * large_n) return SC_LARGE;
  return n > medium_n ? SC_MEDIUM : SC_SMALL;
}

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
  std::condition_variable comp_cv;  // completion-thread wake-ups (a batch finished on the device)
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, Request*> all;
  std::vector<Slot*> slots;
  int64_t bytes_in_use = 0;
  uint64_t next_ticket = 1;
  int64_t next_batch = 1;
  bool stop = false;
  bool log = false;  // KCORE_SERVER_LOG set: one line per batch on stderr
  // workgroups a large batch puts in teams (every graph of it in a team): the team workgroups of all
  // large batches in flight fit in half the device, so every team completes
  int32_t team_wgs = 0;
  int64_t medium_n = 0;  // graphs with more vertices are medium (the batched peel's LDS capacity)
  int medium_slots = 1;  // medium batches in flight at most (half the slots large ones cannot hold)
  std::thread th;       // dispatcher: admission, packing, launches
  std::thread comp_th;  // completion: copies results out of finished slots and frees them
  bool comp_stop = false;

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
  s->comp_cv.notify_all();
}

// Grows a device buffer and, when wanted, its pinned staging twin to hold `need` elements, with
// headroom so that later batches rarely grow them again (freeing device memory waits for the whole
// device). The two grow independently: batches copied from borrowed memory need no staging.
// Outgrown buffers are kept until the server is destroyed instead of being freed on the spot:
// freeing waits for the whole device, and the dispatcher must not stall behind running batches.
template <class T>
int grow_buf(Slot* sl, T*& dev, T*& host, int64_t& dcap, int64_t& hcap, int64_t need, int64_t floor,
             bool want_host) {
  if (need > dcap) {
    const int64_t c = std::max(std::max(need, floor), dcap * 3 / 2);
    if (dev) sl->retired_dev.push_back(dev);
    dev = nullptr;
    dcap = 0;
    if (hipMalloc(&dev, sizeof(T) * (size_t)c) != hipSuccess) return KCORE_ENOMEM;
    dcap = c;
  }
  if (want_host && need > hcap) {
    if (host) sl->retired_host.push_back(host);
    host = nullptr;
    const int64_t c = std::max(std::max(need, floor), hcap * 3 / 2);
    hcap = 0;
    if (hipHostMalloc((void**)&host, sizeof(T) * (size_t)c, hipHostMallocDefault) != hipSuccess)
      return KCORE_ENOMEM;
    hcap = c;
  }
  return 0;
}

// Device and pinned staging buffers of a slot; a batch whose adjacency is copied straight from
// borrowed caller memory needs no pinned adjacency buffer.
int grow(Slot* sl, int64_t V, int64_t E, int64_t G, bool host_adj) {
  int rc = grow_buf(sl, sl->vptr_d, sl->vptr_h, sl->g_cap, sl->gh_cap, G + 1, 4096, true);
  if (!rc) rc = grow_buf(sl, sl->off_d, sl->off_h, sl->v_cap, sl->vh_cap, V + 1, 1 << 20, true);
  if (!rc) rc = grow_buf(sl, sl->adj_d, sl->adj_h, sl->e_cap, sl->eh_cap, E, 16 << 20, host_adj);
  if (!rc) rc = grow_buf(sl, sl->core_d, sl->core_h, sl->c_cap, sl->ch_cap, V, 1 << 20, true);
  return rc;
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
  hipStream_t st = sl->stream;
  // Borrowed large requests are copied to the device straight from the caller's arrays (one DMA
  // each); everything else is packed into the slot's pinned buffer and copied in one piece.
  const bool direct = s->cfg.borrow_inputs && sl->large;
  if (s->cfg.fail_ticket)
    for (const Request* r : sl->reqs)
      if (r->ticket == s->cfg.fail_ticket) return KCORE_EDEVICE;  // injected launch failure
  const double t_start = s->now_us();
  if (int rc = grow(sl, V, E, G, !direct)) return rc;
  const double t_grown = s->now_us();
  std::vector<int64_t> vbs((size_t)G + 1, 0), ebs((size_t)G + 1, 0);
  for (int64_t g = 0; g < G; ++g) {
    vbs[g + 1] = vbs[g] + sl->reqs[g]->n;
    ebs[g + 1] = ebs[g] + sl->reqs[g]->m;
  }
  // Offsets are rebased onto the batch's entry range; adjacency keeps the request's own (local)
  // ids, since the peel is launched in local-id mode. Packing is host memory bandwidth, so the
  // batch is cut into pieces of about 4 MiB (parts of one big request, or runs of small ones) that
  // a few threads take from a shared counter.
  struct Piece {
    int64_t g, v0, v1;  // request and vertex range (offsets); v0 == 0 also copies its adjacency
    int64_t e0, e1;     // adjacency range (entries) copied by this piece
  };
  std::vector<Piece> pieces;
  const int64_t kPiece = 1 << 20;  // elements (4-8 MiB)
  for (int64_t g = 0; g < G; ++g) {
    const Request* r = sl->reqs[g];
    const int64_t nv = r->n, ne = direct ? 0 : r->m;
    const int64_t np = std::max<int64_t>(1, std::max((nv + kPiece - 1) / kPiece, (ne + kPiece - 1) / kPiece));
    for (int64_t q = 0; q < np; ++q)
      pieces.push_back({g, nv * q / np, nv * (q + 1) / np, ne * q / np, ne * (q + 1) / np});
  }
  std::atomic<size_t> next{0};
  auto work = [&] {
    for (size_t i = next.fetch_add(1); i < pieces.size(); i = next.fetch_add(1)) {
      const Piece& pc = pieces[i];
      const Request* r = sl->reqs[pc.g];
      const int64_t vb = vbs[pc.g], eb = ebs[pc.g];
      for (int64_t v = pc.v0; v < pc.v1; ++v) sl->off_h[vb + v] = eb + r->offp[v];
      if (pc.e1 > pc.e0)
        memcpy(sl->adj_h + eb + pc.e0, r->adjp + pc.e0, sizeof(int32_t) * (size_t)(pc.e1 - pc.e0));
      if (pc.v1 == r->n) sl->vptr_h[pc.g + 1] = vbs[pc.g + 1];
    }
  };
  sl->vptr_h[0] = 0;
  const int64_t total_bytes = 8 * V + (direct ? 0 : 4 * E);
  unsigned nt = std::thread::hardware_concurrency();
  nt = nt < 2 ? 2 : (nt > 8 ? 8 : nt);
  if (total_bytes < (4 << 20)) nt = 1;
  {
    std::vector<std::thread> th;
    for (unsigned t = 1; t < nt; ++t) th.emplace_back(work);
    work();
    for (auto& x : th) x.join();
  }
  if (direct) {
    for (int64_t g = 0; g < G; ++g) {
      const Request* r = sl->reqs[g];
      if (r->m && hipMemcpyAsync(sl->adj_d + ebs[g], r->adjp, sizeof(int32_t) * (size_t)r->m,
                                 hipMemcpyHostToDevice, st) != hipSuccess)
        return KCORE_EDEVICE;
    }
  }
  sl->off_h[V] = E;
  const double t_packed = s->now_us();
  if (hipMemcpyAsync(sl->vptr_d, sl->vptr_h, 8 * (G + 1), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(sl->off_d, sl->off_h, 8 * (V + 1), hipMemcpyHostToDevice, st) != hipSuccess ||
      (!direct && E > 0 && hipMemcpyAsync(sl->adj_d, sl->adj_h, 4 * E, hipMemcpyHostToDevice, st) != hipSuccess))
    return KCORE_EDEVICE;
  if (!sl->status_h &&
      hipHostMalloc((void**)&sl->status_h, sizeof(unsigned), hipHostMallocDefault) != hipSuccess)
    return KCORE_ENOMEM;
  *sl->status_h = 0u;
  // a large batch peels each of its graphs with a team of workgroups
  int rc = kc::decompose_batched_local(sl->vptr_d, sl->off_d, sl->adj_d, (int32_t)G, V, sl->core_d, st,
                                       sl->status_h, sl->large ? s->team_wgs : 0);
  if (rc) return rc;
  if (hipMemcpyAsync(sl->core_h, sl->core_d, 4 * V, hipMemcpyDeviceToHost, st) != hipSuccess)
    return KCORE_EDEVICE;
  auto* pr = new std::pair<kcore_server*, Slot*>(s, sl);
  if (hipLaunchHostFunc(st, host_done, pr) != hipSuccess) {
    delete pr;
    return KCORE_EDEVICE;
  }
  if (s->log)
    fprintf(stderr, "[kcore server] batch %lld %s: %lld graphs, %lld vertices, %lld entries; grow %.2f ms, "
            "pack %.2f ms, enqueue %.2f ms\n", (long long)sl->batch_id,
            sl->cls == SC_LARGE ? "large" : sl->cls == SC_MEDIUM ? "medium" : "small",
            (long long)G, (long long)V, (long long)E, (t_grown - t_start) / 1000, (t_packed - t_grown) / 1000,
            (s->now_us() - t_packed) / 1000);
  return 0;
}

// Results of a finished batch into its requests. Runs without s->mu: until finish_slot marks them
// done, the batch's requests and the slot's staging belong to the thread that finishes the slot.
void copy_results(Slot* sl) {
  if (sl->rc == 0 && sl->status_h && *sl->status_h != 0u) sl->rc = KCORE_EDEVICE;
  int64_t vb = 0;
  for (Request* r : sl->reqs) {
    if (sl->rc == 0) r->core.assign(sl->core_h + vb, sl->core_h + vb + r->n);
    vb += r->n;
    std::vector<int64_t>().swap(r->off);
    std::vector<int32_t>().swap(r->adj);
  }
}

void finish_slot(kcore_server* s, Slot* sl) {
  // called with s->mu held, after copy_results
  const double t = s->now_us();
  for (Request* r : sl->reqs) {
    if (sl->rc == 0) {
      r->state = RQ_DONE;
    } else {
      r->state = RQ_FAILED;
      r->err = sl->rc;
    }
    r->st.done_us = t;
    r->offp = nullptr;
    r->adjp = nullptr;
  }
  s->bytes_in_use -= sl->bytes;
  sl->bytes = 0;
  sl->reqs.clear();
  sl->busy = false;
  sl->draining = false;
  sl->rc = 0;
  sl->finished.store(0);
}

// Completion thread: a batch that finished on the device has its results copied out and its slot
// freed here, outside the server lock, so that neither admission nor the runtime's completion
// callbacks wait for the copies of a large batch.
void completer(kcore_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    Slot* sl = nullptr;
    for (Slot* x : s->slots)
      if (x->busy && !x->draining && !x->launching && x->finished.load()) {
        sl = x;
        break;
      }
    if (!sl) {
      if (s->comp_stop) break;
      s->comp_cv.wait_for(lk, std::chrono::microseconds(500));
      continue;
    }
    sl->draining = true;
    lk.unlock();
    copy_results(sl);
    lk.lock();
    finish_slot(s, sl);
    s->done_cv.notify_all();
    s->cv.notify_all();
  }
}

void dispatcher(kcore_server* s) {
  hipSetDevice(s->cfg.device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    int busy = 0;
    Slot* free_slot = nullptr;
    for (Slot* sl : s->slots) {
      if (sl->busy) ++busy;
      else if (!free_slot) free_slot = sl;
    }
    if (s->stop && busy == 0) break;
    if (!s->stop && free_slot && !s->queue.empty() && busy > 0 &&
        (int64_t)s->queue.size() < s->cfg.max_batch_graphs) {
      // the device is busy anyway: give the batch up to batch_wait_us (from its oldest request's
      // arrival) to fill up
      const double age = s->now_us() - s->queue.front()->st.submit_us;
      if (age < s->cfg.batch_wait_us) {
        s->cv.wait_for(lk, std::chrono::microseconds((int64_t)(s->cfg.batch_wait_us - age) + 1));
        continue;
      }
    }
    if (!s->stop && free_slot && !s->queue.empty()) {
      // Admit in arrival order, one size class per batch: the class of the oldest request whose
      // class may take a slot now, then every queued request of that class while the budget and
      // batch limits allow. Large batches hold at most max_large_inflight slots and medium ones at
      // most medium_slots, so small requests always have a slot of their own.
      int busy_cls[3] = {0, 0, 0};
      for (Slot* sl : s->slots)
        if (sl->busy) ++busy_cls[sl->cls];
      const bool one = s->slots.size() == 1;
      const bool ok[3] = {true, one || busy_cls[SC_MEDIUM] < s->medium_slots,
                          one || busy_cls[SC_LARGE] < s->cfg.max_large_inflight};
      int cls = SC_SMALL;
      for (Request* r : s->queue) {
        const int c = size_class(r->n, r->m, s->cfg.large_vertices, s->medium_n);
        if (ok[c]) {
          cls = c;
          break;
        }
      }
      const bool large = cls == SC_LARGE;
      int64_t V = 0, bytes = 0;
      std::vector<Request*> take;
      for (auto it = s->queue.begin(); it != s->queue.end();) {
        Request* r = *it;
        if (size_class(r->n, r->m, s->cfg.large_vertices, s->medium_n) != cls) {
          ++it;
          continue;
        }
        if ((int64_t)take.size() >= s->cfg.max_batch_graphs) break;
        // (a large batch holds at most as many graphs as it has teams)
        if (large && s->team_wgs > 0 && ((int64_t)take.size() + 1) * kc::kTeamSize > s->team_wgs) break;
        if (!take.empty() && (r->solo || take.front()->solo)) break;
        if (!take.empty() && V + r->n > s->cfg.max_batch_vertices) break;
        if (s->bytes_in_use + bytes + r->bytes > s->cfg.hbm_budget_bytes) break;
        it = s->queue.erase(it);
        take.push_back(r);
        V += r->n;
        bytes += r->bytes;
      }
      free_slot->large = large;
      free_slot->cls = cls;
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
        // (the batch may finish on the device before launch_slot returns: the completion thread
        // leaves the slot alone until the dispatcher is done with its requests)
        free_slot->launching = true;
        lk.unlock();
        int rc = launch_slot(s, free_slot);
        const double tl = s->now_us();
        lk.lock();
        for (Request* r : take) r->st.launch_us = tl;
        free_slot->launching = false;
        s->comp_cv.notify_all();
        if (rc) {
          // the failure belongs to this batch only. A batch of several requests is retried one
          // request per batch, at the head of the queue, so that only a failing request fails.
          if (free_slot->reqs.size() > 1) {
            for (auto it = free_slot->reqs.rbegin(); it != free_slot->reqs.rend(); ++it) {
              Request* r = *it;
              r->state = RQ_QUEUED;
              r->solo = true;
              s->queue.push_front(r);
            }
            s->bytes_in_use -= free_slot->bytes;
            free_slot->bytes = 0;
            free_slot->reqs.clear();
            free_slot->busy = false;
          } else {
            free_slot->rc = rc;
            copy_results(free_slot);  // (a failed batch: no results to copy)
            finish_slot(s, free_slot);
            s->done_cv.notify_all();
          }
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
      c.max_request_vertices < 0 || c.batch_wait_us < 0 || c.reserve_vertices < 0 || c.reserve_entries < 0 ||
      c.max_large_inflight < 0 || c.large_vertices < 0) {
    kc::set_error("negative server configuration field");
    return nullptr;
  }
  if (!c.max_inflight) c.max_inflight = 4;
  if (!c.max_batch_graphs) c.max_batch_graphs = 4096;
  if (!c.max_batch_vertices) c.max_batch_vertices = 1 << 24;
  if (!c.hbm_budget_bytes) c.hbm_budget_bytes = 8ll << 30;
  if (!c.batch_wait_us) c.batch_wait_us = 50;
  if (!c.max_large_inflight) c.max_large_inflight = std::max(1, c.max_inflight / 2);
  if (!c.large_vertices) c.large_vertices = 1 << 16;
  if (c.max_inflight > 1 && c.max_large_inflight >= c.max_inflight) c.max_large_inflight = c.max_inflight - 1;
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
  s->log = getenv("KCORE_SERVER_LOG") != nullptr;
  {
    // the team workgroups of all large batches in flight fit in half the device (the other half
    // stays with the small batches); each team completes since nothing it waits for is blocked
    const int res = kc::batched_resident_wgs();
    int tw = res / 2 / c.max_large_inflight / kc::kTeamSize * kc::kTeamSize;
    if (tw > kc::kMaxTeams * kc::kTeamSize) tw = kc::kMaxTeams * kc::kTeamSize;
    s->team_wgs = tw >= kc::kTeamSize ? tw : 0;
    const int64_t lv = kc::batched_lds_vertices();
    s->medium_n = lv > 0 ? lv : INT64_MAX;
    s->medium_slots = std::max(1, (c.max_inflight - c.max_large_inflight) / 2);
    if (s->log)
      fprintf(stderr, "[kcore server] %d slots (large %d, medium %d), %d resident batched workgroups, %d in "
              "teams per large batch, medium above %lld vertices\n", c.max_inflight, c.max_large_inflight,
              s->medium_slots, res, s->team_wgs, (long long)s->medium_n);
  }
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
  if (c.reserve_vertices || c.reserve_entries) {
    for (Slot* sl : s->slots) {
      const int32_t g = c.max_batch_graphs;
      // the batched workspace is sized for the largest batch admission allows
      if (grow(sl, c.reserve_vertices, c.reserve_entries, g, true) ||
          kc::reserve_batched(sl->stream, std::max(c.reserve_vertices, c.max_batch_vertices), g)) {
        kcore_server_destroy(s);
        kc::set_error("could not reserve the slot buffers asked for");
        return nullptr;
      }
    }
  }
  s->th = std::thread(dispatcher, s);
  s->comp_th = std::thread(completer, s);
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

// Hands a finished request's result to the caller. Called with the lock held (lk); the request
// leaves the table first, so the copy runs without the lock (no one else can reach it).
static int take_result(kcore_server* s, Request* r, int32_t* out, kcore_request_stats* st,
                       std::unique_lock<std::mutex>& lk) {
  s->all.erase(r->ticket);
  lk.unlock();
  int rc = KCORE_OK;
  if (r->state == RQ_CANCELED) rc = KCORE_ECANCELED;
  else if (r->state == RQ_FAILED) rc = r->err ? r->err : KCORE_EDEVICE;
  else if (out && r->n) memcpy(out, r->core.data(), sizeof(int32_t) * r->n);
  if (st) *st = r->st;
  delete r;
  return rc;
}

int kcore_poll(kcore_server* s, uint64_t ticket, int32_t* coreness_host_out, kcore_request_stats* st) {
  if (!s) return KCORE_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return KCORE_ENOTFOUND;
  Request* r = it->second;
  if (r->state == RQ_QUEUED || r->state == RQ_RUNNING) return KCORE_PENDING;
  return take_result(s, r, coreness_host_out, st, lk);
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
    if (r->state != RQ_QUEUED && r->state != RQ_RUNNING) return take_result(s, r, coreness_host_out, st, lk);
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
  if (s->th.joinable()) s->th.join();  // (it returns once every slot has been freed)
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->comp_stop = true;
  }
  s->comp_cv.notify_all();
  if (s->comp_th.joinable()) s->comp_th.join();
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
    for (void* p : sl->retired_dev) hipFree(p);
    if (sl->status_h) hipHostFree(sl->status_h);
    for (void* p : sl->retired_host) hipHostFree(p);
    kc::release_batched(sl->stream);
    hipStreamDestroy(sl->stream);
    delete sl;
  }
  for (auto& kv : s->all) delete kv.second;
  delete s;
}

}  // extern "C"
