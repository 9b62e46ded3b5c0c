// C ABI of the k-core library: argument checks, per-(device, stream) workspace cache, launches and
// statistics read-back. Serving lives in kcore_server.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "../../include/kcore.h"
#include "kcore_internal.h"

// Checked builds (a separate library for tests) start every output at -1, so that the kernels can
// verify that each coreness is written exactly once.
#ifndef KCORE_CHECKS
#define KCORE_CHECKS 0
#endif

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(x)                                                                     \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? KCORE_ENOMEM : KCORE_EDEVICE, "%s: %s", #x, \
                  hipGetErrorString(e_));                                              \
  } while (0)

struct DevInfo {
  int cus = 0;
  size_t lds_per_block = 0;
  int peel_bpc = 0;
  int32_t tail_lcap[2] = {0, 0};  // vertices the tail peel's LDS holds: level-sync, chained instance
  size_t batch_lds = 0;           // dynamic LDS per batched workgroup
  int batch_bpc = 0;              // batched workgroups resident per CU with it
};

std::mutex g_mu;
std::map<int, DevInfo> g_dev;

// The peel kernel is a persistent grid that fills the device, and its grid barriers need every one
// of its workgroups resident: two such grids launched from different streams could each hold part
// of the device and wait for the rest forever. So the grids of one device run one after another:
// each launch first waits, in its own stream, for an event recorded after the launch before it
// (stream order only; the host never blocks here).
struct GridOrder {
  hipEvent_t ev = nullptr;
  hipStream_t last = nullptr;
  bool any = false;
};
std::mutex g_grid_mu;
std::map<int, GridOrder> g_grid;

// (also the batched peel when it runs teams: a cooperative grid whose teams wait for each other)
template <class F>
int launch_ordered(int dev, hipStream_t stream, F&& launch) {
  std::lock_guard<std::mutex> lk(g_grid_mu);
  GridOrder& o = g_grid[dev];
  if (!o.ev) HIP_TRY(hipEventCreateWithFlags(&o.ev, hipEventDisableTiming));
  if (o.any && o.last != stream) HIP_TRY(hipStreamWaitEvent(stream, o.ev, 0));
  HIP_TRY(launch());
  HIP_TRY(hipEventRecord(o.ev, stream));
  o.last = stream;
  o.any = true;
  return KCORE_OK;
}

int launch_peel_ordered(int dev, const kc::PeelArgs& a, int blocks, hipStream_t stream) {
  return launch_ordered(dev, stream, [&] { return kc::launch_peel(a, blocks, stream); });
}

int dev_info(int dev, DevInfo& out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_dev.find(dev);
  if (it != g_dev.end()) {
    out = it->second;
    return KCORE_OK;
  }
  DevInfo d;
  HIP_TRY(hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev));
  int lds = 0;
  HIP_TRY(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  d.lds_per_block = (size_t)lds;
  HIP_TRY(kc::peel_occupancy(&d.peel_bpc));
  for (int ch = 0; ch < 2; ++ch) {
    size_t tail_static = 0;
    HIP_TRY(kc::tail_static_lds(ch, &tail_static));
    // 6 bytes per vertex (induced degree and 16-bit queue slot) plus 64 spare slots, in whole
    // 1024-vertex steps, below the 16-bit id limit; the chained instance has almost no static LDS
    // (the level-sync one keeps four 1024-entry scan arrays), so it holds more vertices
    int32_t lc = lds > (int)tail_static + 256 ? (int32_t)(((size_t)lds - tail_static - 256) / 6 / 1024 * 1024) : 0;
    lc = std::min<int32_t>(lc, 64512);
    if (lc > 0) HIP_TRY(kc::tail_allow_lds(ch, lc));
    d.tail_lcap[ch] = lc;
  }
  // batched peel: its registers allow a fixed number of workgroups per CU; give each the most LDS
  // that keeps that number (8 bytes per vertex held in LDS), at least 48 KB when the device has it
  size_t bl = std::min<size_t>(48 * 1024, d.lds_per_block / 2);
  int bb = 0;
  HIP_TRY(kc::batched_occupancy(bl, &bb));
  for (size_t c = d.lds_per_block / 2 / 512 * 512; c > bl; c -= 512) {
    int b2 = 0;
    HIP_TRY(kc::batched_occupancy(c, &b2));
    if (b2 >= bb) {
      bl = c;
      break;
    }
  }
  d.batch_lds = bl;
  d.batch_bpc = bb;
  g_dev[dev] = d;
  out = d;
  return KCORE_OK;
}

// ---- single-graph workspace ---------------------------------------------------------------
struct PeelWs {
  int64_t n_cap = -1, t_cap = -1, r_cap = -1, l_cap = -1, e_cap = -1;
  void* block = nullptr;  // one allocation for everything
  size_t bytes = 0;
  uint32_t* dt = nullptr;
  uint32_t* state = nullptr;
  int32_t* act[2] = {nullptr, nullptr};
  int32_t* fr[2] = {nullptr, nullptr};
  unsigned long long* tl[2] = {nullptr, nullptr};
  long long* aq = nullptr;
  int64_t q_cap = 0;
  long long* rrow = nullptr;
  int32_t* radj = nullptr;
  int32_t* tmap = nullptr;   // tail handoff: id -> local id (n entries)
  int32_t* tgid = nullptr;   //   local id -> id (l_cap)
  long long* trow = nullptr; //   local rows (2 l_cap)
  uint16_t* tadj = nullptr;  //   their entries (e_cap 16-bit local ids)
  // sampling mode (allocated on first use): srate, scnt, sbase, scount (uint32[s_cap] each),
  // scand, srl (int32[s_cap] each)
  void* sblock = nullptr;
  int64_t s_cap = -1;
  uint32_t* srate = nullptr;
  uint32_t* scnt = nullptr;
  uint32_t* sbase = nullptr;
  uint32_t* scount = nullptr;
  int32_t* scand = nullptr;
  int32_t* srl = nullptr;
  // multi-bucket active set (allocated on first use): slots x cap bucket entries, then the
  // per-vertex tags
  void* hblock = nullptr;
  size_t h_bytes = 0;
  int32_t* hbl = nullptr;
  uint32_t* hlo = nullptr;
  kc::PeelCtl* ctl = nullptr;
  unsigned long long* host_stats = nullptr;  // pinned
  unsigned* vstat = nullptr;                 // validation status + xor sum (device)
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

struct BatchWs {
  int64_t v_cap = -1;
  int32_t g_cap = -1;
  void* block = nullptr;
  uint32_t* gdt = nullptr;
  int32_t* gq = nullptr;
  int32_t* ga = nullptr;
  int32_t* order = nullptr;
  kc::BatchCtl* ctl = nullptr;
  unsigned long long* host_stats = nullptr;
  unsigned* vstat = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

using Key = std::pair<int, hipStream_t>;
std::map<Key, PeelWs*> g_peel;
std::map<Key, BatchWs*> g_batch;

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

int peel_ws(int dev, hipStream_t s, int64_t n, int64_t tcap, int64_t rcap, int64_t lcap, int64_t ecap,
            PeelWs*& out) {
  std::lock_guard<std::mutex> lk(g_mu);
  PeelWs*& w = g_peel[Key(dev, s)];
  if (!w) {
    w = new PeelWs;
    HIP_TRY(hipHostMalloc((void**)&w->host_stats, kc::kStatWords * sizeof(unsigned long long) + 64,
                          hipHostMallocDefault));
    HIP_TRY(hipEventCreate(&w->ev0));
    HIP_TRY(hipEventCreate(&w->ev1));
  }
  if (w->n_cap < n || w->t_cap < tcap || w->r_cap < rcap || w->l_cap < lcap || w->e_cap < ecap) {
    if (w->block) {
      HIP_TRY(hipStreamSynchronize(s));
      HIP_TRY(hipFree(w->block));
      w->block = nullptr;
    }
    const int64_t nc = n > w->n_cap ? n + n / 8 : w->n_cap;
    const int64_t tc = tcap > w->t_cap ? tcap + tcap / 8 + 64 : w->t_cap;
    const int64_t rc = rcap > w->r_cap ? rcap : std::max<int64_t>(w->r_cap, 0);
    const int64_t lc = std::max<int64_t>(lcap, std::max<int64_t>(w->l_cap, 0));
    const int64_t ec = std::max<int64_t>(ecap, std::max<int64_t>(w->e_cap, 0));
    const size_t nw = (size_t)((nc + 15) / 16);
    size_t off = 0;
    const size_t o_dt = off; off = align_up(off + 4 * (size_t)nc);
    const size_t o_st = off; off = align_up(off + 4 * nw);
    // active lists are written in per-workgroup segments: room for one 64-entry round-up each
    const size_t na = (size_t)nc + 64 * (size_t)kc::kMaxPeelBlocks;
    const size_t o_a0 = off; off = align_up(off + 4 * na);
    const size_t o_a1 = off; off = align_up(off + 4 * na);
    const size_t o_f0 = off; off = align_up(off + 4 * (size_t)nc);
    const size_t o_f1 = off; off = align_up(off + 4 * (size_t)nc);
    const size_t o_t0 = off; off = align_up(off + 8 * (size_t)tc);
    const size_t o_t1 = off; off = align_up(off + 8 * (size_t)tc);
    const int64_t qc = nc + tc + 256 * 64 * 64;  // entries of one phase + one claim per wave
    const size_t o_q = off; off = align_up(off + 8 * (size_t)qc);
    const size_t o_rr = off; off = align_up(off + (rc > 0 ? 16 * (size_t)nc : 0));
    const size_t o_ra = off; off = align_up(off + 4 * (size_t)rc);
    const size_t o_tm = off; off = align_up(off + (lc > 0 ? 4 * (size_t)nc : 0));
    const size_t o_tg = off; off = align_up(off + 4 * (size_t)lc);
    const size_t o_tr = off; off = align_up(off + 16 * (size_t)lc);
    const size_t o_te = off; off = align_up(off + 2 * (size_t)ec);
    const size_t o_c = off; off = align_up(off + sizeof(kc::PeelCtl));
    const size_t o_v = off; off = align_up(off + 64);
    hipError_t e = hipMalloc(&w->block, off);
    if (e != hipSuccess) {
      w->block = nullptr;
      w->n_cap = w->t_cap = w->r_cap = w->l_cap = w->e_cap = -1;
      return fail(KCORE_ENOMEM, "workspace of %zu bytes: %s", off, hipGetErrorString(e));
    }
    char* b = static_cast<char*>(w->block);
    w->bytes = off;
    w->dt = (uint32_t*)(b + o_dt);
    w->state = (uint32_t*)(b + o_st);
    w->act[0] = (int32_t*)(b + o_a0);
    w->act[1] = (int32_t*)(b + o_a1);
    w->fr[0] = (int32_t*)(b + o_f0);
    w->fr[1] = (int32_t*)(b + o_f1);
    w->tl[0] = (unsigned long long*)(b + o_t0);
    w->tl[1] = (unsigned long long*)(b + o_t1);
    w->aq = (long long*)(b + o_q);
    w->q_cap = qc;
    w->rrow = rc > 0 ? (long long*)(b + o_rr) : nullptr;
    w->radj = rc > 0 ? (int32_t*)(b + o_ra) : nullptr;
    w->r_cap = rc;
    w->tmap = lc > 0 ? (int32_t*)(b + o_tm) : nullptr;
    w->tgid = lc > 0 ? (int32_t*)(b + o_tg) : nullptr;
    w->trow = lc > 0 ? (long long*)(b + o_tr) : nullptr;
    w->tadj = lc > 0 ? (uint16_t*)(b + o_te) : nullptr;
    w->l_cap = lc;
    w->e_cap = ec;
    w->ctl = (kc::PeelCtl*)(b + o_c);
    w->vstat = (unsigned*)(b + o_v);
    w->n_cap = nc;
    w->t_cap = tc;
  }
  out = w;
  return KCORE_OK;
}

// Sampling-mode arrays of a single-graph workspace, grown to n vertices.
int sample_ws(PeelWs* w, hipStream_t s, int64_t n) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (w->s_cap >= n) return KCORE_OK;
  if (w->sblock) {
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipFree(w->sblock));
    w->sblock = nullptr;
    w->s_cap = -1;
  }
  const size_t each = align_up(4 * (size_t)n);
  hipError_t e = hipMalloc(&w->sblock, 6 * each);
  if (e != hipSuccess) {
    w->sblock = nullptr;
    return fail(KCORE_ENOMEM, "sampling workspace of %zu bytes: %s", 6 * each, hipGetErrorString(e));
  }
  char* b = static_cast<char*>(w->sblock);
  w->srate = (uint32_t*)b;
  w->scnt = (uint32_t*)(b + each);
  w->sbase = (uint32_t*)(b + 2 * each);
  w->scount = (uint32_t*)(b + 3 * each);
  w->scand = (int32_t*)(b + 4 * each);
  w->srl = (int32_t*)(b + 5 * each);
  w->s_cap = n;
  return KCORE_OK;
}

// Multi-bucket arrays of a single-graph workspace: slots x cap entries and n tags.
int bucket_ws(PeelWs* w, hipStream_t s, int64_t n, int32_t slots, int64_t cap) {
  std::lock_guard<std::mutex> lk(g_mu);
  const size_t lists = align_up(4 * (size_t)slots * (size_t)cap);
  const size_t need = lists + align_up(4 * (size_t)n);
  if (w->hblock && w->h_bytes >= need) {
    w->hbl = static_cast<int32_t*>(w->hblock);
    w->hlo = reinterpret_cast<uint32_t*>(static_cast<char*>(w->hblock) + lists);
    return KCORE_OK;
  }
  if (w->hblock) {
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipFree(w->hblock));
    w->hblock = nullptr;
    w->h_bytes = 0;
  }
  hipError_t e = hipMalloc(&w->hblock, need);
  if (e != hipSuccess) {
    w->hblock = nullptr;
    return fail(KCORE_ENOMEM, "bucket workspace of %zu bytes: %s", need, hipGetErrorString(e));
  }
  w->h_bytes = need;
  w->hbl = static_cast<int32_t*>(w->hblock);
  w->hlo = reinterpret_cast<uint32_t*>(static_cast<char*>(w->hblock) + lists);
  return KCORE_OK;
}

int batch_ws(int dev, hipStream_t s, int64_t V, int32_t G, BatchWs*& out) {
  std::lock_guard<std::mutex> lk(g_mu);
  BatchWs*& w = g_batch[Key(dev, s)];
  if (!w) {
    w = new BatchWs;
    HIP_TRY(hipHostMalloc((void**)&w->host_stats, kc::kStatWords * sizeof(unsigned long long) + 64,
                          hipHostMallocDefault));
    HIP_TRY(hipEventCreate(&w->ev0));
    HIP_TRY(hipEventCreate(&w->ev1));
  }
  if (w->v_cap < V || w->g_cap < G) {
    if (w->block) {
      HIP_TRY(hipStreamSynchronize(s));
      HIP_TRY(hipFree(w->block));
      w->block = nullptr;
    }
    // headroom: regrowing waits for the stream and frees device memory (a device-wide wait)
    const int64_t vc = V > w->v_cap ? std::max<int64_t>(V, w->v_cap * 3 / 2) : w->v_cap;
    const int64_t gc = G > w->g_cap ? std::max<int64_t>((int64_t)G + 16, (int64_t)w->g_cap * 3 / 2) : w->g_cap;
    size_t off = 0;
    const size_t o_d = off; off = align_up(off + 4 * (size_t)vc);
    const size_t o_q = off; off = align_up(off + 4 * (size_t)vc);
    const size_t o_a = off; off = align_up(off + 4 * (size_t)vc);
    const size_t o_o = off; off = align_up(off + 4 * (size_t)gc);
    const size_t o_c = off; off = align_up(off + sizeof(kc::BatchCtl));
    const size_t o_v = off; off = align_up(off + 64);
    hipError_t e = hipMalloc(&w->block, off);
    if (e != hipSuccess) {
      w->block = nullptr;
      w->v_cap = -1;
      w->g_cap = -1;
      return fail(KCORE_ENOMEM, "batched workspace of %zu bytes: %s", off, hipGetErrorString(e));
    }
    char* b = static_cast<char*>(w->block);
    w->gdt = (uint32_t*)(b + o_d);
    w->gq = (int32_t*)(b + o_q);
    w->ga = (int32_t*)(b + o_a);
    w->order = (int32_t*)(b + o_o);
    w->ctl = (kc::BatchCtl*)(b + o_c);
    w->vstat = (unsigned*)(b + o_v);
    w->v_cap = vc;
    w->g_cap = (int32_t)gc;
  }
  out = w;
  return KCORE_OK;
}

// Entries the CSR of an n-vertex graph can hold when the caller did not say: what is left of the
// device allocation holding adj after adj (the runtime's record of its base and size; no device
// work), capped at n (n - 1). Only a pointer the runtime cannot attribute falls back to reading
// offsets[n] from the device, which blocks.
int entries_bound(const int64_t* offsets, const int32_t* adj, int64_t n, hipStream_t stream, int64_t& m) {
  const int64_t simple = n > 3037000499LL ? INT64_MAX : n * (n - 1);
  if (!adj) {
    m = 0;
    return KCORE_OK;
  }
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<int32_t*>(adj)) == hipSuccess && base && size) {
    const char* b = static_cast<const char*>(base);
    const char* p = reinterpret_cast<const char*>(adj);
    if (p >= b && p < b + size) {
      m = std::min<int64_t>((int64_t)((b + size - p) / sizeof(int32_t)), simple);
      return KCORE_OK;
    }
  }
  (void)hipGetLastError();  // (the failed lookup must not surface in a later call)
  int64_t* pin = nullptr;
  HIP_TRY(hipHostMalloc((void**)&pin, sizeof(int64_t), hipHostMallocDefault));
  hipError_t e1 = hipMemcpyAsync(pin, offsets + n, sizeof(int64_t), hipMemcpyDefault, stream);
  hipError_t e2 = e1 == hipSuccess ? hipStreamSynchronize(stream) : e1;
  m = *pin;
  hipHostFree(pin);
  if (e2 != hipSuccess) return fail(KCORE_EDEVICE, "reading offsets[n]: %s", hipGetErrorString(e2));
  return KCORE_OK;
}

int check_opts(const kcore_options* o) {
  if (!o) return KCORE_OK;
  if (o->mode < 0 || o->mode > 4) return fail(KCORE_EINVAL, "mode %d unknown", o->mode);
  if (o->blocks_per_cu < 0 || o->hub_degree < 0 || o->num_entries < 0 || o->local_budget < 0 ||
      o->tile_edges < 0 || (o->tile_edges % 64) != 0 || o->tile_edges > 32768)
    return fail(KCORE_EINVAL, "negative option, or tile_edges not a multiple of 64 up to 32768");
  if (o->tail < -1) return fail(KCORE_EINVAL, "tail must be >= -1");
  if (o->tile_probe < -1 || o->tile_probe > 0) return fail(KCORE_EINVAL, "tile_probe must be 0 or -1");
  if (o->residual < -1) return fail(KCORE_EINVAL, "residual must be >= -1");
  if (o->block_queue < 0 || o->block_queue > kc::kBlockQ)
    return fail(KCORE_EINVAL, "block_queue must be in [0, %d]", kc::kBlockQ);
  if (o->async_frontier < -1 || o->async_scan < -1 || o->block_tiles < -1)
    return fail(KCORE_EINVAL, "async and block-tile thresholds must be >= -1");
  if (o->buckets < -1) return fail(KCORE_EINVAL, "buckets must be >= -1");
  if (o->batch_teams < -1) return fail(KCORE_EINVAL, "batch_teams must be >= -1");
  if (o->combine_degree < 0 || o->big_phase < 0) return fail(KCORE_EINVAL, "combine_degree and big_phase must be >= 0");
  if (o->team_size < 0 || o->team_size > kc::kMaxTeamSize)
    return fail(KCORE_EINVAL, "team_size must be in [0, %d]", kc::kMaxTeamSize);
  if (o->sample_threshold < 0 || o->sample_mu < 0 || o->debug_phase < 0 || o->test_tail_entries < 0)
    return fail(KCORE_EINVAL, "sampling parameters and test hooks must be >= 0");
  return KCORE_OK;
}

int run_validate(const int64_t* off, const int32_t* adj, int64_t n, const int64_t* vptr, int32_t G,
                 unsigned* vstat, hipStream_t s) {
  HIP_TRY(kc::launch_fill_u32(vstat, 0u, 16, s));
  HIP_TRY(kc::launch_validate(off, adj, n, vptr, G, vstat,
                              reinterpret_cast<unsigned long long*>(vstat + 2), s));
  unsigned h[4] = {0, 0, 0, 0};
  HIP_TRY(hipMemcpyAsync(h, vstat, sizeof h, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h[0] != 0u) return fail(KCORE_EBADGRAPH, "CSR breaks the input contract (offsets, ids or self-loops)");
  if (h[2] != 0u || h[3] != 0u) return fail(KCORE_EBADGRAPH, "CSR is not symmetric");
  return KCORE_OK;
}

void fill_stats(kcore_stats* st, const unsigned long long* hs, unsigned status, float ms) {
  memset(st, 0, sizeof *st);
  st->rounds = (int64_t)hs[kc::ST_ROUNDS];
  st->subrounds = (int64_t)hs[kc::ST_SUBROUNDS];
  st->barriers = (int64_t)hs[kc::ST_BARRIERS];
  st->peeled = (int64_t)hs[kc::ST_PEELED];
  st->edges = (int64_t)hs[kc::ST_EDGES];
  st->decrements = (int64_t)hs[kc::ST_DECR];
  st->combined = (int64_t)hs[kc::ST_COMBINED];
  st->scanned = (int64_t)hs[kc::ST_SCANNED];
  st->kmax = (int32_t)hs[kc::ST_KMAX];
  st->tail_vertices = (int32_t)hs[kc::ST_TAIL];
  st->sampled_vertices = (int32_t)hs[kc::ST_SAMPLED];
  st->sample_recounts = (int32_t)hs[kc::ST_RECOUNTS];
  st->live_decrements = (int64_t)hs[kc::ST_LIVE];
  st->bucket_inserts = (int64_t)hs[kc::ST_BUCKET];
  st->device_status = (int32_t)status;
  st->ms = ms;
}

}  // namespace

void kc::set_error(const char* msg) { g_err = msg ? msg : ""; }

extern "C" {

int kcore_version(void) { return 10200; }

const char* kcore_last_error(void) { return g_err.c_str(); }

// Single graph: the full decomposition (k_query < 0), or the k-core membership for k = k_query >= 1
// (one peeling round at threshold k - 1; out[v] = 1 for the survivors, 0 otherwise).
static int peel_impl(const int64_t* offsets, const int32_t* adj, int64_t n, int32_t* coreness_out,
                     hipStream_t stream, const kcore_options* opt, kcore_stats* stats_host, int64_t k_query) {
  g_err.clear();
  if (n < 0) return fail(KCORE_EINVAL, "n = %lld is negative", (long long)n);
  if (n > 0x7fffffffLL) return fail(KCORE_EINVAL, "n = %lld exceeds the int32 id range", (long long)n);
  if (int rc = check_opts(opt)) return rc;
  if (n == 0) {
    if (stats_host) memset(stats_host, 0, sizeof *stats_host);
    return KCORE_OK;
  }
  if (!offsets || !coreness_out) return fail(KCORE_EINVAL, "null pointer argument");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  DevInfo di;
  if (int rc = dev_info(dev, di)) return rc;

  const int mode = (opt && opt->mode) ? opt->mode : KCORE_MODE_CHAINED;
  const bool sampling = mode == KCORE_MODE_SAMPLING;
  const bool offline = mode == KCORE_MODE_OFFLINE;
  if (sampling && k_query > 0) return fail(KCORE_EINVAL, "the k-core query has no sampling mode");
  if (sampling && n > (1ll << 30))
    return fail(KCORE_EINVAL, "sampling mode takes at most 2^30 vertices (n = %lld)", (long long)n);
  const uint32_t hub = (opt && opt->hub_degree) ? (uint32_t)opt->hub_degree : 256u;
  const int tile = (opt && opt->tile_edges) ? opt->tile_edges : 256;
  // (1,024: a wave hands its queue on to the others after that many; on the road grid, whose time
  // is one asynchronous phase of chains, 25.1 ms against 26.8 ms at 4,096 and 30.4 ms at 256; no
  // change on Chung-Lu or RMAT-16)
  const int budget = (opt && opt->local_budget) ? opt->local_budget : 1024;
  // m: the number of entries the workspace is sized for. The caller's num_entries when given;
  // otherwise the room left in the device allocation that holds adj (no host-device round trip),
  // at most n (n - 1), which a simple graph never exceeds. The kernel checks offsets[n] <= m.
  int64_t m = opt ? opt->num_entries : 0;
  if (m <= 0) {
    if (int rc = entries_bound(offsets, adj, n, stream, m)) return rc;
  }
  if (m < 0) return fail(KCORE_EINVAL, "offsets[n] = %lld is negative", (long long)m);
  if (m > 0 && !adj) return fail(KCORE_EINVAL, "adj is null but the graph has %lld entries", (long long)m);
  // hub tiles address entries with 48 bits
  if (m >= (1ll << 47)) return fail(KCORE_ETOOBIG, "%lld entries exceed the 2^47 limit", (long long)m);
  // tiles pushed over the whole run: sum over hubs of ceil(deg / tile) <= m / tile + #hubs,
  // #hubs <= min(n, m / hub)
  const int64_t hubs = std::min<int64_t>(n, m / (int64_t)hub + 1);
  const int64_t tcap = m / tile + hubs + 64;

  // residual rows (rewritten without peeled neighbours once the active set is small): room for
  // half the adjacency; the rewrite happens only if the live rows fit
  const int32_t ro = opt ? opt->residual : 0;
  // (sampling mode keeps the original rows: its recounts and its biased induced degrees assume them)
  const int64_t resid_vmax = (ro < 0 || sampling) ? -1 : (ro ? ro : std::max<int64_t>(n / 256, 4096));
  const int64_t rcap = resid_vmax < 0 ? 0 : m / 2 + 64;

  // tail handoff: the last live vertices (at most what the tail peel's LDS holds) are peeled by
  // one workgroup; their local rows hold at most min(m, L (L - 1)) entries (simple graph)
  const int32_t to = opt ? opt->tail : 0;
  const int tail_ch = (mode == KCORE_MODE_CHAINED || sampling) ? 1 : 0;  // which tail instance runs
  // (default n / 8: one workgroup streams the rows of what it takes over from one CU, which pays on
  // a large graph's last few thousand rounds but not when the tail would hold much of the graph)
  int64_t tail_vmax = (to < 0 || k_query > 0 || sampling)
                          ? 0
                          : std::min<int64_t>(to ? to : std::max<int64_t>(n / 8, 1), di.tail_lcap[tail_ch]);
  // (local ids are 16-bit: at most 65,535 vertices, 0xffff pads the rows)
  tail_vmax = std::min<int64_t>(std::min<int64_t>(tail_vmax, n), 65535);
  // (plus up to 7 pad entries per row: rows start on 16-byte boundaries)
  const int64_t tail_ecap =
      tail_vmax > 0 ? std::min<int64_t>(m, tail_vmax * (tail_vmax - 1)) + 7 * tail_vmax + 64 : 0;

  PeelWs* w = nullptr;
  if (int rc = peel_ws(dev, stream, n, tcap, rcap, tail_vmax, tail_ecap, w)) return rc;
  if (opt && opt->validate) {
    if (int rc = run_validate(offsets, adj, n, nullptr, 0, w->vstat, stream)) return rc;
  }

  int bpc = (opt && opt->blocks_per_cu) ? opt->blocks_per_cu : di.peel_bpc;
  if (bpc > di.peel_bpc) bpc = di.peel_bpc;
  if (bpc < 1) return fail(KCORE_EDEVICE, "peel kernel cannot be resident on this device");
  int blocks = bpc * di.cus;
  // no more workgroups than there are vertex packets to keep barriers cheap on small graphs
  const int64_t want = (n + 64 * kc::kWaves - 1) / (64 * kc::kWaves);
  if (want < blocks) blocks = (int)std::max<int64_t>(want, 1);
  if (blocks > kc::kMaxPeelBlocks) blocks = kc::kMaxPeelBlocks;

  kc::PeelArgs a;
  a.off = offsets;
  a.adj = adj;
  a.n = n;
  a.m_bound = m;
  a.core = coreness_out;
  a.dt = w->dt;
  a.state = w->state;
  a.act[0] = w->act[0];
  a.act[1] = w->act[1];
  a.fr[0] = w->fr[0];
  a.fr[1] = w->fr[1];
  a.tl[0] = w->tl[0];
  a.tl[1] = w->tl[1];
  a.fcap = w->n_cap;
  a.tcap = w->t_cap;
  a.ctl = w->ctl;
  a.hub = hub;
  // offline mode: every target is combined (Alg. 2's histogram, per workgroup), in every phase
  a.comb_degree = offline ? 0u
                          : (opt && opt->combine_degree) ? (uint32_t)opt->combine_degree : (hub > 1024u ? hub : 1024u);
  a.tile = tile;
  a.chained = (mode == KCORE_MODE_CHAINED || sampling) ? 1 : 0;
  a.lq_budget = budget;
  a.big_phase = offline ? 0 : ((opt && opt->big_phase) ? opt->big_phase : 16384);
  a.aq = w->aq;
  // this call's share of the work queue (the cached workspace may be larger)
  a.qcap = std::min<int64_t>(w->q_cap, n + tcap + 256 * 64 * 64);
  const int32_t af = opt ? opt->async_frontier : 0;
  const int32_t as = opt ? opt->async_scan : 0;
  a.async_small = af < 0 ? -1 : (af ? af : 65536);
  // hub tiles are better spread over every wave by a barrier-separated phase than claimed one
  // by one from the shared queue: frontiers with more than a few tiles stay synchronous
  a.async_tiles = af < 0 ? -1 : 64;
  a.async_scan_max = as < 0 ? -1 : (as ? as : 0);
  const int32_t bt = opt ? opt->block_tiles : 0;
  a.bq_max_tiles = bt < 0 ? 0 : (bt ? bt : 32);
  a.bq_backlog = (opt && opt->block_queue) ? opt->block_queue : 64;
  a.tile_probe_always = !(opt && opt->tile_probe < 0);
  a.k_query = k_query;
  a.rrow = w->rrow;
  a.radj = w->radj;
  a.rcap = rcap;
  a.resid_vmax = w->rrow ? resid_vmax : -1;
  a.tail_vmax = tail_vmax > 0 ? tail_vmax : -1;
  a.tmap = w->tmap;
  a.tgid = w->tgid;
  a.trow = w->trow;
  a.tadj = w->tadj;
  a.tail_ecap = tail_ecap;
  // testing aid: pretend the local rows hold fewer entries, so that handoffs are called off
  if (opt && opt->test_tail_entries > 0) a.tail_ecap = std::min<int64_t>(tail_ecap, opt->test_tail_entries);
  // multi-bucket active set (Sec. 5.2): once at most hbs_vmax vertices are live (k >= 16); each
  // slot holds up to twice that many entries (a vertex enters a slot's range once; a scan that
  // races with a decrement can list it a second time), values below 2^hslots (degrees < n)
  a.hbl = nullptr;
  a.hlo = nullptr;
  a.hcap = 0;
  a.hslots = 0;
  a.hbs_vmax = -1;
  const int32_t bo = opt ? opt->buckets : 0;
  if (bo > 0 && !sampling && k_query <= 0) {
    const int64_t vmax = std::min<int64_t>(bo, n);
    int32_t slots = 1;
    while (slots < 31 && ((int64_t)1 << slots) <= n - 1) ++slots;
    const int64_t cap = 2 * vmax + 1024;
    if (int rc = bucket_ws(w, stream, n, slots, cap)) return rc;
    a.hbl = w->hbl;
    a.hlo = w->hlo;
    a.hcap = cap;
    a.hslots = slots;
    a.hbs_vmax = vmax;
  }
  a.sampling = sampling ? 1 : 0;
  a.s_threshold = a.s_mu = a.s_seed = 0;
  a.srate = a.scnt = a.sbase = a.scount = nullptr;
  a.scand = a.srl = nullptr;
  if (sampling) {
    if (int rc = sample_ws(w, stream, n)) return rc;
    a.srate = w->srate;
    a.scnt = w->scnt;
    a.sbase = w->sbase;
    a.scount = w->scount;
    a.scand = w->scand;
    a.srl = w->srl;
    // Alg. 5's parameters: mu = 4 (c + 2) ln n with c = 1, so that the scheme is correct with
    // probability at least 1 - 1/n (a failure is detected and answered by a second run), at least
    // 16; vertices of degree above 1024 start in sample mode (both can be set in the options)
    a.s_mu = (uint32_t)std::max(16.0, std::ceil(12.0 * std::log((double)std::max<int64_t>(n, 2))));
    a.s_threshold = 1024;
    if (opt && opt->sample_mu > 0) a.s_mu = (uint32_t)opt->sample_mu;
    if (opt && opt->sample_threshold > 0) a.s_threshold = (uint32_t)opt->sample_threshold;
    a.s_seed = 0x2545f491u;
  }
  // debugging aid: record every workgroup's timing in phases [p, p + 64)
  a.dbg_lo = (opt && opt->debug_phase > 0) ? opt->debug_phase : -(1ll << 40);

  HIP_TRY(kc::launch_init_ctl(w->ctl, stream));
  if (a.chained) HIP_TRY(kc::launch_fill_u32(w->aq, 0xffffffffu, 2 * (size_t)a.qcap, stream));
  if (KCORE_CHECKS && k_query <= 0) HIP_TRY(kc::launch_fill_u32(coreness_out, 0xffffffffu, (size_t)n, stream));
  // sampling mode reads its outcome back before returning (a failed sampling run is repeated)
  kcore_stats local_stats;
  if (sampling && !stats_host) stats_host = &local_stats;
  if (stats_host) HIP_TRY(hipEventRecord(w->ev0, stream));
  if (int rc = launch_peel_ordered(dev, a, blocks, stream)) return rc;
  if (tail_vmax > 0) HIP_TRY(kc::launch_tail(a, (int32_t)tail_vmax, stream));
  if (opt && opt->status_out)
    HIP_TRY(hipMemcpyAsync(opt->status_out, &w->ctl->status, sizeof(unsigned), hipMemcpyDefault, stream));
  if (!stats_host) return KCORE_OK;
  HIP_TRY(hipEventRecord(w->ev1, stream));
  // (after the timed region: live decrements from the finished coreness)
  if (k_query <= 0) HIP_TRY(kc::launch_live_count(offsets, coreness_out, n, &w->ctl->stats[kc::ST_LIVE], stream));
  HIP_TRY(hipMemcpyAsync(w->host_stats, w->ctl->stats, kc::kStatWords * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, stream));
  unsigned status = 0;
  HIP_TRY(hipMemcpyAsync(w->host_stats + kc::kStatWords, &w->ctl->status, sizeof(unsigned),
                         hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  memcpy(&status, w->host_stats + kc::kStatWords, sizeof status);
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, w->ev0, w->ev1));
  fill_stats(stats_host, w->host_stats, status, ms);
  if (sampling && status == kc::KC_ERR_SAMPLE) {
    // a sampled vertex was caught below k at a round boundary: the result of this run is void;
    // peel again without sampling (the scheme's answer to its rare failure, so it stays exact)
    const kcore_stats first = *stats_host;
    kcore_options o2;
    memset(&o2, 0, sizeof o2);
    if (opt) o2 = *opt;
    o2.mode = KCORE_MODE_CHAINED;
    o2.num_entries = m;
    const int rc = peel_impl(offsets, adj, n, coreness_out, stream, &o2, stats_host, k_query);
    stats_host->sampled_vertices = first.sampled_vertices;
    stats_host->sample_recounts = first.sample_recounts;
    stats_host->sample_restarts = 1;
    stats_host->ms += first.ms;
    return rc;
  }
  if (status)
    return fail(KCORE_EDEVICE, "device reported failure bits 0x%x (diag %llu %llu %llu %llu)", status,
                w->host_stats[kc::kDiagWord], w->host_stats[kc::kDiagWord + 1],
                w->host_stats[kc::kDiagWord + 2], w->host_stats[kc::kDiagWord + 3]);
  return KCORE_OK;
}

// Debugging aid, not part of kcore.h: copies the phase timeline of the last single-graph call on
// `stream` (rows of eight: start, work done, flushed, barrier passed in 100 MHz ticks, then the
// phase kind word, frontier vertices, hub tiles and active-set size; from row 8192 on, one row per
// round of the tail kernel: start, first frontier extracted, round peeled, -, k, first frontier
// size, vertices peeled so far). Synchronises.
int kcore_debug_trace(hipStream_t stream, unsigned long long* out, int max_phases) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  PeelWs* w = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_peel.find(Key(dev, stream));
    if (it == g_peel.end() || !it->second || !it->second->ctl) return fail(KCORE_ENOTFOUND, "no workspace");
    w = it->second;
  }
  const int np = max_phases < kc::kTracePhases ? max_phases : kc::kTracePhases;
  HIP_TRY(hipStreamSynchronize(stream));
  HIP_TRY(hipMemcpy(out, w->ctl->trace, sizeof(unsigned long long) * 8 * np, hipMemcpyDeviceToHost));
  return KCORE_OK;
}

// Debugging aid, not part of kcore.h: copies the per-workgroup record (kDbgPhases x kDbgBlocks
// rows of start, work done, workgroup-queue tiles, local-queue vertices) of the last single-graph
// call on `stream`. Synchronises.
int kcore_debug_blocks(hipStream_t stream, unsigned long long* out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  PeelWs* w = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_peel.find(Key(dev, stream));
    if (it == g_peel.end() || !it->second || !it->second->ctl) return fail(KCORE_ENOTFOUND, "no workspace");
    w = it->second;
  }
  HIP_TRY(hipStreamSynchronize(stream));
  HIP_TRY(hipMemcpy(out, w->ctl->dbg, sizeof(w->ctl->dbg), hipMemcpyDeviceToHost));
  return KCORE_OK;
}

int kcore_decompose_ex(const int64_t* offsets, const int32_t* adj, int64_t n, int32_t* coreness_out,
                       hipStream_t stream, const kcore_options* opt, kcore_stats* stats_host) {
  return peel_impl(offsets, adj, n, coreness_out, stream, opt, stats_host, -1);
}

int kcore_kcore_subgraph(const int64_t* offsets, const int32_t* adj, int64_t n, int32_t k, int32_t* in_core_out,
                         hipStream_t stream, const kcore_options* opt, kcore_stats* stats_host) {
  if (k <= 0 && n > 0) {
    // every vertex belongs to the 0-core
    g_err.clear();
    if (n > 0x7fffffffLL) return fail(KCORE_EINVAL, "n = %lld exceeds the int32 id range", (long long)n);
    if (int rc = check_opts(opt)) return rc;
    if (!in_core_out) return fail(KCORE_EINVAL, "null pointer argument");
    HIP_TRY(kc::launch_fill_u32(in_core_out, 1u, (size_t)n, stream));
    if (stats_host) {
      HIP_TRY(hipStreamSynchronize(stream));
      memset(stats_host, 0, sizeof *stats_host);
    }
    return KCORE_OK;
  }
  return peel_impl(offsets, adj, n, in_core_out, stream, opt, stats_host, k);
}

int kcore_decompose(const int64_t* offsets, const int32_t* adj, int64_t n, int32_t* coreness_out,
                    hipStream_t stream) {
  return kcore_decompose_ex(offsets, adj, n, coreness_out, stream, nullptr, nullptr);
}

static int batched_impl(const int64_t* graph_vptr, const int64_t* offsets, const int32_t* adj,
                        int32_t num_graphs, int64_t total_vertices, int32_t* coreness_out,
                        hipStream_t stream, const kcore_options* opt, kcore_stats* stats_host,
                        bool local_ids, unsigned* status_out = nullptr, int32_t team_wgs = 0);

int kcore_decompose_batched_ex(const int64_t* graph_vptr, const int64_t* offsets, const int32_t* adj,
                               int32_t num_graphs, int64_t total_vertices, int32_t* coreness_out,
                               hipStream_t stream, const kcore_options* opt, kcore_stats* stats_host) {
  return batched_impl(graph_vptr, offsets, adj, num_graphs, total_vertices, coreness_out, stream, opt,
                      stats_host, false);
}

}  // extern "C"

int kc::reserve_batched(hipStream_t stream, int64_t V, int32_t G) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  BatchWs* w = nullptr;
  return batch_ws(dev, stream, V, G, w);
}

void kc::release_batched(hipStream_t stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_batch.find(Key(dev, stream));
  if (it == g_batch.end()) return;
  BatchWs* w = it->second;
  g_batch.erase(it);
  if (!w) return;
  hipStreamSynchronize(stream);
  if (w->block) hipFree(w->block);
  if (w->host_stats) hipHostFree(w->host_stats);
  if (w->ev0) hipEventDestroy(w->ev0);
  if (w->ev1) hipEventDestroy(w->ev1);
  delete w;
}

int kc::decompose_batched_local(const int64_t* graph_vptr, const int64_t* offsets, const int32_t* adj,
                                int32_t num_graphs, int64_t total_vertices, int32_t* coreness_out,
                                hipStream_t stream, unsigned* status_out, int32_t team_wgs) {
  return batched_impl(graph_vptr, offsets, adj, num_graphs, total_vertices, coreness_out, stream, nullptr,
                      nullptr, true, status_out, team_wgs);
}

int kc::batched_resident_wgs() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  DevInfo di;
  if (dev_info(dev, di)) return 0;
  return di.batch_bpc * di.cus;
}

int64_t kc::batched_lds_vertices() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  DevInfo di;
  if (dev_info(dev, di)) return 0;
  return (int64_t)(di.batch_lds / 8);
}

static int batched_impl(const int64_t* graph_vptr, const int64_t* offsets, const int32_t* adj,
                        int32_t num_graphs, int64_t total_vertices, int32_t* coreness_out,
                        hipStream_t stream, const kcore_options* opt, kcore_stats* stats_host,
                        bool local_ids, unsigned* status_out, int32_t team_wgs) {
  g_err.clear();
  if (num_graphs < 0 || total_vertices < 0)
    return fail(KCORE_EINVAL, "negative num_graphs or total_vertices");
  if (total_vertices > 0x7fffffffLL) return fail(KCORE_EINVAL, "total_vertices exceeds the int32 id range");
  if (int rc = check_opts(opt)) return rc;
  if (num_graphs == 0 || total_vertices == 0) {
    if (stats_host) memset(stats_host, 0, sizeof *stats_host);
    return KCORE_OK;
  }
  if (!graph_vptr || !offsets || !adj || !coreness_out) return fail(KCORE_EINVAL, "null pointer argument");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  DevInfo di;
  if (int rc = dev_info(dev, di)) return rc;
  BatchWs* w = nullptr;
  if (int rc = batch_ws(dev, stream, total_vertices, num_graphs, w)) return rc;
  if (opt && opt->validate) {
    if (int rc = run_validate(offsets, adj, total_vertices, graph_vptr, num_graphs, w->vstat, stream)) return rc;
  }
  // LDS per workgroup: induced degrees + peel queue, 8 bytes per vertex
  const size_t lds = di.batch_lds;
  const int32_t cap = (int32_t)(lds / 8);
  int bpc = di.batch_bpc;
  if (opt && opt->blocks_per_cu && opt->blocks_per_cu < bpc) bpc = opt->blocks_per_cu;
  if (bpc < 1) return fail(KCORE_EDEVICE, "batched kernel cannot be resident on this device");
  const int blocks_full = bpc * di.cus;
  int blocks = std::min(blocks_full, num_graphs);

  HIP_TRY(kc::launch_fill_u32(w->ctl, 0u, sizeof(kc::BatchCtl) / 4, stream));
  if (KCORE_CHECKS) HIP_TRY(kc::launch_fill_u32(coreness_out, 0xffffffffu, (size_t)total_vertices, stream));
  HIP_TRY(kc::launch_order(graph_vptr, offsets, num_graphs, w->order, stream));
  kc::BatchArgs a;
  a.vptr = graph_vptr;
  a.off = offsets;
  a.adj = adj;
  a.G = num_graphs;
  a.core = coreness_out;
  a.order = w->order;
  a.gdt = w->gdt;
  a.gq = w->gq;
  a.ga = w->ga;
  a.local_ids = local_ids ? 1 : 0;
  a.ctl = w->ctl;
  a.lds_cap = cap;
  // barrier-separated subrounds by default: inside one workgroup a barrier is cheap, and peeling a
  // whole frontier edge-balanced over all 512 threads beats 64-vertex packets claimed per wave
  if (opt && (opt->mode == KCORE_MODE_SAMPLING || opt->mode == KCORE_MODE_OFFLINE))
    return fail(KCORE_EINVAL, "the batched peel has neither sampling nor offline mode (its degrees live in LDS)");
  a.chained = (opt && opt->mode == KCORE_MODE_CHAINED) ? 1 : 0;
  // The largest graphs may get teams of workgroups (level-sync mode). A caller's batch runs in a
  // cooperative grid (teams wait for each other, so all must be resident); the serving runtime's
  // large batches (team_wgs > 0) put every graph in a team, in a grid of only the team workgroups
  // whose total over its concurrent batches it keeps within what the device holds.
  const int32_t bt = opt ? opt->batch_teams : 0;
  // (the grid is then the full resident size, whatever the number of graphs: spare workgroups
  // form the teams)
  const bool coop_teams = !local_ids && !a.chained && bt >= 0 && blocks_full >= 4 * kc::kTeamSize &&
                          !(opt && opt->blocks_per_cu);
  const int32_t tsz = opt ? opt->team_size : 0;
  const bool serve_teams = local_ids && team_wgs >= kc::kTeamSize;
  a.teams = (coop_teams || serve_teams) ? 1 : 0;
  if (coop_teams) blocks = blocks_full;
  if (serve_teams) blocks = std::min(blocks_full, team_wgs);
  if (a.teams)
    // (a caller's batch keeps three quarters of its workgroups for the many small graphs)
    HIP_TRY(kc::launch_team_plan(graph_vptr, offsets, num_graphs, w->order, blocks,
                                 serve_teams ? blocks : blocks / 4, tsz, serve_teams ? 1 : 0,
                                 bt > 0 ? bt : 0, w->ctl, stream));
  if (stats_host) HIP_TRY(hipEventRecord(w->ev0, stream));
  if (coop_teams) {
    if (int rc = launch_ordered(dev, stream, [&] { return kc::launch_batched_coop(a, blocks, lds, stream); }))
      return rc;
  } else {
    HIP_TRY(kc::launch_batched(a, blocks, lds, stream));
  }
  // the device status word (failure bits), for callers that check it after the stream
  if (status_out)
    HIP_TRY(hipMemcpyAsync(status_out, &w->ctl->status, sizeof(unsigned), hipMemcpyDeviceToHost, stream));
  if (opt && opt->status_out)
    HIP_TRY(hipMemcpyAsync(opt->status_out, &w->ctl->status, sizeof(unsigned), hipMemcpyDefault, stream));
  if (!stats_host) return KCORE_OK;
  HIP_TRY(hipEventRecord(w->ev1, stream));
  HIP_TRY(kc::launch_live_count(offsets, coreness_out, total_vertices, &w->ctl->stats[kc::ST_LIVE], stream));
  HIP_TRY(hipMemcpyAsync(w->host_stats, w->ctl->stats, kc::kStatWords * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(w->host_stats + kc::kStatWords, &w->ctl->status, sizeof(unsigned),
                         hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  unsigned status = 0;
  memcpy(&status, w->host_stats + kc::kStatWords, sizeof status);
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, w->ev0, w->ev1));
  fill_stats(stats_host, w->host_stats, status, ms);
  stats_host->peeled = total_vertices;
  stats_host->barriers = 0;
  if (status) return fail(KCORE_EDEVICE, "device reported failure bits 0x%x", status);
  return KCORE_OK;
}

// ---- no-allocation batched entry point ---------------------------------------------------
// Its workspace is a file-scope device array (one per GPU, alive until the process ends): the
// control block, the largest-first order of the graphs and the global induced degrees, peel
// queues and active lists of graphs beyond the LDS capacity. Host code reaches it only through
// the address hipGetSymbolAddress reports for the current device.
namespace {
constexpr int64_t kNoAllocVertices = 1ll << 20;  // vertices per call at most
constexpr int32_t kNoAllocGraphs = 1 << 16;      // graphs per call at most
constexpr size_t kNoAllocCtlBytes = (sizeof(kc::BatchCtl) + 255) / 256 * 256;
constexpr size_t kNoAllocOrderOff = kNoAllocCtlBytes;
constexpr size_t kNoAllocStateOff = kNoAllocOrderOff + 4 * (size_t)kNoAllocGraphs;
constexpr size_t kScratchBytes = kNoAllocStateOff + 3 * 4 * (size_t)kNoAllocVertices;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch;  // device -> device address of that device's scratch

// Device address of the current device's scratch array, looked up once per device.
int scratch_ptr(int dev, unsigned char*& out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(dev);
  if (it != g_scratch.end()) {
    out = it->second;
    return KCORE_OK;
  }
  void* ptr = nullptr;
  HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) return fail(KCORE_EDEVICE, "no device address for the scratch array on device %d", dev);
  out = static_cast<unsigned char*>(ptr);
  g_scratch[dev] = out;
  return KCORE_OK;
}
}  // namespace

extern "C" {

int kcore_decompose_batched_noalloc(const int64_t* graph_vptr, const int64_t* offsets, const int32_t* adj,
                                    int32_t num_graphs, int64_t total_vertices, int32_t* coreness_out,
                                    uint32_t* status_out, hipStream_t stream) {
  g_err.clear();
  if (num_graphs < 0 || total_vertices < 0) return fail(KCORE_EINVAL, "negative num_graphs or total_vertices");
  if (total_vertices > kNoAllocVertices || num_graphs > kNoAllocGraphs)
    return fail(KCORE_ETOOBIG, "the no-allocation call takes at most %lld vertices and %d graphs (got %lld, %d)",
                (long long)kNoAllocVertices, kNoAllocGraphs, (long long)total_vertices, num_graphs);
  if (num_graphs == 0 || total_vertices == 0) return KCORE_OK;
  if (!graph_vptr || !offsets || !adj || !coreness_out) return fail(KCORE_EINVAL, "null pointer argument");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  DevInfo di;
  if (int rc = dev_info(dev, di)) return rc;
  unsigned char* sp = nullptr;
  if (int rc = scratch_ptr(dev, sp)) return rc;
  const int32_t cap = (int32_t)(di.batch_lds / 8);
  const int bpc = di.batch_bpc;
  if (bpc < 1) return fail(KCORE_EDEVICE, "batched kernel cannot be resident on this device");
  const int blocks = std::min(bpc * di.cus, num_graphs);
  kc::BatchCtl* ctl = reinterpret_cast<kc::BatchCtl*>(sp);
  // the control block starts at zero in every call (a fill kernel, not a memset node)
  HIP_TRY(kc::launch_fill_u32(ctl, 0u, sizeof(kc::BatchCtl) / 4, stream));
  if (KCORE_CHECKS) HIP_TRY(kc::launch_fill_u32(coreness_out, 0xffffffffu, (size_t)total_vertices, stream));
  int32_t* order = reinterpret_cast<int32_t*>(sp + kNoAllocOrderOff);
  HIP_TRY(kc::launch_order(graph_vptr, offsets, num_graphs, order, stream));
  kc::BatchArgs a;
  a.vptr = graph_vptr;
  a.off = offsets;
  a.adj = adj;
  a.G = num_graphs;
  a.core = coreness_out;
  a.order = order;
  a.gdt = reinterpret_cast<uint32_t*>(sp + kNoAllocStateOff);
  a.gq = reinterpret_cast<int32_t*>(sp + kNoAllocStateOff + 4 * (size_t)kNoAllocVertices);
  a.ga = reinterpret_cast<int32_t*>(sp + kNoAllocStateOff + 8 * (size_t)kNoAllocVertices);
  a.local_ids = 0;
  a.ctl = ctl;
  a.lds_cap = cap;
  a.chained = 0;
  a.teams = 0;  // (teams need the ordered cooperative launch, whose event the library allocates)
  HIP_TRY(kc::launch_batched(a, blocks, di.batch_lds, stream));
  if (status_out)
    HIP_TRY(hipMemcpyAsync(status_out, &ctl->status, sizeof(unsigned), hipMemcpyDefault, stream));
  return KCORE_OK;
}

int kcore_decompose_batched(const int64_t* graph_vptr, const int64_t* offsets, const int32_t* adj,
                            int32_t num_graphs, int64_t total_vertices, int32_t* coreness_out,
                            hipStream_t stream) {
  return kcore_decompose_batched_ex(graph_vptr, offsets, adj, num_graphs, total_vertices, coreness_out,
                                    stream, nullptr, nullptr);
}

int kcore_check(hipStream_t stream) {
  g_err.clear();
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  PeelWs* pw = nullptr;
  BatchWs* bw = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto ip = g_peel.find(Key(dev, stream));
    if (ip != g_peel.end()) pw = ip->second;
    auto ib = g_batch.find(Key(dev, stream));
    if (ib != g_batch.end()) bw = ib->second;
  }
  if ((!pw || !pw->ctl) && (!bw || !bw->ctl))
    return fail(KCORE_ENOTFOUND, "no decomposition ran on this stream of device %d", dev);
  // the status words travel in stream order into each workspace's pinned block
  unsigned* hp = pw && pw->ctl ? reinterpret_cast<unsigned*>(pw->host_stats + kc::kStatWords + 1) : nullptr;
  unsigned* hb = bw && bw->ctl ? reinterpret_cast<unsigned*>(bw->host_stats + kc::kStatWords + 1) : nullptr;
  if (hp) HIP_TRY(hipMemcpyAsync(hp, &pw->ctl->status, sizeof(unsigned), hipMemcpyDeviceToHost, stream));
  if (hb) HIP_TRY(hipMemcpyAsync(hb, &bw->ctl->status, sizeof(unsigned), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  const unsigned sp = hp ? *hp : 0u, sb = hb ? *hb : 0u;
  if (sp || sb)
    return fail(KCORE_EDEVICE, "device reported failure bits 0x%x (single graph), 0x%x (batched)", sp, sb);
  return KCORE_OK;
}

int kcore_release_workspaces(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  HIP_TRY(hipDeviceSynchronize());
  for (auto& kv : g_peel) {
    PeelWs* w = kv.second;
    if (!w) continue;
    if (w->block) hipFree(w->block);
    if (w->sblock) hipFree(w->sblock);
    if (w->hblock) hipFree(w->hblock);
    if (w->host_stats) hipHostFree(w->host_stats);
    if (w->ev0) hipEventDestroy(w->ev0);
    if (w->ev1) hipEventDestroy(w->ev1);
    delete w;
  }
  g_peel.clear();
  for (auto& kv : g_batch) {
    BatchWs* w = kv.second;
    if (!w) continue;
    if (w->block) hipFree(w->block);
    if (w->host_stats) hipHostFree(w->host_stats);
    if (w->ev0) hipEventDestroy(w->ev0);
    if (w->ev1) hipEventDestroy(w->ev1);
    delete w;
  }
  g_batch.clear();
  {
    std::lock_guard<std::mutex> lg(g_grid_mu);
    for (auto& kv : g_grid)
      if (kv.second.ev) hipEventDestroy(kv.second.ev);
    g_grid.clear();
  }
  return KCORE_OK;
}

}  // extern "C"
