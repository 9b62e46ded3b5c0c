// Device code of the k-core library for gfx950 (MI355X).
//
// Two engines:
//  * peel_kernel — one persistent, co-resident grid peels a single graph following the paper's
//    framework (Alg. 1) with the online peel (Alg. 3). Phases are separated by a fence-free grid
//    barrier; a phase either scans the active set (extracting the round's first frontier and
//    refining the set, Alg. 1 extract/refine), expands the current frontier, or (once) rewrites the
//    live rows without peeled neighbours. In chained mode (VGC, Sec. 4.2) a wavefront peels what it
//    pushes through a local queue and a workgroup peels the small hubs it pushes through an LDS tile
//    queue, inside the same phase. Cross-workgroup data (frontiers, active lists, counters) goes
//    through agent-scope relaxed atomics, which the MI355X keeps coherent across its XCD L2
//    caches, so barriers need no L2 write-back or invalidate.
//  * batched_kernel — many independent graphs, one workgroup per graph, with its induced degrees
//    and peel queue in LDS (or, for graphs beyond the LDS, in global memory with a peeled bitmap in
//    LDS), so a graph's rounds and subrounds synchronise at workgroup level only.
#include "kcore_internal.h"

namespace kc {

constexpr uint32_t HUBBIT = 0x80000000u;
constexpr uint32_t DMASK = 0x7fffffffu;

// Checked builds (KCORE_CHECKS=1, a separate library used by tests) verify two invariants of the
// online peel while it runs: every coreness is written exactly once (the output starts filled
// with -1 and each write must find -1 there), and no induced degree is decremented below zero.
// A violation sets KC_ERR_CHECK in the status word; nothing traps. Product builds compile both
// checks away.
#ifndef KCORE_CHECKS
#define KCORE_CHECKS 0
#endif

__device__ __forceinline__ void put_core(int32_t* core, long long v, uint32_t k, unsigned* status) {
  if constexpr (KCORE_CHECKS) {
    if (__hip_atomic_exchange(&core[v], (int32_t)k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != -1)
      __hip_atomic_fetch_or(status, (unsigned)KC_ERR_CHECK, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    (void)status;
    core[v] = (int32_t)k;
  }
}

// (checked builds) a decrement of c that found `before` (its value without flag bits) went below 0
__device__ __forceinline__ void check_decrement(uint32_t before, uint32_t c, unsigned* status) {
  if constexpr (KCORE_CHECKS) {
    if (before < c)
      __hip_atomic_fetch_or(status, (unsigned)KC_ERR_CHECK, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    (void)before;
    (void)c;
    (void)status;
  }
}

template <class T>
__device__ __forceinline__ T ald(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void ast(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T aadd(T* p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T asub(T* p, T v) {
  return __hip_atomic_fetch_sub(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T aor(T* p, T v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T amin(T* p, T v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int rank_in(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}
template <class T>
__device__ __forceinline__ T wave_incl_scan(T x) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T y = __shfl_up(x, o, 64);
    if (l >= o) x += y;
  }
  return x;
}
__device__ __forceinline__ unsigned wave_min(unsigned x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = min(x, (unsigned)__shfl_xor((int)x, o, 64));
  return x;
}

// ------------------------------------------------------------------------------------------
// Grid barrier. Arrivals go to one of kBarGroups counters, the last arrival of each group to a
// top counter, and the last top arrival publishes the new epoch; with ONE set (the level-sync
// kernel instances) every workgroup arrives at the top counter directly. One group (every
// workgroup on one counter) beat 8, 32 and 64 groups in the chained instances; there the grouped
// code with one group also measured faster than the direct form (whose code moved the kernel's
// register allocation), at the cost of a second atomic for the completing arrival only. Counters
// only grow and are tested for equality with the epoch's total, so no reset races. Every thread first waits for its own memory operations to
// complete (s_waitcnt), which with agent-scope accesses makes them visible device-wide before the
// arrival. Waits are bounded: after ~4 s without progress, or if any workgroup has flagged an
// error, every workgroup leaves.
// ------------------------------------------------------------------------------------------
template <bool ONE = false>
__device__ bool grid_sync(PeelCtl* C, unsigned& epoch) {
  __shared__ int s_ok;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned nb = gridDim.x;
    const unsigned target = epoch + 1;
    int ok = 1;
    bool last = false;
    if constexpr (ONE) {
      last = aadd(&C->bar_top, 1u) == target * nb - 1;
    } else {
      const unsigned ng = nb < (unsigned)kBarGroups ? nb : (unsigned)kBarGroups;
      const unsigned grp = blockIdx.x % ng;
      const unsigned gsize = nb / ng + ((nb % ng) > grp ? 1u : 0u);
      const unsigned a = aadd(&C->bar_grp[grp][0], 1u);
      if (a == target * gsize - 1) {
        const unsigned b = aadd(&C->bar_top, 1u);
        if (b == target * ng - 1) last = true;
      }
    }
    if (last) {
      __builtin_amdgcn_s_waitcnt(0);
      ast(&C->bar_gen, target);
    } else {
      const unsigned long long t0 = wall_clock64();
      while (ald(&C->bar_gen) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (wall_clock64() - t0 > 400000000ull) {  // 100 MHz clock: 4 s
          aor(&C->status, (unsigned)KC_ERR_TIMEOUT);
          ok = 0;
          break;
        }
      }
    }
    if (ald(&C->status) != 0u) ok = 0;
    s_ok = ok;
  }
  __syncthreads();
  epoch += 1;
  return s_ok != 0;
}

// ------------------------------------------------------------------------------------------
// Per-wave staging of appends to a global list: entries collect in LDS and go out in bulk, so the
// shared tail counter sees one atomic per flush instead of one per wave step.
// ------------------------------------------------------------------------------------------
struct Stage {
  int32_t* buf;  // LDS, kStage entries
  int cnt;       // wave-uniform
};

__device__ __forceinline__ void stage_flush(Stage& s, unsigned long long* tail, int32_t* dst,
                                            long long cap, unsigned* status) {
  if (s.cnt == 0) return;
  unsigned long long base = 0;
  if (lane_id() == 0) base = aadd(tail, (unsigned long long)s.cnt);
  base = __shfl(base, 0, 64);
  if ((long long)(base + s.cnt) > cap) {
    if (lane_id() == 0) aor(status, (unsigned)KC_ERR_OVERFLOW);
  } else {
    for (int i = lane_id(); i < s.cnt; i += 64) ast(&dst[base + i], s.buf[i]);
  }
  s.cnt = 0;
}

// all lanes call; lanes with p append v
__device__ __forceinline__ void stage_push(Stage& s, bool p, int32_t v, unsigned long long* tail,
                                           int32_t* dst, long long cap, unsigned* status) {
  const unsigned long long m = __ballot(p);
  if (m == 0) return;
  const int c = __popcll(m);
  if (s.cnt + c > kStage) stage_flush(s, tail, dst, cap, status);
  if (p) s.buf[s.cnt + rank_in(m)] = v;
  s.cnt += c;
}

// Block-level final flush of every wave's leftovers with one atomic per block.
__device__ __forceinline__ void block_flush(Stage& s, unsigned long long* tail, int32_t* dst, long long cap,
                            unsigned* status, unsigned long long* s_cnt, unsigned long long* s_base) {
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if (lane_id() == 0) s_cnt[w] = (unsigned long long)s.cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tot = 0;
    for (int i = 0; i < kWaves; ++i) {
      unsigned long long c = s_cnt[i];
      s_cnt[i] = tot;
      tot += c;
    }
    unsigned long long b = tot ? aadd(tail, tot) : 0ull;
    if (tot && (long long)(b + tot) > cap) {
      aor(status, (unsigned)KC_ERR_OVERFLOW);
      tot = 0;
    }
    *s_base = tot ? b : ~0ull;
  }
  __syncthreads();
  const unsigned long long b = *s_base;
  if (b != ~0ull) {
    const unsigned long long o = b + s_cnt[w];
    for (int i = lane_id(); i < s.cnt; i += 64) ast(&dst[o + i], s.buf[i]);
  }
  s.cnt = 0;
  __syncthreads();
}

// Active lists are compacted into one segment per workgroup: a workgroup appends the survivors it
// scanned to its own segment with an LDS counter, so compaction needs no global atomic (a single
// shared tail counter would serialise one atomic per wave flush). Item j of a segmented list is the
// (j - pref[b])-th entry of segment b, where pref holds the exclusive prefix of the segment counts.
__device__ __forceinline__ void seg_flush(Stage& s, int32_t* seg, int* s_used) {
  if (s.cnt == 0) return;
  int base = 0;
  if (lane_id() == 0) base = atomicAdd(s_used, s.cnt);
  base = __shfl(base, 0, 64);
  for (int i = lane_id(); i < s.cnt; i += 64) ast(&seg[base + i], s.buf[i]);
  s.cnt = 0;
}

__device__ __forceinline__ void seg_push(Stage& s, bool p, int32_t v, int32_t* seg, int* s_used) {
  const unsigned long long m = __ballot(p);
  if (m == 0) return;
  const int c = __popcll(m);
  if (s.cnt + c > kStage) seg_flush(s, seg, s_used);
  if (p) s.buf[s.cnt + rank_in(m)] = v;
  s.cnt += c;
}

__device__ __forceinline__ int32_t active_item(const int32_t* alist, bool dense, long long j, long long aseg,
                                               const int* pref, int nb) {
  if (dense) return (int32_t)j;
  int lo = 0, hi = nb - 1;  // last segment with pref[b] <= j
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((long long)pref[mid] <= j) lo = mid; else hi = mid - 1;
  }
  return ald(&alist[(long long)lo * aseg + (j - pref[lo])]);
}

// ------------------------------------------------------------------------------------------
// Single-graph peel.
// ------------------------------------------------------------------------------------------
struct WaveCtx {
  Stage sf;            // next small frontier
  Stage sa;            // compacted active list
  int32_t* lq;         // local queue ring (chained mode)
  int lq_head, lq_cnt; // wave-uniform
  int lq_used;         // vertices peeled from the local queue this phase
  long long edges, decr, scanned, peeled, comb, binserts;  // per-lane statistics
  unsigned mymin;      // per-lane min over kept vertices
  int32_t* ckey;       // LDS combining table (block-shared): target id or -1
  uint32_t* ccnt;      //   decrements collected for it in this phase
  bool precheck;       // phase-uniform: probe peeled bits
  bool combine;        // phase-uniform: collect decrements of hot targets in LDS
  bool async;          // phase-uniform: pushes go to the async work queue
  bool arbitrate;      // phase-uniform: crossings may race with a scan (chained scan phases)
  bool bq_open;        // phase-uniform: small hubs go to the workgroup's tile queue
  unsigned long long* bq;  // LDS, kBlockQ entries: (tile << 32) | vertex, kQEmpty or kQSkip
  int* bqc;            // LDS: claimed, reserved, busy waves, [4..5] debug counts
  const int32_t* adj;  // adjacency the rows point into: the input, or the residual rows
  const long long* rows;  // row bounds: offsets (stride 1) or residual (start, end) pairs (stride 2)
  int rstride;
  bool resid;          // rows come from the residual rows
  bool hbs;            // phase-uniform: the multi-bucket active set is kept (decrements move vertices)
  long long* hlen;     // LDS: entries in each bucket slot before this phase (same in every workgroup)
};

// Row of v: [b, b + d) in c.adj.
__device__ __forceinline__ void row_of(const PeelArgs& a, const WaveCtx& c, int32_t v, long long& b,
                                       long long& d) {
  const long long* r = c.rows + (long long)v * c.rstride;
  b = r[0];
  d = r[1] - b;
}

__device__ __forceinline__ unsigned comb_hash(int32_t u) {
  return ((unsigned)u * 2654435761u) >> (32 - kCombBits);
}

// Adds one decrement of hub target u to the block's LDS table; false when its probe window is
// full (the caller then decrements in global memory directly).
__device__ __forceinline__ bool comb_add(WaveCtx& c, int32_t u) {
  const unsigned h = comb_hash(u);
#pragma unroll
  for (int p = 0; p < kCombProbe; ++p) {
    const unsigned s = (h + p) & (kCombSlots - 1);
    int32_t key = __hip_atomic_load(&c.ckey[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (key == -1) {
      key = atomicCAS(&c.ckey[s], -1, u);
      if (key == -1) key = u;
    }
    if (key == u) {
      atomicAdd(&c.ccnt[s], 1u);
      return true;
    }
  }
  return false;
}

struct PhaseOut {
  PhaseSlot* slot;
  int32_t* fr;  // frontier list written in this phase
  unsigned long long* tl;  // tile list written in this phase (span words)
};

// ------------------------------------------------------------------------------------------
// Multi-bucket active set (HBS, Sec. 5.2). Relative to the current round k, a live vertex with
// induced degree x > k belongs to bucket b = the highest bit in which x and k differ (x has a 1
// there, k a 0): the ranges above k are aligned blocks of 1, 2, 4, ... values, so the bucket of a
// value only changes for values in the block that k itself enters. When k moves to k' > k, the
// buckets above H = the highest bit of k ^ k' keep their ranges, bucket H holds exactly the values
// from k' up to its block's end (redistributed by the next scan into lower buckets, with the
// vertices at k' extracted), and the buckets below H held only values below k' (all peeled), so
// they start empty. Buckets are append-only lists; a vertex whose induced degree drops into a
// lower bucket is appended there (the old copy goes stale and is dropped when read). A per-vertex
// tag (the lower end of the range it was last filed into) keeps a vertex from being appended
// twice to one range: every change of the tag comes with an append, so a vertex is always listed
// in the bucket of its current value.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ int hbs_bucket(uint32_t x, uint32_t k) { return 31 - __clz(x ^ k); }
__device__ __forceinline__ uint32_t hbs_lo(uint32_t k, int b) { return ((k >> b) | 1u) << b; }

// Appends v to bucket slot b for the lanes with want: one reservation per distinct slot in the
// wave. All lanes call.
__device__ __forceinline__ void hbs_append(const PeelArgs& a, WaveCtx& c, const PhaseOut& o, bool want,
                                           int32_t v, int b) {
  unsigned long long pend = __ballot(want);
  while (pend) {
    const int leader = __ffsll((long long)pend) - 1;
    const int bl = __shfl(b, leader, 64);
    const bool mine = want && b == bl;
    const unsigned long long mm = __ballot(mine);
    unsigned long long base = 0;
    if (lane_id() == leader && bl < a.hslots) base = aadd(&o.slot->hadd[bl], (unsigned long long)__popcll(mm));
    base = __shfl(base, leader, 64);
    if (mine) {
      const long long pos = c.hlen[bl] + (long long)base + rank_in(mm);
      if (bl < a.hslots && pos < a.hcap) {
        ast(&a.hbl[(long long)bl * a.hcap + pos], v);
        c.binserts += 1;
      } else {
        aor(&a.ctl->status, (unsigned)KC_ERR_OVERFLOW);
      }
    }
    pend &= ~mm;
  }
}

// A decrement took u from xo to xn in round k: if xn > k lies in a lower bucket than xo, u is
// filed there unless its tag says it already is. All lanes call.
__device__ __forceinline__ void hbs_move(const PeelArgs& a, WaveCtx& c, const PhaseOut& o, bool did, int32_t u,
                                         uint32_t xo, uint32_t xn, uint32_t k) {
  bool want = false;
  int b = 0;
  if (did && xn > k && xn < xo) {
    b = hbs_bucket(xn, k);
    if (b < hbs_bucket(xo, k)) {
      const uint32_t lo = hbs_lo(k, b);
      want = __hip_atomic_exchange(&a.hlo[u], lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != lo;
    }
  }
  hbs_append(a, c, o, want, u, b);
}

// A scan read v live with x > k (keep) after reading its tag t: file it into its bucket, unless
// the tag already names that range or changed meanwhile (then whoever changed it filed v). All
// lanes call.
__device__ __forceinline__ void hbs_file(const PeelArgs& a, WaveCtx& c, const PhaseOut& o, bool keep, int32_t v,
                                         uint32_t x, uint32_t t, uint32_t k) {
  bool want = false;
  int b = 0;
  if (keep) {
    b = hbs_bucket(x, k);
    const uint32_t lo = hbs_lo(k, b);
    if (t != lo) want = atomicCAS(&a.hlo[v], t, lo) == t;
  }
  hbs_append(a, c, o, want, v, b);
}

// Pushes crossed/extracted vertices: hubs are split into tiles on the global tile list, small
// vertices go to the wave's local queue (chained mode, while it has room) or the staged frontier.
// All lanes call.
// Async work queue entry: low word vertex, high word tile index, or kWholeRow for a whole row.
constexpr uint32_t kWholeRow = 0xffffffffu;
constexpr long long kQEmpty = -1ll;
constexpr long long kQSkip = -2ll;  // a reserved workgroup-queue slot that holds no work

// A hub tile as one word: position of its first adjacency entry (high 48 bits) and its length (low
// 16 bits), so that peeling it needs no lookup of the row's offsets. Lengths never reach 0xfffe,
// so a span never equals kQEmpty or kQSkip.
__device__ __forceinline__ unsigned long long span_word(long long pos, long long len) {
  return ((unsigned long long)pos << 16) | (unsigned long long)len;
}

template <class T>
__device__ __forceinline__ T lds_ld(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <class T>
__device__ __forceinline__ void lds_st(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Chained mode: appends the cnt tiles of row [rb, rb + deg) of each lane with cnt > 0 to the
// workgroup's tile queue. Either
// the whole wave's request fits, or none of it does (its reserved slots are then marked empty of
// work and the caller sends the tiles to the global list). All lanes call; true for lanes whose
// tiles were queued.
__device__ __forceinline__ bool block_push(WaveCtx& c, long long rb, long long deg, long long tile, long long cnt,
                                           int backlog_max) {
  const long long incl = wave_incl_scan(cnt);
  const long long tot = __shfl(incl, 63, 64);
  if (tot == 0) return false;
  int base = -1;
  if (lane_id() == 0) {
    // a burst of hubs (more than backlog_max tiles waiting) is better spread over the whole grid
    // by the next phase than worked off by this workgroup's 16 waves
    const int waiting = lds_ld(&c.bqc[1]) - lds_ld(&c.bqc[0]);
    if ((long long)waiting + tot <= backlog_max) base = atomicAdd(&c.bqc[1], (int)tot);
  }
  base = __shfl(base, 0, 64);
  if (base < 0) return false;
  const int cap = kBlockQ;
  const bool fits = (long long)base + tot <= cap;
  const long long s0 = (long long)base + incl - cnt;
  for (long long j = 0; j < cnt; ++j) {
    const long long sl = s0 + j;
    if (sl < cap)
      lds_st(&c.bq[sl], fits ? span_word(rb + j * tile, min(tile, deg - j * tile)) : (unsigned long long)kQSkip);
  }
  return fits && cnt > 0;
}

// Appends work for the lanes with cnt > 0 to the phase's async queue: a whole row (cnt == 1 and
// !tiles) or cnt tiles of a hub row. The tail counter doubles as the count of created entries: it
// grows before an entry becomes visible, which the quiescence test relies on. All lanes call.
__device__ __forceinline__ void queue_push(const PeelArgs& a, const PhaseOut& o, int32_t v, long long cnt,
                                           bool tiles) {
  const long long incl = wave_incl_scan(cnt);
  const long long tot = __shfl(incl, 63, 64);
  if (tot == 0) return;
  unsigned long long base = 0;
  if (lane_id() == 0) base = aadd(&o.slot->qtail, (unsigned long long)tot);
  base = __shfl(base, 0, 64);
  if ((long long)base + tot > a.qcap) {
    if (lane_id() == 0) aor(&a.ctl->status, (unsigned)KC_ERR_OVERFLOW);
    return;
  }
  const long long s0 = (long long)base + incl - cnt;
  for (long long j = 0; j < cnt; ++j) {
    const unsigned long long hi = tiles ? (unsigned long long)j : (unsigned long long)kWholeRow;
    ast(&a.aq[s0 + j], (long long)((hi << 32) | (unsigned)v));
  }
}

// Pushes crossed/extracted vertices: hubs are split into tiles, small vertices go to the wave's
// local queue (chained mode, while it has room). Outside async phases the rest goes to the next
// frontier (staged) and the tile list; in async phases both go to the async queue. All lanes call.
template <bool CH>
__device__ __forceinline__ void push_vertices(const PeelArgs& a, WaveCtx& c, const PhaseOut& o,
                                              bool p, int32_t v, bool hub) {
  const bool ps = p && !hub;
  const unsigned long long ms = __ballot(ps);
  if (ms) {
    const int cnt = __popcll(ms);
    if (CH && c.lq_cnt + cnt <= kLocalQ) {
      if (ps) c.lq[(c.lq_head + c.lq_cnt + rank_in(ms)) & (kLocalQ - 1)] = v;
      c.lq_cnt += cnt;
    } else if (CH && c.async) {
      queue_push(a, o, v, ps ? 1 : 0, false);
    } else {
      stage_push(c.sf, ps, v, &o.slot->small, o.fr, a.fcap, &a.ctl->status);
    }
  }
  const bool ph = p && hub;
  const unsigned long long mh = __ballot(ph);
  if (mh) {
    long long nt = 0, rb = 0, deg = 0;
    if (ph) {
      row_of(a, c, v, rb, deg);
      nt = (deg + a.tile - 1) / a.tile;
    }
    if (lane_id() == 0) aadd(&o.slot->hubv, (unsigned long long)__popcll(mh));
    if (CH && c.async) {
      queue_push(a, o, v, nt, true);
      return;
    }
    bool pg = ph;
    if (CH && c.bq_open && block_push(c, rb, deg, a.tile, (ph && nt <= a.bq_max_tiles) ? nt : 0, a.bq_backlog))
      pg = false;
    if (!pg) nt = 0;
    if (__ballot(pg) == 0) return;
    const long long incl = wave_incl_scan(nt);
    const long long tot = __shfl(incl, 63, 64);
    unsigned long long base = 0;
    if (lane_id() == 0) base = aadd(&o.slot->tiles, (unsigned long long)tot);
    base = __shfl(base, 0, 64);
    if ((long long)base + tot > a.tcap) {
      if (lane_id() == 0) aor(&a.ctl->status, (unsigned)KC_ERR_OVERFLOW);
    } else if (pg) {
      const long long s0 = (long long)base + incl - nt;
      for (long long j = 0; j < nt; ++j) ast(&o.tl[s0 + j], span_word(rb + j * a.tile, min((long long)a.tile, deg - j * a.tile)));
    }
  }
}

// ------------------------------------------------------------------------------------------
// Sampling mode (Sec. 4.1, Alg. 4/5). A vertex of degree above s_threshold starts in sample mode:
// bit 30 of its induced degree is set (so no decrement ever takes it to k and no scan extracts it)
// and the "hot" bits of the state words mark it. Removing one of its neighbours then increments its
// hit count with probability rate = mu / ((1 - r) d*), r = 1/10, instead of decrementing it: in
// large phases, where the state word is read anyway, no atomic is spent on its induced degree;
// in small ones the decrement lands on the biased value and is ignored. Validation (Error of
// Alg. 5) and recounts run at round boundaries, where no expansion is pending, so a recount from
// the peeled bits is exact; a vertex found below k there was missed in an earlier round, which
// the host answers by peeling again without sampling (the scheme stays exact).
// ------------------------------------------------------------------------------------------
constexpr uint32_t SAMPLEBIT = 0x40000000u;

// Hit threshold on a uniform 32-bit draw for the rate mu / ((1 - r) d), r = 1/10.
__device__ __forceinline__ uint32_t sample_rate32(uint32_t mu, uint32_t d) {
  const double rate = (double)mu / (0.9 * (double)d);
  return rate >= 1.0 ? 0xffffffffu : (uint32_t)(rate * 4294967296.0);
}

// Smallest round k at which Error (Alg. 5) fails for a vertex with induced degree b at its last
// (re)initialisation, hit threshold thr and cnt hits: d* r <= k, or cnt >= rate (d* - k) / 4, i.e.
// k >= d* - 4 cnt / rate. Rounded down (validated early rather than late); 0 once mu hits are in.
__device__ __forceinline__ uint32_t sample_valk(uint32_t b, uint32_t thr, uint32_t cnt, uint32_t mu) {
  if (cnt >= mu || thr == 0u) return 0u;
  const uint32_t k1 = (b + 9u) / 10u;
  const unsigned long long t = ((((unsigned long long)cnt) << 34) + thr - 1u) / thr;  // ceil(4 cnt / rate)
  const uint32_t k2 = t >= b ? 0u : b - (uint32_t)t;
  return k1 < k2 ? k1 : k2;
}

// Error (Alg. 5) at round k: true while the vertex may stay in sample mode.
__device__ __forceinline__ bool sample_safe(uint32_t b, uint32_t thr, uint32_t cnt, uint32_t k) {
  if ((unsigned long long)b <= 10ull * k) return false;
  return ((unsigned long long)cnt << 34) < (unsigned long long)thr * (unsigned long long)(b - k);
}

// The coin: murmur3's 32-bit finaliser over the seed, the lane's global index and its count of
// entries processed so far (a distinct counter value for every removal the lane handles).
__device__ __forceinline__ uint32_t sample_coin(uint32_t seed, uint32_t lane, uint32_t ctr) {
  uint32_t h = seed ^ (lane * 0x9e3779b1u) ^ (ctr * 0x85ebca77u);
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// One removal of a neighbour of sampled vertex u: a hit with the vertex's rate; a hit moves the
// round of its next validation forward when needed.
__device__ __forceinline__ void sample_hit(const PeelArgs& a, const WaveCtx& c, int32_t u) {
  const uint32_t thr = ald(&a.srate[u]);
  const uint32_t gl = blockIdx.x * blockDim.x + threadIdx.x;
  if (sample_coin(a.s_seed, gl, (uint32_t)c.edges) >= thr) return;
  const uint32_t cnt = aadd(&a.scnt[u], 1u) + 1u;
  const uint32_t kb = sample_valk(ald(&a.sbase[u]), thr, cnt, a.s_mu);
  if (kb < ald(&a.ctl->s_valk)) amin(&a.ctl->s_valk, kb);
}

// Up to U adjacency entries per lane: the online decrement of Alg. 3. All loads, and
// then all atomics, of a lane are issued before any result is used, so one pass costs a few memory
// round trips however many entries it covers. In large phases (c.precheck) a neighbour whose
// peeled bit is already set is skipped and hub targets go to the LDS combining table; in small,
// latency-bound phases the probe is skipped (decrementing a peeled vertex is harmless: it can
// never cross k again, and each neighbour decrements it once, so it never drops below zero).
// The lane whose decrement takes u from k+1 to k pushes it.
template <bool S, bool H, bool CH, int U>
__device__ __forceinline__ void edges_batch(const PeelArgs& a, WaveCtx& c, const PhaseOut& o,
                                            const int32_t (&u)[U], unsigned valid, uint32_t k) {
  uint32_t sw[U];
#pragma unroll
  for (int j = 0; j < U; ++j) sw[j] = 0u;
  if (c.precheck) {
#pragma unroll
    for (int j = 0; j < U; ++j)
      if ((valid >> j) & 1u) sw[j] = ald(&a.state[u[j] >> 4]);
  }
  uint32_t old[U];
  unsigned did = 0u;
#pragma unroll
  for (int j = 0; j < U; ++j) {
    old[j] = 0u;
    if (!((valid >> j) & 1u)) continue;
    c.edges += 1;
    if ((sw[j] >> (u[j] & 15)) & 1u) continue;  // already peeled
    if constexpr (S) {
      // sampling mode: the state word marks sampled targets (large phases read it anyway)
      if ((sw[j] >> (16 + (u[j] & 15))) & 1u) {
        sample_hit(a, c, u[j]);
        continue;
      }
    } else {
      // hub targets collect their decrements in LDS for the rest of the phase (the flush applies
      // them with one atomic per target); everything else is decremented right away
      if (c.combine && ((sw[j] >> (16 + (u[j] & 15))) & 1u) && comb_add(c, u[j])) {
        c.comb += 1;
        continue;
      }
    }
    old[j] = asub(&a.dt[u[j]], 1u);
    c.decr += 1;
    did |= 1u << j;
  }
  if constexpr (S) {
    // a decrement that landed on a sampled vertex (small phases do not read the state word)
#pragma unroll
    for (int j = 0; j < U; ++j)
      if (((did >> j) & 1u) && (old[j] & SAMPLEBIT)) sample_hit(a, c, u[j]);
  }
  if constexpr (!S && KCORE_CHECKS) {
#pragma unroll
    for (int j = 0; j < U; ++j)
      if ((did >> j) & 1u) check_decrement(old[j] & DMASK, 1u, &a.ctl->status);
  }
  if constexpr (!S && H) {
    if (c.hbs) {
#pragma unroll
      for (int j = 0; j < U; ++j) {
        const uint32_t xo = old[j] & DMASK;
        hbs_move(a, c, o, ((did >> j) & 1u) != 0u, u[j], xo, xo - 1u, k);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < U; ++j) {
    bool crossed = ((did >> j) & 1u) && (old[j] & DMASK) == k + 1u;
    const bool hub = (old[j] & HUBBIT) != 0u;
    if (crossed) {
      const uint32_t bit = 1u << (u[j] & 15);
      if (CH && c.arbitrate) {
        // a scan of this phase may find u at the same time: the peeled bit decides ownership
        if (aor(&a.state[u[j] >> 4], bit) & bit) crossed = false;
      } else {
        // only one decrement crosses k, so the lane owns u: set the bit without waiting for it
        __hip_atomic_fetch_or(&a.state[u[j] >> 4], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (crossed) {
        if (a.k_query <= 0) put_core(a.core, u[j], k, &a.ctl->status);
        c.peeled += 1;
      }
    }
    push_vertices<CH>(a, c, o, crossed, u[j], hub);
  }
}

// Expands the rows of up to 64 vertices (one per lane, -1 = none) edge-balanced across the wave:
// an exclusive scan of the degrees, then each lane finds the row of each of its entries by binary
// search over the scan.
template <bool S, bool H, bool CH>
__device__ __forceinline__ void expand_rows(const PeelArgs& a, WaveCtx& c, const PhaseOut& o, int32_t v, uint32_t k) {
  long long b = 0, d = 0;
  if (v >= 0) row_of(a, c, v, b, d);
  const long long incl = wave_incl_scan(d);
  const long long excl = incl - d;
  const long long total = __shfl(incl, 63, 64);
  const int l = lane_id();
  for (long long e0 = 0; e0 < total; e0 += 64 * kEdgeUnroll) {
    int32_t u[kEdgeUnroll];
    unsigned valid = 0u;
#pragma unroll
    for (int q = 0; q < kEdgeUnroll; ++q) {
      const long long t = e0 + 64 * q + l;
      int j = 0;
#pragma unroll
      for (int step = 32; step >= 1; step >>= 1) {
        const int cand = j + step;
        const long long ex = __shfl(excl, cand & 63, 64);
        if (cand < 64 && ex <= t) j = cand;
      }
      const long long pos = __shfl(b, j, 64) + (t - __shfl(excl, j, 64));
      u[q] = 0;
      if (t < total) {
        u[q] = c.adj[pos];
        valid |= 1u << q;
      }
    }
    edges_batch<S, H, CH>(a, c, o, u, valid, k);
  }
}

// A hub tile: adjacency entries [pos, pos + len), len <= 64 * kTileUnroll for default tiles.
template <bool S, bool H, bool CH>
__device__ __forceinline__ void expand_span(const PeelArgs& a, WaveCtx& c, const PhaseOut& o, long long pos,
                                            long long len, uint32_t k) {
  // hub rows mostly point at vertices peeled long ago: probe the peeled bits here (in every phase
  // unless only large phases are asked for). Rewritten rows hold live neighbours only, so small
  // phases save the probe's round trip there.
  const bool saved = c.precheck;
  c.precheck = saved || (a.tile_probe_always && !c.resid);
  const long long e = pos + len;
  for (long long p0 = pos; p0 < e; p0 += 64 * kTileUnroll) {
    int32_t u[kTileUnroll];
    unsigned valid = 0u;
#pragma unroll
    for (int q = 0; q < kTileUnroll; ++q) {
      const long long i = p0 + 64 * q + lane_id();
      u[q] = 0;
      if (i < e) {
        u[q] = c.adj[i];
        valid |= 1u << q;
      }
    }
    edges_batch<S, H, CH>(a, c, o, u, valid, k);
  }
  c.precheck = saved;
}

// Tile j of the row of v (async queue entries name the vertex).
template <bool S, bool H, bool CH>
__device__ __forceinline__ void expand_tile(const PeelArgs& a, WaveCtx& c, const PhaseOut& o, int32_t v, int32_t j,
                                            uint32_t k) {
  long long rb = 0, d = 0;
  row_of(a, c, v, rb, d);
  const long long b = rb + (long long)j * a.tile;
  expand_span<S, H, CH>(a, c, o, b, min(rb + d, b + a.tile) - b, k);
}

// Applies the block's combined decrements: one atomic subtraction of c per target; exactly one
// subtraction takes a target from above k to k or below (old > k >= old - c), and that one pushes
// it. Clears the table for the next phase. All threads of the block call.
template <bool H, bool CH>
__device__ __forceinline__ void comb_flush(const PeelArgs& a, WaveCtx& c, const PhaseOut& o, uint32_t k) {
  __syncthreads();
  for (int s0 = 0; s0 < kCombSlots; s0 += kPeelThreads) {
    const int s = s0 + threadIdx.x;
    const int32_t u = c.ckey[s];
    bool crossed = false, hub = false;
    uint32_t hxo = 0, hxn = 0;
    if (u >= 0) {
      const uint32_t cnt = c.ccnt[s];
      c.ckey[s] = -1;
      c.ccnt[s] = 0;
      const uint32_t old = asub(&a.dt[u], cnt);
      c.decr += 1;
      const uint32_t ox = old & DMASK;
      hxo = ox;
      hxn = ox - cnt;
      check_decrement(ox, cnt, &a.ctl->status);
      if (ox > k && ox - cnt <= k) {
        const uint32_t bit = 1u << (u & 15);
        if (!(aor(&a.state[u >> 4], bit) & bit)) {
          crossed = true;
          hub = (old & HUBBIT) != 0u;
          if (a.k_query <= 0) put_core(a.core, u, k, &a.ctl->status);
          c.peeled += 1;
        }
      }
    }
    if constexpr (H) {
      if (c.hbs) hbs_move(a, c, o, u >= 0 && hxo >= hxn, u, hxo, hxn, k);
    }
    push_vertices<CH>(a, c, o, crossed, u, hub);
  }
  __syncthreads();
}

// Chained mode: peel what the wave queued locally, in packets of up to 64 vertices, until the
// queue is empty or the wave's budget for this phase is spent; what is left joins the frontier.
template <bool S, bool H, bool CH>
__device__ __forceinline__ void drain_local(const PeelArgs& a, WaveCtx& c, const PhaseOut& o, uint32_t k) {
  while (c.lq_cnt > 0 && c.lq_used < a.lq_budget) {
    const int take = c.lq_cnt < 64 ? c.lq_cnt : 64;
    const int32_t v = lane_id() < take ? c.lq[(c.lq_head + lane_id()) & (kLocalQ - 1)] : -1;
    c.lq_head = (c.lq_head + take) & (kLocalQ - 1);
    c.lq_cnt -= take;
    c.lq_used += take;
    if (lane_id() == 0) atomicAdd(&c.bqc[5], take);
    expand_rows<S, H, CH>(a, c, o, v, k);
  }
  while (c.lq_cnt > 0) {
    const int take = c.lq_cnt < 64 ? c.lq_cnt : 64;
    const bool p = lane_id() < take;
    const int32_t v = p ? c.lq[(c.lq_head + lane_id()) & (kLocalQ - 1)] : 0;
    c.lq_head = (c.lq_head + take) & (kLocalQ - 1);
    c.lq_cnt -= take;
    if (c.async)
      queue_push(a, o, v, p ? 1 : 0, false);
    else
      stage_push(c.sf, p, v, &o.slot->small, o.fr, a.fcap, &a.ctl->status);
  }
}

// Chained mode, after a wave's static share: the workgroup's 16 waves peel the small hubs pushed
// into its tile queue in this phase, and whatever those tiles push in turn, so a chain through hubs
// continues inside the phase instead of waiting for the next one. A wave leaves once it sees no
// busy wave (busy first) and then no unclaimed slot: entries are only reserved by busy waves, and a
// wave that reserved entries stays until it sees them claimed, so no entry is left behind. Waits
// are bounded.
template <bool S, bool H, bool CH>
__device__ __forceinline__ void block_loop(const PeelArgs& a, WaveCtx& c, const PhaseOut& o, uint32_t k) {
  int* head = &c.bqc[0];
  int* tail = &c.bqc[1];
  int* busy = &c.bqc[2];
  for (;;) {
    int state = 0;  // 1 got an entry, 2 done, 3 error
    long long e = kQEmpty;
    if (lane_id() == 0) {
      bool counted = true;  // every wave starts the phase counted as busy
      const unsigned long long t0 = wall_clock64();
      for (int spin = 0;; ++spin) {
        const int h = lds_ld(head);
        const int t = min(lds_ld(tail), kBlockQ);
        if (h < t) {
          if (!counted) {
            atomicAdd(busy, 1);
            counted = true;
          }
          if (atomicCAS(head, h, h + 1) == h) {
            // the producer reserved the slot before writing it: wait for the entry
            for (int s2 = 0;; ++s2) {
              e = (long long)lds_ld(&c.bq[h]);
              if (e != kQEmpty) break;
              if ((s2 & 255) == 255 && wall_clock64() - t0 > 400000000ull) break;
            }
            state = e == kQEmpty ? 3 : 1;
            atomicAdd(&c.bqc[4], 1);
            break;
          }
          continue;
        }
        if (counted) {
          atomicSub(busy, 1);
          counted = false;
          continue;
        }
        if (lds_ld(busy) == 0) {
          if (lds_ld(head) >= min(lds_ld(tail), kBlockQ)) {
            state = 2;
            break;
          }
          continue;
        }
        __builtin_amdgcn_s_sleep(1);
        if ((spin & 255) == 255 && wall_clock64() - t0 > 400000000ull) {
          state = 3;
          break;
        }
      }
      if (state == 3) aor(&a.ctl->status, (unsigned)KC_ERR_TIMEOUT);
    }
    state = __shfl(state, 0, 64);
    if (state != 1) return;
    e = __shfl(e, 0, 64);
    if (e == kQSkip) continue;
    expand_span<S, H, CH>(a, c, o, (long long)((unsigned long long)e >> 16), e & 0xffff, k);
    drain_local<S, H, CH>(a, c, o, k);
  }
}

// Async phase, dynamic part: each wave claims one queue slot at a time, waits until the slot is
// filled or the phase is quiescent, and peels what it holds (a whole row or a hub tile), together
// with the local chain it starts. Quiescent = every workgroup finished its static share and every
// created entry is done; done is counted after an entry's pushes, so when done equals the tail
// (read after done) nothing is left in flight and nothing more can be created. Only wave 0 of a
// workgroup polls those shared counters (and publishes the outcome in LDS for its siblings), so
// waiting waves do not slow down the atomics of working ones. Waits are bounded.
template <bool S, bool H, bool CH>
__device__ __forceinline__ void async_loop(const PeelArgs& a, WaveCtx& c, const PhaseOut& o, uint32_t k,
                                           volatile int* s_quiet) {
  PhaseSlot* PS = o.slot;
  const unsigned nb = gridDim.x;
  const bool watcher = (threadIdx.x >> 6) == 0;
  for (;;) {
    unsigned long long idx = 0;
    if (lane_id() == 0) idx = aadd(&PS->qhead, 1ull);
    idx = __shfl(idx, 0, 64);
    long long e = kQEmpty;
    int state = 0;  // 0 waiting, 1 got entry, 2 quiescent, 3 error
    if (lane_id() == 0) {
      const unsigned long long t0 = wall_clock64();
      for (int spin = 0;; ++spin) {
        if ((long long)idx < a.qcap) {
          e = ald(&a.aq[idx]);
          if (e != kQEmpty) {
            state = 1;
            break;
          }
        }
        const int q = *s_quiet;
        if (q) {
          state = q;
          break;
        }
        if (watcher) {
          if (ald(&PS->bdone) >= nb) {
            const unsigned long long dn = ald(&PS->qdone);
            const unsigned long long tl = ald(&PS->qtail);
            if (dn == tl && (long long)idx >= (long long)tl) {
              *s_quiet = 2;
              state = 2;
              break;
            }
          }
          if (ald(&a.ctl->status) != 0u) {
            *s_quiet = 3;
            state = 3;
            break;
          }
        }
        __builtin_amdgcn_s_sleep(2);
        if ((spin & 255) == 255 && wall_clock64() - t0 > 400000000ull) {
          aor(&a.ctl->status, (unsigned)KC_ERR_TIMEOUT);
          *s_quiet = 3;
          state = 3;
          break;
        }
      }
    }
    state = __shfl(state, 0, 64);
    if (state != 1) return;
    e = __shfl(e, 0, 64);
    if (lane_id() == 0) ast(&a.aq[idx], kQEmpty);  // slots start empty in every async phase
    const int32_t v = (int32_t)(e & 0xffffffffll);
    const uint32_t j = (uint32_t)((unsigned long long)e >> 32);
    c.lq_used = 0;
    if (j == kWholeRow)
      expand_rows<S, H, CH>(a, c, o, lane_id() == 0 ? v : -1, k);
    else
      expand_tile<S, H, CH>(a, c, o, v, (int32_t)j, k);
    if (CH) drain_local<S, H, CH>(a, c, o, k);
    __builtin_amdgcn_s_waitcnt(0);
    if (lane_id() == 0) aadd(&PS->qdone, 1ull);
  }
}

enum PhaseKind { PH_SCAN = 0, PH_EXPAND = 1, PH_ASYNC = 2, PH_RESIDUAL = 3, PH_TAIL = 4, PH_SAMPLE = 5 };

template <bool S, bool H, bool CH>
__global__ __launch_bounds__(kPeelThreads, 2) void peel_kernel(PeelArgs a) {
  __shared__ int32_t s_sf[kWaves][kStage];
  __shared__ int32_t s_sa[kWaves][kStage];
  __shared__ int32_t s_lq[kWaves][kLocalQ];
  __shared__ unsigned long long s_cnt[kWaves];
  __shared__ unsigned long long s_base;
  __shared__ unsigned s_red[kWaves];
  __shared__ long long s_red64[kWaves];
  __shared__ long long s_out[8];
  __shared__ int s_quiet;
  __shared__ int32_t s_ckey[kCombSlots];
  __shared__ uint32_t s_ccnt[kCombSlots];
  __shared__ unsigned long long s_bq[kBlockQ];
  __shared__ int s_bqc[8];
  __shared__ int s_apref[kMaxPeelBlocks + 1];  // segment prefix of the current active list
  __shared__ int s_anew;                        // survivors this workgroup appended in this phase
  __shared__ long long s_hlen[kBucketSlots];    // entries in each bucket slot (multi-bucket mode)

  const int w = threadIdx.x >> 6;
  const int l = lane_id();
  // wave order interleaves workgroups, so a short list (a small active set or frontier) is spread
  // over every workgroup, and with it the hub tiles their workgroup queues take
  const long long gw = (long long)w * gridDim.x + blockIdx.x;
  const long long W = (long long)gridDim.x * kWaves;
  const long long gt = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long GT = (long long)gridDim.x * blockDim.x;
  PeelCtl* C = a.ctl;
  const int64_t n = a.n;

  WaveCtx c;
  c.sf.buf = s_sf[w];
  c.sf.cnt = 0;
  c.sa.buf = s_sa[w];
  c.sa.cnt = 0;
  c.lq = s_lq[w];
  c.lq_head = 0;
  c.lq_cnt = 0;
  c.lq_used = 0;
  c.edges = c.decr = c.scanned = c.peeled = c.comb = c.binserts = 0;
  c.hbs = false;
  c.hlen = s_hlen;
  if (threadIdx.x < kBucketSlots) s_hlen[threadIdx.x] = 0;
  c.mymin = 0xffffffffu;
  c.ckey = s_ckey;
  c.ccnt = s_ccnt;
  for (int i = threadIdx.x; i < kCombSlots; i += kPeelThreads) {
    s_ckey[i] = -1;
    s_ccnt[i] = 0;
  }
  c.bq = s_bq;
  c.bqc = s_bqc;
  c.bq_open = false;
  if (threadIdx.x == 0) s_anew = 0;
  c.adj = a.adj;
  c.rows = reinterpret_cast<const long long*>(a.off);
  c.rstride = 1;
  c.resid = false;
  for (int i = threadIdx.x; i < kBlockQ; i += kPeelThreads) s_bq[i] = (unsigned long long)kQEmpty;
  if (threadIdx.x < 8) s_bqc[threadIdx.x] = threadIdx.x == 2 ? kWaves : 0;

  unsigned epoch = 0;
  long long st_rounds = 0, st_sub = 0, st_bar = 0;
  uint32_t kmax_seen = 0;

  // ---- phase 0: induced degree = degree (Alg. 1 initialisation), hub flags, min degree
  {
    // the workspace was sized for at most m_bound entries: a larger offsets[n] stops the run at the
    // first barrier, before any adjacency entry is read
    if (gt == 0 && a.off[n] > a.m_bound) aor(&C->status, (unsigned)KC_ERR_OVERFLOW);
    const long long nw = (n + 15) >> 4;
    unsigned mn = 0xffffffffu;
    for (long long wd = gt; wd < nw; wd += GT) {
      uint32_t bits = 0;
      for (int j = 0; j < 16; ++j) {
        const long long v = wd * 16 + j;
        if (v >= n) break;
        const long long d = a.off[v + 1] - a.off[v];
        const bool hub = d >= (long long)a.hub;        // rows split into tiles when peeled
        bool hot = d >= (long long)a.comb_degree;      // decrements combined in LDS
        uint32_t sbit = 0u;
        if constexpr (S) {
          // InitSampler (Alg. 5) at k = 0: sample mode for degrees above the threshold; the hot
          // bit then marks sampled vertices (there is no LDS combining in this mode)
          hot = d > (long long)a.s_threshold;
          if (hot) {
            const uint32_t thr = sample_rate32(a.s_mu, (uint32_t)d);
            ast(&a.srate[v], thr);
            ast(&a.scnt[v], 0u);
            ast(&a.sbase[v], (uint32_t)d);
            const uint32_t slot = aadd(&C->s_ncand, 1u);
            ast(&a.scand[slot], (int32_t)v);
            const uint32_t kb = sample_valk((uint32_t)d, thr, 0u, a.s_mu);
            if (kb < ald(&C->s_valk)) amin(&C->s_valk, kb);
            sbit = SAMPLEBIT;
          }
        }
        ast(&a.dt[v], (uint32_t)d | (hub ? HUBBIT : 0u) | sbit);
        if (H && a.hlo) ast(&a.hlo[v], 0u);  // filed nowhere yet
        bits |= (hot ? 1u : 0u) << (16 + j);
        mn = min(mn, (unsigned)d);
      }
      ast(&a.state[wd], bits);
    }
    mn = wave_min(mn);
    if (l == 0) s_red[w] = mn;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned m = 0xffffffffu;
      for (int i = 0; i < kWaves; ++i) m = min(m, s_red[i]);
      if (m < ald(&C->slot[0].minv)) amin(&C->slot[0].minv, m);
    }
  }
  if (!grid_sync<!CH>(C, epoch)) return;
  st_bar++;

  if (threadIdx.x == 0) {
    s_out[0] = (long long)ald(&C->slot[0].minv);
    s_out[5] = (long long)ald(&C->s_valk);
  }
  __syncthreads();
  // round being extracted or expanded; a k-core query runs the single round k - 1
  long long kx = a.k_query > 0 ? a.k_query - 1 : s_out[0];
  int kind = PH_SCAN;
  if constexpr (S) {
    // sampled vertices due for validation at the first round are validated before its scan
    if (s_out[5] <= kx) kind = PH_SAMPLE;
  }
  __syncthreads();
  bool dense = true, compact = false;
  long long asize = n;   // items of the current active list
  long long aseg = 0;    // its segment length (segmented lists)
  int acur = 0;
  const int nb = (int)gridDim.x;
  long long removed_since = 0, total_peeled = 0;
  long long fs = 0, ft = 0;
  // the rows are rewritten once the active set is at most this large (-1: done, or never); a
  // rewrite called off for lack of room is tried again when the active set has halved
  long long resid_limit = a.resid_vmax;
  // the live vertices go to the tail peel once at most this many remain (-1: never); a handoff
  // called off for lack of room is tried again when half as many remain
  long long tail_limit = a.k_query > 0 ? -1 : a.tail_vmax;
  const long long max_phases = 4 * n + 64;
  // multi-bucket active set: on from the round it starts at; hk = the round the buckets are
  // relative to; hscan = the slot the current scan reads (-1: the active list, when it starts)
  bool hbs_on = false;
  uint32_t hk = 0;
  int hscan = -1;

  for (long long p = 1;; ++p) {
    if (p > max_phases) {
      if (threadIdx.x == 0) aor(&C->status, (unsigned)KC_ERR_PHASES);
      break;
    }
    PhaseOut o;
    o.slot = &C->slot[p % 3];
    o.fr = a.fr[p & 1];
    o.tl = a.tl[p & 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      PhaseSlot* r = &C->slot[(p + 1) % 3];
      ast(&r->small, 0ull);
      ast(&r->tiles, 0ull);
      ast(&r->hubv, 0ull);
      ast(&r->active, 0ull);
      ast(&r->peeled, 0ull);
      ast(&r->qhead, 0ull);
      ast(&r->qtail, 0ull);
      ast(&r->qdone, 0ull);
      ast(&r->bdone, 0u);
      ast(&r->minv, 0xffffffffu);
    }
    if (blockIdx.x == 0 && threadIdx.x < kBucketSlots) ast(&C->slot[(p + 1) % 3].hadd[threadIdx.x], 0ull);
    const uint32_t k = (uint32_t)kx;
    const bool tr = blockIdx.x == 0 && threadIdx.x == 0 && p < kTracePhases;
    if (tr) C->trace[p][0] = wall_clock64();
    const bool dbg = threadIdx.x == 0 && blockIdx.x < kDbgBlocks && p >= a.dbg_lo && p < a.dbg_lo + kDbgPhases;
    if (dbg) C->dbg[p - a.dbg_lo][blockIdx.x][0] = wall_clock64();
    if constexpr (S) {
      if (kind == PH_SAMPLE) {
        // Validation and recounts of the sampled vertices at the start of round kx (Alg. 4's loop
        // over sample-mode vertices, Error and SetSampler of Alg. 5). Every expansion has landed,
        // so a live neighbour is one whose peeled bit is clear. (1) Check each sampled vertex;
        // those that fail are marked (rate 0) and their row tiles listed; (2) count the live
        // entries of each listed tile; (3) re-initialise each recounted vertex (InitSampler) or
        // return it to exact counting, and collect the round of the next validation.
        PhaseSlot* slot = o.slot;
        const long long ncand = (long long)ald(&C->s_ncand);
        if (blockIdx.x == 0 && threadIdx.x == 0) ast(&C->s_valk, 0xffffffffu);  // rebuilt in (3)
        for (long long i0 = gw * 64; i0 < ncand; i0 += W * 64) {
          const long long i = i0 + l;
          int32_t v = -1;
          bool redo = false;
          long long nt = 0;
          if (i < ncand) {
            v = ald(&a.scand[i]);
            const uint32_t thr = ald(&a.srate[v]);
            if (thr != 0u && !sample_safe(ald(&a.sbase[v]), thr, ald(&a.scnt[v]), k)) {
              redo = true;
              ast(&a.srate[v], 0u);
              ast(&a.scount[v], 0u);
              nt = (a.off[v + 1] - a.off[v] + a.tile - 1) / a.tile;
            }
          }
          const unsigned long long rm = __ballot(redo);
          if (rm == 0) continue;
          unsigned long long rbase = 0;
          if (l == 0) rbase = aadd(&slot->small, (unsigned long long)__popcll(rm));
          rbase = __shfl(rbase, 0, 64);
          const long long tincl = wave_incl_scan(nt);
          const long long ttot = __shfl(tincl, 63, 64);
          unsigned long long tbase = 0;
          if (l == 0 && ttot) tbase = aadd(&slot->tiles, (unsigned long long)ttot);
          tbase = __shfl(tbase, 0, 64);
          if ((long long)tbase + ttot > a.qcap) {
            if (l == 0) aor(&C->status, (unsigned)KC_ERR_OVERFLOW);
          } else if (redo) {
            ast(&a.srl[rbase + rank_in(rm)], v);
            const long long t0 = (long long)tbase + tincl - nt;
            for (long long j = 0; j < nt; ++j)
              ast(&a.aq[t0 + j], (long long)(((unsigned long long)j << 32) | (unsigned)v));
          }
        }
        if (!grid_sync<!CH>(C, epoch)) break;
        st_bar++;
        if (threadIdx.x == 0) {
          s_out[0] = (long long)ald(&slot->tiles);
          s_out[1] = (long long)ald(&slot->small);
        }
        __syncthreads();
        const long long ntl = s_out[0] <= a.qcap ? s_out[0] : a.qcap;
        const long long nrl = s_out[1];
        __syncthreads();
        // (2) live entries of each listed tile
        for (long long it = gw; it < ntl; it += W) {
          const long long e = ald(&a.aq[it]);
          const int32_t v = (int32_t)(e & 0xffffffffll);
          const long long j = (long long)((unsigned long long)e >> 32);
          const long long ob = a.off[v], oe = a.off[v + 1];
          const long long b = ob + j * a.tile, en = min(oe, b + a.tile);
          int cnt = 0;
          for (long long q = b + l; q < en; q += 64) {
            const int32_t u = a.adj[q];
            cnt += ((ald(&a.state[u >> 4]) >> (u & 15)) & 1u) ? 0 : 1;
          }
          for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
          if (l == 0) {
            if (cnt) aadd(&a.scount[v], (uint32_t)cnt);
            ast(&a.aq[it], kQEmpty);  // the async queue starts every phase empty
          }
        }
        if (!grid_sync<!CH>(C, epoch)) break;
        st_bar++;
        // (3) InitSampler for the recounted vertices; the others report their next validation
        for (long long i = gt; i < nrl; i += GT) {
          const int32_t v = ald(&a.srl[i]);
          const uint32_t cnt = ald(&a.scount[v]);
          const uint32_t hubf = (a.off[v + 1] - a.off[v]) >= (long long)a.hub ? HUBBIT : 0u;
          if (cnt < k) {
            // live at the start of round k with fewer than k live neighbours: it should have been
            // peeled in an earlier round (the rare failure of the sampling scheme)
            aor(&C->status, (unsigned)KC_ERR_SAMPLE);
          } else if ((unsigned long long)cnt > 10ull * k && cnt > a.s_threshold) {
            const uint32_t thr = sample_rate32(a.s_mu, cnt);
            ast(&a.sbase[v], cnt);
            ast(&a.scnt[v], 0u);
            ast(&a.srate[v], thr);
            ast(&a.dt[v], cnt | hubf | SAMPLEBIT);
            const uint32_t kb = max(sample_valk(cnt, thr, 0u, a.s_mu), k + 1u);
            amin(&C->s_valk, kb);
          } else {
            ast(&a.dt[v], cnt | hubf);
            __hip_atomic_fetch_and(&a.state[v >> 4], ~(1u << (16 + (v & 15))), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
          }
          aadd(&C->stats[ST_RECOUNTS], 1ull);
        }
        for (long long i = gt; i < ncand; i += GT) {
          const int32_t v = ald(&a.scand[i]);
          const uint32_t thr = ald(&a.srate[v]);
          if (thr == 0u) continue;
          const uint32_t kb = max(sample_valk(ald(&a.sbase[v]), thr, ald(&a.scnt[v]), a.s_mu), k + 1u);
          if (kb < ald(&C->s_valk)) amin(&C->s_valk, kb);
        }
        if (tr) {
          C->trace[p][1] = C->trace[p][2] = wall_clock64();
          C->trace[p][4] = (unsigned long long)PH_SAMPLE | ((unsigned long long)k << 8);
          C->trace[p][5] = (unsigned long long)nrl;
          C->trace[p][6] = (unsigned long long)ntl;
          C->trace[p][7] = (unsigned long long)asize;
        }
        if (!grid_sync<!CH>(C, epoch)) break;
        st_bar++;
        if (tr) C->trace[p][3] = wall_clock64();
        kind = PH_SCAN;
        continue;
      }
    }
    if (kind == PH_RESIDUAL || kind == PH_TAIL) {
      // Rewrites the rows of the live vertices without their peeled neighbours. It runs at a round
      // boundary: every decrement has landed, so a live vertex's induced degree is its number of
      // live neighbours and sizes its new row exactly. (1) Reserve the new rows and list the tiles
      // of the current ones; (2) copy the live neighbours of each tile to the new row (order within
      // a row is free). When the new rows do not fit their buffer the rewrite is called off after
      // (1) and nothing changes.
      //  * PH_RESIDUAL (once): the grid goes on peeling from the new rows, whose hub flags follow
      //    the new row lengths.
      //  * PH_TAIL: hands the live vertices to the single-workgroup tail peel. At a round boundary
      //    they form the kx-core, and a vertex of the kx-core has the same coreness in it as in the
      //    whole graph, so the tail peel needs only this subgraph: the live vertices are numbered
      //    0..L-1 in (1), and (2) writes their rows in those local ids. The grid then stops.
      const bool to_tail = kind == PH_TAIL;
      long long* nrow = to_tail ? a.trow : a.rrow;
      int32_t* nadj = a.radj;  // (the tail's rows are 16-bit local ids in a.tadj)
      const long long ncap = to_tail ? a.tail_ecap : a.rcap;
      PhaseSlot* slot = o.slot;
      const int32_t* alist = a.act[acur];
      for (long long i0 = gw * 64; i0 < asize; i0 += W * 64) {
        const long long i = i0 + l;
        int32_t v = -1;
        if (i < asize) v = active_item(alist, dense, i, aseg, s_apref, nb);
        bool live = false;
        long long len = 0, nt = 0;
        if (v >= 0) {
          live = !((ald(&a.state[v >> 4]) >> (v & 15)) & 1u);
          if (live) {
            long long ob = 0, od = 0;
            row_of(a, c, v, ob, od);
            len = ald(&a.dt[v]) & DMASK;
            nt = (od + a.tile - 1) / a.tile;
          }
        }
        const unsigned long long lm = __ballot(live);
        if (lm == 0) continue;
        unsigned long long vbase = 0;
        if (l == 0 && to_tail) vbase = aadd(&slot->active, (unsigned long long)__popcll(lm));
        vbase = __shfl(vbase, 0, 64);
        // local rows start on 16-byte boundaries (lengths padded to 8 16-bit entries with 0xffff)
        // so that the tail peel streams them with 16-byte loads
        const long long rlen = to_tail ? (len + 7) & ~7ll : len;
        const long long incl = wave_incl_scan(rlen);
        const long long tot = __shfl(incl, 63, 64);
        unsigned long long base = 0;
        if (l == 0 && tot) base = aadd(&slot->small, (unsigned long long)tot);
        base = __shfl(base, 0, 64);
        const long long tincl = wave_incl_scan(nt);
        const long long ttot = __shfl(tincl, 63, 64);
        unsigned long long tbase = 0;
        if (l == 0 && ttot) tbase = aadd(&slot->tiles, (unsigned long long)ttot);
        tbase = __shfl(tbase, 0, 64);
        if ((long long)base + tot > ncap || (long long)tbase + ttot > a.qcap ||
            (to_tail && (long long)(vbase + __popcll(lm)) > a.tail_vmax)) {
          if (l == 0) ast(&slot->hubv, 1ull);  // the new rows do not fit: called off
        } else if (live) {
          long long r = v;  // new row index: the vertex, or its local id
          if (to_tail) {
            r = (long long)vbase + rank_in(lm);
            ast(&a.tmap[v], (int32_t)r);
            ast(&a.tgid[r], v);
          }
          const long long rb = (long long)base + incl - rlen;
          ast(&nrow[2 * r], rb);      // first entry
          ast(&nrow[2 * r + 1], rb);  // fill cursor, the row's end once filled
          for (long long x = rb + len; x < rb + rlen; ++x) a.tadj[x] = 0xffffu;
          const long long t0 = (long long)tbase + tincl - nt;
          for (long long j = 0; j < nt; ++j)
            ast(&a.aq[t0 + j], (long long)(((unsigned long long)j << 32) | (unsigned)v));
        }
      }
      if (!grid_sync<!CH>(C, epoch)) break;
      st_bar++;
      if (threadIdx.x == 0) {
        s_out[0] = (long long)ald(&slot->tiles);
        s_out[1] = (long long)ald(&slot->hubv);
        s_out[2] = (long long)ald(&slot->active);
      }
      __syncthreads();
      const long long ntl = s_out[0] <= a.qcap ? s_out[0] : a.qcap;
      const bool called_off = s_out[1] != 0;
      const long long nlive = s_out[2];
      __syncthreads();
      for (long long it = gw; it < ntl; it += W) {
        const long long e = ald(&a.aq[it]);
        if (called_off) {
          // entries past a refused reservation were never written: clear every slot
          if (l == 0) ast(&a.aq[it], kQEmpty);
          continue;
        }
        const int32_t v = (int32_t)(e & 0xffffffffll);
        const long long j = (long long)((unsigned long long)e >> 32);
        long long ob = 0, od = 0;
        row_of(a, c, v, ob, od);
        const long long b = ob + j * a.tile, en = min(ob + od, b + a.tile);
        const long long len = (long long)(ald(&a.dt[v]) & DMASK);
        const long long r = to_tail ? (long long)ald(&a.tmap[v]) : (long long)v;
        const long long lim = ald(&nrow[2 * r]) + len;
        // hub flag for the new row length (only the flag bit changes)
        if (!to_tail && j == 0 && l == 0) ast(&a.dt[v], (uint32_t)len | (len >= (long long)a.hub ? HUBBIT : 0u));
        // 256 entries per pass: all loads, then all probes, then one reservation for the pass
        for (long long p0 = b; p0 < en; p0 += 64 * kTileUnroll) {
          int32_t u[kTileUnroll];
          uint32_t sw[kTileUnroll];
#pragma unroll
          for (int q = 0; q < kTileUnroll; ++q) {
            const long long x = p0 + 64 * q + l;
            u[q] = x < en ? c.adj[x] : -1;
          }
#pragma unroll
          for (int q = 0; q < kTileUnroll; ++q) sw[q] = u[q] >= 0 ? ald(&a.state[u[q] >> 4]) : 1u;
          unsigned long long mk[kTileUnroll];
          int cnt = 0;
#pragma unroll
          for (int q = 0; q < kTileUnroll; ++q) {
            const bool lv = u[q] >= 0 && !((sw[q] >> (u[q] & 15)) & 1u);
            // entries to peeled neighbours are done with here (they count as expanded)
            c.edges += (u[q] >= 0 && !lv) ? 1 : 0;
            if (lv && to_tail) u[q] = ald(&a.tmap[u[q]]);
            mk[q] = __ballot(lv);
            cnt += __popcll(mk[q]);
          }
          if (cnt == 0) continue;
          long long pos = 0;
          if (l == 0)
            pos = (long long)aadd(reinterpret_cast<unsigned long long*>(&nrow[2 * r + 1]),
                                  (unsigned long long)cnt);
          pos = __shfl(pos, 0, 64);
          if (pos + cnt > lim) {
            if (l == 0) aor(&C->status, (unsigned)KC_ERR_OVERFLOW);
            continue;
          }
#pragma unroll
          for (int q = 0; q < kTileUnroll; ++q) {
            if ((mk[q] >> l) & 1ull) {
              // (the tail kernel, a later launch, is the only reader of the tail's rows)
              if (to_tail)
                a.tadj[pos + rank_in(mk[q])] = (uint16_t)u[q];
              else
                ast(&nadj[pos + rank_in(mk[q])], u[q]);
            }
            pos += __popcll(mk[q]);
          }
        }
        if (l == 0) ast(&a.aq[it], kQEmpty);  // the async queue starts every phase empty
      }
      if (tr) {
        C->trace[p][1] = C->trace[p][2] = wall_clock64();
        C->trace[p][4] = (unsigned long long)kind | ((unsigned long long)k << 8);
        C->trace[p][5] = C->trace[p][6] = 0;
        C->trace[p][7] = (unsigned long long)asize;
      }
      if (!grid_sync<!CH>(C, epoch)) break;
      st_bar++;
      if (tr) C->trace[p][3] = wall_clock64();
      if (to_tail) {
        if (!called_off) {
          if (blockIdx.x == 0 && threadIdx.x == 0) {
            ast(&C->tail_k, (unsigned long long)kx);
            ast(&C->tail_n, (unsigned long long)nlive);
          }
          break;
        }
        tail_limit = (n - total_peeled) / 2;
      } else if (!called_off) {
        c.resid = true;
        c.adj = a.radj;
        c.rows = a.rrow;
        c.rstride = 2;
        resid_limit = -1;
      } else {
        const long long aset = hbs_on ? n - total_peeled : asize;
        resid_limit = aset / 2 > 0 ? aset / 2 : -1;
      }
      kind = PH_SCAN;
      continue;
    }
    c.lq_used = 0;
    if (H && kind == PH_SCAN && a.hbs_vmax > 0) {
      if (!hbs_on && kx >= (long long)kBucketMinK && n - total_peeled <= a.hbs_vmax) {
        // the multi-bucket set starts: this scan files every live vertex of the active list
        // (frozen from now on; the row rewrite and the tail handoff still read it, with the
        // peeled bits telling which entries are live)
        hbs_on = true;
        hscan = -1;
        hk = (uint32_t)kx;
        compact = false;
        if (threadIdx.x < kBucketSlots) s_hlen[threadIdx.x] = 0;
        __syncthreads();
      } else if (hbs_on && (uint32_t)kx != hk) {
        // a new round: read the bucket that holds kx; the buckets below it held only values
        // below kx (every such vertex is peeled) and start empty
        hscan = hbs_bucket((uint32_t)kx, hk);
        hk = (uint32_t)kx;
        if (threadIdx.x < hscan) s_hlen[threadIdx.x] = 0;
        __syncthreads();
      }
    }
    c.hbs = hbs_on;
    // the list a scan reads: the active list, or (multi-bucket mode) one bucket slot
    const bool hb_list = kind == PH_SCAN && hbs_on && hscan >= 0;
    // (a slot that overflowed has already stopped the run at the barrier; never read past it)
    const long long slen = hb_list ? min(s_hlen[hscan], (long long)a.hcap) : asize;
    // large phases are bandwidth bound: probe peeled bits and combine hub decrements; small ones
    // are latency bound: skip the probe and spread the frontier over as many waves as possible
    c.precheck = kind == PH_SCAN ? slen >= a.big_phase * 16 : (fs + ft * (a.tile / 16)) >= a.big_phase;
    // chained mode folds the round's whole peel into its scan phase once the active set is small
    const bool async_scan = kind == PH_SCAN && CH && !hbs_on && asize <= a.async_scan_max;
    // deferred (combined) decrements would hide work from the async quiescence test
    c.async = kind == PH_ASYNC || async_scan;
    c.combine = c.precheck && !c.async;
    c.arbitrate = kind == PH_SCAN && CH;
    c.bq_open = CH && a.bq_max_tiles > 0 && !c.async;
    if (tr) {
      C->trace[p][4] = (unsigned long long)kind | (c.precheck ? 16ull : 0ull) | (c.async ? 32ull : 0ull) |
                       ((unsigned long long)k << 8);
      C->trace[p][5] = (unsigned long long)fs;
      C->trace[p][6] = (unsigned long long)ft;
      C->trace[p][7] = (unsigned long long)slen;
    }
    long long peeled_before = c.peeled;
    if (kind == PH_SCAN) {
      // Alg. 1: F = {v in A : induced degree <= k}; survivors refine A (or, in multi-bucket
      // mode, move to the bucket of their induced degree: GetNextBucket of Sec. 5.2).
      int32_t* alist = a.act[acur];
      const int32_t* hlist = hb_list ? a.hbl + (long long)hscan * a.hcap : nullptr;
      // this workgroup's segment of the next list: at most the items it scans (64-entry chunks
      // dealt round-robin over workgroups)
      const long long nseg = 64 * (((asize + 63) / 64 + nb - 1) / nb);
      int32_t* myseg = a.act[acur ^ 1] + (long long)blockIdx.x * nseg;
      for (long long i0 = gw * 64; i0 < slen; i0 += W * 64) {
        const long long i = i0 + l;
        const bool valid = i < slen;
        int32_t v = -1;
        if (valid) v = hb_list ? ald(&hlist[i]) : active_item(alist, dense, i, aseg, s_apref, nb);
        uint32_t word = 0, x = 0, tag = 0;
        bool alive = false;
        if (valid) {
          // (multi-bucket mode: the tag is read before the induced degree, see hbs_file)
          if (hbs_on) tag = ald(&a.hlo[v]);
          // liveness comes from the peeled bit, not from the induced degree: in chained mode a
          // chain of this round may already have taken a vertex due for extraction below k
          const uint32_t sw = ald(&a.state[v >> 4]);
          word = ald(&a.dt[v]);
          x = word & DMASK;
          alive = !((sw >> (v & 15)) & 1u);
          c.scanned += 1;
        }
        bool ext = alive && (long long)x <= kx;
        const bool keep = alive && (long long)x > kx;
        if (keep) c.mymin = min(c.mymin, x);
        if (compact) seg_push(c.sa, keep, v, myseg, &s_anew);
        if (hbs_on) hbs_file(a, c, o, keep, v, x, tag, (uint32_t)kx);
        if (ext) {
          const uint32_t bit = 1u << (v & 15);
          if (aor(&a.state[v >> 4], bit) & bit) {
            ext = false;  // already peeled in this round by a chain (chained mode)
          } else {
            if (a.k_query <= 0) put_core(a.core, v, k, &C->status);
            c.peeled += 1;
          }
        }
        push_vertices<CH>(a, c, o, ext, v, (word & HUBBIT) != 0u);
      }
    } else {
      // Alg. 3 over the frontier: packets of small vertices, then hub tiles (the static share of
      // an async phase is the same).
      const int32_t* fcur = a.fr[(p - 1) & 1];
      const unsigned long long* tcur = a.tl[(p - 1) & 1];
      int per = 64;  // frontier vertices per wave item: fewer when the frontier is small
      while (per > 1 && (fs + per - 1) / per < W) per >>= 1;
      const long long npk = (fs + per - 1) / per;
      const long long items = npk + ft;
      for (long long it = gw; it < items; it += W) {
        if (it < npk) {
          const long long i = it * per + l;
          const int32_t v = (l < per && i < fs) ? ald(&fcur[i]) : -1;
          expand_rows<S, H, CH>(a, c, o, v, k);
        } else {
          const unsigned long long sw = ald(&tcur[it - npk]);
          expand_span<S, H, CH>(a, c, o, (long long)(sw >> 16), (long long)(sw & 0xffff), k);
        }
      }
    }
    if (CH) drain_local<S, H, CH>(a, c, o, k);
    if (c.bq_open) {
      block_loop<S, H, CH>(a, c, o, k);
      c.bq_open = false;
    }
    if (CH && c.async) {
      if (threadIdx.x == 0) s_quiet = 0;
      __syncthreads();
      if (threadIdx.x == 0) {
        __builtin_amdgcn_s_waitcnt(0);
        aadd(&o.slot->bdone, 1u);
      }
      // a few waves per workgroup take part in the dynamic part: every claim is an atomic on one
      // shared counter, so thousands of claimers would serialise there
      if ((threadIdx.x >> 6) < kAsyncWaves) async_loop<S, H, CH>(a, c, o, k, &s_quiet);
    }
    comb_flush<H, CH>(a, c, o, k);
    // every wave has left the tile queue (comb_flush starts with a workgroup barrier): reset it for
    // the next phase; the barriers of the flushes below order this before its next use
    for (int i = threadIdx.x; i < kBlockQ; i += kPeelThreads) s_bq[i] = (unsigned long long)kQEmpty;
    if (threadIdx.x < 4) s_bqc[threadIdx.x] = threadIdx.x == 2 ? kWaves : 0;
    if (CH) drain_local<S, H, CH>(a, c, o, k);
    if (tr) C->trace[p][1] = wall_clock64();
    if (dbg) C->dbg[p - a.dbg_lo][blockIdx.x][1] = wall_clock64();

    // ---- phase end: block-level flushes and reductions
    block_flush(c.sf, &o.slot->small, o.fr, a.fcap, &C->status, s_cnt, &s_base);
    if (kind == PH_SCAN && compact) {
      const long long nseg = 64 * (((asize + 63) / 64 + nb - 1) / nb);
      seg_flush(c.sa, a.act[acur ^ 1] + (long long)blockIdx.x * nseg, &s_anew);
      __syncthreads();
      if (threadIdx.x == 0) {
        ast(&C->acnt[acur ^ 1][blockIdx.x], (unsigned)s_anew);
        if (s_anew) aadd(&o.slot->active, (unsigned long long)s_anew);
        s_anew = 0;
      }
    }
    {
      const unsigned mn = wave_min(c.mymin);
      long long pc = c.peeled - peeled_before;
      for (int off = 32; off > 0; off >>= 1) pc += __shfl_xor(pc, off, 64);
      if (l == 0) {
        s_red[w] = mn;
        s_red64[w] = pc;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        unsigned m = 0xffffffffu;
        long long tp = 0;
        for (int i = 0; i < kWaves; ++i) {
          m = min(m, s_red[i]);
          tp += s_red64[i];
        }
        if (m != 0xffffffffu && m < ald(&o.slot->minv)) amin(&o.slot->minv, m);
        if (tp) aadd(&o.slot->peeled, (unsigned long long)tp);
      }
      c.mymin = 0xffffffffu;
    }
    if (tr) C->trace[p][2] = wall_clock64();
    if (threadIdx.x == 0) {
      // the flushes above end with a workgroup barrier: the phase's counts are complete
      if (dbg) {
        C->dbg[p - a.dbg_lo][blockIdx.x][2] = (unsigned long long)s_bqc[4];
        C->dbg[p - a.dbg_lo][blockIdx.x][3] = (unsigned long long)s_bqc[5];
      }
      s_bqc[4] = 0;
      s_bqc[5] = 0;
    }
    if (!grid_sync<!CH>(C, epoch)) break;
    st_bar++;
    if (tr) C->trace[p][3] = wall_clock64();

    // ---- decide the next phase (identical in every workgroup); one thread reads the outcome
    if (threadIdx.x == 0) {
      s_out[0] = (long long)ald(&o.slot->small);
      s_out[1] = (long long)ald(&o.slot->tiles);
      s_out[2] = (long long)ald(&o.slot->active);
      s_out[3] = (long long)ald(&o.slot->minv);
      s_out[4] = (long long)ald(&o.slot->peeled);
      if constexpr (S) s_out[5] = (long long)ald(&C->s_valk);
    }
    __syncthreads();
    const long long nfs = s_out[0];
    const long long nft = s_out[1];
    const long long nact = s_out[2];
    const unsigned mv = (unsigned)s_out[3];
    const long long npeel = s_out[4];
    const long long valk = S ? s_out[5] : (long long)0xffffffffu;  // next validation (sampling)
    if (hbs_on) {
      // bucket lengths after the phase (the same in every workgroup); a scanned slot has been
      // redistributed into lower ones and is empty
      if (threadIdx.x < kBucketSlots) {
        s_hlen[threadIdx.x] += (long long)ald(&o.slot->hadd[threadIdx.x]);
        if (hb_list && (int)threadIdx.x == hscan) s_hlen[threadIdx.x] = 0;
      }
    }
    __syncthreads();
    if (nfs > a.fcap || nft > a.tcap || nact > n) {
      // a list overflowed (its entries were not written): stop before reading them
      if (threadIdx.x == 0) aor(&C->status, (unsigned)KC_ERR_OVERFLOW);
      break;
    }
    total_peeled += npeel;
    removed_since += npeel;
    if (kind != PH_SCAN) st_sub++;
    // small frontiers of chained mode are peeled by the async phase
    const bool go_async = CH && nfs <= a.async_small && nft <= a.async_tiles;
    if (npeel > 0) kmax_seen = k;
    if (kind == PH_SCAN && compact) {
      aseg = 64 * (((asize + 63) / 64 + nb - 1) / nb);
      asize = nact;
      acur ^= 1;
      dense = false;
      removed_since = npeel;
      // segment prefix of the new list (every workgroup computes the same one)
      const int b = threadIdx.x;
      const long long cnt = b < nb ? (long long)ald(&C->acnt[acur][b]) : 0;
      const long long incl = wave_incl_scan(cnt);
      if (l == 63) s_red64[w] = incl;
      __syncthreads();
      if (threadIdx.x == 0) {
        long long t = 0;
        for (int i = 0; i < kWaves; ++i) {
          const long long x = s_red64[i];
          s_red64[i] = t;
          t += x;
        }
      }
      __syncthreads();
      if (b < nb) s_apref[b] = (int)(s_red64[w] + incl - cnt);
      if (b == nb - 1) s_apref[nb] = (int)(s_red64[w] + incl);
      __syncthreads();
    }
    if (kind == PH_SCAN) {
      if (npeel > 0) st_rounds++;
      if (nfs + nft > 0) {
        kind = go_async ? PH_ASYNC : PH_EXPAND;
        fs = nfs;
        ft = nft;
      } else if (total_peeled >= n) {
        break;
      } else if (npeel > 0) {
        // the round completed inside the scan (chained mode)
        kx = kx + 1;
        compact = !hbs_on && removed_since * 8 >= asize;
      } else {
        // no live vertex has induced degree <= kx: jump to the smallest one (next non-empty round)
        long long jump = (long long)mv;
        if (hbs_on && mv == 0xffffffffu) {
          // nothing live in the bucket just read: the next round starts at the lowest range that
          // still lists vertices (its entries may all be stale: its scan then moves on again)
          for (int b = 0; b < kBucketSlots; ++b)
            if (s_hlen[b] > 0) {
              jump = (long long)hbs_lo(hk, b);
              break;
            }
        }
        if (jump == 0xffffffffll) {
          if (threadIdx.x == 0) aor(&C->status, (unsigned)KC_ERR_PHASES);
          if (blockIdx.x == 0 && threadIdx.x == 0) {
            ast(&C->stats[kDiagWord], (unsigned long long)total_peeled);
            ast(&C->stats[kDiagWord + 1], (unsigned long long)kx);
            ast(&C->stats[kDiagWord + 2], (unsigned long long)p);
            ast(&C->stats[kDiagWord + 3], (unsigned long long)asize);
          }
          break;
        }
        // (in sampling mode not past the next validation)
        kx = S ? min(jump, max(valk, kx + 1)) : jump;
        compact = false;
      }
    } else {
      if (nfs + nft > 0) {
        kind = go_async ? PH_ASYNC : PH_EXPAND;
        fs = nfs;
        ft = nft;
      } else if (total_peeled >= n) {
        break;
      } else {
        kx = kx + 1;
        kind = PH_SCAN;
        compact = !hbs_on && removed_since * 8 >= asize;
      }
    }
    // a k-core query ends with its one round: the survivors are the k-core
    if (a.k_query > 0 && kind == PH_SCAN) break;
    // sampling mode: sampled vertices due for validation are checked before the round's scan
    if (S && kind == PH_SCAN && valk <= kx) kind = PH_SAMPLE;
    // at a round boundary with few live vertices left: hand them to the tail peel; else, with a
    // small active set whose live rows fit: rewrite the rows once
    if (kind == PH_SCAN && tail_limit > 0 && n - total_peeled <= tail_limit)
      kind = PH_TAIL;
    else if (kind == PH_SCAN && resid_limit >= 0 && (hbs_on ? n - total_peeled : asize) <= resid_limit)
      kind = PH_RESIDUAL;
  }
  if (a.k_query > 0) {
    // membership: every workgroup left the loop after the same barrier, so the peeled bits are final.
    // This is the only write of the output in a query (no coreness is written while peeling): plain
    // stores to one address from workgroups on different XCDs have no defined order.
    for (long long v = gt; v < n; v += GT) a.core[v] = ((ald(&a.state[v >> 4]) >> (v & 15)) & 1u) ? 0 : 1;
  }

  // ---- statistics: per-lane counters reduced per block, one atomic each per block
  {
    long long v4[6] = {c.edges, c.decr, c.scanned, c.peeled, c.comb, c.binserts};
    for (int q = 0; q < 6; ++q) {
      long long x = v4[q];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
      if (l == 0) s_red64[w] = x;
      __syncthreads();
      if (threadIdx.x == 0) {
        long long t = 0;
        for (int i = 0; i < kWaves; ++i) t += s_red64[i];
        const int idx = q == 0 ? ST_EDGES : q == 1 ? ST_DECR : q == 2 ? ST_SCANNED : q == 3 ? ST_PEELED
                      : q == 4 ? ST_COMBINED : ST_BUCKET;
        if (t) aadd(&C->stats[idx], (unsigned long long)t);
      }
      __syncthreads();
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ast(&C->stats[ST_ROUNDS], (unsigned long long)st_rounds);
      ast(&C->stats[ST_SUBROUNDS], (unsigned long long)st_sub);
      ast(&C->stats[ST_BARRIERS], (unsigned long long)st_bar);
      ast(&C->stats[ST_KMAX], (unsigned long long)kmax_seen);
      if (S) ast(&C->stats[ST_SAMPLED], (unsigned long long)ald(&C->s_ncand));
    }
  }
}

hipError_t launch_peel(const PeelArgs& a, int blocks, hipStream_t s) {
  void* args[] = {const_cast<PeelArgs*>(&a)};
  // instances: sampling (always chained), multi-bucket active set, neither; each in a chained and a
  // level-synchronous form (each keeps the others' code out of its registers)
  const void* f = a.sampling ? reinterpret_cast<const void*>(peel_kernel<true, false, true>)
                  : a.hbs_vmax > 0
                      ? (a.chained ? reinterpret_cast<const void*>(peel_kernel<false, true, true>)
                                   : reinterpret_cast<const void*>(peel_kernel<false, true, false>))
                      : (a.chained ? reinterpret_cast<const void*>(peel_kernel<false, false, true>)
                                   : reinterpret_cast<const void*>(peel_kernel<false, false, false>));
  return hipLaunchCooperativeKernel(f, dim3(blocks),
                                    dim3(kPeelThreads), args, 0, s);
}

hipError_t peel_occupancy(int* blocks_per_cu) {
  int b0 = 0, b1 = 0;
  int b2 = 0;
  int b3 = 0, b4 = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b0, peel_kernel<false, false, true>, kPeelThreads, 0);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b1, peel_kernel<true, false, true>, kPeelThreads, 0);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b2, peel_kernel<false, true, true>, kPeelThreads, 0);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b3, peel_kernel<false, false, false>, kPeelThreads, 0);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b4, peel_kernel<false, true, false>, kPeelThreads, 0);
  if (b2 < b1) b1 = b2;
  if (b3 < b1) b1 = b3;
  if (b4 < b1) b1 = b4;
  *blocks_per_cu = b0 < b1 ? b0 : b1;
  return e;
}


// ------------------------------------------------------------------------------------------
// Batched peel: one workgroup per graph, graphs claimed largest-first from a shared counter.
// Induced degrees and the peel queue live in LDS when the graph fits (lds_cap vertices), else in
// the global workspace at the graph's own vertex range; either way only this workgroup touches
// them, so decrements are workgroup-scope atomics and every (sub)round ends at __syncthreads.
// The queue holds vertices in peel order; since each vertex is peeled once, n slots suffice and
// the current frontier is always the queue segment between two marks.
// ------------------------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T wsub(T* p, T v) {
  return __hip_atomic_fetch_sub(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ long long block_excl_scan(long long x, long long* s_w, long long& total) {
  const int w = threadIdx.x >> 6, l = lane_id();
  const long long incl = wave_incl_scan(x);
  if (l == 63) s_w[w] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int i = 0; i < kBatchThreads / 64; ++i) {
      const long long c = s_w[i];
      s_w[i] = t;
      t += c;
    }
    s_w[kBatchThreads / 64] = t;
  }
  __syncthreads();
  total = s_w[kBatchThreads / 64];
  const long long r = s_w[w] + incl - x;
  __syncthreads();
  return r;
}

template <class QT>
__device__ __forceinline__ void team_push(bool p, int32_t v, QT* q, int* s_tail) {
  const unsigned long long m = __ballot(p);
  if (!m) return;
  int base = 0;
  if (lane_id() == 0) base = atomicAdd(s_tail, __popcll(m));
  base = __shfl(base, 0, 64);
  if (p) q[base + rank_in(m)] = (QT)v;
}

// Chained round of one graph (VGC, Sec. 4.2, at workgroup level): the round's queue segment grows
// while it is worked off; each wave claims up to 64 queued vertices at a time, expands their rows
// edge-balanced across its lanes and appends the vertices it takes to k to the same queue. A wave
// leaves when it sees no busy wave (busy first) and then no unclaimed entry; entries are reserved
// before they are written, so claimed entries are read once they are no longer -1. False on a
// timeout. All threads call.
__device__ __forceinline__ bool batch_chain(const BatchArgs& a, uint32_t* d, int32_t* q, uint32_t* pb,
                                            const int64_t* off, int64_t base, bool inl, uint32_t k,
                                            int* s_claim, int* s_tail, int* s_busy, long long& st_edges,
                                            long long& st_decr) {
  const int l = lane_id();
  const unsigned long long t_start = wall_clock64();
  for (;;) {
    int state = 0, h = 0, cnt = 0;  // state: 1 claimed, 2 done, 3 timeout
    if (l == 0) {
      bool counted = true;
      for (int spin = 0;; ++spin) {
        const int hh = lds_ld(s_claim);
        const int tt = lds_ld(s_tail);
        if (hh < tt) {
          if (!counted) {
            atomicAdd(s_busy, 1);
            counted = true;
          }
          const int n = min(64, tt - hh);
          if (atomicCAS(s_claim, hh, hh + n) == hh) {
            h = hh;
            cnt = n;
            state = 1;
            break;
          }
          continue;
        }
        if (counted) {
          atomicSub(s_busy, 1);
          counted = false;
          continue;
        }
        if (lds_ld(s_busy) == 0) {
          if (lds_ld(s_claim) >= lds_ld(s_tail)) {
            state = 2;
            break;
          }
          continue;
        }
        __builtin_amdgcn_s_sleep(1);
        if ((spin & 255) == 255 && wall_clock64() - t_start > 400000000ull) {
          state = 3;
          break;
        }
      }
    }
    state = __shfl(state, 0, 64);
    if (state != 1) return state == 2;
    h = __shfl(h, 0, 64);
    cnt = __shfl(cnt, 0, 64);
    int32_t v = -1;
    if (l < cnt) {
      for (int spin = 0;; ++spin) {
        v = lds_ld(&q[h + l]);
        if (v >= 0) break;
        if ((spin & 255) == 255 && wall_clock64() - t_start > 400000000ull) break;
      }
    }
    if (__ballot(l < cnt && v < 0)) return false;
    long long rb = 0, dg = 0;
    if (v >= 0) {
      rb = off[v];
      dg = off[v + 1] - rb;
    }
    const long long incl = wave_incl_scan(dg);
    const long long excl = incl - dg;
    const long long total = __shfl(incl, 63, 64);
    for (long long e0 = 0; e0 < total; e0 += 64) {
      const long long t = e0 + l;
      int j = 0;
#pragma unroll
      for (int step = 32; step >= 1; step >>= 1) {
        const int cand = j + step;
        const long long ex = __shfl(excl, cand & 63, 64);
        if (cand < 64 && ex <= t) j = cand;
      }
      const long long pos = __shfl(rb, j, 64) + (t - __shfl(excl, j, 64));
      bool crossed = false;
      int32_t ul = 0;
      if (t < total) {
        ul = a.adj[pos] - (a.local_ids ? 0 : (int32_t)base);
        st_edges++;
        const bool live = pb ? !((pb[ul >> 5] >> (ul & 31)) & 1u) : d[ul] > k;
        if (live) {
          const unsigned old = inl ? atomicSub(&d[ul], 1u) : wsub(&d[ul], 1u);
          st_decr++;
          check_decrement(old, 1u, &a.ctl->status);
          crossed = old == k + 1;
        }
      }
      if (crossed) {
        if (pb) atomicOr(&pb[ul >> 5], 1u << (ul & 31));
        put_core(a.core, base + ul, k, &a.ctl->status);
      }
      const unsigned long long m = __ballot(crossed);
      if (m) {
        int b = 0;
        if (l == 0) b = atomicAdd(s_tail, __popcll(m));
        b = __shfl(b, 0, 64);
        if (crossed) lds_st(&q[b + rank_in(m)], ul);
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Teams: a graph too large for one workgroup's share of the batch is peeled by team_size
// workgroups together (the launch is cooperative, so they are all resident). Induced degrees and
// the peel queue live in global memory at the graph's own vertex range; decrements are agent-scope
// atomics, and the team synchronises at every round scan and subround with a counter barrier
// (fence-free, as the grid barrier of the single-graph peel). Level-synchronous Alg. 1 + Alg. 3:
// a round's scan reads every vertex (x == k: extract; x > k: min for a jump; x < k: peeled), each
// subround splits the frontier into one contiguous share per member, expanded edge-balanced over
// the member's threads.
// ------------------------------------------------------------------------------------------
// Team barrier. The last arrival records the queue tail (every push of the phase has landed: each
// member waited for its memory operations before arriving) and then releases the team, so all
// members see the same tail even though the fastest may start pushing again at once. Waits are
// bounded (~4 s, or any failure bit set). Returns false when the team must stop; `tail` receives
// the recorded tail.
__device__ bool team_sync(TeamCtl* T, unsigned size, unsigned& epoch, unsigned* status, long long& tail) {
  __shared__ int s_tok;
  __shared__ long long s_tail;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned target = epoch + 1;
    int ok = 1;
    if (aadd(&T->bar, 1u) == target * size - 1) {
      ast(&T->snap[epoch & 1], ald(&T->tail));
      __builtin_amdgcn_s_waitcnt(0);
      ast(&T->gen, target);
    } else {
      const unsigned long long t0 = wall_clock64();
      while (ald(&T->gen) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (wall_clock64() - t0 > 400000000ull) {  // 100 MHz clock: 4 s
          aor(status, (unsigned)KC_ERR_TIMEOUT);
          ok = 0;
          break;
        }
      }
    }
    if (ald(status) != 0u) ok = 0;
    s_tok = ok;
    s_tail = (long long)ald(&T->snap[epoch & 1]);
  }
  __syncthreads();
  epoch += 1;
  tail = s_tail;
  return s_tok != 0;
}

__device__ __forceinline__ void team_push(bool p, int32_t v, int32_t* q, unsigned long long* tail) {
  const unsigned long long m = __ballot(p);
  if (!m) return;
  unsigned long long b = 0;
  if (lane_id() == 0) b = aadd(tail, (unsigned long long)__popcll(m));
  b = __shfl(b, 0, 64);
  if (p) ast(&q[b + rank_in(m)], v);
}

constexpr int kTeamScan = 8;  // degrees per thread a team's round scan loads at once

__device__ __forceinline__ void team_peel(const BatchArgs& a, int team, int member, long long* s_pref, long long* s_rb,
                                       long long* s_w, unsigned* s_min, long long& st_edges, long long& st_decr,
                                       long long& st_rounds, long long& st_sub, long long& st_scanned,
                                       unsigned& kmax_all) {
  TeamCtl* T = &a.ctl->team[team];
  unsigned* status = &a.ctl->status;
  const int32_t g = a.order[team];
  const int64_t base = a.vptr[g];
  const int64_t ng = a.vptr[g + 1] - base;
  const int64_t* off = a.off + base;
  uint32_t* d = a.gdt + base;
  int32_t* q = a.gq + base;
  const int tid = threadIdx.x, l = lane_id(), w = threadIdx.x >> 6;
  const int tsz = (int)a.ctl->team_size;
  const long long gtid = (long long)member * kBatchThreads + tid;
  const long long GT = (long long)tsz * kBatchThreads;
  unsigned epoch = 0;
  const bool lead = member == 0;

  // induced degree = degree; k = min degree
  unsigned mn = 0xffffffffu;
  for (long long i = gtid; i < ng; i += GT) {
    const unsigned dg = (unsigned)(off[i + 1] - off[i]);
    ast(&d[i], dg);
    mn = min(mn, dg);
  }
  mn = wave_min(mn);
  if (l == 0) s_min[w] = mn;
  __syncthreads();
  if (tid == 0) {
    unsigned m = 0xffffffffu;
    for (int i = 0; i < kBatchThreads / 64; ++i) m = min(m, s_min[i]);
    if (m != 0xffffffffu) __hip_atomic_fetch_max(&T->rmx[2], ~m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  long long tail = 0;
  if (!team_sync(T, tsz, epoch, status, tail)) return;
  unsigned k = ~ald(&T->rmx[2]);
  long long head = 0;
  for (long long r = 0;; ++r) {
    unsigned* rmx = &T->rmx[r % 3];
    if (lead && tid == 0) ast(&T->rmx[(r + 1) % 3], 0u);  // (last read two rounds ago)
    // the round's first frontier, and the min over the others: kTeamScan degrees per thread in
    // flight at once (the loads are independent; one at a time, a round's scan of a 100K-vertex
    // graph by a team of 8 would be ~25 dependent memory round trips)
    unsigned nm = 0xffffffffu;
    for (long long b = 0; b < ng; b += GT * kTeamScan) {
      unsigned x[kTeamScan];
#pragma unroll
      for (int r = 0; r < kTeamScan; ++r) {
        const long long i = b + r * GT + gtid;
        x[r] = i < ng ? ald(&d[i]) : 0u;
      }
#pragma unroll
      for (int r = 0; r < kTeamScan; ++r) {
        const long long i = b + r * GT + gtid;
        const bool in = i < ng;
        st_scanned += in ? 1 : 0;
        const bool ext = in && x[r] == k;
        if (in && x[r] > k) nm = min(nm, x[r]);
        if (ext) put_core(a.core, base + i, k, status);
        team_push(ext, (int32_t)i, q, &T->tail);
      }
    }
    nm = wave_min(nm);
    if (l == 0) s_min[w] = nm;
    __syncthreads();
    if (tid == 0) {
      unsigned m = 0xffffffffu;
      for (int i = 0; i < kBatchThreads / 64; ++i) m = min(m, s_min[i]);
      if (m != 0xffffffffu) __hip_atomic_fetch_max(rmx, ~m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!team_sync(T, tsz, epoch, status, tail)) return;
    if (tail == head) {
      const unsigned mv = ~ald(rmx);
      if (mv == 0xffffffffu || tail >= ng) return;  // (nothing live: cannot happen before tail == ng)
      k = mv;
      continue;
    }
    if (lead) st_rounds++;
    kmax_all = max(kmax_all, k);
    while (head < tail) {
      if (lead) st_sub++;
      const long long c0 = head + (tail - head) * member / tsz;
      const long long c1 = head + (tail - head) * (member + 1) / tsz;
      for (long long cb = c0; cb < c1; cb += kBatchThreads) {
        const long long i = cb + tid;
        long long dg = 0, rb = 0;
        if (i < c1) {
          const int32_t v = ald(&q[i]);
          rb = off[v];
          dg = off[v + 1] - rb;
        }
        long long total;
        const long long ex = block_excl_scan(dg, s_w, total);
        s_pref[tid] = ex;
        s_rb[tid] = rb;
        __syncthreads();
        for (long long e0 = 0; e0 < total; e0 += kBatchThreads) {
          const long long t = e0 + tid;
          bool crossed = false;
          int32_t ul = 0;
          if (t < total) {
            int lo = 0, hi = kBatchThreads - 1;  // largest j with s_pref[j] <= t
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (s_pref[mid] <= t) lo = mid; else hi = mid - 1;
            }
            ul = a.adj[s_rb[lo] + (t - s_pref[lo])] - (a.local_ids ? 0 : (int32_t)base);
            st_edges++;
            {  // (no liveness probe: a peeled target is at or below k, so its decrement never crosses)
              const unsigned old = asub(&d[ul], 1u);
              st_decr++;
              check_decrement(old, 1u, status);
              crossed = old == k + 1;
            }
          }
          if (crossed) put_core(a.core, base + ul, k, status);
          team_push(crossed, ul, q, &T->tail);
        }
        __syncthreads();
      }
      head = tail;
      if (!team_sync(T, tsz, epoch, status, tail)) return;
    }
    if (tail >= ng) return;
    k = k + 1;
  }
}

__global__ __launch_bounds__(kBatchThreads) void batched_kernel(BatchArgs a) {
  extern __shared__ uint32_t s_dyn[];
  __shared__ long long s_pref[kBatchThreads];
  __shared__ long long s_rb[kBatchThreads];
  __shared__ long long s_w[kBatchThreads / 64 + 1];
  __shared__ unsigned s_min[kBatchThreads / 64];
  __shared__ int s_tail;
  __shared__ int s_claim, s_busy;
  __shared__ long long s_g;

  long long st_edges = 0, st_decr = 0, st_rounds = 0, st_sub = 0, st_scanned = 0;
  unsigned kmax_all = 0;
  const int tid = threadIdx.x, l = lane_id(), w = threadIdx.x >> 6;
  // the leading nteams graphs of the order are peeled by teams of the first workgroups
  const int nteams = a.teams ? (int)a.ctl->nteams : 0;
  const int tsz = a.teams ? (int)a.ctl->team_size : 1;
  if ((int)blockIdx.x < nteams * tsz)
    team_peel(a, blockIdx.x / tsz, blockIdx.x % tsz, s_pref, s_rb, s_w, s_min, st_edges, st_decr, st_rounds, st_sub,
              st_scanned, kmax_all);

  for (;;) {
    if (tid == 0) s_g = (long long)aadd(&a.ctl->next, 1ull) + nteams;
    __syncthreads();
    const long long gi = s_g;
    __syncthreads();
    if (gi >= a.G) break;
    const int32_t g = a.order ? a.order[gi] : (int32_t)gi;
    const int64_t base = a.vptr[g];
    const int64_t ng = a.vptr[g + 1] - base;
    if (ng <= 0) continue;
    const bool inl = ng <= a.lds_cap;
    const int64_t* off = a.off + base;
    // A level-sync graph whose rows fit beside its degrees and queue keeps them in LDS too: row
    // starts relative to its first entry, then its adjacency as 16-bit local ids (ng <= lds_cap <
    // 65,536), copied once with coalesced loads, so that no subround waits on global memory.
    const int64_t mg = inl ? off[ng] - off[0] : 0;
    const bool staged = inl && !a.chained && 12 * ng + 4 + 2 * mg <= 8ll * a.lds_cap;
    uint32_t* d = inl ? s_dyn : a.gdt + base;
    int32_t* q = staged ? reinterpret_cast<int32_t*>(s_dyn + ng)
                        : inl ? reinterpret_cast<int32_t*>(s_dyn + a.lds_cap) : a.gq + base;
    uint32_t* srow = staged ? s_dyn + 2 * ng : nullptr;                           // ng + 1 starts
    uint16_t* sadj = staged ? reinterpret_cast<uint16_t*>(s_dyn + 3 * ng + 1) : nullptr;  // mg ids
    // a graph held in global memory keeps a peeled bitmap in the (then unused) LDS, so that the
    // liveness test before a decrement costs no global load
    uint32_t* pb = (!inl && ng <= 64ll * a.lds_cap) ? s_dyn : nullptr;

    // induced degree = degree; k = min degree
    unsigned mn = 0xffffffffu;
    for (long long i = tid; i < ng; i += kBatchThreads) {
      const unsigned dg = (unsigned)(off[i + 1] - off[i]);
      d[i] = dg;
      mn = min(mn, dg);
    }
    if (staged) {
      const int64_t e0 = off[0];
      const int32_t shift = a.local_ids ? 0 : (int32_t)base;
      for (long long i = tid; i <= ng; i += kBatchThreads) srow[i] = (uint32_t)(off[i] - e0);
      for (long long e = tid; e < mg; e += kBatchThreads) sadj[e] = (uint16_t)(a.adj[e0 + e] - shift);
    }
    if (pb)
      for (long long i = tid; i < (ng + 31) / 32; i += kBatchThreads) pb[i] = 0u;
    if (a.chained)
      for (long long i = tid; i < ng; i += kBatchThreads) q[i] = -1;  // unwritten queue entries
    mn = wave_min(mn);
    if (l == 0) s_min[w] = mn;
    if (tid == 0) s_tail = 0;
    __syncthreads();
    unsigned k = 0xffffffffu;
    for (int i = 0; i < kBatchThreads / 64; ++i) k = min(k, s_min[i]);
    __syncthreads();

    int head = 0;
    // Graphs held in global memory keep a compacted active list (Alg. 1 refine): each round's
    // scan reads the survivors of the previous one and writes its own survivors in place (a
    // survivor never moves forward, and a chunk is read before it is overwritten). LDS-resident
    // graphs are small enough to scan whole.
    int32_t* act = inl ? nullptr : a.ga + base;
    long long asz = ng;
    bool dense_b = true;
    for (;;) {
      // extraction of round k's first frontier (at round start every live vertex has d >= k);
      // also the min over the others for a jump
      unsigned nm = 0xffffffffu;
      long long wpos = 0;
      // four consecutive slots per thread: independent loads, and one compaction scan per 2048
      // slots (order preserving, so the in-place compaction never overwrites an unread slot)
      for (long long i0 = 0; i0 < asz; i0 += 4 * kBatchThreads) {
        int32_t vi[4];
        unsigned x[4];
        bool ext[4], keep[4];
        int nk = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const long long i = i0 + 4 * tid + r;
          vi[r] = (i < asz) ? (dense_b ? (int32_t)i : act[i]) : -1;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = vi[r] >= 0 ? d[vi[r]] : 0u;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          ext[r] = vi[r] >= 0 && x[r] == k;
          keep[r] = vi[r] >= 0 && x[r] > k;
          if (vi[r] >= 0) st_scanned++;
          if (keep[r]) {
            nm = min(nm, x[r]);
            ++nk;
          }
          if (ext[r]) {
            put_core(a.core, base + vi[r], k, &a.ctl->status);
            if (pb) atomicOr(&pb[vi[r] >> 5], 1u << (vi[r] & 31));
          }
          team_push(ext[r], vi[r], q, &s_tail);
        }
        if (!inl) {
          long long kept;
          long long ex = block_excl_scan(nk, s_w, kept);
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (keep[r]) act[wpos + ex++] = vi[r];
          wpos += kept;
          __syncthreads();
        }
      }
      if (!inl) {
        asz = wpos;
        dense_b = false;
      }
      nm = wave_min(nm);
      if (l == 0) s_min[w] = nm;
      __syncthreads();
      int tail = s_tail;
      unsigned nextmin = 0xffffffffu;
      for (int i = 0; i < kBatchThreads / 64; ++i) nextmin = min(nextmin, s_min[i]);
      __syncthreads();
      if (tail == head) {
        // empty round: jump to the next non-empty one
        if (nextmin == 0xffffffffu) break;
        k = nextmin;
        continue;
      }
      st_rounds++;
      if (k > kmax_all) kmax_all = k;
      if (a.chained) {
        if (tid == 0) {
          s_claim = head;
          s_busy = kBatchThreads / 64;
        }
        __syncthreads();
        if (!batch_chain(a, d, q, pb, off, base, inl, k, &s_claim, &s_tail, &s_busy, st_edges, st_decr) &&
            l == 0)
          aor(&a.ctl->status, (unsigned)KC_ERR_TIMEOUT);
        __syncthreads();
        st_sub++;
        head = tail = s_tail;
        __syncthreads();
      }
      // level-synchronous subrounds: frontier = q[head, tail)
      while (head < tail) {
        st_sub++;
        for (long long c0 = head; c0 < tail; c0 += kBatchThreads) {
          const long long i = c0 + tid;
          long long dg = 0, rb = 0;
          if (i < tail) {
            const int32_t v = q[i];
            if (staged) {
              rb = srow[v];
              dg = srow[v + 1] - rb;
            } else {
              rb = off[v];
              dg = off[v + 1] - rb;
            }
          }
          long long total;
          const long long ex = block_excl_scan(dg, s_w, total);
          s_pref[tid] = ex;
          s_rb[tid] = rb;
          __syncthreads();
          for (long long e0 = 0; e0 < total; e0 += kBatchThreads) {
            const long long t = e0 + tid;
            bool crossed = false;
            int32_t ul = 0;
            if (t < total) {
              int lo = 0, hi = kBatchThreads - 1;  // largest j with s_pref[j] <= t
              while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_pref[mid] <= t) lo = mid; else hi = mid - 1;
              }
              const long long pos = s_rb[lo] + (t - s_pref[lo]);
              ul = staged ? (int32_t)sadj[pos] : a.adj[pos] - (a.local_ids ? 0 : (int32_t)base);
              st_edges++;
              const bool live = pb ? !((pb[ul >> 5] >> (ul & 31)) & 1u) : d[ul] > k;
              if (live) {
                const unsigned old = inl ? atomicSub(&d[ul], 1u) : wsub(&d[ul], 1u);
                st_decr++;
                check_decrement(old, 1u, &a.ctl->status);
                crossed = old == k + 1;
              }
            }
            if (crossed && pb) atomicOr(&pb[ul >> 5], 1u << (ul & 31));
            team_push(crossed, ul, q, &s_tail);
            if (crossed) put_core(a.core, base + ul, k, &a.ctl->status);
          }
          __syncthreads();
        }
        head = tail;
        tail = s_tail;
        __syncthreads();
      }
      if (tail >= ng) break;
      k = k + 1;
    }
    __syncthreads();
  }
  // statistics
  long long v5[3] = {st_edges, st_decr, st_scanned};
  for (int qd = 0; qd < 3; ++qd) {
    long long x = v5[qd];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (l == 0 && x) aadd(&a.ctl->stats[qd == 0 ? ST_EDGES : qd == 1 ? ST_DECR : ST_SCANNED], (unsigned long long)x);
  }
  if (tid == 0) {
    if (st_rounds) aadd(&a.ctl->stats[ST_ROUNDS], (unsigned long long)st_rounds);
    if (st_sub) aadd(&a.ctl->stats[ST_SUBROUNDS], (unsigned long long)st_sub);
    __hip_atomic_fetch_max(&a.ctl->stats[ST_KMAX], (unsigned long long)kmax_all, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  }
}

hipError_t launch_batched(const BatchArgs& a, int blocks, size_t lds_bytes, hipStream_t s) {
  hipLaunchKernelGGL(batched_kernel, dim3(blocks), dim3(kBatchThreads), lds_bytes, s, a);
  return hipGetLastError();
}

hipError_t launch_batched_coop(const BatchArgs& a, int blocks, size_t lds_bytes, hipStream_t s) {
  void* args[] = {const_cast<BatchArgs*>(&a)};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(batched_kernel), dim3(blocks), dim3(kBatchThreads),
                                    args, (unsigned)lds_bytes, s);
}

// Team plan: the leading graphs of the order (largest first by power of two of their entries)
// with more entries than min_entries (default: half a workgroup's average share of the batch; every
// leading graph when `all`) get a team; at most kMaxTeams, and at most team_wgs workgroups in teams.
// One workgroup peels a graph held in global memory several times slower per entry than the
// LDS-resident small graphs that make up most of a batch, hence the low default threshold. Teams
// have team_size workgroups, or (team_size 0) an equal share of team_wgs, at least kTeamSize and
// at most kMaxTeamSize, so that a few huge graphs get large teams and many big ones teams of 8.
__global__ __launch_bounds__(64) void team_plan_kernel(const int64_t* vptr, const int64_t* off, int32_t G,
                                                       const int32_t* order, int32_t blocks, int32_t team_wgs,
                                                       int32_t team_size, int32_t all, long long min_entries,
                                                       BatchCtl* ctl) {
  if (threadIdx.x != 0) return;
  const long long total = off[vptr[G]] - off[vptr[0]];
  const long long share = total / (blocks > 0 ? blocks : 1);
  const long long thr = min_entries > 0 ? min_entries : share / 2;
  int want = 0;
  while (want < kMaxTeams && want < G) {
    const int32_t g = order[want];
    const long long e = off[vptr[g + 1]] - off[vptr[g]];
    if (!all && e <= thr) break;
    ++want;
  }
  int ts = team_size;
  if (ts <= 0) ts = want > 0 ? max(kTeamSize, min(kMaxTeamSize, team_wgs / want)) : kTeamSize;
  int nt = min(want, team_wgs / ts);
  ctl->nteams = (unsigned)nt;
  ctl->team_size = (unsigned)ts;
}

hipError_t launch_team_plan(const int64_t* vptr, const int64_t* off, int32_t G, const int32_t* order,
                            int32_t blocks, int32_t team_wgs, int32_t team_size, int32_t all, int64_t min_entries,
                            BatchCtl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(team_plan_kernel, dim3(1), dim3(64), 0, s, vptr, off, G, order, blocks, team_wgs, team_size,
                     all, (long long)min_entries, ctl);
  return hipGetLastError();
}

hipError_t batched_occupancy(size_t lds_bytes, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, batched_kernel, kBatchThreads,
                                                      lds_bytes);
}

// ------------------------------------------------------------------------------------------
// Tail peel: one workgroup finishes the decomposition on the live vertices peel_kernel handed over
// (Alg. 1 with the online peel of Alg. 3: chained rounds in chained mode, level-synchronous
// subrounds in level-sync mode) with their induced degrees in LDS, so its rounds synchronise at
// workgroup level instead of grid-wide. The local rows hold live neighbours only, in local ids. A
// round scans every local vertex: at its start a live vertex has induced degree >= k, and a vertex
// peeled earlier stays below k (it is never decremented once at or below the current k), so
// degree == k picks the round's first frontier. The queue holds vertices in peel order; a
// subround's frontier is the queue segment between two marks.
// ------------------------------------------------------------------------------------------
// A tail vertex's coreness is recorded when its row is claimed (every peeled vertex is claimed
// exactly once, in the round that peels it), as -(k + 1) in the end word of its local row bounds,
// which nothing reads after the claim; one pass at the end of the tail peel moves the recorded
// values to the output. So no store on the peel's critical path waits for the local-to-global id
// lookup. Returns the row end read before the overwrite.
__device__ __forceinline__ long long tail_claim(const PeelArgs& a, int32_t v, uint32_t k) {
  long long* p = &a.trow[2 * (long long)v + 1];
  const long long e = *p;
  if (KCORE_CHECKS && e < 0) {  // claimed twice
    aor(&a.ctl->status, (unsigned)KC_ERR_CHECK);
    return p[-1];
  }
  *p = -(long long)k - 1;
  return e;
}

// Decrements of the induced degrees of N neighbours per lane (local ids; a lane with no entry
// passes L + lane, a private spare slot past the vertices, so that no lane branches). A vertex
// peeled before is at or below k and stays there, and every neighbour decrements it once, so its
// degree never wraps and never returns to k + 1; the decrement that takes u from k + 1 to k pushes
// it (slot reserved first, then written: chained rounds read slots as they fill). Every atomic of
// the batch is issued before any result is looked at. All lanes of the wavefront call.
template <int N>
__device__ __forceinline__ void tail_edges(const PeelArgs& a, uint32_t* d, uint16_t* q, int* s_tail, int L,
                                           const int32_t (&u)[N], uint32_t k) {
  uint32_t old[N];
#pragma unroll
  for (int j = 0; j < N; ++j) old[j] = atomicSub(&d[u[j]], 1u);
  unsigned cm = 0;  // this lane's crossings
#pragma unroll
  for (int j = 0; j < N; ++j) {
    cm |= (old[j] == k + 1 ? 1u : 0u) << j;
    if (KCORE_CHECKS && u[j] < L) check_decrement(old[j], 1u, &a.ctl->status);
  }
  if (!__ballot(cm != 0)) return;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const bool crossed = (cm >> j) & 1u;
    const unsigned long long m = __ballot(crossed);
    if (!m) continue;
    int b = 0;
    if (lane_id() == 0) b = atomicAdd(s_tail, __popcll(m));
    b = __shfl(b, 0, 64);
    if (crossed) lds_st(&q[b + rank_in(m)], (uint16_t)u[j]);
  }
}

// tail_edges for 16 entries held as 8 packed words of two 16-bit local ids: entry e is the
// (e & 1) half of word e >> 1, valid when e < lim (lim <= 0: none); an invalid entry decrements
// the lane's spare slot. Ids are unpacked where they are used, so the packed words are all that
// stays live. All lanes of the wavefront call.
__device__ __forceinline__ void tail_edges16(const PeelArgs& a, uint32_t* d, uint16_t* q, int* s_tail, int L,
                                             const uint32_t (&w)[8], const int (&lim)[2], uint32_t k) {
  const int spare = L + lane_id();
  uint32_t old[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int32_t id = (int32_t)((w[e >> 1] >> (16 * (e & 1))) & 0xffffu);
    old[e] = atomicSub(&d[(e & 7) < lim[e >> 3] ? id : spare], 1u);
  }
  unsigned cm = 0;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    cm |= (old[e] == k + 1 ? 1u : 0u) << e;
    if (KCORE_CHECKS && (e & 7) < lim[e >> 3]) check_decrement(old[e], 1u, &a.ctl->status);
  }
  if (!__ballot(cm != 0)) return;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const bool crossed = (cm >> e) & 1u;
    const unsigned long long m = __ballot(crossed);
    if (!m) continue;
    const int32_t u = (int32_t)((w[e >> 1] >> (16 * (e & 1))) & 0xffffu);
    int b = 0;
    if (lane_id() == 0) b = atomicAdd(s_tail, __popcll(m));
    b = __shfl(b, 0, 64);
    if (crossed) lds_st(&q[b + rank_in(m)], (uint16_t)u);
  }
}

// Entries [tb, tb + len) of the local rows, len <= kTailTile, through one wavefront with 16-byte
// loads of eight 16-bit local ids each, every load in flight before the first decrement (tb on a
// 16-byte boundary; rows are padded to whole 16-byte words); the decrements go in two halves of
// 16 entries per lane. All lanes call with the same range.
__device__ __forceinline__ void tail_tile(const PeelArgs& a, uint32_t* d, uint16_t* q, int* s_tail, int L, int tb,
                                          int len, uint32_t k) {
  static_assert(kTailTile == 2048, "four 16-byte loads of 8 entries per lane");
  const int l = lane_id();
  uint4 x[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int r = 512 * j + 8 * l;
    x[j] = r < len ? *reinterpret_cast<const uint4*>(a.tadj + (tb + r)) : make_uint4(0u, 0u, 0u, 0u);
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const uint32_t w[8] = {x[2 * h].x, x[2 * h].y, x[2 * h].z, x[2 * h].w,
                           x[2 * h + 1].x, x[2 * h + 1].y, x[2 * h + 1].z, x[2 * h + 1].w};
    const int lim[2] = {len - (1024 * h + 8 * l), len - (1024 * h + 512 + 8 * l)};
    tail_edges16(a, d, q, s_tail, L, w, lim, k);
  }
}

// Chained round of the tail peel (VGC, Sec. 4.2, at workgroup level): the round's queue segment
// grows while it is worked off. A wavefront claims a share of the waiting vertices (all waiting
// ones split over the wavefronts, at most 64), streams each long row itself and expands the short
// ones edge-balanced across its lanes; what it takes to k joins the same queue. A wave leaves when
// it sees no busy wave (busy first) and then no unclaimed entry; entries are reserved before they
// are written, so a claimed slot is read once it is no longer -1. False on a timeout. All threads
// call.
// Tiles of long rows a wavefront claimed are shared with the other wavefronts through a small
// LDS ring (start << 16 | length, kTileEmpty = free slot), so that a chain level with a few long
// rows keeps all wavefronts busy; when the ring has no room the claiming wavefront streams them.
constexpr int kTailRing = 256;
constexpr unsigned long long kTileEmpty = ~0ull;

__device__ __forceinline__ bool tail_chain(const PeelArgs& a, uint32_t* d, uint16_t* q, int L, uint32_t k,
                                           int* s_claim, int* s_tail, int* s_busy, unsigned long long* s_ring,
                                           int* s_rclaim, int* s_rtail, long long& st_edges) {
  constexpr int nw = kTailThreads / 64;
  const int l = lane_id();
  const unsigned long long t_start = wall_clock64();
  for (;;) {
    int state = 0, h = 0, cnt = 0;  // state: 1 vertices claimed, 4 a tile claimed, 2 done, 3 timeout
    if (l == 0) {
      bool counted = true;
      for (int spin = 0;; ++spin) {
        // shared tiles first: they finish rows that are already under way
        const int rh = lds_ld(s_rclaim);
        if (rh < lds_ld(s_rtail)) {
          if (!counted) {
            atomicAdd(s_busy, 1);
            counted = true;
          }
          if (atomicCAS(s_rclaim, rh, rh + 1) == rh) {
            h = rh;
            state = 4;
            break;
          }
          continue;
        }
        const int hh = lds_ld(s_claim);
        const int tt = lds_ld(s_tail);
        if (hh < tt) {
          if (!counted) {
            atomicAdd(s_busy, 1);
            counted = true;
          }
          const int n = min(64, (tt - hh + nw - 1) / nw);
          if (atomicCAS(s_claim, hh, hh + n) == hh) {
            h = hh;
            cnt = n;
            state = 1;
            break;
          }
          continue;
        }
        if (counted) {
          atomicSub(s_busy, 1);
          counted = false;
          continue;
        }
        if (lds_ld(s_busy) == 0) {
          if (lds_ld(s_claim) >= lds_ld(s_tail) && lds_ld(s_rclaim) >= lds_ld(s_rtail)) {
            state = 2;
            break;
          }
          continue;
        }
        __builtin_amdgcn_s_sleep(1);
        if ((spin & 255) == 255 && wall_clock64() - t_start > 400000000ull) {
          state = 3;
          break;
        }
      }
    }
    state = __shfl(state, 0, 64);
    if (state == 4) {
      // a shared tile: its slot was reserved before it was written, so wait for the entry, then
      // free the slot and stream the tile
      h = __shfl(h, 0, 64);
      unsigned long long e = kTileEmpty;
      int full = 0;
      if (l == 0) {
        unsigned long long* slot = &s_ring[h & (kTailRing - 1)];
        for (int spin = 0;; ++spin) {
          e = lds_ld(slot);
          if (e != kTileEmpty) break;
          if ((spin & 255) == 255 && wall_clock64() - t_start > 400000000ull) break;
        }
        if (e != kTileEmpty) lds_st(slot, kTileEmpty);
        full = lds_ld(s_tail) >= L;
      }
      e = __shfl(e, 0, 64);
      if (e == kTileEmpty) return false;
      const int tlen = (int)(e & 0xffffull);
      if (l == 0) st_edges += tlen;
      if (!__shfl(full, 0, 64)) tail_tile(a, d, q, s_tail, L, (int)(e >> 16), tlen, k);
      continue;
    }
    if (state != 1) return state == 2;
    h = __shfl(h, 0, 64);
    cnt = __shfl(cnt, 0, 64);
    int32_t v = -1;
    if (l < cnt) {
      for (int spin = 0;; ++spin) {
        const uint16_t x = lds_ld(&q[h + l]);
        v = x == kTailQEmpty ? -1 : (int32_t)x;
        if (v >= 0) break;
        if ((spin & 255) == 255 && wall_clock64() - t_start > 400000000ull) break;
      }
    }
    if (__ballot(l < cnt && v < 0)) return false;
    int rb = 0, dg = 0;
    if (v >= 0) {
      rb = (int)a.trow[2 * (long long)v];
      dg = (int)(tail_claim(a, v, k) - rb);
    }
    // once every local vertex is queued, the rows still waiting can only decrement peeled vertices
    // (the last round of a dense core queues all of it after a fraction of its rows): they count
    // as expanded without being read
    int full = 0;
    if (l == 0) full = lds_ld(s_tail) >= L;
    if (__shfl(full, 0, 64)) {
      const int tot = __shfl(wave_incl_scan(dg), 63, 64);
      if (l == 0) st_edges += tot;
      continue;
    }
    unsigned long long big = __ballot(dg >= kTailBig);
    if (big) {
      // hand the long rows' tiles to the ring when it has room for all of them
      const int nt = dg >= kTailBig ? (dg + kTailTile - 1) / kTailTile : 0;
      const int tincl = wave_incl_scan(nt);
      const int ttot = __shfl(tincl, 63, 64);
      int base = -1;
      if (l == 0 && ttot > 1) {  // (a single tile is streamed by the wave that holds it)
        for (;;) {
          const int rt = lds_ld(s_rtail);
          if (rt + ttot - lds_ld(s_rclaim) > kTailRing) break;
          if (atomicCAS(s_rtail, rt, rt + ttot) == rt) {
            base = rt;
            break;
          }
        }
      }
      base = __shfl(base, 0, 64);
      if (base >= 0) {
        bool late = false;
        for (int j = 0; j < nt; ++j) {
          // (a slot may still hold an older tile that was claimed but not yet read)
          unsigned long long* slot = &s_ring[(base + tincl - nt + j) & (kTailRing - 1)];
          for (int spin = 0; lds_ld(slot) != kTileEmpty; ++spin)
            if ((spin & 255) == 255 && wall_clock64() - t_start > 400000000ull) {
              late = true;
              break;
            }
          lds_st(slot, ((unsigned long long)(rb + j * kTailTile) << 16) |
                           (unsigned long long)min(kTailTile, dg - j * kTailTile));
        }
        if (__ballot(late)) return false;
        big = 0;
      }
    }
    while (big) {
      const int j = __ffsll((long long)big) - 1;
      big &= big - 1;
      const int rs = __shfl(rb, j, 64), len = __shfl(dg, j, 64);
      if (l == 0) st_edges += len;
      if (l == 0) full = lds_ld(s_tail) >= L;
      if (__shfl(full, 0, 64)) continue;  // (as above, row by row)
      for (int o = 0; o < len; o += kTailTile)
        tail_tile(a, d, q, s_tail, L, rs + o, min(len - o, kTailTile), k);
    }
    const int sd = dg >= kTailBig ? 0 : dg;
    const int incl = wave_incl_scan(sd);
    const int excl = incl - sd;
    const int total = __shfl(incl, 63, 64);
    if (l == 0) st_edges += total;
    if (l == 0) full = lds_ld(s_tail) >= L;
    const bool skip = __shfl(full, 0, 64) != 0;
    for (int e0 = 0; !skip && e0 < total; e0 += 64 * kTailUnroll) {
      int32_t u[kTailUnroll];
#pragma unroll
      for (int r = 0; r < kTailUnroll; ++r) {
        const int t = e0 + 64 * r + l;
        int j = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
          const int cand = j + step;
          const int ex = __shfl(excl, cand & 63, 64);
          if (cand < 64 && ex <= t) j = cand;
        }
        const int pos = __shfl(rb, j, 64) + (t - __shfl(excl, j, 64));
        u[r] = t < total ? (int32_t)a.tadj[pos] : L + l;
      }
      tail_edges(a, d, q, s_tail, L, u, k);
    }
  }
}

__device__ __forceinline__ int tail_excl_scan(int x, int* s_w, int& total) {
  constexpr int nw = kTailThreads / 64;
  const int w = threadIdx.x >> 6, l = lane_id();
  const int incl = wave_incl_scan(x);
  if (l == 63) s_w[w] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int i = 0; i < nw; ++i) {
      const int c = s_w[i];
      s_w[i] = t;
      t += c;
    }
    s_w[nw] = t;
  }
  __syncthreads();
  total = s_w[nw];
  const int r = s_w[w] + incl - x;
  __syncthreads();
  return r;
}

// LDS of the tail peel: per vertex an induced degree and a queue slot, plus 64 spare degree slots
// (one per lane) that lanes without an entry decrement.
constexpr size_t tail_dyn_lds(int32_t lcap) { return (size_t)lcap * 6 + 64 * 4; }

template <bool kChained>
__global__ __launch_bounds__(kTailThreads) void tail_kernel(PeelArgs a, int32_t lcap) {
  extern __shared__ uint32_t s_dyn[];
  __shared__ int s_pref[kTailThreads];   // chunk prefix of short-row entries
  __shared__ int s_tpref[kTailThreads];  // chunk prefix of long-row tiles
  __shared__ int s_rb[kTailThreads];     // row start
  __shared__ int s_len[kTailThreads];    // row length
  __shared__ int s_w[kTailThreads / 64 + 1];
  __shared__ unsigned s_min[kTailThreads / 64];
  __shared__ int s_tail;
  __shared__ int s_claim, s_busy;
  __shared__ unsigned long long s_ring[kChained ? kTailRing : 1];  // shared long-row tiles
  __shared__ int s_rclaim, s_rtail;
  const int tid = threadIdx.x, l = lane_id(), w = tid >> 6;
  const long long Ln = (long long)ald(&a.ctl->tail_n);
  if (Ln == 0) return;
  if (Ln > lcap) {
    if (tid == 0) aor(&a.ctl->status, (unsigned)KC_ERR_OVERFLOW);
    return;
  }
  const int L = (int)Ln;
  uint32_t* d = s_dyn;                                       // L degrees, then 64 spare slots
  uint16_t* q = reinterpret_cast<uint16_t*>(s_dyn + lcap + 64);  // lcap 16-bit queue slots
  const long long* rows = a.trow;
  // per-round timeline in the upper half of the phase timeline (100 MHz clock): start, first
  // frontier extracted, round peeled; then k, first frontier size, vertices peeled so far
  unsigned long long* trc = nullptr;
  int ntr = 0;
  long long st_edges = 0, st_scanned = 0, st_rounds = 0, st_sub = 0;

  // induced degree = length of the local row (its live neighbours); k = the smallest
  unsigned mn = 0xffffffffu;
  for (int i = tid; i < L; i += kTailThreads) {
    const unsigned dg = (unsigned)(rows[2 * (long long)i + 1] - rows[2 * (long long)i]);
    d[i] = dg;
    q[i] = kTailQEmpty;  // unwritten queue slot
    mn = min(mn, dg);
  }
  if (tid < 64) d[L + tid] = 0x7fffffffu;  // spare slots: never near any k
  if (kChained)
    for (int i = tid; i < kTailRing; i += kTailThreads) s_ring[i] = kTileEmpty;
  mn = wave_min(mn);
  if (l == 0) s_min[w] = mn;
  if (tid == 0) s_tail = 0;
  __syncthreads();
  unsigned k = 0xffffffffu;
  for (int i = 0; i < kTailThreads / 64; ++i) k = min(k, s_min[i]);
  __syncthreads();
  unsigned kmax = 0;
  int head = 0;
  for (;;) {
    trc = (tid == 0 && ntr < kTracePhases / 2) ? a.ctl->trace[kTracePhases / 2 + ntr] : nullptr;
    if (trc) trc[0] = wall_clock64();
    // the round's first frontier, and the smallest degree above k for a jump over empty rounds
    unsigned nm = 0xffffffffu;
    for (int i0 = 0; i0 < L; i0 += 4 * kTailThreads) {
      unsigned x[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + r * kTailThreads + tid;
        x[r] = i < L ? d[i] : 0u;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + r * kTailThreads + tid;
        const bool ext = i < L && x[r] == k;
        if (x[r] > k) nm = min(nm, x[r]);
        team_push(ext, i, q, &s_tail);
      }
    }
    if (tid == 0) st_scanned += L;
    nm = wave_min(nm);
    if (l == 0) s_min[w] = nm;
    __syncthreads();
    int tail = s_tail;
    unsigned nextmin = 0xffffffffu;
    for (int i = 0; i < kTailThreads / 64; ++i) nextmin = min(nextmin, s_min[i]);
    __syncthreads();
    if (tail == head) {
      if (nextmin == 0xffffffffu) break;  // (cannot happen while vertices are live)
      k = nextmin;
      continue;
    }
    st_rounds++;
    kmax = k;
    if (trc) {
      trc[1] = wall_clock64();
      trc[4] = k;
      trc[5] = (unsigned long long)(tail - head);
    }
    if (kChained) {
      if (tid == 0) {
        s_claim = head;
        s_busy = kTailThreads / 64;
        s_rclaim = 0;
        s_rtail = 0;
      }
      __syncthreads();
      if (!tail_chain(a, d, q, L, k, &s_claim, &s_tail, &s_busy, s_ring, &s_rclaim, &s_rtail, st_edges) && l == 0)
        aor(&a.ctl->status, (unsigned)KC_ERR_TIMEOUT);
      __syncthreads();
      st_sub++;
      head = tail = s_tail;
      __syncthreads();
    }
    // level-synchronous subrounds: frontier = q[head, tail). Short rows are expanded
    // edge-balanced over the workgroup (one search per entry); long rows are cut into tiles that
    // a wavefront streams with 16-byte loads.
    while (!kChained && head < tail) {
      st_sub++;
      const bool full = tail >= L;  // every local vertex queued: rows counted, not read
      for (int c0 = head; c0 < tail; c0 += kTailThreads) {
        const int i = c0 + tid;
        int rb = 0, dg = 0;
        if (i < tail) {
          const int32_t v = (int32_t)q[i];
          rb = (int)rows[2 * (long long)v];
          dg = (int)(tail_claim(a, v, k) - rb);
        }
        const bool big = dg >= kTailBig;
        int total, tiles;
        const int ex = tail_excl_scan(big ? 0 : dg, s_w, total);
        const int tex = tail_excl_scan(big ? (dg + kTailTile - 1) / kTailTile : 0, s_w, tiles);
        s_pref[tid] = ex;
        s_tpref[tid] = tex;
        s_rb[tid] = rb;
        s_len[tid] = dg;
        if (tid == 0) st_edges += total;
        if (big) st_edges += dg;
        __syncthreads();
        for (int e0 = 0; !full && e0 < total; e0 += kTailThreads * kTailUnroll) {
          int32_t u[kTailUnroll];
#pragma unroll
          for (int r = 0; r < kTailUnroll; ++r) {
            const int t = e0 + r * kTailThreads + tid;
            u[r] = L + l;
            if (t < total) {
              int lo = 0, hi = kTailThreads - 1;  // largest j with s_pref[j] <= t
              while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_pref[mid] <= t) lo = mid; else hi = mid - 1;
              }
              u[r] = (int32_t)a.tadj[s_rb[lo] + (t - s_pref[lo])];
            }
          }
          tail_edges(a, d, q, &s_tail, L, u, k);
        }
        for (int tt = w; !full && tt < tiles; tt += kTailThreads / 64) {
          int lo = 0, hi = kTailThreads - 1;  // largest j with s_tpref[j] <= tt (wave-uniform)
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_tpref[mid] <= tt) lo = mid; else hi = mid - 1;
          }
          // the row starts on a 16-byte boundary and is padded to whole 16-byte words
          const int o = (tt - s_tpref[lo]) * kTailTile;
          tail_tile(a, d, q, &s_tail, L, s_rb[lo] + o, min(s_len[lo] - o, kTailTile), k);
        }
        __syncthreads();
      }
      head = tail;
      tail = s_tail;
      __syncthreads();
    }
    if (trc) {
      trc[2] = wall_clock64();
      trc[6] = (unsigned long long)tail;
      ntr++;
    }
    if (tail >= L) break;
    k = k + 1;
  }
  // every local vertex has been claimed: its coreness goes to the output
  __syncthreads();
  for (int i = tid; i < L; i += kTailThreads) {
    const long long x = a.trow[2 * (long long)i + 1];
    if (KCORE_CHECKS && x >= 0) aor(&a.ctl->status, (unsigned)KC_ERR_CHECK);  // never claimed
    put_core(a.core, a.tgid[i], (uint32_t)(-x - 1), &a.ctl->status);
  }
  // statistics: the tail's share of the decomposition's counters (its decrements are LDS
  // operations, not counted with the global ones)
  long long v5[2] = {st_edges, st_scanned};
  for (int qd = 0; qd < 2; ++qd) {
    long long x = v5[qd];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (l == 0 && x) aadd(&a.ctl->stats[qd == 0 ? ST_EDGES : ST_SCANNED], (unsigned long long)x);
  }
  if (tid == 0) {
    aadd(&a.ctl->stats[ST_PEELED], (unsigned long long)L);
    ast(&a.ctl->stats[ST_TAIL], (unsigned long long)L);
    if (st_rounds) aadd(&a.ctl->stats[ST_ROUNDS], (unsigned long long)st_rounds);
    if (st_sub) aadd(&a.ctl->stats[ST_SUBROUNDS], (unsigned long long)st_sub);
    __hip_atomic_fetch_max(&a.ctl->stats[ST_KMAX], (unsigned long long)kmax, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  }
}

hipError_t launch_tail(const PeelArgs& a, int32_t lcap, hipStream_t s) {
  if (a.chained)
    hipLaunchKernelGGL(tail_kernel<true>, dim3(1), dim3(kTailThreads), tail_dyn_lds(lcap), s, a, lcap);
  else
    hipLaunchKernelGGL(tail_kernel<false>, dim3(1), dim3(kTailThreads), tail_dyn_lds(lcap), s, a, lcap);
  return hipGetLastError();
}

hipError_t tail_static_lds(int chained, size_t* bytes) {
  hipFuncAttributes fa;
  const void* f = chained ? reinterpret_cast<const void*>(tail_kernel<true>)
                          : reinterpret_cast<const void*>(tail_kernel<false>);
  hipError_t e = hipFuncGetAttributes(&fa, f);
  if (e == hipSuccess) *bytes = fa.sharedSizeBytes;
  return e;
}
hipError_t tail_allow_lds(int chained, int32_t lcap) {
  const void* f = chained ? reinterpret_cast<const void*>(tail_kernel<true>)
                          : reinterpret_cast<const void*>(tail_kernel<false>);
  return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)tail_dyn_lds(lcap));
}

// Largest-first order of the graphs of a batch: counting sort on floor(log2(edges + 1)),
// descending, in a single workgroup (order inside a size class is arbitrary).
__global__ __launch_bounds__(1024) void order_kernel(const int64_t* vptr, const int64_t* off, int32_t G,
                                                     int32_t* order) {
  __shared__ int s_cnt[64];
  if (threadIdx.x < 64) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  for (int g = threadIdx.x; g < G; g += blockDim.x) {
    const long long m = off[vptr[g + 1]] - off[vptr[g]];
    atomicAdd(&s_cnt[63 - __clzll(m + 1)], 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int b = 63; b >= 0; --b) {
      const int c = s_cnt[b];
      s_cnt[b] = t;
      t += c;
    }
  }
  __syncthreads();
  for (int g = threadIdx.x; g < G; g += blockDim.x) {
    const long long m = off[vptr[g + 1]] - off[vptr[g]];
    order[atomicAdd(&s_cnt[63 - __clzll(m + 1)], 1)] = g;
  }
}

hipError_t launch_order(const int64_t* vptr, const int64_t* off, int32_t G, int32_t* order,
                        hipStream_t s) {
  hipLaunchKernelGGL(order_kernel, dim3(1), dim3(1024), 0, s, vptr, off, G, order);
  return hipGetLastError();
}

// Live decrements of a finished decomposition: a vertex receives exactly deg(v) - coreness(v)
// decrements while its induced degree is above the round's k (those taking it from deg(v) down to
// k, whatever the order), so their total is offsets[n] - sum of coreness. Adds that to *out.
__global__ __launch_bounds__(1024) void live_count_kernel(const int64_t* off, const int32_t* core, int64_t n,
                                                          unsigned long long* out) {
  __shared__ long long s_w[16];
  long long acc = 0;
  for (long long v = blockIdx.x * 1024ll + threadIdx.x; v < n; v += (long long)gridDim.x * 1024)
    acc += core[v];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane_id() == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int i = 0; i < 16; ++i) t += s_w[i];
    if (blockIdx.x == 0) t = off[n] - off[0] - t;
    else t = -t;
    aadd(out, (unsigned long long)t);
  }
}

hipError_t launch_live_count(const int64_t* off, const int32_t* core, int64_t n, unsigned long long* out,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n + 1023) / 1024;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(live_count_kernel, dim3((unsigned)blocks), dim3(1024), 0, s, off, core, n, out);
  return hipGetLastError();
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void init_ctl_kernel(PeelCtl* c) {
  uint32_t* w = reinterpret_cast<uint32_t*>(c);
  for (size_t i = threadIdx.x; i < offsetof(PeelCtl, trace) / 4; i += blockDim.x) w[i] = 0u;
  __syncthreads();
  if (threadIdx.x < 3) c->slot[threadIdx.x].minv = 0xffffffffu;
  if (threadIdx.x == 0) c->s_valk = 0xffffffffu;
}

hipError_t launch_init_ctl(PeelCtl* c, hipStream_t s) {
  hipLaunchKernelGGL(init_ctl_kernel, dim3(1), dim3(256), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_fill_u32(void* p, uint32_t v, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<uint32_t*>(p), v, count);
  return hipGetLastError();
}

// Input check: offsets start at 0 and never decrease, ids are in range (within the own graph for a
// batch), no self-loops, and every edge appears in both directions (an XOR-sum over a symmetric
// hash of each entry's endpoints cancels exactly when every entry has its reverse, up to hash
// collisions). Duplicates are not detected.
__device__ __forceinline__ unsigned long long pair_hash(unsigned a, unsigned b) {
  unsigned long long lo = a < b ? a : b, hi = a < b ? b : a;
  unsigned long long x = (hi << 32) | lo;
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

__global__ void validate_kernel(const int64_t* off, const int32_t* adj, int64_t n, const int64_t* vptr,
                                int32_t G, unsigned* status, unsigned long long* xsum) {
  const long long gt = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long GT = (long long)gridDim.x * blockDim.x;
  if (gt == 0 && off[0] != 0) atomicOr(status, (unsigned)KC_ERR_BADGRAPH);
  unsigned long long acc = 0;
  for (long long v = gt; v < n; v += GT) {
    const long long b = off[v], e = off[v + 1];
    if (e < b) {
      atomicOr(status, (unsigned)KC_ERR_BADGRAPH);
      continue;
    }
    long long lo = 0, hi = n;
    if (vptr) {
      int l = 0, h = G - 1;  // graph of v: largest g with vptr[g] <= v
      while (l < h) {
        const int mid = (l + h + 1) >> 1;
        if (vptr[mid] <= v) l = mid; else h = mid - 1;
      }
      lo = vptr[l];
      hi = vptr[l + 1];
    }
    for (long long p = b; p < e; ++p) {
      const int32_t u = adj[p];
      if (u < lo || u >= hi || u == v) {
        atomicOr(status, (unsigned)KC_ERR_BADGRAPH);
        break;
      }
      acc ^= pair_hash((unsigned)v, (unsigned)u);
    }
  }
  for (int o = 32; o > 0; o >>= 1) acc ^= __shfl_xor(acc, o, 64);
  if (lane_id() == 0 && acc) atomicXor(xsum, acc);
}

hipError_t launch_validate(const int64_t* off, const int32_t* adj, int64_t n, const int64_t* vptr,
                           int32_t G, unsigned* status, unsigned long long* xsum, hipStream_t s) {
  hipLaunchKernelGGL(validate_kernel, dim3(2048), dim3(256), 0, s, off, adj, n, vptr, G, status, xsum);
  return hipGetLastError();
}

}  // namespace kc
