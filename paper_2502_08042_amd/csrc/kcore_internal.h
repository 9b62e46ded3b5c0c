// Internal declarations shared by the device code and the host-side C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kc {

constexpr int kPeelThreads = 1024;   // threads per persistent workgroup (16 waves)
constexpr int kWaves = kPeelThreads / 64;
constexpr int kStage = 256;          // per-wave LDS staging entries for frontier appends
constexpr int kLocalQ = 512;         // per-wave local queue (chained mode)
constexpr int kCombBits = 13;
constexpr int kCombSlots = 1 << kCombBits;  // per-workgroup LDS combining table for hub targets
constexpr int kCombProbe = 4;               // linear-probe window of that table
constexpr int kEdgeUnroll = 2;              // adjacency entries in flight per lane (rows)
constexpr int kTileUnroll = 4;              //   (hub tiles: a default tile is one pass)
constexpr int kMaxPeelBlocks = 1024;  // workgroups of the persistent grid at most (segmented lists)
static_assert(kPeelThreads >= kMaxPeelBlocks, "one thread per segment when prefixing segment counts");
constexpr int kDbgPhases = 64;             // phases of the per-workgroup debug record
constexpr int kDbgBlocks = 256;
constexpr int kBlockQ = 1024;              // workgroup-local hub tile queue (chained mode)
constexpr int kAsyncWaves = 2;              // waves per workgroup claiming async work
constexpr int kBarGroups = 1;        // arrival groups of the grid barrier (chained instances)
constexpr int kBatchThreads = 512;   // threads per workgroup of the batched peel
constexpr int kTracePhases = 16384;   // phases whose timeline workgroup 0 records
constexpr int kTailThreads = 1024;    // threads of the single-workgroup tail peel
constexpr int kTailUnroll = 4;        //   short rows: adjacency entries in flight per thread
constexpr int kTailBig = 256;         //   rows at least this long are streamed in tiles ...
constexpr int kTailTile = 2048;       //   ... of this many entries (4 16-byte loads of 8 ids per lane)
constexpr uint16_t kTailQEmpty = 0xffffu;  // unwritten slot of the tail's 16-bit queue (ids < 65,535)
constexpr int kBucketSlots = 32;      // multi-bucket active set: one slot per bit of an induced degree
constexpr uint32_t kBucketMinK = 16;  //   kept from the first round with k >= 16 (Sec. 5.2's threshold)

// ST_LIVE: decrements that landed on a vertex still above k (one per peeled vertex and live
// neighbour), computed after the run as offsets[n] - sum of coreness.
// ST_BUCKET: insertions into the multi-bucket active set (placements and moves).
enum StatIdx {
  ST_ROUNDS = 0, ST_SUBROUNDS, ST_BARRIERS, ST_PEELED, ST_EDGES, ST_DECR, ST_COMBINED, ST_SCANNED,
  ST_KMAX, ST_TAIL, ST_SAMPLED, ST_RECOUNTS, ST_LIVE, ST_BUCKET, ST_NUM
};
constexpr int kStatWords = 24;   // statistics words of a control block
constexpr int kDiagWord = 20;    // [20, 24): diagnostics of a failed run

// Counters produced during one phase (three-way rotation, see the peel kernel).
struct alignas(128) PhaseSlot {
  unsigned long long small;   // next small-vertex frontier tail
  unsigned long long tiles;   // next hub-tile list tail
  unsigned long long hubv;    // hub vertices pushed
  unsigned long long active;  // compacted active-list tail
  unsigned long long peeled;  // vertices given a coreness in the phase
  unsigned long long qhead;   // async queue: next slot to claim
  unsigned long long qtail;   //   entries created (= slots filled or being filled)
  unsigned long long qdone;   //   entries fully processed
  unsigned int bdone;         //   workgroups done with their static share
  unsigned int minv;          // min induced degree over vertices kept by a scan
  unsigned int pad[6];
  unsigned long long hadd[kBucketSlots];  // entries appended to each bucket slot in the phase
};

struct alignas(128) PeelCtl {
  unsigned int bar_gen;
  unsigned int pad0[31];
  unsigned int bar_top;
  unsigned int pad1[31];
  unsigned int bar_grp[kBarGroups][32];
  PhaseSlot slot[3];
  unsigned int status;        // error bits (KC_ERR_*)
  unsigned int pad2[31];
  // live vertices handed to the tail peel (0 = none) and the round at which they were handed over
  unsigned long long tail_n;
  unsigned long long tail_k;
  // sampling mode: smallest round at which a sampled vertex must be validated, candidates listed
  unsigned int s_valk;
  unsigned int s_ncand;
  unsigned long long pad3[13];
  unsigned long long stats[kStatWords];
  // survivors each workgroup wrote into its segment of active list 0 / 1 (see the peel kernel)
  unsigned int acnt[2][kMaxPeelBlocks];
  // phase timeline of workgroup 0, not cleared between launches: 100 MHz wall clock at start,
  // work done, flushed and barrier passed; then kind | precheck << 4 | async << 5 | k << 8, the
  // frontier's vertices, its hub tiles and the active-set size
  unsigned long long trace[kTracePhases][8];
  // per-workgroup record of the phases [dbg_lo, dbg_lo + kDbgPhases) when asked for: start, work
  // done, tiles taken from the workgroup queue, vertices peeled from local queues
  unsigned long long dbg[kDbgPhases][kDbgBlocks][4];
};

// KC_ERR_SAMPLE: a sampled vertex was found below k at a round boundary (the Las Vegas check of
// the sampling scheme); the host then runs the decomposition again without sampling.
// KC_ERR_CHECK: (checked builds only) a coreness written twice or an induced degree decremented
// below zero.
enum : unsigned { KC_ERR_TIMEOUT = 1u, KC_ERR_OVERFLOW = 2u, KC_ERR_PHASES = 4u, KC_ERR_BADGRAPH = 8u,
                  KC_ERR_SAMPLE = 16u, KC_ERR_CHECK = 32u };

struct PeelArgs {
  const int64_t* off;
  const int32_t* adj;
  int64_t n;
  int64_t m_bound;     // entries adj holds at most; the kernel stops with KC_ERR_OVERFLOW when
                       // offsets[n] exceeds it (the workspace was sized from it)
  int32_t* core;
  uint32_t* dt;        // induced degree, bit 31 = hub flag
  uint32_t* state;     // per 16 vertices: bits 0..15 peeled, 16..31 hub
  int32_t* act[2];     // compacted active lists
  int32_t* fr[2];      // small-vertex frontiers
  unsigned long long* tl[2];  // hub tiles: first entry << 16 | length
  int64_t fcap;        // frontier capacity (entries)
  int64_t tcap;        // tile list capacity
  PeelCtl* ctl;
  uint32_t hub;        // rows of vertices with at least this degree are split into tiles
  uint32_t comb_degree;// decrements to vertices with at least this degree are combined in LDS
  int32_t tile;        // edges per tile (multiple of 64)
  int32_t chained;     // 1: local queues (chained mode)
  int32_t lq_budget;   // max vertices a wave peels from its local queue per phase
  int64_t big_phase;   // frontier size from which a phase probes peeled bits and combines hubs
  long long* aq;       // async work queue (entries, -1 = empty), qcap slots
  int64_t qcap;
  int64_t async_small; // chained mode: frontiers up to this many small vertices ...
  int64_t async_tiles; //   ... and tiles are peeled by an async phase
  int64_t async_scan_max; // chained mode: active sets up to this size scan and peel in one phase
  int32_t bq_max_tiles;   // chained mode: hubs of at most this many tiles stay in the workgroup (0 = off)
  int32_t bq_backlog;     //   while at most this many tiles wait unclaimed in the workgroup's queue
  int64_t dbg_lo;         // first phase of the per-workgroup debug record (-1 = none)
  int32_t tile_probe_always; // hub tiles probe peeled bits in every phase (else in large ones only)
  long long* rrow;        // residual rows: [2v] first entry, [2v + 1] end, in radj
  int32_t* radj;          // residual adjacency (live neighbours only), rcap entries
  int64_t rcap;
  int64_t resid_vmax;     // rewrite the rows once the active set is at most this large (-1 = never)
  int64_t k_query;        // >= 1: only the k_query-core (one round at k_query - 1, membership out)
  // tail handoff: once at most tail_vmax vertices are live at a round boundary (-1 = never), they
  // are renumbered 0..L-1 (tmap: id -> local id, tgid: local id -> id) and their rows rewritten
  // with live neighbours only, in local ids (trow: [2i] first entry, [2i + 1] end, in tadj)
  int64_t tail_vmax;
  int32_t* tmap;
  int32_t* tgid;
  long long* trow;
  uint16_t* tadj;         // 16-bit local ids (the tail holds fewer than 65,535 vertices)
  int64_t tail_ecap;      // entries tadj holds
  // multi-bucket active set (Sec. 5.2): slot b holds the vertices whose induced degree x > k has
  // its highest bit differing from k at bit b, entries [b * hcap, b * hcap + length) of hbl;
  // hlo[v] is the lower bound of the range v was last filed into (0 = none), hslots the slots in
  // use (values below 2^hslots); started at the first round boundary with k >= kBucketMinK and at
  // most hbs_vmax live vertices (-1 = never)
  int32_t* hbl;
  uint32_t* hlo;
  int64_t hcap;
  int32_t hslots;
  int64_t hbs_vmax;
  // sampling mode (Alg. 4/5): vertices of degree above s_threshold start in sample mode; per vertex
  // the hit threshold of the counter-based coin (rate x 2^32, 0 = not sampled), the hits, the
  // induced degree at the last (re)initialisation and a recount accumulator; the candidates list
  // and the list of vertices being recounted
  int32_t sampling;
  uint32_t s_threshold;
  uint32_t s_mu;          // hits expected before a resample (mu of Alg. 5)
  uint32_t s_seed;
  uint32_t* srate;
  uint32_t* scnt;
  uint32_t* sbase;
  uint32_t* scount;
  int32_t* scand;
  int32_t* srl;
};

constexpr int kMaxTeams = 64;       // batched peel: largest graphs peeled by a team of workgroups
constexpr int kTeamSize = 8;        //   workgroups per team (default; at most kMaxTeamSize)
constexpr int kMaxTeamSize = 32;

// One team's control block: barrier arrivals, the graph's peel-queue tail, and the per-round
// minimum of the kept induced degrees (three-way rotation, stored complemented so that zero
// initialisation and atomic max give "no value yet").
struct alignas(128) TeamCtl {
  unsigned int bar;               // arrivals (monotone)
  unsigned int gen;               // barriers released (written by the last arrival)
  unsigned int pad0[30];
  unsigned long long tail;        // the graph's peel-queue tail
  unsigned long long snap[2];     // tail as the last arrival of barrier e saw it, in snap[e & 1]
  unsigned int rmx[3];
  unsigned int pad1[23];
};

struct BatchCtl {
  unsigned long long next;
  unsigned int status;
  unsigned int nteams;    // leading graphs of the processing order peeled by teams
  unsigned int team_size; // workgroups per team
  unsigned int pad[27];
  unsigned long long stats[kStatWords];
  TeamCtl team[kMaxTeams];
};

struct BatchArgs {
  const int64_t* vptr;
  const int64_t* off;
  const int32_t* adj;
  int32_t G;
  int32_t* core;
  const int32_t* order;   // processing order (largest first)
  uint32_t* gdt;          // global induced degrees for graphs beyond the LDS capacity
  int32_t* gq;            // global peel queues for those graphs
  int32_t* ga;            // global active lists for those graphs
  int32_t local_ids;      // adjacency holds per-graph local ids (serving) instead of global ids
  BatchCtl* ctl;
  int32_t lds_cap;        // vertices per graph held in LDS
  int32_t chained;        // 1: each round is peeled through a dynamic workgroup queue (no subround barriers)
  int32_t teams;          // 1: the plan kernel may give the largest graphs teams of workgroups (it
                          // writes ctl->nteams and ctl->team_size; teams wait for each other: see
                          // the launch)
};

// Error text returned by kcore_last_error (thread-local; defined in kcore_api.cpp).
void set_error(const char* msg);

// kcore_decompose_batched with per-graph local ids in adj (used by the serving runtime, which
// then packs requests without rewriting their adjacency). Defined in kcore_api.cpp.
// Grows the batched-peel workspace of (current device, stream) to V vertices and G graphs now.
int reserve_batched(hipStream_t stream, int64_t V, int32_t G);
// Frees the batched-peel workspace of (current device, stream), if any (before the stream goes).
void release_batched(hipStream_t stream);
// team_wgs > 0: every graph of the batch (up to kMaxTeams, within team_wgs workgroups) is peeled
// by a team, in a grid launched without co-residency guarantee; the caller keeps the team
// workgroups of all such batches that may run at once within what the device holds resident (other
// workgroups do not wait on anything, so teams then always complete).
int decompose_batched_local(const int64_t* graph_vptr, const int64_t* offsets, const int32_t* adj,
                            int32_t num_graphs, int64_t total_vertices, int32_t* coreness_out,
                            hipStream_t stream, unsigned* status_out, int32_t team_wgs = 0);
// Workgroups of the batched peel resident on the current device at once (0 if unknown).
int batched_resident_wgs();
int64_t batched_lds_vertices();  // vertices of a graph the batched peel keeps in LDS

// Launch helpers (defined in kcore_device.hip).
hipError_t launch_peel(const PeelArgs& a, int blocks, hipStream_t s);
hipError_t peel_occupancy(int* blocks_per_cu);
hipError_t launch_batched(const BatchArgs& a, int blocks, size_t lds_bytes, hipStream_t s);
hipError_t launch_batched_coop(const BatchArgs& a, int blocks, size_t lds_bytes, hipStream_t s);
hipError_t batched_occupancy(size_t lds_bytes, int* blocks_per_cu);
hipError_t launch_order(const int64_t* vptr, const int64_t* off, int32_t G, int32_t* order,
                        hipStream_t s);
// Picks the leading graphs of `order` whose entries exceed half a workgroup's average share
// (blocks workgroups; every leading graph when `all`) for teams of team_size workgroups (0: sized
// from team_wgs), using at most team_wgs workgroups; writes ctl->nteams and ctl->team_size.
// min_entries > 0 replaces the size rule: graphs with more entries than that get teams.
hipError_t launch_team_plan(const int64_t* vptr, const int64_t* off, int32_t G, const int32_t* order,
                            int32_t blocks, int32_t team_wgs, int32_t team_size, int32_t all, int64_t min_entries,
                            BatchCtl* ctl, hipStream_t s);
hipError_t launch_fill_u32(void* p, uint32_t v, size_t count, hipStream_t s);
// Adds offsets[n] - offsets[0] - sum(core[0..n)) (the live decrements of a finished decomposition)
// to *out.
hipError_t launch_live_count(const int64_t* off, const int32_t* core, int64_t n, unsigned long long* out,
                             hipStream_t s);
hipError_t launch_init_ctl(PeelCtl* c, hipStream_t s);
// Single-workgroup peel of the live vertices handed over by peel_kernel (returns at once when none
// were); lcap = vertices its LDS holds.
hipError_t launch_tail(const PeelArgs& a, int32_t lcap, hipStream_t s);
// Static LDS of the chained (1) or level-sync (0) instance, and allowing it lcap vertices.
hipError_t tail_static_lds(int chained, size_t* bytes);
hipError_t tail_allow_lds(int chained, int32_t lcap);
hipError_t launch_validate(const int64_t* off, const int32_t* adj, int64_t n, const int64_t* vptr,
                           int32_t G, unsigned* status, unsigned long long* xsum, hipStream_t s);

}  // namespace kc
