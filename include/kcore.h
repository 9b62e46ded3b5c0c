/*
 * kcore.h — exact k-core decomposition on AMD Instinct MI355X (gfx950).
 *
 * Computes the coreness of every vertex of an undirected simple graph: the largest k such that the
 * vertex belongs to the k-core, the largest subgraph whose vertices all have degree >= k
 * (paper: "Parallel k-Core Decomposition: Theory and Practice", Sec. 1 and Sec. 2, Notations).
 * The method is the paper's work-efficient framework (Alg. 1) — rounds k = 0, 1, ... over an
 * active set, each round peeling frontiers of vertices whose induced degree is at most k in
 * subrounds — with the online peel of Alg. 3: peeling v atomically decrements the induced degree
 * of each live neighbour u, and the decrement that takes u from above k to k or below pushes u
 * into the next frontier.
 *
 * Graph layout (all entry points): CSR with both directions of every undirected edge stored.
 *   offsets  int64[n+1], offsets[0] = 0, non-decreasing; row v is adj[offsets[v] .. offsets[v+1])
 *   adj      int32[offsets[n]], neighbour ids in [0, n)
 * The graph must be simple and symmetric: no self-loops, no duplicate entries in a row, and u in
 * row v iff v in row u. Rows need not be sorted. Inputs that break this contract are peeled
 * literally (memory-safe as long as every id is in range); set kcore_options.validate to have the
 * device reject them with KCORE_EBADGRAPH instead.
 *
 * Calls are stream-ordered and asynchronous unless stated: a return of KCORE_OK means the work is
 * enqueued on `stream`; coreness_out is valid once the stream reaches that point, and the host
 * never waits for the device. Argument errors are reported synchronously and enqueue nothing.
 * Failures the device detects while peeling (a bounded wait that gave up, a list that overflowed,
 * offsets[n] beyond what adj can hold) leave coreness_out incomplete and are reported through the
 * device status word: read it with kcore_check(stream) after the work, have it copied to
 * kcore_options.status_out in stream order, or pass a kcore_stats* (synchronous). The caller
 * owns every buffer it passes; the library owns its device workspace, cached per (device, stream)
 * and reused across calls (see kcore_release_workspaces). Calls on distinct streams may run concurrently; calls on one stream
 * are serialised by it. Exception: the single-graph peel (kcore_decompose*, kcore_kcore_subgraph)
 * runs a persistent grid that fills the device, so those grids run one at a time per device, each
 * after the one launched before it (ordered through the streams; the host does not block).
 * hipStream_t 0 is the legacy default stream.
 */
#ifndef KCORE_H_
#define KCORE_H_

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KCORE_OK = 0,
  KCORE_PENDING = 1,      /* kcore_poll: request not finished yet */
  KCORE_EINVAL = -1,      /* bad argument (null pointer, negative size, bad option) */
  KCORE_ENOMEM = -2,      /* device or host allocation failed */
  KCORE_EDEVICE = -3,     /* HIP runtime error, or the device reported an internal failure */
  KCORE_ETOOBIG = -4,     /* request can never fit the configured limits */
  KCORE_ENOTFOUND = -5,   /* kcore_poll: unknown ticket, or result already taken */
  KCORE_ECANCELED = -6,   /* kcore_poll: request was cancelled */
  KCORE_EBADGRAPH = -7    /* validate mode: CSR breaks the input contract */
} kcore_status;

/* Peeling schedules of the single-graph path. */
typedef enum {
  KCORE_MODE_AUTO = 0,      /* library choice (currently KCORE_MODE_CHAINED) */
  KCORE_MODE_LEVELSYNC = 1, /* Alg. 1 + Alg. 3 literally: one grid-wide barrier per subround; the
                               frontiers, and so the subround count rho (Sec. 3.2, span analysis),
                               equal those of the sequential framework */
  KCORE_MODE_CHAINED = 2,   /* vertices that drop to k inside a round are peeled in the same
                               pass by whichever workgroup finds them, without waiting for a
                               barrier (the idea of vertical granularity control, Sec. 4.2);
                               one grid-wide barrier per round */
  KCORE_MODE_SAMPLING = 3,  /* chained, with the sampling scheme of Sec. 4.1 (Alg. 4/5) for
                               vertices of degree above 1024 instead of LDS combining: removing a
                               neighbour counts a hit with probability mu / (0.9 d*) instead of
                               decrementing, sampled vertices are validated and recounted at round
                               boundaries; a sampled vertex found below k there voids the run,
                               which is repeated in chained mode (the result is always exact).
                               The call then synchronises `stream`. No tail handoff, no residual
                               rows; at most 2^30 vertices; not for kcore_kcore_subgraph */
  KCORE_MODE_OFFLINE = 4    /* level-sync subrounds with the offline peel of Alg. 2: within a
                               subround each workgroup first counts the decrements per target in
                               an LDS table (the histogram), then applies each count once with the
                               batch rule old > k >= old - c; targets that find no free slot of the
                               8,192 are decremented directly. Frontiers and rho are those of
                               KCORE_MODE_LEVELSYNC */
} kcore_mode;

typedef struct {
  int32_t mode;          /* kcore_mode */
  int32_t validate;      /* nonzero: check the CSR on the device first (KCORE_EBADGRAPH);
                            makes the call synchronous on `stream` */
  int32_t blocks_per_cu; /* persistent workgroups per compute unit; 0 = library choice */
  int32_t hub_degree;    /* vertices with at least this degree are split into tiles of
                            `tile_edges` adjacency entries when peeled; 0 = library choice */
  int64_t num_entries;   /* offsets[n] when the caller knows it, to size the workspace exactly;
                            0 = unknown: the workspace is then sized for the device allocation
                            that holds adj (from its base and size as the HIP runtime reports
                            them, at most n (n - 1) entries), with no host-device round trip; only
                            for a pointer the runtime cannot attribute to an allocation is
                            offsets[n] read with a blocking 8-byte copy. Either way the device
                            checks offsets[n] against the size used before it reads any entry
                            (a failure reported through the status word, see kcore_check) */
  int32_t local_budget;  /* chained mode: vertices one wavefront may peel from its local queue per
                            phase (or per asynchronous queue entry) before handing the rest to the
                            global frontier or queue; 0 = default (1024) */
  int32_t tile_edges;    /* adjacency entries per hub tile (multiple of 64, at most 32768);
                            0 = default */
  int32_t async_frontier;/* chained mode: a frontier of at most this many vertices (and as many
                            hub tiles) is peeled by one asynchronous phase with a shared work
                            queue instead of barrier-separated subrounds; 0 = default, -1 = never */
  int32_t async_scan;    /* chained mode: while the active set has at most this many vertices the
                            round's scan and its whole peel run as one asynchronous phase (one
                            barrier per round); 0 = default, -1 = never */
  int32_t block_tiles;   /* chained mode: a hub of at most this many tiles, pushed during a phase,
                            is peeled in the same phase by the 16 wavefronts of the workgroup that
                            pushed it (workgroup-local tile queue) instead of in the next phase by
                            the whole grid; 0 = default, -1 = never */
  int32_t block_queue;   /* chained mode: a workgroup queues a hub's tiles only while at most this
                            many tiles wait unclaimed in its queue (at most 1024); otherwise they
                            go to the next phase's global list, so a burst of hubs is spread over
                            the grid instead of holding one workgroup up; 0 = default */
  int32_t tile_probe;    /* 0 = default: hub tiles skip neighbours already peeled (one probe of a
                            bitmap per entry, fewer atomics); -1 = only in large phases, so small
                            latency-bound phases save a memory round trip per tile */
  int32_t residual;      /* chained and level-sync modes: once the active set has at most this many
                            vertices (at a round boundary), the rows of the live vertices are
                            rewritten once without their peeled neighbours, so later rounds stop
                            reading dead entries; costs 16 bytes per vertex and half the adjacency
                            in workspace; 0 = default (n / 256, at least 4096), -1 = never */
  int32_t tail;          /* once at most this many vertices are live at a round boundary (they then
                            form the k-core of that round, whose coreness is the same inside it
                            as in the whole graph), one workgroup finishes the decomposition on
                            them with their induced degrees in LDS, so the last, small rounds
                            synchronise at workgroup level instead of grid-wide (the k-core
                            query never hands over); costs 4 bytes per vertex plus
                            min(m, tail^2) 16-bit entries of workspace; capped at what the
                            workgroup's LDS holds at 6 bytes per vertex (on a 160 KB-LDS device
                            26,624 in chained mode, 23,552 in the level-sync and offline modes,
                            whose tail keeps 16 KB of scan arrays); 0 = default, min(that cap,
                            n / 8); -1 = never */
  int32_t buckets;       /* chained and level-sync modes: multi-bucket active set (Sec. 5.2, HBS).
                            From the first round boundary with k >= 16 at which at most this many
                            vertices are live, live vertices are kept in buckets by the highest bit
                            in which their induced degree differs from k (ranges 1, 2, 4, ... above
                            k, aligned to powers of two), so a round reads only the bucket that
                            holds the new k and moves its other entries to lower buckets; a
                            decrement that takes a vertex below its bucket's range moves it.
                            Costs 2 x 31 int32 slots per such vertex plus 4 bytes per vertex of
                            workspace. 0 = default (off), -1 = never, > 0 = that many vertices */
  int32_t sample_threshold; /* sampling mode: vertices of degree above this start sampled;
                            0 = default (1024) */
  int32_t sample_mu;     /* sampling mode: hits expected before a resample (mu of Alg. 5);
                            0 = default (4 (c + 2) ln n with c = 1, at least 16) */
  int32_t debug_phase;   /* debugging: record every workgroup's timing in phases
                            [debug_phase, debug_phase + 64) (read with kcore_debug_blocks, not
                            part of this header); 0 = off */
  int64_t test_tail_entries; /* testing: pretend the tail's local rows hold at most this many
                            entries, so that handoffs are called off and retried; 0 = off */
  int32_t team_size;     /* batched peel: workgroups per team (see batch_teams); 0 = default (the
                            teams share a quarter of the grid equally, 8 to 32 workgroups each),
                            at most 32 */
  int32_t combine_degree;/* chained and level-sync modes: in large phases, decrements of vertices of at
                            least this degree are combined in the workgroup's LDS table and applied
                            once per target; 0 = default (max(1024, hub_degree)) */
  int32_t big_phase;     /* frontier size (entries of small vertices plus 16 per hub tile) from
                            which a phase probes peeled bits before decrementing and combines; 0 =
                            default (16384) */
  int32_t batch_teams;   /* batched peel (level-sync): a graph with more adjacency entries than this
                            is peeled by a team of workgroups; 0 = default (half a workgroup's
                            average share of the batch's entries), -1 = never */
  uint32_t* status_out;  /* nullable, device or pinned host memory: receives the device status word
                            of the call (0 = success, else internal failure bits) when `stream`
                            reaches the end of the call */
} kcore_options;

/* Counters of one decomposition (filled when a kcore_stats* is passed; that call synchronises
 * `stream`). Field meanings follow the paper's framework. */
typedef struct {
  int64_t rounds;          /* non-empty rounds = number of distinct coreness values */
  int64_t subrounds;       /* peel passes over a non-empty frontier (rho in level-sync mode) */
  int64_t barriers;        /* grid-wide synchronisations executed */
  int64_t peeled;          /* vertices given a coreness (= n) */
  int64_t edges;           /* adjacency entries expanded (= m; entries dropped when rows are
                              rewritten without peeled neighbours count as expanded there, and so
                              do the tail's rows left unread once all its vertices are queued) */
  int64_t decrements;      /* global atomic decrements issued */
  int64_t combined;        /* decrements absorbed by LDS combining */
  int64_t scanned;         /* active-set slots scanned (Thm. 3.1 bounds this by n + m) */
  int32_t kmax;            /* largest coreness */
  int32_t device_status;   /* 0, or internal failure bits */
  float ms;                /* device time of the call in milliseconds */
  int32_t tail_vertices;   /* vertices peeled by the single-workgroup tail (0 = no handoff); its
                              decrements are LDS operations and not counted in `decrements` */
  int32_t sampled_vertices;/* sampling mode: vertices that started in sample mode */
  int32_t sample_recounts; /* sampling mode: validations that recounted a vertex's live degree */
  int32_t sample_restarts; /* sampling mode: 1 if the sampled run failed and was repeated */
  int32_t reserved[1];
  int64_t live_decrements; /* decrements that land on a vertex still above k (Alg. 1's test
                              "induced degree > k"): one per peeled vertex and live neighbour, at
                              most m / 2 on a simple graph. A vertex receives exactly deg - coreness
                              of them whatever the order, so this is computed after the run as
                              offsets[n] - sum of coreness (0 for the k-core query) */
  int64_t bucket_inserts;  /* insertions into the multi-bucket active set (kcore_options.buckets):
                              placements, moves to lower buckets and redistributions */
} kcore_stats;

/* Single graph. n == 0 is a no-op; adj may be null when offsets[n] == 0; KCORE_ETOOBIG when
 * offsets[n] >= 2^47. */
int kcore_decompose(const int64_t* offsets, const int32_t* adj, int64_t n, int32_t* coreness_out,
                    hipStream_t stream);

/* As kcore_decompose with options (nullable: defaults) and statistics (nullable; non-null makes
 * the call synchronous on `stream`). */
int kcore_decompose_ex(const int64_t* offsets, const int32_t* adj, int64_t n, int32_t* coreness_out,
                       hipStream_t stream, const kcore_options* opt, kcore_stats* stats_host);

/* Maximum k-core subgraph (App. B): the framework with its peeling condition fixed at "induced
 * degree below k", i.e. one round at threshold k - 1 with the same (chained) subrounds, after which
 * the survivors form the k-core (the largest subgraph of minimum degree >= k).
 *   in_core_out  int32[n] on the device: 1 if v belongs to the k-core, else 0
 * k <= 0 marks every vertex. Arguments, options, statistics (rounds <= 1) and errors as
 * kcore_decompose_ex. */
int kcore_kcore_subgraph(const int64_t* offsets, const int32_t* adj, int64_t n, int32_t k,
                         int32_t* in_core_out, hipStream_t stream, const kcore_options* opt,
                         kcore_stats* stats_host);

/* Many independent graphs in one segmented CSR (device pointers). Graph g owns the global vertex
 * range [graph_vptr[g], graph_vptr[g+1]); its rows use global ids inside that range. The k-cores
 * of a disjoint union are the unions of the k-cores of its parts, so every graph is peeled on its
 * own k cursor; one launch covers the whole batch.
 *   graph_vptr  int64[num_graphs+1] on the device, graph_vptr[0] = 0,
 *               graph_vptr[num_graphs] = total_vertices, non-decreasing
 *   offsets     int64[total_vertices+1], adj int32[offsets[total_vertices]] (global ids; must be
 *               non-null even when the batch has no edges)
 *   coreness_out int32[total_vertices]
 * Options of the _ex form: mode LEVELSYNC (= AUTO) peels each round in barrier-separated
 * subrounds inside the graph's workgroup; CHAINED works each round off through a dynamic
 * workgroup queue. validate, blocks_per_cu and status_out apply; the other fields are ignored.
 * A device failure is reported as for the single-graph calls (kcore_check, status_out, or
 * stats_host). */
int kcore_decompose_batched(const int64_t* graph_vptr, const int64_t* offsets, const int32_t* adj,
                            int32_t num_graphs, int64_t total_vertices, int32_t* coreness_out,
                            hipStream_t stream);

int kcore_decompose_batched_ex(const int64_t* graph_vptr, const int64_t* offsets,
                               const int32_t* adj, int32_t num_graphs, int64_t total_vertices,
                               int32_t* coreness_out, hipStream_t stream, const kcore_options* opt,
                               kcore_stats* stats_host);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): kcore_decompose_batched without any allocation. Same
 * arguments, layout and result as kcore_decompose_batched (level-sync mode); its workspace is a
 * device array inside the library, one per GPU, held until the process ends: 12.8 MB for at most
 * 2^20 vertices and 2^16 graphs per call (larger batches: KCORE_ETOOBIG, nothing enqueued). Every
 * call on a GPU shares that GPU's array, so calls that overlap on one GPU (from several streams
 * or threads) race and must be serialised by the caller. The control block is cleared by a kernel
 * at the start of each call (no memset node), so the call can be captured into a graph.
 *   status_out  nullable, device or pinned host memory: receives the device status word (0 =
 *               success) when `stream` reaches the end of the call */
int kcore_decompose_batched_noalloc(const int64_t* graph_vptr, const int64_t* offsets, const int32_t* adj,
                                    int32_t num_graphs, int64_t total_vertices, int32_t* coreness_out,
                                    uint32_t* status_out, hipStream_t stream);

/* Frees every cached workspace after synchronising the device. */
int kcore_release_workspaces(void);

/* Waits for `stream`, then reads the device status words of the last single-graph and the last
 * batched call made on it (blocks the calling thread). KCORE_OK when neither reported a failure,
 * KCORE_EDEVICE otherwise (kcore_last_error names the bits), KCORE_ENOTFOUND when no call ran on
 * this stream of the current device. */
int kcore_check(hipStream_t stream);

/* ------------------------------------------------------------------------------------------------
 * Serving: continuous batching of independent graph requests on one device.
 *
 * kcore_submit copies a HOST graph before it returns (the caller may free its buffers at once)
 * unless borrow_inputs is set, and hands back a ticket. A dispatcher thread admits queued requests while
 * their device footprint fits the HBM budget and a batch slot is free, packs them into a segmented
 * CSR and launches the batched peel; up to max_inflight batches run concurrently on separate
 * streams, so requests that arrive while others are on the GPU start as soon as a slot and memory
 * free up. Results are copied back to pinned host memory; kcore_poll hands them out.
 * ---------------------------------------------------------------------------------------------- */
typedef struct kcore_server kcore_server;

typedef struct {
  int32_t device;              /* HIP device ordinal */
  int32_t max_inflight;        /* concurrent batches on the device, one stream each (>= 1; 0 = 4);
                                  each stream needs a hardware queue of its own, else batches
                                  share queues and wait for each other: HIP gives a process
                                  GPU_MAX_HW_QUEUES of them (4 unless the environment says
                                  otherwise before HIP initialises), and the runtime takes some
                                  for itself (cooperative launches use one), so leave room */
  int32_t max_batch_graphs;    /* graphs per batch (0 = 4096) */
  int32_t max_large_inflight;  /* batches of large requests (see large_vertices) in flight at
                                  once, each graph of them peeled by a team of workgroups within
                                  half the device (0 = max_inflight / 2, at least 1, below
                                  max_inflight). Requests between the batched peel's LDS capacity
                                  (about 9,000 vertices, by device) and the large class are
                                  medium: batched apart from the small ones, in at most half of
                                  the other slots (at least 1), so that small requests always have
                                  slots that no slower graph holds up */
  int64_t max_batch_vertices;  /* vertices per batch (0 = 1 << 24) */
  int64_t hbm_budget_bytes;    /* device bytes all in-flight batches may hold (0 = 8 GiB) */
  int64_t max_request_vertices;/* larger requests are rejected with KCORE_ETOOBIG (0 = no limit) */
  double batch_wait_us;        /* how long the dispatcher waits to grow a batch while the device
                                  is busy (0 = 50 us) */
  int32_t borrow_inputs;       /* nonzero: kcore_submit does not copy; the caller keeps offsets and
                                  adj unchanged and alive until kcore_poll/kcore_wait returns the
                                  result (host-to-device copies then read them directly, at DMA
                                  speed when the caller's memory is pinned) */
  int32_t large_vertices;      /* requests with at least this many vertices, or 32 times as many
                                  adjacency entries, are large (0 = 65,536, i.e. also 2^21 entries) */
  int64_t reserve_vertices;    /* nonzero: every slot allocates, at creation, device and pinned
                                  buffers for batches of this many vertices and reserve_entries
                                  adjacency entries, and a peel workspace for max_batch_vertices,
                                  so that serving rarely stops to allocate or pin memory (buffers
                                  a slot outgrows are kept until kcore_server_destroy) */
  int64_t reserve_entries;
  uint64_t fail_ticket;        /* testing: the launch of any batch holding this ticket fails with
                                  KCORE_EDEVICE before it touches the device (0 = none); as with a
                                  real launch failure, the batch's requests are retried one per
                                  batch, so only the failing request ends in an error */
} kcore_server_config;

typedef struct {
  double submit_us;   /* submit time, microseconds on the server's steady clock */
  double admit_us;    /* admitted into a batch */
  double launch_us;   /* batch packed and enqueued on its stream */
  double done_us;     /* result visible to kcore_poll */
  int64_t batch_id;   /* batch the request ran in */
  int32_t batch_graphs;
  int32_t reserved;
} kcore_request_stats;

/* Returns null on failure (see kcore_last_error). */
kcore_server* kcore_server_create(const kcore_server_config* cfg);

/* Host CSR (offsets int64[n+1], adj int32[offsets[n]]), copied before return unless the server
 * borrows inputs (kcore_server_config.borrow_inputs). */
int kcore_submit(kcore_server* s, const int64_t* offsets_host, const int32_t* adj_host, int64_t n,
                 uint64_t* ticket_out);

/* KCORE_PENDING until done; then KCORE_OK once (coreness_host_out int32[n] filled, stats if
 * non-null), after which the ticket is forgotten (KCORE_ENOTFOUND). */
int kcore_poll(kcore_server* s, uint64_t ticket, int32_t* coreness_host_out,
               kcore_request_stats* st);

/* Blocks until the ticket is done (or timeout_us elapses: KCORE_PENDING), then behaves as
 * kcore_poll. */
int kcore_wait(kcore_server* s, uint64_t ticket, int32_t* coreness_host_out,
               kcore_request_stats* st, double timeout_us);

/* Cancels a queued request (KCORE_OK) or reports KCORE_PENDING if it is already on the device. */
int kcore_cancel(kcore_server* s, uint64_t ticket);

/* Microseconds on the server's steady clock (the time base of kcore_request_stats). */
double kcore_server_now_us(const kcore_server* s);

/* Drains in-flight batches, then frees everything. */
void kcore_server_destroy(kcore_server* s);

/* Message of the last error on the calling thread ("" if none). */
const char* kcore_last_error(void);

/* Library version: major * 10000 + minor * 100 + patch. */
int kcore_version(void);

#ifdef __cplusplus
}
#endif
#endif /* KCORE_H_ */
