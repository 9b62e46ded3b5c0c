// Seeded synthetic graph generators shared by the tests, the oracle checks and the benchmark.
//
// This module holds no k-core arithmetic: it only draws graphs and lays them out as a simple
// undirected CSR (int64 row offsets, int32 neighbour ids, both directions of every edge stored,
// rows sorted, no self-loops, no duplicate entries). Every random choice comes from a
// counter-based splitmix64 stream keyed by (seed, stream id, index), so a graph is a pure
// function of its parameters and does not depend on the number of host threads.
//
// Families (sizes and distributions follow the workloads the method is evaluated on):
//   * R-MAT with quadrant probabilities a,b,c,d (social/web-like skew)
//   * a 2D grid with random edge deletions and random unit-square diagonals (road-like)
//   * Chung-Lu power law with a planted dense G(n_b, p) block (high-coreness core + hubs)
//   * Erdos-Renyi G(n, p) by geometric skipping over the pair index space
//   * a batch of many small ER / R-MAT graphs packed into one segmented CSR
//   * arbitrary edge lists (symmetrised, de-duplicated) for hand-built test graphs
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>
#include <omp.h>
#include <chrono>
#include <cstdio>

namespace {

struct Timer {
  const char* what;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  explicit Timer(const char* w) : what(w) {}
  ~Timer() {
    if (std::getenv("GG_VERBOSE"))
      std::fprintf(stderr, "[graphgen] %s %.3f s\n", what,
                   std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
  }
};

inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// Counter-based stream: value number `i` of stream `s` under `seed`.
inline uint64_t stream_key(uint64_t seed, uint64_t s) {
  return splitmix64(seed ^ splitmix64(s + 0x632BE59BD9B4E019ull));
}
inline uint64_t rnd(uint64_t seed, uint64_t s, uint64_t i) { return splitmix64(stream_key(seed, s) + i); }
// Uniform double in [0, 1) with 53 random bits.
inline double u01(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

struct Csr {
  int64_t n = 0;
  std::vector<int64_t> off;
  std::vector<int32_t> adj;
};

// Builds a symmetric, sorted, duplicate-free, loop-free CSR from undirected pairs.
// Pairs with a negative endpoint are ignored (used to mark rejected draws).
void build_csr(int64_t n, const std::vector<int32_t>& src, const std::vector<int32_t>& dst, Csr& g) {
  const int64_t P = (int64_t)src.size();
  std::vector<int64_t> cnt(n + 1, 0);
  {
    Timer t_("csr count");
    std::atomic<int64_t>* c = reinterpret_cast<std::atomic<int64_t>*>(cnt.data());
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < P; ++i) {
      int32_t u = src[i], v = dst[i];
      if (u < 0 || v < 0 || u == v) continue;
      c[u].fetch_add(1, std::memory_order_relaxed);
      c[v].fetch_add(1, std::memory_order_relaxed);
    }
  }
  std::vector<int64_t> start(n + 1, 0);
  for (int64_t v = 0; v < n; ++v) start[v + 1] = start[v] + cnt[v];
  std::vector<int32_t> tmp((size_t)start[n]);
  {
    Timer t_("csr scatter");
    std::vector<int64_t> cur(start.begin(), start.end() - 1);
    std::atomic<int64_t>* c = reinterpret_cast<std::atomic<int64_t>*>(cur.data());
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < P; ++i) {
      int32_t u = src[i], v = dst[i];
      if (u < 0 || v < 0 || u == v) continue;
      tmp[c[u].fetch_add(1, std::memory_order_relaxed)] = v;
      tmp[c[v].fetch_add(1, std::memory_order_relaxed)] = u;
    }
  }
  std::vector<int64_t> ndeg(n, 0);
  Timer t_sort("csr sort+copy");
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < n; ++v) {
    int32_t* b = tmp.data() + start[v];
    int32_t* e = tmp.data() + start[v + 1];
    std::sort(b, e);
    ndeg[v] = std::unique(b, e) - b;
  }
  g.n = n;
  g.off.assign(n + 1, 0);
  for (int64_t v = 0; v < n; ++v) g.off[v + 1] = g.off[v] + ndeg[v];
  g.adj.resize((size_t)g.off[n]);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < n; ++v)
    std::memcpy(g.adj.data() + g.off[v], tmp.data() + start[v], sizeof(int32_t) * ndeg[v]);
}

// One R-MAT endpoint pair drawn with `levels` quadrant choices from counter position `i`.
inline void rmat_pair(uint64_t seed, uint64_t stream, uint64_t i, int levels, double a, double b,
                      double c, int64_t& u, int64_t& v) {
  u = 0;
  v = 0;
  const uint64_t key = stream_key(seed, stream);
  for (int l = 0; l < levels; ++l) {
    double r = u01(splitmix64(key + i * 64 + (uint64_t)l));
    int64_t bu = 0, bv = 0;
    if (r < a) {
    } else if (r < a + b) {
      bv = 1;
    } else if (r < a + b + c) {
      bu = 1;
    } else {
      bu = 1;
      bv = 1;
    }
    u = (u << 1) | bu;
    v = (v << 1) | bv;
  }
}

void gen_rmat(int scale, int64_t edge_factor, double a, double b, double c, uint64_t seed, Csr& g) {
  const int64_t n = (int64_t)1 << scale;
  const int64_t E = edge_factor * n;
  std::vector<int32_t> src(E), dst(E);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < E; ++i) {
    int64_t u, v;
    rmat_pair(seed, 1, (uint64_t)i, scale, a, b, c, u, v);
    src[i] = (int32_t)u;
    dst[i] = (int32_t)v;
  }
  build_csr(n, src, dst, g);
}

// R-MAT restricted to n vertices: draws at scale ceil(log2 n); a draw with an endpoint >= n is
// redrawn (up to 64 attempts, then dropped).
void gen_rmat_n(int64_t n, int64_t draws, double a, double b, double c, uint64_t seed, Csr& g) {
  int scale = 0;
  while (((int64_t)1 << scale) < n) ++scale;
  std::vector<int32_t> src(draws), dst(draws);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < draws; ++i) {
    int64_t u = -1, v = -1;
    for (int t = 0; t < 64; ++t) {
      rmat_pair(seed, 2 + (uint64_t)t, (uint64_t)i, scale, a, b, c, u, v);
      if (u < n && v < n) break;
      u = v = -1;
    }
    src[i] = (int32_t)u;
    dst[i] = (int32_t)v;
  }
  build_csr(n, src, dst, g);
}

// s x s grid, id = i*s + j. Each of the 2*s*(s-1) lattice edges is deleted with probability
// p_del; each of the (s-1)^2 unit squares receives one diagonal with probability p_diag, whose
// orientation is a fair coin. Built row by row in sorted order, no sort needed.
void gen_grid_road(int64_t s, double p_del, double p_diag, uint64_t seed, Csr& g) {
  const int64_t n = s * s;
  auto hkeep = [&](int64_t i, int64_t j) {  // edge (i,j)-(i,j+1)
    return u01(rnd(seed, 11, (uint64_t)(i * s + j))) >= p_del;
  };
  auto vkeep = [&](int64_t i, int64_t j) {  // edge (i,j)-(i+1,j)
    return u01(rnd(seed, 12, (uint64_t)(i * s + j))) >= p_del;
  };
  // square (i,j) spans rows i,i+1 and columns j,j+1. 0 = none, 1 = main (i,j)-(i+1,j+1),
  // 2 = anti (i,j+1)-(i+1,j).
  auto diag = [&](int64_t i, int64_t j) -> int {
    uint64_t r = rnd(seed, 13, (uint64_t)(i * s + j));
    if (u01(r) >= p_diag) return 0;
    return (rnd(seed, 14, (uint64_t)(i * s + j)) & 1) ? 1 : 2;
  };
  auto neigh = [&](int64_t i, int64_t j, int32_t* out) -> int {
    int c = 0;
    auto id = [&](int64_t a, int64_t b) { return (int32_t)(a * s + b); };
    // in increasing id order: (i-1,j-1) (i-1,j) (i-1,j+1) (i,j-1) (i,j+1) (i+1,j-1) (i+1,j) (i+1,j+1)
    if (i > 0 && j > 0 && diag(i - 1, j - 1) == 1) { if (out) out[c] = id(i - 1, j - 1); ++c; }
    if (i > 0 && vkeep(i - 1, j)) { if (out) out[c] = id(i - 1, j); ++c; }
    if (i > 0 && j + 1 < s && diag(i - 1, j) == 2) { if (out) out[c] = id(i - 1, j + 1); ++c; }
    if (j > 0 && hkeep(i, j - 1)) { if (out) out[c] = id(i, j - 1); ++c; }
    if (j + 1 < s && hkeep(i, j)) { if (out) out[c] = id(i, j + 1); ++c; }
    if (i + 1 < s && j > 0 && diag(i, j - 1) == 2) { if (out) out[c] = id(i + 1, j - 1); ++c; }
    if (i + 1 < s && vkeep(i, j)) { if (out) out[c] = id(i + 1, j); ++c; }
    if (i + 1 < s && j + 1 < s && diag(i, j) == 1) { if (out) out[c] = id(i + 1, j + 1); ++c; }
    return c;
  };
  g.n = n;
  g.off.assign(n + 1, 0);
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) g.off[v + 1] = neigh(v / s, v % s, nullptr);
  for (int64_t v = 0; v < n; ++v) g.off[v + 1] += g.off[v];
  g.adj.resize((size_t)g.off[n]);
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) neigh(v / s, v % s, g.adj.data() + g.off[v]);
}

// Walker/Vose alias table over non-negative weights.
struct Alias {
  std::vector<double> prob;
  std::vector<int32_t> alias;
  void build(const std::vector<double>& w) {
    const int64_t n = (int64_t)w.size();
    double sum = 0;
    for (double x : w) sum += x;
    prob.assign(n, 0.0);
    alias.assign(n, 0);
    std::vector<double> p(n);
    std::vector<int32_t> small, large;
    small.reserve(n);
    large.reserve(n);
    for (int64_t i = 0; i < n; ++i) {
      p[i] = w[i] * (double)n / sum;
      (p[i] < 1.0 ? small : large).push_back((int32_t)i);
    }
    while (!small.empty() && !large.empty()) {
      int32_t s = small.back(), l = large.back();
      small.pop_back();
      prob[s] = p[s];
      alias[s] = l;
      p[l] = (p[l] + p[s]) - 1.0;
      if (p[l] < 1.0) {
        large.pop_back();
        small.push_back(l);
      }
    }
    for (int32_t l : large) prob[l] = 1.0;
    for (int32_t s : small) prob[s] = 1.0;
  }
  int32_t draw(uint64_t r1, uint64_t r2) const {
    int64_t i = (int64_t)(u01(r1) * (double)prob.size());
    if (i >= (int64_t)prob.size()) i = (int64_t)prob.size() - 1;
    return u01(r2) < prob[i] ? (int32_t)i : alias[i];
  }
};

// Chung-Lu: expected degree of vertex i proportional to (i+1)^(-1/(gamma-1)), scaled so the
// expected degrees sum to 2*pairs, each capped at max_deg (scale found by bisection). `pairs`
// endpoint pairs are drawn independently proportional to those weights. A dense block of block_n
// distinct vertices (uniform over [0,n)) is planted with every block pair present with
// probability block_p.
// Block pair index t -> (a, b), a < b, row-major over the strict upper triangle of block positions.
inline void block_pair(int64_t t, int64_t block_n, int64_t& a, int64_t& b) {
  const double B = (double)block_n;
  a = (int64_t)std::floor((2 * B - 1 - std::sqrt((2 * B - 1) * (2 * B - 1) - 8.0 * (double)t)) / 2);
  if (a < 0) a = 0;
  auto row_start = [&](int64_t r) { return r * (2 * block_n - r - 1) / 2; };
  while (a > 0 && row_start(a) > t) --a;
  while (row_start(a + 1) <= t) ++a;
  b = a + 1 + (t - row_start(a));
}

// Chung-Lu: expected degree of vertex i proportional to (i+1)^(-1/(gamma-1)), scaled so the
// expected degrees sum to 2*pairs, each capped at max_deg (scale found by bisection). `pairs`
// endpoint pairs are drawn independently proportional to those weights (alias method). A dense
// block of block_n distinct vertices (uniform over [0,n)) is planted with every block pair present
// with probability block_p.
void chung_lu_setup(int64_t n, double gamma, int64_t pairs, int64_t max_deg, int64_t block_n,
                    double block_p, uint64_t seed, Alias& al, std::vector<int32_t>& blk,
                    std::vector<int64_t>& bsel) {
  Timer t_setup("chung-lu setup");
  std::vector<double> w(n);
  const double ex = -1.0 / (gamma - 1.0);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) w[i] = std::pow((double)(i + 1), ex);
  const double target = 2.0 * (double)pairs;
  double lo = 0, hi = 1;
  auto total = [&](double c) {
    double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t i = 0; i < n; ++i) s += std::min(c * w[i], (double)max_deg);
    return s;
  };
  while (total(hi) < target) hi *= 2;
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    (total(mid) < target ? lo : hi) = mid;
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) w[i] = std::min(hi * w[i], (double)max_deg);
  {
    Timer t_("alias");
    al.build(w);
  }
  // block members: the first block_n distinct values of a uniform draw sequence
  blk.clear();
  {
    std::vector<char> used(block_n > 0 ? n : 0, 0);
    for (uint64_t t = 0; (int64_t)blk.size() < block_n; ++t) {
      int32_t x = (int32_t)(rnd(seed, 21, t) % (uint64_t)n);
      if (used[x]) continue;
      used[x] = 1;
      blk.push_back(x);
    }
  }
  const int64_t bpairs = block_n * (block_n - 1) / 2;
  bsel.clear();
  if (bpairs > 0) {
    const uint64_t key = stream_key(seed, 22);
    std::vector<std::vector<int64_t>> part(omp_get_max_threads());
#pragma omp parallel
    {
      auto& mine = part[omp_get_thread_num()];
#pragma omp for schedule(static)
      for (int64_t t = 0; t < bpairs; ++t)
        if (u01(splitmix64(key + (uint64_t)t)) < block_p) mine.push_back(t);
    }
    for (auto& p : part) bsel.insert(bsel.end(), p.begin(), p.end());
  }
}

void gen_chung_lu(int64_t n, double gamma, int64_t pairs, int64_t max_deg, int64_t block_n,
                  double block_p, uint64_t seed, Csr& g) {
  Timer t_all("chung-lu total");
  Alias al;
  std::vector<int32_t> blk;
  std::vector<int64_t> bsel;
  chung_lu_setup(n, gamma, pairs, max_deg, block_n, block_p, seed, al, blk, bsel);
  const int64_t E = pairs + (int64_t)bsel.size();
  std::vector<int32_t> src(E), dst(E);
  {
    Timer t_samp("sample");
    const uint64_t k23 = stream_key(seed, 23), k24 = stream_key(seed, 24);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < pairs; ++i) {
      const uint64_t j = 2 * (uint64_t)i;
      src[i] = al.draw(splitmix64(k23 + j), splitmix64(k24 + j));
      dst[i] = al.draw(splitmix64(k23 + j + 1), splitmix64(k24 + j + 1));
    }
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < (int64_t)bsel.size(); ++q) {
      int64_t a, b;
      block_pair(bsel[q], block_n, a, b);
      src[pairs + q] = blk[a];
      dst[pairs + q] = blk[b];
    }
  }
  build_csr(n, src, dst, g);
}

// G(n, p) by geometric skipping over the n(n-1)/2 pair indices (stream `stream`).
void gen_er(int64_t n, double p, uint64_t seed, uint64_t stream, Csr& g) {
  std::vector<int32_t> src, dst;
  const int64_t total = n * (n - 1) / 2;
  if (p > 0 && n > 1) {
    const double lq = std::log1p(-std::min(p, 1.0 - 1e-12));
    int64_t t = -1;
    uint64_t k = 0;
    for (;;) {
      double r = u01(rnd(seed, stream, k++));
      int64_t skip = (p >= 1.0) ? 0 : (int64_t)std::floor(std::log1p(-r) / lq);
      t += 1 + skip;
      if (t >= total) break;
      double N = (double)n;
      int64_t a = (int64_t)std::floor((2 * N - 1 - std::sqrt((2 * N - 1) * (2 * N - 1) - 8.0 * (double)t)) / 2);
      if (a < 0) a = 0;
      auto row_start = [&](int64_t r) { return r * (2 * n - r - 1) / 2; };
      while (a > 0 && row_start(a) > t) --a;
      while (row_start(a + 1) <= t) ++a;
      int64_t b = a + 1 + (t - row_start(a));
      src.push_back((int32_t)a);
      dst.push_back((int32_t)b);
    }
  }
  build_csr(n, src, dst, g);
}

}  // namespace

extern "C" {

struct gg_graph {
  Csr g;
  std::vector<int64_t> vptr;  // segmented batches only
};

static gg_graph* wrap(Csr&& g) {
  gg_graph* h = new (std::nothrow) gg_graph;
  if (!h) return nullptr;
  h->g = std::move(g);
  return h;
}

gg_graph* gg_rmat(int scale, int64_t edge_factor, double a, double b, double c, uint64_t seed) {
  if (scale < 1 || scale > 30 || edge_factor < 0) return nullptr;
  Csr g;
  gen_rmat(scale, edge_factor, a, b, c, seed, g);
  return wrap(std::move(g));
}

gg_graph* gg_rmat_n(int64_t n, int64_t draws, double a, double b, double c, uint64_t seed) {
  if (n < 1 || draws < 0) return nullptr;
  Csr g;
  gen_rmat_n(n, draws, a, b, c, seed, g);
  return wrap(std::move(g));
}

gg_graph* gg_grid_road(int64_t s, double p_del, double p_diag, uint64_t seed) {
  if (s < 1 || s > 46340) return nullptr;
  Csr g;
  gen_grid_road(s, p_del, p_diag, seed, g);
  return wrap(std::move(g));
}

gg_graph* gg_chung_lu(int64_t n, double gamma, int64_t pairs, int64_t max_deg, int64_t block_n,
                      double block_p, uint64_t seed) {
  if (n < 2 || gamma <= 1.0 || pairs < 0 || block_n < 0 || block_n > n) return nullptr;
  Csr g;
  gen_chung_lu(n, gamma, pairs, max_deg, block_n, block_p, seed, g);
  return wrap(std::move(g));
}

gg_graph* gg_erdos_renyi(int64_t n, double p, uint64_t seed) {
  if (n < 0) return nullptr;
  Csr g;
  gen_er(n, p, seed, 31, g);
  return wrap(std::move(g));
}

// Undirected edge list -> symmetric CSR (loops dropped, duplicates merged).
gg_graph* gg_from_edges(int64_t n, int64_t ne, const int32_t* src, const int32_t* dst) {
  if (n < 0 || ne < 0) return nullptr;
  for (int64_t i = 0; i < ne; ++i)
    if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return nullptr;
  std::vector<int32_t> s(src, src + ne), d(dst, dst + ne);
  Csr g;
  build_csr(n, s, d, g);
  return wrap(std::move(g));
}

// Per-graph vertex count of the batched workload: round(exp(N(ln median, sigma))) redrawn until it
// lies in [lo, hi]; normal deviates by Box-Muller from the counter stream.
static int64_t batch_size(uint64_t seed, int64_t gidx, double median, double sigma, int64_t lo, int64_t hi) {
  for (uint64_t t = 0;; ++t) {
    double u1 = u01(rnd(seed, 41, (uint64_t)gidx * 1024 + 2 * t));
    double u2 = u01(rnd(seed, 41, (uint64_t)gidx * 1024 + 2 * t + 1));
    if (u1 <= 0) u1 = 1e-300;
    double z = std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    int64_t nv = (int64_t)std::llround(std::exp(std::log(median) + sigma * z));
    if (nv >= lo && nv <= hi) return nv;
    if (t > 1000) return std::min(std::max(nv, lo), hi);
  }
}

// Batch of `G` independent graphs packed in one segmented CSR with global ids. Graph g has
// n_g vertices (lognormal, see batch_size); even g is G(n_g, avg_deg/(n_g-1)), odd g is R-MAT
// with rmat_factor*n_g draws restricted to n_g vertices. Graph g uses sub-seed mix(seed, g), so
// graph g is identical whatever batch it is packed in (first_graph offsets the index).
gg_graph* gg_batch(int32_t G, int64_t first_graph, uint64_t seed, double median, double sigma, int64_t lo,
                   int64_t hi, double avg_deg, int64_t rmat_factor, double a, double b, double c) {
  if (G < 0 || lo < 1 || hi < lo) return nullptr;
  std::vector<Csr> parts(G);
  std::vector<int64_t> sizes(G);
  std::vector<int32_t> order(G);
  for (int32_t q = 0; q < G; ++q) {
    sizes[q] = batch_size(seed, first_graph + q, median, sigma, lo, hi);
    order[q] = q;
  }
  // largest first, one graph per thread (nested parallel regions inside run single-threaded)
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return sizes[x] > sizes[y]; });
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t oq = 0; oq < G; ++oq) {
    const int32_t q = order[oq];
    int64_t gi = first_graph + q;
    uint64_t sub = splitmix64(seed * 0x100000001B3ull + (uint64_t)gi);
    int64_t nv = sizes[q];
    if ((gi & 1) == 0)
      gen_er(nv, avg_deg / (double)(nv > 1 ? nv - 1 : 1), sub, 31, parts[q]);
    else
      gen_rmat_n(nv, rmat_factor * nv, a, b, c, sub, parts[q]);
  }
  gg_graph* h = new (std::nothrow) gg_graph;
  if (!h) return nullptr;
  h->vptr.assign(G + 1, 0);
  int64_t nnz = 0;
  for (int32_t q = 0; q < G; ++q) {
    h->vptr[q + 1] = h->vptr[q] + parts[q].n;
    nnz += (int64_t)parts[q].adj.size();
  }
  Csr& out = h->g;
  out.n = h->vptr[G];
  out.off.assign(out.n + 1, 0);
  out.adj.resize((size_t)nnz);
  int64_t e = 0;
  for (int32_t q = 0; q < G; ++q) {
    const Csr& p = parts[q];
    const int64_t base = h->vptr[q];
    for (int64_t v = 0; v < p.n; ++v) out.off[base + v] = e + p.off[v];
    for (size_t i = 0; i < p.adj.size(); ++i) out.adj[(size_t)e + i] = p.adj[i] + (int32_t)base;
    e += (int64_t)p.adj.size();
  }
  out.off[out.n] = e;
  return h;
}

// Chung-Lu sampling tables (exactly those gen_chung_lu uses) and the planted block's edge list,
// for drawing the same graph elsewhere: prob/alias are [n], block pairs are returned through a
// gg_graph handle whose adj holds (a, b) pairs flattened.
struct gg_cl_tables {
  std::vector<double> prob;
  std::vector<int32_t> alias;
  std::vector<int32_t> bpairs;
};

gg_cl_tables* gg_chung_lu_tables(int64_t n, double gamma, int64_t pairs, int64_t max_deg, int64_t block_n,
                                 double block_p, uint64_t seed) {
  if (n < 2 || gamma <= 1.0 || pairs < 0 || block_n < 0 || block_n > n) return nullptr;
  auto* t = new (std::nothrow) gg_cl_tables;
  if (!t) return nullptr;
  Alias al;
  std::vector<int32_t> blk;
  std::vector<int64_t> bsel;
  chung_lu_setup(n, gamma, pairs, max_deg, block_n, block_p, seed, al, blk, bsel);
  t->prob = std::move(al.prob);
  t->alias = std::move(al.alias);
  t->bpairs.resize(2 * bsel.size());
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < (int64_t)bsel.size(); ++q) {
    int64_t a, b;
    block_pair(bsel[q], block_n, a, b);
    t->bpairs[2 * q] = blk[a];
    t->bpairs[2 * q + 1] = blk[b];
  }
  return t;
}
int64_t gg_cl_block_pairs(const gg_cl_tables* t) { return t ? (int64_t)t->bpairs.size() / 2 : -1; }
void gg_cl_fill(const gg_cl_tables* t, double* prob, int32_t* alias, int32_t* bpairs) {
  std::memcpy(prob, t->prob.data(), sizeof(double) * t->prob.size());
  std::memcpy(alias, t->alias.data(), sizeof(int32_t) * t->alias.size());
  if (!t->bpairs.empty()) std::memcpy(bpairs, t->bpairs.data(), sizeof(int32_t) * t->bpairs.size());
}
void gg_cl_free(gg_cl_tables* t) { delete t; }

int64_t gg_num_vertices(const gg_graph* h) { return h ? h->g.n : -1; }
int64_t gg_num_entries(const gg_graph* h) { return h ? (int64_t)h->g.adj.size() : -1; }
int64_t gg_num_graphs(const gg_graph* h) { return h && !h->vptr.empty() ? (int64_t)h->vptr.size() - 1 : 0; }

// Copies the CSR out; buffers sized [n+1], [nnz], and [G+1] (vptr may be null).
int gg_fill(const gg_graph* h, int64_t* offsets, int32_t* adj, int64_t* vptr) {
  if (!h) return -1;
  std::memcpy(offsets, h->g.off.data(), sizeof(int64_t) * (h->g.n + 1));
  if (!h->g.adj.empty()) std::memcpy(adj, h->g.adj.data(), sizeof(int32_t) * h->g.adj.size());
  if (vptr && !h->vptr.empty()) std::memcpy(vptr, h->vptr.data(), sizeof(int64_t) * h->vptr.size());
  return 0;
}

void gg_free(gg_graph* h) { delete h; }

// Counter-based uniform draws for host-side workload decisions (arrival times, pool picks).
void gg_uniform(uint64_t seed, uint64_t stream, uint64_t first, int64_t count, double* out) {
  for (int64_t i = 0; i < count; ++i) out[i] = u01(rnd(seed, stream, first + (uint64_t)i));
}

}  // extern "C"
