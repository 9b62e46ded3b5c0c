/*
 * CPU oracle for exact k-core decomposition (coreness of every vertex).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the library's product path may call, link or load this
 * file; only the test suite, the package smoke check and the benchmark's CPU-baseline leg use it.
 * It shares no code, headers, tables or helpers with the GPU library.
 *
 * Input convention (all functions): an undirected simple graph as CSR with both directions of
 * every edge stored: offsets[0..n] (int64, offsets[0] = 0, non-decreasing), adj[offsets[n]]
 * (int32 ids in [0, n)), no self-loops, no duplicate entries in a row.
 *
 * What is computed (paper, Sec. 1 and Sec. 2 "Notations"): the k-core G_k is the largest subgraph
 * whose vertices all have degree >= k; the coreness of v is the largest k with v in G_k. The result
 * is unique, so every function below must agree exactly.
 *
 *   oracle_bz        Batagelj-Zaversnik bucket peel, the sequential O(n+m) baseline the paper
 *                    compares against (Sec. 1, Sec. 6.1 "Baselines"). Primary oracle.
 *   oracle_brute     the definition itself: for each k, delete vertices with fewer than k live
 *                    neighbours until none is left to delete. Tiny graphs only.
 *   oracle_hindex    h-index iteration c <- H({c(u) : u in N(v)}) from c = degree, which
 *                    converges to coreness (Lu et al., Nat. Commun. 2016); a third, independent
 *                    computation, not from the paper.
 *   oracle_levelsync the paper's framework (Alg. 1) with its sequential peel, run round by round
 *                    and subround by subround, reporting the structural counts the paper defines:
 *                    subrounds rho (Sec. 3.2, span analysis), non-empty rounds, the total size of
 *                    all active sets (Thm. 3.1) and the subround in which each vertex is peeled.
 *
 * Every function returns 0 on success, -1 on bad arguments, -2 when out of memory.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int bad_args(int64_t n, const int64_t* offsets, const int32_t* adj, const int32_t* core) {
  return n < 0 || (n > 0 && (!offsets || !core)) || (n > 0 && offsets[n] > 0 && !adj);
}

/* ---------------------------------------------------------------------------------------------
 * Batagelj-Zaversnik. Vertices are kept in an array ordered by current degree, with bin[d] the
 * first position holding degree d. Taking vertices in that order, the vertex v at the front has the
 * minimum current degree; its degree is final (its coreness). Each neighbour u with a larger current
 * degree loses one: u is swapped with the first vertex of its bin, that bin's start advances by one,
 * so u now sits at the end of the next-lower bin, and its degree drops by one.
 * ------------------------------------------------------------------------------------------- */
int oracle_bz(int64_t n, const int64_t* offsets, const int32_t* adj, int32_t* core) {
  if (bad_args(n, offsets, adj, core)) return -1;
  if (n == 0) return 0;
  int64_t maxd = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t d = offsets[v + 1] - offsets[v];
    if (d < 0) return -1;
    if (d > maxd) maxd = d;
  }
  int32_t* deg = core; /* current degree, becomes the coreness */
  int64_t* bin = (int64_t*)calloc((size_t)maxd + 2, sizeof(int64_t));
  int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int32_t* vert = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!bin || !pos || !vert) {
    free(bin);
    free(pos);
    free(vert);
    return -2;
  }
  for (int64_t v = 0; v < n; ++v) {
    deg[v] = (int32_t)(offsets[v + 1] - offsets[v]);
    bin[deg[v]]++;
  }
  /* counts -> first position of each degree */
  int64_t at = 0;
  for (int64_t d = 0; d <= maxd; ++d) {
    int64_t c = bin[d];
    bin[d] = at;
    at += c;
  }
  for (int64_t v = 0; v < n; ++v) {
    pos[v] = bin[deg[v]];
    vert[pos[v]] = (int32_t)v;
    bin[deg[v]]++;
  }
  /* the placement advanced every start by its count; shift back */
  for (int64_t d = maxd; d > 0; --d) bin[d] = bin[d - 1];
  bin[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t v = vert[i];
    for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e) {
      const int32_t u = adj[e];
      if (deg[u] > deg[v]) {
        const int32_t du = deg[u];
        const int64_t pu = pos[u];
        const int64_t pw = bin[du];
        const int32_t w = vert[pw];
        if (u != w) {
          vert[pu] = w;
          pos[w] = pu;
          vert[pw] = u;
          pos[u] = pw;
        }
        bin[du]++;
        deg[u] = du - 1;
      }
    }
  }
  free(bin);
  free(pos);
  free(vert);
  return 0;
}

/* ---------------------------------------------------------------------------------------------
 * Definition-level brute force: for k = 0, 1, 2, ... compute G_k by repeatedly deleting every
 * vertex with fewer than k live neighbours until a full pass deletes nothing; every vertex still
 * alive gets coreness >= k. Stops at the first k whose core is empty. O(kmax * n * m).
 * ------------------------------------------------------------------------------------------- */
int oracle_brute(int64_t n, const int64_t* offsets, const int32_t* adj, int32_t* core) {
  if (bad_args(n, offsets, adj, core)) return -1;
  if (n == 0) return 0;
  char* alive = (char*)malloc((size_t)n);
  if (!alive) return -2;
  for (int64_t v = 0; v < n; ++v) core[v] = 0; /* every vertex is in G_0 */
  for (int64_t k = 1;; ++k) {
    for (int64_t v = 0; v < n; ++v) alive[v] = 1;
    int changed = 1;
    while (changed) {
      changed = 0;
      for (int64_t v = 0; v < n; ++v) {
        if (!alive[v]) continue;
        int64_t live = 0;
        for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e) live += alive[adj[e]];
        if (live < k) {
          alive[v] = 0;
          changed = 1;
        }
      }
    }
    int64_t left = 0;
    for (int64_t v = 0; v < n; ++v)
      if (alive[v]) {
        core[v] = (int32_t)k;
        ++left;
      }
    if (left == 0) break;
  }
  free(alive);
  return 0;
}

/* ---------------------------------------------------------------------------------------------
 * h-index iteration. H(x_1..x_d) = the largest h such that at least h of the x_i are >= h.
 * Starting from c = degree, all vertices are updated together from the previous values until
 * nothing changes; the fixed point reached this way is the coreness. *iters_out = sweeps made.
 * ------------------------------------------------------------------------------------------- */
int oracle_hindex(int64_t n, const int64_t* offsets, const int32_t* adj, int32_t* core,
                  int64_t* iters_out) {
  if (bad_args(n, offsets, adj, core)) return -1;
  if (iters_out) *iters_out = 0;
  if (n == 0) return 0;
  int64_t maxd = 0;
  for (int64_t v = 0; v < n; ++v)
    if (offsets[v + 1] - offsets[v] > maxd) maxd = offsets[v + 1] - offsets[v];
  int32_t* cur = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* nxt = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int64_t* cnt = (int64_t*)calloc((size_t)maxd + 2, sizeof(int64_t));
  if (!cur || !nxt || !cnt) {
    free(cur);
    free(nxt);
    free(cnt);
    return -2;
  }
  for (int64_t v = 0; v < n; ++v) cur[v] = (int32_t)(offsets[v + 1] - offsets[v]);
  int64_t sweeps = 0;
  for (;;) {
    int changed = 0;
    ++sweeps;
    for (int64_t v = 0; v < n; ++v) {
      const int64_t d = offsets[v + 1] - offsets[v];
      for (int64_t h = 0; h <= d; ++h) cnt[h] = 0;
      for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e) {
        int64_t x = cur[adj[e]];
        cnt[x < d ? x : d]++;
      }
      /* scan h from d down: at_least = #{x_i >= h} */
      int64_t at_least = 0, h = d;
      for (; h > 0; --h) {
        at_least += cnt[h];
        if (at_least >= h) break;
      }
      nxt[v] = (int32_t)h;
      if (nxt[v] != cur[v]) changed = 1;
    }
    int32_t* t = cur;
    cur = nxt;
    nxt = t;
    if (!changed) break;
  }
  memcpy(core, cur, sizeof(int32_t) * (size_t)n);
  if (iters_out) *iters_out = sweeps;
  free(cur);
  free(nxt);
  free(cnt);
  return 0;
}

/* ---------------------------------------------------------------------------------------------
 * The paper's framework (Alg. 1) with its sequential peel, executed literally:
 *   induced degree <- degree; active set A <- V; k <- 0
 *   while A is not empty:                                   (a round)
 *     F <- { v in A : induced degree of v = k }
 *     while F is not empty:                                 (a subround)
 *       coreness of every v in F <- k
 *       F' <- {}; for v in F, for u in N(v): decrement u; if it now equals k, append u to F'
 *       F <- F'
 *     A <- { v in A : induced degree of v > k };  k <- k + 1
 * Within a subround the set F' does not depend on the visiting order (a vertex joins F' when its
 * induced degree passes from k+1 to k, which happens at most once), so the subround structure is
 * deterministic. Reported counts:
 *   st[0] rounds executed (k = 0 .. kmax, empty ones included)
 *   st[1] non-empty rounds (= number of distinct coreness values)
 *   st[2] subrounds rho (number of non-empty frontiers)
 *   st[3] sum of all frontier sizes (= n: every vertex is peeled exactly once)
 *   st[4] sum over rounds of |A| (Thm. 3.1: = sum over v of (1 + coreness(v)))
 *   st[5] adjacency entries expanded (= m)
 *   st[6] largest number of subrounds in one round
 * sub_out (nullable): for every vertex the 1-based subround, within its round, that peeled it.
 * ------------------------------------------------------------------------------------------- */
int oracle_levelsync(int64_t n, const int64_t* offsets, const int32_t* adj, int32_t* core,
                     int32_t* sub_out, int64_t* st) {
  if (bad_args(n, offsets, adj, core) || !st) return -1;
  for (int i = 0; i < 7; ++i) st[i] = 0;
  if (n == 0) return 0;
  int64_t* dt = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int32_t* A = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* F = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* Fn = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!dt || !A || !F || !Fn) {
    free(dt);
    free(A);
    free(F);
    free(Fn);
    return -2;
  }
  int64_t na = n;
  for (int64_t v = 0; v < n; ++v) {
    dt[v] = offsets[v + 1] - offsets[v];
    A[v] = (int32_t)v;
    core[v] = -1;
  }
  for (int64_t k = 0; na > 0; ++k) {
    st[0]++;
    st[4] += na;
    int64_t nf = 0;
    for (int64_t i = 0; i < na; ++i)
      if (dt[A[i]] == k) F[nf++] = A[i];
    if (nf > 0) st[1]++;
    int64_t s = 0;
    while (nf > 0) {
      ++s;
      st[2]++;
      st[3] += nf;
      for (int64_t i = 0; i < nf; ++i) {
        core[F[i]] = (int32_t)k;
        if (sub_out) sub_out[F[i]] = (int32_t)s;
      }
      int64_t nn = 0;
      for (int64_t i = 0; i < nf; ++i) {
        const int32_t v = F[i];
        for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e) {
          const int32_t u = adj[e];
          st[5]++;
          dt[u] -= 1;
          if (dt[u] == k) Fn[nn++] = u;
        }
      }
      int32_t* t = F;
      F = Fn;
      Fn = t;
      nf = nn;
    }
    if (s > st[6]) st[6] = s;
    int64_t keep = 0;
    for (int64_t i = 0; i < na; ++i)
      if (dt[A[i]] > k) A[keep++] = A[i];
    na = keep;
  }
  free(dt);
  free(A);
  free(F);
  free(Fn);
  return 0;
}
