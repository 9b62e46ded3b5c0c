"""Pins for the CPU oracle (no GPU).

The oracle is trusted only because these tests tie it to things other than itself:
the k-core definition by brute force on every small graph, closed-form coreness of graph families,
the subround structure the paper's framework implies on grids and paths, the identities of the
work analysis (Thm. 3.1), the h-index fixed point and an O(m) exactness certificate.
"""
import itertools
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
import graphs as G

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def all_four(off, adj, lib=None):
    c_bz = oracle.bz(off, adj, lib)
    c_br = oracle.brute(off, adj, lib)
    c_hi, _ = oracle.hindex(off, adj, lib)
    c_ls, _, _ = oracle.levelsync(off, adj, lib)
    return c_bz, c_br, c_hi, c_ls


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_exhaustive_small_graphs_match_definition(n):
    parts = G.all_graphs(n)
    want = np.concatenate([G.brute_py(*p) for p in parts])
    off, adj = G.union(parts)
    for got in all_four(off, adj):
        np.testing.assert_array_equal(got, want)


def test_exhaustive_six_vertices():
    # all 32768 labelled graphs on 6 vertices, checked as one disjoint union against the C brute
    # force (itself pinned above) and per graph against pure-Python brute force on a sample
    parts = G.all_graphs(6)
    off, adj = G.union(parts)
    c_bz, c_br, c_hi, c_ls = all_four(off, adj)
    np.testing.assert_array_equal(c_bz, c_br)
    np.testing.assert_array_equal(c_hi, c_br)
    np.testing.assert_array_equal(c_ls, c_br)
    rng = np.random.default_rng(0)
    for gi in rng.choice(len(parts), 300, replace=False):
        np.testing.assert_array_equal(c_bz[6 * gi:6 * gi + 6], G.brute_py(*parts[gi]))


@pytest.mark.parametrize("seed", range(12))
def test_random_graphs_match_definition(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 65))
    p = float(rng.choice([0.03, 0.08, 0.2, 0.5, 0.9]))
    g = gg.erdos_renyi(n, p, seed)
    want = G.brute_py(g.offsets, g.adj)
    for got in all_four(g.offsets, g.adj):
        np.testing.assert_array_equal(got, want)


def closed_forms():
    rng = np.random.default_rng(7)
    yield "K1", G.csr(1, []), [0]
    for n in (2, 3, 7, 30):
        yield f"K{n}", G.complete(n), [n - 1] * n
    for n in (3, 4, 11, 100):
        yield f"C{n}", G.cycle(n), [2] * n
    for n in (2, 3, 10, 101):
        yield f"P{n}", G.path(n), [1] * n
    for leaves in (1, 5, 64):
        yield f"star{leaves}", G.star(leaves), [1] * (leaves + 1)
    for n in (2, 17, 200):
        yield f"tree{n}", G.random_tree(n, rng), [1] * n
    for s in (2, 3, 8, 31):
        yield f"grid{s}", G.grid(s), [2] * (s * s)
    for s in (2, 3, 6):
        yield f"cube{s}", G.cube(s), [3] * (s ** 3)
    for a, b in ((1, 1), (2, 5), (4, 4), (7, 3)):
        yield f"K{a},{b}", G.complete_bipartite(a, b), [min(a, b)] * (a + b)
    for d in (1, 2, 3, 6):
        yield f"Q{d}", G.hypercube(d), [d] * (1 << d)
    yield "petersen", G.petersen(), [3] * 10
    for K in (2, 5, 40):
        yield f"hcns{K}", G.hcns(K), G.hcns_expected(K).tolist()
    yield "isolated5", G.csr(5, []), [0] * 5


@pytest.mark.parametrize("name,graph,want", list(closed_forms()), ids=lambda x: x if isinstance(x, str) else "")
def test_closed_forms(name, graph, want):
    off, adj = graph
    for got in all_four(off, adj):
        np.testing.assert_array_equal(got, np.asarray(want, dtype=np.int32), err_msg=name)


def test_disjoint_union_concatenates():
    parts = [G.complete(5), G.cycle(7), G.grid(4), G.star(3), G.hcns(6)]
    off, adj = G.union(parts)
    want = np.concatenate([oracle.bz(*p) for p in parts])
    for got in all_four(off, adj):
        np.testing.assert_array_equal(got, want)


def test_golden_fixtures():
    gdir = os.path.join(HERE, "golden")
    files = sorted(f for f in os.listdir(gdir) if f.endswith(".json"))
    assert files
    for f in files:
        fx = json.load(open(os.path.join(gdir, f)))
        assert fx.get("citation"), f
        off, adj = G.csr(fx["n"], fx["edges"])
        want = np.asarray(fx["coreness"], dtype=np.int32)
        for got in all_four(off, adj):
            np.testing.assert_array_equal(got, want, err_msg=f)
        if "kmax" in fx:
            assert int(want.max()) == fx["kmax"]


def test_hcns_printed_size_matches_construction():
    # Table 2 prints n = 0.1M and m = 5.0B for the k_max = 50000 staircase graph (Sec. 6.1.1);
    # the staircase reading gives n = 2K and 2K^2 directed entries. Check the formula on small K
    # against the built graph, then evaluate it at K = 50000.
    for K in (2, 3, 9, 40):
        off, adj = G.hcns(K)
        assert len(off) - 1 == 2 * K and len(adj) == 2 * K * K
    K = 50_000
    assert 2 * K == 100_000 and 2 * K * K == 5_000_000_000


# ---- structural counts of the framework (Alg. 1) ------------------------------------------

@pytest.mark.parametrize("s", [2, 3, 4, 7, 10, 33, 64])
def test_levelsync_grid_peel_times(s):
    # On an s x s grid every vertex has coreness 2; round 2 starts at the four corners and a
    # vertex falls one subround after two of its neighbours do, so vertex (i,j) is peeled in
    # subround 1 + min(i, s-1-i) + min(j, s-1-j), and rho = s-1 (s even) or s (s odd).
    off, adj = G.grid(s)
    core, sub, st = oracle.levelsync(off, adj)
    i, j = np.divmod(np.arange(s * s), s)
    want = 1 + np.minimum(i, s - 1 - i) + np.minimum(j, s - 1 - j)
    np.testing.assert_array_equal(sub, want)
    assert st["subrounds"] == (s - 1 if s % 2 == 0 else s)
    assert st["nonempty_rounds"] == 1 and st["rounds"] == 3


@pytest.mark.parametrize("n", [2, 3, 8, 9, 50])
def test_levelsync_path_peel_times(n):
    off, adj = G.path(n)
    core, sub, st = oracle.levelsync(off, adj)
    idx = np.arange(n)
    np.testing.assert_array_equal(sub, 1 + np.minimum(idx, n - 1 - idx))
    assert st["subrounds"] == (n + 1) // 2


def test_levelsync_star_and_clique():
    off, adj = G.star(9)
    core, sub, st = oracle.levelsync(off, adj)
    assert sub[0] == 2 and np.all(sub[1:] == 1) and st["subrounds"] == 2
    off, adj = G.complete(12)
    core, sub, st = oracle.levelsync(off, adj)
    assert np.all(sub == 1) and st["subrounds"] == 1 and st["rounds"] == 12


@pytest.mark.parametrize("which", ["rmat", "er", "hcns", "grid_road"])
def test_levelsync_identities(which):
    if which == "rmat":
        g = gg.rmat(12, 16, 11)
        off, adj = g.offsets, g.adj
    elif which == "er":
        g = gg.erdos_renyi(3000, 0.004, 5)
        off, adj = g.offsets, g.adj
    elif which == "hcns":
        off, adj = G.hcns(60)
    else:
        g = gg.grid_road(96, 0.05, 0.01, 2)
        off, adj = g.offsets, g.adj
    n, m = len(off) - 1, len(adj)
    core, sub, st = oracle.levelsync(off, adj)
    c64 = core.astype(np.int64)
    assert st["frontier_total"] == n                    # every vertex in exactly one frontier
    assert st["edges_expanded"] == m                    # every adjacency entry expanded once
    assert st["active_total"] == int((1 + c64).sum())   # Thm. 3.1 identity
    assert st["rounds"] == int(core.max()) + 1
    assert st["nonempty_rounds"] == len(np.unique(core))
    assert not G.core_certificate(off, adj, core, sub)
    np.testing.assert_array_equal(oracle.bz(off, adj), core)
    np.testing.assert_array_equal(oracle.hindex(off, adj)[0], core)


def test_certificate_rejects_wrong_answers():
    off, adj = G.complete(4)
    assert G.core_certificate(off, adj, np.full(4, 3), np.ones(4))  == []
    # c = 0 everywhere is an h-index fixed point on K4 but not the coreness
    assert G.core_certificate(off, adj, np.zeros(4), np.ones(4))
    assert G.core_certificate(off, adj, np.full(4, 4), np.ones(4))


def test_hindex_fixed_point_on_bz_output():
    g = gg.rmat(13, 8, 3)
    core = oracle.bz(g.offsets, g.adj)
    n = g.n
    for v in range(0, n, 97):
        nb = core[g.adj[g.offsets[v]:g.offsets[v + 1]]]
        h = max([h for h in range(len(nb) + 1) if (nb >= h).sum() >= h])
        assert h == core[v]


def test_empty_and_bad_inputs():
    z = np.zeros(1, np.int64)
    assert oracle.bz(z, np.zeros(0, np.int32)).shape == (0,)
    assert oracle.levelsync(z, np.zeros(0, np.int32))[2]["rounds"] == 0
    with pytest.raises(RuntimeError):
        oracle.bz(np.array([0, -1], np.int64), np.zeros(0, np.int32))


# ---- the pins have teeth: plant plausible mistakes in a copy of the oracle -------------------

MUTANTS = {
    "bz_strict_vs_nonstrict": ("if (deg[u] > deg[v]) {", "if (deg[u] >= deg[v]) {"),
    "bz_bin_not_advanced": ("        bin[du]++;\n        deg[u] = du - 1;", "        deg[u] = du - 1;"),
    "bz_no_bin_shift": ("for (int64_t d = maxd; d > 0; --d) bin[d] = bin[d - 1];", ""),
    "brute_off_by_one": ("if (live < k) {", "if (live <= k) {"),
    "hindex_cap_wrong": ("cnt[x < d ? x : d]++;", "cnt[x < d ? x : d - 1]++;"),
    "levelsync_le_instead_of_eq": ("if (dt[u] == k) Fn[nn++] = u;", "if (dt[u] <= k && dt[u] >= k - 1) Fn[nn++] = u;"),
    "levelsync_refine_ge": ("if (dt[A[i]] > k) A[keep++] = A[i];", "if (dt[A[i]] >= k) A[keep++] = A[i];"),
}


def pins_pass(lib) -> bool:
    """A condensed pin suite run against an arbitrary compiled oracle."""
    try:
        for n in (3, 4, 5):
            parts = G.all_graphs(n)
            want = np.concatenate([oracle.brute(*p) for p in parts])  # trusted, pinned build
            off, adj = G.union(parts)
            for got in all_four(off, adj, lib):
                if not np.array_equal(got, want):
                    return False
        for name, (off, adj), want in closed_forms():
            for got in all_four(off, adj, lib):
                if not np.array_equal(got, np.asarray(want, dtype=np.int32)):
                    return False
        for s in (4, 7):
            off, adj = G.grid(s)
            _, sub, st = oracle.levelsync(off, adj, lib)
            if st["subrounds"] != (s - 1 if s % 2 == 0 else s):
                return False
        g = gg.rmat(11, 8, 2)
        core, sub, st = oracle.levelsync(g.offsets, g.adj, lib)
        if st["active_total"] != int((1 + core.astype(np.int64)).sum()):
            return False
    except Exception:
        return False
    return True


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_pins_catch_planted_mistake(mutant, tmp_path):
    # the mutant runs in a child process: a planted mistake may also crash it, which counts as
    # caught
    import subprocess
    import sys
    src = open(oracle._SRC).read()
    old, new = MUTANTS[mutant]
    assert src.count(old) == 1, mutant
    bad = tmp_path / "oracle_mut.c"
    bad.write_text(src.replace(old, new))
    so = oracle.build(force=True, src=str(bad), out=str(tmp_path / "liboracle_mut.so"))
    code = ("import sys; sys.path[:0] = [%r, %r]; import oracle, test_oracle; "
            "sys.exit(0 if test_oracle.pins_pass(oracle.load(%r)) else 3)" % (ROOT, HERE, so))
    rc = subprocess.run([sys.executable, "-c", code], capture_output=True).returncode
    assert rc != 0, f"pins did not catch {mutant}"


def test_unmutated_oracle_passes_condensed_pins():
    assert pins_pass(oracle.load())
