"""GPU parity: the HIP library against the CPU oracle, element by element (coreness is exact).

Every case prints its name before touching the GPU so that a failing run names it.
"""
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
import graphs as G
from gpu_util import say, run_single, run_batched, first_mismatch

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
MODES = ["levelsync", "chained"]


def small_cases():
    yield "K1", G.csr(1, [])
    yield "isolated7", G.csr(7, [])
    yield "K2", G.complete(2)
    yield "K30", G.complete(30)
    yield "C100", G.cycle(100)
    yield "P101", G.path(101)
    yield "star64", G.star(64)
    yield "grid31", G.grid(31)
    yield "cube6", G.cube(6)
    yield "K7,3", G.complete_bipartite(7, 3)
    yield "Q6", G.hypercube(6)
    yield "petersen", G.petersen()
    yield "hcns40", G.hcns(40)
    yield "union", G.union([G.complete(5), G.cycle(7), G.grid(4), G.star(3), G.hcns(6), G.csr(3, [])])
    for f in sorted(os.listdir(os.path.join(HERE, "golden"))):
        if f.endswith(".json"):
            fx = json.load(open(os.path.join(HERE, "golden", f)))
            yield f, G.csr(fx["n"], fx["edges"])


@pytest.mark.parametrize("tail", [0, -1])
@pytest.mark.parametrize("mode", MODES)
def test_small_graphs(mode, tail):
    for name, (off, adj) in small_cases():
        say(f"[gpu] small {name} mode={mode} tail={tail} n={len(off) - 1} m={len(adj)}")
        got, st = run_single(off, adj, mode=mode, tail=tail)
        want = oracle.bz(off, adj)
        assert not first_mismatch(got, want), f"{name}: {first_mismatch(got, want)}"
        assert st["peeled"] == len(off) - 1, (name, st)
        assert st["edges"] == len(adj), (name, st)
        assert st["device_status"] == 0


@pytest.mark.parametrize("tail", [0, -1])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("which", ["rmat12", "er3000", "road128", "hcns200", "rmat16", "road1024"])
def test_medium_graphs(mode, which, tail):
    if which == "rmat12":
        g = gg.rmat(12, 16, 11)
        off, adj = g.offsets, g.adj
    elif which == "er3000":
        g = gg.erdos_renyi(3000, 0.004, 5)
        off, adj = g.offsets, g.adj
    elif which == "road128":
        g = gg.grid_road(128, 0.05, 0.01, 2)
        off, adj = g.offsets, g.adj
    elif which == "hcns200":
        off, adj = G.hcns(200)
    elif which == "road1024":
        # deep peel chains: in chained mode scans and chains race for the same vertices, and
        # every vertex must still be peeled exactly once (peeled == n, edges == m)
        g = gg.grid_road(1024, 0.05, 0.01, 2)
        off, adj = g.offsets, g.adj
    else:
        g = gg.config_rmat16()
        off, adj = g.offsets, g.adj
    say(f"[gpu] medium {which} mode={mode} tail={tail} n={len(off) - 1} m={len(adj)}")
    got, st = run_single(off, adj, mode=mode, tail=tail)
    want, sub, ls = oracle.levelsync(off, adj)
    assert not first_mismatch(got, want), first_mismatch(got, want)
    assert st["peeled"] == len(off) - 1 and st["edges"] == len(adj)
    assert st["rounds"] == ls["nonempty_rounds"], (st, ls)
    assert st["kmax"] == int(want.max())
    # each vertex takes deg - coreness decrements while above k: m - sum of the oracle's coreness
    assert st["live_decrements"] == len(adj) - int(want.astype(np.int64).sum()), st
    if mode == "levelsync":
        # Alg. 1 + Alg. 3 frontiers are order independent: the subround count must equal the
        # sequential framework's rho
        assert st["subrounds"] == ls["subrounds"], (st, ls)
    else:
        assert st["subrounds"] <= ls["subrounds"]


@pytest.mark.parametrize("mode", MODES)
def test_tuning_knobs_do_not_change_results(mode):
    g = gg.rmat(13, 16, 7)
    want = oracle.bz(g.offsets, g.adj)
    for hub, tile, budget, bpc in ((8, 64, 1, 1), (64, 128, 64, 1), (1 << 30, 1024, 100000, 0)):
        say(f"[gpu] knobs mode={mode} hub={hub} tile={tile} budget={budget}")
        got, st = run_single(g.offsets, g.adj, mode=mode, hub_degree=hub, tile_edges=tile,
                             local_budget=budget, blocks_per_cu=bpc)
        assert not first_mismatch(got, want), first_mismatch(got, want)


def test_cached_tuned_options_are_exact():
    """Every option set the shipped tuning cache holds for a single-graph class, applied to graphs
    of other shapes (they are plain launch and threshold choices), gives the oracle's coreness."""
    import paper_2502_08042_amd.autotune as A
    cases = [("rmat13", gg.rmat(13, 16, 7)), ("road256", gg.grid_road(256, 0.05, 0.01, 3))]
    off, adj = G.hcns(300)
    sets = [(dev, cls, o["options"]) for dev, classes in A.load_cache().items()
            for cls, o in classes.items() if cls.startswith("single/")]
    assert sets
    for dev, cls, opts in sets:
        for name, o_np, a_np in [(nm, g.offsets, g.adj) for nm, g in cases] + [("hcns300", off, adj)]:
            want = oracle.bz(o_np, a_np)
            tuning = A._resolve({k: v for k, v in opts.items() if v != 0}, len(o_np) - 1)
            say(f"[gpu] tuned {dev} {cls} on {name}: {tuning}")
            got, st = run_single(o_np, a_np, mode="chained", **tuning)
            assert not first_mismatch(got, want), (cls, name, first_mismatch(got, want))
            assert st["device_status"] == 0


def test_chained_work_queues_do_not_change_results():
    """Chained mode's in-phase work sharing: the workgroup tile queue (off, one tile, a few tiles,
    more tiles than the queue holds, which spills to the global list) and the asynchronous phases
    (never, default, scan folded in) must all give the oracle's coreness, every vertex peeled once."""
    cases = [("rmat13", gg.rmat(13, 16, 7)), ("road256", gg.grid_road(256, 0.05, 0.01, 3))]
    for name, g in cases:
        want = oracle.bz(g.offsets, g.adj)
        for bt, bq, af, asc, tp in ((-1, 0, -1, -1, 0), (1, 0, -1, -1, 0), (4, 0, 0, 0, -1),
                                    (2000, 0, -1, -1, 0), (4, 8, -1, -1, -1), (0, 0, 0, 1 << 30, 0),
                                    (0, 0, 0, 0, 0), (0, 0, 0, 0, -1)):
            say(f"[gpu] queues {name} block_tiles={bt} block_queue={bq} async_frontier={af} "
                f"async_scan={asc} tile_probe={tp}")
            got, st = run_single(g.offsets, g.adj, mode="chained", hub_degree=16, tile_edges=64,
                                 block_tiles=bt, block_queue=bq, async_frontier=af, async_scan=asc,
                                 tile_probe=tp)
            assert not first_mismatch(got, want), first_mismatch(got, want)
            assert st["peeled"] == g.n and st["edges"] == g.m and st["device_status"] == 0


@pytest.mark.parametrize("mode", MODES)
def test_residual_rows_do_not_change_results(mode):
    """Rows rewritten without peeled neighbours (at the first round boundary the threshold allows,
    from a small and from a large threshold) must give the oracle's coreness, and so must runs
    that never rewrite them."""
    cases = [("rmat13", gg.rmat(13, 16, 7)), ("road256", gg.grid_road(256, 0.05, 0.01, 3)),
             ("hcns120", None)]
    for name, g in cases:
        off, adj = (g.offsets, g.adj) if g is not None else G.hcns(120)
        want = oracle.bz(off, adj)
        for resid in (-1, 1, 64, 1 << 30):
            for hub in (0, 16):
                say(f"[gpu] residual {name} mode={mode} residual={resid} hub={hub}")
                got, st = run_single(off, adj, mode=mode, residual=resid, hub_degree=hub,
                                     tile_edges=64 if hub else 0)
                assert not first_mismatch(got, want), first_mismatch(got, want)
                assert st["peeled"] == len(off) - 1 and st["device_status"] == 0


def _tail_cases():
    # rmat16x4: 23,472 vertices are live at the boundary of round 2, so the largest handoff fills
    # nearly the whole tail capacity (16-bit local ids and queue slots up to 23,471)
    return [("rmat13", gg.rmat(13, 16, 7)), ("road256", gg.grid_road(256, 0.05, 0.01, 3)),
            ("hcns120", None), ("er5000", gg.erdos_renyi(5000, 0.01, 8)), ("rmat16x4", gg.rmat(16, 4, 9))]


@pytest.mark.parametrize("mode", MODES)
def test_tail_handoff_sizes(mode):
    """The last live vertices (the k-core of the round boundary where at most `tail` remain) are
    peeled by one workgroup: from a handoff of a single vertex up to the whole graph after its first
    round, with and without rewritten rows before, the coreness must be the oracle's, every vertex
    and entry counted once, the round count that of the sequential framework, and in level-sync
    mode the subround count its rho."""
    for name, g in _tail_cases():
        off, adj = (g.offsets, g.adj) if g is not None else G.hcns(120)
        want, sub, ls = oracle.levelsync(off, adj)
        for tail in (1, 2, 64, 1000, 1 << 30):
            for resid in (-1, 0, 1 << 30):
                say(f"[gpu] tail {name} mode={mode} tail={tail} residual={resid}")
                got, st = run_single(off, adj, mode=mode, tail=tail, residual=resid)
                assert not first_mismatch(got, want), first_mismatch(got, want)
                assert st["peeled"] == len(off) - 1 and st["edges"] == len(adj), st
                assert st["device_status"] == 0 and st["kmax"] == int(want.max())
                assert st["rounds"] == ls["nonempty_rounds"], (st, ls)
                if mode == "levelsync":
                    assert st["subrounds"] == ls["subrounds"], (st, ls)
                if name == "rmat16x4" and tail == 1 << 30:
                    assert st["tail_vertices"] > 17408, st


def test_tail_handoff_called_off():
    """A handoff whose local rows do not fit is called off and retried when half as many
    vertices are live (or never happens): the grid keeps peeling and the result is unchanged."""
    for name, g in _tail_cases():
        off, adj = (g.offsets, g.adj) if g is not None else G.hcns(120)
        want = oracle.bz(off, adj)
        for ecap in (1, 50, 2000):
            say(f"[gpu] tail called off {name} ecap={ecap}")
            got, st = run_single(off, adj, mode="chained", test_tail_entries=ecap)
            assert not first_mismatch(got, want), first_mismatch(got, want)
            assert st["peeled"] == len(off) - 1 and st["edges"] == len(adj), st
            assert st["device_status"] == 0


@pytest.mark.parametrize("tail", [0, -1])
def test_offline_mode_keeps_levelsync_frontiers(tail):
    """Offline mode (Alg. 2): each subround's decrements are counted per target in a workgroup
    table and applied once with the batch rule old > k >= old - c. Coreness must be the oracle's
    and, the frontiers being order independent, the subround count the sequential framework's
    rho."""
    cases = [("rmat12", gg.rmat(12, 16, 11)), ("er3000", gg.erdos_renyi(3000, 0.004, 5)),
             ("road128", gg.grid_road(128, 0.05, 0.01, 2)), ("hcns200", None),
             ("rmat16", gg.config_rmat16())]
    for name, g in cases:
        off, adj = (g.offsets, g.adj) if g is not None else G.hcns(200)
        say(f"[gpu] offline {name} tail={tail}")
        want, sub, ls = oracle.levelsync(off, adj)
        got, st = run_single(off, adj, mode="offline", tail=tail)
        assert not first_mismatch(got, want), first_mismatch(got, want)
        assert st["peeled"] == len(off) - 1 and st["edges"] == len(adj), st
        assert st["rounds"] == ls["nonempty_rounds"] and st["subrounds"] == ls["subrounds"], (st, ls)
        assert st["device_status"] == 0, st
        if tail == -1:  # (with the tail, small graphs go to the single workgroup after round one)
            assert st["combined"] > 0, st


def _sample_knobs(knobs):
    if knobs is None:
        return {}
    th, mu = knobs
    return {"sample_threshold": th, "sample_mu": mu}


@pytest.mark.parametrize("mode,knobs", [("offline", None), ("sampling", None), ("sampling", (2, 4))])
def test_small_graphs_other_modes(mode, knobs):
    """Exact graph families and golden fixtures in offline and sampling mode (with nearly every
    vertex in sample mode for threshold 2)."""
    for name, (off, adj) in small_cases():
        say(f"[gpu] small {name} mode={mode} knobs={knobs}")
        got, st = run_single(off, adj, mode=mode, **_sample_knobs(knobs))
        want = oracle.bz(off, adj)
        assert not first_mismatch(got, want), f"{name}: {first_mismatch(got, want)}"
        assert st["peeled"] == len(off) - 1 and st["device_status"] == 0, (name, st)


def test_sampling_mode_is_exact():
    """Sampling mode (Alg. 4/5): hubs count hits instead of decrementing and are validated and
    recounted at round boundaries; the coreness must still be the oracle's, every vertex peeled
    and every entry expanded once. Low thresholds put many vertices in sample mode."""
    cases = [("rmat13", gg.rmat(13, 16, 7)), ("rmat16", gg.config_rmat16()),
             ("road256", gg.grid_road(256, 0.05, 0.01, 3)), ("hcns120", None),
             ("er5000", gg.erdos_renyi(5000, 0.01, 8))]
    for name, g in cases:
        off, adj = (g.offsets, g.adj) if g is not None else G.hcns(120)
        want = oracle.bz(off, adj)
        for knobs in (None, (128, 100), (16, 32), (8, 400)):
            say(f"[gpu] sampling {name} threshold,mu={knobs}")
            got, st = run_single(off, adj, mode="sampling", **_sample_knobs(knobs))
            assert not first_mismatch(got, want), first_mismatch(got, want)
            assert st["peeled"] == len(off) - 1 and st["edges"] == len(adj), st
            assert st["device_status"] == 0 and st["kmax"] == int(want.max())
            thr = 1024 if knobs is None else knobs[0]
            assert st["sampled_vertices"] == int((np.diff(off) > thr).sum()), st


def test_sampling_failure_is_detected_and_repeated():
    """A star's centre in sample mode with one expected hit (mu = 1) loses every neighbour in
    round 1 unseen: the recount at a later round boundary finds it below k, the run is void and
    is repeated without sampling, and the result is still exact."""
    off, adj = G.star(64)
    want = oracle.bz(off, adj)
    say("[gpu] sampling failure on star64")
    got, st = run_single(off, adj, mode="sampling", sample_threshold=4, sample_mu=1)
    assert not first_mismatch(got, want), first_mismatch(got, want)
    assert st["sample_restarts"] == 1 and st["sampled_vertices"] == 1, st
    assert st["device_status"] == 0 and st["peeled"] == len(off) - 1


@pytest.mark.parametrize("mode", MODES)
def test_kcore_subgraph_query(mode):
    """Maximum k-core subgraph (App. B): membership equals coreness >= k from the oracle, for k
    below, at and above the largest coreness, on graphs with hubs, chains and a dense core."""
    import paper_2502_08042_amd as K
    import torch
    from gpu_util import to_dev
    cases = [("rmat13", gg.rmat(13, 16, 7)), ("road256", gg.grid_road(256, 0.05, 0.01, 3)),
             ("hcns60", None)]
    for name, g in cases:
        off, adj = (g.offsets, g.adj) if g is not None else G.hcns(60)
        core = oracle.bz(off, adj)
        d_off, d_adj = to_dev(off, adj)
        kmax = int(core.max())
        for k in sorted({0, 1, 2, 3, max(kmax // 2, 1), kmax, kmax + 1}):
            say(f"[gpu] k-core query {name} mode={mode} k={k}")
            got, st = K.kcore_subgraph(d_off, d_adj, k, mode=mode, stats=True)
            torch.cuda.synchronize()
            want = (core >= k).astype(np.int32)
            assert np.array_equal(got.cpu().numpy(), want), (name, k)
            assert st["device_status"] == 0 and st["rounds"] <= 1


@pytest.mark.parametrize("mode", MODES)
def test_batched_small(mode):
    b = gg.batch(64, 4, hi=20000)
    say(f"[gpu] batched 64 graphs V={b.n} m={b.m} mode={mode}")
    got, st = run_batched(b.offsets, b.adj, b.vptr, mode=mode)
    want = oracle.bz(b.offsets, b.adj)
    assert not first_mismatch(got, want), first_mismatch(got, want)
    assert st["edges"] == b.m


@pytest.mark.parametrize("mode", MODES)
def test_batched_equals_per_graph_and_handles_empty_graphs(mode):
    parts = [G.complete(9), G.csr(0, []), G.csr(5, []), G.hcns(30), G.grid(12), G.csr(1, [])]
    off, adj = G.union(parts)
    vptr = np.cumsum([0] + [len(p[0]) - 1 for p in parts]).astype(np.int64)
    say(f"[gpu] batched with empty graphs V={len(off) - 1} mode={mode}")
    got, _ = run_batched(off, adj, vptr, mode=mode)
    want = np.concatenate([oracle.bz(*p) for p in parts])
    assert not first_mismatch(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("mode", MODES)
def test_batched_large_graph_in_global_memory(mode):
    # graphs above the LDS capacity (6,144 to ~9,200 vertices, by what the device's LDS allows at
    # the kernel's occupancy) keep their state in the global workspace, with a peeled bitmap in LDS
    # up to 64 times that capacity (R-MAT scale 19) and without one above (scale 20)
    r15, r19, r20 = gg.rmat(15, 8, 3), gg.rmat(19, 4, 12), gg.rmat(20, 2, 13)
    road = gg.grid_road(200, 0.05, 0.01, 9)
    parts = [(r15.offsets, r15.adj), G.complete(40), (road.offsets, road.adj), (r19.offsets, r19.adj),
             (r20.offsets, r20.adj)]
    off, adj = G.union(parts)
    vptr = np.cumsum([0] + [len(p[0]) - 1 for p in parts]).astype(np.int64)
    say(f"[gpu] batched large graphs V={len(off) - 1} m={len(adj)} mode={mode}")
    got, _ = run_batched(off, adj, vptr, mode=mode)
    want = oracle.bz(off, adj)
    assert not first_mismatch(got, want), first_mismatch(got, want)


def test_batched_rows_staged_in_lds_and_not():
    """LDS-resident graphs of the level-sync batched peel whose rows fit beside their degrees and
    queue (12 bytes per vertex + 2 per entry within the workgroup's LDS) are peeled from an LDS copy
    of their rows; denser ones of the same size read their rows from global memory. A batch of both
    kinds, and of graphs on either side of the limit, must match the oracle graph by graph."""
    # complete graphs: K_n holds n(n-1) entries, so 12n + 2n(n-1) bytes; the limit lies between
    # K_120 (29 KB) and K_260 (136 KB) for any LDS share the device gives a workgroup
    parts = [G.complete(n) for n in (60, 120, 170, 185, 200, 260)]
    small = gg.batch(40, 8, hi=6000)
    parts += [small.subgraph(g) for g in range(40)]
    parts = [(p.offsets, p.adj) if hasattr(p, "offsets") else p for p in parts]
    off, adj = G.union(parts)
    vptr = np.cumsum([0] + [len(p[0]) - 1 for p in parts]).astype(np.int64)
    want = oracle.bz(off, adj)
    for mode in ("levelsync", "chained"):
        say(f"[gpu] batched staged rows mode={mode} V={len(off) - 1} m={len(adj)}")
        got, st = run_batched(off, adj, vptr, mode=mode)
        assert not first_mismatch(got, want), first_mismatch(got, want)
        assert st["device_status"] == 0 and st["edges"] == len(adj)


def test_batched_plain_entry_point_large_graphs():
    # the plain entry point (no options, no statistics) on graphs above the LDS capacity
    import torch
    import paper_2502_08042_amd as K
    from gpu_util import to_dev
    r15 = gg.rmat(15, 8, 3)
    road = gg.grid_road(200, 0.05, 0.01, 9)
    parts = [(r15.offsets, r15.adj), G.complete(40), (road.offsets, road.adj)]
    off, adj = G.union(parts)
    vptr = np.cumsum([0] + [len(p[0]) - 1 for p in parts]).astype(np.int64)
    say(f"[gpu] batched large graphs, plain entry point, V={len(off) - 1} m={len(adj)}")
    d_off, d_adj, d_vptr = to_dev(off, adj, vptr)
    out = torch.empty(len(off) - 1, dtype=torch.int32, device="cuda")
    rc = K._lib.kcore_decompose_batched(d_vptr.data_ptr(), d_off.data_ptr(), d_adj.data_ptr(), len(parts),
                                        len(off) - 1, out.data_ptr(), None)
    torch.cuda.synchronize()
    assert rc == 0, K.last_error()
    got, want = out.cpu().numpy(), oracle.bz(off, adj)
    assert not first_mismatch(got, want), first_mismatch(got, want)


def test_repeat_is_deterministic():
    g = gg.rmat(14, 16, 5)
    say("[gpu] repeat x5 levelsync rmat14")
    res = [run_single(g.offsets, g.adj, mode="levelsync") for _ in range(5)]
    for core, st in res[1:]:
        assert np.array_equal(core, res[0][0])
        assert st["subrounds"] == res[0][1]["subrounds"]


def test_validate_rejects_bad_csr():
    import paper_2502_08042_amd as K
    from gpu_util import to_dev
    off, adj = G.cycle(10)
    say("[gpu] validate good/bad")
    d_off, d_adj = to_dev(off, adj)
    K.decompose(d_off, d_adj, validate=True)
    bad = adj.copy()
    bad[0] = 5  # 0-5 entry without its reverse
    d_off, d_adj = to_dev(off, bad)
    with pytest.raises(K.KcoreError) as e:
        K.decompose(d_off, d_adj, validate=True)
    assert e.value.code == -7
    loop = adj.copy()
    loop[0] = 0
    d_off, d_adj = to_dev(off, loop)
    with pytest.raises(K.KcoreError):
        K.decompose(d_off, d_adj, validate=True)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("tail", [0, -1])
def test_multi_bucket_active_set(mode, tail):
    """Multi-bucket active set (Sec. 5.2): rounds read only the bucket holding the new k, and
    decrements move vertices to lower buckets. Coreness must be the oracle's; in level-sync mode
    the frontiers do not change, so rho must still be the sequential framework's."""
    cases = [("hcns300", None), ("hcns2000", None), ("rmat16", gg.config_rmat16()),
             ("road1024", gg.grid_road(1024, 0.05, 0.01, 2)), ("er5000", gg.erdos_renyi(5000, 0.02, 8)),
             ("rmat14", gg.rmat(14, 32, 3))]
    for name, g in cases:
        off, adj = (g.offsets, g.adj) if g is not None else G.hcns(int(name[4:]))
        want, sub, ls = oracle.levelsync(off, adj)
        for thr in (1 << 30, 1000):
            say(f"[gpu] buckets {name} mode={mode} tail={tail} threshold={thr}")
            got, st = run_single(off, adj, mode=mode, tail=tail, buckets=thr)
            assert not first_mismatch(got, want), f"{name}: {first_mismatch(got, want)}"
            assert st["peeled"] == len(off) - 1 and st["edges"] == len(adj), (name, st)
            assert st["device_status"] == 0, (name, st)
            assert st["rounds"] == ls["nonempty_rounds"], (name, st, ls)
            if mode == "levelsync":
                assert st["subrounds"] == ls["subrounds"], (name, st, ls)
            if int(want.max()) >= 16 and thr == 1 << 30 and tail == -1:
                assert st["bucket_inserts"] > 0, (name, st)
                assert st["live_decrements"] == len(adj) - int(want.astype(np.int64).sum())


def test_batched_teams_for_the_largest_graphs():
    """A batch whose few largest graphs each hold far more than a workgroup's share of the entries:
    those are peeled by teams of workgroups (cooperative launch, team barriers); every graph must
    still match the oracle, alone and with the small ones."""
    import torch
    parts = [gg.rmat(15, 16, 21), gg.rmat(14, 16, 22), gg.grid_road(256, 0.05, 0.01, 3)]
    small = gg.batch(300, 6, hi=3000)
    offs = [(p.offsets, p.adj) for p in parts] + [small.subgraph(g) for g in range(300)]
    offs = [(o.offsets, o.adj) if hasattr(o, "offsets") else o for o in offs]
    off, adj = G.union(offs)
    sizes = [len(o) - 1 for o, _ in offs]
    vptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    want = oracle.bz(off, adj)
    for mode in ("levelsync", "auto"):
        say(f"[gpu] batched teams mode={mode} G={len(sizes)} V={len(off) - 1} m={len(adj)}")
        got, st = run_batched(off, adj, vptr, mode=mode)
        assert not first_mismatch(got, want), first_mismatch(got, want)
        assert st["device_status"] == 0, st
        assert st["edges"] == len(adj), st
