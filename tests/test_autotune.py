"""Host logic of the autotuner (no GPU): workload classes, symbolic option values, and the
coordinate descent that must keep only candidates whose coreness equals the default's."""
import torch

import paper_2502_08042_amd.autotune as A


def test_workload_class_bins():
    # 4 vertices, avg degree 2: sparse, flat; a star of 1000 leaves: skewed
    off = torch.tensor([0, 2, 4, 6, 8], dtype=torch.int64)
    assert A.workload_class(off) == "single/1/sparse/flat"
    star = torch.cat([torch.tensor([0, 1000]), 1000 + torch.arange(1, 1001)]).to(torch.int64)
    assert A.workload_class(star).endswith("/sparse/skewed")
    dense = torch.arange(0, 65 * 40, 40, dtype=torch.int64)  # 64 vertices of degree 40
    assert A.workload_class(dense) == "single/3/dense/flat"
    assert A.workload_class(off, batched=True) == "batched/1"


def test_symbolic_values_resolve_per_graph():
    r = A._resolve({"tail": "n/32", "buckets": "n", "residual": -1, "tile_edges": 512}, 6400)
    assert r == {"tail": 200, "buckets": 6400, "residual": -1, "tile_edges": 512}
    assert A._resolve({"tail": "n/32"}, 10)["tail"] == 1


def test_descent_keeps_only_exact_and_faster_candidates():
    ref = torch.arange(10)
    cost = {("a", 1): 5.0, ("a", 2): 1.0, ("b", 7): 0.5}

    def run(o):
        ms = 10.0
        for k, v in o.items():
            ms = min(ms, cost.get((k, v), 10.0))
        # a=2 is fastest but gives a different answer: it must be rejected
        core = ref + 1 if o.get("a") == 2 else ref
        return ms, core

    best, best_ms, ref_ms, trials = A.tune({"a": [0, 1, 2], "b": [0, 7]}, run, log=lambda *x: None)
    assert ref_ms == 10.0
    assert best["a"] != 2
    assert best["b"] == 7 and best_ms == 0.5
    assert any(t.get("exact") is False for t in trials)


def test_shipped_cache_names_only_known_options():
    """The cache that ships with the package: every entry's options are fields the binding passes
    to the library (single graph: kcore_options; batched: the batched call's keywords)."""
    import paper_2502_08042_amd as K
    cache = A.load_cache()
    fields = {f for f, _ in K.Options._fields_}
    batched_kw = {"mode", "blocks_per_cu", "team_size", "batch_teams"}
    for dev, classes in cache.items():
        for cls, ent in classes.items():
            keys = set(ent["options"])
            if cls.startswith("batched/"):
                assert keys <= batched_kw, (dev, cls, keys)
            else:
                assert keys <= fields, (dev, cls, keys - fields)
            assert ent["ms"] <= ent["default_ms"] + 1e-9, (dev, cls)
