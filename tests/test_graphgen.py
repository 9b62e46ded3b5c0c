"""Generators (no k-core arithmetic): the device HCNS builder draws the same graph as the small
test builder, here on CPU tensors."""
import numpy as np
import pytest

import graphs as G


@pytest.mark.parametrize("K", [2, 3, 7, 40, 129])
def test_hcns_device_builder_matches_reference_construction(K):
    import graphgen.gpu as gp
    off, adj = gp.hcns_device(K, device="cpu", rows_per_chunk=7)
    o2, a2 = G.hcns(K)
    off, adj = off.numpy(), adj.numpy()
    assert np.array_equal(off, o2)
    assert int(off[-1]) == 2 * K * K
    for v in range(2 * K):
        assert sorted(adj[off[v]:off[v + 1]].tolist()) == sorted(a2[o2[v]:o2[v + 1]].tolist())
