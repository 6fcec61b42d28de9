"""The seeded input generators (`graphgen`) keep the properties their
recipes state: every graph is a canonical edge list (u < v, sorted, no
duplicates, no self-loops), the same seed gives the same graph, and each
family has the shape its recipe promises.  CPU only."""
import numpy as np
import pytest

import graphgen as gg


def _canonical(g):
    assert g.u.dtype == np.int32 and g.v.dtype == np.int32
    assert np.all(g.u < g.v)
    key = g.u.astype(np.int64) * g.num_vertices + g.v
    assert np.all(np.diff(key) > 0)                 # sorted, distinct
    assert g.v.max(initial=-1) < g.num_vertices and g.u.min(initial=0) >= 0


@pytest.mark.parametrize("make", [
    lambda s: gg.bipartite_uniform(300, 200, 2000, seed=s),
    lambda s: gg.rmat(10, 8, seed=s),
    lambda s: gg.chung_lu(3000, 2.3, 8.0, seed=s),
    lambda s: gg.gnm_random(500, 3000, seed=s),
    lambda s: gg.hub_graph(20, 300, 1000, seed=s),
    lambda s: gg.user_item(400, 150, 10, 30, 1.0, seed=s),
])
def test_canonical_and_seeded(make):
    g1, g2, g3 = make(7), make(7), make(8)
    _canonical(g1)
    assert np.array_equal(g1.u, g2.u) and np.array_equal(g1.v, g2.v)
    assert not (g1.num_edges == g3.num_edges and np.array_equal(g1.u, g3.u) and np.array_equal(g1.v, g3.v))


def test_bipartite_uniform_shape():
    g = gg.bipartite_uniform(300, 200, 2000, seed=1)
    assert g.num_edges == 2000 and g.n_left == 300 and g.num_vertices == 500
    assert g.u.max() < 300 and g.v.min() >= 300


def test_hub_graph_shape():
    g = gg.hub_graph(20, 300, 1000, seed=2)
    deg = g.degrees()
    assert np.all(deg[:20] == 300)                   # every hub at exactly hub_degree
    assert g.u.max() < 20 and g.v.min() >= 20        # leaves only meet hubs


def test_user_item_shape():
    g = gg.user_item(400, 150, 10, 30, 1.0, seed=3)
    deg = g.degrees()
    assert g.n_left == 400 and g.num_vertices == 550
    assert g.u.max() < 400 and g.v.min() >= 400      # ratings join a user and an item
    assert deg[:400].min() >= 10 and deg[:400].max() <= 30
    # long tail: the most popular item is rated far more often than the median one
    items = deg[400:]
    assert items.max() >= 5 * max(1, np.median(items))


def test_batch_bipartite_shape():
    gs = gg.batch_bipartite(6, scale_div=64)
    for k, g in enumerate(gs):
        nr = g.num_vertices - g.n_left
        assert 16 <= g.n_left <= 1024 and 16 <= nr <= 1024
        assert 4.0 * g.n_left - 1 <= g.num_edges <= min(16.0 * g.n_left + 1, g.n_left * nr)
        assert g.u.max() < g.n_left and g.v.min() >= g.n_left
    again = gg.batch_bipartite(6, scale_div=64)
    assert all(np.array_equal(a.u, b.u) and np.array_equal(a.v, b.v) for a, b in zip(gs, again))


def test_rmat_size():
    g = gg.rmat(12, 16, seed=2)
    assert g.num_vertices == 4096
    assert 0.5 * 16 * 4096 < g.num_edges <= 16 * 4096   # loops and duplicates removed
