"""Batched execution (many uneven matching LPs in the same kernels): every
instance is checked on its own against facts that do not come from the
library -- the exact LP optimum (maximum matching size by Hopcroft-Karp, for
bipartite graphs the matching LP is integral, Section 3), feasibility of the
returned x and the (1 + eps) bracket -- and against the single-instance
solver on the same graph."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import maximum_bipartite_matching

import graphgen as gg

pytestmark = pytest.mark.gpu

EPS = 0.1


def _nu(g):
    nl = g.n_left
    A = sp.csr_matrix((np.ones(g.num_edges), (g.u, g.v - nl)), shape=(nl, g.num_vertices - nl))
    return int((maximum_bipartite_matching(A, perm_type="column") >= 0).sum())


def _instances():
    gs = gg.batch_bipartite(14, scale_div=64)            # sides 16 .. 1024, uneven
    gs.append(gg.complete_bipartite(3, 5))                # OPT = 3
    gs.append(gg.complete_bipartite(1, 6))                # star: OPT = 1
    gs.append(gg.Graph(2, np.array([0], np.int32), np.array([1], np.int32), n_left=1))   # one edge
    gs.append(gg.bipartite_uniform(300, 40, 900, seed=9))  # lopsided
    return gs


def _check(g, r, nu):
    assert r.certified, (r.lower, r.upper)
    assert r.lower - 1e-9 * nu <= nu <= r.upper * (1 + 1e-12)
    assert r.objective * (1 + EPS) >= nu * (1 - 1e-12)
    load = np.bincount(g.u, weights=r.x, minlength=g.num_vertices) + \
        np.bincount(g.v, weights=r.x, minlength=g.num_vertices)
    assert load.max() <= 1.0 + 1e-9 and r.x.min() >= 0.0
    assert abs(r.x.sum() - r.objective) <= 1e-9 * max(1.0, r.objective)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_matches_exact_optimum(precision):
    import paper_2307_03307_amd as mwu
    gs = _instances()
    with mwu.BatchSolver([(g.num_vertices, g.u, g.v) for g in gs], precision=precision) as b:
        res = b.solve()
    assert len(res) == len(gs)
    for g, r in zip(gs, res):
        _check(g, r, _nu(g))


def test_batch_agrees_with_single_instance_solver():
    import paper_2307_03307_amd as mwu
    gs = _instances()[:6]
    with mwu.BatchSolver([(g.num_vertices, g.u, g.v) for g in gs], precision=0) as b:
        res = b.solve()
    for g, r in zip(gs, res):
        with mwu.bmatch(g.num_vertices, g.u, g.v, precision=0) as s:
            r1 = s.solve()
        assert r1.certified and r.certified
        # both are certified (1 + eps) answers of the same LP
        assert max(r.objective, r1.objective) <= (1 + EPS) * min(r.objective, r1.objective)
        assert max(r.lower, r1.lower) <= min(r.upper, r1.upper) * (1 + 1e-12)


def test_batch_medium_uneven():
    """64 instances, sides 128 .. 8192, mean degree 4 .. 16, mixed form."""
    import paper_2307_03307_amd as mwu
    gs = gg.batch_bipartite(64, scale_div=8)
    with mwu.BatchSolver([(g.num_vertices, g.u, g.v) for g in gs]) as b:
        res = b.solve()
    for g, r in zip(gs, res):
        _check(g, r, _nu(g))


def test_batch_solve_twice_is_identical():
    """A second solve on the same handle starts again from the initial brackets
    and reproduces the first bit for bit (fixed-order reductions)."""
    import paper_2307_03307_amd as mwu
    gs = _instances()[:5]
    with mwu.BatchSolver([(g.num_vertices, g.u, g.v) for g in gs]) as b:
        r1 = b.solve()
        r2 = b.solve()
    for a, c in zip(r1, r2):
        assert a.total_iterations == c.total_iterations > 0
        assert a.objective == c.objective and a.lower == c.lower and a.upper == c.upper
        assert np.array_equal(a.x, c.x)


def test_batch_full_c5():
    """The full C5 batch (512 instances, sides uniform in [1024, 65536], mean
    degree uniform in [4, 16], 164M edges) in the chosen form with the layout
    the autotuner picks, as bench.py runs it: every instance certified, and
    for every 16th instance the exact optimum in the bracket with a feasible
    x (per-vertex loads at most 1)."""
    import paper_2307_03307_amd as mwu
    gs = gg.batch_bipartite(512)
    with mwu.BatchSolver([(g.num_vertices, g.u, g.v) for g in gs]) as b:
        res = b.solve()
    assert sum(r.certified for r in res) == len(gs)
    for k in range(0, len(gs), 16):
        _check(gs[k], res[k], _nu(gs[k]))


# ------------------------------------------------------------------ autotuner

TILE_E = {1024, 2048, 4096, 8192}
TILE_V = {1024, 2048, 4096, 8192, 16384}


def test_autotuner_sweeps_then_reuses(tmp_path):
    """The first create times a sweep and appends its choice to the cache
    file; a second create of the same batch shape reads it back; a record
    written by hand for the same key is taken as it stands; the tuned layout
    solves every instance to the exact optimum's bracket."""
    import paper_2307_03307_amd as mwu
    from paper_2307_03307_amd import _lib
    gs = gg.batch_bipartite(64, scale_div=8)
    spec = [(g.num_vertices, g.u, g.v) for g in gs]
    cache = tmp_path / "layouts.txt"
    with mwu.BatchSolver(spec, tune_cache=str(cache)) as b:
        lay = b.layout()
        print("tuned layout", lay)
        assert lay["source"] in (_lib.LAYOUT_TUNED, _lib.LAYOUT_CACHED)
        if lay["source"] == _lib.LAYOUT_TUNED:
            assert lay["candidates_timed"] >= 4 and lay["edge_iters_per_sec"] > 0
        assert lay["tile_edges"] in TILE_E and lay["tile_vertices"] in TILE_V
        assert lay["workgroups_per_cu"] in (2, 4, 8) and lay["search_launches"] in (1, 2, 3)
        res = b.solve()
    for g, r in zip(gs, res):
        _check(g, r, _nu(g))
    lines = [ln for ln in cache.read_text().split("\n") if ln.strip()]
    assert len(lines) == 1   # a sweep's record, or the process's record for the same shape
    with mwu.BatchSolver(spec, tune_cache=str(cache)) as b:
        again = b.layout()
    assert again["source"] == _lib.LAYOUT_CACHED
    assert all(again[f] == lay[f] for f in ("tile_edges", "tile_vertices", "workgroups_per_cu",
                                            "search_launches"))
    key = lines[-1].split()[0]
    hand = tmp_path / "hand.txt"
    hand.write_text("garbage line\n" + f"{key} 1024 8192 4 1 1.0e9\n")
    with mwu.BatchSolver(spec, tune_cache=str(hand)) as b:
        got = b.layout()
        res = b.solve()
    assert (got["tile_edges"], got["tile_vertices"], got["workgroups_per_cu"],
            got["search_launches"], got["source"]) == (1024, 8192, 4, 1, _lib.LAYOUT_CACHED)
    for g, r in zip(gs, res):
        _check(g, r, _nu(g))


def test_untuned_layout_is_the_default():
    import paper_2307_03307_amd as mwu
    from paper_2307_03307_amd import _lib
    gs = _instances()[:4]
    with mwu.BatchSolver([(g.num_vertices, g.u, g.v) for g in gs], tune=False) as b:
        lay = b.layout()
    assert lay["source"] == _lib.LAYOUT_DEFAULT and lay["candidates_timed"] == 0
    assert (lay["tile_edges"], lay["tile_vertices"], lay["workgroups_per_cu"],
            lay["search_launches"]) == (2048, 4096, 8, 2)


@pytest.mark.parametrize("precision", [0, 1])
def test_every_layout_solves(precision):
    """Extreme layouts (one-wave tiles, one workgroup per CU, one search
    launch per slot; 64Ki tiles, four search launches) give certified
    answers around the exact optimum; an invalid layout is rejected and the
    handle keeps working."""
    import paper_2307_03307_amd as mwu
    from paper_2307_03307_amd import _lib
    gs = _instances()
    nus = [_nu(g) for g in gs]
    with mwu.BatchSolver([(g.num_vertices, g.u, g.v) for g in gs], precision=precision,
                         tune=False) as b:
        for lay in [(256, 256, 1, 1), (65536, 65536, 16, 4), (1024, 2048, 2, 3)]:
            b.set_layout(*lay)
            got = b.layout()
            assert (got["tile_edges"], got["tile_vertices"], got["workgroups_per_cu"],
                    got["search_launches"]) == lay and got["source"] == _lib.LAYOUT_SET
            for g, r, nu in zip(gs, b.solve(), nus):
                _check(g, r, nu)
        for bad in [(300, 4096, 8, 2), (2048, 0, 8, 2), (2048, 4096, 0, 2), (2048, 4096, 8, 5),
                    (131072, 4096, 8, 2)]:
            with pytest.raises(_lib.MwuError) as e:
                b.set_layout(*bad)
            assert e.value.code == -1
        for g, r, nu in zip(gs, b.solve(), nus):
            _check(g, r, nu)
