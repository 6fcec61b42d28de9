"""Dominating set LP at full C4 size on the generic CSR engine: the seeded
Chung-Lu graph with 2M vertices (exponent 2.3, mean degree 10), C = I + A in
CSR (pattern only), eps = 0.1.  No exact optimum is available at this size:
the check is the certified bracket (weak-duality lower bound, rescaled
feasible upper bound within 1 + eps) and feasibility of the returned x."""
import time

import numpy as np
import pytest
import scipy.sparse as sp

import graphgen as gg

pytestmark = pytest.mark.gpu

EPS = 0.1


@pytest.mark.parametrize("precision", [1, 0])
def test_domset_chung_lu_2m(precision):
    import paper_2307_03307_amd as mwu
    g = gg.cached("chunglu2m_g23_d10_s4", lambda: gg.chung_lu(2_000_000, 2.3, 10.0, seed=4))
    ptr, col = gg.adjacency_csr(g, with_identity=True)
    n = g.num_vertices
    t = time.perf_counter()
    with mwu.dominating_set(ptr, col, n, precision=precision) as s:
        create = time.perf_counter() - t
        t = time.perf_counter()
        r = s.solve()
        wall = time.perf_counter() - t
    print(f"C4 precision {precision}: create {create:.2f}s solve {wall:.3f}s obj {r.objective:.2f} "
          f"bracket [{r.lower:.2f}, {r.upper:.2f}] iters {r.total_iterations} probes {r.probes} "
          f"passes {r.search_passes}")
    assert r.status == mwu.CERTIFIED
    assert r.lower <= r.objective <= r.upper * (1 + 1e-12)
    assert r.upper <= (1 + EPS) * r.lower * (1 + 1e-12)
    A = sp.csr_matrix((np.ones(col.shape[0]), col, ptr), shape=(n, n))
    cov = A @ r.x
    assert cov.min() >= 1.0 - 1e-9
    assert abs(r.x.sum() - r.objective) <= 1e-9 * r.objective
