"""mwu_potential_backward_noalloc against mwu_potential_backward (and the
value of mwu_potential_forward), through the C ABI: the same gradient and
value with every reduction record and chunk partial in the library's static
device array.  Two calls in a row, the second on a smaller problem (another
program), so that a stale record left in the shared array would show; then
the first problem again."""
import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


def _domset(precision):
    import paper_2307_03307_amd as mwu
    g = gg.chung_lu(20000, 2.1, 8.0, seed=41)       # power-law rows longer than one tile
    ptr, col = gg.adjacency_csr(g, with_identity=True)
    n = g.num_vertices
    rng = np.random.default_rng(3)
    x = rng.uniform(0.02, 0.12, n)
    return mwu.dominating_set(ptr, col, n, precision=precision), 0.05 * n, x


def _densest(precision):
    import paper_2307_03307_amd as mwu
    g = gg.gnm_random(300, 2000, seed=42)
    rng = np.random.default_rng(4)
    x = rng.uniform(0.1, 0.6, 2 * g.num_edges)
    return mwu.densest_subgraph(g.num_vertices, g.u, g.v, precision=precision), 1.3 * g.num_edges / 300, x


def _both(make, precision, grad_scale):
    import torch
    s, param, x = make(precision)
    with s:
        n = s.sizes().n
        assert n == x.shape[0]
        s.probe_begin(param)
        xt = torch.tensor(x, dtype=torch.float64, device="cuda")
        g_ref = torch.zeros(n, dtype=torch.float64, device="cuda")
        g_new = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
        v_ref = s.potential_forward(xt.data_ptr())
        s.potential_backward(xt.data_ptr(), grad_scale, g_ref.data_ptr())
        v_new = s.potential_backward_noalloc(xt.data_ptr(), grad_scale, g_new.data_ptr())
        torch.cuda.synchronize()
        a, b = g_ref.cpu().numpy(), g_new.cpu().numpy()
    return n, v_ref, v_new, a, b


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_backward(precision):
    out = []
    for make, scale in ((_domset, 1.0), (_densest, -0.75), (_domset, 2.5)):
        n, v_ref, v_new, a, b = _both(make, precision, scale)
        err = float(np.max(np.abs(a - b)) / max(np.max(np.abs(a)), 1e-300))
        out.append((make.__name__, n, err, v_ref, v_new))
        assert np.all(np.isfinite(b))
        # same kernels, same reduction order: the results agree to rounding
        # (and are expected to be bitwise equal)
        assert err <= 1e-12, (make.__name__, err)
        assert v_new == pytest.approx(v_ref, rel=1e-12, abs=1e-15)
    assert out[1][1] < out[0][1]          # the second call is on a smaller problem
    print(out)
