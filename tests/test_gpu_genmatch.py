"""Generalized matching (the mixed feasibility LP of the paper's appendix):
exists x >= 0 with l <= M x <= u, M the vertex-edge incidence of a
user-item rating graph; users matched between 3 and 5 times, items at most
`cap` times, no lower bound for items (so items have no covering row).  The
Netflix and KDD rating data are not available: seeded synthetic user-item
graphs with a long-tailed item popularity stand in for them.

The packing side is M with right-hand side u (edge-list incidence), the
covering side the user rows of M with right-hand side l (CSR); one
feasibility probe at lambda = 1.  The oracle runs the same probe on the
normalised matrices.  Reported along the way: the max violation
max{0, max(Px) - 1, 1 - min(Cx)} of the paper's comparison (the appendix
figure), at checkpoints of the probe."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_common import EPS, rel_err
import paper_2307_03307_amd as mwu

pytestmark = pytest.mark.gpu

LB, UB = 3.0, 5.0


def genmatch_problem(g, cap):
    """(GPU solver factory, oracle P, oracle C): P is M with rows scaled by
    1/u, C the user rows of M scaled by 1/l."""
    import paper_2307_03307_amd as mwu
    users = g.n_left
    E, V = g.num_edges, g.num_vertices
    ub = np.where(np.arange(V) < users, UB, float(cap))
    lb = np.full(users, LB)
    e = np.arange(E)
    # oracle: rows normalised by their right-hand sides
    P = oracle.CSR.from_coo(V, E, np.concatenate([g.u, g.v]), np.concatenate([e, e]),
                            np.concatenate([1.0 / ub[g.u], 1.0 / ub[g.v]]))
    C = oracle.CSR.from_coo(users, E, g.u, e, np.full(E, 1.0 / LB))
    # GPU: the incidence from the edge list, the user rows as CSR (edges are
    # sorted by user, so each user's edges are contiguous)
    ptr = np.zeros(users + 1, np.int64)
    np.cumsum(np.bincount(g.u, minlength=users), out=ptr[1:])

    def make(**kw):
        return mwu.Solver(mwu.MIXED, P=mwu.incidence(V, g.u, g.v),
                          C=mwu.csr_matrix(ptr, e.astype(np.int32), shape=(users, E)),
                          b_P=ub, b_C=lb, fixed_lambda=1.0, **kw)
    return make, P, C


def rows(M, x):
    out = np.zeros(M.rows)
    oracle.lib().orc_matvec(M.c, 1.0, np.ascontiguousarray(x).ctypes.data, out.ctypes.data)
    return out


def violation(P, C, x):
    return max(0.0, rows(P, x).max() - 1.0, 1.0 - rows(C, x).min())


@pytest.fixture(scope="module")
def small():
    return gg.user_item(2000, 400, 10, 30, 1.0, seed=31)


def test_genmatch_fp64_follows_oracle(small):
    """FP64: the GPU's free-running probe takes the oracle's steps one for
    one, ends with its verdict, and its iterate matches; the max violation
    falls along the probe (oracle replay of the GPU's steps)."""
    import paper_2307_03307_amd as mwu
    make, P, C = genmatch_problem(small, cap=60)
    with make(precision=mwu.FP64) as s:
        s.probe_begin(1.0)
        info = s.probe_run(5000)
        alphas = s.probe_read("alpha", info.iterations)
        xg = s.probe_read("x", s.sizes().n)
    r = oracle.probe(P, 1.0, C, 1.0, EPS)
    assert info.status == r.status == oracle.FEASIBLE
    assert info.iterations == r.iterations and np.array_equal(alphas, r.alphas)
    # same steps; the iterate carries the reduction-order differences of g
    # and h, amplified by the steps (R13; observed 2.8e-8 on the sum and
    # 1.2e-6 on the largest coordinate difference here; bounds about 4x)
    e_sum = abs(xg.sum() - r.x.sum()) / r.x.sum()
    e_x = rel_err(xg, r.x)
    print(f"genmatch FP64 iterate: sum rel err {e_sum:.2e}, x rel err {e_x:.2e}")
    assert e_sum <= 1e-7
    assert e_x <= 5e-6
    curve = []
    for t in sorted({1, 2, 4, 8, 16, 32, r.iterations} & set(range(1, r.iterations + 1))):
        rt = oracle.probe(P, 1.0, C, 1.0, EPS, max_iter=t, forced_alpha=alphas[:t])
        curve.append((t, violation(P, C, rt.x)))
    print("genmatch max violation by iteration: " + ", ".join(f"{t}: {v:.3g}" for t, v in curve))
    assert curve[-1][1] <= EPS          # feasible: covering rows met, packing within (1 + eps)
    assert curve[-1][1] < curve[0][1]


@pytest.mark.parametrize("precision", [0, 1])
def test_genmatch_solve(small, precision):
    """The fixed-lambda solve in both forms: a feasible verdict whose point
    meets every bound within the reported max violation, and whose reported
    objective is the lambda of that same point."""
    make, P, C = genmatch_problem(small, cap=60)
    with make(precision=precision) as s:
        r = s.solve()
    print(f"genmatch precision {precision}: status {r.status} iterations {r.total_iterations} "
          f"max violation {r.max_violation:.3g}")
    assert r.status == mwu.FEASIBLE_POINT
    assert r.max_violation <= EPS
    assert violation(P, C, r.x) <= r.max_violation * (1 + 1e-6) + 1e-9
    assert rows(C, r.x).min() >= 1 - 1e-9
    # lambda of the returned point: the largest packing row (P carries 1/u)
    assert r.objective == pytest.approx(rows(P, r.x).max(), rel=1e-9)
