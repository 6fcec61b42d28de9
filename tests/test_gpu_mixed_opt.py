"""Mixed packing/covering optimization (MWU_MIXED_MAX / MWU_MIXED_MIN: the
objective embedded as one more row at a searched level M, the last sentence
of Section 2.2, reading R23) against HiGHS and the CPU oracle, through the
C ABI.

  per pass   a probe at a given M (the objective row at level 1/M, rewritten
             on the device before the probe): g, h, d, y, z, Pd, Cd and Psi,
             Phi at the Algorithm 1 point against the oracle's iteration on
             the matrices with that row appended, FP64 within 1e-9.
  solves     random LPs with uneven right-hand sides and costs, both senses,
             both precisions: the bracket certified within 1 + eps and
             consistent with HiGHS's optimum (infeasible verdicts are exact
             bounds), the returned point feasible within the reported
             violation; FP64 probe counts and brackets equal to the oracle's,
             the oracle's point within the same band.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog

import oracle
import paper_2307_03307_amd as mwu

from gpu_common import EPS, rel_err

pytestmark = pytest.mark.gpu

MAX_ITER = 20000


def _lp(seed, n=60, mP=25, mC=15, dens=0.15, rhs=True):
    rng = np.random.default_rng(seed)
    draw = lambda k: rng.uniform(0.5, 2.0, k)
    P = sp.random(mP, n, density=dens, random_state=rng, data_rvs=draw).tolil()
    C = sp.random(mC, n, density=dens, random_state=rng, data_rvs=draw).tolil()
    for j in range(n):
        if P[:, j].nnz == 0:
            P[rng.integers(mP), j] = 1.0
    for i in range(mC):
        if C[i].nnz == 0:
            C[i, rng.integers(n)] = 1.0
    bP = rng.uniform(0.5, 3.0, mP) if rhs else np.ones(mP)
    bC = rng.uniform(0.5, 3.0, mC) if rhs else np.ones(mC)
    c = rng.uniform(0.5, 2.0, n) if rhs else np.ones(n)
    return P.tocsr(), C.tocsr(), bP, bC, c


def _gpu(P, C, bP, bC, c, form, **kw):
    Pm = mwu.csr_matrix(P.indptr, P.indices, P.data, shape=P.shape)
    Cm = mwu.csr_matrix(C.indptr, C.indices, C.data, shape=C.shape)
    return mwu.Solver(form, P=Pm, C=Cm, b_P=bP, b_C=bC, c=c, **kw)


def _ocsr(A):
    A = sp.csr_matrix(A)
    return oracle.CSR(A.shape[0], A.shape[1], A.indptr.astype(np.int64), A.indices.astype(np.int32),
                      A.data.astype(np.float64))


def _normalized(P, C, bP, bC):
    return sp.diags(1.0 / bP) @ P, sp.diags(1.0 / bC) @ C


@pytest.mark.parametrize("maximize", [True, False])
def test_objective_row_per_pass_fp64(maximize):
    """A probe at level M: the device rewrites the embedded row to 1/M in
    both of its structures (and, minimizing, the column maxima of the
    Algorithm 1 point); the iteration at the start point then matches the
    oracle's on the matrices with the row (1/M) 1^T appended."""
    P, C, bP, bC, c = _lp(5, rhs=False)
    M = 7.5 if maximize else 3.0
    n = P.shape[1]
    obj = sp.csr_matrix(np.full((1, n), 1.0 / M))
    Pp, Cp = (P, sp.vstack([C, obj])) if maximize else (sp.vstack([P, obj]), C)
    Po, Co = _ocsr(Pp), _ocsr(Cp)
    x0 = np.zeros(n)
    oracle.lib().orc_initial_point(Po.c, 1.0, EPS, x0.ctypes.data)
    ref = oracle.iteration_terms(Po, 1.0, Co, 1.0, EPS, x0, alphas=[1.0, 4.0, 32.0])
    form = mwu.MIXED_MAX if maximize else mwu.MIXED_MIN
    with _gpu(P, C, bP, bC, c, form, precision=mwu.FP64) as s:
        sz = s.sizes()
        assert (sz.m_P, sz.m_C) == (Pp.shape[0], Cp.shape[0])
        s.probe_begin(M)
        s.probe_direction()
        got = {k: s.probe_read(k, m) for k, m in (("x", n), ("g", n), ("h", n), ("d", n), ("y", sz.m_P),
                                                   ("z", sz.m_C), ("dy", sz.m_P), ("dz", sz.m_C))}
        psi, phi, zm = s.probe_eval_steps([1.0, 4.0, 32.0])
    errs = {k: rel_err(got[k], ref[k]) for k in ("g", "h", "d", "y", "z", "dy", "dz")}
    errs["x"] = rel_err(got["x"], x0)
    errs["psi"] = rel_err(psi, ref["psi"])
    errs["phi"] = rel_err(phi, ref["phi"])
    print(f"mixed optimization per pass ({'max' if maximize else 'min'}): "
          + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    assert all(v <= 1e-9 for v in errs.values()), errs


@pytest.mark.parametrize("precision", [mwu.FP64, mwu.MIXED_FP32_FP64])
@pytest.mark.parametrize("maximize", [True, False])
@pytest.mark.parametrize("seed", [0, 2, 4])
def test_mixed_optimization_solves(seed, maximize, precision):
    P, C, bP, bC, c = _lp(seed)
    form = mwu.MIXED_MAX if maximize else mwu.MIXED_MIN
    # a near-optimum probe can take several thousand iterations; a probe cut
    # off by max_iter proves nothing and leaves the bracket open
    with _gpu(P, C, bP, bC, c, form, precision=precision, max_iter=MAX_ITER) as s:
        r = s.solve()
    x, viol = r.x, r.max_violation
    sgn = -1.0 if maximize else 1.0
    A = sp.vstack([P, -C]).toarray()

    def lp(slack):
        b = np.concatenate([bP * (1.0 + slack), -bC])
        res = linprog(sgn * c, A_ub=A, b_ub=b, bounds=(0, None))
        assert res.status == 0
        return sgn * res.fun

    opt, relaxed = lp(0.0), lp(viol)
    print(f"seed {seed} {'max' if maximize else 'min'} precision {precision}: OPT {opt:.6g}, bracket "
          f"[{r.lower:.6g}, {r.upper:.6g}], objective {r.objective:.6g}, violation {viol:.2e}, "
          f"{r.probes} probes, {r.total_iterations} iterations")
    assert r.certified and r.upper <= (1 + EPS) * r.lower * (1 + 1e-12)
    assert (C @ x / bC).min() >= 1 - 1e-9 and x.min() >= 0
    assert (P @ x / bP).max() <= 1 + viol + 1e-9 and viol <= EPS
    assert r.objective == pytest.approx(float(c @ x), rel=1e-9)
    if maximize:
        assert opt <= r.upper * (1 + 1e-9)
        assert r.objective >= r.lower * (1 - 1e-9) and r.objective <= relaxed * (1 + 1e-9)
    else:
        assert r.lower <= opt * (1 + 1e-9)
        assert r.objective >= relaxed * (1 - 1e-9) and r.objective <= r.upper * (1 + viol) * (1 + 1e-9)
    if precision == mwu.FP64:
        Pn, Cn = _normalized(P, C, bP, bC)
        ro, oviol = oracle.solve_mixed_opt(_ocsr(Pn), _ocsr(Cn), c, maximize, max_iter=MAX_ITER)
        assert ro.probes == r.probes
        assert r.lower == pytest.approx(ro.lower, rel=1e-9) and r.upper == pytest.approx(ro.upper, rel=1e-9)
        # the returned points come from runs of hundreds of iterations whose
        # last bits amplify (R13: the device scales columns by c where the
        # oracle puts c / M in the row), so both objectives are held to the
        # same certified band rather than to each other
        print(f"  oracle: objective {ro.objective:.9g} (relative difference "
              f"{abs(r.objective - ro.objective) / ro.objective:.1e}), violation {oviol:.2e}")
        if maximize:
            assert ro.lower * (1 - 1e-9) <= ro.objective <= lp(oviol) * (1 + 1e-9)
        else:
            assert lp(oviol) * (1 - 1e-9) <= ro.objective <= ro.upper * (1 + oviol) * (1 + 1e-9)


@pytest.mark.parametrize("precision", [mwu.FP64, mwu.MIXED_FP32_FP64])
@pytest.mark.parametrize("maximize", [True, False])
def test_mixed_optimization_infeasible_lp(maximize, precision):
    """An LP with no feasible point (HiGHS says so; seed 1 of the generator):
    every probe is infeasible, the search ends without a point or a
    certified bracket -- maximizing, the upper end shrinks to the bottom of
    the search range; minimizing, the level grows fourfold until the probes
    run out -- and in FP64 the probe count and the bracket equal the
    oracle's."""
    P, C, bP, bC, c = _lp(1)
    A = sp.vstack([P, -C]).toarray()
    assert linprog(c, A_ub=A, b_ub=np.concatenate([bP, -bC]), bounds=(0, None)).status == 2
    form = mwu.MIXED_MAX if maximize else mwu.MIXED_MIN
    with _gpu(P, C, bP, bC, c, form, precision=precision, max_probes=12) as s:
        r = s.solve()
    print(f"infeasible LP {'max' if maximize else 'min'} precision {precision}: status {r.status}, "
          f"bracket [{r.lower:.6g}, {r.upper:.6g}], {r.probes} probes")
    assert r.status == mwu.INFEASIBLE and not r.certified and r.probes == 12
    assert np.all(r.x == 0.0)
    if precision == mwu.FP64:
        Pn, Cn = _normalized(P, C, bP, bC)
        ro, _ = oracle.solve_mixed_opt(_ocsr(Pn), _ocsr(Cn), c, maximize, max_probes=12)
        assert not ro.certified and ro.probes == r.probes and not np.any(ro.x)
        assert r.lower == pytest.approx(ro.lower, rel=1e-9) and r.upper == pytest.approx(ro.upper, rel=1e-9)


def test_columns_without_covering_entries_leave_the_lp():
    """The min-lambda mixed form keeps only the columns with a covering
    entry; their packing entries leave the structure with them (they were
    once renumbered to -1).  The LP then solves bit for bit as the LP with
    those columns deleted, and they come back as 0."""
    P, C, bP, bC, _ = _lp(0, rhs=False)
    keep = np.asarray((C != 0).sum(axis=0)).ravel() > 0
    gone = ~keep & (np.asarray((P != 0).sum(axis=0)).ravel() > 0)
    assert gone.sum() >= 3
    with _gpu(P, C, bP, bC, None, mwu.MIXED, precision=mwu.FP64) as s:
        r = s.solve()
    Pk, Ck = P[:, keep].tocsr(), C[:, keep].tocsr()
    with _gpu(Pk, Ck, bP, bC, None, mwu.MIXED, precision=mwu.FP64) as s:
        rk = s.solve()
    print(f"{gone.sum()} packing-only columns: bracket [{r.lower:.9g}, {r.upper:.9g}], {r.probes} probes")
    assert r.certified and (r.lower, r.upper, r.probes) == (rk.lower, rk.upper, rk.probes)
    assert np.array_equal(r.x[keep], rk.x) and np.all(r.x[~keep] == 0.0)


@pytest.mark.parametrize("rule,drop", [(mwu.STEP_BIN_WARM, False), (mwu.STEP_NEWTON, False),
                                       (mwu.STEP_BIN, True), (mwu.STEP_BIN_WARM, True)])
@pytest.mark.parametrize("maximize", [True, False])
def test_mixed_optimization_step_rules_and_drop(maximize, rule, drop):
    """The embedded objective row with the warm-started and the Newton step
    searches and with met covering rows dropped (the objective row among
    them when maximizing): in FP64 the probe count and the bracket equal the
    oracle's run with the same rule and flag; the point is feasible."""
    P, C, bP, bC, c = _lp(0)
    form = mwu.MIXED_MAX if maximize else mwu.MIXED_MIN
    flags = mwu._lib.FLAG_DROP_SATISFIED if drop else 0
    with _gpu(P, C, bP, bC, c, form, precision=mwu.FP64, max_iter=MAX_ITER, step_rule=rule, flags=flags) as s:
        r = s.solve()
    Pn, Cn = _normalized(P, C, bP, bC)
    ro, _ = oracle.solve_mixed_opt(_ocsr(Pn), _ocsr(Cn), c, maximize, max_iter=MAX_ITER, step_rule=rule, drop=drop)
    print(f"{'max' if maximize else 'min'} rule {rule} drop {drop}: bracket [{r.lower:.6g}, {r.upper:.6g}] "
          f"(oracle [{ro.lower:.6g}, {ro.upper:.6g}]), {r.probes} probes, {r.total_iterations} iterations "
          f"(oracle {ro.total_iterations})")
    assert r.certified and ro.certified and r.probes == ro.probes
    assert r.lower == pytest.approx(ro.lower, rel=1e-9) and r.upper == pytest.approx(ro.upper, rel=1e-9)
    assert (C @ r.x / bC).min() >= 1 - 1e-9 and (P @ r.x / bP).max() <= 1 + r.max_violation + 1e-9
