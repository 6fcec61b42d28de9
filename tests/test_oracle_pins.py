"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: every expected value comes from
a high-precision evaluation of the plain definitions, a closed form, a
textbook theorem evaluated by an independent library routine (Hopcroft-Karp,
HiGHS), or brute force over all subsets.
"""
import itertools
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog
from scipy.sparse.csgraph import maximum_bipartite_matching

import graphgen as gg

getcontext().prec = 60
EPS = 0.1


# ------------------------------------------------------------- definitions

def d_smax(y, eta):
    """smax_eta(y) = (1/eta) ln sum exp(eta y_i), Section 2.2, in 60 digits."""
    eta = Decimal(repr(eta))
    return sum((eta * Decimal(repr(float(v)))).exp() for v in y).ln() / eta


def d_smin(z, eta):
    eta = Decimal(repr(eta))
    return -sum((-eta * Decimal(repr(float(v)))).exp() for v in z).ln() / eta


def test_smax_smin_match_definition(oracle_mod):
    rng = np.random.default_rng(0)
    for m in (1, 2, 3, 7, 40):
        for eta in (2.5, 30.0, 800.0):
            y = rng.uniform(0, 1.5, m)
            v, w = oracle_mod.smax(y, eta)
            assert abs(Decimal(repr(float(v))) - d_smax(y, eta)) < Decimal("1e-14")
            v2, u = oracle_mod.smin(y, eta)
            assert abs(Decimal(repr(float(v2))) - d_smin(y, eta)) < Decimal("1e-14")
            # gradients are the softmax / softmin probability vectors
            ed = [(Decimal(repr(eta)) * Decimal(repr(float(t)))).exp() for t in y]
            s = sum(ed)
            for i in range(m):
                assert abs(Decimal(repr(float(w[i]))) - ed[i] / s) < Decimal("1e-14")
            assert abs(u.sum() - 1.0) < 1e-13 and np.all(u >= 0)
            # smooth max/min are within ln(m)/eta of max/min (Section 2.2, eta choice)
            assert y.max() - 1e-12 <= v <= y.max() + math.log(m) / eta + 1e-12
            assert y.min() - math.log(m) / eta - 1e-12 <= v2 <= y.min() + 1e-12


def test_single_entry_is_exact(oracle_mod):
    # smax and smin of one entry are the entry (end of Section 2.2)
    for val in (0.0, 0.37, 5.0):
        assert oracle_mod.smax([val], 900.0)[0] == pytest.approx(val, abs=1e-15)
        assert oracle_mod.smin([val], 900.0)[0] == pytest.approx(val, abs=1e-15)


def _phi_psi_decimal(y, dy, z, dz, eta, alpha):
    yp = [float(a) + alpha * float(b) for a, b in zip(y, dy)]
    zp = [float(a) + alpha * float(b) for a, b in zip(z, dz)]
    psi = d_smax(yp, eta) - d_smax(y, eta)
    phi = d_smin(zp, eta) - d_smin(z, eta)
    return float(psi), float(phi)


@pytest.mark.parametrize("alpha", [1e-3, 0.5, 1.0, 7.0, 300.0, 5e4])
def test_phi_psi_forms_match_definition(oracle_mod, alpha):
    """Section 4.1: Psi, Phi are differences of smax/smin; the oracle's
    cancellation-free evaluation must agree with a 60-digit evaluation of the
    plain differences, over alpha ranges hitting every branch."""
    rng = np.random.default_rng(int(alpha * 1000) % 997)
    eta = 200.0
    m = 9
    y = rng.uniform(0.2, 0.9, m)
    dy = rng.uniform(0, 2e-3, m)
    z = rng.uniform(0.1, 0.8, m)
    dz = rng.uniform(0, 4e-3, m)
    LP, w = oracle_mod.smax(y, eta)
    LC, u = oracle_mod.smin(z, eta)
    psi = oracle_mod.psi(y, dy, w, eta, LP, alpha)
    phi, zmn = oracle_mod.phi(z, dz, u, eta, LC, alpha)
    e_psi, e_phi = _phi_psi_decimal(y, dy, z, dz, eta, alpha)
    assert psi == pytest.approx(e_psi, rel=1e-10, abs=1e-300)
    assert phi == pytest.approx(e_phi, rel=1e-10, abs=1e-300)
    assert zmn == pytest.approx(float(np.min(z + alpha * dz)), rel=1e-15)


@pytest.mark.parametrize("alpha", [300.0, 3000.0])
def test_phi_psi_large_steps_match_definition(oracle_mod, alpha):
    """Section 4.1 at steps where eta*alpha*d reaches the thousands and the
    moved point keeps several comparable rows (near-uniform dy and dz), so
    that both log-sum terms of the shifted forms matter: 60-digit evaluation
    of the plain differences."""
    rng = np.random.default_rng(int(alpha))
    eta = 200.0
    m = 9
    y = rng.uniform(0.2, 0.21, m)
    dy = 1e-2 * (1 + rng.uniform(0, 1e-5, m))
    z = rng.uniform(0.1, 0.11, m)
    dz = 2e-2 * (1 + rng.uniform(0, 1e-5, m))
    LP, w = oracle_mod.smax(y, eta)
    LC, u = oracle_mod.smin(z, eta)
    psi = oracle_mod.psi(y, dy, w, eta, LP, alpha)
    phi, _ = oracle_mod.phi(z, dz, u, eta, LC, alpha)
    e_psi, e_phi = _phi_psi_decimal(y, dy, z, dz, eta, alpha)
    assert psi == pytest.approx(e_psi, rel=1e-12)
    assert phi == pytest.approx(e_phi, rel=1e-12)


def test_bang_for_buck_is_monotone(oracle_mod):
    """Proposition 1 (Section 4.1): f = Phi/Psi decreases in alpha."""
    rng = np.random.default_rng(7)
    eta = 150.0
    for trial in range(5):
        y = rng.uniform(0, 1, 12)
        dy = rng.uniform(0, 1e-2, 12)
        z = rng.uniform(0, 1, 15)
        dz = rng.uniform(0, 1e-2, 15)
        LP, w = oracle_mod.smax(y, eta)
        LC, u = oracle_mod.smin(z, eta)
        alphas = np.geomspace(1e-3, 1e3, 60)
        f = [oracle_mod.phi(z, dz, u, eta, LC, a)[0] / oracle_mod.psi(y, dy, w, eta, LP, a)
             for a in alphas]
        assert np.all(np.diff(f) <= 1e-9 * np.abs(f[:-1]))


def _scan(oracle_mod, y, dy, z, dz, eta):
    LP, w = oracle_mod.smax(y, eta)
    LC, u = oracle_mod.smin(z, eta)
    T = lambda a: oracle_mod.phi(z, dz, u, eta, LC, a)[0] >= oracle_mod.psi(y, dy, w, eta, LP, a)
    return LP, w, LC, u, T


def test_algorithm3_brackets_the_largest_step(oracle_mod):
    """Algorithm 3 returns lb with T(lb) true and T(ub) false, ub-lb <= eps*lb,
    so by monotonicity the largest admissible step lies in [lb, (1+eps) lb]."""
    rng = np.random.default_rng(11)
    eta = 300.0
    hits = 0
    for trial in range(12):
        y = rng.uniform(0, 0.5, 20)
        dy = rng.uniform(0, 1e-3, 20)
        z = rng.uniform(0, 0.3, 25)
        dz = rng.uniform(1e-4, 2e-3, 25) * rng.uniform(0.5, 4)
        LP, w, LC, u, T = _scan(oracle_mod, y, dy, z, dz, eta)
        a, ev = oracle_mod.step_search(y, dy, w, LP, z, dz, u, LC, eta, EPS)
        if not T(1.0):
            assert a < 1.0
            continue
        assert a >= 1.0 and T(a)
        if np.min(z + a * dz) >= 1.0:
            continue  # early return
        hits += 1
        assert not T(a * (1 + EPS) * 1.0000001) or not T(2 * a)
        # fine scan: the true crossing is within [a, (1+eps) a]
        grid = a * np.linspace(1.0, 2.0, 401)
        ok = np.array([T(b) for b in grid])
        cross = grid[np.argmin(ok)] if not ok.all() else 2 * a
        assert a <= cross <= a * (1 + EPS) * (1 + 1e-9)
    assert hits > 3


def test_algorithm3_early_return(oracle_mod):
    """If T(alpha) holds and min(z + alpha dz) >= 1 the search returns alpha
    immediately (Algorithm 3, early return)."""
    eta = 50.0
    y = np.array([0.1, 0.2])
    dy = np.array([1e-6, 1e-6])
    z = np.array([0.9, 0.95])
    dz = np.array([0.06, 0.06])
    LP, w = oracle_mod.smax(y, eta)
    LC, u = oracle_mod.smin(z, eta)
    a, ev = oracle_mod.step_search(y, dy, w, LP, z, dz, u, LC, eta, EPS)
    # alpha = 1 already makes z >= 0.96 < 1; alpha = 2 gives >= 1.02
    assert a == 2.0 and ev == 2


def _crossing(T, a, hi_factor=2.0, n=401):
    """First grid point in [a, hi_factor a] where T fails (hi_factor a if none)."""
    grid = a * np.linspace(1.0, hi_factor, n)
    ok = np.array([T(b) for b in grid])
    return grid[np.argmin(ok)] if not ok.all() else hi_factor * a


def test_warm_search_brackets_from_any_start(oracle_mod):
    """Warm start (reading R19): from any start above 1, upward or downward,
    the search still returns lb with T(lb) true and the largest admissible
    step within [lb, (1+eps) lb]; a failing T(1) still gives alpha < 1."""
    rng = np.random.default_rng(12)
    eta = 300.0
    down = up = 0
    for trial in range(10):
        y = rng.uniform(0, 0.5, 20)
        dy = rng.uniform(0, 1e-3, 20)
        z = rng.uniform(0, 0.3, 25)
        dz = rng.uniform(1e-4, 2e-3, 25) * rng.uniform(0.5, 4)
        LP, w, LC, u, T = _scan(oracle_mod, y, dy, z, dz, eta)
        a3, _ = oracle_mod.step_search(y, dy, w, LP, z, dz, u, LC, eta, EPS)
        for s in (1.5, 3.0 * max(a3, 1.0), 37.0 * max(a3, 1.0), 0.4 * max(a3, 1.0)):
            if s <= 1.0:
                continue
            a, ev = oracle_mod.step_search(y, dy, w, LP, z, dz, u, LC, eta, EPS, start=s)
            if not T(1.0):
                assert a < 1.0
                continue
            assert a >= 1.0 and T(a)
            if T(s):
                up += 1
            else:
                down += 1
                assert a < s
            if np.min(z + a * dz) >= 1.0:
                continue  # early return
            cross = _crossing(T, a)
            assert a <= cross <= a * (1 + EPS) * (1 + 1e-9)
    assert down > 3 and up > 3


def test_warm_search_from_one_is_algorithm3(oracle_mod):
    """Start 1 is Algorithm 3 as printed: same step, same evaluation count."""
    rng = np.random.default_rng(13)
    eta = 200.0
    for trial in range(5):
        y = rng.uniform(0, 0.5, 10)
        dy = rng.uniform(0, 1e-3, 10)
        z = rng.uniform(0, 0.3, 12)
        dz = rng.uniform(1e-4, 2e-3, 12)
        LP, w, LC, u, _ = _scan(oracle_mod, y, dy, z, dz, eta)
        assert (oracle_mod.step_search(y, dy, w, LP, z, dz, u, LC, eta, EPS, start=1.0)
                == oracle_mod.step_search(y, dy, w, LP, z, dz, u, LC, eta, EPS))


def test_warm_search_counts(oracle_mod):
    """Evaluation counts of the warm start: from s with T(s) true and T(2s)
    false, one doubling then at most 4 bisection steps (width s/16 <= eps s);
    from 2^k s it halves k times first; an early return on the way down
    stops at once."""
    rng = np.random.default_rng(14)
    eta = 300.0
    y = rng.uniform(0, 0.5, 20)
    dy = rng.uniform(0, 1e-3, 20)
    z = rng.uniform(0, 0.3, 25)
    dz = rng.uniform(1e-4, 2e-3, 25)
    LP, w, LC, u, T = _scan(oracle_mod, y, dy, z, dz, eta)
    a3, ev3 = oracle_mod.step_search(y, dy, w, LP, z, dz, u, LC, eta, EPS)
    assert a3 > 8.0 and np.min(z + a3 * dz) < 1.0      # a case with a long doubling phase
    cross = _crossing(T, a3)
    s = cross / 1.5                                     # T(s) holds, T(2 s) fails
    assert T(s) and not T(2 * s)
    a, ev = oracle_mod.step_search(y, dy, w, LP, z, dz, u, LC, eta, EPS, start=s)
    assert 5 <= ev <= 6 and ev < ev3
    assert a <= cross <= a * (1 + EPS) * (1 + 1e-9)
    a8, ev8 = oracle_mod.step_search(y, dy, w, LP, z, dz, u, LC, eta, EPS, start=8 * s)
    assert ev8 == ev + 3 - 1      # 8s, 4s, 2s fail, s holds (s itself not doubled again)
    # downward early return: T fails at s0, holds at s0 / 2^k, which covers
    # every row (Psi overtakes the linear Phi = 0.06 alpha near alpha = 5)
    y2 = np.array([0.1, 0.2])
    dy2 = np.array([0.08, 0.01])
    z2 = np.array([0.9, 0.95])
    dz2 = np.array([0.06, 0.06])
    eta2 = 50.0
    LP2, w2 = oracle_mod.smax(y2, eta2)
    LC2, u2 = oracle_mod.smin(z2, eta2)
    T2 = lambda b: (oracle_mod.phi(z2, dz2, u2, eta2, LC2, b)[0]
                    >= oracle_mod.psi(y2, dy2, w2, eta2, LP2, b))
    assert T2(2.0) and not T2(64.0)
    s0 = 2.0
    while T2(s0) and s0 < 64.0:
        s0 *= 2.0
    a2, ev2 = oracle_mod.step_search(y2, dy2, w2, LP2, z2, dz2, u2, LC2, eta2, EPS, start=s0)
    assert T2(a2) and np.min(z2 + a2 * dz2) >= 1.0
    k = int(round(np.log2(s0 / a2)))
    assert k >= 1 and a2 == s0 / 2 ** k and ev2 == k + 1


# --------------------------------------------------------- whole iterations

def _bmatch_problem(g):
    import oracle
    P = oracle.incidence(g)
    return P


def test_iteration_invariants(oracle_mod):
    """Algorithm 1/2 facts: P x0 <= eps; d >= 0 with d_i <= s x_i/eta; every
    accepted step keeps T; the potential smax(Px) - smin(Cx) never grows."""
    g = gg.bipartite_uniform(40, 40, 200, seed=3)
    P = oracle_mod.incidence(g)
    n = P.cols
    ones = oracle_mod.CSR(1, n, np.array([0, n]), np.arange(n), np.ones(n))
    M = 30.0
    x0 = np.zeros(n)
    import ctypes
    oracle_mod.lib().orc_initial_point(P.c, 1.0, EPS, x0.ctypes.data)
    assert (P.dense() @ x0).max() <= EPS * (1 + 1e-12)
    x = x0.copy()
    eta = oracle_mod.eta(P.rows + 1, EPS)
    pot_prev = None
    for it in range(25):
        t = oracle_mod.iteration_terms(P, 1.0, ones, 1.0 / M, EPS, x, alphas=[1.0])
        assert np.all(t["d"] >= 0)
        assert np.all(t["d"] <= (1.0 / eta) * x * (1 + 1e-12))   # s = 1: one covering row
        pot = t["LP"] - t["LC"]
        if pot_prev is not None:
            assert pot <= pot_prev + 1e-12
        pot_prev = pot
        if t["z"].min() >= 1:
            break
        a, _ = oracle_mod.step_search(t["y"], t["dy"], t["w"], t["LP"], t["z"], t["dz"], t["u"],
                                      t["LC"], eta, EPS)
        assert a >= 1.0
        tt = oracle_mod.iteration_terms(P, 1.0, ones, 1.0 / M, EPS, x, alphas=[a])
        assert tt["phi"][0] >= tt["psi"][0]
        x = x + a * t["d"]


def _weighted_mixed(mP, mC, n, seed):
    """Dense P (mP x n) and C (mC x n) with spread positive entries; column 0
    has tiny packing entries and a unit entry in every covering row, so its
    ratio g_0/h_0 is below 1e-6 at any point."""
    rng = np.random.default_rng(seed)
    P = rng.uniform(0.05, 2.0, (mP, n)) * (rng.random((mP, n)) < 0.5)
    C = rng.uniform(0.05, 2.0, (mC, n)) * (rng.random((mC, n)) < 0.5)
    P[:, 0] = 1e-7
    C[:, 0] = 1.0
    P[0, 1:] = np.where(P[0, 1:] > 0, P[0, 1:], 0.3)      # every column has a packing entry
    return P, C


@pytest.mark.parametrize("mP,mC,s", [(30, 20, 0.5), (25, 1, 1.0), (1, 18, 1.0)])
def test_smoothing_and_step_constants(oracle_mod, mP, mC, s):
    """Algorithm 1 fixes eta = 10 ln(m)/eps with m the rows of both sides, and
    Algorithm 2's direction scale s/eta, with s = 1/2 and s = 1 when one side
    is a single row (end of Section 2.2).  The smoothed max and min the probe
    carries equal 60-digit evaluations of their definitions at that eta, and a
    coordinate whose packing weight is negligible against its covering weight
    moves by (s/eta) x_i, the largest step the direction allows."""
    n = 40
    Pd, Cd = _weighted_mixed(mP, mC, n, seed=mP + 7 * mC)
    P, C = oracle_mod.CSR.from_dense(Pd), oracle_mod.CSR.from_dense(Cd)
    eta = 10.0 * math.log(mP + mC) / EPS
    x = np.random.default_rng(1).uniform(0.01, 0.05, n)
    t = oracle_mod.iteration_terms(P, 1.0, C, 1.0, EPS, x)
    assert t["LP"] == pytest.approx(float(d_smax(Pd @ x, eta)), rel=1e-13, abs=1e-14)
    assert t["LC"] == pytest.approx(float(d_smin(Cd @ x, eta)), rel=1e-13, abs=1e-14)
    ratio = t["d"] / x * eta / s
    assert ratio.max() <= 1 + 1e-12
    assert ratio[0] >= 1 - 1e-5


def test_initial_point_tight_per_column(oracle_mod):
    """Algorithm 1's start: every coordinate sits at eps/n of its tightest
    packing row, so P x0 <= eps 1 whatever the column scales (here spread
    over two orders of magnitude)."""
    Pd, Cd = _weighted_mixed(12, 5, 30, seed=3)
    P = oracle_mod.CSR.from_dense(Pd)
    n = P.cols
    x0 = np.zeros(n)
    assert oracle_mod.lib().orc_initial_point(P.c, 1.0, EPS, x0.ctypes.data) == 0
    assert (Pd @ x0).max() <= EPS * (1 + 1e-12)
    np.testing.assert_allclose((Pd * x0).max(axis=0), EPS / n, rtol=1e-14)


def test_probe_stops_at_first_covered_iterate(oracle_mod):
    """Algorithm 2 returns as soon as Cx >= 1: the iterate one accepted step
    earlier (the forced replay of all steps but the last) still has an
    uncovered row, and the returned one has none."""
    g = gg.bipartite_uniform(50, 60, 300, seed=4)
    P = oracle_mod.incidence(g)
    n = P.cols
    ones = oracle_mod.CSR(1, n, np.array([0, n]), np.arange(n), np.ones(n))
    opt = hopcroft_karp(g)
    rng = np.random.default_rng(5)
    Pd = rng.uniform(0.05, 2.0, (20, 30)) * (rng.random((20, 30)) < 0.5)
    Pd[0] = np.where(Pd[0] > 0, Pd[0], 0.3)
    Cd = rng.uniform(0.05, 2.0, (12, 30)) * (rng.random((12, 30)) < 0.5)
    Cd[:, 0] += 0.1
    cases = [(P, ones, 1.0 / (0.8 * opt)), (P, ones, 1.0 / (0.95 * opt)),
             (oracle_mod.CSR.from_dense(Pd), oracle_mod.CSR.from_dense(Cd), 2.0)]
    for Pc, Cc, sC in cases:
        r = oracle_mod.probe(Pc, 1.0, Cc, sC, EPS)
        assert r.status == oracle_mod.FEASIBLE and r.iterations >= 2
        assert (sC * Cc.dense() @ r.x).min() >= 1.0
        prev = oracle_mod.probe(Pc, 1.0, Cc, sC, EPS, max_iter=r.iterations - 1,
                                forced_alpha=r.alphas[:-1])
        assert prev.status == oracle_mod.MAX_ITER
        assert (sC * Cc.dense() @ prev.x).min() < 1.0


def test_probe_trajectory_matches_forced_replay(oracle_mod):
    """Decision replay: forcing the probe to its own step sequence reproduces
    its iterate bit for bit (the replay hook used against the GPU)."""
    g = gg.bipartite_uniform(50, 60, 300, seed=4)
    P = oracle_mod.incidence(g)
    n = P.cols
    ones = oracle_mod.CSR(1, n, np.array([0, n]), np.arange(n), np.ones(n))
    r1 = oracle_mod.probe(P, 1.0, ones, 1.0 / 40.0)
    r2 = oracle_mod.probe(P, 1.0, ones, 1.0 / 40.0, forced_alpha=r1.alphas)
    assert r1.status == r2.status and r1.iterations == r2.iterations
    assert np.array_equal(r1.x, r2.x)


# ------------------------------------------------------------ graph LP pins

def hopcroft_karp(g):
    B = sp.csr_matrix((np.ones(g.num_edges), (g.u, g.v - g.n_left)),
                      shape=(g.n_left, g.num_vertices - g.n_left))
    return int((maximum_bipartite_matching(B, perm_type="column") >= 0).sum())


def _check_packing(g, r, opt):
    import oracle
    M = oracle.incidence(g).dense()
    assert r.lower <= opt * (1 + 1e-9) and opt <= r.upper * (1 + 1e-9)
    assert (M @ r.x).max() <= 1 + 1e-9 and r.x.min() >= 0
    assert r.x.sum() == pytest.approx(r.objective, rel=1e-9)
    assert opt / r.objective <= 1 + EPS + 1e-9


@pytest.mark.parametrize("seed,nl,nr,ne", [(1, 30, 30, 90), (2, 50, 40, 160), (3, 80, 80, 400),
                                            (4, 200, 150, 900)])
def test_bmatch_equals_maximum_matching(oracle_mod, seed, nl, nr, ne):
    """No integrality gap for bipartite matching (Section 3): LP optimum =
    maximum matching size, computed by Hopcroft-Karp."""
    g = gg.bipartite_uniform(nl, nr, ne, seed=seed)
    r = oracle_mod.solve_bmatch(g)
    assert r.certified
    _check_packing(g, r, hopcroft_karp(g))


@pytest.mark.parametrize("a,b", [(3, 3), (4, 7), (9, 2)])
def test_bmatch_complete_bipartite(oracle_mod, a, b):
    g = gg.complete_bipartite(a, b)
    r = oracle_mod.solve_bmatch(g)
    _check_packing(g, r, min(a, b))


def test_bmatch_config_size(oracle_mod):
    """The 2000+2000 vertex, 20000 edge bipartite matching workload: within
    (1+eps) of the Hopcroft-Karp optimum."""
    g = gg.bipartite_uniform(2000, 2000, 20000, seed=1)
    r = oracle_mod.solve_bmatch(g)
    assert r.certified
    _check_packing(g, r, hopcroft_karp(g))


def _check_covering(C_dense, r, opt):
    assert r.lower <= opt * (1 + 1e-9) and opt <= r.upper * (1 + 1e-9)
    assert (C_dense @ r.x).min() >= 1 - 1e-9 and r.x.min() >= 0
    assert r.x.sum() == pytest.approx(r.objective, rel=1e-9)
    assert r.objective / opt <= 1 + EPS + 1e-9


def _double_cover_matching(g):
    """nu(G x K2): maximum matching of the bipartite double cover."""
    n = g.num_vertices
    r = np.concatenate([g.u, g.v])
    c = np.concatenate([g.v, g.u])
    B = sp.csr_matrix((np.ones(r.shape[0]), (r, c)), shape=(n, n))
    return int((maximum_bipartite_matching(B, perm_type="column") >= 0).sum())


@pytest.mark.parametrize("seed,n,m", [(1, 30, 60), (2, 60, 200), (3, 120, 300)])
def test_vcover_lp_equals_half_double_cover_matching(oracle_mod, seed, n, m):
    """Vertex cover LP optimum = fractional matching number = nu(G x K2)/2
    (LP duality plus half-integrality); cross-checked with HiGHS."""
    g = gg.gnm_random(n, m, seed=seed)
    r = oracle_mod.solve_vcover(g)
    opt = _double_cover_matching(g) / 2.0
    C, keep = oracle_mod.vertex_cover_matrix(g)
    A = C.dense()
    lp = linprog(np.ones(A.shape[1]), A_ub=-A, b_ub=-np.ones(A.shape[0]), bounds=(0, None))
    assert lp.fun == pytest.approx(opt, abs=1e-7)
    full = oracle_mod.incidence(g, drop_isolated=False).dense().T
    _check_covering(full, r, opt)


def test_vcover_bipartite_koenig(oracle_mod):
    """Koenig: on bipartite graphs the vertex cover LP equals the maximum matching."""
    g = gg.bipartite_uniform(60, 50, 250, seed=9)
    r = oracle_mod.solve_vcover(g)
    full = oracle_mod.incidence(g, drop_isolated=False).dense().T
    _check_covering(full, r, hopcroft_karp(g))


@pytest.mark.parametrize("make,opt", [
    (lambda: gg.regular_circulant(30, 4), 30 / 5),
    (lambda: gg.regular_circulant(24, 6), 24 / 7),
    (lambda: gg.complete_graph(9), 1.0),
    (lambda: gg.star_graph(12), 1.0),
    (lambda: gg.cycle_graph(21), 7.0),
])
def test_domset_closed_forms(oracle_mod, make, opt):
    """Dominating set LP: k-regular -> n/(k+1); K_n and stars -> 1; cycles -> n/3."""
    g = make()
    r = oracle_mod.solve_domset(g)
    _check_covering(oracle_mod.dominating_set_matrix(g).dense(), r, opt)


def test_domset_matches_highs(oracle_mod):
    g = gg.chung_lu(300, 2.3, 6.0, seed=4)
    D = oracle_mod.dominating_set_matrix(g).dense()
    lp = linprog(np.ones(D.shape[1]), A_ub=-D, b_ub=-np.ones(D.shape[0]), bounds=(0, None))
    r = oracle_mod.solve_domset(g)
    _check_covering(D, r, lp.fun)


def brute_force_density(g):
    best = 0.0
    n = g.num_vertices
    for mask in range(1, 1 << n):
        inS = np.array([(mask >> i) & 1 for i in range(n)], dtype=bool)
        e = int(np.sum(inS[g.u] & inS[g.v]))
        best = max(best, e / inS.sum())
    return best


def _check_densest(oracle_mod, g, r, opt):
    assert r.lower <= opt * (1 + 1e-9) and opt <= r.upper * (1 + 1e-9)
    O, W, keep = oracle_mod.densest_matrices(g)
    z = r.x
    assert (W.dense() @ z).min() >= 1 - 1e-9 and z.min() >= 0
    assert (O.dense() @ z).max() == pytest.approx(r.objective, rel=1e-9)
    assert r.objective / opt <= 1 + EPS + 1e-9


@pytest.mark.parametrize("seed,n,m", [(5, 14, 30), (6, 12, 40), (7, 16, 25)])
def test_densest_brute_force(oracle_mod, seed, n, m):
    """Densest subgraph LP = max over subsets of |E(S)|/|S| (Charikar)."""
    g = gg.gnm_random(n, m, seed=seed)
    r = oracle_mod.solve_densest(g)
    _check_densest(oracle_mod, g, r, brute_force_density(g))


@pytest.mark.parametrize("make,opt", [
    (lambda: gg.complete_graph(8), 3.5),
    (lambda: gg.cycle_graph(15), 1.0),
    (lambda: gg.path_graph(10), 0.9),
    (lambda: gg.random_tree(25, seed=3), 24 / 25),
])
def test_densest_closed_forms(oracle_mod, make, opt):
    """K_n -> (n-1)/2; cycles -> 1; trees (and paths) -> (n-1)/n."""
    g = make()
    r = oracle_mod.solve_densest(g)
    _check_densest(oracle_mod, g, r, opt)


def test_level_set_density_brute_force(oracle_mod):
    """The level-set rounding returns the best prefix density, which is the
    true maximum when scored by the indicator of a densest set."""
    g = gg.gnm_random(12, 30, seed=21)
    best = brute_force_density(g)
    n = g.num_vertices
    found = None
    for mask in range(1, 1 << n):
        inS = np.array([(mask >> i) & 1 for i in range(n)], dtype=bool)
        if np.sum(inS[g.u] & inS[g.v]) / inS.sum() == best:
            found = inS
            break
    v = oracle_mod.level_set_density(n, g.u, g.v, found.astype(float))
    assert v == pytest.approx(best, rel=1e-12)
    rng = np.random.default_rng(0)
    for _ in range(5):
        s = rng.random(n)
        order = np.argsort(-s, kind="stable")
        want = 0.0
        for k in range(1, n + 1):
            S = np.zeros(n, bool)
            S[order[:k]] = True
            want = max(want, np.sum(S[g.u] & S[g.v]) / k)
        assert oracle_mod.level_set_density(n, g.u, g.v, s) == pytest.approx(want, rel=1e-12)


def test_weak_duality_bounds(oracle_mod):
    """Every iteration's 1/min(P^T w) bounds the packing optimum from above and
    1/max(C^T u) bounds the covering optimum from below."""
    g = gg.bipartite_uniform(40, 40, 150, seed=12)
    opt = hopcroft_karp(g)
    P = oracle_mod.incidence(g)
    n = P.cols
    ones = oracle_mod.CSR(1, n, np.array([0, n]), np.arange(n), np.ones(n))
    for M in (0.6 * opt, 0.95 * opt, 1.3 * opt):
        pr = oracle_mod.probe(P, 1.0, ones, 1.0 / M)
        assert pr.pack_bound >= opt * (1 - 1e-12)
    C, keep = oracle_mod.vertex_cover_matrix(g)
    onesC = oracle_mod.CSR(1, C.cols, np.array([0, C.cols]), np.arange(C.cols), np.ones(C.cols))
    for M in (0.6 * opt, 1.3 * opt):
        pr = oracle_mod.probe(onesC, 1.0 / M, C, 1.0)
        assert pr.cover_bound <= opt * (1 + 1e-12)


def test_infeasible_probe_reports_infeasible(oracle_mod):
    """A probe with M well above the optimum cannot be feasible; the theorem of
    Section 4.1 says MWU then reports INFEASIBLE (and never FEASIBLE)."""
    g = gg.bipartite_uniform(40, 40, 150, seed=12)
    opt = hopcroft_karp(g)
    P = oracle_mod.incidence(g)
    n = P.cols
    ones = oracle_mod.CSR(1, n, np.array([0, n]), np.arange(n), np.ones(n))
    pr = oracle_mod.probe(P, 1.0, ones, 1.0 / (1.5 * opt))
    assert pr.status == oracle_mod.INFEASIBLE
    pr = oracle_mod.probe(P, 1.0, ones, 1.0 / (0.7 * opt))
    assert pr.status == oracle_mod.FEASIBLE
    # (1+eps)-relative point (Theorem, Section 4.1).  The early return of
    # Algorithm 3 may overshoot the covering side, so the statement is checked
    # on x / min(Cx), which keeps Cx >= 1: max(Px) / min(Cx) <= 1 + eps.
    Px = P.dense() @ pr.x
    z = pr.x.sum() / (0.7 * opt)
    assert z >= 1.0 and Px.max() / z <= 1 + EPS + 1e-12


def test_genmatch_probe_agrees_with_highs(oracle_mod):
    """Generalized matching (appendix): l <= M x <= u with users matched 3 to 5
    times and items at most `cap` times, as a fixed-lambda probe over P = M
    scaled by 1/u and C = the user rows scaled by 1/l.  HiGHS gives the
    smallest feasible cap (here set by a bottleneck of popular items, well
    above the average load) and decides each cap independently.  The theorem
    of Section 4.1 binds the verdicts: FEASIBLE only where the (1 + eps)-relaxed
    LP is feasible, with Px <= 1 + eps and Cx >= 1; INFEASIBLE only where the
    exact LP is infeasible.  With 5% slack on either side the verdict must be
    reached."""
    g = gg.user_item(60, 40, 3, 5, 1.5, seed=3)
    U, V, E = g.n_left, g.num_vertices, g.num_edges
    e = np.arange(E)
    M = np.zeros((V, E))
    M[g.u, e] = 1.0
    M[g.v, e] = 1.0
    Mu, Mi = M[:U], M[U:]
    lo, hi = 3.0, 5.0

    def lp_feasible(user_hi, cap):
        A = np.vstack([Mi, Mu, -Mu])
        b = np.concatenate([np.full(V - U, cap), np.full(U, user_hi), np.full(U, -lo)])
        st = linprog(np.zeros(E), A_ub=A, b_ub=b, bounds=(0, None)).status
        assert st in (0, 2)
        return st == 0

    # smallest cap: min t s.t. Mi x <= t, lo <= Mu x <= hi, x >= 0
    A = np.block([[Mi, -np.ones((V - U, 1))], [Mu, np.zeros((U, 1))], [-Mu, np.zeros((U, 1))]])
    b = np.concatenate([np.zeros(V - U), np.full(U, hi), np.full(U, -lo)])
    cap_star = linprog(np.r_[np.zeros(E), 1.0], A_ub=A, b_ub=b, bounds=(0, None)).fun
    assert cap_star > 1.5 * lo * U / (V - U)
    decided = {1.05 * cap_star: oracle_mod.FEASIBLE, 0.98 * cap_star / (1 + EPS): oracle_mod.INFEASIBLE}
    for cap in sorted(set(decided) | {0.7 * cap_star, 0.9 * cap_star, 1.2 * cap_star, 2.0 * cap_star}):
        ub = np.where(np.arange(V) < U, hi, cap)
        P = oracle_mod.CSR.from_coo(V, E, np.r_[g.u, g.v], np.r_[e, e], np.r_[1.0 / ub[g.u], 1.0 / ub[g.v]])
        C = oracle_mod.CSR.from_coo(U, E, g.u, e, np.full(E, 1.0 / lo))
        r = oracle_mod.probe(P, 1.0, C, 1.0, EPS)
        if cap in decided:
            assert r.status == decided[cap], (cap / cap_star, r.status)
        if r.status == oracle_mod.FEASIBLE:
            assert lp_feasible((1 + EPS) * hi, (1 + EPS) * cap)
            assert (Mi @ r.x).max() <= (1 + EPS) * cap * (1 + 1e-12)
            assert (Mu @ r.x).max() <= (1 + EPS) * hi * (1 + 1e-12)
            assert (Mu @ r.x).min() >= lo * (1 - 1e-12) and r.x.min() >= 0
        elif r.status == oracle_mod.INFEASIBLE:
            assert not lp_feasible(hi, cap)


def test_step_rule_effect(oracle_mod):
    """Table 2: the standard step needs orders of magnitude more iterations than
    the searched step on the same probe."""
    g = gg.bipartite_uniform(60, 60, 300, seed=2)
    P = oracle_mod.incidence(g)
    n = P.cols
    ones = oracle_mod.CSR(1, n, np.array([0, n]), np.arange(n), np.ones(n))
    M = 0.8 * hopcroft_karp(g)
    bin_ = oracle_mod.probe(P, 1.0, ones, 1.0 / M, step_rule=oracle_mod.STEP_BIN)
    std = oracle_mod.probe(P, 1.0, ones, 1.0 / M, step_rule=oracle_mod.STEP_STD, max_iter=200000)
    assert bin_.status == std.status == oracle_mod.FEASIBLE
    assert std.iterations >= 30 * bin_.iterations


def test_general_lp_normalization(oracle_mod):
    """Weighted packing max c^T x s.t. A x <= b via P = A/(b c^T) (Section 2.1),
    against HiGHS."""
    rng = np.random.default_rng(5)
    A = (rng.random((15, 25)) < 0.3) * rng.uniform(0.5, 3.0, (15, 25))
    A[0, :] += 0.1  # every column covered
    b = rng.uniform(1, 4, 15)
    c = rng.uniform(0.5, 2, 25)
    lp = linprog(-c, A_ub=A, b_ub=b, bounds=(0, None))
    P = oracle_mod.normalize_packing(oracle_mod.CSR.from_dense(A), b, c)
    r = oracle_mod.solve_packing(P)
    x = r.x / c
    assert (A @ x <= b * (1 + 1e-9)).all()
    assert -lp.fun / (c @ x) <= 1 + EPS + 1e-9
    assert r.lower <= -lp.fun * (1 + 1e-9) <= r.upper * (1 + 1e-9) * (1 + 1e-9)


# ------------------------------------------------------------- potential (autograd)

def _d_potential(Pd, sP, Cd, sC, eta, x):
    """smax(sP P x) - smin(sC C x) from the definitions, in 60 digits."""
    D = lambda v: Decimal(repr(float(v)))
    xd = [D(t) for t in x]
    y = [D(sP) * sum(D(Pd[r, c]) * xd[c] for c in range(len(x))) for r in range(Pd.shape[0])]
    z = [D(sC) * sum(D(Cd[r, c]) * xd[c] for c in range(len(x))) for r in range(Cd.shape[0])]
    e = D(eta)
    smax = sum((e * t).exp() for t in y).ln() / e
    smin = -sum((-e * t).exp() for t in z).ln() / e
    return smax - smin


@pytest.mark.parametrize("eta", [3.0, 60.0, 900.0])
def test_potential_value_and_gradient(oracle_mod, eta):
    """Section 4.1 potential and its gradient g - h: the value against the
    definitions in 60 digits, every gradient coordinate against a 60-digit
    central difference of the definitions (step 1e-25, truncation ~1e-45)."""
    rng = np.random.default_rng(int(eta))
    n, mP, mC = 6, 3, 4
    Pd = (rng.random((mP, n)) < 0.6) * rng.uniform(0.3, 2.0, (mP, n))
    Cd = (rng.random((mC, n)) < 0.6) * rng.uniform(0.3, 2.0, (mC, n))
    Pd[0, :] += 0.1
    Cd[0, :] += 0.1
    P, C = oracle_mod.CSR.from_dense(Pd), oracle_mod.CSR.from_dense(Cd)
    sP, sC = 0.7, 1.3
    x = rng.uniform(0.05, 0.6, n)
    v, gr = oracle_mod.potential(P, sP, C, sC, eta, x)
    ref = _d_potential(Pd, sP, Cd, sC, eta, x)
    assert abs(Decimal(repr(float(v))) - ref) < Decimal("1e-13") * max(Decimal(1), abs(ref))
    h = Decimal("1e-25")
    for i in range(n):
        xp = [Decimal(repr(float(t))) for t in x]
        xm = list(xp)
        xp[i] += h
        xm[i] -= h
        # _d_potential takes floats; evaluate the perturbed points in decimal directly
        def pot(xs):
            e = Decimal(repr(eta))
            y = [Decimal(repr(sP)) * sum(Decimal(repr(float(Pd[r, c]))) * xs[c] for c in range(n))
                 for r in range(mP)]
            z = [Decimal(repr(sC)) * sum(Decimal(repr(float(Cd[r, c]))) * xs[c] for c in range(n))
                 for r in range(mC)]
            return sum((e * t).exp() for t in y).ln() / e + sum((-e * t).exp() for t in z).ln() / e
        fd = (pot(xp) - pot(xm)) / (2 * h)
        assert abs(Decimal(repr(float(gr[i]))) - fd) < Decimal("1e-12") * max(Decimal(1), abs(fd))


# ------------------------------------------------------------------ probe-to-probe reuse (R21)

@pytest.mark.parametrize("seed", [1, 2])
def test_reuse_solves_bracket_exact_optima(oracle_mod, seed):
    """Outer searches whose probes start from their predecessor's rescaled
    point (and, warm-started, from its last step) still end certified around
    the exact optima: Hopcroft-Karp for matching, the double-cover matching
    for vertex cover, brute force for densest, HiGHS for dominating set."""
    for rule in (oracle_mod.STEP_BIN, oracle_mod.STEP_BIN_WARM):
        g = gg.bipartite_uniform(80, 80, 400, seed=seed)
        r = oracle_mod.solve_bmatch(g, step_rule=rule, reuse=True)
        assert r.certified and r.probes >= 2
        _check_packing(g, r, hopcroft_karp(g))
        g = gg.gnm_random(60, 200, seed=seed)
        C, keep = oracle_mod.vertex_cover_matrix(g)
        r = oracle_mod.solve_vcover(g, step_rule=rule, reuse=True)
        assert r.certified
        opt = _double_cover_matching(g) / 2.0
        assert r.lower <= opt * (1 + 1e-9) and opt <= r.upper * (1 + 1e-9)
        g = gg.gnm_random(14, 30, seed=seed + 4)
        r = oracle_mod.solve_densest(g, step_rule=rule, reuse=True)
        _check_densest(oracle_mod, g, r, brute_force_density(g))
        g = gg.chung_lu(200, 2.3, 6.0, seed=seed)
        D = oracle_mod.dominating_set_matrix(g).dense()
        opt = linprog(np.ones(D.shape[1]), A_ub=-D, b_ub=-np.ones(D.shape[0]), bounds=(0, None)).fun
        r = oracle_mod.solve_domset(g, step_rule=rule, reuse=True)
        assert r.certified
        _check_covering(D, r, opt)


def test_reuse_start_level_and_first_step(oracle_mod):
    """The reused start sits where the Algorithm 1 point does, max(P x0) = eps
    under the next probe's scale, and a warm-started probe given a start
    step searches its first step from there: the first accepted step is the
    warm search from that value on the same vectors, with the same number of
    tests (counted by the probe)."""
    g = gg.bipartite_uniform(60, 50, 300, seed=3)
    P = oracle_mod.incidence(g)
    n = P.cols
    one = oracle_mod.CSR(1, n, np.array([0, n]), np.arange(n), np.ones(n))
    nu = hopcroft_karp(g)
    r1 = oracle_mod.probe(P, 1.0, one, 1.0 / (0.9 * nu), EPS)
    x0 = oracle_mod.reuse_start(P, 1.0, EPS, r1.x)
    assert (P.dense() @ x0).max() == pytest.approx(EPS, rel=1e-14)
    assert np.allclose(x0 / r1.x, x0[0] / r1.x[0], rtol=1e-14)   # a uniform rescaling
    # and under a scaled P (the covering form's objective row (1/M) 1^T)
    C, keep = oracle_mod.vertex_cover_matrix(gg.gnm_random(40, 120, seed=2))
    nc = C.cols
    row = oracle_mod.CSR(1, nc, np.array([0, nc]), np.arange(nc), np.ones(nc))
    xc = np.random.default_rng(5).uniform(0.1, 1.0, nc)
    xs = oracle_mod.reuse_start(row, 1.0 / 37.0, EPS, xc)
    assert xs.sum() / 37.0 == pytest.approx(EPS, rel=1e-14)
    M2 = 0.95 * nu
    start = float(r1.last_alpha)
    assert start > 1.0
    r2 = oracle_mod.probe(P, 1.0, one, 1.0 / M2, EPS, x0=x0, step_rule=oracle_mod.STEP_BIN_WARM,
                          start_alpha=start, max_iter=1)
    t = oracle_mod.iteration_terms(P, 1.0, one, 1.0 / M2, EPS, x0)
    eta = oracle_mod.eta(P.rows + 1, EPS)
    a, ev = oracle_mod.step_search(t["y"], t["dy"], t["w"], t["LP"], t["z"], t["dz"], t["u"], t["LC"],
                                   eta, EPS, start=start)
    assert r2.iterations == 1 and r2.alphas[0] == a and r2.evaluations == ev
    # without a start step the first search is Algorithm 3 from 1
    r3 = oracle_mod.probe(P, 1.0, one, 1.0 / M2, EPS, x0=x0, step_rule=oracle_mod.STEP_BIN_WARM, max_iter=1)
    a1, ev1 = oracle_mod.step_search(t["y"], t["dy"], t["w"], t["LP"], t["z"], t["dz"], t["u"], t["LC"],
                                     eta, EPS)
    assert r3.alphas[0] == a1 and r3.evaluations == ev1


# ------------------------------------------------------------------ Newton step search (R20)

@pytest.mark.parametrize("alpha", [0.5, 7.0, 300.0])
def test_newton_derivatives_match_definition(oracle_mod, alpha):
    """Psi'(alpha) and Phi'(alpha) against 60-digit central differences of
    the definitions (differences of smax and smin, Section 4.1)."""
    rng = np.random.default_rng(int(alpha * 10) + 3)
    eta = 200.0
    m = 9
    y = rng.uniform(0.2, 0.9, m)
    dy = rng.uniform(0, 2e-3, m)
    z = rng.uniform(0.1, 0.8, m)
    dz = rng.uniform(0, 4e-3, m)
    dpsi, dphi = oracle_mod.step_derivatives(y, dy, z, dz, eta, alpha)
    D = lambda v: Decimal(repr(float(v)))
    E = D(eta)

    def moved(base, step, a, sign):            # sign*ln sum exp(sign*eta*(base+a*step)) / eta
        return sum((sign * E * (D(b) + a * D(t))).exp() for b, t in zip(base, step)).ln() / E

    a0, h = D(alpha), D(alpha) * Decimal("1e-12")
    e_psi = (moved(y, dy, a0 + h, 1) - moved(y, dy, a0 - h, 1)) / (2 * h)
    e_phi = (moved(z, dz, a0 - h, -1) - moved(z, dz, a0 + h, -1)) / (2 * h)
    assert dpsi == pytest.approx(float(e_psi), rel=1e-12)
    assert dphi == pytest.approx(float(e_phi), rel=1e-12)
    # a single row is its own average: the closed form of the embedded objective row
    a, b = oracle_mod.step_derivatives(y[:1], dy[:1], z[:1], dz[:1], eta, alpha)
    assert a == dy[0] and b == dz[0]


def test_newton_search_lands_below_the_crossing(oracle_mod):
    """The Newton search returns a step where the test holds (Phi >= Psi),
    at least 1, within (1 - eps)^2 of the largest admissible step (bracketed
    by Algorithm 3), from starts far below or above it too (the safeguard
    steps of R20), unless it returned early with every covering row met;
    from a start near the crossing it needs few tests."""
    rng = np.random.default_rng(21)
    eta = 300.0
    checked = 0
    near_evals = []
    for trial in range(12):
        y = rng.uniform(0, 0.5, 20)
        dy = rng.uniform(0, 1e-3, 20)
        z = rng.uniform(0, 0.3, 25)
        dz = rng.uniform(1e-4, 2e-3, 25) * rng.uniform(0.5, 4)
        LP, w, LC, u, T = _scan(oracle_mod, y, dy, z, dz, eta)
        if not T(1.0):
            a, _ = oracle_mod.newton_search(y, dy, w, LP, z, dz, u, LC, eta, EPS, 3.0)
            assert a < 1.0
            continue
        a3, _ = oracle_mod.step_search(y, dy, w, LP, z, dz, u, LC, eta, EPS)
        for s in (1.0, 0.7 * a3 + 0.3, (1 + EPS) * a3, 1.3 * a3, 20.0 * a3):
            a, ev = oracle_mod.newton_search(y, dy, w, LP, z, dz, u, LC, eta, EPS, max(s, 1.0))
            assert a >= 1.0 and T(a)
            if s in (0.7 * a3 + 0.3, 1.3 * a3):
                near_evals.append(ev)
            if np.min(z + a * dz) >= 1.0:
                continue                      # early return (R2)
            # T is monotone and Algorithm 3 brackets the largest admissible step in [a3, (1+eps) a3]
            assert a <= (1 + EPS) * a3 and a >= (1 - EPS) ** 2 * a3
            checked += 1
    assert checked >= 20
    # near its root Newton converges in a few steps: within 30% of the
    # crossing, three tests per search on average (Algorithm 3 needs 8-15 here)
    assert len(near_evals) >= 20 and np.mean(near_evals) <= 3.0


def test_newton_back_off_and_first_iteration(oracle_mod):
    """Reading R20 on a probe: its first iteration takes Algorithm 3's step
    from 1 (same step, same count of tests), and a failing test at 1 ends
    the search below 1 (the probe is infeasible)."""
    g = gg.bipartite_uniform(60, 50, 300, seed=3)
    P = oracle_mod.incidence(g)
    n = P.cols
    one = oracle_mod.CSR(1, n, np.array([0, n]), np.arange(n), np.ones(n))
    M = 0.9 * hopcroft_karp(g)
    r_n = oracle_mod.probe(P, 1.0, one, 1.0 / M, EPS, step_rule=oracle_mod.STEP_NEWTON, max_iter=1)
    r_b = oracle_mod.probe(P, 1.0, one, 1.0 / M, EPS, step_rule=oracle_mod.STEP_BIN, max_iter=1)
    assert r_n.alphas[0] == r_b.alphas[0] and r_n.evaluations == r_b.evaluations
    # T(1) failing: d pointing out of the packing region
    y = np.array([0.98, 0.5])
    dy = np.array([0.5, 0.0])
    z = np.array([0.2, 0.3])
    dz = np.array([1e-6, 2e-6])
    eta = 300.0
    LP, w = oracle_mod.smax(y, eta)
    LC, u = oracle_mod.smin(z, eta)
    assert oracle_mod.psi(y, dy, w, eta, LP, 1.0) > oracle_mod.phi(z, dz, u, eta, LC, 1.0)[0]
    a, ev = oracle_mod.newton_search(y, dy, w, LP, z, dz, u, LC, eta, EPS, 5.0)
    assert a < 1.0


@pytest.mark.parametrize("seed", [1, 2])
def test_newton_solves_bracket_exact_optima(oracle_mod, seed):
    """Outer searches with the Newton step (R20) end certified around the
    exact optima; the Newton search tests fewer steps per iteration than
    Algorithm 3 (Table 2's Nwt and Bin columns)."""
    rule = oracle_mod.STEP_NEWTON
    g = gg.bipartite_uniform(80, 80, 400, seed=seed)
    r = oracle_mod.solve_bmatch(g, step_rule=rule)
    assert r.certified
    _check_packing(g, r, hopcroft_karp(g))
    rb = oracle_mod.solve_bmatch(g)
    assert r.evaluations / r.total_iterations < rb.evaluations / rb.total_iterations
    g = gg.gnm_random(60, 200, seed=seed)
    r = oracle_mod.solve_vcover(g, step_rule=rule)
    assert r.certified
    opt = _double_cover_matching(g) / 2.0
    assert r.lower <= opt * (1 + 1e-9) and opt <= r.upper * (1 + 1e-9)
    g = gg.gnm_random(14, 30, seed=seed + 4)
    r = oracle_mod.solve_densest(g, step_rule=rule)
    _check_densest(oracle_mod, g, r, brute_force_density(g))
    g = gg.chung_lu(200, 2.3, 6.0, seed=seed)
    D = oracle_mod.dominating_set_matrix(g).dense()
    opt = linprog(np.ones(D.shape[1]), A_ub=-D, b_ub=-np.ones(D.shape[0]), bounds=(0, None)).fun
    r = oracle_mod.solve_domset(g, step_rule=rule)
    assert r.certified
    _check_covering(D, r, opt)


# ------------------------------------------------------------ general (non-bipartite) matching

def _fractional_matching_number(g):
    """nu_f(G) = nu(G x K2) / 2: the fractional matching LP has a
    half-integral optimum, and half-integral matchings of G correspond to
    matchings of its bipartite double cover."""
    return _double_cover_matching(g) / 2.0


@pytest.mark.parametrize("name", ["C5", "C9", "K5", "K8", "gnm", "chunglu", "odd-components"])
def test_general_matching_lp_equals_fractional_matching_number(oracle_mod, name):
    """Section 3's matching LP on graphs that are not bipartite: the packing
    LP max 1^T x s.t. M x <= 1 has the fractional matching number as its
    optimum, which exceeds the maximum matching on odd cycles (n/2 against
    (n-1)/2); certified brackets around nu(G x K2)/2, cross-checked with
    HiGHS, and a feasible x within (1 + eps)."""
    g = {"C5": lambda: gg.cycle_graph(5), "C9": lambda: gg.cycle_graph(9),
         "K5": lambda: gg.complete_graph(5), "K8": lambda: gg.complete_graph(8),
         "gnm": lambda: gg.gnm_random(80, 240, seed=31),
         "chunglu": lambda: gg.chung_lu(300, 2.3, 5.0, seed=32),
         # three disjoint triangles and a 5-cycle: nu_f = 3 * 1.5 + 2.5 = 7, nu = 5
         "odd-components": lambda: gg._from_pairs(14, [(0, 1), (1, 2), (2, 0), (3, 4), (4, 5), (5, 3),
                                                      (6, 7), (7, 8), (8, 6), (9, 10), (10, 11), (11, 12),
                                                      (12, 13), (13, 9)])}[name]()
    opt = _fractional_matching_number(g)
    M = oracle_mod.incidence(g).dense()
    highs = linprog(-np.ones(M.shape[1]), A_ub=M, b_ub=np.ones(M.shape[0]), bounds=(0, None)).fun
    assert -highs == pytest.approx(opt, rel=1e-9)
    closed = {"C5": 2.5, "C9": 4.5, "K5": 2.5, "K8": 4.0, "odd-components": 7.0}
    if name in closed:
        assert opt == closed[name]
    r = oracle_mod.solve_bmatch(g)
    assert r.certified
    _check_packing(g, r, opt)


# ------------------------------------------------------------ dropping satisfied covering rows (R22)

@pytest.mark.parametrize("name", ["vcover", "domset"])
def test_drop_is_the_iteration_on_the_unsatisfied_rows(oracle_mod, name):
    """Algorithm 2's drop line C <- {c_i : c_i^T x < 1} (R22): at a point
    where part of the covering rows is met, the iteration with dropping is
    the plain iteration (no dropping) on the LP whose covering side holds
    only the unmet rows, with the eta of the full row count: the same
    smoothed minimum, u (and 0 on the met rows), h, d, Cd on the kept rows,
    Psi, Phi and min z'.  Keeping the met rows changes h."""
    rng = np.random.default_rng(7)
    if name == "vcover":
        g = gg.gnm_random(80, 300, seed=8)
        C, keep = oracle_mod.vertex_cover_matrix(g)
    else:
        C = oracle_mod.dominating_set_matrix(gg.chung_lu(150, 2.3, 5.0, seed=9))
    n = C.cols
    one = oracle_mod.CSR(1, n, np.array([0, n]), np.arange(n), np.ones(n))
    Cd = C.dense()
    if name == "vcover":
        # every z_e = x_u + x_w within 2% of 1: the met rows still carry weight
        x = 0.5 + rng.uniform(-0.01, 0.01, n)
    else:
        x = rng.uniform(0.0, 0.8, n) / np.maximum(1.0, Cd.sum(axis=1).mean() / 2)
    z = Cd @ x
    met = z >= 1.0
    assert 0.2 < met.mean() < 0.8, met.mean()
    sP = 1.0 / (0.6 * n)
    alphas = [0.5, 3.0, 40.0]
    full = oracle_mod.iteration_terms(one, sP, C, 1.0, EPS, x, alphas=alphas, drop=True)
    R = Cd[~met]
    Rs = sp.csr_matrix(R)
    red = oracle_mod.CSR(R.shape[0], n, Rs.indptr.astype(np.int64), Rs.indices.astype(np.int32), Rs.data)
    ref = oracle_mod.iteration_terms(one, sP, red, 1.0, EPS, x, alphas=alphas, eta_=full["eta"])
    assert full["LC"] == pytest.approx(ref["LC"], rel=1e-14)
    assert np.array_equal(full["u"][met], np.zeros(met.sum()))
    assert np.allclose(full["u"][~met], ref["u"], rtol=1e-13, atol=0)
    for k in ("h", "d", "g"):
        assert np.allclose(full[k], ref[k], rtol=1e-13, atol=1e-300), k
    assert np.allclose(full["dz"][~met], ref["dz"], rtol=1e-13, atol=0)
    for k in ("psi", "phi", "zmin_new"):
        assert np.allclose(full[k], ref[k], rtol=1e-12, atol=0), k
    if name == "vcover":
        kept = oracle_mod.iteration_terms(one, sP, C, 1.0, EPS, x)
        # variables all of whose rows are met lose their h (and so their step)
        gone = (full["h"] == 0.0) & (kept["h"] > 0.0)
        assert gone.sum() >= 3


@pytest.mark.parametrize("seed", [1, 2])
def test_drop_solves_bracket_exact_optima(oracle_mod, seed):
    """Outer searches whose probes drop satisfied covering rows end certified
    around the exact optima of the covering LPs and the densest subgraph."""
    g = gg.gnm_random(60, 200, seed=seed)
    r = oracle_mod.solve_vcover(g, drop=True)
    assert r.certified
    opt = _double_cover_matching(g) / 2.0
    assert r.lower <= opt * (1 + 1e-9) and opt <= r.upper * (1 + 1e-9)
    C, keep = oracle_mod.vertex_cover_matrix(g)
    assert (C.dense() @ r.x[keep]).min() >= 1 - 1e-9
    g = gg.chung_lu(200, 2.3, 6.0, seed=seed)
    D = oracle_mod.dominating_set_matrix(g).dense()
    dopt = linprog(np.ones(D.shape[1]), A_ub=-D, b_ub=-np.ones(D.shape[0]), bounds=(0, None)).fun
    r = oracle_mod.solve_domset(g, drop=True)
    assert r.certified
    _check_covering(D, r, dopt)
    g = gg.gnm_random(14, 30, seed=seed + 4)
    r = oracle_mod.solve_densest(g, drop=True)
    _check_densest(oracle_mod, g, r, brute_force_density(g))


# ------------------------------------------------------------ mixed optimization (R23)

def _rand_mixed_lp(seed, n=30, mP=12, mC=8, dens=0.25):
    rng = np.random.default_rng(seed)
    draw = lambda k: rng.uniform(0.5, 2.0, k)
    P = sp.random(mP, n, density=dens, random_state=rng, data_rvs=draw).tolil()
    C = sp.random(mC, n, density=dens, random_state=rng, data_rvs=draw).tolil()
    for j in range(n):                       # every variable in some packing row
        if P[:, j].nnz == 0:
            P[rng.integers(mP), j] = 1.0
    for i in range(mC):                      # no empty covering row
        if C[i].nnz == 0:
            C[i, rng.integers(n)] = 1.0
    return P.tocsr(), C.tocsr(), rng.uniform(0.5, 2.0, n)


def _as_csr(oracle_mod, A):
    return oracle_mod.CSR(A.shape[0], A.shape[1], A.indptr.astype(np.int64), A.indices.astype(np.int32),
                          A.data.astype(np.float64))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("maximize", [True, False])
def test_mixed_optimization_brackets_the_lp_optimum(oracle_mod, seed, maximize):
    """End of Section 2.2: a mixed packing/covering optimization LP solved by
    embedding its objective as one more row and searching its level (R23).
    Against HiGHS on random LPs: the infeasible verdicts bound OPT exactly
    (maximizing: OPT <= upper; minimizing: lower <= OPT), the returned x
    meets every covering row and the objective level of the bracket end it
    comes from, it is feasible for the packing rows relaxed by the reported
    violation (so its objective is at most / at least the relaxed LP's
    optimum), the violation stays within eps, and the bracket is certified
    within 1 + eps."""
    P, C, c = _rand_mixed_lp(seed)
    r, viol = oracle_mod.solve_mixed_opt(_as_csr(oracle_mod, P), _as_csr(oracle_mod, C), c, maximize)
    sgn = -1.0 if maximize else 1.0
    A = np.vstack([P.toarray(), -C.toarray()])

    def lp(slack):
        b = np.concatenate([np.full(P.shape[0], 1.0 + slack), -np.ones(C.shape[0])])
        res = linprog(sgn * c, A_ub=A, b_ub=b, bounds=(0, None))
        assert res.status == 0
        return sgn * res.fun

    opt, relaxed = lp(0.0), lp(viol)
    x = r.x
    assert r.certified and r.upper <= (1 + EPS) * r.lower * (1 + 1e-12)
    assert (C.toarray() @ x).min() >= 1 - 1e-9 and x.min() >= 0
    assert (P.toarray() @ x).max() <= 1 + viol + 1e-12 and viol <= EPS
    assert r.objective == pytest.approx(float(c @ x), rel=1e-12)
    if maximize:
        assert opt <= r.upper * (1 + 1e-12)
        assert r.objective >= r.lower * (1 - 1e-12) and r.objective <= relaxed * (1 + 1e-9)
    else:
        assert r.lower <= opt * (1 + 1e-12)
        assert r.objective >= relaxed * (1 - 1e-9)
        assert r.objective <= r.upper * (1 + viol) * (1 + 1e-12)   # the objective row, within the violation
