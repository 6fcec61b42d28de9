"""GPU parity against the CPU oracle, through the C ABI.

Modes (oracle vs gfx950 library):
  per-pass      identical x fed to both: y = Px, z = Cx, g, h, d, Pd, Cd and
                Psi, Phi, min(z + a Cd) at candidate steps.  FP64 form: max
                relative error <= 1e-9.  Mixed FP32/FP64 form: per-quantity
                bounds in units of 2^-24 (MIXED_TOL).
  replay        the oracle is forced to the GPU's step sequence: FP64 final x
                objective within 1e-9 (final x within 1e-6), mixed form final
                objective within 1e-5.
  free run      both solve; both certified within (1+eps) of the exact optimum
                and within eps of each other.  Exact agreement is not a
                property of the method: with steps of 1e3-1e4 the MWU map
                amplifies last-bit differences about tenfold per iteration, so
                two correct FP64 runs drift apart late in a long probe (the
                replay tests bound this) and may then take different
                decisions and probes.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2307_03307_amd as mwu

from gpu_common import (EPS, bmatch_case, densest_case, domset_case, ones_row, rel_err, start_point,
                        vcover_case, weighted_packing_case)

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-9
# Chosen form, per quantity, in units of the FP32 unit roundoff U = 2^-24:
# x, y, z are FP32-stored values and FP32 row sums; g and h are normalized
# weights, whose common shift (the LSE total) cancels the rounding of the
# dominant rows, so they keep O(U) too; d = (s/eta) q x multiplies the
# rounding of g/h by x and the products Pd, Cd sum it over the rows; Psi and
# Phi (relative to the scale of the test Phi >= Psi) carry the FP32 terms of
# the search.  Each bound is about 3x the largest error seen over the cases
# below, so an error ten times larger fails.
U = 2.0 ** -24
MIXED_TOL = {"x": 4 * U, "y": 6 * U, "z": 6 * U, "g": 6 * U, "h": 24 * U, "d": 64 * U, "dy": 32 * U,
             "dz": 64 * U, "psi": 24 * U, "phi": 12 * U, "psi_list": 24 * U, "phi_list": 12 * U,
             "zmin": 4 * U, "zmin_list": 4 * U}
EXP_ALPHAS = [float(2 ** k) for k in range(8)]    # one exponential-grid pass
LIST_ALPHAS = [0.37, 1.0, 3.5, 11.0, 70.0]


def _cases():
    bip = gg.bipartite_uniform(700, 650, 9000, seed=21)          # several tiles, ragged tail
    gnm = gg.gnm_random(900, 7000, seed=22)
    star = gg.star_graph(5000)
    pl = gg.chung_lu(3000, 2.3, 8.0, seed=23)                     # power-law rows
    return {
        "bmatch": lambda: bmatch_case(bip),
        "vcover": lambda: vcover_case(gnm),
        "vcover-generic": lambda: vcover_case(gnm, generic=True),
        "vcover-star": lambda: vcover_case(star, param=2.0),       # a row of 5000 > one tile
        # 600 rows of 2100 > one tile: more long rows than the pass A finisher
        # takes, completed by the direction pass
        "vcover-hubs": lambda: vcover_case(gg.hub_graph(600, 2100, 20000, seed=26), param=400.0),
        "domset": lambda: domset_case(pl),
        "domset-star": lambda: domset_case(gg.star_graph(6000), param=3.0),
        "densest": lambda: densest_case(gg.gnm_random(400, 3000, seed=24)),
        "densest-generic": lambda: densest_case(gg.gnm_random(400, 3000, seed=24), generic=True),
        "densest-powerlaw": lambda: densest_case(gg.chung_lu(3000, 2.1, 8.0, seed=25)),   # long vertex rows
        "weighted": lambda: weighted_packing_case(),
        # matching LP on a graph with odd cycles (not bipartite), probed at
        # 0.8 of its fractional matching number nu(G x K2)/2 = 450
        "gmatch": lambda: bmatch_case(gg.gnm_random(900, 5000, seed=41), param=360.0),
    }


CASES = _cases()


def _per_pass(case, precision, tol, seed=0, direction=True):
    x0 = start_point(case, seed)
    sP, sC = case.sP(case.param), case.sC(case.param)
    ref = oracle.iteration_terms(case.P, sP, case.C, sC, EPS, x0,
                                 alphas=EXP_ALPHAS)
    ref_list = oracle.iteration_terms(case.P, sP, case.C, sC, EPS, x0, alphas=LIST_ALPHAS)
    with case.make_gpu(precision=precision) as s:
        sz = s.sizes()
        assert sz.n == case.P.cols
        assert sz.eta == pytest.approx(ref["eta"], rel=1e-15)
        s.probe_begin(case.param, x0)
        s.probe_direction()
        got = {k: s.probe_read(k, n) for k, n in
               (("x", sz.n), ("d", sz.n), ("g", sz.n), ("h", sz.n), ("y", sz.m_P),
                ("z", sz.m_C), ("dy", sz.m_P), ("dz", sz.m_C))}
        errs = {k: rel_err(got[k], ref[k]) for k in ("d", "g", "h", "y", "z", "dy", "dz")}
        errs["x"] = rel_err(got["x"], x0)
        psi, phi, zm = s.probe_eval_steps(EXP_ALPHAS)
        psi2, phi2, zm2 = s.probe_eval_steps(LIST_ALPHAS)
    for name, (a, b, other) in {"psi": (psi, ref["psi"], ref["phi"]), "phi": (phi, ref["phi"], ref["psi"]),
                                "psi_list": (psi2, ref_list["psi"], ref_list["phi"]),
                                "phi_list": (phi2, ref_list["phi"], ref_list["psi"])}.items():
        if precision == mwu.FP64:
            scale = np.abs(b)
        else:
            # the mixed form is held to the scale of the test Phi >= Psi that the
            # values feed: a Psi far below Phi may underflow in FP32 per term
            scale = np.maximum(np.abs(b), np.abs(other))
        errs[name] = float(np.max(np.abs(a - b) / np.maximum(scale, 1e-300)))
    errs["zmin"] = rel_err(zm, ref["zmin_new"])
    errs["zmin_list"] = rel_err(zm2, ref_list["zmin_new"])
    if not direction:
        # d, Pd, Cd and the step sums depend on coordinates whose weights lie
        # below float range; their error is reported, not bounded
        for k in ("d", "dy", "dz", "psi", "phi", "psi_list", "phi_list", "zmin", "zmin_list"):
            errs.pop(k)
    print(f"per-pass {case.name} precision {precision}: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    bad = {k: v for k, v in errs.items() if not v <= (tol[k] if isinstance(tol, dict) else tol)}
    assert not bad, (case.name, bad)
    return errs


@pytest.mark.parametrize("name", list(CASES))
def test_per_pass_fp64(name):
    _per_pass(CASES[name](), mwu.FP64, FP64_TOL)


# g of the general-matching case: a CPU emulation of the chosen form's row
# values (float32 row sums of float32 x in CSR order, FP64 weights formed from
# them) puts 12.8 U into g on this graph against 1.8 U on the bipartite case:
# the vertex rows holding most of the weight carry eta (about 680) times the
# rounding of their own y, which the common shift does not cancel.  The bound
# is three times the emulated error.
MIXED_TOL_CASE = {"gmatch": dict(MIXED_TOL, g=40 * U)}


@pytest.mark.parametrize("name", ["bmatch", "vcover", "vcover-star", "vcover-hubs", "domset", "weighted",
                                  "densest", "densest-powerlaw", "gmatch"])
def test_per_pass_mixed(name):
    """The fused densest program forms g_i / h_i in the log domain, so its FP32
    direction matches even where both FP32 weights underflow."""
    _per_pass(CASES[name](), mwu.MIXED_FP32_FP64, MIXED_TOL_CASE.get(name, MIXED_TOL))


def test_per_pass_mixed_densest_generic_weights():
    """Generic engine on the densest-subgraph LP in the mixed form: both sides
    are exponential weights, so coordinates whose weights underflow float get
    d = 0; the weights, g and h themselves still match to float accuracy."""
    # h sums one covering weight per variable (single-weight rows): observed 2.8e-6
    tol = dict(MIXED_TOL, h=128 * U)
    _per_pass(CASES["densest-generic"](), mwu.MIXED_FP32_FP64, tol, direction=False)


def _replay(case, precision):
    sP, sC = case.sP(case.param), case.sC(case.param)
    with case.make_gpu(precision=precision) as s:
        s.probe_begin(case.param)
        info = s.probe_run(5000)
        alphas = s.probe_read("alpha", info.iterations)
        xg = s.probe_read("x", s.sizes().n)
    r = oracle.probe(case.P, sP, case.C, sC, EPS, forced_alpha=alphas)
    return info, alphas, xg, r


@pytest.mark.parametrize("name", ["bmatch", "vcover", "domset", "densest", "densest-generic", "weighted",
                                  "gmatch"])
def test_decision_replay_fp64(name):
    case = CASES[name]()
    info, alphas, xg, r = _replay(case, mwu.FP64)
    assert info.status == r.status
    assert info.iterations == r.iterations
    # per-iteration quantities agree to 1e-9 (per-pass tests); over a whole
    # probe, steps of up to 1e5 amplify last-bit differences of coordinates
    # with g_i/h_i near 1, so the iterate is held to 1e-6 and its objective to 1e-9
    assert abs(xg.sum() - r.x.sum()) <= FP64_TOL * r.x.sum()
    assert rel_err(xg, r.x) <= 1e-6
    # free-running oracle takes the same decisions in FP64
    sP, sC = case.sP(case.param), case.sC(case.param)
    free = oracle.probe(case.P, sP, case.C, sC, EPS)
    assert free.iterations == info.iterations and np.array_equal(free.alphas, alphas)
    # the device counts the tests of Algorithm 3 as the sequential oracle makes them
    assert info.evaluations == free.evaluations


@pytest.mark.parametrize("name", ["bmatch", "vcover", "domset", "densest", "densest-generic"])
def test_decision_replay_fp64_warm(name):
    """Warm-started search (reading R19, MWU_STEP_BIN_WARM): in FP64 the GPU's
    free run takes the warm-started oracle's decisions step for step, halvings
    from a failing start included."""
    case = CASES[name]()
    sP, sC = case.sP(case.param), case.sC(case.param)
    with case.make_gpu(precision=mwu.FP64, step_rule=mwu.STEP_BIN_WARM) as s:
        s.probe_begin(case.param)
        info = s.probe_run(5000)
        alphas = s.probe_read("alpha", info.iterations)
        xg = s.probe_read("x", s.sizes().n)
    free = oracle.probe(case.P, sP, case.C, sC, EPS, step_rule=oracle.STEP_BIN_WARM)
    down = int(np.sum(alphas[1:] < alphas[:-1]))   # searches that went below their start
    bin3 = oracle.probe(case.P, sP, case.C, sC, EPS)
    print(f"{name}: warm {info.iterations} iterations, {info.search_passes} passes, "
          f"{free.evaluations} oracle evaluations ({down} downward); Algorithm 3 from 1: "
          f"{bin3.iterations} iterations, {bin3.evaluations} evaluations")
    assert info.status == free.status
    assert info.iterations == free.iterations and np.array_equal(alphas, free.alphas)
    assert abs(xg.sum() - free.x.sum()) <= FP64_TOL * free.x.sum()
    assert rel_err(xg, free.x) <= 1e-6


# The chosen form's weights and search terms are FP32; the oracle replays the
# GPU's steps.  Rows that sum many weights (matching, covers) average the FP32
# rounding of the direction out.  The densest program has single-weight rows
# and steps up to ~3e5, where a 1e-7 relative perturbation of the direction
# grows to 1e-5..1e-2 in a probe's objective, so its direction state (x, d,
# Pd, Cd, the log-domain ratio) is FP64 and only its weights are FP32.
MIXED_REPLAY_TOL = {"bmatch": 1e-5, "vcover": 1e-5, "domset": 1e-5, "densest": 1e-5}


@pytest.mark.parametrize("name", list(MIXED_REPLAY_TOL))
def test_decision_replay_mixed(name):
    case = CASES[name]()
    info, alphas, xg, r = _replay(case, mwu.MIXED_FP32_FP64)
    assert info.status == r.status
    err = abs(xg.sum() - r.x.sum()) / r.x.sum()
    print(f"{name}: mixed replay objective rel err {err:.2e}")
    assert err <= MIXED_REPLAY_TOL[name]


@pytest.mark.parametrize("precision", [mwu.FP64, mwu.MIXED_FP32_FP64])
def test_sparse_transpose_pass(precision):
    """Per-pass parity of the transpose and direction passes over the active
    lists (R17): 600 iterations into a near-optimum vertex-cover probe most
    covering rows carry exactly zero weight in FP32 and the transpose pass
    visits only the active neighbours; g, h and d at that point match the
    oracle's full sums at the same x."""
    g = gg.rmat(13, 16, seed=2)
    C, keep = oracle.vertex_cover_matrix(g)
    n = C.cols
    param = 1.02 * _opt_vcover(g)
    sP = 1.0 / param
    with mwu.vertex_cover(g.num_vertices, g.u, g.v, precision=precision) as s:
        s.probe_begin(param)
        info = s.probe_run(600)
        assert info.status == mwu._lib.PROBE_RUNNING
        _, _, nnz = s.time_pass(0, 2)      # nonzeros the transpose pass visits now
        s.probe_direction()
        x = s.probe_read("x", n)            # the point the passes saw (pending step committed)
        got = {k: s.probe_read(k, n) for k in ("g", "h", "d")}
    ref = oracle.iteration_terms(ones_row(n), sP, C, 1.0, EPS, x)
    errs = {k: rel_err(got[k], ref[k]) for k in ("g", "h", "d")}
    print(f"precision {precision}: transpose pass over {nnz:.0f} of {2 * C.rows} nonzeros; {errs}")
    if precision == mwu.MIXED_FP32_FP64:
        assert nnz < 0.6 * 2 * C.rows
    # observed 1.6e-7 on h and d in the chosen form
    tol = {k: 1e-9 for k in errs} if precision == mwu.FP64 else {"g": 6 * U, "h": 8 * U, "d": 8 * U}
    assert all(v <= tol[k] for k, v in errs.items()), errs


def _opt_bmatch(g):
    import scipy.sparse as sp
    from scipy.sparse.csgraph import maximum_bipartite_matching
    B = sp.csr_matrix((np.ones(g.num_edges), (g.u, g.v - g.n_left)),
                      shape=(g.n_left, g.num_vertices - g.n_left))
    return int((maximum_bipartite_matching(B, perm_type="column") >= 0).sum())


def _opt_vcover(g):
    import scipy.sparse as sp
    from scipy.sparse.csgraph import maximum_bipartite_matching
    n = g.num_vertices
    r = np.concatenate([g.u, g.v])
    c = np.concatenate([g.v, g.u])
    B = sp.csr_matrix((np.ones(r.shape[0]), (r, c)), shape=(n, n))
    return int((maximum_bipartite_matching(B, perm_type="column") >= 0).sum()) / 2.0


@pytest.mark.parametrize("precision", [mwu.FP64, mwu.MIXED_FP32_FP64])
def test_solve_bmatch(precision):
    g = gg.bipartite_uniform(2000, 2000, 20000, seed=1)   # the 2000+2000 / 20000 workload
    opt = _opt_bmatch(g)
    with mwu.bmatch(g.num_vertices, g.u, g.v, precision=precision) as s:
        r = s.solve()
    assert r.certified
    assert r.lower <= opt <= r.upper * (1 + 1e-12)
    assert opt / r.objective <= 1 + EPS
    load = np.bincount(g.u, weights=r.x, minlength=g.num_vertices) + \
        np.bincount(g.v, weights=r.x, minlength=g.num_vertices)
    assert load.max() <= 1 + 1e-9 and r.x.min() >= 0
    assert r.x.sum() == pytest.approx(r.objective, rel=1e-9)
    if precision == mwu.FP64:
        ro = oracle.solve_bmatch(g)
        assert ro.certified and r.objective == pytest.approx(ro.objective, rel=EPS)


@pytest.mark.parametrize("precision", [mwu.FP64, mwu.MIXED_FP32_FP64])
def test_solve_general_matching(precision):
    """The matching LP of Section 3 on graphs that are not bipartite: its
    optimum is the fractional matching number nu(G x K2)/2 (half-integral
    LP), above the maximum matching wherever odd cycles are left over.
    Certified brackets around it, a feasible x, and agreement with the
    oracle's certified answer."""
    graphs = {"K7": gg.complete_graph(7),                  # nu_f = 3.5, nu = 3
              "C9": gg.cycle_graph(9),                     # nu_f = 4.5, nu = 4
              "gnm": gg.gnm_random(3000, 15000, seed=42),
              "powerlaw": gg.chung_lu(5000, 2.2, 6.0, seed=43)}
    for name, g in graphs.items():
        opt = _opt_vcover(g)                    # = nu(G x K2)/2, the fractional matching number
        with mwu.bmatch(g.num_vertices, g.u, g.v, precision=precision) as s:
            r = s.solve()
        assert r.certified, name
        assert r.lower <= opt * (1 + 1e-12) and opt <= r.upper * (1 + 1e-12), (name, r.lower, opt, r.upper)
        assert opt / r.objective <= 1 + EPS + 1e-12, name
        load = np.bincount(g.u, weights=r.x, minlength=g.num_vertices) + \
            np.bincount(g.v, weights=r.x, minlength=g.num_vertices)
        assert load.max() <= 1 + 1e-9 and r.x.min() >= 0, name
        if name in ("K7", "C9"):
            assert opt == {"K7": 3.5, "C9": 4.5}[name]
        if precision == mwu.FP64 and g.num_vertices <= 3000:
            ro = oracle.solve_bmatch(g)
            assert ro.certified and r.objective == pytest.approx(ro.objective, rel=EPS)


@pytest.mark.parametrize("precision", [mwu.FP64, mwu.MIXED_FP32_FP64])
@pytest.mark.parametrize("generic", [False, True])
def test_solve_vcover(precision, generic):
    g = gg.rmat(13, 16, seed=2)                       # power-law, isolated vertices
    opt = _opt_vcover(g)
    flags = mwu._lib.FLAG_GENERIC if generic else 0
    with mwu.vertex_cover(g.num_vertices, g.u, g.v, precision=precision, flags=flags) as s:
        r = s.solve()
    assert r.certified
    assert r.lower <= opt * (1 + 1e-12) and opt <= r.upper * (1 + 1e-12)
    assert r.objective / opt <= 1 + EPS
    assert (r.x[g.u] + r.x[g.v]).min() >= 1 - 1e-9 and r.x.min() >= 0
    deg = g.degrees()
    assert np.all(r.x[deg == 0] == 0)
    if precision == mwu.FP64:
        ro = oracle.solve_vcover(g)
        assert ro.certified and r.objective == pytest.approx(ro.objective, rel=EPS)


@pytest.mark.parametrize("precision", [mwu.FP64, mwu.MIXED_FP32_FP64])
def test_solve_domset(precision):
    from scipy.optimize import linprog
    g = gg.chung_lu(400, 2.3, 6.0, seed=4)
    ptr, col = gg.adjacency_csr(g, with_identity=True)
    D = oracle.dominating_set_matrix(g).dense()
    opt = linprog(np.ones(D.shape[1]), A_ub=-D, b_ub=-np.ones(D.shape[0]), bounds=(0, None)).fun
    with mwu.dominating_set(ptr, col, g.num_vertices, precision=precision) as s:
        r = s.solve()
    assert r.certified
    assert r.lower <= opt * (1 + 1e-9) and opt <= r.upper * (1 + 1e-9)
    assert (D @ r.x).min() >= 1 - 1e-9
    if precision == mwu.FP64:
        ro = oracle.solve_domset(g)
        assert ro.certified and r.objective == pytest.approx(ro.objective, rel=EPS)


@pytest.mark.parametrize("precision", [mwu.FP64, mwu.MIXED_FP32_FP64])
@pytest.mark.parametrize("generic", [False, True])
def test_solve_densest(precision, generic):
    g = gg.gnm_random(16, 34, seed=5)
    best = 0.0
    for mask in range(1, 1 << 16):
        S = np.array([(mask >> i) & 1 for i in range(16)], bool)
        best = max(best, np.sum(S[g.u] & S[g.v]) / S.sum())
    flags = mwu._lib.FLAG_GENERIC if generic else 0
    with mwu.densest_subgraph(g.num_vertices, g.u, g.v, precision=precision, flags=flags) as s:
        r = s.solve()
    assert r.certified
    assert r.lower <= best * (1 + 1e-9) and best <= r.upper * (1 + 1e-9)
    assert r.objective / best <= 1 + EPS
    z = r.x
    assert (z[0::2] + z[1::2]).min() >= 1 - 1e-9
    load = np.bincount(g.u, weights=z[0::2], minlength=16) + np.bincount(g.v, weights=z[1::2], minlength=16)
    assert load.max() == pytest.approx(r.objective, rel=1e-9)


@pytest.mark.parametrize("precision", [mwu.FP64, mwu.MIXED_FP32_FP64])
def test_solve_warm_start(precision):
    """Whole solves with the warm-started search: the vertex cover and the
    densest subgraph of the tests above, certified around the exact optima,
    and in FP64 within the oracle's warm-started result."""
    g = gg.rmat(13, 16, seed=2)
    opt = _opt_vcover(g)
    with mwu.vertex_cover(g.num_vertices, g.u, g.v, precision=precision,
                          step_rule=mwu.STEP_BIN_WARM) as s:
        r = s.solve()
    assert r.certified
    assert r.lower <= opt * (1 + 1e-12) and opt <= r.upper * (1 + 1e-12)
    assert r.objective / opt <= 1 + EPS
    assert (r.x[g.u] + r.x[g.v]).min() >= 1 - 1e-9 and r.x.min() >= 0
    if precision == mwu.FP64:
        ro = oracle.solve_vcover(g, step_rule=oracle.STEP_BIN_WARM)
        assert ro.certified and r.objective == pytest.approx(ro.objective, rel=EPS)
    gd = gg.gnm_random(16, 34, seed=5)
    best = 0.0
    for mask in range(1, 1 << 16):
        S = np.array([(mask >> i) & 1 for i in range(16)], bool)
        best = max(best, np.sum(S[gd.u] & S[gd.v]) / S.sum())
    with mwu.densest_subgraph(gd.num_vertices, gd.u, gd.v, precision=precision,
                              step_rule=mwu.STEP_BIN_WARM) as s:
        rd = s.solve()
    assert rd.certified
    assert rd.lower <= best * (1 + 1e-9) and best <= rd.upper * (1 + 1e-9)


def test_solve_weighted_packing():
    case = weighted_packing_case()
    from scipy.optimize import linprog
    lp = linprog(-case.c, A_ub=case.A, b_ub=case.b, bounds=(0, None))
    with case.make_gpu(precision=mwu.FP64) as s:
        r = s.solve()
    assert r.certified
    assert (case.A @ r.x <= case.b * (1 + 1e-9)).all()
    assert -lp.fun / (case.c @ r.x) <= 1 + EPS + 1e-9
    ro = oracle.solve_packing(case.P)
    assert ro.certified and r.objective == pytest.approx(ro.objective, rel=EPS)


def test_tiny_and_degenerate():
    # one edge: matching 1, vertex cover 1
    with mwu.bmatch(2, [0], [1], precision=mwu.FP64) as s:
        r = s.solve()
    assert r.certified and r.objective == pytest.approx(1.0, rel=0.1)
    with mwu.vertex_cover(5, [3], [1], precision=mwu.FP64) as s:
        r = s.solve()
    assert r.certified and 1.0 <= r.objective <= 1.1
    assert r.x[0] == r.x[2] == r.x[4] == 0.0
    # an infeasible fixed-lambda probe reports INFEASIBLE
    g = gg.complete_graph(6)
    with mwu.densest_subgraph(6, g.u, g.v, precision=mwu.FP64, fixed_lambda=1.0) as s:
        r = s.solve()
    assert r.status == mwu.INFEASIBLE
    with mwu.densest_subgraph(6, g.u, g.v, precision=mwu.FP64, fixed_lambda=4.0) as s:
        r = s.solve()
    # a feasible verdict: x covers every edge, its lambda (max vertex load) is
    # the reported objective, within (1 + eps) of the lambda asked for
    assert r.status == mwu.FEASIBLE_POINT and r.objective <= 4.0 * (1 + EPS)
    z = r.x
    assert (z[0::2] + z[1::2]).min() >= 1 - 1e-9
    load = np.bincount(g.u, weights=z[0::2], minlength=6) + np.bincount(g.v, weights=z[1::2], minlength=6)
    assert r.objective == pytest.approx(load.max(), rel=1e-9)


@pytest.mark.parametrize("step_rule", [mwu.STEP_BIN, mwu.STEP_BIN_WARM])
def test_deterministic_rerun(step_rule):
    g = gg.rmat(12, 8, seed=6)
    out = []
    for _ in range(2):
        with mwu.vertex_cover(g.num_vertices, g.u, g.v, step_rule=step_rule) as s:
            out.append(s.solve())
    assert out[0].objective == out[1].objective
    assert np.array_equal(out[0].x, out[1].x)
    assert out[0].total_iterations == out[1].total_iterations


def test_max_iter_and_standard_step():
    g = gg.bipartite_uniform(100, 100, 600, seed=7)
    with mwu.bmatch(g.num_vertices, g.u, g.v, precision=mwu.FP64, max_iter=1, max_probes=3) as s:
        r = s.solve()
    assert r.status == mwu.FEASIBLE_UNCERTIFIED
    case = bmatch_case(g, param=0.8 * _opt_bmatch(g))
    with case.make_gpu(precision=mwu.FP64, step_rule=mwu.STEP_STD, max_iter=100000) as s:
        s.probe_begin(case.param)
        info = s.probe_run(100000)
    ref = oracle.probe(case.P, 1.0, case.C, 1.0 / case.param, EPS, step_rule=oracle.STEP_STD,
                       max_iter=100000)
    assert info.status == ref.status and info.iterations == ref.iterations


# probes long enough to interrupt (FP64 oracle iteration counts: bmatch 134,
# vcover 180, domset 177, densest 53)
LONG_PROBES = {
    "bmatch": lambda: bmatch_case(gg.bipartite_uniform(700, 650, 9000, seed=21), param=630.0),
    "vcover": lambda: vcover_case(gg.gnm_random(900, 7000, seed=22), param=495.0),
    "domset": lambda: domset_case(gg.chung_lu(3000, 2.3, 8.0, seed=23), param=646.5),
    "densest": CASES["densest"],
}


@pytest.mark.parametrize("name", list(LONG_PROBES))
def test_probe_resumes_after_direction(name):
    """Running, forming the direction (and evaluating steps along it), then
    running again takes exactly the steps of an uninterrupted run (FP64)."""
    case = LONG_PROBES[name]()
    with case.make_gpu(precision=mwu.FP64) as s:
        s.probe_begin(case.param)
        ref = s.probe_run(5000)
        ref_alphas = s.probe_read("alpha", ref.iterations)
        assert ref.iterations > 20
        s.probe_begin(case.param)
        first = s.probe_run(7)
        assert first.status == mwu._lib.PROBE_RUNNING and first.iterations == 7
        s.probe_direction()
        s.probe_eval_steps(EXP_ALPHAS)
        info = s.probe_run(5000)
        alphas = s.probe_read("alpha", info.iterations)
    assert info.status == ref.status and info.iterations == ref.iterations
    assert np.array_equal(alphas, ref_alphas)


@pytest.mark.parametrize("name", list(LONG_PROBES))
def test_probe_continues_after_time_pass(name):
    """mwu_time_pass commits the pending step and times held launches; the
    probe then continues from the committed point and takes the steps an
    uninterrupted run takes from there (FP64; the LSE totals are renormalized
    by a row pass with no step, so the comparison covers the next 10 steps)."""
    case = LONG_PROBES[name]()
    with case.make_gpu(precision=mwu.FP64) as s:
        s.probe_begin(case.param)
        ref = s.probe_run(5000)
        ref_alphas = s.probe_read("alpha", ref.iterations)
        assert ref.iterations > 20
        s.probe_begin(case.param)
        s.probe_run(5)
        for which in (1, 2, 3, 4, 5, 0):
            s.time_pass(which, 2)
        info = s.probe_run(10)
        alphas = s.probe_read("alpha", info.iterations)
    assert info.iterations == 15
    assert np.array_equal(alphas, ref_alphas[:15])


# ------------------------------------------------------------------ probe-to-probe reuse (R21)

def _reuse_start(P, sP, x, eps=EPS):
    """The previous iterate scaled so that its largest packing row (values
    scaled by sP) is eps, as the oracle's outer search does."""
    y = np.zeros(P.rows)
    oracle.lib().orc_matvec(P.c, sP, np.ascontiguousarray(x).ctypes.data, y.ctypes.data)
    return x * (eps / y.max())


@pytest.mark.parametrize("name", ["vcover", "densest", "domset"])
def test_probe_from_reused_point_fp64(name):
    """A probe started from the previous probe's rescaled iterate (FP64).  At
    that point the direction, g and h match the oracle's to 1e-9; from it the
    GPU takes the oracle's first 16 steps exactly and ends with its verdict.
    Whole trajectories are compared for the densest probe only: the covering
    probes here run 160-170 iterations from a non-uniform start, and the
    oracle itself amplifies a 1e-13 perturbation of that start 1e11- to
    1e12-fold by their end (R13), so their late steps are not a kernel check."""
    case = LONG_PROBES[name]()
    p2 = case.param * (0.97 if name == "densest" else 1.03)
    sP2, sC2 = case.sP(p2), case.sC(p2)
    with case.make_gpu(precision=mwu.FP64) as s:
        n = s.sizes().n
        s.probe_begin(case.param)
        first = s.probe_run(5000)
        x_prev = s.probe_read("x", n)
        x0 = _reuse_start(case.P, sP2, x_prev)
        s.probe_begin(p2, x0)
        s.probe_direction()
        got = {k: s.probe_read(k, n) for k in ("g", "h", "d")}
        info = s.probe_run(5000)
        alphas = s.probe_read("alpha", info.iterations)
        xg = s.probe_read("x", n)
    ref = oracle.iteration_terms(case.P, sP2, case.C, sC2, EPS, x0)
    errs = {k: rel_err(got[k], ref[k]) for k in ("g", "h", "d")}
    free = oracle.probe(case.P, sP2, case.C, sC2, EPS, x0=x0)
    print(f"{name}: first probe {first.iterations} iterations; reused start {info.iterations} "
          f"(from the Algorithm 1 point: {oracle.probe(case.P, sP2, case.C, sC2, EPS).iterations}); {errs}")
    assert all(v <= FP64_TOL for v in errs.values()), errs
    assert info.iterations > 16 and np.array_equal(alphas[:16], free.alphas[:16])
    assert info.status == free.status
    if name == "densest":
        r = oracle.probe(case.P, sP2, case.C, sC2, EPS, x0=x0, forced_alpha=alphas)
        assert np.array_equal(alphas, free.alphas) and info.iterations == r.iterations
        assert abs(xg.sum() - r.x.sum()) <= 1e-9 * r.x.sum()


@pytest.mark.parametrize("precision", [mwu.FP64, mwu.MIXED_FP32_FP64])
def test_solve_with_reuse(precision):
    """Whole outer searches with MWU_FLAG_REUSE: certified brackets around the
    exact optima (vertex cover, dominating set, densest subgraph, matching)."""
    from scipy.optimize import linprog
    F = mwu._lib.FLAG_REUSE
    g = gg.rmat(13, 16, seed=2)
    opt = _opt_vcover(g)
    with mwu.vertex_cover(g.num_vertices, g.u, g.v, precision=precision, flags=F) as s:
        r = s.solve()
    assert r.certified and r.lower <= opt * (1 + 1e-12) and opt <= r.upper * (1 + 1e-12)
    pl = gg.chung_lu(400, 2.3, 6.0, seed=4)
    ptr, col = gg.adjacency_csr(pl, with_identity=True)
    D = oracle.dominating_set_matrix(pl).dense()
    dopt = linprog(np.ones(D.shape[1]), A_ub=-D, b_ub=-np.ones(D.shape[0]), bounds=(0, None)).fun
    with mwu.dominating_set(ptr, col, pl.num_vertices, precision=precision, flags=F) as s:
        rd = s.solve()
    assert rd.certified and rd.lower <= dopt * (1 + 1e-9) and dopt <= rd.upper * (1 + 1e-9)
    gd = gg.gnm_random(16, 34, seed=5)
    best = 0.0
    for mask in range(1, 1 << 16):
        S = np.array([(mask >> i) & 1 for i in range(16)], bool)
        best = max(best, np.sum(S[gd.u] & S[gd.v]) / S.sum())
    with mwu.densest_subgraph(gd.num_vertices, gd.u, gd.v, precision=precision, flags=F) as s:
        rn = s.solve()
    assert rn.certified and rn.lower <= best * (1 + 1e-9) and best <= rn.upper * (1 + 1e-9)
    b = gg.bipartite_uniform(2000, 2000, 20000, seed=1)
    bopt = _opt_bmatch(b)
    with mwu.bmatch(b.num_vertices, b.u, b.v, precision=precision, flags=F) as s:
        rb = s.solve()
    assert rb.certified and rb.lower <= bopt <= rb.upper * (1 + 1e-12)
    print(f"reuse precision {precision}: vcover {r.probes} probes {r.total_iterations} iterations; "
          f"domset {rd.probes}/{rd.total_iterations}; densest {rn.probes}/{rn.total_iterations}; "
          f"bmatch {rb.probes}/{rb.total_iterations}")
