"""Newton step search (MWU_STEP_NEWTON, Section 4.2, reading R20) against the
CPU oracle, through the C ABI.

  Newton pass   at the same x and direction: Psi, Phi and the derivatives
                Psi', Phi' at chosen steps, including steps whose packing
                exponent is past the direct form (the FP64 program refines
                them in two exact passes, the chosen form max-shifts them).
                FP64 within 1e-9; chosen form in units of 2^-24.
  free run      FP64: the GPU's first 16 steps and their test counts equal
                the oracle's Newton search; later steps are checked with the
                oracle forced to the GPU's earlier steps (the MWU map
                amplifies last-bit differences over a long probe, R13).
  solves        certified brackets around exact optima in both precisions,
                on the fused programs, the generic engine and the batch.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2307_03307_amd as mwu

from gpu_common import EPS, rel_err, start_point, vcover_case
from test_gpu_parity import CASES, LONG_PROBES, _opt_bmatch, _opt_vcover

pytestmark = pytest.mark.gpu

NEWTON = mwu.STEP_NEWTON
U = 2.0 ** -24
# Chosen form: Psi' is a weighted mean of Pd, formed from FP32 terms
# w dy e^{eta a dy} over FP32 direction products (errors up to 32 U of
# max |Pd| in the per-pass tests; Cd 64 U).  An error delta of Pd moves each
# exponent by eta a delta, so the log-weights of the mean carry errors up to
# B = eta a max |Pd| times 32 U, and the mean moves by at most that times
# max |Pd|.  Psi' is held to 64 U (1 + B_P) max |Pd| and Phi' to
# 128 U (1 + B_C) max |Cd| (the errors below are reported in units of
# (1 + B) max |Pd| and (1 + B) max |Cd|).  FP64: relative to the value.
MIXED_DTOL = {"psi": 24 * U, "phi": 12 * U, "dpsi": 64 * U, "dphi": 128 * U}


def _newton_pass(case, precision):
    x0 = start_point(case, 0)
    sP, sC = case.sP(case.param), case.sC(case.param)
    ref0 = oracle.iteration_terms(case.P, sP, case.C, sC, EPS, x0)
    eta = ref0["eta"]
    # 1, a middle step, and one whose packing exponent eta a max(Pd) is 1.5x
    # the FP64 direct-form limit of 700 (refined) where Pd has a nonzero entry
    dymax = float(np.max(ref0["dy"]))
    alphas = [1.0, 37.5]
    if dymax > 0:
        alphas.append(1050.0 / (eta * dymax))
    ref = oracle.iteration_terms(case.P, sP, case.C, sC, EPS, x0, alphas=alphas)
    got = []
    with case.make_gpu(precision=precision, step_rule=NEWTON) as s:
        s.probe_begin(case.param, x0)
        s.probe_direction()
        for a in alphas:
            got.append(s.probe_eval_newton(a))
    errs = {"psi": 0.0, "phi": 0.0, "dpsi": 0.0, "dphi": 0.0}
    mixed = precision == mwu.MIXED_FP32_FP64
    for k, a in enumerate(alphas):
        dps, dph = oracle.step_derivatives(ref["y"], ref["dy"], ref["z"], ref["dz"], eta, a)
        psi, phi = ref["psi"][k], ref["phi"][k]
        # the mixed form's Psi, Phi are held to the scale of the test Phi >= Psi
        vscale = max(abs(psi), abs(phi)) if mixed else None
        mdy, mdz = float(np.max(np.abs(ref["dy"]))), float(np.max(np.abs(ref["dz"])))
        dscale = {"dpsi": (1.0 + eta * a * mdy) * mdy, "dphi": (1.0 + eta * a * mdz) * mdz}
        for name, g, r in (("psi", got[k][0], psi), ("phi", got[k][1], phi),
                           ("dpsi", got[k][2], dps), ("dphi", got[k][3], dph)):
            if not mixed:
                sc = abs(r)
            else:
                sc = dscale[name] if name in dscale else vscale
            e = abs(g - r) / max(sc, 1e-300)
            print(f"  a={a:.6g} {name}: gpu {g:.12e} oracle {r:.12e} err {e:.2e}")
            errs[name] = max(errs[name], e)
    print(f"Newton pass {case.name} precision {precision} alphas {[f'{a:.4g}' for a in alphas]}: "
          + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    return errs


@pytest.mark.parametrize("name", ["bmatch", "vcover", "vcover-star", "domset", "densest", "densest-generic",
                                  "densest-powerlaw", "weighted"])
def test_newton_pass_fp64(name):
    errs = _newton_pass(CASES[name](), mwu.FP64)
    assert all(v <= 1e-9 for v in errs.values()), errs


@pytest.mark.parametrize("name", ["bmatch", "vcover", "domset", "densest", "densest-powerlaw", "weighted"])
def test_newton_pass_mixed(name):
    errs = _newton_pass(CASES[name](), mwu.MIXED_FP32_FP64)
    bad = {k: v for k, v in errs.items() if not v <= MIXED_DTOL[k]}
    assert not bad, bad


@pytest.mark.parametrize("name", list(LONG_PROBES) + ["densest-generic", "weighted"])
def test_newton_probe_follows_oracle_fp64(name):
    """FP64 free run with the Newton search.  The first 16 steps equal the
    oracle's to 1e-8 with the same number of tests (Newton iterates are not
    dyadic values: last-bit differences of Psi and Phi reach them, and the
    MWU map amplifies them from step to step, R13).  At sampled later
    iterations k the oracle is handed the GPU's own iterate x_k and last step
    and takes one Newton search from there: same step to 1e-9, same number
    of tests, and the same next iterate x_(k+1) to 1e-9.  Same verdict as
    the free oracle.  Whole trajectories are not compared: these probes sit
    near the optimum, where even the oracle forced to the GPU's steps drifts
    from the GPU's iterate by a percent within 110 iterations (the forced
    map has no step search to damp the amplification of R13), and the
    iteration at which min Cx crosses 1 moves with it."""
    case = CASES[name]() if name in CASES and name not in LONG_PROBES else LONG_PROBES[name]()
    sP, sC = case.sP(case.param), case.sC(case.param)
    with case.make_gpu(precision=mwu.FP64, step_rule=NEWTON) as s:
        n = s.sizes().n
        s.probe_begin(case.param)
        info = s.probe_run(5000)
        alphas = s.probe_read("alpha", info.iterations)
        # the same probe again, stopped at sampled iterations (stopping, forming
        # the direction and resuming does not change the steps taken)
        ks = sorted(set(int(k) for k in np.linspace(16, info.iterations - 2, 6) if 1 <= k < info.iterations - 1))
        states = []
        s.probe_begin(case.param)
        head = s.probe_run(16)
        head_alphas = s.probe_read("alpha", head.iterations)
        done, prev = head.iterations, head
        for k in ks:
            if k > done:
                prev = s.probe_run(k - done)
            if prev.iterations != k:
                break
            s.probe_direction()
            xk = s.probe_read("x", n)
            nxt = s.probe_run(1)
            a_k = s.probe_read("alpha", nxt.iterations)[k]
            s.probe_direction()                      # applies step k+1
            states.append((k, xk, a_k, nxt.evaluations - prev.evaluations, s.probe_read("x", n)))
            done, prev = nxt.iterations, nxt
    ref16 = oracle.probe(case.P, sP, case.C, sC, EPS, step_rule=oracle.STEP_NEWTON, max_iter=16)
    free = oracle.probe(case.P, sP, case.C, sC, EPS, step_rule=oracle.STEP_NEWTON)
    bin3 = oracle.probe(case.P, sP, case.C, sC, EPS)
    print(f"{name}: Newton {info.iterations} iterations, {info.search_passes} passes, "
          f"{info.evaluations} tests (oracle {free.iterations} / {free.evaluations}); "
          f"Algorithm 3: {bin3.iterations} iterations, {bin3.evaluations} tests")
    assert head.iterations == ref16.iterations
    assert np.allclose(head_alphas, ref16.alphas, rtol=1e-8, atol=0)
    assert head.evaluations == ref16.evaluations
    assert info.status == free.status
    assert len(states) == len(ks)
    for k, xk, a_gpu, ev_gpu, xk1 in states:
        assert np.array_equal(alphas[k], a_gpu)          # the resumed run took the same step
        r = oracle.probe(case.P, sP, case.C, sC, EPS, step_rule=oracle.STEP_NEWTON, x0=xk,
                         start_alpha=alphas[k - 1], max_iter=1)
        print(f"  iteration {k}: GPU step {a_gpu:.12g} ({ev_gpu} tests), oracle from x_k {r.alphas[0]:.12g} "
              f"({r.evaluations} tests); x_(k+1) {rel_err(xk1, r.x):.1e}")
        assert abs(r.alphas[0] - a_gpu) <= 1e-9 * a_gpu and r.evaluations == ev_gpu, k
        assert rel_err(xk1, r.x) <= 1e-9, k


@pytest.mark.parametrize("precision", [mwu.FP64, mwu.MIXED_FP32_FP64])
def test_newton_solves_bracket_exact_optima(precision):
    """Whole outer searches with the Newton step on the fused programs and the
    generic engine, with and without probe-to-probe reuse: certified brackets
    around exact optima, and fewer step tests per iteration than Algorithm 3
    (Table 2's Nwt and Bin columns)."""
    from scipy.optimize import linprog
    g = gg.rmat(13, 16, seed=2)
    opt = _opt_vcover(g)
    for flags in (0, mwu._lib.FLAG_GENERIC, mwu._lib.FLAG_REUSE):
        with mwu.vertex_cover(g.num_vertices, g.u, g.v, precision=precision, flags=flags,
                              step_rule=NEWTON) as s:
            r = s.solve()
        assert r.certified and r.lower <= opt * (1 + 1e-12) and opt <= r.upper * (1 + 1e-12), flags
    with mwu.vertex_cover(g.num_vertices, g.u, g.v, precision=precision) as s:
        rb = s.solve()
    print(f"vcover rmat13 precision {precision}: Newton {r.total_iterations} iterations "
          f"{r.evaluations / r.total_iterations:.2f} tests/iteration; Bin {rb.total_iterations} "
          f"{rb.evaluations / rb.total_iterations:.2f}")
    assert r.evaluations / r.total_iterations < rb.evaluations / rb.total_iterations
    pl = gg.chung_lu(400, 2.3, 6.0, seed=4)
    ptr, col = gg.adjacency_csr(pl, with_identity=True)
    D = oracle.dominating_set_matrix(pl).dense()
    dopt = linprog(np.ones(D.shape[1]), A_ub=-D, b_ub=-np.ones(D.shape[0]), bounds=(0, None)).fun
    with mwu.dominating_set(ptr, col, pl.num_vertices, precision=precision, step_rule=NEWTON) as s:
        rd = s.solve()
    assert rd.certified and rd.lower <= dopt * (1 + 1e-9) and dopt <= rd.upper * (1 + 1e-9)
    gd = gg.gnm_random(16, 34, seed=5)
    best = 0.0
    for mask in range(1, 1 << 16):
        S = np.array([(mask >> i) & 1 for i in range(16)], bool)
        best = max(best, np.sum(S[gd.u] & S[gd.v]) / S.sum())
    for flags in (0, mwu._lib.FLAG_GENERIC):
        with mwu.densest_subgraph(gd.num_vertices, gd.u, gd.v, precision=precision, flags=flags,
                                  step_rule=NEWTON) as s:
            rn = s.solve()
        assert rn.certified and rn.lower <= best * (1 + 1e-9) and best <= rn.upper * (1 + 1e-9), flags
    b = gg.bipartite_uniform(2000, 2000, 20000, seed=1)
    bopt = _opt_bmatch(b)
    with mwu.bmatch(b.num_vertices, b.u, b.v, precision=precision, step_rule=NEWTON) as s:
        rm = s.solve()
    assert rm.certified and rm.lower <= bopt <= rm.upper * (1 + 1e-12)


@pytest.mark.parametrize("precision", [mwu.FP64, mwu.MIXED_FP32_FP64])
def test_newton_batch_matches_exact_optimum(precision):
    """The batched kernels run the same Newton replay: every instance ends
    certified around its exact matching number."""
    from test_gpu_batch import _check, _instances, _nu
    gs = _instances()
    with mwu.BatchSolver([(g.num_vertices, g.u, g.v) for g in gs], precision=precision,
                         step_rule=NEWTON) as b:
        res = b.solve()
    for g, r in zip(gs, res):
        _check(g, r, _nu(g))


def test_newton_batch_probes_follow_oracle_fp64():
    """FP64 batched probes with the Newton search: each instance's first 16
    steps and final verdict are the oracle's.  The steps are held to 1e-6:
    batched probes cannot be stopped and handed to the oracle mid-way, and
    near-optimum instances amplify last-bit differences to ~1e-8 within 16
    Newton steps (R13)."""
    from test_gpu_batch import _instances, _oracle_mats, _probe_params
    gs = _instances()
    params = _probe_params(gs)
    with mwu.BatchSolver([(g.num_vertices, g.u, g.v) for g in gs], precision=mwu.FP64, tune=False,
                         step_rule=NEWTON) as b:
        infos = b.probe_run(params)
        got = [b.probe_read(k, "alpha", infos[k].iterations) for k in range(len(gs))]
    for k, g in enumerate(gs):
        P, C = _oracle_mats(g)
        r = oracle.probe(P, 1.0, C, 1.0 / params[k], EPS, step_rule=oracle.STEP_NEWTON)
        assert infos[k].status == r.status, k
        m = min(16, r.iterations)
        d = np.max(np.abs(got[k][:m] - r.alphas[:m]) / r.alphas[:m]) if m else 0.0
        print(f"instance {k}: {infos[k].iterations} iterations (oracle {r.iterations}), "
              f"first {m} steps within {d:.1e}")
        assert len(got[k]) >= m and d <= 1e-6, k
