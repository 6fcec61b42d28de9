"""Dropping satisfied covering rows (MWU_FLAG_DROP_SATISFIED; the line
C <- {c_i : c_i^T x < 1} of Algorithms 1 and 2, reading R22) against the
CPU oracle, through the C ABI.

  per pass    at a point where part of the covering rows is met: y, z, g, h,
              d, Pd, Cd and Psi, Phi, min z' of the oracle's iteration with
              the met rows left out.  FP64 within 1e-9; the chosen form adds
              no error to that of the same point with the rows kept.
  free run    FP64 near-optimum probes: the GPU takes the dropping oracle's
              first steps exactly (the steps of Algorithm 3 are dyadic
              values) and reaches the same verdict.
  solves      certified brackets around exact optima in both precisions,
              on the fused programs and the generic engine.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2307_03307_amd as mwu

from gpu_common import (EPS, densest_case, domset_case, rel_err, start_point, vcover_case)
from test_gpu_parity import MIXED_TOL, U, _opt_vcover

pytestmark = pytest.mark.gpu

DROP = mwu._lib.FLAG_DROP_SATISFIED


def _with_drop(case):
    """The same case with the flag set on the GPU side (make_plain: without)."""
    make = case.make_gpu
    case.make_plain = make
    case.make_gpu = lambda **kw: make(**dict(kw, flags=kw.get("flags", 0) | DROP))
    return case


# near-optimum probes (long enough for rows to be met before the end)
LONG = {
    "vcover": lambda: vcover_case(gg.gnm_random(900, 7000, seed=22), param=495.0),
    "vcover-generic": lambda: vcover_case(gg.gnm_random(900, 7000, seed=22), param=495.0, generic=True),
    "domset": lambda: domset_case(gg.chung_lu(3000, 2.3, 8.0, seed=23), param=646.5),
    "densest": lambda: densest_case(gg.gnm_random(400, 3000, seed=24)),
    "densest-generic": lambda: densest_case(gg.gnm_random(400, 3000, seed=24), generic=True),
}

CASES = {
    "vcover": lambda: vcover_case(gg.gnm_random(900, 7000, seed=22)),
    "vcover-generic": lambda: vcover_case(gg.gnm_random(900, 7000, seed=22), generic=True),
    "domset": lambda: domset_case(gg.chung_lu(3000, 2.3, 8.0, seed=23)),
    "densest": lambda: densest_case(gg.gnm_random(400, 3000, seed=24)),
    "densest-generic": lambda: densest_case(gg.gnm_random(400, 3000, seed=24), generic=True),
}


def _half_met_point(case):
    """A positive point whose covering rows are half met (median z = 1)."""
    x = start_point(case, 3)
    sC = case.sC(case.param)
    z = np.zeros(case.C.rows)
    oracle.lib().orc_matvec(case.C.c, sC, x.ctypes.data, z.ctypes.data)
    return x / np.median(z)


def _pass_errors(case, precision, x0, drop, alphas):
    sP, sC = case.sP(case.param), case.sC(case.param)
    ref = oracle.iteration_terms(case.P, sP, case.C, sC, EPS, x0, alphas=alphas, drop=drop)
    make = case.make_gpu if drop else case.make_plain
    with make(precision=precision) as s:
        sz = s.sizes()
        s.probe_begin(case.param, x0)
        s.probe_direction()
        got = {k: s.probe_read(k, n) for k, n in
               (("d", sz.n), ("g", sz.n), ("h", sz.n), ("y", sz.m_P), ("z", sz.m_C), ("dy", sz.m_P),
                ("dz", sz.m_C))}
        psi, phi, zm = s.probe_eval_steps(alphas)
    errs = {k: rel_err(got[k], ref[k]) for k in got}
    for nm, a, b, other in (("psi", psi, ref["psi"], ref["phi"]), ("phi", phi, ref["phi"], ref["psi"])):
        scale = np.abs(b) if precision == mwu.FP64 else np.maximum(np.abs(b), np.abs(other))
        errs[nm] = float(np.max(np.abs(a - b) / np.maximum(scale, 1e-300)))
    errs["zmin"] = rel_err(zm, ref["zmin_new"])
    return errs, got, ref


@pytest.mark.parametrize("precision", [mwu.FP64, mwu.MIXED_FP32_FP64])
@pytest.mark.parametrize("name", list(CASES))
def test_per_pass_with_met_rows_left_out(name, precision):
    """FP64: every quantity within 1e-9 of the dropping oracle's.  Chosen
    form: dropping adds no error of its own -- at the same point each
    quantity is within twice (plus 4 U) the chosen form's error without
    dropping, or within the per-pass bound of the other tests (the half-met
    point here has larger row values than those tests' points, and the
    weights carry eta times their rounding).  The generic engine's FP32
    direction on the densest LP is reported, not bounded (d = 0 where both
    FP32 weights underflow, as in the tests without dropping)."""
    case = _with_drop(CASES[name]())
    x0 = _half_met_point(case)
    alphas = [1.0, 3.5, 11.0, 70.0]
    errs, got, ref = _pass_errors(case, precision, x0, True, alphas)
    met = ref["z"] >= 1.0
    assert 0.3 < met.mean() < 0.7
    # the met rows carry no weight: the variables all of whose rows are met
    # get h = 0 and no step on both sides
    gone = ref["h"] == 0.0
    print(f"drop per-pass {name} precision {precision}: {met.mean():.0%} rows met, {gone.sum()} variables "
          f"without h; " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    assert gone.sum() > 0 and np.all(got["d"][gone] == 0.0)
    if precision == mwu.FP64:
        bad = {k: v for k, v in errs.items() if not v <= 1e-9}
    else:
        base, _, _ = _pass_errors(case, precision, x0, False, alphas)
        print("  same point, rows kept: " + ", ".join(f"{k} {v:.2e}" for k, v in base.items()))
        skip = ("d", "dy", "dz", "psi", "phi", "zmin") if name == "densest-generic" else ()
        bad = {k: v for k, v in errs.items()
               if k not in skip and not (v <= MIXED_TOL[k] or v <= 2 * base[k] + 4 * U)}
    assert not bad, bad


@pytest.mark.parametrize("name", list(LONG))
def test_drop_probe_follows_oracle_fp64(name):
    """FP64 free run of a near-optimum probe with the met rows dropped: the
    GPU takes the dropping oracle's first 16 steps exactly (dyadic values of
    Algorithm 3) and reaches its verdict; where the whole run matches, so
    do the number of tests and the iterate's objective (1e-9).  Longer
    near-optimum probes amplify last-bit differences (R13)."""
    case = _with_drop(LONG[name]())
    sP, sC = case.sP(case.param), case.sC(case.param)
    with case.make_gpu(precision=mwu.FP64) as s:
        s.probe_begin(case.param)
        info = s.probe_run(5000)
        alphas = s.probe_read("alpha", info.iterations)
        xg = s.probe_read("x", s.sizes().n)
    free = oracle.probe(case.P, sP, case.C, sC, EPS, drop=True)
    kept = oracle.probe(case.P, sP, case.C, sC, EPS)
    same = info.iterations == free.iterations and np.array_equal(alphas, free.alphas)
    print(f"{name}: drop {info.iterations} iterations (oracle {free.iterations}, whole run "
          f"{'equal' if same else 'differs'}), keeping the rows {kept.iterations}")
    assert info.status == free.status
    m = min(16, free.iterations)
    assert info.iterations >= m and np.array_equal(alphas[:m], free.alphas[:m])
    if same:
        assert info.evaluations == free.evaluations
        assert abs(xg.sum() - free.x.sum()) <= 1e-9 * free.x.sum()


@pytest.mark.parametrize("precision", [mwu.FP64, mwu.MIXED_FP32_FP64])
def test_drop_solves_bracket_exact_optima(precision):
    """Whole outer searches with the met rows dropped, on the fused programs
    and the generic engine: certified brackets around the exact optima."""
    from scipy.optimize import linprog
    g = gg.rmat(13, 16, seed=2)
    opt = _opt_vcover(g)
    for flags in (DROP, DROP | mwu._lib.FLAG_GENERIC):
        with mwu.vertex_cover(g.num_vertices, g.u, g.v, precision=precision, flags=flags) as s:
            r = s.solve()
        assert r.certified and r.lower <= opt * (1 + 1e-12) and opt <= r.upper * (1 + 1e-12), flags
        cover = r.x[g.u] + r.x[g.v]
        assert cover.min() >= 1 - 1e-9
    pl = gg.chung_lu(400, 2.3, 6.0, seed=4)
    ptr, col = gg.adjacency_csr(pl, with_identity=True)
    D = oracle.dominating_set_matrix(pl).dense()
    dopt = linprog(np.ones(D.shape[1]), A_ub=-D, b_ub=-np.ones(D.shape[0]), bounds=(0, None)).fun
    with mwu.dominating_set(ptr, col, pl.num_vertices, precision=precision, flags=DROP) as s:
        rd = s.solve()
    assert rd.certified and rd.lower <= dopt * (1 + 1e-9) and dopt <= rd.upper * (1 + 1e-9)
    gd = gg.gnm_random(16, 34, seed=5)
    best = 0.0
    for mask in range(1, 1 << 16):
        S = np.array([(mask >> i) & 1 for i in range(16)], bool)
        best = max(best, np.sum(S[gd.u] & S[gd.v]) / S.sum())
    for flags in (DROP, DROP | mwu._lib.FLAG_GENERIC):
        with mwu.densest_subgraph(gd.num_vertices, gd.u, gd.v, precision=precision, flags=flags) as s:
            rn = s.solve()
        assert rn.certified and rn.lower <= best * (1 + 1e-9) and best <= rn.upper * (1 + 1e-9), flags
