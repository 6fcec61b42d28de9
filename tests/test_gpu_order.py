"""The generic engine's internal locality order (MWU_FLAG_LOCALITY_ORDER:
columns by number of nonzeros, rows of each side likewise, both descending)
against the CPU oracle and against the caller's order (MWU_FLAG_KEEP_ORDER),
through the C ABI.  Every vector is read back, and every given vector taken,
in the caller's order.

  per pass    forced on, every generic-engine case of the parity tests: x,
              d, g, h, y, z, Pd, Cd and Psi, Phi, min z' at a random start
              point within 1e-9 of the oracle in FP64; in the chosen form no
              error beyond that of the caller's order at the same point.
  objective   the mixed optimization's embedded row in both senses (on the
              packing side it enters the column maxima of the start point)
              per pass at a given level, FP64 within 1e-9.
  potential   value and gradient for x given, and the gradient written, in
              the caller's order (mapped on the device), equal to the
              caller's-order engine's to 1e-12 in FP64, through the
              allocating and the no-allocation entry points.
  solves      whole solves with the order on and off, both certified around
              the exact optimum.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import graphgen as gg
import oracle
import paper_2307_03307_amd as mwu

from gpu_common import EPS, rel_err
from test_gpu_parity import CASES, FP64_TOL, MIXED_TOL, MIXED_TOL_CASE, U, _per_pass

pytestmark = pytest.mark.gpu

LOC = mwu._lib.FLAG_LOCALITY_ORDER
KEEP = mwu._lib.FLAG_KEEP_ORDER
GENERIC_CASES = ["bmatch", "gmatch", "vcover-generic", "domset", "domset-star", "densest-generic", "weighted"]


def _with_flags(case, flags):
    make = case.make_gpu
    case.make_gpu = lambda **kw: make(**dict(kw, flags=kw.get("flags", 0) | flags))
    return case


@pytest.mark.parametrize("precision", [mwu.FP64, mwu.MIXED_FP32_FP64])
@pytest.mark.parametrize("name", GENERIC_CASES)
def test_per_pass_in_locality_order(name, precision):
    """FP64: the oracle's values within 1e-9.  Chosen form: the order adds
    no error of its own -- each quantity within the per-quantity bound of
    the parity tests, or within twice (plus 4 U) its error in the caller's
    order at the same point (the FP32 sums only change their order).  The
    densest LP on the generic engine leaves d = 0 where both FP32 weights
    underflow, in either order (reported, not bounded)."""
    if precision == mwu.FP64:
        _per_pass(_with_flags(CASES[name](), LOC), precision, FP64_TOL)
        return
    direction = name != "densest-generic"
    loc = _per_pass(_with_flags(CASES[name](), LOC), precision, math.inf, direction=direction)
    keep = _per_pass(_with_flags(CASES[name](), KEEP), precision, math.inf, direction=direction)
    tol = MIXED_TOL_CASE.get(name, MIXED_TOL)
    bad = {k: (v, keep[k]) for k, v in loc.items() if not (v <= tol[k] or v <= 2 * keep[k] + 4 * U)}
    assert not bad, bad


def _lp(seed, n=300, mP=120, mC=80, dens=0.03):
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
    # a few long columns and rows, so that the order moves them
    for j in rng.choice(n, 4, replace=False):
        for i in rng.choice(mP, mP // 2, replace=False):
            P[i, j] = 1.5
    return P.tocsr(), C.tocsr()


def _ocsr(A):
    A = sp.csr_matrix(A)
    return oracle.CSR(A.shape[0], A.shape[1], A.indptr.astype(np.int64), A.indices.astype(np.int32),
                      A.data.astype(np.float64))


@pytest.mark.parametrize("maximize", [True, False])
def test_objective_row_in_locality_order(maximize):
    P, C = _lp(6)
    n = P.shape[1]
    M = 40.0 if maximize else 6.0
    obj = sp.csr_matrix(np.full((1, n), 1.0 / M))
    Pp, Cp = (P, sp.vstack([C, obj])) if maximize else (sp.vstack([P, obj]), C)
    Po, Co = _ocsr(Pp), _ocsr(Cp)
    x0 = np.zeros(n)
    oracle.lib().orc_initial_point(Po.c, 1.0, EPS, x0.ctypes.data)
    ref = oracle.iteration_terms(Po, 1.0, Co, 1.0, EPS, x0, alphas=[1.0, 4.0, 32.0])
    Pm = mwu.csr_matrix(P.indptr, P.indices, P.data, shape=P.shape)
    Cm = mwu.csr_matrix(C.indptr, C.indices, C.data, shape=C.shape)
    form = mwu.MIXED_MAX if maximize else mwu.MIXED_MIN
    with mwu.Solver(form, P=Pm, C=Cm, c=np.ones(n), precision=mwu.FP64, flags=LOC) as s:
        sz = s.sizes()
        s.probe_begin(M)
        s.probe_direction()
        got = {k: s.probe_read(k, m) for k, m in (("x", n), ("g", n), ("h", n), ("d", n), ("y", sz.m_P),
                                                   ("z", sz.m_C), ("dy", sz.m_P), ("dz", sz.m_C))}
        psi, phi, _ = s.probe_eval_steps([1.0, 4.0, 32.0])
    errs = {k: rel_err(got[k], ref[k]) for k in ("g", "h", "d", "y", "z", "dy", "dz")}
    errs["x"] = rel_err(got["x"], x0)
    errs["psi"] = rel_err(psi, ref["psi"])
    errs["phi"] = rel_err(phi, ref["phi"])
    print(f"objective row in locality order ({'max' if maximize else 'min'}): "
          + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    assert all(v <= 1e-9 for v in errs.values()), errs


def test_potential_in_callers_order():
    import torch
    g = gg.chung_lu(20000, 2.1, 8.0, seed=43)
    ptr, col = gg.adjacency_csr(g, with_identity=True)
    n = g.num_vertices
    x = np.random.default_rng(5).uniform(0.02, 0.12, n)
    out = {}
    for tag, flags in (("keep", KEEP), ("locality", LOC)):
        with mwu.dominating_set(ptr, col, n, precision=mwu.FP64, flags=flags) as s:
            s.probe_begin(0.05 * n)
            xt = torch.tensor(x, dtype=torch.float64, device="cuda")
            ga = torch.zeros(n, dtype=torch.float64, device="cuda")
            gb = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
            v = s.potential_forward(xt.data_ptr())
            s.potential_backward(xt.data_ptr(), 1.5, ga.data_ptr())
            vb = s.potential_backward_noalloc(xt.data_ptr(), 1.5, gb.data_ptr())
            torch.cuda.synchronize()
            out[tag] = (v, vb, ga.cpu().numpy(), gb.cpu().numpy())
    (v0, vb0, a0, b0), (v1, vb1, a1, b1) = out["keep"], out["locality"]
    errs = (rel_err(a1, a0), rel_err(b1, a0), abs(v1 - v0) / abs(v0), abs(vb1 - v0) / abs(v0))
    print(f"potential, locality against caller's order: gradient {errs[0]:.2e} (no-alloc {errs[1]:.2e}), "
          f"value {errs[2]:.2e} (no-alloc {errs[3]:.2e})")
    assert np.all(np.isfinite(b1)) and max(errs) <= 1e-12


@pytest.mark.parametrize("precision", [mwu.FP64, mwu.MIXED_FP32_FP64])
def test_solves_in_both_orders(precision):
    from scipy.optimize import linprog
    g = gg.chung_lu(1500, 2.2, 6.0, seed=44)
    ptr, col = gg.adjacency_csr(g, with_identity=True)
    D = oracle.dominating_set_matrix(g).dense()
    opt = linprog(np.ones(D.shape[1]), A_ub=-D, b_ub=-np.ones(D.shape[0]), bounds=(0, None)).fun
    res = {}
    for tag, flags in (("keep", KEEP), ("locality", LOC)):
        with mwu.dominating_set(ptr, col, g.num_vertices, precision=precision, flags=flags) as s:
            r = s.solve()
        cover = D @ r.x
        print(f"{tag} order, precision {precision}: bracket [{r.lower:.6g}, {r.upper:.6g}] (OPT {opt:.6g}), "
              f"{r.probes} probes, {r.total_iterations} iterations")
        assert r.certified and r.lower <= opt * (1 + 1e-9) and opt <= r.upper * (1 + 1e-9), tag
        assert cover.min() >= 1 - 1e-9 and r.x.min() >= 0
        res[tag] = r
