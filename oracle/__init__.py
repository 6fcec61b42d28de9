"""Plain FP64 CPU oracle for the MWU positive-LP solver (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports it and
shares no code with it; the two meet only through the seeded inputs of
``graphgen``.

The C part (``mwu_oracle.c``) implements the iteration, Algorithm 3 and the
outer searches on explicit CSR matrices.  This module builds those explicit
matrices straight from the definitions in Section 3 of the paper:

* vertex-edge incidence M (n x m): M[u, e] = 1 iff u is an endpoint of e;
* dominating set: I + A;
* vertex cover: M^T;
* densest subgraph: interweaved identity W (m x 2m) with W[e, 2e] =
  W[e, 2e+1] = 1, and vertex-edge pair matrix O (n x 2m) with O[u, 2e] = 1
  for e = (u, .) and O[v, 2e+1] = 1 for e = (., v).

General LPs  max c^T x s.t. A x <= b  are normalized as P = A / (b c^T)
(Section 2.1) with x' = c * x.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mwu_oracle.c")
_LIB = os.path.join(_HERE, "libmwu_oracle.so")

STATUS_NAMES = {0: "RUNNING", 1: "FEASIBLE", 2: "INFEASIBLE", 3: "MAX_ITER"}
FEASIBLE, INFEASIBLE, MAX_ITER = 1, 2, 3
STEP_STD, STEP_BIN, STEP_BIN_WARM, STEP_NEWTON = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no OpenMP, no intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Mat(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("ptr", ctypes.c_void_p), ("idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class _ProbeResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int64),
                ("evaluations", ctypes.c_int64), ("pack_bound", ctypes.c_double),
                ("cover_bound", ctypes.c_double), ("last_alpha", ctypes.c_double),
                ("max_violation", ctypes.c_double)]


class _SolveResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("objective", ctypes.c_double),
                ("lower", ctypes.c_double), ("upper", ctypes.c_double),
                ("probes", ctypes.c_int64), ("total_iterations", ctypes.c_int64),
                ("final_probe_iterations", ctypes.c_int64), ("evaluations", ctypes.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        L.orc_probe.argtypes = [P(_Mat), ctypes.c_double, P(_Mat), ctypes.c_double, ctypes.c_double,
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, ctypes.c_int64,
                                vp, ctypes.c_int64, P(_ProbeResult)]
        L.orc_probe_from.argtypes = [P(_Mat), ctypes.c_double, P(_Mat), ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, ctypes.c_int64,
                                     vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, P(_ProbeResult)]
        L.orc_iteration_terms.argtypes = [P(_Mat), ctypes.c_double, P(_Mat), ctypes.c_double,
                                          ctypes.c_double, vp] + [vp] * 9 + [vp, vp, vp,
                                                                             ctypes.c_int64, vp, vp, vp,
                                                                             ctypes.c_int32, ctypes.c_double]
        for name in ("orc_solve_packing", "orc_solve_covering"):
            getattr(L, name).argtypes = [P(_Mat), ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, vp, P(_SolveResult)]
        L.orc_solve_densest.argtypes = [P(_Mat), P(_Mat), vp, vp, ctypes.c_double, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, P(_SolveResult)]
        L.orc_solve_mixed_opt.argtypes = [P(_Mat), P(_Mat), vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp,
                                          P(_SolveResult)]
        L.orc_smax.argtypes = [vp, ctypes.c_int64, ctypes.c_double, vp]
        L.orc_smax.restype = ctypes.c_double
        L.orc_smin.argtypes = [vp, ctypes.c_int64, ctypes.c_double, vp]
        L.orc_smin.restype = ctypes.c_double
        L.orc_psi.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double]
        L.orc_psi.restype = ctypes.c_double
        L.orc_phi.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, vp]
        L.orc_phi.restype = ctypes.c_double
        L.orc_eta.argtypes = [ctypes.c_int64, ctypes.c_double]
        L.orc_eta.restype = ctypes.c_double
        L.orc_level_set_density.argtypes = [ctypes.c_int64, ctypes.c_int64, vp, vp, vp]
        L.orc_level_set_density.restype = ctypes.c_double
        L.orc_matvec.argtypes = [P(_Mat), ctypes.c_double, vp, vp]
        L.orc_matvec_t.argtypes = [P(_Mat), ctypes.c_double, vp, vp]
        L.orc_initial_point.argtypes = [P(_Mat), ctypes.c_double, ctypes.c_double, vp]
        L.orc_step_search_terms.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_double,
                                            vp, vp, vp, ctypes.c_int64, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, vp]
        L.orc_step_search_terms.restype = ctypes.c_double
        L.orc_step_search_terms_from.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_double,
                                                 vp, vp, vp, ctypes.c_int64, ctypes.c_double,
                                                 ctypes.c_double, ctypes.c_double, ctypes.c_double, vp]
        L.orc_step_search_terms_from.restype = ctypes.c_double
        L.orc_newton_search_terms.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_double,
                                              vp, vp, vp, ctypes.c_int64, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_double, ctypes.c_double, vp]
        L.orc_newton_search_terms.restype = ctypes.c_double
        L.orc_step_derivatives.argtypes = [vp, vp, ctypes.c_int64, vp, vp, ctypes.c_int64, ctypes.c_double,
                                           ctypes.c_double, vp, vp]
        L.orc_step_derivatives.restype = None
        L.orc_reuse_start.argtypes = [P(_Mat), ctypes.c_double, ctypes.c_double, vp]
        L.orc_reuse_start.restype = ctypes.c_int
        L.orc_potential.argtypes = [P(_Mat), ctypes.c_double, P(_Mat), ctypes.c_double,
                                    ctypes.c_double, vp, vp]
        L.orc_potential.restype = ctypes.c_double
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


# ------------------------------------------------------------------ matrices

@dataclasses.dataclass
class CSR:
    """Explicit CSR with values (the oracle's only matrix format)."""
    rows: int
    cols: int
    ptr: np.ndarray   # int64
    idx: np.ndarray   # int32
    val: np.ndarray   # float64

    def __post_init__(self):
        self.ptr = np.ascontiguousarray(self.ptr, dtype=np.int64)
        self.idx = np.ascontiguousarray(self.idx, dtype=np.int32)
        self.val = np.ascontiguousarray(self.val, dtype=np.float64)
        self._c = _Mat(self.rows, self.cols, self.ptr.ctypes.data, self.idx.ctypes.data,
                       self.val.ctypes.data)
        # the struct holds raw addresses: let it own the arrays, so that
        # `.c` of a temporary CSR stays valid for the call it is passed to
        self._c._arrays = (self.ptr, self.idx, self.val)

    @property
    def c(self):
        return ctypes.byref(self._c)

    def dense(self) -> np.ndarray:
        A = np.zeros((self.rows, self.cols))
        for r in range(self.rows):
            for k in range(self.ptr[r], self.ptr[r + 1]):
                A[r, self.idx[k]] += self.val[k]
        return A

    @staticmethod
    def from_coo(rows: int, cols: int, r: np.ndarray, c: np.ndarray,
                 v: Optional[np.ndarray] = None) -> "CSR":
        r = np.asarray(r, dtype=np.int64)
        c = np.asarray(c, dtype=np.int64)
        v = np.ones(r.shape[0]) if v is None else np.asarray(v, dtype=np.float64)
        order = np.lexsort((c, r))
        r, c, v = r[order], c[order], v[order]
        ptr = np.zeros(rows + 1, dtype=np.int64)
        np.cumsum(np.bincount(r, minlength=rows), out=ptr[1:])
        return CSR(rows, cols, ptr, c.astype(np.int32), v)

    @staticmethod
    def from_dense(A: np.ndarray) -> "CSR":
        r, c = np.nonzero(A)
        return CSR.from_coo(A.shape[0], A.shape[1], r, c, A[r, c])


def _nonisolated(g):
    deg = np.bincount(g.u, minlength=g.num_vertices) + np.bincount(g.v, minlength=g.num_vertices)
    keep = np.nonzero(deg > 0)[0]
    newid = np.full(g.num_vertices, -1, dtype=np.int64)
    newid[keep] = np.arange(keep.shape[0])
    return keep, newid


def incidence(g, drop_isolated: bool = True) -> CSR:
    """M: rows = vertices, columns = edges (eq. incidence, Section 3)."""
    e = np.arange(g.num_edges)
    if drop_isolated:
        keep, newid = _nonisolated(g)
        u, v, nv = newid[g.u], newid[g.v], keep.shape[0]
    else:
        u, v, nv = g.u.astype(np.int64), g.v.astype(np.int64), g.num_vertices
    return CSR.from_coo(nv, g.num_edges, np.concatenate([u, v]), np.concatenate([e, e]))


def vertex_cover_matrix(g):
    """C = M^T (rows = edges, columns = non-isolated vertices); returns (C, kept ids)."""
    keep, newid = _nonisolated(g)
    e = np.arange(g.num_edges)
    C = CSR.from_coo(g.num_edges, keep.shape[0], np.concatenate([e, e]),
                     np.concatenate([newid[g.u], newid[g.v]]))
    return C, keep


def dominating_set_matrix(g) -> CSR:
    """C = I + A (Section 3, dominating set)."""
    n = g.num_vertices
    ar = np.arange(n)
    r = np.concatenate([g.u, g.v, ar])
    c = np.concatenate([g.v, g.u, ar])
    return CSR.from_coo(n, n, r, c)


def densest_matrices(g):
    """(O, W, kept ids): O (n' x 2m) vertex-edge pairs, W (m x 2m) interweaved identity."""
    keep, newid = _nonisolated(g)
    m = g.num_edges
    e = np.arange(m)
    O = CSR.from_coo(keep.shape[0], 2 * m, np.concatenate([newid[g.u], newid[g.v]]),
                     np.concatenate([2 * e, 2 * e + 1]))
    W = CSR.from_coo(m, 2 * m, np.concatenate([e, e]), np.concatenate([2 * e, 2 * e + 1]))
    return O, W, keep


def normalize_packing(A: CSR, b: Optional[np.ndarray] = None, c: Optional[np.ndarray] = None) -> CSR:
    """P_ij = A_ij / (b_i c_j)  (Section 2.1 normalization)."""
    b = np.ones(A.rows) if b is None else np.asarray(b, dtype=np.float64)
    c = np.ones(A.cols) if c is None else np.asarray(c, dtype=np.float64)
    rows = np.repeat(np.arange(A.rows), np.diff(A.ptr))
    return CSR(A.rows, A.cols, A.ptr.copy(), A.idx.copy(), A.val / (b[rows] * c[A.idx]))


# ------------------------------------------------------------------ wrappers

@dataclasses.dataclass
class ProbeResult:
    status: int
    iterations: int
    evaluations: int
    pack_bound: float
    cover_bound: float
    last_alpha: float
    max_violation: float
    x: np.ndarray
    alphas: np.ndarray


def probe(P: CSR, sP: float, C: CSR, sC: float, eps: float = 0.1, max_iter: int = 5000,
          step_rule: int = STEP_BIN, x0: Optional[np.ndarray] = None,
          forced_alpha: Optional[Sequence[float]] = None, start_alpha: float = 0.0,
          drop: bool = False) -> ProbeResult:
    """One MWU feasibility probe (Algorithm 2 + Algorithm 3); drop: leave the
    satisfied covering rows out of every iteration (R22)."""
    n = P.cols
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    fa = None if forced_alpha is None else np.ascontiguousarray(forced_alpha, dtype=np.float64)
    trace = np.zeros(max_iter)
    r = _ProbeResult()
    rc = lib().orc_probe_from(P.c, sP, C.c, sC, eps, max_iter, step_rule, int(x0 is not None),
                         x.ctypes.data, _p(fa), 0 if fa is None else fa.shape[0],
                         trace.ctypes.data, max_iter, start_alpha, int(drop), ctypes.byref(r))
    if rc != 0:
        raise RuntimeError(f"orc_probe failed: {rc}")
    return ProbeResult(r.status, r.iterations, r.evaluations, r.pack_bound, r.cover_bound,
                       r.last_alpha, r.max_violation, x, trace[:r.iterations].copy())


def reuse_start(P: CSR, sP: float, eps: float, x: np.ndarray) -> np.ndarray:
    """The start of a probe that reuses its predecessor's point (R21): x
    scaled so that max(sP P x) = eps."""
    out = np.array(x, dtype=np.float64)
    if not lib().orc_reuse_start(P.c, sP, eps, out.ctypes.data):
        raise ValueError("no positive packing row")
    return out


def iteration_terms(P: CSR, sP: float, C: CSR, sC: float, eps: float, x: np.ndarray,
                    alphas: Sequence[float] = (), drop: bool = False, eta_: Optional[float] = None) -> dict:
    """All per-iteration vectors at point x, plus (Psi, Phi, min z') at each
    alpha; drop leaves the satisfied covering rows out (R22); eta_ replaces
    the eta of the row count."""
    n, mP, mC = P.cols, P.rows, C.rows
    out = {k: np.zeros(n) for k in ("g", "h", "d")}
    out.update({k: np.zeros(mP) for k in ("y", "w", "dy")})
    out.update({k: np.zeros(mC) for k in ("z", "u", "dz")})
    a = np.ascontiguousarray(alphas, dtype=np.float64)
    k = a.shape[0]
    psi, phi, zmn = np.zeros(k), np.zeros(k), np.zeros(k)
    LP, LC = ctypes.c_double(), ctypes.c_double()
    x = np.ascontiguousarray(x, dtype=np.float64)
    rc = lib().orc_iteration_terms(P.c, sP, C.c, sC, eps, x.ctypes.data,
                                   *[out[q].ctypes.data for q in ("y", "z", "w", "u", "g", "h",
                                                                   "d", "dy", "dz")],
                                   ctypes.addressof(LP), ctypes.addressof(LC),
                                   _p(a) if k else None, k, psi.ctypes.data, phi.ctypes.data,
                                   zmn.ctypes.data, int(drop), float(eta_ or 0.0))
    if rc != 0:
        raise RuntimeError(f"orc_iteration_terms failed: {rc}")
    out.update(LP=LP.value, LC=LC.value, psi=psi, phi=phi, zmin_new=zmn,
               eta=eta_ if eta_ else eta(mP + mC, eps))
    return out


def eta(rows_total: int, eps: float) -> float:
    return lib().orc_eta(rows_total, eps)


@dataclasses.dataclass
class SolveResult:
    certified: bool
    objective: float
    lower: float
    upper: float
    probes: int
    total_iterations: int
    final_probe_iterations: int
    evaluations: int
    x: np.ndarray


def _flags(reuse: bool, drop: bool) -> int:
    """Outer-search flags: probe-to-probe reuse (R21), dropping satisfied
    covering rows (R22)."""
    return (1 if reuse else 0) | (2 if drop else 0)


def _solve_result(r, x) -> SolveResult:
    return SolveResult(r.status == 0, r.objective, r.lower, r.upper, r.probes,
                       r.total_iterations, r.final_probe_iterations, r.evaluations, x)


def solve_packing(P: CSR, eps: float = 0.1, max_iter: int = 5000, max_probes: int = 64,
                  step_rule: int = STEP_BIN, reuse: bool = False, drop: bool = False) -> SolveResult:
    x = np.zeros(P.cols)
    r = _SolveResult()
    rc = lib().orc_solve_packing(P.c, eps, max_iter, max_probes, step_rule, _flags(reuse, drop), x.ctypes.data,
                                 ctypes.byref(r))
    if rc != 0:
        raise RuntimeError(f"orc_solve_packing failed: {rc}")
    return _solve_result(r, x)


def solve_covering(C: CSR, eps: float = 0.1, max_iter: int = 5000, max_probes: int = 64,
                   step_rule: int = STEP_BIN, reuse: bool = False, drop: bool = False) -> SolveResult:
    x = np.zeros(C.cols)
    r = _SolveResult()
    rc = lib().orc_solve_covering(C.c, eps, max_iter, max_probes, step_rule, _flags(reuse, drop), x.ctypes.data,
                                  ctypes.byref(r))
    if rc != 0:
        raise RuntimeError(f"orc_solve_covering failed: {rc}")
    return _solve_result(r, x)


def solve_mixed_opt(P: CSR, C: CSR, c, maximize: bool, eps: float = 0.1, max_iter: int = 5000,
                    max_probes: int = 64, step_rule: int = STEP_BIN, reuse: bool = False, drop: bool = False):
    """max (maximize) or min c^T x s.t. P x <= 1, C x >= 1, x >= 0 with the
    objective embedded as one more row and its level M searched (R23).
    Returns (SolveResult, violation), violation = max{0, max(P x) - 1} of
    the returned x."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    x = np.zeros(P.cols)
    v = ctypes.c_double()
    r = _SolveResult()
    rc = lib().orc_solve_mixed_opt(P.c, C.c, c.ctypes.data, int(maximize), eps, max_iter, max_probes, step_rule,
                                   _flags(reuse, drop), x.ctypes.data, ctypes.addressof(v), ctypes.byref(r))
    if rc != 0:
        raise RuntimeError(f"orc_solve_mixed_opt failed: {rc}")
    return _solve_result(r, x), v.value


def solve_densest(g, eps: float = 0.1, max_iter: int = 5000, max_probes: int = 64,
                  step_rule: int = STEP_BIN, reuse: bool = False, drop: bool = False) -> SolveResult:
    O, W, keep = densest_matrices(g)
    _, newid = _nonisolated(g)
    eu = np.ascontiguousarray(newid[g.u], dtype=np.int32)
    ev = np.ascontiguousarray(newid[g.v], dtype=np.int32)
    z = np.zeros(O.cols)
    r = _SolveResult()
    rc = lib().orc_solve_densest(O.c, W.c, eu.ctypes.data, ev.ctypes.data, eps, max_iter,
                                 max_probes, step_rule, _flags(reuse, drop), z.ctypes.data, ctypes.byref(r))
    if rc != 0:
        raise RuntimeError(f"orc_solve_densest failed: {rc}")
    return _solve_result(r, z)


def potential(P: CSR, sP: float, C: CSR, sC: float, eta_: float, x):
    """(smax(sP P x) - smin(sC C x), its gradient): the smoothed potential of
    Section 4.1 and g - h of Algorithm 2."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    gr = np.zeros(P.cols)
    v = lib().orc_potential(P.c, sP, C.c, sC, eta_, x.ctypes.data, gr.ctypes.data)
    return v, gr


def smax(y, eta_):
    y = np.ascontiguousarray(y, dtype=np.float64)
    gr = np.zeros_like(y)
    v = lib().orc_smax(y.ctypes.data, y.shape[0], eta_, gr.ctypes.data)
    return v, gr


def smin(z, eta_):
    z = np.ascontiguousarray(z, dtype=np.float64)
    gr = np.zeros_like(z)
    v = lib().orc_smin(z.ctypes.data, z.shape[0], eta_, gr.ctypes.data)
    return v, gr


def psi(y, dy, w, eta_, L, alpha):
    y, dy, w = (np.ascontiguousarray(a, dtype=np.float64) for a in (y, dy, w))
    return lib().orc_psi(y.ctypes.data, dy.ctypes.data, w.ctypes.data, y.shape[0], eta_, L, alpha)


def phi(z, dz, u, eta_, L, alpha):
    z, dz, u = (np.ascontiguousarray(a, dtype=np.float64) for a in (z, dz, u))
    zm = ctypes.c_double()
    v = lib().orc_phi(z.ctypes.data, dz.ctypes.data, u.ctypes.data, z.shape[0], eta_, L, alpha,
                      ctypes.addressof(zm))
    return v, zm.value


def step_search(y, dy, w, LP, z, dz, u, LC, eta_, eps, start=None):
    """Algorithm 3 on given vectors; returns (alpha, number of T evaluations).
    start (above 1): the warm-started search of reading R19 from that step."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (y, dy, w, z, dz, u)]
    ev = ctypes.c_int64()
    head = (arrs[0].ctypes.data, arrs[1].ctypes.data, arrs[2].ctypes.data, arrs[0].shape[0], LP,
            arrs[3].ctypes.data, arrs[4].ctypes.data, arrs[5].ctypes.data, arrs[3].shape[0], LC,
            eta_, eps)
    if start is None:
        a = lib().orc_step_search_terms(*head, ctypes.addressof(ev))
    else:
        a = lib().orc_step_search_terms_from(*head, float(start), ctypes.addressof(ev))
    return a, ev.value


def newton_search(y, dy, w, LP, z, dz, u, LC, eta_, eps, start):
    """The Newton step search of reading R20 from `start` on given vectors;
    returns (alpha, number of T evaluations)."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (y, dy, w, z, dz, u)]
    ev = ctypes.c_int64()
    a = lib().orc_newton_search_terms(arrs[0].ctypes.data, arrs[1].ctypes.data, arrs[2].ctypes.data,
                                      arrs[0].shape[0], LP, arrs[3].ctypes.data, arrs[4].ctypes.data,
                                      arrs[5].ctypes.data, arrs[3].shape[0], LC, eta_, eps, float(start),
                                      ctypes.addressof(ev))
    return a, ev.value


def step_derivatives(y, dy, z, dz, eta_, alpha):
    """(Psi'(alpha), Phi'(alpha)) as the Newton search forms them."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (y, dy, z, dz)]
    a, b = ctypes.c_double(), ctypes.c_double()
    lib().orc_step_derivatives(arrs[0].ctypes.data, arrs[1].ctypes.data, arrs[0].shape[0],
                               arrs[2].ctypes.data, arrs[3].ctypes.data, arrs[2].shape[0], eta_, float(alpha),
                               ctypes.addressof(a), ctypes.addressof(b))
    return a.value, b.value


def level_set_density(nv: int, eu: np.ndarray, ev: np.ndarray, score: np.ndarray) -> float:
    eu = np.ascontiguousarray(eu, dtype=np.int32)
    ev = np.ascontiguousarray(ev, dtype=np.int32)
    s = np.ascontiguousarray(score, dtype=np.float64)
    return lib().orc_level_set_density(nv, eu.shape[0], eu.ctypes.data, ev.ctypes.data,
                                       s.ctypes.data)


# ------------------------------------------------------------ graph problems

def solve_bmatch(g, **kw) -> SolveResult:
    """Maximum (bipartite) matching LP: max 1^T x s.t. M x <= 1 (pure packing)."""
    return solve_packing(incidence(g), **kw)


def solve_vcover(g, **kw):
    """Vertex cover LP: min 1^T x s.t. M^T x >= 1; x over non-isolated vertices,
    returned scattered back to all vertices (isolated ones at 0)."""
    C, keep = vertex_cover_matrix(g)
    r = solve_covering(C, **kw)
    full = np.zeros(g.num_vertices)
    full[keep] = r.x
    r.x = full
    return r


def solve_domset(g, **kw) -> SolveResult:
    """Dominating set LP: min 1^T x s.t. (I + A) x >= 1."""
    return solve_covering(dominating_set_matrix(g), **kw)
