"""MI355X (gfx950) multiplicative-weight-update solver for positive LPs.

A thin Python binding over the C ABI of ``libmwu.so`` (``include/mwu.h``):
argument marshalling only, every step of the solver runs in the HIP
library.  Importing the package does not load the library; the first call
does, and fails loudly when it has not been built.

Method: Ju, Yesil, Sun, Chekuri, Solomonik, arXiv 2307.03307 (Algorithm 2
with the step search of Algorithm 3; graph LPs of Section 3).
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import (CERTIFIED, COVERING, FEASIBLE_POINT, FEASIBLE_UNCERTIFIED, FP64, INFEASIBLE, MAX_ITER,
                   MIXED, MIXED_FP32_FP64, MIXED_MAX, MIXED_MIN, PACKING, STEP_BIN, STEP_BIN_WARM, STEP_NEWTON,
                   STEP_STD, MwuError)

__all__ = ["Solver", "BatchSolver", "Result", "csr_matrix", "incidence", "incidence_t", "edge_pair",
           "interweave", "bmatch", "vertex_cover", "dominating_set", "densest_subgraph",
           "MwuError", "PACKING", "COVERING", "MIXED", "MIXED_MAX", "MIXED_MIN", "FP64", "MIXED_FP32_FP64", "STEP_BIN", "STEP_BIN_WARM",
           "STEP_NEWTON", "STEP_STD", "CERTIFIED", "FEASIBLE_UNCERTIFIED", "INFEASIBLE", "MAX_ITER", "FEASIBLE_POINT"]

VEC = {"x": 0, "d": 1, "g": 2, "h": 3, "y": 4, "z": 5, "dy": 6, "dz": 7, "alpha": 8}


@dataclasses.dataclass
class _Mat:
    kind: int
    rows: int = 0
    cols: int = 0
    row_ptr: Optional[np.ndarray] = None
    col_idx: Optional[np.ndarray] = None
    values: Optional[np.ndarray] = None
    num_vertices: int = 0
    num_edges: int = 0
    edge_u: Optional[np.ndarray] = None
    edge_v: Optional[np.ndarray] = None

    def c(self) -> _lib.Matrix:
        p = lambda a: None if a is None else a.ctypes.data
        return _lib.Matrix(self.kind, self.rows, self.cols, p(self.row_ptr), p(self.col_idx),
                           p(self.values), self.num_vertices, self.num_edges, p(self.edge_u),
                           p(self.edge_v))


def csr_matrix(row_ptr, col_idx, values=None, shape=None) -> _Mat:
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    rows = row_ptr.shape[0] - 1
    cols = shape[1] if shape is not None else int(col_idx.max()) + 1
    vals = None if values is None else np.ascontiguousarray(values, dtype=np.float64)
    return _Mat(_lib.MAT_CSR, rows, cols, row_ptr, col_idx, vals)


def _edges(kind, num_vertices, u, v) -> _Mat:
    u = np.ascontiguousarray(u, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.int32)
    return _Mat(kind, num_vertices=int(num_vertices), num_edges=int(u.shape[0]), edge_u=u, edge_v=v)


def incidence(num_vertices, u, v) -> _Mat:
    """M (vertices x edges), eq. incidence of Section 3."""
    return _edges(_lib.MAT_INCIDENCE, num_vertices, u, v)


def incidence_t(num_vertices, u, v) -> _Mat:
    """M^T (edges x vertices): the vertex cover rows x_u + x_v."""
    return _edges(_lib.MAT_INCIDENCE_T, num_vertices, u, v)


def edge_pair(num_vertices, u, v) -> _Mat:
    """O (vertices x 2 edges), eq. oddshifted of Section 3."""
    return _edges(_lib.MAT_EDGE_PAIR, num_vertices, u, v)


def interweave(num_vertices, u, v) -> _Mat:
    """W (edges x 2 edges), eq. interweaved of Section 3."""
    return _edges(_lib.MAT_INTERWEAVE, num_vertices, u, v)


@dataclasses.dataclass
class Result:
    x: np.ndarray
    objective: float
    status: int
    lower: float
    upper: float
    total_iterations: int
    final_probe_iterations: int
    search_passes: int
    probes: int
    max_violation: float
    seconds: float
    evaluations: int = 0

    @property
    def certified(self) -> bool:
        return self.status == CERTIFIED


class Solver:
    """One LP on one GPU (``mwu_create`` ... ``mwu_destroy``)."""

    def __init__(self, form: int, P: Optional[_Mat] = None, C: Optional[_Mat] = None,
                 b_P=None, b_C=None, c=None, eps: float = 0.1, max_iter: int = 5000,
                 max_probes: int = 64, step_rule: int = STEP_BIN,
                 precision: int = MIXED_FP32_FP64, iters_per_launch: int = 0, device: int = 0,
                 stream: Optional[int] = None, fixed_lambda: float = 0.0, flags: int = 0):
        L = _lib.load()
        self._L = L
        self._keep = []
        arr = lambda a: None if a is None else self._hold(np.ascontiguousarray(a, dtype=np.float64))
        empty = _Mat(_lib.MAT_CSR)
        prob = _lib.Problem(form, (P or empty).c(), (C or empty).c(), arr(b_P), arr(b_C), arr(c))
        self._mats = (P, C)
        opt = _lib.Options()
        L.mwu_default_options(ctypes.byref(opt))
        opt.eps, opt.max_iter, opt.max_probes = eps, max_iter, max_probes
        opt.step_rule, opt.precision, opt.iters_per_launch = step_rule, precision, iters_per_launch
        opt.device = device
        opt.hip_stream = stream
        opt.mixed_fixed_lambda = fixed_lambda
        opt.flags = flags
        h = ctypes.c_void_p()
        _lib.check(L.mwu_create(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(h)), "mwu_create")
        self._h = h
        self._keep = []

    def _hold(self, a):
        self._keep.append(a)
        return a.ctypes.data

    @property
    def handle(self):
        return self._h

    @property
    def num_variables(self) -> int:
        return int(self._L.mwu_num_variables(self._h))

    def solve(self, want_x: bool = True) -> Result:
        n = self.num_variables
        x = np.zeros(n) if want_x else None
        obj = ctypes.c_double()
        it = ctypes.c_int64()
        info = _lib.ResultInfo()
        _lib.check(self._L.mwu_solve(self._h, None if x is None else x.ctypes.data,
                                     ctypes.addressof(obj), ctypes.addressof(it),
                                     ctypes.byref(info)), "mwu_solve")
        return Result(x, info.objective, info.status, info.lower_bound, info.upper_bound,
                      info.total_iterations, info.final_probe_iterations, info.search_passes,
                      info.probes, info.max_violation, info.seconds_solve, info.evaluations)

    # ---- probe-level access -------------------------------------------------
    def sizes(self) -> _lib.Sizes:
        s = _lib.Sizes()
        _lib.check(self._L.mwu_probe_sizes(self._h, ctypes.byref(s)), "mwu_probe_sizes")
        return s

    def probe_begin(self, param: float, x0: Optional[np.ndarray] = None) -> None:
        x0 = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        _lib.check(self._L.mwu_probe_begin(self._h, float(param),
                                           None if x0 is None else x0.ctypes.data),
                   "mwu_probe_begin")

    def probe_run(self, max_iters: int, forced_alpha: Optional[Sequence[float]] = None
                  ) -> _lib.ProbeInfo:
        info = _lib.ProbeInfo()
        fa = None if forced_alpha is None else np.ascontiguousarray(forced_alpha, dtype=np.float64)
        _lib.check(self._L.mwu_probe_run(self._h, int(max_iters),
                                         None if fa is None else fa.ctypes.data,
                                         0 if fa is None else fa.shape[0], ctypes.byref(info)),
                   "mwu_probe_run")
        return info

    def probe_direction(self) -> None:
        _lib.check(self._L.mwu_probe_direction(self._h), "mwu_probe_direction")

    def probe_read(self, which: str, length: int) -> np.ndarray:
        out = np.zeros(length)
        _lib.check(self._L.mwu_probe_read(self._h, VEC[which], out.ctypes.data, length),
                   "mwu_probe_read")
        return out

    def probe_eval_steps(self, alphas: Sequence[float]):
        a = np.ascontiguousarray(alphas, dtype=np.float64)
        k = a.shape[0]
        psi, phi, zm = np.zeros(k), np.zeros(k), np.zeros(k)
        _lib.check(self._L.mwu_probe_eval_steps(self._h, a.ctypes.data, k, psi.ctypes.data,
                                                phi.ctypes.data, zm.ctypes.data),
                   "mwu_probe_eval_steps")
        return psi, phi, zm

    def probe_eval_newton(self, alpha: float):
        """(Psi, Phi, Psi', Phi') at step alpha: the Newton pass of STEP_NEWTON."""
        out = [ctypes.c_double() for _ in range(4)]
        _lib.check(self._L.mwu_probe_eval_newton(self._h, float(alpha), *[ctypes.byref(v) for v in out]),
                   "mwu_probe_eval_newton")
        return tuple(v.value for v in out)

    def time_pass(self, which: int, reps: int = 20):
        """(average microseconds, algorithmic bytes, nonzeros) of one pass launch."""
        us, by, nz = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _lib.check(self._L.mwu_time_pass(self._h, int(which), int(reps), ctypes.addressof(us),
                                         ctypes.addressof(by), ctypes.addressof(nz)), "mwu_time_pass")
        return us.value, by.value, nz.value

    # ---- smoothed potential (device pointers) ---------------------------------
    def potential_forward(self, x_dev_ptr: int, stream: Optional[int] = None) -> float:
        """smax(Px) - smin(Cx) at the current probe's param; x_dev_ptr is the
        device address of n doubles (internal variable order)."""
        v = ctypes.c_double()
        _lib.check(self._L.mwu_potential_forward(self._h, ctypes.c_void_p(x_dev_ptr),
                                                 ctypes.addressof(v), ctypes.c_void_p(stream or 0)),
                   "mwu_potential_forward")
        return v.value

    def potential_backward(self, x_dev_ptr: int, grad_scale: float, grad_dev_ptr: int,
                           stream: Optional[int] = None) -> None:
        """grad_dev <- grad_scale * (P^T grad smax(Px) - C^T grad smin(Cx))."""
        _lib.check(self._L.mwu_potential_backward(self._h, ctypes.c_void_p(x_dev_ptr),
                                                  float(grad_scale), ctypes.c_void_p(grad_dev_ptr),
                                                  ctypes.c_void_p(stream or 0)),
                   "mwu_potential_backward")

    def potential_backward_noalloc(self, x_dev_ptr: int, grad_scale: float, grad_dev_ptr: int,
                                   stream: Optional[int] = None) -> float:
        """potential_backward with every scratch buffer in the library's static
        device array (no allocation in the call); returns the potential at x."""
        v = ctypes.c_double()
        _lib.check(self._L.mwu_potential_backward_noalloc(self._h, ctypes.c_void_p(x_dev_ptr),
                                                          float(grad_scale), ctypes.c_void_p(grad_dev_ptr),
                                                          ctypes.addressof(v), ctypes.c_void_p(stream or 0)),
                   "mwu_potential_backward_noalloc")
        return v.value

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.mwu_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class BatchSolver:
    """Many independent bipartite-matching LPs solved together in the same
    kernels (``mwu_create_batch``): every instance keeps its own probe state
    and outer search, and all of them advance in one captured launch
    sequence.  ``graphs`` is a sequence of (num_vertices, u, v)."""

    def __init__(self, graphs, eps: float = 0.1, max_iter: int = 5000, max_probes: int = 64,
                 step_rule: int = STEP_BIN, precision: int = MIXED_FP32_FP64, device: int = 0,
                 flags: int = 0, iters_per_launch: int = 0, tune: bool = False,
                 tune_cache: Optional[str] = None):
        L = _lib.load()
        self._L = L
        mats = [incidence(nv, u, v) for (nv, u, v) in graphs]
        empty = _Mat(_lib.MAT_CSR)
        arr = (_lib.Problem * len(mats))()
        for k, m in enumerate(mats):
            arr[k] = _lib.Problem(PACKING, m.c(), empty.c(), None, None, None)
        self._mats = mats
        self._sizes = [int(m.num_edges) for m in mats]
        opt = _lib.Options()
        L.mwu_default_options(ctypes.byref(opt))
        opt.eps, opt.max_iter, opt.max_probes = eps, max_iter, max_probes
        opt.step_rule, opt.precision, opt.device = step_rule, precision, device
        opt.flags = flags | (_lib.FLAG_TUNE if tune else 0)
        opt.iters_per_launch = iters_per_launch
        self._cache = tune_cache.encode() if tune_cache else None   # kept alive for the call
        opt.tune_cache = self._cache
        h = ctypes.c_void_p()
        _lib.check(L.mwu_create_batch(arr, len(mats), ctypes.byref(opt), ctypes.byref(h)),
                   "mwu_create_batch")
        self._h = h

    @property
    def count(self) -> int:
        return len(self._sizes)

    def layout(self) -> dict:
        """The handle's layout (``mwu_batch_get_layout``) as a dict."""
        lay = _lib.BatchLayout()
        _lib.check(self._L.mwu_batch_get_layout(self._h, ctypes.byref(lay)), "mwu_batch_get_layout")
        return {f: getattr(lay, f) for f, _ in _lib.BatchLayout._fields_}

    def set_layout(self, tile_edges: int, tile_vertices: int, workgroups_per_cu: int,
                   search_launches: int) -> None:
        lay = _lib.BatchLayout(tile_edges, tile_vertices, workgroups_per_cu, search_launches, 0, 0, 0.0)
        _lib.check(self._L.mwu_batch_set_layout(self._h, ctypes.byref(lay)), "mwu_batch_set_layout")

    def solve(self):
        """List of per-instance Results (x per instance, in edge order)."""
        n = sum(self._sizes)
        x = np.zeros(n)
        obj = np.zeros(self.count)
        it = ctypes.c_int64()
        info = (_lib.ResultInfo * self.count)()
        _lib.check(self._L.mwu_solve(self._h, x.ctypes.data, obj.ctypes.data, ctypes.addressof(it),
                                     ctypes.addressof(info)), "mwu_solve")
        out, off = [], 0
        for k, ne in enumerate(self._sizes):
            r = info[k]
            out.append(Result(x[off:off + ne].copy(), r.objective, r.status, r.lower_bound,
                              r.upper_bound, r.total_iterations, r.final_probe_iterations,
                              r.search_passes, r.probes, r.max_violation, r.seconds_solve,
                              r.evaluations))
            off += ne
        return out

    def probe_run(self, params: Sequence[float], max_iters: int = 0):
        """One probe per instance at params[k] in the batched kernels
        (``mwu_batch_probe_run``); list of per-instance ProbeInfo."""
        p = np.ascontiguousarray(params, dtype=np.float64)
        assert p.shape == (self.count,)
        info = (_lib.ProbeInfo * self.count)()
        _lib.check(self._L.mwu_batch_probe_run(self._h, p.ctypes.data, int(max_iters), ctypes.addressof(info)),
                   "mwu_batch_probe_run")
        return [info[k] for k in range(self.count)]

    def probe_read(self, instance: int, which: str, length: int) -> np.ndarray:
        out = np.zeros(length)
        _lib.check(self._L.mwu_batch_probe_read(self._h, int(instance), VEC[which], out.ctypes.data, length),
                   "mwu_batch_probe_read")
        return out

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.mwu_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


# ---------------------------------------------------------------- graph LPs

def bmatch(num_vertices, u, v, **kw) -> Solver:
    """Maximum (bipartite) matching LP: max 1^T x s.t. M x <= 1 (Section 3)."""
    return Solver(PACKING, P=incidence(num_vertices, u, v), **kw)


def vertex_cover(num_vertices, u, v, **kw) -> Solver:
    """Vertex cover LP: min 1^T x s.t. M^T x >= 1 (Section 3)."""
    return Solver(COVERING, C=incidence_t(num_vertices, u, v), **kw)


def dominating_set(row_ptr, col_idx, n, **kw) -> Solver:
    """Dominating set LP: min 1^T x s.t. (I + A) x >= 1; pass the pattern of I + A."""
    return Solver(COVERING, C=csr_matrix(row_ptr, col_idx, shape=(n, n)), **kw)


def densest_subgraph(num_vertices, u, v, **kw) -> Solver:
    """Densest subgraph through the dual LP: min D s.t. W z >= 1, O z <= D (Section 3)."""
    return Solver(MIXED, P=edge_pair(num_vertices, u, v), C=interweave(num_vertices, u, v), **kw)
