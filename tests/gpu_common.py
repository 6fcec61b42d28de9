"""Problem builders shared by the GPU parity tests: each returns the GPU
solver factory and the oracle's explicit matrices of the same LP."""
import numpy as np

import graphgen as gg
import oracle
import paper_2307_03307_amd as mwu

EPS = 0.1


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / scale) if b.size else 0.0


# the chosen form moves a coordinate only when q = 1 - g/h exceeds 2^-16
MIXED_QMIN = 2.0 ** -16


def direction_err(d, ref, qmin, margin=0.25):
    """Error of a direction d against the oracle's (exact rule q > 0), with
    the chosen form's threshold q > qmin taken apart.  Returns (far, near):
    far is the infinity-relative error over the coordinates whose oracle q
    lies outside (0, (1 + margin) qmin] (the GPU's q carries FP32 rounding
    of g and h, well inside the margin at qmin); near is, over the others,
    the largest distance of the GPU's d_i from the nearer of 0 (dropped by
    the threshold) and the oracle's d_i, relative to max |d|.  The dropped
    coordinates alone can differ by qmin x_i (s / eta), which relative to
    max |d| grows with x_i / max (q x) and has no fixed bound."""
    d = np.asarray(d, dtype=np.float64)
    rd = np.asarray(ref["d"], dtype=np.float64)
    h = np.asarray(ref["h"], dtype=np.float64)
    g = np.asarray(ref["g"], dtype=np.float64)
    q = np.where(h > 0, 1.0 - g / np.where(h > 0, h, 1.0), 0.0)
    near = (q > 0) & (q <= qmin * (1 + margin)) if qmin > 0 else np.zeros(d.shape, bool)
    scale = max(np.max(np.abs(rd)), 1e-300)
    far = float(np.max(np.abs(d[~near] - rd[~near])) / scale) if (~near).any() else 0.0
    nb = float(np.max(np.minimum(np.abs(d[near]), np.abs(d[near] - rd[near]))) / scale) if near.any() else 0.0
    return far, nb


def _merge_flags(kw, flags):
    """Keyword arguments of a solver factory with `flags` or-ed into any the
    caller passes."""
    out = dict(kw)
    out["flags"] = out.get("flags", 0) | flags
    return out


def ones_row(n):
    return oracle.CSR(1, n, np.array([0, n]), np.arange(n), np.ones(n))


class Case:
    """form, oracle matrices (P, C) with probe scales as functions of param,
    and a GPU solver factory."""

    def __init__(self, name, make_gpu, P, C, sP, sC, param):
        self.name, self.make_gpu, self.P, self.C = name, make_gpu, P, C
        self.sP, self.sC, self.param = sP, sC, param


def bmatch_case(g, param=None):
    P = oracle.incidence(g)
    n = P.cols
    param = param or 0.8 * min(g.n_left or g.num_vertices, g.num_vertices - (g.n_left or 0))
    return Case("bmatch", lambda **kw: mwu.bmatch(g.num_vertices, g.u, g.v, **kw), P, ones_row(n),
                lambda p: 1.0, lambda p: 1.0 / p, param)


def vcover_case(g, param=None, generic=False):
    C, keep = oracle.vertex_cover_matrix(g)
    n = C.cols
    flags = mwu._lib.FLAG_GENERIC if generic else 0
    param = param or 0.3 * n
    return Case("vcover" + ("-generic" if generic else ""),
                lambda **kw: mwu.vertex_cover(g.num_vertices, g.u, g.v, **_merge_flags(kw, flags)),
                ones_row(n), C, lambda p: 1.0 / p, lambda p: 1.0, param)


def domset_case(g, param=None):
    ptr, col = gg.adjacency_csr(g, with_identity=True)
    C = oracle.dominating_set_matrix(g)
    n = C.cols
    param = param or 0.1 * n
    return Case("domset", lambda **kw: mwu.dominating_set(ptr, col, n, **kw), ones_row(n), C,
                lambda p: 1.0 / p, lambda p: 1.0, param)


def densest_case(g, param=None, generic=False):
    O, W, keep = oracle.densest_matrices(g)
    param = param or 1.2 * g.num_edges / keep.shape[0]
    flags = mwu._lib.FLAG_GENERIC if generic else 0
    return Case("densest" + ("-generic" if generic else ""),
                lambda **kw: mwu.densest_subgraph(g.num_vertices, g.u, g.v, **_merge_flags(kw, flags)), O, W,
                lambda p: 1.0 / p, lambda p: 1.0, param)


def weighted_packing_case(seed=3, rows=300, cols=900, density=0.02):
    rng = np.random.default_rng(seed)
    A = (rng.random((rows, cols)) < density) * rng.uniform(0.5, 3.0, (rows, cols))
    A[rng.integers(0, rows, cols), np.arange(cols)] += 1.0     # no empty column
    b = rng.uniform(1, 4, rows)
    c = rng.uniform(0.5, 2, cols)
    Ao = oracle.CSR.from_dense(A)
    P = oracle.normalize_packing(Ao, b, c)
    r, k = np.nonzero(A)
    ptr = np.zeros(rows + 1, np.int64)
    np.cumsum(np.bincount(r, minlength=rows), out=ptr[1:])
    make = lambda **kw: mwu.Solver(mwu.PACKING, P=mwu.csr_matrix(ptr, k, A[r, k], shape=A.shape),
                                   b_P=b, c=c, **kw)
    case = Case("weighted-packing", make, P, ones_row(cols), lambda p: 1.0, lambda p: 1.0 / p, 5.0)
    case.A, case.b, case.c = A, b, c
    return case


def start_point(case, seed=0):
    """A positive point with O(1) packing and covering row values."""
    rng = np.random.default_rng(seed)
    n = case.P.cols
    x = rng.uniform(0.5, 1.5, n)
    sP, sC = case.sP(case.param), case.sC(case.param)
    y = np.zeros(case.P.rows)
    z = np.zeros(case.C.rows)
    oracle.lib().orc_matvec(case.P.c, sP, x.ctypes.data, y.ctypes.data)
    oracle.lib().orc_matvec(case.C.c, sC, x.ctypes.data, z.ctypes.data)
    # packing rows near 0.6, covering rows mostly below 1
    f = min(0.6 / y.max(), 0.8 / np.median(z))
    return x * f
