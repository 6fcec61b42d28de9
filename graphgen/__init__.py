"""Seeded synthetic graph generators.

This module only produces inputs: edge lists and CSR patterns drawn from a
seed.  It holds none of the solver's arithmetic, so both the plain CPU
reference under ``oracle/`` and the GPU library can take their inputs from it
without sharing any of the method.

Conventions
-----------
* An undirected edge list is returned canonically: ``u < v``, rows sorted by
  ``(u, v)``, no self-loops and no duplicates.  Edge ``e`` is its position in
  that order.
* A bipartite edge list numbers the left side ``0 .. n_left-1`` and the right
  side ``n_left .. n_left+n_right-1`` so that it is also a plain undirected
  graph; ``u`` is always the left endpoint.
* All draws use numpy's ``PCG64`` bit generator with the given seed.

The graph families follow the workloads the paper measures on (Graph500
Kronecker graphs, random geometric graphs, power-law real graphs; Section 6.3)
as synthetic stand-ins: R-MAT with a/b/c = 0.57/0.19/0.19 is the Graph500
Kronecker generator, Chung-Lu gives a power-law degree sequence, and uniform
bipartite pairs give the bipartite matching inputs.
"""
from __future__ import annotations

import dataclasses
import os
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "Graph", "canonical_edges", "bipartite_uniform", "rmat", "chung_lu",
    "batch_bipartite", "complete_graph", "cycle_graph", "path_graph",
    "star_graph", "complete_bipartite", "random_tree", "gnm_random",
    "grid_graph", "regular_circulant", "adjacency_csr", "bfs_induced_subgraph",
    "relabel_compact", "cached",
]


@dataclasses.dataclass
class Graph:
    """An undirected simple graph as a canonical edge list."""
    num_vertices: int
    u: np.ndarray  # int32, u < v, sorted by (u, v)
    v: np.ndarray  # int32
    n_left: Optional[int] = None  # set for bipartite graphs

    @property
    def num_edges(self) -> int:
        return int(self.u.shape[0])

    def degrees(self) -> np.ndarray:
        deg = np.bincount(self.u, minlength=self.num_vertices)
        deg += np.bincount(self.v, minlength=self.num_vertices)
        return deg.astype(np.int64)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def canonical_edges(u: np.ndarray, v: np.ndarray, num_vertices: int
                    ) -> Tuple[np.ndarray, np.ndarray]:
    """Orient every pair as (min, max), drop self-loops, sort and dedupe."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    key = np.unique(lo * np.int64(num_vertices) + hi)
    return (key // num_vertices).astype(np.int32), (key % num_vertices).astype(np.int32)


def bipartite_uniform(n_left: int, n_right: int, num_edges: int, seed: int) -> Graph:
    """Exactly ``num_edges`` distinct uniform (left, right) pairs.

    Pairs are drawn uniformly with replacement and duplicates rejected until the
    requested count is reached.
    """
    if num_edges > n_left * n_right:
        raise ValueError("more edges than vertex pairs")
    rng = _rng(seed)
    keys = np.empty(0, dtype=np.int64)
    while keys.shape[0] < num_edges:
        need = num_edges - keys.shape[0]
        draw = max(need + need // 8 + 16, 64)
        a = rng.integers(0, n_left, size=draw, dtype=np.int64)
        b = rng.integers(0, n_right, size=draw, dtype=np.int64)
        new = a * n_right + b
        # keep first occurrences in draw order, then merge with what we have
        _, first = np.unique(new, return_index=True)
        new = new[np.sort(first)]
        new = new[~np.isin(new, keys)]
        keys = np.concatenate([keys, new[:need]])
    keys = np.sort(keys)
    u = (keys // n_right).astype(np.int32)
    v = (keys % n_right + n_left).astype(np.int32)
    return Graph(n_left + n_right, u, v, n_left=n_left)


def user_item(users: int, items: int, deg_lo: int, deg_hi: int, zipf: float, seed: int) -> Graph:
    """A user-item rating graph (bipartite, users [0, users), items after):
    every user rates distinct items, as many as a uniform draw from
    [deg_lo, deg_hi] (fewer only if its draws hold fewer distinct items),
    with item popularity proportional to (rank + 1)^-zipf (a long tail, as in
    rating data).  Each user draws 3 deg_hi items with replacement, the
    distinct ones are put in a random order and the first ones kept."""
    rng = _rng(seed)
    w = (np.arange(items, dtype=np.float64) + 1.0) ** -zipf
    cdf = np.cumsum(w / w.sum())
    cdf[-1] = 1.0
    deg = rng.integers(deg_lo, deg_hi + 1, size=users)
    draws = np.searchsorted(cdf, rng.random((users, 3 * deg_hi)), side="right").astype(np.int64)
    pairs = np.unique(np.arange(users, dtype=np.int64)[:, None] * items + draws)
    pu, pi = pairs // items, pairs % items
    order = np.lexsort((rng.random(pairs.shape[0]), pu))
    pu, pi = pu[order], pi[order]
    first = np.searchsorted(pu, np.arange(users))
    keep = np.arange(pu.shape[0]) - first[pu] < deg[pu]
    cu, cv = canonical_edges(pu[keep], users + pi[keep], users + items)
    return Graph(users + items, cu, cv, n_left=users)


def rmat(scale: int, edge_factor: int, seed: int, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, relabel: bool = True) -> Graph:
    """Graph500-style R-MAT: ``edge_factor * 2**scale`` sampled pairs.

    Per bit the quadrant (row bit, column bit) is (0,0) with probability a,
    (0,1) with b, (1,0) with c and (1,1) with 1-a-b-c.  Vertex ids are then
    permuted at random (so id carries no degree information), self-loops are
    dropped and duplicates merged.
    """
    n = 1 << scale
    m = edge_factor * n
    rng = _rng(seed)
    u = np.zeros(m, dtype=np.int64)
    v = np.zeros(m, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for bit in range(scale):
        r = rng.random(m, dtype=np.float32)
        ubit = r >= np.float32(ab)
        vbit = ((r >= np.float32(a)) & (r < np.float32(ab))) | (r >= np.float32(abc))
        u |= ubit.astype(np.int64) << bit
        v |= vbit.astype(np.int64) << bit
        del r, ubit, vbit
    if relabel:
        perm = rng.permutation(n).astype(np.int64)
        u = perm[u]
        v = perm[v]
    cu, cv = canonical_edges(u, v, n)
    return Graph(n, cu, cv)


def chung_lu(n: int, gamma: float, mean_degree: float, seed: int) -> Graph:
    """Chung-Lu power-law graph.

    Vertex i gets weight (i+1)^(-1/(gamma-1)); ``n*mean_degree/2`` endpoint
    pairs are drawn i.i.d. with probability proportional to weight; ids are
    permuted, self-loops dropped and duplicates merged.
    """
    rng = _rng(seed)
    w = np.power(np.arange(1, n + 1, dtype=np.float64), -1.0 / (gamma - 1.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    pairs = int(round(n * mean_degree / 2.0))
    a = np.searchsorted(cdf, rng.random(pairs), side="right")
    b = np.searchsorted(cdf, rng.random(pairs), side="right")
    a = np.minimum(a, n - 1)
    b = np.minimum(b, n - 1)
    perm = rng.permutation(n).astype(np.int64)
    cu, cv = canonical_edges(perm[a], perm[b], n)
    return Graph(n, cu, cv)


def batch_bipartite(count: int, base_seed: int = 5_000_000, side_lo: int = 1024,
                    side_hi: int = 65536, deg_lo: float = 4.0, deg_hi: float = 16.0,
                    scale_div: int = 1) -> List[Graph]:
    """Independent uniform bipartite instances of uneven size.

    Instance k draws its shape with seed ``base_seed + k``: both side sizes
    uniform in [side_lo, side_hi] and the mean left degree uniform in
    [deg_lo, deg_hi]; its ``round(n_left * degree)`` distinct uniform pairs
    come from seed ``base_seed + k + 7919 count``.  ``scale_div`` divides the
    side range (for small test batches).
    """
    out = []
    for k in range(count):
        rng = _rng(base_seed + k)
        lo, hi = max(2, side_lo // scale_div), max(3, side_hi // scale_div)
        nl = int(rng.integers(lo, hi + 1))
        nr = int(rng.integers(lo, hi + 1))
        deg = float(rng.uniform(deg_lo, deg_hi))
        ne = min(int(round(nl * deg)), nl * nr)
        out.append(bipartite_uniform(nl, nr, ne, seed=base_seed + k + 7919 * count))
    return out


# ---------------------------------------------------------------- small families

def _from_pairs(n: int, pairs) -> Graph:
    pairs = np.asarray(list(pairs), dtype=np.int64).reshape(-1, 2)
    if pairs.shape[0] == 0:
        return Graph(n, np.zeros(0, np.int32), np.zeros(0, np.int32))
    u, v = canonical_edges(pairs[:, 0], pairs[:, 1], n)
    return Graph(n, u, v)


def hub_graph(hubs: int, hub_degree: int, leaves: int, seed: int) -> Graph:
    """Vertices [0, hubs) each joined to hub_degree distinct uniform leaves
    among [hubs, hubs + leaves): many rows longer than one tile at once."""
    rng = _rng(seed)
    u = np.repeat(np.arange(hubs, dtype=np.int64), hub_degree)
    v = np.concatenate([hubs + rng.choice(leaves, hub_degree, replace=False) for _ in range(hubs)])
    n = hubs + leaves
    cu, cv = canonical_edges(u, v, n)
    return Graph(n, cu, cv)


def complete_graph(n: int) -> Graph:
    return _from_pairs(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def cycle_graph(n: int) -> Graph:
    return _from_pairs(n, [(i, (i + 1) % n) for i in range(n)])


def path_graph(n: int) -> Graph:
    return _from_pairs(n, [(i, i + 1) for i in range(n - 1)])


def star_graph(leaves: int) -> Graph:
    return _from_pairs(leaves + 1, [(0, i) for i in range(1, leaves + 1)])


def complete_bipartite(a: int, b: int) -> Graph:
    g = _from_pairs(a + b, [(i, a + j) for i in range(a) for j in range(b)])
    g.n_left = a
    return g


def random_tree(n: int, seed: int) -> Graph:
    rng = _rng(seed)
    return _from_pairs(n, [(i, int(rng.integers(0, i))) for i in range(1, n)])


def gnm_random(n: int, m: int, seed: int) -> Graph:
    rng = _rng(seed)
    keys = set()
    while len(keys) < m:
        a, b = int(rng.integers(0, n)), int(rng.integers(0, n))
        if a != b:
            keys.add((min(a, b), max(a, b)))
    return _from_pairs(n, sorted(keys))


def grid_graph(rows: int, cols: int) -> Graph:
    pairs = []
    for r in range(rows):
        for c in range(cols):
            i = r * cols + c
            if c + 1 < cols:
                pairs.append((i, i + 1))
            if r + 1 < rows:
                pairs.append((i, i + cols))
    return _from_pairs(rows * cols, pairs)


def regular_circulant(n: int, k: int) -> Graph:
    """k-regular circulant graph (k even): i ~ i±1..i±k/2 (mod n)."""
    if k % 2 or k >= n:
        raise ValueError("k must be even and < n")
    return _from_pairs(n, [(i, (i + s) % n) for i in range(n) for s in range(1, k // 2 + 1)])


# ---------------------------------------------------------------- derived inputs

def adjacency_csr(g: Graph, with_identity: bool = False) -> Tuple[np.ndarray, np.ndarray]:
    """Pattern-only symmetric adjacency as CSR (int64 row_ptr, int32 col_idx).

    With ``with_identity`` the diagonal is included, giving the pattern of
    A + I.  Columns are sorted within each row.
    """
    n = g.num_vertices
    rows = [g.u.astype(np.int64), g.v.astype(np.int64)]
    cols = [g.v.astype(np.int64), g.u.astype(np.int64)]
    if with_identity:
        ar = np.arange(n, dtype=np.int64)
        rows.append(ar)
        cols.append(ar)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    order = np.lexsort((c, r))
    r, c = r[order], c[order]
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=ptr[1:])
    return ptr, c.astype(np.int32)


def relabel_compact(g: Graph) -> Tuple[Graph, np.ndarray]:
    """Drop isolated vertices; returns the new graph and the kept old ids."""
    deg = g.degrees()
    keep = np.nonzero(deg > 0)[0]
    newid = np.full(g.num_vertices, -1, dtype=np.int64)
    newid[keep] = np.arange(keep.shape[0])
    u, v = canonical_edges(newid[g.u], newid[g.v], keep.shape[0])
    return Graph(int(keep.shape[0]), u, v), keep


def bfs_induced_subgraph(g: Graph, size: int) -> Graph:
    """Induced subgraph on the first ``size`` vertices of a BFS from the
    maximum-degree vertex (ties to the smallest id), relabelled 0..size-1 in
    BFS order."""
    ptr, col = adjacency_csr(g)
    deg = np.diff(ptr)
    src = int(np.argmax(deg))
    order = [src]
    seen = np.zeros(g.num_vertices, dtype=bool)
    seen[src] = True
    head = 0
    while head < len(order) and len(order) < size:
        x = order[head]
        head += 1
        for y in col[ptr[x]:ptr[x + 1]]:
            if not seen[y]:
                seen[y] = True
                order.append(int(y))
                if len(order) >= size:
                    break
    order = np.asarray(order[:size], dtype=np.int64)
    newid = np.full(g.num_vertices, -1, dtype=np.int64)
    newid[order] = np.arange(order.shape[0])
    mu, mv = newid[g.u], newid[g.v]
    keep = (mu >= 0) & (mv >= 0)
    u, v = canonical_edges(mu[keep], mv[keep], order.shape[0])
    return Graph(int(order.shape[0]), u, v)


def cached(name: str, make, cache_dir: Optional[str] = None) -> Graph:
    """Memoise a generated graph as an ``.npz`` file (uncommitted cache)."""
    cache_dir = cache_dir or os.environ.get(
        "MWU_GRAPH_CACHE", os.path.join(os.path.dirname(os.path.dirname(__file__)), ".graph_cache"))
    path = os.path.join(cache_dir, name + ".npz")
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        nl = int(z["n_left"]) if int(z["n_left"]) >= 0 else None
        return Graph(int(z["n"]), z["u"], z["v"], n_left=nl)
    g = make()
    os.makedirs(cache_dir, exist_ok=True)
    tmp = path + ".tmp.npz"
    np.savez(tmp, n=g.num_vertices, u=g.u, v=g.v,
             n_left=-1 if g.n_left is None else g.n_left)
    os.replace(tmp, path)
    return g
