"""Graph families used by the paper's experiments (Results and Diagnostic
controls sections): binary and balanced trees, random (Pruefer) trees, stars,
complete graphs, random 3-regular graphs, cycles, circulants and generalized
Petersen graphs.

Every generator is deterministic; random ones take a numpy seed and draw from
``numpy.random.default_rng(seed)`` (PCG64) in the order documented per function.
Vertices are 0..n-1 and vertex v is qubit v, i.e. bit v of a basis index z.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np


@dataclass
class Graph:
    """Undirected simple graph; ``edges`` are (u, v) pairs with u < v, sorted."""

    n: int
    edges: List[Tuple[int, int]]
    name: str = ""
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        es = sorted({(min(u, v), max(u, v)) for (u, v) in self.edges})
        if len(es) != len(self.edges):
            raise ValueError("duplicate edges")
        for u, v in es:
            if u == v or not (0 <= u < self.n and 0 <= v < self.n):
                raise ValueError(f"bad edge {(u, v)} for n={self.n}")
        self.edges = es

    @property
    def m(self) -> int:
        return len(self.edges)

    def adjacency(self) -> List[List[int]]:
        adj = [[] for _ in range(self.n)]
        for u, v in self.edges:
            adj[u].append(v)
            adj[v].append(u)
        for a in adj:
            a.sort()
        return adj

    def edge_array(self) -> np.ndarray:
        """int32 array of shape (m, 2)."""
        return np.asarray(self.edges, dtype=np.int32).reshape(-1, 2)

    def degrees(self) -> List[int]:
        return [len(a) for a in self.adjacency()]


def full_rary_tree(r: int, n: int) -> Graph:
    """Tree on n vertices where vertex i has children r*i+1 .. r*i+r (those < n).

    This is the construction behind the 'binary tree G(V,E)' rows of Tables 1
    and 3 (r = 2) and the balanced trees of Tables 2 and 4.
    """
    edges = []
    for i in range(n):
        for j in range(1, r + 1):
            c = r * i + j
            if c < n:
                edges.append((i, c))
    return Graph(n, edges, name=f"rary_tree(r={r},n={n})")


def binary_tree(n: int) -> Graph:
    g = full_rary_tree(2, n)
    g.name = f"binary_tree({n})"
    return g


def balanced_tree(r: int, h: int) -> Graph:
    """Perfect r-ary tree of height h: (r^(h+1)-1)/(r-1) vertices."""
    n = (r ** (h + 1) - 1) // (r - 1) if r > 1 else h + 1
    g = full_rary_tree(r, n)
    g.name = f"balanced_tree(r={r},h={h})"
    return g


def prufer_decode(seq: Sequence[int], n: int) -> Graph:
    """Tree from a Pruefer sequence, repeatedly joining the smallest leaf."""
    seq = [int(s) for s in seq]
    if len(seq) != n - 2:
        raise ValueError("Pruefer sequence must have n-2 entries")
    degree = [1] * n
    for s in seq:
        degree[s] += 1
    edges = []
    import heapq

    leaves = [v for v in range(n) if degree[v] == 1]
    heapq.heapify(leaves)
    for s in seq:
        leaf = heapq.heappop(leaves)
        edges.append((leaf, s))
        degree[s] -= 1
        if degree[s] == 1:
            heapq.heappush(leaves, s)
    u = heapq.heappop(leaves)
    v = heapq.heappop(leaves)
    edges.append((u, v))
    return Graph(n, edges, name=f"prufer_tree(n={n})")


def prufer_tree(n: int, seed: int) -> Graph:
    """Random labelled tree: seq = default_rng(seed).integers(0, n, n-2)."""
    rng = np.random.default_rng(seed)
    seq = rng.integers(0, n, n - 2)
    g = prufer_decode(seq, n)
    g.name = f"prufer_tree(n={n},seed={seed})"
    g.meta["prufer"] = [int(s) for s in seq]
    return g


def prufer_tree_from_rng(n: int, rng: np.random.Generator) -> Graph:
    seq = rng.integers(0, n, n - 2) if n > 2 else np.zeros(0, dtype=np.int64)
    if n == 1:
        return Graph(1, [], name="tree(1)")
    if n == 2:
        return Graph(2, [(0, 1)], name="tree(2)")
    g = prufer_decode(seq, n)
    g.meta["prufer"] = [int(s) for s in seq]
    return g


def star(num_leaves: int) -> Graph:
    """Hub 0 joined to leaves 1..num_leaves (n = num_leaves + 1)."""
    return Graph(num_leaves + 1, [(0, i) for i in range(1, num_leaves + 1)], name=f"star({num_leaves + 1})")


def complete(n: int) -> Graph:
    return Graph(n, [(i, j) for i in range(n) for j in range(i + 1, n)], name=f"K_{n}")


def cycle(n: int) -> Graph:
    return Graph(n, [(i, (i + 1) % n) for i in range(n)], name=f"C_{n}")


def circulant(n: int, jumps: Sequence[int]) -> Graph:
    es = set()
    for i in range(n):
        for j in jumps:
            a, b = i, (i + j) % n
            es.add((min(a, b), max(a, b)))
    return Graph(n, sorted(es), name=f"C_{n}({','.join(map(str, jumps))})")


def generalized_petersen(n: int, k: int) -> Graph:
    """GP(n,k): outer cycle 0..n-1, spokes i--n+i, inner star polygon n+i--n+(i+k)%n."""
    es = set()
    for i in range(n):
        es.add((i, (i + 1) % n) if i < (i + 1) % n else ((i + 1) % n, i))
        es.add((i, n + i))
        a, b = n + i, n + (i + k) % n
        es.add((min(a, b), max(a, b)))
    return Graph(2 * n, sorted(es), name=f"GP({n},{k})")


def random_regular(d: int, n: int, seed: int | None = None, rng: np.random.Generator | None = None) -> Graph:
    """Random simple d-regular graph by the pairing (configuration) model.

    Draw order: repeatedly ``rng.permutation(n*d)`` of the d*n half-edge
    points, pair consecutive points, and accept the first pairing that has no
    self-loop and no repeated edge.
    """
    if (n * d) % 2 != 0 or d >= n:
        raise ValueError("n*d must be even and d < n")
    if rng is None:
        rng = np.random.default_rng(seed)
    points = np.repeat(np.arange(n), d)
    for _ in range(100000):
        perm = rng.permutation(n * d)
        pts = points[perm].reshape(-1, 2)
        ok = True
        es = set()
        for a, b in pts:
            a, b = int(a), int(b)
            if a == b:
                ok = False
                break
            e = (min(a, b), max(a, b))
            if e in es:
                ok = False
                break
            es.add(e)
        if ok:
            return Graph(n, sorted(es), name=f"random_{d}_regular(n={n},seed={seed})")
    raise RuntimeError("pairing model did not produce a simple graph")


FROZEN_RR_3_22_SEED7 = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden",
                                    "random_regular_3_22_seed7.json")


def networkx_random_regular_3_22_seed7() -> Graph:
    """The 3-regular graph on 22 vertices that ``networkx.random_regular_graph(3, 22, seed=7)``
    returns, read from its frozen edge list (written by tests/golden/make_references.py), so
    the instance does not depend on the installed networkx."""
    with open(FROZEN_RR_3_22_SEED7) as f:
        d = json.load(f)
    return Graph(int(d["n"]), [tuple(e) for e in d["edges"]], name="random_3_regular(n=22,seed=7,networkx)")
