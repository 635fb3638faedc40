"""Aut(G) edge orbits (Algorithm 1 of the paper, "Automorphism-Based Graph
Processing" section) without nauty.

Two steps, as in the paper: (1) obtain permutations that generate (enough of)
Aut(G); (2) close the sorted edge list under those generators by a breadth-first
search, seeding a new class at each still-unclassified edge.  The paper gets
the generators from nauty's ``sparsenauty``; here they come from a small
individualisation-refinement search written for this project.  Step (1) is
driven by the orbits themselves: whenever two edges that could be equivalent
(equal colour-refinement invariants) are still in different classes, the
search looks for an automorphism mapping one onto the other, adds it to the
generator set and recloses.  The result is therefore the exact orbit partition
of the edges under the full group Aut(G), the reading taken for the phrase
"mapped onto each other via a generator" (orbits of the generated group).

Edge (u, v) is stored with u < v; the image of an edge under a permutation is
normalised to (min, max) before lookup.

With integer edge weights (weighted MaxCut, the paper's H_P with its w_ij) the group is the
weight-preserving automorphisms: refinement sees (neighbour colour, edge weight) pairs,
a candidate permutation must map every edge onto an edge of the same weight, and edges of
different weights are never compared.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

from .graphs import Graph


def _refine(adj: List[List[int]], colors: List[int], wadj: Optional[List[List[int]]] = None) -> List[int]:
    """Colour refinement (1-dimensional Weisfeiler-Leman) to a stable colouring;
    ``wadj[v][k]`` is the weight of the edge to ``adj[v][k]`` (all 1 when None).

    Colour names are canonical: they depend only on the multiset structure, so
    two disjoint copies refined together get comparable colours.
    """
    cur = list(colors)
    ncls = len(set(cur))
    if wadj is None:
        wadj = [[1] * len(a) for a in adj]
    while True:
        sigs = [(cur[v], tuple(sorted((cur[w], x) for w, x in zip(adj[v], wadj[v])))) for v in range(len(adj))]
        table = {s: i for i, s in enumerate(sorted(set(sigs)))}
        new = [table[s] for s in sigs]
        k = len(table)
        if k == ncls:
            return new
        cur, ncls = new, k


class _Searcher:
    """Finds automorphisms of G that extend a partial vertex mapping."""

    def __init__(self, g: Graph, weights: Optional[Sequence[int]] = None):
        self.n = g.n
        self.adj = g.adjacency()
        n = self.n
        wt = {}
        for k, (u, v) in enumerate(g.edges):
            wt[(u, v)] = wt[(v, u)] = 1 if weights is None else int(weights[k])
        self.wadj = [[wt[(v, w)] for w in self.adj[v]] for v in range(n)]
        self.adjsets = [{(w, x) for w, x in zip(self.adj[v], self.wadj[v])} for v in range(n)]
        # disjoint union of two copies: vertex v in copy 0, n + v in copy 1
        self.adj2 = [list(a) for a in self.adj] + [[n + w for w in a] for a in self.adj]
        self.wadj2 = self.wadj + self.wadj
        self.base = _refine(self.adj, [0] * n, self.wadj)

    def is_automorphism(self, phi: Sequence[int]) -> bool:
        for v in range(self.n):
            img = {(phi[w], x) for w, x in zip(self.adj[v], self.wadj[v])}
            if img != self.adjsets[phi[v]]:
                return False
        return True

    def extend(self, pairs: Sequence[Tuple[int, int]]) -> Optional[List[int]]:
        """Return an automorphism phi with phi[a] = b for every (a, b), or None."""
        n = self.n
        colors = [1] * (2 * n)
        for i, (a, b) in enumerate(pairs):
            colors[a] = i + 2
            colors[n + b] = i + 2
        return self._search(colors, len(pairs) + 2)

    def _search(self, colors: List[int], next_color: int) -> Optional[List[int]]:
        n = self.n
        col = _refine(self.adj2, colors, self.wadj2)
        cnt0: Dict[int, int] = {}
        cnt1: Dict[int, int] = {}
        for v in range(n):
            cnt0[col[v]] = cnt0.get(col[v], 0) + 1
            cnt1[col[n + v]] = cnt1.get(col[n + v], 0) + 1
        if cnt0 != cnt1:
            return None
        # target cell: smallest non-singleton colour class (ties: smallest colour)
        cell = None
        for c, k in sorted(cnt0.items(), key=lambda t: (t[1], t[0])):
            if k > 1:
                cell = c
                break
        if cell is None:
            where = {col[n + v]: v for v in range(n)}
            phi = [where[col[v]] for v in range(n)]
            return phi if self.is_automorphism(phi) else None
        x = min(v for v in range(n) if col[v] == cell)
        for y in (v for v in range(n) if col[n + v] == cell):
            c2 = list(col)
            # shift existing colours so the new individualised colour is fresh
            c2 = [c + 1 for c in c2]
            c2[x] = 0
            c2[n + y] = 0
            phi = self._search(c2, next_color + 1)
            if phi is not None:
                return phi
        return None


@dataclass
class EdgeOrbits:
    """Edge-orbit partition: ``orbit_of[e]`` is the class id of edge index e
    (edge index = position in the sorted edge list); ``orbits[m]`` lists the
    edge indices of class m in discovery order (the first one is the seed edge
    of Algorithm 1, the lowest-index edge of the class)."""

    orbit_of: List[int]
    orbits: List[List[int]]
    generators: List[List[int]]

    @property
    def count(self) -> int:
        return len(self.orbits)

    def sizes(self) -> List[int]:
        return [len(o) for o in self.orbits]

    def representatives(self, rng=None) -> List[int]:
        """One edge index per class: the seed edge, or a uniformly random member
        if ``rng`` (a numpy Generator) is given (the paper picks at random)."""
        if rng is None:
            return [o[0] for o in self.orbits]
        return [int(o[int(rng.integers(0, len(o)))]) for o in self.orbits]


def close_under_generators(g: Graph, generators: Sequence[Sequence[int]]) -> Tuple[List[int], List[List[int]]]:
    """Algorithm 1's classification loop: BFS closure of the sorted edge list
    under the given vertex permutations."""
    index = {e: i for i, e in enumerate(g.edges)}
    orbit_of = [-1] * g.m
    orbits: List[List[int]] = []
    for e0 in range(g.m):
        if orbit_of[e0] >= 0:
            continue
        cid = len(orbits)
        cls = [e0]
        orbit_of[e0] = cid
        q = deque([e0])
        while q:
            u, v = g.edges[q.popleft()]
            for gen in generators:
                a, b = gen[u], gen[v]
                e2 = index.get((min(a, b), max(a, b)))
                if e2 is None:
                    raise ValueError("generator is not an automorphism")
                if orbit_of[e2] < 0:
                    orbit_of[e2] = cid
                    cls.append(e2)
                    q.append(e2)
        orbits.append(cls)
    return orbit_of, orbits


def edge_orbits(g: Graph, weights: Optional[Sequence[int]] = None) -> EdgeOrbits:
    """Exact Aut(G) edge orbits of g (weight-preserving automorphisms when integer edge
    ``weights`` are given, one per edge in the graph's edge order)."""
    if g.m == 0:
        return EdgeOrbits([], [], [])
    s = _Searcher(g, weights)
    gens: List[List[int]] = []
    inv = [tuple(sorted((s.base[u], s.base[v]))) + ((1 if weights is None else int(weights[k])),)
           for k, (u, v) in enumerate(g.edges)]
    tested = set()
    while True:
        orbit_of, orbits = close_under_generators(g, gens)
        merged = False
        # for each pair of classes with equal invariants, try to map seed to seed
        seeds = [o[0] for o in orbits]
        for i in range(len(seeds)):
            for j in range(i + 1, len(seeds)):
                ei, ej = seeds[i], seeds[j]
                if inv[ei] != inv[ej] or (ei, ej) in tested:
                    continue
                tested.add((ei, ej))
                (a, b), (c, d) = g.edges[ei], g.edges[ej]
                phi = s.extend([(a, c), (b, d)]) or s.extend([(a, d), (b, c)])
                if phi is not None:
                    gens.append(phi)
                    merged = True
                    break
            if merged:
                break
        if not merged:
            return EdgeOrbits(orbit_of, orbits, gens)


def automorphism_generators(g: Graph) -> List[List[int]]:
    """Automorphisms found while computing the edge orbits, plus those needed
    to make the vertex orbits exact (used by invariance tests)."""
    eo = edge_orbits(g)
    s = _Searcher(g)
    gens = list(eo.generators)
    # vertex-orbit completion
    while True:
        parent = list(range(g.n))

        def find(x):
            while parent[x] != x:
                parent[x] = parent[parent[x]]
                x = parent[x]
            return x

        for phi in gens:
            for v in range(g.n):
                a, b = find(v), find(phi[v])
                if a != b:
                    parent[a] = b
        reps = sorted({find(v) for v in range(g.n)})
        added = False
        for i in range(len(reps)):
            for j in range(i + 1, len(reps)):
                u, v = reps[i], reps[j]
                if s.base[u] != s.base[v]:
                    continue
                phi = s.extend([(u, v)])
                if phi is not None:
                    gens.append(phi)
                    added = True
                    break
            if added:
                break
        if not added:
            return gens
