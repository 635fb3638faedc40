"""Combined reverse-causal-cone coverage eta_p (plain Python, exact rationals where it matters).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's structural descriptor (subsection "Structural descriptor: combined-RCC
coverage", Eq. for eta_p):

    eta_p = 1 - |union over representatives e of RCC_p(e)| / |E|,

the fraction of the graph's edges outside the combined cone of the representative edges.
The reverse causal cone of e = (i, j) (the "Reverse Causal Cone" subsection, eqs. rcc1 to
rcc4) is read here as the set of cost gates that do not commute through to Z_i Z_j: in the
last layer the gates on i or j, in every earlier layer one hop further out, so after p
layers the edges with an endpoint within graph distance p - 1 of {i, j}; its qubits are
the vertices within distance p (N({i, j}) at p = 1).  The tables report eta_p as a mean
over a random choice of representatives; ``eta_mean`` takes the plain definition of that
mean: the average over every combination of one edge per orbit (each equally likely).
"""
from __future__ import annotations

import itertools
from collections import deque
from fractions import Fraction
from typing import Dict, List, Sequence, Tuple


def _adjacency(n: int, edges: Sequence[Tuple[int, int]]) -> List[List[int]]:
    adj: List[List[int]] = [[] for _ in range(n)]
    for u, v in edges:
        adj[u].append(v)
        adj[v].append(u)
    return adj


def distances(n: int, edges: Sequence[Tuple[int, int]], sources: Sequence[int]) -> Dict[int, int]:
    """Graph distance from the nearest source, breadth-first (unreached vertices absent)."""
    adj = _adjacency(n, edges)
    d = {s: 0 for s in sources}
    q = deque(sources)
    while q:
        u = q.popleft()
        for w in adj[u]:
            if w not in d:
                d[w] = d[u] + 1
                q.append(w)
    return d


def rcc_edges(n: int, edges: Sequence[Tuple[int, int]], e: int, p: int) -> set:
    """Indices of the cost gates in the depth-p cone of edge e: an endpoint within p - 1."""
    d = distances(n, edges, list(edges[e]))
    far = p + 1
    return {f for f, (u, v) in enumerate(edges) if min(d.get(u, far), d.get(v, far)) <= p - 1}


def rcc_vertices(n: int, edges: Sequence[Tuple[int, int]], e: int, p: int) -> set:
    """Qubits of the depth-p cone of edge e: the vertices within distance p of its endpoints."""
    return {v for v, dv in distances(n, edges, list(edges[e])).items() if dv <= p}


def eta(n: int, edges: Sequence[Tuple[int, int]], reps: Sequence[int], p: int) -> Fraction:
    """eta_p for one choice of representative edges (exact)."""
    cov = set()
    for e in reps:
        cov |= rcc_edges(n, edges, e, p)
    return 1 - Fraction(len(cov), len(edges))


def vertex_cover(n: int, edges: Sequence[Tuple[int, int]], reps: Sequence[int], p: int) -> set:
    """Union of the qubits of the representatives' cones."""
    cov = set()
    for e in reps:
        cov |= rcc_vertices(n, edges, e, p)
    return cov


def qubit_elimination(n: int, edges: Sequence[Tuple[int, int]], reps: Sequence[int], p: int) -> Fraction:
    """Share of the n qubits outside the union of the representatives' cone qubits (the
    qubit-elimination fraction of the structural-descriptor figure, under that reading)."""
    return 1 - Fraction(len(vertex_cover(n, edges, reps, p)), n)


def _mean(fn, n, edges, orbit_of, p) -> Fraction:
    orbits: Dict[int, List[int]] = {}
    for f, m in enumerate(orbit_of):
        orbits.setdefault(int(m), []).append(f)
    groups = [orbits[m] for m in sorted(orbits)]
    total, count = Fraction(0), 0
    for choice in itertools.product(*groups):
        total += fn(n, edges, choice, p)
        count += 1
    return total / count


def eta_mean(n: int, edges: Sequence[Tuple[int, int]], orbit_of: Sequence[int], p: int) -> Fraction:
    """Mean of eta_p over every choice of one representative per orbit (brute force: the
    product of the orbit sizes must stay small)."""
    return _mean(eta, n, edges, orbit_of, p)


def qubit_elimination_mean(n: int, edges: Sequence[Tuple[int, int]], orbit_of: Sequence[int], p: int) -> Fraction:
    """Mean of the qubit-elimination fraction over every choice of representatives."""
    return _mean(qubit_elimination, n, edges, orbit_of, p)
