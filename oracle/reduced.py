"""Independent reduced formulations of the same QAOA quantities (FP64 NumPy).

TEST INFRASTRUCTURE ONLY (see the package docstring).  These pin the
full-state C oracle from outside itself:

* ``p1_energy``: the standard closed form of <C_uv> at p = 1 for MaxCut QAOA
  (Wang, Hadfield, Jiang, Rieffel, PRA 97, 022304 (2018)) with d = deg u - 1,
  e = deg v - 1 and f = number of triangles on (u, v), for the convention
  U_P = e^{-i gamma H_C}, U_M = e^{-i beta sum X}.
* ``p1_weighted_energy``: the single-layer expectation of Z_u Z_v for an Ising cost with
  couplings (Ozaeta, van Dam, McMahon, Quantum Sci. Technol. 7, 045036 (2022)), written
  for the weighted cut phase exp(-i gamma sum_e w_e (1 - Z Z)/2), theta_e = gamma w_e:
  <ZZ>_uv = -(1/2) sin 4b sin theta_uv [prod_{x in N(u)-v} cos theta_ux + prod_{x in N(v)-u} cos theta_vx]
            -(1/2) sin^2 2b [prod_{x != u,v} cos(theta_ux + theta_vx) - prod_{x != u,v} cos(theta_ux - theta_vx)]
  (theta = 0 for a non-edge).  With every w = 1 it reduces to the formula above.
* ``complete_graph_energy``: K_n evolves inside the symmetric (Dicke) subspace;
  C = k(n-k) for Hamming weight k and <k+1| sum X |k> = sqrt((k+1)(n-k)).
* ``star_energy``: hub (x) Dicke subspace of the leaves, 2(L+1) dimensions.
* ``light_cone_*``: <Z_u Z_v> after p layers only depends on the subgraph
  induced by the vertices within distance p of {u, v} (reverse causal cone
  section, eqs. rcc1-rcc4).
"""
from __future__ import annotations

import math
from collections import deque
from typing import List, Sequence, Tuple

import numpy as np

from . import energy as _full_energy
from . import energy_grad as _full_energy_grad


# ------------------------------------------------------------------ p = 1
def edge_structure(n: int, edges) -> Tuple[List[set], dict]:
    adj = [set() for _ in range(n)]
    for u, v in np.asarray(edges).reshape(-1, 2):
        adj[int(u)].add(int(v))
        adj[int(v)].add(int(u))
    return adj, {}


def p1_edge_cut_probability(du: int, dv: int, tri: int, gamma: float, beta: float) -> float:
    """<(1 - Z_u Z_v)/2> at p = 1 for an edge whose endpoints have degrees du, dv
    and which lies on ``tri`` triangles."""
    d, e, f = du - 1, dv - 1, tri
    cg = math.cos(gamma)
    return (0.5 + 0.25 * math.sin(4 * beta) * math.sin(gamma) * (cg ** d + cg ** e)
            - 0.25 * math.sin(2 * beta) ** 2 * cg ** (d + e - 2 * f) * (1 - math.cos(2 * gamma) ** f))


def p1_energy(n: int, edges, terms, gamma: float, beta: float) -> float:
    """sum_t w_t <(1 - Z_i Z_j)/2> at p = 1; every term must be an edge of the graph."""
    adj, _ = edge_structure(n, edges)
    ti, tj, tw = terms
    tot = 0.0
    for i, j, w in zip(ti, tj, tw):
        i, j = int(i), int(j)
        if j not in adj[i]:
            raise ValueError("closed form needs each term to be an edge")
        tri = len(adj[i] & adj[j])
        tot += float(w) * p1_edge_cut_probability(len(adj[i]), len(adj[j]), tri, gamma, beta)
    return tot


def p1_weighted_zz(n: int, edges, weights, u: int, v: int, gamma: float, beta: float) -> float:
    """<Z_u Z_v> at p = 1 for the weighted cut phase (the Ising single-layer formula)."""
    th = np.zeros((n, n))
    for (a, b), w in zip(np.asarray(edges).reshape(-1, 2), np.asarray(weights).reshape(-1)):
        th[int(a), int(b)] = th[int(b), int(a)] = gamma * float(w)
    others = [x for x in range(n) if x != u and x != v]
    pu = math.prod(math.cos(th[u, x]) for x in others)
    pv = math.prod(math.cos(th[v, x]) for x in others)
    pplus = math.prod(math.cos(th[u, x] + th[v, x]) for x in others)
    pminus = math.prod(math.cos(th[u, x] - th[v, x]) for x in others)
    return (-0.5 * math.sin(4 * beta) * math.sin(th[u, v]) * (pu + pv)
            - 0.5 * math.sin(2 * beta) ** 2 * (pplus - pminus))


def p1_weighted_energy(n: int, edges, weights, terms, gamma: float, beta: float) -> float:
    """sum_t (w_t/2)(1 - <Z_i Z_j>_t) at p = 1 under the weighted cut phase."""
    ti, tj, tw = terms
    return sum(0.5 * float(w) * (1.0 - p1_weighted_zz(n, edges, weights, int(i), int(j), gamma, beta))
               for i, j, w in zip(ti, tj, tw))


def p1_dEdgamma_dbeta(n: int, edges, terms, gamma: float, beta: float, h: float = 1e-6):
    """Derivatives of the p = 1 closed form (central differences of the closed
    form itself; the closed form is smooth, so h = 1e-6 gives ~1e-9 accuracy)."""
    dg = (p1_energy(n, edges, terms, gamma + h, beta) - p1_energy(n, edges, terms, gamma - h, beta)) / (2 * h)
    db = (p1_energy(n, edges, terms, gamma, beta + h) - p1_energy(n, edges, terms, gamma, beta - h)) / (2 * h)
    return dg, db


# ------------------------------------------------------------------ subspaces
def _expm_sym(B: np.ndarray, beta: float) -> np.ndarray:
    """exp(-i beta B) for a real symmetric B (eigen-decomposition)."""
    mu, V = np.linalg.eigh(B)
    return (V * np.exp(-1j * beta * mu)) @ V.T


def _dicke_mixer(L: int) -> np.ndarray:
    B = np.zeros((L + 1, L + 1))
    for k in range(L):
        B[k + 1, k] = B[k, k + 1] = math.sqrt((k + 1) * (L - k))
    return B


def _dicke_plus(L: int) -> np.ndarray:
    k = np.arange(L + 1)
    return np.sqrt([math.comb(L, int(x)) for x in k]) / 2.0 ** (L / 2)


def complete_graph_energy(n: int, gamma: Sequence[float], beta: Sequence[float]) -> float:
    """<H_C> on K_n at any depth, in the (n+1)-dimensional symmetric subspace."""
    k = np.arange(n + 1)
    C = k * (n - k)
    a = _dicke_plus(n).astype(np.complex128)
    B = _dicke_mixer(n)
    for g, b in zip(gamma, beta):
        a = a * np.exp(-1j * g * C)
        a = _expm_sym(B, b) @ a
    return float(np.sum(np.abs(a) ** 2 * C))


def star_energy(num_leaves: int, gamma: Sequence[float], beta: Sequence[float]) -> float:
    """<H_C> on the star (hub 0, L leaves) at any depth, in hub (x) Dicke(L)."""
    L = num_leaves
    k = np.arange(L + 1)
    C = np.stack([k, L - k])  # C[h, k]: hub bit h
    a = np.outer(np.ones(2) / math.sqrt(2.0), _dicke_plus(L)).astype(np.complex128)
    B = _dicke_mixer(L)
    X = np.array([[0.0, 1.0], [1.0, 0.0]])
    for g, b in zip(gamma, beta):
        a = a * np.exp(-1j * g * C)
        a = _expm_sym(X, b) @ a @ _expm_sym(B, b).T
    return float(np.sum(np.abs(a) ** 2 * C))


# ------------------------------------------------------------------ light cone
def ball(n: int, edges, sources: Sequence[int], radius: int) -> List[int]:
    adj, _ = edge_structure(n, edges)
    dist = {int(s): 0 for s in sources}
    q = deque(dist.keys())
    while q:
        x = q.popleft()
        if dist[x] == radius:
            continue
        for y in adj[x]:
            if y not in dist:
                dist[y] = dist[x] + 1
                q.append(y)
    return sorted(dist)


def _cone(n, edges, i, j, p, weights=None):
    verts = ball(n, edges, [int(i), int(j)], p)
    idx = {v: k for k, v in enumerate(verts)}
    es = np.asarray(edges).reshape(-1, 2)
    keep = [k for k, (u, v) in enumerate(es) if int(u) in idx and int(v) in idx]
    sub = np.asarray([(idx[int(es[k, 0])], idx[int(es[k, 1])]) for k in keep], dtype=np.int32).reshape(-1, 2)
    sw = None if weights is None else np.asarray(weights, dtype=np.int32).reshape(-1)[keep]
    return verts, idx, sub, sw


def light_cone_energy(n: int, edges, terms, gamma, beta, weights=None) -> float:
    """sum_t (w_t/2)(1 - <Z_i Z_j>_t), each term simulated on its cone subgraph (with the
    cone's edge weights when ``weights`` are given)."""
    p = len(np.atleast_1d(gamma))
    ti, tj, tw = terms
    tot = 0.0
    for i, j, w in zip(ti, tj, tw):
        verts, idx, sub, sw = _cone(n, edges, i, j, p, weights)
        t = ([idx[int(i)]], [idx[int(j)]], [float(w)])
        tot += _full_energy(len(verts), sub, t, gamma, beta, weights=sw)
    return tot


def light_cone_energy_grad(n: int, edges, terms, gamma, beta, weights=None):
    """Energy and gradient, each term's contribution by the FP64 adjoint on its cone."""
    gamma = np.asarray(gamma, dtype=np.float64).reshape(-1)
    beta = np.asarray(beta, dtype=np.float64).reshape(-1)
    p = gamma.shape[0]
    ti, tj, tw = terms
    e = 0.0
    dg = np.zeros(p)
    db = np.zeros(p)
    max_ball = 0
    for i, j, w in zip(ti, tj, tw):
        verts, idx, sub, sw = _cone(n, edges, i, j, p, weights)
        max_ball = max(max_ball, len(verts))
        t = ([idx[int(i)]], [idx[int(j)]], [float(w)])
        en, g, b = _full_energy_grad(len(verts), sub, t, gamma, beta, weights=sw)
        e += en
        dg += g
        db += b
    return e, dg, db, max_ball
