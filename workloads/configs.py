"""Concrete seeded workloads shaped like the paper's experiments.

The paper's instances are generator-made graphs (binary/balanced trees up to
34 vertices; K_n, stars and random 3-regular graphs as diagnostic controls), so
these seeded synthetic inputs *are* the workloads; no dataset is involved.
Every random draw uses ``numpy.random.default_rng(seed)`` in the order given
in each function's docstring.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Tuple

import numpy as np

from . import graphs as G
from .graphs import Graph
from .orbits import EdgeOrbits, edge_orbits

OBS_HC = 0    # full cost Hamiltonian H_C (one ZZ term per edge, weight 1)
OBS_HRED = 1  # orbit-reduced H_red (one ZZ term per edge orbit, weight = orbit size)


@dataclass
class Problem:
    """A MaxCut QAOA instance: graph plus its edge orbits and chosen representatives."""

    graph: Graph
    orbits: EdgeOrbits
    reps: List[int]  # representative edge index per orbit
    weights: Optional[np.ndarray] = None  # integer edge weights (weighted MaxCut), None: all 1

    @property
    def n(self) -> int:
        return self.graph.n

    @property
    def m(self) -> int:
        return self.graph.m

    def edges(self) -> np.ndarray:
        return self.graph.edge_array()

    def orbit_rep(self) -> np.ndarray:
        return np.asarray(self.reps, dtype=np.int32)

    def orbit_size(self) -> np.ndarray:
        return np.asarray(self.orbits.sizes(), dtype=np.int32)

    def edge_orbit(self) -> np.ndarray:
        return np.asarray(self.orbits.orbit_of, dtype=np.int32)

    def edge_weight(self) -> np.ndarray:
        if self.weights is None:
            return np.ones(self.m, dtype=np.int32)
        return np.asarray(self.weights, dtype=np.int32)

    def terms(self, observable: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        """(i, j, w) arrays of the ZZ terms of the observable (H_C: every edge with its
        weight; H_red: one representative per orbit, weight orbit size x edge weight)."""
        e = self.edges()
        w = self.edge_weight()
        if observable == OBS_HC:
            return e[:, 0].copy(), e[:, 1].copy(), w.copy()
        if observable == OBS_HRED:
            r = self.orbit_rep()
            return e[r, 0].copy(), e[r, 1].copy(), (self.orbit_size() * w[r]).astype(np.int32)
        raise ValueError("observable must be 0 (H_C) or 1 (H_red)")


def make_problem(g: Graph, rep_rng: Optional[np.random.Generator] = None, weights=None) -> Problem:
    """The instance with its (weight-preserving, when integer ``weights`` are given) edge
    orbits and the seed edge (or a random member) of each as representative."""
    w = None if weights is None else np.asarray(weights, dtype=np.int32).reshape(-1)
    eo = edge_orbits(g, w)
    return Problem(g, eo, eo.representatives(rep_rng), w)


# ---------------------------------------------------------------- config 1
def config1():
    """Perfect binary tree on 15 vertices, p = 1, 16 x 16 grid
    gamma_a = a*pi/15, beta_b = b*pi/30 (a, b = 0..15), complex128."""
    prob = make_problem(G.binary_tree(15))
    a = np.arange(16)
    gam = a * math.pi / 15
    bet = a * math.pi / 30
    gg, bb = np.meshgrid(gam, bet, indexing="ij")
    return prob, 1, gg.reshape(-1, 1).copy(), bb.reshape(-1, 1).copy()


# ---------------------------------------------------------------- config 2
def _points(seed: int, count: int, p: int):
    rng = np.random.default_rng(seed)
    gam = rng.uniform(0.0, math.pi, (count, p))
    bet = rng.uniform(0.0, math.pi / 2, (count, p))
    return gam, bet


def config2():
    """Orbit-reduction diagnostics, complex64, 256 points per graph drawn from
    default_rng(0): gamma ~ U[0,pi]^(256,p), then beta ~ U[0,pi/2]^(256,p).
    (a) K_16, p=1; (b) star with 19 leaves (n=20), p=2; (c) the random 3-regular
    graph networkx.random_regular_graph(3, 22, seed=7) (frozen edge list), p=3."""
    out = []
    for name, g, p in (
        ("K16", G.complete(16), 1),
        ("star20", G.star(19), 2),
        ("3reg22", G.networkx_random_regular_3_22_seed7(), 3),
    ):
        gam, bet = _points(0, 256, p)
        out.append((name, make_problem(g), p, gam, bet))
    return out


# ---------------------------------------------------------------- config 3
def config3(num_points: int = 32):
    """Random tree n=26 (Pruefer sequence from default_rng(3)), p=4, 32 points
    from default_rng(0): gamma ~ U[0,pi]^(32,4), then beta ~ U[0,pi/2]^(32,4)."""
    prob = make_problem(G.prufer_tree(26, 3))
    gam, bet = _points(0, num_points, 4)
    return prob, 4, gam, bet


# ---------------------------------------------------------------- config 4
def config4(count: int = 512, seed: int = 11):
    """Mixed batch: for each instance, in order, from default_rng(11):
    n = integers(8, 19); family = eligible[integers(len(eligible))] with
    eligible = [tree, star] + [K_n if n <= 12] + [3-regular if n even];
    tree: Pruefer seq = integers(0, n, n-2); 3-regular: pairing model seeded
    with integers(2**31); then gamma ~ U[0,pi]^2, beta ~ U[0,pi/2]^2. p = 2."""
    rng = np.random.default_rng(seed)
    probs, gams, bets = [], [], []
    for _ in range(count):
        n = int(rng.integers(8, 19))
        elig = ["tree", "star"]
        if n <= 12:
            elig.append("complete")
        if n % 2 == 0:
            elig.append("3reg")
        fam = elig[int(rng.integers(0, len(elig)))]
        if fam == "tree":
            g = G.prufer_tree_from_rng(n, rng)
        elif fam == "star":
            g = G.star(n - 1)
        elif fam == "complete":
            g = G.complete(n)
        else:
            g = G.random_regular(3, n, seed=int(rng.integers(0, 2 ** 31)))
        g.meta["family"] = fam
        probs.append(make_problem(g))
        gams.append(rng.uniform(0.0, math.pi, 2))
        bets.append(rng.uniform(0.0, math.pi / 2, 2))
    return probs, 2, np.asarray(gams), np.asarray(bets)


# ---------------------------------------------------------------- config 5
def config5a(num_points: int = 32):
    """Random tree n=34 (Pruefer, default_rng(5)), p=1, forward energy only;
    points from default_rng(0)."""
    prob = make_problem(G.prufer_tree(34, 5))
    gam, bet = _points(0, num_points, 1)
    return prob, 1, gam, bet


def config5b(num_points: int = 4):
    """Random tree n=33 (Pruefer, default_rng(5)), p=2, energy + gradient."""
    prob = make_problem(G.prufer_tree(33, 5))
    gam, bet = _points(0, num_points, 2)
    return prob, 2, gam, bet
