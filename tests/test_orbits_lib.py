"""Edge orbits computed by the library (aaq_edge_orbits, host only): the paper's printed
orbit counts, brute-force automorphism enumeration on small graphs, agreement with the
Python orbit tool, input-order independence, and the error paths."""
import itertools
import json
import os

import numpy as np
import pytest

import paper_2410_22247_amd as A
from workloads import graphs as G
from workloads.orbits import edge_orbits

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_orbit_counts.json")


def lib_orbits(g):
    of, rep, size = A.aaq_edge_orbits(g.n, g.edge_array())
    return of, rep, size


def partition(edges, of):
    """The orbit partition as a set of frozensets of normalised edges."""
    cls = {}
    for e, c in zip(edges, of):
        u, v = int(e[0]), int(e[1])
        cls.setdefault(int(c), set()).add((min(u, v), max(u, v)))
    return {frozenset(s) for s in cls.values()}


def test_paper_table_counts():
    gold = json.load(open(GOLD))
    for n, k in gold["binary_tree"].items():
        assert len(lib_orbits(G.binary_tree(int(n)))[1]) == k, n
    for r, h, n, k in gold["balanced_tree"]:
        g = G.balanced_tree(r, h)
        assert g.n == n and len(lib_orbits(g)[1]) == k
    for n, k in gold["complete"].items():
        assert len(lib_orbits(G.complete(int(n)))[1]) == k
    for n, k in gold["star_vertices"].items():
        assert len(lib_orbits(G.star(int(n) - 1))[1]) == k
    assert len(lib_orbits(G.cycle(13))[1]) == gold["cycle_13"]
    assert len(lib_orbits(G.generalized_petersen(5, 2))[1]) == gold["generalized_petersen_5_2"]
    assert len(lib_orbits(G.circulant(13, [1, 2]))[1]) == gold["circulant_13_1_2"]


def brute_force_partition(n, edges):
    es = {(min(u, v), max(u, v)) for u, v in edges}
    auts = [phi for phi in itertools.permutations(range(n))
            if {(min(phi[u], phi[v]), max(phi[u], phi[v])) for u, v in es} == es]
    seen, parts = set(), set()
    for e in sorted(es):
        if e in seen:
            continue
        orb = {(min(phi[e[0]], phi[e[1]]), max(phi[e[0]], phi[e[1]])) for phi in auts}
        seen |= orb
        parts.add(frozenset(orb))
    return parts


@pytest.mark.parametrize("seed", range(12))
def test_matches_brute_force_small(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 8))
    pe = float(rng.choice([0.3, 0.5, 0.7]))
    es = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < pe] or [(0, 1)]
    of, rep, size = A.aaq_edge_orbits(n, np.array(es))
    assert partition(es, of) == brute_force_partition(n, es)


@pytest.mark.parametrize("g", [G.prufer_tree(26, 3), G.prufer_tree(34, 5), G.prufer_tree(33, 5), G.complete(16),
                               G.star(19), G.random_regular(3, 22, seed=7), G.random_regular(3, 12, seed=0),
                               G.generalized_petersen(8, 3), G.binary_tree(31)], ids=lambda g: g.name)
def test_matches_python_tool_and_is_consistent(g):
    of, rep, size = lib_orbits(g)
    eo = edge_orbits(g)
    assert partition(g.edges, of) == partition(g.edges, eo.orbit_of)
    # representatives are the lowest edge index of their class, sizes add up, and the
    # arrays pass the library's own orbit validation
    for c, (r, s) in enumerate(zip(rep, size)):
        members = np.where(of == c)[0]
        assert r == members.min() and s == members.size
    assert size.sum() == g.m
    A.aaq_validate(A.Problem(g.n, g.edge_array(), rep, size, of), 1)


def test_edge_order_does_not_change_the_partition():
    g = G.prufer_tree(20, 4)
    rng = np.random.default_rng(3)
    es = g.edge_array()
    perm = rng.permutation(len(es))
    flipped = np.array([(v, u) if rng.random() < 0.5 else (u, v) for u, v in es[perm]])
    of1, _, _ = A.aaq_edge_orbits(g.n, es)
    of2, _, _ = A.aaq_edge_orbits(g.n, flipped)
    assert partition(es, of1) == partition(flipped, of2)


def test_from_edges_builds_a_valid_problem():
    g = G.binary_tree(15)
    pr = A.Problem.from_edges(g.n, g.edge_array())
    assert pr.num_orbits == 3 and sorted(pr.orbit_size.tolist()) == [2, 4, 8]
    A.aaq_validate(pr, 2)


def test_errors():
    with pytest.raises(A.AAQError) as e:
        A.aaq_edge_orbits(3, np.array([(0, 0)]))
    assert e.value.status == 2  # AAQ_ERR_GRAPH
    with pytest.raises(A.AAQError):
        A.aaq_edge_orbits(3, np.array([(0, 1), (1, 0)]))
    with pytest.raises(A.AAQError):
        A.aaq_edge_orbits(3, np.array([(0, 3)]))
    of, rep, size = A.aaq_edge_orbits(4, np.zeros((0, 2), dtype=np.int32))
    assert of.size == 0 and rep.size == 0
