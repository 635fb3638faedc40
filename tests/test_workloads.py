"""Input generators and the host orbit finder (Algorithm 1), pinned to the
paper's printed orbit counts and to brute-force automorphism enumeration."""
import itertools
import json
import os

import numpy as np
import pytest

from workloads import graphs as G
from workloads.configs import config1, config2, config3, config5a, config5b, make_problem, OBS_HC, OBS_HRED
from workloads.orbits import close_under_generators, edge_orbits, automorphism_generators

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_orbit_counts.json")


def paper_counts():
    with open(GOLD) as f:
        return json.load(f)


def test_binary_tree_orbits_match_table1():
    for n, cnt in paper_counts()["binary_tree"].items():
        assert edge_orbits(G.binary_tree(int(n))).count == cnt, n


def test_balanced_tree_orbits_match_table2():
    for r, h, n, cnt in paper_counts()["balanced_tree"]:
        g = G.balanced_tree(r, h)
        assert g.n == n and g.m == n - 1
        assert edge_orbits(g).count == cnt


def test_control_family_orbits():
    pc = paper_counts()
    for n, c in pc["complete"].items():
        assert edge_orbits(G.complete(int(n))).count == c
    for n, c in pc["star_vertices"].items():
        assert edge_orbits(G.star(int(n) - 1)).count == c
    assert edge_orbits(G.cycle(13)).count == pc["cycle_13"]
    assert edge_orbits(G.generalized_petersen(5, 2)).count == pc["generalized_petersen_5_2"]
    assert edge_orbits(G.circulant(13, [1, 2])).count == pc["circulant_13_1_2"]


def brute_orbits(g):
    """Edge orbits by enumerating every vertex permutation (tiny graphs only)."""
    es = set(g.edges)
    auts = []
    for perm in itertools.permutations(range(g.n)):
        if all((min(perm[u], perm[v]), max(perm[u], perm[v])) in es for u, v in g.edges):
            auts.append(perm)
    oid = {}
    classes = []
    for e in g.edges:
        if e in oid:
            continue
        orb = {(min(a[e[0]], a[e[1]]), max(a[e[0]], a[e[1]])) for a in auts}
        for f in orb:
            oid[f] = len(classes)
        classes.append(orb)
    return sorted(sorted(c) for c in classes), len(auts)


@pytest.mark.parametrize("seed", range(12))
def test_orbits_equal_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(3, 8))
    if seed % 3 == 0:
        g = G.prufer_tree_from_rng(n, rng)
    else:
        es = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < 0.45]
        if not es:
            es = [(0, 1)]
        g = G.Graph(n, es)
    eo = edge_orbits(g)
    got = sorted(sorted(g.edges[e] for e in o) for o in eo.orbits)
    want, _ = brute_orbits(g)
    assert got == want


def test_generators_are_automorphisms_and_close_to_orbits():
    g = G.binary_tree(20)
    gens = automorphism_generators(g)
    es = set(g.edges)
    for phi in gens:
        assert sorted(phi) == list(range(g.n))
        assert all((min(phi[u], phi[v]), max(phi[u], phi[v])) in es for u, v in g.edges)
    oid, orbs = close_under_generators(g, gens)
    assert len(orbs) == edge_orbits(g).count


def test_prufer_decoding_matches_networkx():
    nx = pytest.importorskip("networkx")
    rng = np.random.default_rng(5)
    for n in (3, 5, 10, 26):
        seq = [int(x) for x in rng.integers(0, n, n - 2)]
        ours = G.prufer_decode(seq, n).edges
        theirs = sorted((min(u, v), max(u, v)) for u, v in nx.from_prufer_sequence(seq).edges())
        assert ours == theirs


def test_rary_trees_match_networkx():
    nx = pytest.importorskip("networkx")
    for n in (5, 10, 15, 34):
        assert G.binary_tree(n).edges == sorted((min(u, v), max(u, v)) for u, v in nx.full_rary_tree(2, n).edges())
    for r, h in ((2, 2), (3, 2), (2, 4)):
        assert G.balanced_tree(r, h).edges == sorted(
            (min(u, v), max(u, v)) for u, v in nx.balanced_tree(r, h).edges())


def test_random_regular_is_simple_regular_and_seeded():
    a = G.random_regular(3, 22, seed=7)
    b = G.random_regular(3, 22, seed=7)
    assert a.edges == b.edges and a.m == 33
    assert all(d == 3 for d in a.degrees())


def test_config_shapes_and_orbit_ratios():
    prob, p, gam, bet = config1()
    assert (prob.n, prob.m, prob.orbits.count, p) == (15, 14, 3, 1) and gam.shape == (256, 1)
    assert sorted(prob.orbits.sizes()) == [2, 4, 8]
    c2 = config2()
    assert [(x[1].n, x[1].m, x[1].orbits.count, x[2]) for x in c2] == [(16, 120, 1, 1), (20, 19, 1, 2),
                                                                         (22, 33, 33, 3)]
    prob, p, gam, bet = config3()
    assert (prob.n, prob.m, prob.orbits.count, p, gam.shape) == (26, 25, 20, 4, (32, 4))
    assert (gam >= 0).all() and (gam <= np.pi).all() and (bet >= 0).all() and (bet <= np.pi / 2).all()
    prob, p, *_ = config5a()
    assert (prob.n, prob.m, prob.orbits.count, p) == (34, 33, 29, 1)
    prob, p, *_ = config5b()
    assert (prob.n, prob.m, prob.orbits.count, p) == (33, 32, 29, 2)


def test_terms():
    prob = make_problem(G.binary_tree(15))
    ti, tj, tw = prob.terms(OBS_HC)
    assert len(ti) == 14 and (tw == 1).all()
    ri, rj, rw = prob.terms(OBS_HRED)
    assert len(ri) == 3 and rw.sum() == 14
