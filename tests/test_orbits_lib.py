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


# ------------------------------------------------------------------ closed forms at larger n
def _partition_of(groups):
    return {frozenset((min(u, v), max(u, v)) for u, v in grp) for grp in groups}


def _closed_form_cases():
    """(name, n, edges, expected partition) for families whose edge orbits are known in
    closed form, up to 34 vertices: the automorphism group of K_n, of a star, of a cycle,
    of K_{a,b}, of a hypercube and of a torus grid acts transitively on the edges; a path
    has only its reversal (edge i with edge n-2-i); a wheel keeps spokes and rim apart;
    two disjoint cycles of different lengths keep their two edge sets apart."""
    cases = []
    for n in (12, 20, 34):
        es = [(u, v) for u in range(n) for v in range(u + 1, n)]
        cases.append((f"K{n}", n, es, [es]))
    for n in (17, 34):
        es = [(0, v) for v in range(1, n)]
        cases.append((f"star{n}", n, es, [es]))
    for n in (5, 23, 34):
        es = [(v, (v + 1) % n) for v in range(n)]
        cases.append((f"C{n}", n, es, [es]))
    for n in (9, 18, 34):
        es = [(i, i + 1) for i in range(n - 1)]
        groups = [[es[i], es[n - 2 - i]] for i in range((n - 1) // 2)]
        if (n - 1) % 2:
            groups.append([es[(n - 1) // 2]])
        cases.append((f"P{n}", n, es, groups))
    for m in (6, 33):  # hub 0 and a rim cycle of m vertices
        spokes = [(0, v) for v in range(1, m + 1)]
        rim = [(v, v % m + 1) for v in range(1, m + 1)]
        cases.append((f"W{m + 1}", m + 1, spokes + rim, [spokes, rim]))
    for a, b in ((3, 7), (17, 17)):
        es = [(u, a + v) for u in range(a) for v in range(b)]
        cases.append((f"K{a},{b}", a + b, es, [es]))
    for d in (4, 5):
        n = 1 << d
        es = [(z, z | (1 << k)) for z in range(n) for k in range(d) if not (z >> k) & 1]
        cases.append((f"Q{d}", n, es, [es]))
    for m in (5, 6):  # torus C_m x C_m
        idx = lambda i, j: (i % m) * m + (j % m)  # noqa: E731
        es = [(idx(i, j), idx(i, j + 1)) for i in range(m) for j in range(m)] + \
             [(idx(i, j), idx(i + 1, j)) for i in range(m) for j in range(m)]
        cases.append((f"T{m}x{m}", m * m, es, [es]))
    c1 = [(v, (v + 1) % 15) for v in range(15)]
    c2 = [(15 + v, 15 + (v + 1) % 19) for v in range(19)]
    cases.append(("C15+C19", 34, c1 + c2, [c1, c2]))
    return cases


@pytest.mark.parametrize("case", _closed_form_cases(), ids=lambda c: c[0])
def test_closed_form_orbits_up_to_34_vertices(case):
    name, n, edges, groups = case
    rng = np.random.default_rng(len(edges))
    perm = rng.permutation(len(edges))  # input order must not matter
    es = np.asarray(edges, dtype=np.int32)[perm]
    of, rep, size = A.aaq_edge_orbits(n, es)
    assert partition(es, of) == _partition_of(groups), name
    assert sorted(size) == sorted(len(set(map(tuple, map(sorted, grp)))) for grp in groups)
    for o, r in enumerate(rep):
        assert of[r] == o
