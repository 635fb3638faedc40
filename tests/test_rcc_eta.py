"""eta_p, the combined reverse-causal-cone coverage of the representative edges (CPU only).

Oracle pins (oracle/rcc.py, brute force over every choice of representatives):
* Tables 1 and 2: the mean eta_1 and eta_2 of every binary and balanced tree printed there,
  within 0.01 (the printed values are two-decimal means over a random selection);
* the G(29,28) example: with each orbit's lowest-index edge as representative, the cones at
  p = 1 cover exactly the printed vertices;
* closed forms: the cycle C_n has eta_p = 1 - (2p + 1)/n; K_n (one orbit) has
  eta_1 = 1 - (2n - 3)/C(n, 2), rising with n as the paper says; a star has eta_p = 0; a graph
  with trivial automorphism group (every edge its own orbit) has eta_p = 0; eta_p never
  grows with p; the qubit-elimination fraction is 0 for K_n, stars and trivial groups (as
  the paper's figure of descriptors states) and 1 - (2p + 2)/n for cycles.
Library (aaq_rcc_eta) against the oracle: exact means and single choices on trees, cycles,
circulants, Petersen-type, complete, star, random 3-regular and random graphs; the vertex
cover; the argument errors."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import paper_2410_22247_amd as A
from oracle import rcc as R
from workloads import graphs as G
from workloads.orbits import edge_orbits

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_eta.json")))


def orbits_of(g):
    return [int(m) for m in edge_orbits(g).orbit_of]


def lowest_reps(orbit_of):
    reps = {}
    for f, m in enumerate(orbit_of):
        reps.setdefault(m, f)
    return [reps[m] for m in sorted(reps)]


TABLE = [(G.binary_tree(int(n)), v) for n, v in GOLD["binary_tree"].items()] + \
        [(G.balanced_tree(r, h), [e1, e2]) for r, h, e1, e2 in GOLD["balanced_tree"]]


@pytest.mark.parametrize("g,printed", TABLE, ids=lambda x: getattr(x, "name", None) or str(x))
def test_oracle_eta_matches_tables(g, printed):
    of = orbits_of(g)
    for p, want in zip((1, 2), printed):
        got = float(R.eta_mean(g.n, g.edges, of, p))
        assert abs(got - want) <= 0.01, (p, got, want)


def test_oracle_g29_cover_matches_example():
    g = G.binary_tree(29)
    of = orbits_of(g)
    assert len(set(of)) == 12
    cover = R.vertex_cover(g.n, g.edges, lowest_reps(of), 1)
    assert sorted(cover) == GOLD["g29_p1_covered_vertices"]


def test_oracle_closed_forms():
    for n in (7, 13, 20):
        g = G.cycle(n)
        for p in (1, 2, 3):
            assert R.eta_mean(g.n, g.edges, orbits_of(g), p) == 1 - Fraction(2 * p + 1, n)
    prev = -1
    for n in (5, 8, 12, 16):
        g = G.complete(n)
        e1 = R.eta_mean(g.n, g.edges, orbits_of(g), 1)
        assert e1 == 1 - Fraction(2 * n - 3, n * (n - 1) // 2)
        assert e1 > prev
        prev = e1
        assert R.eta_mean(g.n, g.edges, orbits_of(g), 2) == 0
    for n in (6, 12, 21):
        g = G.star(n)
        for p in (1, 2):
            assert R.eta_mean(g.n, g.edges, orbits_of(g), p) == 0
    g = G.random_regular(3, 16, seed=3)
    assert len(set(orbits_of(g))) == g.m  # trivial group
    assert R.eta(g.n, g.edges, list(range(g.m)), 1) == 0
    # qubit elimination (share of qubits outside the cones): the paper's figure has it
    # identically 0 for K_n, stars and trivial groups, rising for edge-transitive families
    for g in (G.complete(9), G.complete(14), G.star(10), G.random_regular(3, 16, seed=3)):
        assert R.qubit_elimination_mean(g.n, g.edges, orbits_of(g), 1) == 0
    for n in (9, 13, 30):
        g = G.cycle(n)
        for p in (1, 2, 3):
            assert R.qubit_elimination_mean(g.n, g.edges, orbits_of(g), p) == 1 - Fraction(2 * p + 2, n)
    for g in (G.binary_tree(20), G.balanced_tree(3, 2), G.prufer_tree(18, 2)):
        of = orbits_of(g)
        vals = [R.eta_mean(g.n, g.edges, of, p) for p in (1, 2, 3, 4)]
        assert all(a >= b for a, b in zip(vals, vals[1:])) and all(0 <= v <= 1 for v in vals)


def graphs_for_library():
    return [G.binary_tree(15), G.binary_tree(29), G.balanced_tree(3, 2), G.prufer_tree(16, 4), G.cycle(11),
            G.circulant(13, [1, 2]), G.generalized_petersen(5, 2), G.complete(7), G.star(9),
            G.random_regular(3, 12, seed=5), G.full_rary_tree(3, 17)]


@pytest.mark.parametrize("g", graphs_for_library(), ids=lambda g: g.name)
def test_library_matches_oracle(g):
    of = orbits_of(g)
    e = np.asarray(g.edges, dtype=np.int32)
    combos = math.prod(np.bincount(of).tolist())
    rng = np.random.default_rng(g.n)
    for p in (1, 2, 3):
        if combos <= 4096:
            eta, qe = A.aaq_rcc_eta(g.n, e, of, p, qubits=True)
            assert abs(eta - float(R.eta_mean(g.n, g.edges, of, p))) <= 1e-12
            assert abs(qe - float(R.qubit_elimination_mean(g.n, g.edges, of, p))) <= 1e-12
            assert A.aaq_rcc_eta(g.n, e, of, p) == eta
        for _ in range(3):
            reps = [int(rng.choice([f for f, m in enumerate(of) if m == k])) for k in range(max(of) + 1)]
            eta, qe, cov = A.aaq_rcc_eta(g.n, e, of, p, rep=reps, vertex_cover=True, qubits=True)
            assert abs(eta - float(R.eta(g.n, g.edges, reps, p))) <= 1e-12
            assert abs(qe - float(R.qubit_elimination(g.n, g.edges, reps, p))) <= 1e-12
            assert sorted(np.flatnonzero(cov).tolist()) == sorted(R.vertex_cover(g.n, g.edges, reps, p))


def test_library_g29_example_and_errors():
    g = G.binary_tree(29)
    of = orbits_of(g)
    e = np.asarray(g.edges, dtype=np.int32)
    _, cov = A.aaq_rcc_eta(g.n, e, of, 1, rep=lowest_reps(of), vertex_cover=True)
    assert np.flatnonzero(cov).tolist() == GOLD["g29_p1_covered_vertices"]
    with pytest.raises(A.AAQError) as x:
        A.aaq_rcc_eta(g.n, e, of, 0)
    assert x.value.status == 1  # p < 1
    assert of[5] != max(of)
    empty = [m if m != of[5] else m + 1 for m in of]  # orbit of[5] now empty, ids still 0..11
    with pytest.raises(A.AAQError) as x:
        A.aaq_rcc_eta(g.n, e, empty, 1)
    assert x.value.status == 3  # AAQ_ERR_ORBITS
    reps = lowest_reps(of)
    reps[0] = reps[1]  # a representative outside its orbit
    with pytest.raises(A.AAQError) as x:
        A.aaq_rcc_eta(g.n, e, of, 1, rep=reps)
    assert x.value.status == 3
    loop = e.copy()
    loop[0] = [4, 4]
    with pytest.raises(A.AAQError) as x:
        A.aaq_rcc_eta(g.n, loop, of, 1)
    assert x.value.status == 2  # AAQ_ERR_GRAPH
