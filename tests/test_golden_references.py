"""Pins of the stored expected values that the full-size configuration tests read
(tests/golden/make_references.py writes them with the FP64 oracle).  Each check uses a
route other than the one that wrote the value: closed forms, reduced subspaces, the exact
identity <H_red> = <H_C> of the paper's reduced Hamiltonian, and the agreement of two
independent derivative routes."""
import json
import math
import os

import numpy as np

from oracle import reduced as Rd
from workloads import configs as C
from workloads import graphs as G
from workloads.configs import OBS_HC, OBS_HRED
from workloads.orbits import edge_orbits

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_frozen_random_regular_graph():
    """The frozen networkx instance is a simple 3-regular graph on 22 vertices with a
    trivial automorphism group (33 singleton edge orbits, so H_red = H_C term by term)."""
    g = G.networkx_random_regular_3_22_seed7()
    assert g.n == 22 and g.m == 33 and set(g.degrees()) == {3}
    eo = edge_orbits(g)
    assert len(eo.sizes()) == 33 and set(eo.sizes()) == {1}
    cfg = [c for c in C.config2() if c[0] == "3reg22"][0]
    assert sorted(map(tuple, cfg[1].edges().tolist())) == g.edges


def test_random_regular_energies():
    """256 stored energies of each observable: equal (trivial group: the same terms), within
    [0, |E|], and at two points equal to the independent numpy per-gate simulator."""
    from oracle import derivs as D

    d = _load("random_regular_3_22_seed7.json")
    e_hc, e_hred = np.asarray(d["energy_hc"]), np.asarray(d["energy_hred"])
    assert e_hc.shape == (256,) and np.max(np.abs(e_hc - e_hred)) <= 1e-12 * 33
    assert np.all((e_hc >= 0) & (e_hc <= 33))
    name, wp, p, gam, bet = [c for c in C.config2() if c[0] == "3reg22"][0]
    for k in (0, 201):
        e = D.per_gate_energy(wp.n, wp.edges(), wp.terms(OBS_HC), gam[k], bet[k])
        assert abs(e - e_hc[k]) <= 1e-10 * abs(e), (k, e, e_hc[k])


def test_tree26_references():
    """At the 32 points: the light-cone FP64 adjoint and the central differences of the
    light-cone energy (independent routes) agree within the differences' truncation error
    h^2 |f'''| / 6 (observed 3.6e-8 of ||g||, bound 3e-7); the energies lie in [0, |E|]; the points
    are the seeded ones."""
    d = _load("tree26_p4_references.json")
    wp, p, gam, bet = C.config3(32)
    assert d["fd_step"] == 1e-4 and len(d["points"]) == 32
    worst = 0.0
    for k, r in enumerate(d["points"]):
        assert r["gamma"] == gam[k].tolist() and r["beta"] == bet[k].tolist()
        assert 0 <= r["energy_lc"] <= wp.m and r["max_cone"] <= 20
        g = np.asarray(r["dgamma_lc"] + r["dbeta_lc"])
        f = np.asarray(r["dgamma_fd"] + r["dbeta_fd"])
        worst = max(worst, np.linalg.norm(g - f) / np.linalg.norm(g))
    assert worst <= 3e-7, worst


def test_mixed512_references():
    """The 512 stored energies and gradients: the complete graphs against the Dicke-subspace
    oracle and the stars against the hub x Dicke oracle (independent simulators), every
    energy within [0, |E|]."""
    d = _load("mixed512_p2_references.json")["units"]
    probs, p, gam, bet = C.config4()
    assert len(d) == len(probs) == 512
    h = 1e-5
    checked = 0
    for u, (r, wp) in enumerate(zip(d, probs)):
        assert r["n"] == wp.n and r["family"] == wp.graph.meta["family"]
        assert 0 <= r["energy"] <= wp.m
        fam = r["family"]
        if fam not in ("complete", "star") or u % 3:
            continue
        if fam == "complete":
            f = lambda g_, b_: Rd.complete_graph_energy(wp.n, g_, b_)  # noqa: E731
        else:
            f = lambda g_, b_: Rd.star_energy(wp.n - 1, g_, b_)  # noqa: E731
        assert abs(f(gam[u], bet[u]) - r["energy"]) <= 1e-11 * max(1.0, r["energy"])
        # central differences of the reduced-subspace energy against the stored adjoint
        fd = []
        for which in (0, 1):
            for l in range(p):
                e = np.zeros(p)
                e[l] = h
                if which == 0:
                    fd.append((f(gam[u] + e, bet[u]) - f(gam[u] - e, bet[u])) / (2 * h))
                else:
                    fd.append((f(gam[u], bet[u] + e) - f(gam[u], bet[u] - e)) / (2 * h))
        g = np.asarray(r["dgamma"] + r["dbeta"])
        assert np.linalg.norm(np.asarray(fd) - g) <= 1e-5 * max(np.linalg.norm(g), 1.0), (u, fd, g)
        checked += 1
    assert checked >= 60
