"""Writes the stored expected values of the full-size configuration parity tests.

Every value comes from the FP64 oracle (``oracle/``) on the seeded inputs of
``workloads/``; nothing here touches the HIP library.  Run from the repository root:

    python tests/golden/make_references.py [c2c] [c3] [c4]

Files (JSON, next to this script):
* ``random_regular_3_22_seed7.json``: the edge list that ``networkx.random_regular_graph(3, 22,
  seed=7)`` returns (networkx 3.4.2), frozen so the instance does not depend on the installed
  version, and the full-state FP64 energy of both observables at the 256 points of the
  orbit-reduction diagnostic (p = 3; its automorphism group is trivial, 33 singleton orbits).
* ``tree26_p4_references.json``: the 32 points of the adjoint-gradient configuration (Pruefer
  tree n = 26, p = 4, H_red): per point the light-cone FP64 energy and adjoint gradient (exact
  for the QAOA state: a term's <Z_i Z_j> only depends on the subgraph within distance p of its
  edge), and the central finite differences (h = 1e-4) of the light-cone FP64 energy.
* ``mixed512_p2_references.json``: the 512 instances of the batched configuration (p = 2, H_red):
  FP64 energy and adjoint gradient of each.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from oracle import derivs as D  # noqa: E402
from oracle import reduced as Rd  # noqa: E402
from workloads import configs as C  # noqa: E402
from workloads.configs import OBS_HC, OBS_HRED  # noqa: E402

RR_FILE = os.path.join(HERE, "random_regular_3_22_seed7.json")
C3_FILE = os.path.join(HERE, "tree26_p4_references.json")
C4_FILE = os.path.join(HERE, "mixed512_p2_references.json")


def _dump(path, obj):
    with open(path, "w") as f:
        json.dump(obj, f, indent=1)
        f.write("\n")
    print("wrote", path, flush=True)


def make_c2c():
    import networkx as nx

    g = nx.random_regular_graph(3, 22, seed=7)
    edges = sorted((min(u, v), max(u, v)) for u, v in g.edges())
    obj = {"source": "networkx.random_regular_graph(3, 22, seed=7)", "networkx": nx.__version__, "n": 22,
           "edges": [list(e) for e in edges]}
    _dump(RR_FILE, obj)  # the configuration reads the edge list from here
    name, wp, p, gam, bet = [c for c in C.config2() if c[0] == "3reg22"][0]
    assert sorted(map(tuple, wp.edges().tolist())) == edges
    out = {}
    for key, obs in (("energy_hc", OBS_HC), ("energy_hred", OBS_HRED)):
        t0 = time.time()
        out[key] = [O.energy(wp.n, wp.edges(), wp.terms(obs), gam[k], bet[k]) for k in range(gam.shape[0])]
        print(key, f"{time.time() - t0:.1f} s", flush=True)
    obj.update({"p": p, "num_orbits": int(len(wp.orbit_rep())), "points_seed": 0, **out})
    _dump(RR_FILE, obj)


def make_c3():
    wp, p, gam, bet = C.config3(32)
    terms = wp.terms(OBS_HRED)
    rows = []
    t0 = time.time()
    for k in range(gam.shape[0]):
        e, dg, db, mb = Rd.light_cone_energy_grad(wp.n, wp.edges(), terms, gam[k], bet[k])
        f = lambda g, b: Rd.light_cone_energy(wp.n, wp.edges(), terms, g, b)
        fg, fb = D.central_fd(f, gam[k], bet[k], h=1e-4)
        rows.append({"gamma": gam[k].tolist(), "beta": bet[k].tolist(), "energy_lc": e, "dgamma_lc": dg.tolist(),
                     "dbeta_lc": db.tolist(), "dgamma_fd": fg.tolist(), "dbeta_fd": fb.tolist(), "max_cone": mb})
        print(f"point {k}: E {e:.12f}  {time.time() - t0:.1f} s", flush=True)
    _dump(C3_FILE, {"workload": "Pruefer tree n=26 (rng 3), p=4, H_red, points from rng 0", "fd_step": 1e-4,
                    "points": rows})


def make_c4():
    probs, p, gam, bet = C.config4()
    rows = []
    t0 = time.time()
    for u, wp in enumerate(probs):
        e, dg, db = O.energy_grad(wp.n, wp.edges(), wp.terms(OBS_HRED), gam[u], bet[u])
        rows.append({"n": wp.n, "family": wp.graph.meta["family"], "energy": e, "dgamma": dg.tolist(),
                     "dbeta": db.tolist()})
    print(f"c4: {time.time() - t0:.1f} s", flush=True)
    _dump(C4_FILE, {"workload": "512 mixed instances (rng 11), p=2, H_red", "units": rows})


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2c", "c3", "c4"]
    for w in which:
        {"c2c": make_c2c, "c3": make_c3, "c4": make_c4}[w]()
