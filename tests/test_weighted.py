"""Weighted MaxCut (integer edge weights w_ij in the cost Hamiltonian H_P of the QAOA
section): the cut C(z) = sum w_ij [z_i != z_j] stays an exact integer, the edge orbits are
those of the weight-preserving automorphisms, and H_red's terms carry orbit size x weight.

CPU: the library's weighted orbits against brute-force enumeration of the
weight-preserving permutations and against the Python orbit tool; validation errors.
GPU (through the C ABI): cut values bit-exact for every tile layout; energies, per-term
<ZZ>, gradients (uncompute and checkpointed), batched plans, light cones and sampling
against the weighted FP64 oracle (tolerances as in test_gpu_parity); the n = 26, p = 4
tree with weights against the weighted light-cone FP64 adjoint."""
import itertools
import math

import numpy as np
import pytest

import oracle as O
import paper_2410_22247_amd as A
from oracle import reduced as Rd
from workloads import graphs as G
from workloads.configs import OBS_HC, OBS_HRED, config3, make_problem
from workloads.orbits import edge_orbits

EREL, GREL = 1e-5, 1e-5


def rand_graph(n, pe, seed):
    rng = np.random.default_rng(seed)
    es = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < pe]
    return G.Graph(n, es or [(0, 1)], name=f"G({n},{pe},{seed})")


def depth_weights(g):
    """Weights constant on the unweighted edge orbits (1, 3, 5, 2, 4 by orbit id): every
    automorphism preserves them, so the orbits do not split."""
    of = np.asarray(make_problem(g).orbits.orbit_of)
    return (1 + (2 * of) % 5).astype(np.int32)


def random_weights(g, seed, hi=4):
    return np.random.default_rng(seed).integers(1, hi + 1, g.m).astype(np.int32)


def wproblem(g, w):
    wp = make_problem(g, weights=w)
    return wp, A.Problem.from_workload(wp)


def check_energy(e, ref, rel=EREL):
    assert abs(e - ref) <= rel * max(abs(ref), 1e-12), (e, ref)


def check_grad(g, ref, rel=GREL):
    """Normwise and per-component relative error (the tolerances of test_gpu_parity)."""
    g, ref = np.asarray(g), np.asarray(ref)
    nrm = np.linalg.norm(ref)
    assert np.linalg.norm(g - ref) <= rel * max(nrm, 1e-12), (g, ref)
    assert np.all(np.abs(g - ref) <= rel * np.maximum(np.abs(ref), nrm) + 1e-14), (g, ref)
    return float(np.linalg.norm(g - ref) / max(nrm, 1e-300))


def partition(edges, of):
    cls = {}
    for e, c in zip(edges, of):
        u, v = int(e[0]), int(e[1])
        cls.setdefault(int(c), set()).add((min(u, v), max(u, v)))
    return {frozenset(s) for s in cls.values()}


def brute_force_partition(n, edges, w):
    wt = {(min(u, v), max(u, v)): int(x) for (u, v), x in zip(edges, w)}
    auts = [phi for phi in itertools.permutations(range(n))
            if all(wt.get((min(phi[u], phi[v]), max(phi[u], phi[v]))) == x for (u, v), x in wt.items())]
    seen, parts = set(), set()
    for e in sorted(wt):
        if e in seen:
            continue
        orb = {(min(phi[e[0]], phi[e[1]]), max(phi[e[0]], phi[e[1]])) for phi in auts}
        seen |= orb
        parts.add(frozenset(orb))
    return parts


# ------------------------------------------------------------------ host (CPU)
@pytest.mark.parametrize("seed", range(12))
def test_weighted_orbits_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(3, 8))
    es = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < 0.6] or [(0, 1)]
    w = rng.integers(1, 3, len(es)).astype(np.int32)
    want = brute_force_partition(n, es, w)
    of, _, _ = A.aaq_edge_orbits(n, np.array(es), w)
    assert partition(es, of) == want
    assert partition(es, edge_orbits(G.Graph(n, es), w).orbit_of) == want


@pytest.mark.parametrize("g,w", [(G.binary_tree(31), None), (G.complete(8), "rand"), (G.generalized_petersen(8, 3), "rand"),
                                 (G.star(12), "rand"), (G.prufer_tree(26, 3), "rand"), (G.cycle(12), "alt")],
                         ids=["tree31-depth", "K8", "GP83", "star12", "tree26", "C12-alt"])
def test_weighted_orbits_match_python_tool(g, w):
    if w is None:
        w = depth_weights(g)
    elif w == "alt":
        w = np.array([1 + (k % 2) for k in range(g.m)], dtype=np.int32)
    else:
        w = random_weights(g, g.n, 2)
    of, rep, size = A.aaq_edge_orbits(g.n, g.edge_array(), w)
    assert partition(g.edges, of) == partition(g.edges, edge_orbits(g, w).orbit_of)
    for c in range(len(rep)):  # every class holds one weight
        assert np.ptp(w[of == c]) == 0
    pr = A.Problem.from_edges(g.n, g.edge_array(), w)
    A.aaq_validate(pr, 2)
    if w is not None and g.name.startswith("binary_tree"):
        assert len(rep) == len(make_problem(g).orbits.orbits)  # orbit-constant weights split nothing


def test_weighted_validation_errors():
    g = G.binary_tree(7)
    wp = make_problem(g)
    with pytest.raises(A.AAQError) as e:
        A.aaq_validate(A.Problem(g.n, g.edge_array(), wp.orbit_rep(), wp.orbit_size(), None,
                                 np.array([1, 1, 0, 1, 1, 1])), 1)
    assert e.value.status == 2  # AAQ_ERR_GRAPH: weight < 1
    big = G.complete(20)
    with pytest.raises(A.AAQError) as e:
        A.aaq_validate(A.Problem(big.n, big.edge_array(), edge_weight=np.full(big.m, 3)), 1)
    assert e.value.status == 6  # AAQ_ERR_UNSUPPORTED: total weight 570 > 561
    A.aaq_validate(A.Problem(big.n, big.edge_array(), edge_weight=np.concatenate([np.full(185, 3), np.ones(5)])), 1)  # 560
    with pytest.raises(A.AAQError) as e:  # unweighted orbits with weights that differ inside one
        A.aaq_validate(A.Problem(g.n, g.edge_array(), wp.orbit_rep(), wp.orbit_size(), wp.edge_orbit(),
                                 np.arange(1, 7)), 1)
    assert e.value.status == 3  # AAQ_ERR_ORBITS
    with pytest.raises(A.AAQError):
        A.aaq_edge_orbits(3, np.array([(0, 1), (1, 2)]), np.array([1, 0]))


def test_weighted_lightcone_info():
    g = G.prufer_tree(26, 3)
    w = random_weights(g, 5)
    _, pr = wproblem(g, w)
    _, pu = wproblem(g, None)
    assert A.aaq_lightcone_info(pr, 4, OBS_HC) == A.aaq_lightcone_info(pu, 4, OBS_HC)


# ------------------------------------------------------------------ GPU
W_CASES = [(G.Graph(2, [(0, 1)]), [3], 2), (G.binary_tree(7), "depth", 2), (rand_graph(9, 0.5, 4), "rand", 2),
           (G.complete(11), "rand", 1), (G.binary_tree(15), "depth", 3), (G.prufer_tree(14, 1), "rand", 2),
           (G.star(16), "rand", 2), (G.generalized_petersen(9, 2), "depth", 2), (G.prufer_tree(20, 6), "rand", 3),
           (rand_graph(22, 0.12, 9), "rand", 1)]


def case_weights(g, w):
    if isinstance(w, list):
        return np.array(w, dtype=np.int32)
    return depth_weights(g) if w == "depth" else random_weights(g, g.n * 3 + 1)


@pytest.mark.gpu
@pytest.mark.parametrize("g,w", [(c[0], c[1]) for c in W_CASES if c[0].n <= 20], ids=lambda x: getattr(x, "name", None) or "w")
def test_weighted_cut_values_bit_exact_every_layout(g, w):
    import torch

    w = case_weights(g, w)
    wp, pr = wproblem(g, w)
    ws = torch.empty(1 << 17, dtype=torch.uint8, device="cuda")
    out = torch.empty(1 << g.n, dtype=torch.int32, device="cuda")
    ref_c = O.cut_values(g.n, g.edge_array(), w)
    ref_h = O.term_values(g.n, wp.terms(OBS_HRED)).astype(np.int64)
    for prec in (A.AAQ_PREC_C64, A.AAQ_PREC_C128):
        for s in range(A.aaq_num_sets(g.n, prec)):
            for arr in (0, 1):
                for obs, ref in ((A.AAQ_OBS_HC, ref_c), (A.AAQ_OBS_HRED, ref_h)):
                    out.fill_(-1)
                    A.aaq_cut_values_layout(pr, obs, s, arr, prec, ws, out)
                    assert np.array_equal(out.cpu().numpy(), ref), (prec, s, arr, obs)


@pytest.mark.gpu
@pytest.mark.parametrize("g,w,p", W_CASES, ids=lambda x: getattr(x, "name", None) or str(x))
def test_weighted_energy_and_gradient_match_oracle(g, w, p, record_property):
    w = case_weights(g, w)
    worst = 0.0
    wp, pr = wproblem(g, w)
    rng = np.random.default_rng(g.n * 11 + p)
    gam, bet = rng.uniform(0, math.pi / 2, p), rng.uniform(0, math.pi / 2, p)
    e_hc = None
    for obs in (OBS_HC, OBS_HRED):
        e_ref, dg_ref, db_ref = O.energy_grad(g.n, g.edge_array(), wp.terms(obs), gam, bet, weights=w)
        if e_hc is None:
            e_hc = e_ref
        assert abs(e_ref - e_hc) < 1e-10 * max(1.0, abs(e_hc))  # weighted exact identity
        for prec, tol in ((A.AAQ_PREC_C128, 1e-10), (A.AAQ_PREC_C64, EREL)):
            est = A.Estimator(pr, p, obs, prec, grad=True)
            e, _, nrm = est.energy(gam, bet)
            check_energy(e, e_ref, tol)
            e, dg, db, nrm = est.energy_grad(gam, bet)
            check_energy(e, e_ref, tol)
            err = check_grad(np.concatenate([dg, db]), np.concatenate([dg_ref, db_ref]), tol)
            if prec == A.AAQ_PREC_C64:
                worst = max(worst, err)
            assert abs(nrm - 1) <= (1e-5 if prec == A.AAQ_PREC_C64 else 1e-12)
    record_property("c64_max_rel_err_grad_normwise", worst)


@pytest.mark.gpu
@pytest.mark.parametrize("agg", [A.AAQ_AGG_PER_TERM, A.AAQ_AGG_PASS_PER_TERM], ids=["per_term", "pass_per_term"])
def test_weighted_per_term_aggregation(agg):
    g = G.binary_tree(15)
    w = depth_weights(g)
    wp, pr = wproblem(g, w)
    gam, bet = np.array([0.3, 0.9]), np.array([0.4, 0.2])
    est = A.Estimator(pr, 2, OBS_HC, A.AAQ_PREC_C64, grad=False, agg=agg)
    for obs in (OBS_HC, OBS_HRED):
        e_ref, _, zz_ref, _ = O.energy(g.n, g.edge_array(), wp.terms(obs), gam, bet, full=True, weights=w)
        e, zz, _ = est.energy(gam, bet, obs=obs, agg=agg)
        assert np.max(np.abs(zz - zz_ref)) <= 1e-5
        check_energy(e, e_ref)


@pytest.mark.gpu
@pytest.mark.parametrize("g,p", [(G.prufer_tree(15, 2), 3), (G.prufer_tree(23, 6), 2)], ids=["n15", "n23"])
def test_weighted_checkpointed_gradient(g, p):
    w = random_weights(g, 7)
    wp, pr = wproblem(g, w)
    rng = np.random.default_rng(3)
    gam, bet = rng.uniform(0, math.pi / 2, p), rng.uniform(0, math.pi / 2, p)
    e_ref, dg_ref, db_ref = O.energy_grad(g.n, g.edge_array(), wp.terms(OBS_HRED), gam, bet, weights=w)
    est = A.Estimator(pr, p, OBS_HRED, A.AAQ_PREC_C64, grad=True, checkpoint=True)
    e, dg, db, _ = est.energy_grad(gam, bet)
    check_energy(e, e_ref)
    check_grad(np.concatenate([dg, db]), np.concatenate([dg_ref, db_ref]))


@pytest.mark.gpu
def test_weighted_plan_mixed_units():
    """Weighted and unweighted units, small (one tile) and large (several tile sets), in one
    batched plan with graph replays."""
    import torch

    gs = [(G.star(7), "rand"), (G.complete(9), None), (G.prufer_tree(12, 1), "rand"), (G.binary_tree(15), "depth"),
          (G.prufer_tree(18, 4), "rand"), (G.random_regular(3, 16, seed=3), None)]
    wps, prs, ws_ = [], [], []
    for g, w in gs:
        w = None if w is None else case_weights(g, w)
        wp, pr = wproblem(g, w)
        wps.append(wp)
        prs.append(pr)
        ws_.append(w)
    p = 2
    rng = np.random.default_rng(21)
    units = prs * 2
    gam = rng.uniform(0, math.pi / 2, (len(units), p))
    bet = rng.uniform(0, math.pi / 2, (len(units), p))
    for obs in (OBS_HRED, OBS_HC):
        plan = A.Plan(units, p, obs, with_grad=True, use_graph=True)
        plan.params.copy_(torch.from_numpy(np.concatenate([gam, bet], 1)))
        for _ in range(2):
            out = plan.execute().cpu().numpy()
            torch.cuda.synchronize()
            for u in range(len(units)):
                k = u % len(prs)
                wp = wps[k]
                e_ref, dg_ref, db_ref = O.energy_grad(wp.n, wp.edges(), wp.terms(obs), gam[u], bet[u], weights=ws_[k])
                check_energy(out[u, 0], e_ref)
                check_grad(out[u, 2:], np.concatenate([dg_ref, db_ref]))
        plan.close()


@pytest.mark.gpu
@pytest.mark.parametrize("g,p", [(G.binary_tree(15), 2), (G.prufer_tree(16, 2), 3), (rand_graph(12, 0.3, 4), 2)],
                         ids=["tree15", "prufer16", "rand12"])
def test_weighted_lightcone_matches_oracle(g, p):
    w = random_weights(g, g.n)
    wp, pr = wproblem(g, w)
    rng = np.random.default_rng(g.n + p)
    gam, bet = rng.uniform(0, math.pi / 2, p), rng.uniform(0, math.pi / 2, p)
    for obs in (OBS_HRED, OBS_HC):
        e_ref, dg_ref, db_ref = O.energy_grad(g.n, g.edge_array(), wp.terms(obs), gam, bet, weights=w)
        lc = A.LightCone(pr, p, obs, with_grad=True)
        e, dg, db, _ = lc.energy_grad(gam, bet)
        check_energy(e, e_ref)
        check_grad(np.concatenate([dg, db]), np.concatenate([dg_ref, db_ref]))
        lc.close()


@pytest.mark.gpu
def test_weighted_sampling_cut_values():
    g = G.prufer_tree(14, 2)
    w = random_weights(g, 9, 5)
    _, pr = wproblem(g, w)
    gam, bet = np.array([0.2, 0.5]), np.array([0.6, 0.3])
    u = np.random.default_rng(1).random(2000)
    z, cuts, best, mean = A.Sampler(pr, 2, u.size).sample(gam, bet, u)
    zo, co, cdf = O.sample(g.n, g.edge_array(), gam, bet, u, weights=w)
    z = z.astype(np.int64)
    assert np.array_equal(cuts, O.cut_values(g.n, g.edge_array(), w)[z])
    lo = np.where(z > 0, cdf[np.maximum(z - 1, 0)], 0.0)
    assert np.all(lo - 1e-5 <= u) and np.all(u < cdf[z] + 1e-5)
    assert best == cuts.max() and mean == pytest.approx(cuts.mean(), rel=1e-15, abs=0)


@pytest.mark.gpu
def test_weighted_n26_config3_tree_against_light_cone_oracle(record_property):
    import torch

    wp0, p, gams, bets = config3(1)
    g = wp0.graph
    w = random_weights(g, 26)
    wp, pr = wproblem(g, w)
    est = A.Estimator(pr, p, OBS_HRED, A.AAQ_PREC_C64, grad=True, checkpoint=True)
    e, dg, db, _ = est.energy_grad(gams[0], bets[0])
    e_lc, dg_lc, db_lc, _ = Rd.light_cone_energy_grad(wp.n, wp.edges(), wp.terms(OBS_HRED), gams[0], bets[0],
                                                      weights=w)
    check_energy(e, e_lc)
    record_property("max_rel_err_grad_normwise", check_grad(np.concatenate([dg, db]), np.concatenate([dg_lc, db_lc])))
    del est
    torch.cuda.empty_cache()
