"""Light-cone evaluation (aaq_lightcone_*): every observable term simulated on the
subgraph within distance p of its edge.

CPU: the library's cone construction against the oracle's own breadth-first ball
(unit counts, largest cone, total amplitudes) and the error paths.
GPU: energies and gradients against the full-state FP64 oracle (small n), against the
light-cone FP64 adjoint at the full configuration sizes, and against the full-state HIP
path on the same GPU; H_red = H_C; graph replays with new parameters.
Tolerances as in test_gpu_parity (1e-5 relative for complex64, 1e-10 for complex128)."""
import math

import numpy as np
import pytest

import oracle as O
import paper_2410_22247_amd as A
from oracle import reduced as Rd
from workloads import graphs as G
from workloads.configs import OBS_HC, OBS_HRED, config3, config5a, config5b, make_problem

EREL, GREL = 1e-5, 1e-5


def rand_graph(n, pe, seed):
    rng = np.random.default_rng(seed)
    es = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < pe]
    return G.Graph(n, es or [(0, 1)], name=f"G({n},{pe},{seed})")


def check_energy(e, ref, rel=EREL):
    assert abs(e - ref) <= rel * max(abs(ref), 1e-12), (e, ref)


def check_grad(g, ref, rel=GREL):
    g, ref = np.asarray(g), np.asarray(ref)
    nrm = np.linalg.norm(ref)
    assert np.linalg.norm(g - ref) <= rel * max(nrm, 1e-12), (g, ref)
    assert np.all(np.abs(g - ref) <= rel * np.maximum(np.abs(ref), nrm) + 1e-14), (g, ref)


# ------------------------------------------------------------------ host (CPU)
CONE_GRAPHS = [(G.binary_tree(15), 1), (G.binary_tree(15), 2), (G.prufer_tree(26, 3), 4), (G.prufer_tree(34, 5), 1),
               (G.prufer_tree(33, 5), 2), (G.complete(9), 1), (G.star(12), 3), (G.random_regular(3, 22, seed=7), 2),
               (rand_graph(14, 0.2, 3), 2), (G.Graph(2, [(0, 1)]), 5)]


@pytest.mark.parametrize("g,p", CONE_GRAPHS, ids=lambda x: getattr(x, "name", str(x)))
def test_lightcone_info_matches_oracle_balls(g, p):
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    for obs in (OBS_HC, OBS_HRED):
        ti, tj, _ = wp.terms(obs)
        sizes = [len(Rd.ball(g.n, g.edge_array(), [int(i), int(j)], p)) for i, j in zip(ti, tj)]
        units, mq, amp = A.aaq_lightcone_info(pr, p, obs)
        assert units == len(ti)
        assert mq == max(sizes)
        assert amp == float(sum(2 ** s for s in sizes))


def test_lightcone_config_sizes():
    """The cone sizes of the n=26 p=4, n=34 p=1 and n=33 p=2 trees (largest balls 20, 7, 16)."""
    for fn, mq_ref in ((config3, 20), (config5a, 7), (config5b, 16)):
        wp, p, _, _ = fn(1)
        pr = A.Problem.from_workload(wp)
        units, mq, _ = A.aaq_lightcone_info(pr, p, OBS_HRED)
        assert units == wp.orbits.count and mq == mq_ref


def test_lightcone_errors():
    empty = A.Problem(3, np.zeros((0, 2), dtype=np.int32))
    with pytest.raises(A.AAQError) as e:
        A.aaq_lightcone_info(empty, 1, OBS_HC)
    assert e.value.status == 6  # AAQ_ERR_UNSUPPORTED
    pr = A.Problem.from_workload(make_problem(G.binary_tree(7)))
    with pytest.raises(A.AAQError) as e:
        A.aaq_lightcone_info(pr, 0, OBS_HC)
    assert e.value.status == 1  # AAQ_ERR_INVALID_ARG
    with pytest.raises(A.AAQError):
        A.aaq_lightcone_workspace_size(pr, 2, 7, True)


# ------------------------------------------------------------------ GPU
LC_CASES = [(G.binary_tree(15), 1), (G.binary_tree(13), 2), (G.prufer_tree(16, 2), 3), (G.complete(8), 2),
            (G.star(11), 2), (rand_graph(12, 0.3, 4), 2), (G.random_regular(3, 14, seed=3), 2),
            (G.generalized_petersen(7, 2), 1), (G.Graph(2, [(0, 1)]), 3)]


@pytest.mark.gpu
@pytest.mark.parametrize("g,p", LC_CASES, ids=lambda x: getattr(x, "name", str(x)))
def test_lightcone_matches_full_state_oracle(g, p):
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    rng = np.random.default_rng(g.n * 17 + p)
    gam, bet = rng.uniform(0, math.pi, p), rng.uniform(0, math.pi / 2, p)
    for obs in (OBS_HRED, OBS_HC):
        e_ref, dg_ref, db_ref = O.energy_grad(g.n, g.edge_array(), wp.terms(obs), gam, bet)
        for prec, tol in ((A.AAQ_PREC_C64, EREL), (A.AAQ_PREC_C128, 1e-10)):
            lc = A.LightCone(pr, p, obs, with_grad=True, prec=prec)
            e, dg, db, nrm = lc.energy_grad(gam, bet)
            check_energy(e, e_ref, tol)
            check_grad(np.concatenate([dg, db]), np.concatenate([dg_ref, db_ref]), tol)
            assert abs(nrm - 1) <= (1e-5 if prec == A.AAQ_PREC_C64 else 1e-12)
            lc.close()


@pytest.mark.gpu
def test_lightcone_energy_only_and_replays():
    g = G.prufer_tree(18, 7)
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    lc = A.LightCone(pr, 2, OBS_HRED, with_grad=False)
    rng = np.random.default_rng(1)
    for _ in range(3):  # the captured graph replays with new parameters
        gam, bet = rng.uniform(0, math.pi, 2), rng.uniform(0, math.pi / 2, 2)
        e = lc.energy_grad(gam, bet)[0]
        check_energy(e, O.energy(g.n, g.edge_array(), wp.terms(OBS_HRED), gam, bet))
    lc.close()


@pytest.mark.gpu
def test_lightcone_n26_config3_against_light_cone_oracle_and_full_state():
    import torch

    wp, p, gams, bets = config3(2)
    pr = A.Problem.from_workload(wp)
    lc = A.LightCone(pr, p, OBS_HRED, with_grad=True)
    lc_hc = A.LightCone(pr, p, OBS_HC, with_grad=True)
    est = A.Estimator(pr, p, OBS_HRED, A.AAQ_PREC_C64, grad=True)
    for k in range(2):
        e, dg, db, _ = lc.energy_grad(gams[k], bets[k])
        e_lc, dg_lc, db_lc, _ = Rd.light_cone_energy_grad(wp.n, wp.edges(), wp.terms(OBS_HRED), gams[k], bets[k])
        check_energy(e, e_lc)
        check_grad(np.concatenate([dg, db]), np.concatenate([dg_lc, db_lc]))
        e2, dg2, db2, _ = lc_hc.energy_grad(gams[k], bets[k])
        check_energy(e2, e_lc)
        check_grad(np.concatenate([dg2, db2]), np.concatenate([dg_lc, db_lc]))
        ef, dgf, dbf, _ = est.energy_grad(gams[k], bets[k])  # the full 2^26 state on the same GPU
        check_energy(e, ef, 2 * EREL)
        check_grad(np.concatenate([dg, db]), np.concatenate([dgf, dbf]), 2 * GREL)
    lc.close()
    lc_hc.close()
    del est
    torch.cuda.empty_cache()


@pytest.mark.gpu
def test_lightcone_n34_and_n33_configs():
    wp, p, gams, bets = config5a(4)
    pr = A.Problem.from_workload(wp)
    lc = A.LightCone(pr, p, OBS_HRED, with_grad=True)
    for k in range(4):
        e, dg, db, _ = lc.energy_grad(gams[k], bets[k])
        check_energy(e, Rd.p1_energy(wp.n, wp.edges(), wp.terms(OBS_HRED), gams[k, 0], bets[k, 0]))
        _, dg_lc, db_lc, _ = Rd.light_cone_energy_grad(wp.n, wp.edges(), wp.terms(OBS_HRED), gams[k], bets[k])
        check_grad(np.concatenate([dg, db]), np.concatenate([dg_lc, db_lc]))
    lc.close()
    wp, p, gams, bets = config5b(2)
    pr = A.Problem.from_workload(wp)
    for obs in (OBS_HRED, OBS_HC):
        lc = A.LightCone(pr, p, obs, with_grad=True)
        e, dg, db, _ = lc.energy_grad(gams[1], bets[1])
        e_lc, dg_lc, db_lc, _ = Rd.light_cone_energy_grad(wp.n, wp.edges(), wp.terms(obs), gams[1], bets[1])
        check_energy(e, e_lc)
        check_grad(np.concatenate([dg, db]), np.concatenate([dg_lc, db_lc]))
        lc.close()
