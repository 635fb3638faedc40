"""The spin-flip half state (aaq_set_half_state): single-instance and resident evaluations
that store only the amplitudes with bit n-1 = 0 give the full-state results.

CPU: the switch.
GPU: half against full on the same GPU (complex128 to 1e-12 relative, complex64 to the
parity tolerance) and half against the FP64 oracle, over graph sizes with two to four
tile sets (12- and 13-bit tiles), energies, per-term <ZZ>, gradients in both modes,
weighted instances and the resident evaluator; sizes where the half state does not apply
(one tile set, sampling) run unchanged."""
import math

import numpy as np
import pytest

import oracle as O
import paper_2410_22247_amd as A
from workloads import graphs as G
from workloads.configs import OBS_HC, OBS_HRED, make_problem


def test_switch():
    assert A.aaq_get_half_state()
    A.aaq_set_half_state(False)
    assert not A.aaq_get_half_state()
    A.aaq_set_half_state(True)
    assert A.aaq_get_half_state()


def both(fn):
    """fn() with the half state on, then off (restored to on)."""
    try:
        A.aaq_set_half_state(True)
        h = fn()
        A.aaq_set_half_state(False)
        f = fn()
    finally:
        A.aaq_set_half_state(True)
    return h, f


def close(a, b, rel):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return np.all(np.abs(a - b) <= rel * np.maximum(np.abs(b), np.max(np.abs(b)) + 1e-300))


CASES = [(G.binary_tree(13), 2), (G.prufer_tree(16, 3), 3), (G.complete(14), 1), (G.prufer_tree(19, 5), 2),
         (G.star(21), 2), (G.random_regular(3, 22, seed=7), 1), (G.prufer_tree(24, 2), 2)]


@pytest.mark.gpu
@pytest.mark.parametrize("g,p", CASES, ids=lambda x: getattr(x, "name", None) or str(x))
def test_half_equals_full_and_oracle(g, p):
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    rng = np.random.default_rng(g.n * 5 + p)
    gam, bet = rng.uniform(0, math.pi, p), rng.uniform(0, math.pi / 2, p)
    for obs in (OBS_HRED, OBS_HC):
        e_ref, dg_ref, db_ref = O.energy_grad(g.n, g.edge_array(), wp.terms(obs), gam, bet)
        for prec, tol, ftol in ((A.AAQ_PREC_C128, 1e-10, 1e-12), (A.AAQ_PREC_C64, 1e-5, 2e-6)):
            for ckpt in (False, True):
                est = A.Estimator(pr, p, obs, prec, grad=True, checkpoint=ckpt)
                h, f = both(lambda: est.energy_grad(gam, bet))
                gh, gf = np.concatenate([h[1], h[2]]), np.concatenate([f[1], f[2]])
                assert close(h[0], f[0], ftol) and close(gh, gf, ftol) and abs(h[3] - f[3]) < 10 * ftol
                assert abs(h[0] - e_ref) <= tol * abs(e_ref)
                gr = np.concatenate([dg_ref, db_ref])
                assert np.linalg.norm(gh - gr) <= tol * np.linalg.norm(gr)
            est = A.Estimator(pr, p, obs, prec, grad=False)
            h, f = both(lambda: est.energy(gam, bet))
            assert close(h[0], f[0], ftol) and abs(h[0] - e_ref) <= tol * abs(e_ref)


@pytest.mark.gpu
def test_half_per_term_weighted_and_resident():
    import torch

    g = G.prufer_tree(20, 9)
    w = np.random.default_rng(2).integers(1, 4, g.m).astype(np.int32)
    wp = make_problem(g, weights=w)
    pr = A.Problem.from_workload(wp)
    gam, bet = np.array([0.5, 0.9, 0.2]), np.array([0.3, 0.6, 0.1])
    # per-term <ZZ>
    est = A.Estimator(pr, 3, OBS_HC, A.AAQ_PREC_C128, grad=False, agg=A.AAQ_AGG_PER_TERM)
    h, f = both(lambda: est.energy(gam, bet, agg=A.AAQ_AGG_PER_TERM))
    assert close(h[0], f[0], 1e-12) and close(h[1], f[1], 1e-11)
    _, _, zz_ref, _ = O.energy(g.n, g.edge_array(), wp.terms(OBS_HC), gam, bet, full=True, weights=w)
    assert np.max(np.abs(h[1] - zz_ref)) < 1e-10
    # weighted gradient (run-time sweep path) and the resident evaluator
    e_ref, dg_ref, db_ref = O.energy_grad(g.n, g.edge_array(), wp.terms(OBS_HRED), gam, bet, weights=w)
    for prec, tol in ((A.AAQ_PREC_C128, 1e-10), (A.AAQ_PREC_C64, 1e-5)):
        r = A.Resident(pr, 3, OBS_HRED, with_grad=True, checkpoint=True, prec=prec)
        e, dg, db, nrm = r.energy_grad(gam, bet)
        assert abs(e - e_ref) <= tol * abs(e_ref)
        scale = max(np.linalg.norm(np.concatenate([dg_ref, db_ref])), abs(e_ref) if prec == A.AAQ_PREC_C64 else 0)
        assert np.linalg.norm(np.concatenate([dg - dg_ref, db - db_ref])) <= tol * scale
        r.close()
    torch.cuda.synchronize()


@pytest.mark.gpu
def test_half_does_not_apply_to_small_or_sampling():
    """One tile set (n <= 12) and sampling run the full state whatever the switch says."""
    g = G.binary_tree(11)
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    est = A.Estimator(pr, 2, OBS_HRED, A.AAQ_PREC_C128, grad=True)
    h, f = both(lambda: est.energy_grad([0.3, 0.4], [0.5, 0.6]))
    assert h[0] == f[0]
    g2 = G.prufer_tree(16, 4)
    pr2 = A.Problem.from_workload(make_problem(g2))
    u = np.random.default_rng(0).random(500)
    s = A.Sampler(pr2, 2, u.size)
    h, f = both(lambda: s.sample([0.3, 0.4], [0.5, 0.6], u))
    assert np.array_equal(h[0], f[0]) and np.array_equal(h[1], f[1])


@pytest.mark.gpu
def test_n26_energy_both_state_modes():
    """The n = 26, p = 4 tree, energy only: the half state (one 256 MiB state, default-policy
    loads) and the full state (512 MiB, non-temporal loads) both give the light-cone FP64
    value, and agree with each other within rounding."""
    import torch

    from oracle import reduced as Rd
    from workloads.configs import config3

    wp, p, gams, bets = config3(1)
    pr = A.Problem.from_workload(wp)
    est = A.Estimator(pr, p, OBS_HRED, A.AAQ_PREC_C64, grad=False)
    h, f = both(lambda: est.energy(gams[0], bets[0]))
    e_ref = Rd.light_cone_energy(wp.n, wp.edges(), wp.terms(OBS_HRED), gams[0], bets[0])
    for e in (h[0], f[0]):
        assert abs(e - e_ref) <= 1e-5 * abs(e_ref), (e, e_ref)
    assert abs(h[0] - f[0]) <= 2e-6 * abs(e_ref)
    del est
    torch.cuda.empty_cache()


@pytest.mark.gpu
@pytest.mark.parametrize("n,p,prec", [(30, 1, A.AAQ_PREC_C64), (31, 1, A.AAQ_PREC_C64), (29, 1, A.AAQ_PREC_C128)],
                         ids=["c64-n30-full", "c64-n31-64bit", "c128-n29-full"])
def test_half_state_with_64bit_addresses(n, p, prec):
    """States whose stored half exceeds 4 GiB (n = 31 in complex64) take 64-bit addresses
    with the mirrored registers; n = 30 (complex64) and n = 29 (complex128), whose full
    index range exceeds 4 GiB but whose half does not, keep the full state.  Energy and
    gradient with the switch on and off, against each other and the light-cone FP64
    adjoint."""
    import torch
    from oracle import reduced as Rd

    g = G.prufer_tree(n, 7)
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    gam, bet = np.array([0.83]), np.array([0.37])
    e_lc, dg_lc, db_lc, _ = Rd.light_cone_energy_grad(n, wp.edges(), wp.terms(OBS_HRED), gam, bet)
    tol = 1e-5 if prec == A.AAQ_PREC_C64 else 1e-10

    def run():
        est = A.Estimator(pr, p, OBS_HRED, prec, grad=True)
        r = est.energy_grad(gam, bet)
        del est
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        return r

    h, f = both(run)
    for e, dg, db, nrm in (h, f):
        assert abs(e - e_lc) <= tol * abs(e_lc)
        gr, gv = np.concatenate([dg_lc, db_lc]), np.concatenate([dg, db])
        assert np.linalg.norm(gv - gr) <= tol * np.linalg.norm(gr)
        assert abs(nrm - 1) <= (1e-5 if prec == A.AAQ_PREC_C64 else 1e-12)
