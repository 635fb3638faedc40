"""Resident evaluator (aaq_resident_*): the fused evaluation with device parameters and
device outputs, queued without host synchronisation.

CPU: sizes and the argument checks (no device work).
GPU: against the FP64 oracle (energy, norm, gradient; complex64 and complex128; with and
without forward-state checkpoints; weighted); many executions queued back to back with
different parameter rows give, row by row, the synchronous host API's results; the
energy-only evaluator leaves the gradient entries 0; the n = 26, p = 4 tree against the
light-cone FP64 adjoint."""
import math

import numpy as np
import pytest

import oracle as O
import paper_2410_22247_amd as A
from oracle import reduced as Rd
from workloads import graphs as G
from workloads.configs import OBS_HC, OBS_HRED, config3, make_problem

EREL = 1e-5


def check(e, dg, db, e_ref, dg_ref, db_ref, tol):
    """Energy relative error; gradient normwise relative to ||g_ref||."""
    assert abs(e - e_ref) <= tol * abs(e_ref), (e, e_ref)
    g, gr = np.concatenate([dg, db]), np.concatenate([dg_ref, db_ref])
    scale = max(np.linalg.norm(gr), 1e-12)
    assert np.linalg.norm(g - gr) <= tol * scale, (g, gr)


# ------------------------------------------------------------------ host (CPU)
def test_resident_sizes_and_errors():
    g = G.prufer_tree(20, 2)
    pr = A.Problem.from_workload(make_problem(g))
    wb, sb = A.aaq_resident_workspace_size(pr, 3, OBS_HRED, True, False)
    assert wb > 0 and sb == A.aaq_state_bytes(pr, A.AAQ_PREC_C64)
    wbc, sbc = A.aaq_resident_workspace_size(pr, 3, OBS_HRED, True, True)
    assert sb < sbc <= A.aaq_checkpoint_bytes(pr, 3, A.AAQ_PREC_C64)  # the chosen tile size only
    with pytest.raises(A.AAQError) as e:
        A.aaq_resident_workspace_size(pr, 0, OBS_HRED, True, False)
    assert e.value.status == 1
    with pytest.raises(A.AAQError) as e:  # NULL buffers are refused before any device work
        A.aaq_resident_create(pr, 3, OBS_HRED, True, False, A.AAQ_PREC_C64, None, None, None, stream=0)
    assert e.value.status == 1
    with pytest.raises(A.AAQError) as e:
        A.aaq_resident_execute(None, None, None, stream=0)
    assert e.value.status == 1


# ------------------------------------------------------------------ GPU
CASES = [(G.binary_tree(13), 2, None), (G.prufer_tree(16, 3), 3, None), (G.complete(10), 2, None),
         (G.prufer_tree(21, 8), 2, None), (G.binary_tree(15), 2, "w")]


@pytest.mark.gpu
@pytest.mark.parametrize("g,p,w", CASES, ids=lambda x: getattr(x, "name", None) or str(x))
def test_resident_matches_oracle(g, p, w):
    weights = None if w is None else np.random.default_rng(3).integers(1, 4, g.m).astype(np.int32)
    wp = make_problem(g, weights=weights)
    pr = A.Problem.from_workload(wp)
    rng = np.random.default_rng(g.n + 5 * p)
    gam, bet = rng.uniform(0, math.pi / 2, p), rng.uniform(0, math.pi / 2, p)
    for obs in (OBS_HRED, OBS_HC):
        e_ref, dg_ref, db_ref = O.energy_grad(g.n, g.edge_array(), wp.terms(obs), gam, bet, weights=weights)
        for prec, tol in ((A.AAQ_PREC_C128, 1e-10), (A.AAQ_PREC_C64, EREL)):
            for ckpt in (False, True):
                r = A.Resident(pr, p, obs, with_grad=True, checkpoint=ckpt, prec=prec)
                e, dg, db, nrm = r.energy_grad(gam, bet)
                check(e, dg, db, e_ref, dg_ref, db_ref, tol)
                assert abs(nrm - 1) <= (1e-12 if prec == A.AAQ_PREC_C128 else 1e-5)
                r.close()


@pytest.mark.gpu
def test_resident_queued_rows_equal_host_api():
    """40 executions queued back to back (new parameter row and output row each, no
    synchronisation between them) give the host API's results for the same points."""
    import torch

    g = G.prufer_tree(22, 4)
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    p = 3
    rng = np.random.default_rng(8)
    gam, bet = rng.uniform(0, math.pi, (40, p)), rng.uniform(0, math.pi / 2, (40, p))
    params = torch.from_numpy(np.concatenate([gam, bet], 1)).cuda()
    out = torch.zeros(40, 2 + 2 * p, dtype=torch.float64, device="cuda")
    for ckpt in (True, False):
        r = A.Resident(pr, p, OBS_HRED, with_grad=True, checkpoint=ckpt)
        est = A.Estimator(pr, p, OBS_HRED, A.AAQ_PREC_C64, grad=True, checkpoint=ckpt)
        out.zero_()
        for k in range(40):
            r.execute(params[k], out[k])
        got = out.cpu().numpy()
        for k in range(40):
            e, dg, db, nrm = est.energy_grad(gam[k], bet[k])
            # the same kernels in the same order: identical results
            assert np.array_equal(got[k], np.concatenate([[e, nrm], dg, db])), k
        r.close()


@pytest.mark.gpu
def test_resident_energy_only():
    g = G.binary_tree(15)
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    gam, bet = np.array([0.4, 0.8]), np.array([0.3, 0.6])
    r = A.Resident(pr, 2, OBS_HC, with_grad=False)
    e, dg, db, nrm = r.energy_grad(gam, bet)
    assert abs(e - O.energy(g.n, g.edge_array(), wp.terms(OBS_HC), gam, bet)) <= EREL * abs(e)
    assert not np.any(dg) and not np.any(db) and abs(nrm - 1) < 1e-5
    r.close()


@pytest.mark.gpu
def test_resident_n26_config3():
    import torch

    wp, p, gams, bets = config3(2)
    pr = A.Problem.from_workload(wp)
    r = A.Resident(pr, p, OBS_HRED, with_grad=True, checkpoint=True)
    for k in range(2):
        e, dg, db, _ = r.energy_grad(gams[k], bets[k])
        e_lc, dg_lc, db_lc, _ = Rd.light_cone_energy_grad(wp.n, wp.edges(), wp.terms(OBS_HRED), gams[k], bets[k])
        check(e, dg, db, e_lc, dg_lc, db_lc, EREL)
    r.close()
    del r
    torch.cuda.empty_cache()


@pytest.mark.gpu
def test_resident_adam_matches_host_adam():
    """The device-resident Adam loop follows the host-API loop (identical gradients per
    evaluation; only the optimizer's own rounding on GPU vs CPU can differ) and raises
    the expected cut."""
    from paper_2410_22247_amd.autograd import adam_maximize, adam_maximize_resident

    g = G.binary_tree(15)
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    r = A.Resident(pr, 2, OBS_HRED, with_grad=True)
    est = A.Estimator(pr, 2, OBS_HRED, A.AAQ_PREC_C64, grad=True)
    g_r, b_r, h_r = adam_maximize_resident(r, [0.4, 0.9], [0.6, 0.3], steps=30, lr=0.05)
    g_h, b_h, h_h = adam_maximize(est, [0.4, 0.9], [0.6, 0.3], steps=30, lr=0.05)
    assert np.max(np.abs(h_r[:, 0] - h_h)) <= 1e-9 * np.max(np.abs(h_h))
    assert np.allclose(np.concatenate([g_r, b_r]), np.concatenate([g_h, b_h]), rtol=0, atol=1e-9)
    assert h_r[-1, 0] > h_r[0, 0] + 0.5
    e_end = O.energy(g.n, g.edge_array(), wp.terms(OBS_HRED), g_r, b_r)
    e_dev = r.energy_grad(g_r, b_r)[0]
    assert abs(e_dev - e_end) <= EREL * abs(e_end)
    r.close()
