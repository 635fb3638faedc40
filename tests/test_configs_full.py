"""The measured configurations at full size, every point and instance, on the GPU.

* Orbit-reduction diagnostics (K_16 p=1, star n=20 p=2, the networkx 3-regular graph
  n=22 p=3): all 256 seeded points, both observables, complex64, through the batched plan
  the benchmark times and through single-instance calls; K_16 against the Dicke-subspace
  oracle, the star against the hub x Dicke oracle, the 3-regular graph against the stored
  full-state FP64 oracle energies.
* Adjoint gradients (Pruefer tree n=26, p=4, H_red): all 32 seeded points through the
  device-resident evaluator with forward-state checkpoints (the benchmark's launch
  configuration): energy and gradient against the stored light-cone FP64 adjoint, the
  gradient against the stored central finite differences (h = 1e-4) of the light-cone FP64
  energy, and against the layer-level parameter-shift rule (Wierichs, Izaac, Wang, Lin,
  Quantum 6, 677 (2022)) evaluated with complex128 energies of the same GPU path.
* Batched mixed workload (512 instances, n = 8..18, p=2, H_red energy + gradient): every
  instance through a plan built with the options aaq_plan_autotune picks, replayed as a HIP
  graph, against the stored FP64 oracle values, and equal to single-instance calls.

Stored values: tests/golden/make_references.py (FP64 oracle only).  Tolerances: energies
1e-5 relative; gradients 1e-5 of ||g_ref|| normwise and per component 1e-5 of
max(|g_ref,k|, ||g_ref||); the finite differences carry their own truncation error
(stated at the test).  Each test records its observed maximum errors as junit properties.
"""
import json
import math
import os

import numpy as np
import pytest

import paper_2410_22247_amd as A
from oracle import derivs as D
from oracle import reduced as Rd
from workloads import configs as C
from workloads.configs import OBS_HC, OBS_HRED

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
EREL = GREL = 1e-5


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def rel_energy(e, ref):
    return np.abs(np.asarray(e) - np.asarray(ref)) / np.maximum(np.abs(np.asarray(ref)), 1e-12)


def grad_errors(g, ref):
    """(normwise relative error, max per-component error relative to max(|ref_k|, ||ref||))."""
    g, ref = np.asarray(g, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    nrm = max(np.linalg.norm(ref), 1e-300)
    return (float(np.linalg.norm(g - ref) / nrm),
            float(np.max(np.abs(g - ref) / np.maximum(np.abs(ref), nrm))))


# ------------------------------------------------------------------ orbit-reduction diagnostics
def _c2_reference(name, wp, gam, bet, obs):
    if name == "K16":
        return np.array([Rd.complete_graph_energy(16, gam[i], bet[i]) for i in range(gam.shape[0])])
    if name == "star20":
        return np.array([Rd.star_energy(19, gam[i], bet[i]) for i in range(gam.shape[0])])
    d = _load("random_regular_3_22_seed7.json")
    assert sorted(map(tuple, wp.edges().tolist())) == sorted(map(tuple, d["edges"]))
    return np.asarray(d["energy_hc" if obs == OBS_HC else "energy_hred"])


@pytest.mark.parametrize("cfg", C.config2(), ids=lambda c: c[0])
def test_orbit_diagnostics_all_points(cfg, record_property):
    name, wp, p, gam, bet = cfg
    pr = A.Problem.from_workload(wp)
    worst = 0.0
    for obs in (OBS_HC, OBS_HRED):
        ref = _c2_reference(name, wp, gam, bet, obs)
        plan = A.Plan([pr] * gam.shape[0], p, obs, with_grad=False)
        plan.params.copy_(torch.from_numpy(np.concatenate([gam, bet], 1)))
        for _ in range(2):  # graph replays
            out = plan.execute().cpu().numpy()
            err = rel_energy(out[:, 0], ref)
            assert err.max() <= EREL, (name, obs, err.max(), int(err.argmax()))
            assert np.max(np.abs(out[:, 1] - 1)) <= 1e-5
        plan.close()
        worst = max(worst, float(err.max()))
        est = A.Estimator(pr, p, obs, A.AAQ_PREC_C64, grad=False)
        single = np.array([est.energy(gam[i], bet[i])[0] for i in range(gam.shape[0])])
        err_s = rel_energy(single, ref)
        assert err_s.max() <= EREL, (name, obs, err_s.max(), int(err_s.argmax()))
        worst = max(worst, float(err_s.max()))
        del est
    record_property("max_rel_err_energy", worst)


# ------------------------------------------------------------------ adjoint gradients, n = 26
@pytest.fixture(scope="module")
def tree26():
    wp, p, gam, bet = C.config3(32)
    ref = _load("tree26_p4_references.json")["points"]
    assert len(ref) == 32
    for k, r in enumerate(ref):  # the stored points are the seeded ones
        assert np.allclose(r["gamma"], gam[k], rtol=0, atol=0) and np.allclose(r["beta"], bet[k], rtol=0, atol=0)
    return wp, p, gam, bet, ref


@pytest.fixture(scope="module")
def tree26_adjoint(tree26):
    """The complex64 energy + adjoint gradient at the 32 points, in the benchmark's launch
    configuration (device-resident, forward-state checkpoints, spin-flip half state)."""
    wp, p, gam, bet, _ = tree26
    res = A.Resident(A.Problem.from_workload(wp), p, OBS_HRED, with_grad=True, checkpoint=True)
    prm = torch.from_numpy(np.concatenate([gam, bet], 1)).cuda()
    out = torch.zeros(32, 2 + 2 * p, dtype=torch.float64, device="cuda")
    for k in range(32):  # queued without synchronisation, as the benchmark runs them
        res.execute(params=prm[k], out=out[k])
    o = out.cpu().numpy()
    res.close()
    del res
    torch.cuda.empty_cache()
    return o


def test_tree26_all_points_vs_light_cone_adjoint(tree26, tree26_adjoint, record_property):
    wp, p, gam, bet, ref = tree26
    o = tree26_adjoint
    e_ref = np.array([r["energy_lc"] for r in ref])
    g_ref = np.array([r["dgamma_lc"] + r["dbeta_lc"] for r in ref])
    err_e = rel_energy(o[:, 0], e_ref)
    errs = [grad_errors(o[k, 2:], g_ref[k]) for k in range(32)]
    record_property("max_rel_err_energy", float(err_e.max()))
    record_property("max_rel_err_grad_normwise", max(e[0] for e in errs))
    record_property("max_rel_err_grad_component", max(e[1] for e in errs))
    assert err_e.max() <= EREL, (err_e.max(), int(err_e.argmax()))
    assert max(e[0] for e in errs) <= GREL and max(e[1] for e in errs) <= GREL, errs
    assert np.max(np.abs(o[:, 1] - 1)) <= 1e-5


def test_tree26_all_points_vs_finite_differences(tree26, tree26_adjoint, record_property):
    """Central differences of the FP64 light-cone energy with h = 1e-4 carry a truncation
    error h^2 |f'''| / 6 per component; the stored values agree with the exact light-cone
    adjoint within 3.6e-8 of ||g|| (checked on the CPU by test_golden_references), so the
    1e-5 bound applies to the complex64 adjoint unchanged."""
    wp, p, gam, bet, ref = tree26
    o = tree26_adjoint
    g_fd = np.array([r["dgamma_fd"] + r["dbeta_fd"] for r in ref])
    errs = [grad_errors(o[k, 2:], g_fd[k]) for k in range(32)]
    record_property("max_rel_err_grad_normwise", max(e[0] for e in errs))
    assert max(e[0] for e in errs) <= GREL and max(e[1] for e in errs) <= GREL, errs


def test_tree26_all_points_vs_parameter_shift_complex128(tree26, tree26_adjoint, record_property):
    """Layer-level parameter shift: gamma_l's generator C(z) has integer spectrum 0..|E|
    (R = |E| frequencies), beta_l's generator sum_q X_q has eigenvalues n - 2k, i.e. R = n
    frequencies in x = 2 beta.  The shifted energies are complex128 evaluations of the same
    sweeps (Sum |coef| = R amplifies their rounding, so complex64 energies would not do)."""
    wp, p, gam, bet, ref = tree26
    m, n = wp.m, wp.n
    xg, cg = D.shift_points(m)
    xb, cb = D.shift_points(n)
    res = A.Resident(A.Problem.from_workload(wp), p, OBS_HRED, with_grad=False, checkpoint=False,
                     prec=A.AAQ_PREC_C128)
    worst, worst_ref = 0.0, 0.0
    for k in range(32):
        rows = []
        for l in range(p):
            for x in xg:
                g = gam[k].copy()
                g[l] += x
                rows.append(np.concatenate([g, bet[k]]))
        for l in range(p):
            for x in xb:
                b = bet[k].copy()
                b[l] += x / 2
                rows.append(np.concatenate([gam[k], b]))
        prm = torch.from_numpy(np.asarray(rows)).cuda()
        out = torch.zeros(len(rows), 2 + 2 * p, dtype=torch.float64, device="cuda")
        for r in range(len(rows)):
            res.execute(params=prm[r], out=out[r])
        e = out[:, 0].cpu().numpy()
        eg, eb = e[:p * len(xg)].reshape(p, -1), e[p * len(xg):].reshape(p, -1)
        dg = np.array([np.dot(cg, eg[l]) for l in range(p)])
        db = np.array([2 * np.dot(cb, eb[l]) for l in range(p)])
        g_shift = np.concatenate([dg, db])
        # the shift rule itself against the exact FP64 light-cone adjoint
        wr = grad_errors(g_shift, ref[k]["dgamma_lc"] + ref[k]["dbeta_lc"])[0]
        assert wr <= 1e-9, (k, wr)
        err = grad_errors(tree26_adjoint[k, 2:], g_shift)
        assert err[0] <= GREL and err[1] <= GREL, (k, err)
        worst, worst_ref = max(worst, err[0]), max(worst_ref, wr)
    res.close()
    record_property("max_rel_err_grad_normwise", worst)
    record_property("shift_c128_vs_light_cone_adjoint", worst_ref)


# ------------------------------------------------------------------ batched mixed workload
def test_mixed512_every_instance_autotuned_plan(record_property):
    probs, p, gam, bet = C.config4()
    ref = _load("mixed512_p2_references.json")["units"]
    assert [r["n"] for r in ref] == [w.n for w in probs]
    prs = [A.Problem.from_workload(w) for w in probs]
    prm = np.concatenate([gam, bet], 1)
    plan = A.Plan.autotuned(prs, p, OBS_HRED, True, params=prm, reps=2)
    plan.params.copy_(torch.from_numpy(prm))
    e_ref = np.array([r["energy"] for r in ref])
    g_ref = np.array([r["dgamma"] + r["dbeta"] for r in ref])
    for _ in range(3):  # graph replays with eager work in between
        out = plan.execute().cpu().numpy()
        plan.params.mul_(1.0)
        err_e = rel_energy(out[:, 0], e_ref)
        errs = np.array([grad_errors(out[u, 2:], g_ref[u]) for u in range(len(prs))])
        assert err_e.max() <= EREL, (err_e.max(), int(err_e.argmax()))
        assert errs[:, 0].max() <= GREL and errs[:, 1].max() <= GREL, (errs.max(0), errs.argmax(0))
        assert np.max(np.abs(out[:, 1] - 1)) <= 1e-5
    plan.close()
    record_property("tuned_opts", json.dumps(plan.tuned_opts))
    record_property("max_rel_err_energy", float(err_e.max()))
    record_property("max_rel_err_grad_normwise", float(errs[:, 0].max()))
    # the same instances through single-instance calls (the plain loop the plan is timed against)
    ests = {}
    single = np.zeros_like(out)
    for u, w in enumerate(probs):
        key = (w.n, tuple(w.graph.edges))
        if key not in ests:
            ests[key] = A.Estimator(prs[u], p, OBS_HRED, A.AAQ_PREC_C64, grad=True)
        e, dg, db, nrm = ests[key].energy_grad(gam[u], bet[u])
        single[u] = np.concatenate([[e, nrm], dg, db])
    err_s = rel_energy(single[:, 0], e_ref)
    errs_s = np.array([grad_errors(single[u, 2:], g_ref[u]) for u in range(len(prs))])
    assert err_s.max() <= EREL and errs_s[:, 0].max() <= GREL and errs_s[:, 1].max() <= GREL
    # batched and single calls run the same arithmetic up to the tile shapes: within the tolerance
    diff = rel_energy(out[:, 0], single[:, 0])
    assert diff.max() <= 2 * EREL
