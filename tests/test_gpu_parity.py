"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (the accuracy target of the complex64 path, normwise reading for
gradients whose components can vanish):
  energies   |E - E_ref| <= 1e-5 |E_ref|           (complex128: 1e-10)
  gradients  ||g - g_ref|| <= 1e-5 ||g_ref|| and per component
             |g_k - g_ref,k| <= 1e-5 max(|g_ref,k|, ||g_ref||)
  <ZZ>       absolute 1e-5
  cut values bit-exact
"""
import math

import numpy as np
import pytest

import oracle as O
import paper_2410_22247_amd as A
from oracle import reduced as Rd
from workloads import graphs as G
from workloads.configs import OBS_HC, OBS_HRED, make_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EREL = 1e-5
GREL = 1e-5


def dev_bytes(nbytes):
    return torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")


def rand_graph(n, pe, seed):
    rng = np.random.default_rng(seed)
    es = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < pe]
    return G.Graph(n, es or [(0, 1)], name=f"G({n},{pe},{seed})")


def check_energy(e, ref, rel=EREL):
    assert abs(e - ref) <= rel * max(abs(ref), 1e-12), (e, ref, abs(e - ref) / max(abs(ref), 1e-12))


def check_grad(g, ref, rel=GREL):
    g, ref = np.asarray(g), np.asarray(ref)
    nrm = np.linalg.norm(ref)
    assert np.linalg.norm(g - ref) <= rel * max(nrm, 1e-12), (g, ref)
    assert np.all(np.abs(g - ref) <= rel * np.maximum(np.abs(ref), nrm) + 1e-14), (g, ref)


# ------------------------------------------------------------------ cut values (bit-exact)
CUT_GRAPHS = [G.binary_tree(5), rand_graph(9, 0.5, 1), G.complete(13), G.star(13), G.prufer_tree(14, 3),
              G.generalized_petersen(8, 3), rand_graph(17, 0.3, 2), G.random_regular(3, 22, seed=7)]


@pytest.mark.parametrize("g", CUT_GRAPHS, ids=lambda g: f"{g.name}-n{g.n}")
def test_cut_values_bit_exact_every_layout(g):
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    ws = dev_bytes(1 << 16)
    out = torch.empty(1 << g.n, dtype=torch.int32, device="cuda")
    ref_c = O.cut_values(g.n, g.edge_array())
    ref_h = O.term_values(g.n, wp.terms(OBS_HRED)).astype(np.int64)
    for prec in (A.AAQ_PREC_C64, A.AAQ_PREC_C128):
        for s in range(A.aaq_num_sets(g.n, prec)):
            for arr in (0, 1):
                for obs, ref in ((A.AAQ_OBS_HC, ref_c), (A.AAQ_OBS_HRED, ref_h)):
                    out.fill_(-1)
                    A.aaq_cut_values_layout(pr, obs, s, arr, prec, ws, out)
                    got = out.cpu().numpy()
                    assert np.array_equal(got, ref), (prec, s, arr, obs)
    out.fill_(-1)
    A.aaq_cut_values(pr, A.AAQ_OBS_HC, ws, out)
    assert np.array_equal(out.cpu().numpy(), ref_c)


def test_cut_values_bit_exact_every_layout_large():
    """n = 28, whose high tile sets each hold one of qubits 26 and 27 beside a run of other
    qubits (13-bit tiles, three sets): every set, arrangement, observable and precision
    against the oracle over all 2^28 indices (the comparison runs on the device against
    the oracle's values copied there)."""
    n = 28
    g = G.prufer_tree(n, 40 + n)
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    ref_c = torch.from_numpy(O.cut_values(g.n, g.edge_array())).cuda()
    ref_h = torch.from_numpy(O.term_values(g.n, wp.terms(OBS_HRED)).astype(np.int32)).cuda()
    ws = dev_bytes(1 << 16)
    out = torch.empty(1 << g.n, dtype=torch.int32, device="cuda")
    assert A.aaq_num_sets(n) == 3
    for prec in (A.AAQ_PREC_C64, A.AAQ_PREC_C128):
        for s in range(A.aaq_num_sets(n, prec)):
            for arr in (0, 1):
                for obs, ref in ((A.AAQ_OBS_HC, ref_c), (A.AAQ_OBS_HRED, ref_h)):
                    out.fill_(-1)
                    A.aaq_cut_values_layout(pr, obs, s, arr, prec, ws, out)
                    assert torch.equal(out, ref), (prec, s, arr, obs)
    del out, ref_c, ref_h
    torch.cuda.empty_cache()


@pytest.mark.parametrize("g", [G.prufer_tree(33, 5), G.prufer_tree(34, 5), rand_graph(33, 0.3, 7)],
                         ids=lambda g: f"{g.name or 'tree'}-n{g.n}")
def test_cut_values_64bit_sampled(g):
    """n > 32, where index masks take 64 bits and the tile's uniform part of C(z) is formed
    across the wave (one lane per vertex): every set, arrangement, observable and precision
    dumped whole (32 or 64 GiB), 2^20 seeded indices against the oracle's per-index values,
    and the complement symmetry C(z) = C(~z) over every index on the device.  The dense
    graph (144 edges) puts edges among the thread-bit vertices and between them and the
    register bits, which trees rarely do."""
    n = g.n
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    rng = np.random.default_rng(100 + n)
    idx = rng.integers(0, 1 << n, 1 << 20, dtype=np.uint64)
    ref_c = O.cut_values_at(idx, g.edge_array())
    ref_h = O.term_values_at(idx, wp.terms(OBS_HRED))
    didx = torch.from_numpy(idx.astype(np.int64)).cuda()
    ws = dev_bytes(1 << 16)
    out = torch.empty(1 << n, dtype=torch.int32, device="cuda")
    chunk = 1 << 28
    N = 1 << n
    for prec in (A.AAQ_PREC_C64, A.AAQ_PREC_C128):
        for s in range(A.aaq_num_sets(n, prec)):
            for arr in (0, 1):
                for obs, ref in ((A.AAQ_OBS_HC, ref_c), (A.AAQ_OBS_HRED, ref_h)):
                    out.fill_(-1)
                    A.aaq_cut_values_layout(pr, obs, s, arr, prec, ws, out)
                    got = out[didx].cpu().numpy()
                    assert np.array_equal(got.astype(np.float64), np.asarray(ref, dtype=np.float64)), (prec, s, arr, obs)
                    for a in range(0, N // 2, chunk):
                        assert torch.equal(out[a:a + chunk], out[N - a - chunk:N - a].flip(0)), (prec, s, arr, obs, a)
    del out, didx
    torch.cuda.empty_cache()


# ------------------------------------------------------------------ energies
ENERGY_CASES = [
    (G.Graph(1, []), 1), (G.Graph(2, [(0, 1)]), 2), (G.binary_tree(5), 3), (rand_graph(8, 0.5, 4), 2),
    (G.complete(12), 1), (G.binary_tree(13), 2), (G.prufer_tree(14, 1), 3), (G.star(16), 2),
    (G.generalized_petersen(9, 2), 2), (G.prufer_tree(20, 6), 3), (rand_graph(22, 0.15, 9), 1),
]


@pytest.mark.parametrize("g,p", ENERGY_CASES, ids=lambda x: getattr(x, "name", str(x)))
def test_energy_matches_oracle(g, p):
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    rng = np.random.default_rng(g.n * 31 + p)
    gam, bet = rng.uniform(0, math.pi, p), rng.uniform(0, math.pi / 2, p)
    st = dev_bytes(A.aaq_state_bytes(pr, A.AAQ_PREC_C128))
    for obs in (OBS_HC, OBS_HRED):
        ref = O.energy(g.n, g.edge_array(), wp.terms(obs), gam, bet) if g.m else 0.0
        for prec, tol in ((A.AAQ_PREC_C64, EREL), (A.AAQ_PREC_C128, 1e-10)):
            ws = dev_bytes(A.aaq_workspace_size(pr, p, False, obs, A.AAQ_AGG_FUSED, prec))
            e, _, nrm = A.aaq_energy(pr, gam, bet, obs, A.AAQ_AGG_FUSED, prec, st, ws)
            if g.m:
                check_energy(e, ref, tol)
            else:
                assert e == 0.0
            assert abs(nrm - 1) <= (1e-5 if prec == A.AAQ_PREC_C64 else 1e-12)


def test_energy_hred_equals_hc_and_closed_form():
    g = G.binary_tree(15)
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    est = A.Estimator(pr, 1, A.AAQ_OBS_HRED, A.AAQ_PREC_C128, grad=False)
    for gam, bet in [(math.pi / 3, math.pi / 8), (0.4, 1.3)]:
        cf = 7 + 0.25 * math.sin(4 * bet) * math.sin(gam) * (8 + 2 * math.cos(gam) + 18 * math.cos(gam) ** 2)
        eh = est.energy([gam], [bet], obs=A.AAQ_OBS_HC)[0]
        er = est.energy([gam], [bet], obs=A.AAQ_OBS_HRED)[0]
        assert abs(eh - cf) < 1e-11 and abs(er - cf) < 1e-11


@pytest.mark.parametrize("agg", [A.AAQ_AGG_PER_TERM, A.AAQ_AGG_PASS_PER_TERM], ids=["per_term", "pass_per_term"])
@pytest.mark.parametrize("g,p", [(G.binary_tree(11), 2), (G.complete(16), 1), (G.prufer_tree(18, 2), 2)],
                         ids=["tree11", "K16", "prufer18"])
def test_per_term_aggregation(agg, g, p):
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    rng = np.random.default_rng(5)
    gam, bet = rng.uniform(0, math.pi, p), rng.uniform(0, math.pi / 2, p)
    est = A.Estimator(pr, p, A.AAQ_OBS_HC, A.AAQ_PREC_C64, grad=False, agg=agg)
    for obs in (OBS_HC, OBS_HRED):
        e_ref, _, zz_ref, _ = O.energy(g.n, g.edge_array(), wp.terms(obs), gam, bet, full=True)
        e, zz, _ = est.energy(gam, bet, obs=obs, agg=agg)
        assert np.max(np.abs(zz - zz_ref)) <= 1e-5
        check_energy(e, e_ref)
    # Eq. A3 on the device: per-edge <ZZ> equal within every orbit
    _, zz, _ = est.energy(gam, bet, obs=OBS_HC, agg=agg)
    for orb in wp.orbits.orbits:
        assert np.ptp(zz[orb]) <= 2e-6


def test_per_term_reduction_is_bitwise_deterministic():
    """Per-term <ZZ> sums are added in a fixed order (waves in turn, then tiles in order):
    repeated calls give identical bits, for both observables and tile sizes."""
    g = G.prufer_tree(20, 5)
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    gam, bet = np.array([0.9, 2.3]), np.array([0.4, 1.2])
    for obs in (OBS_HC, OBS_HRED):
        for tile in (12, 13):
            A.aaq_set_tile_bits(g.n, A.AAQ_PREC_C64, False, tile)
            try:
                est = A.Estimator(pr, 2, obs, A.AAQ_PREC_C64, grad=False, agg=A.AAQ_AGG_PER_TERM)
                runs = [est.energy(gam, bet) for _ in range(3)]
            finally:
                A.aaq_set_tile_bits(g.n, A.AAQ_PREC_C64, False, 0)
            for e, zz, nrm in runs[1:]:
                assert e == runs[0][0] and nrm == runs[0][2] and np.array_equal(zz, runs[0][1])
            zz_ref = O.energy(g.n, g.edge_array(), wp.terms(obs), gam, bet, full=True)[2]
            assert np.max(np.abs(runs[0][1] - zz_ref)) <= 1e-5


# ------------------------------------------------------------------ gradients
GRAD_CASES = [
    (G.Graph(2, [(0, 1)]), 1), (G.binary_tree(6), 2), (rand_graph(9, 0.5, 2), 3), (G.complete(10), 2),
    (G.binary_tree(13), 1), (G.prufer_tree(14, 5), 2), (G.star(17), 3), (G.prufer_tree(21, 8), 2),
]


@pytest.mark.parametrize("g,p", GRAD_CASES, ids=lambda x: getattr(x, "name", str(x)))
def test_energy_grad_matches_oracle_adjoint(g, p):
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    rng = np.random.default_rng(g.n * 7 + p)
    gam, bet = rng.uniform(0, math.pi, p), rng.uniform(0, math.pi / 2, p)
    for obs in (OBS_HRED, OBS_HC):
        e_ref, dg_ref, db_ref = O.energy_grad(g.n, g.edge_array(), wp.terms(obs), gam, bet)
        est = A.Estimator(pr, p, obs, A.AAQ_PREC_C64, grad=True)
        e, dg, db, nrm = est.energy_grad(gam, bet)
        check_energy(e, e_ref)
        check_grad(np.concatenate([dg, db]), np.concatenate([dg_ref, db_ref]))
        assert abs(nrm - 1) < 1e-5


@pytest.mark.parametrize("g,p,prec", [(G.prufer_tree(12, 4), 2, A.AAQ_PREC_C64), (G.prufer_tree(15, 2), 3, A.AAQ_PREC_C64),
                                      (G.star(19), 2, A.AAQ_PREC_C128), (G.prufer_tree(23, 6), 3, A.AAQ_PREC_C64),
                                      (G.random_regular(3, 20, seed=9), 2, A.AAQ_PREC_C64)],
                         ids=["n12", "n15", "star19-c128", "n23", "3reg20"])
def test_checkpointed_gradient(g, p, prec):
    """Forward-state checkpoints give the oracle's energy and gradient, for both tile sizes."""
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    rng = np.random.default_rng(g.n * 13 + p)
    gam, bet = rng.uniform(0, math.pi, p), rng.uniform(0, math.pi / 2, p)
    e_ref, dg_ref, db_ref = O.energy_grad(g.n, g.edge_array(), wp.terms(OBS_HRED), gam, bet)
    tol = 1e-10 if prec == A.AAQ_PREC_C128 else EREL
    est = A.Estimator(pr, p, A.AAQ_OBS_HRED, prec, grad=True, checkpoint=True)
    assert est.state.numel() == A.aaq_checkpoint_bytes(pr, p, prec)
    try:
        for tile in (12, 13):
            A.aaq_set_tile_bits(g.n, prec, True, tile)
            e, dg, db, nrm = est.energy_grad(gam, bet)
            check_energy(e, e_ref, tol)
            check_grad(np.concatenate([dg, db]), np.concatenate([dg_ref, db_ref]), tol)
            assert abs(nrm - 1) < (1e-12 if prec == A.AAQ_PREC_C128 else 1e-5)
    finally:
        A.aaq_set_tile_bits(g.n, prec, True, 0)


def test_energy_grad_complex128():
    g = G.prufer_tree(15, 4)
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    gam, bet = np.array([0.7, 2.1]), np.array([0.3, 1.2])
    e_ref, dg_ref, db_ref = O.energy_grad(g.n, g.edge_array(), wp.terms(OBS_HRED), gam, bet)
    est = A.Estimator(pr, 2, OBS_HRED, A.AAQ_PREC_C128, grad=True)
    e, dg, db, _ = est.energy_grad(gam, bet)
    check_energy(e, e_ref, 1e-11)
    check_grad(np.concatenate([dg, db]), np.concatenate([dg_ref, db_ref]), 1e-10)


def test_energy_grad_n26_config3_point():
    """Full configuration-3 size (n = 26, p = 4, 2^26 amplitudes): gradient against
    the light-cone FP64 adjoint (exact for the QAOA state), energy also against the
    full-state oracle at one point."""
    from workloads.configs import config3

    wp, p, gams, bets = config3(2)
    pr = A.Problem.from_workload(wp)
    est = A.Estimator(pr, p, OBS_HRED, A.AAQ_PREC_C64, grad=True)
    terms = wp.terms(OBS_HRED)
    for k in range(2):
        e, dg, db, nrm = est.energy_grad(gams[k], bets[k])
        e_lc, dg_lc, db_lc, mb = Rd.light_cone_energy_grad(wp.n, wp.edges(), terms, gams[k], bets[k])
        assert mb <= 20
        check_energy(e, e_lc)
        check_grad(np.concatenate([dg, db]), np.concatenate([dg_lc, db_lc]))
        eh = est.energy(gams[k], bets[k], obs=OBS_HC)[0]
        check_energy(eh, e_lc)
    e_full = O.energy(wp.n, wp.edges(), terms, gams[0], bets[0])
    check_energy(est.energy(gams[0], bets[0])[0], e_full)


def test_energy_grad_n26_config3_complex128():
    """The same kernels instantiated for complex128 at the full n = 26, p = 4 size (two
    1 GiB states, and checkpoints), against the light-cone FP64 adjoint at 1e-10."""
    from workloads.configs import config3

    wp, p, gams, bets = config3(1)
    pr = A.Problem.from_workload(wp)
    e_lc, dg_lc, db_lc, _ = Rd.light_cone_energy_grad(wp.n, wp.edges(), wp.terms(OBS_HRED), gams[0], bets[0])
    for ckpt in (False, True):
        est = A.Estimator(pr, p, OBS_HRED, A.AAQ_PREC_C128, grad=True, checkpoint=ckpt)
        e, dg, db, nrm = est.energy_grad(gams[0], bets[0])
        check_energy(e, e_lc, 1e-10)
        check_grad(np.concatenate([dg, db]), np.concatenate([dg_lc, db_lc]), 1e-10)
        assert abs(nrm - 1) < 1e-12
        _release(est)


def _release(*objs):
    for o in objs:
        del o
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_energy_grad_n26_config3_checkpointed():
    """The launch configuration the benchmark times (n = 26, p = 4, forward-state
    checkpoints, 4 GiB of checkpoint slots): energy and gradient against the
    light-cone FP64 adjoint at three points, and equal to the uncompute mode within the
    sum of the two modes' tolerances (their complex64 rounding differs)."""
    from workloads.configs import config3

    wp, p, gams, bets = config3(3)
    pr = A.Problem.from_workload(wp)
    terms = wp.terms(OBS_HRED)
    est = A.Estimator(pr, p, OBS_HRED, A.AAQ_PREC_C64, grad=True, checkpoint=True)
    res = []
    for k in range(3):
        e, dg, db, nrm = est.energy_grad(gams[k], bets[k])
        e_lc, dg_lc, db_lc, _ = Rd.light_cone_energy_grad(wp.n, wp.edges(), terms, gams[k], bets[k])
        check_energy(e, e_lc)
        check_grad(np.concatenate([dg, db]), np.concatenate([dg_lc, db_lc]))
        assert abs(nrm - 1) < 1e-5
        res.append(np.concatenate([[e], dg, db]))
    _release(est)
    est = A.Estimator(pr, p, OBS_HRED, A.AAQ_PREC_C64, grad=True, checkpoint=False)
    for k in range(3):
        e, dg, db, _ = est.energy_grad(gams[k], bets[k])
        check_energy(e, res[k][0], 2 * EREL)
        check_grad(np.concatenate([dg, db]), res[k][1:], 2 * GREL)
    _release(est)


def test_energy_n34_config5a_full_size():
    """n = 34, p = 1: one 128 GiB complex64 state on 13-bit tiles in 4 tile sets.
    Energies of both observables against the p = 1 closed form at four points."""
    from workloads.configs import config5a

    wp, p, gams, bets = config5a(4)
    pr = A.Problem.from_workload(wp)
    assert A.aaq_state_bytes(pr) == 8 << 34
    est = A.Estimator(pr, p, OBS_HRED, A.AAQ_PREC_C64, grad=False)
    for k in range(4):
        for obs in (OBS_HRED, OBS_HC):
            e, _, nrm = est.energy(gams[k], bets[k], obs=obs)
            ref = Rd.p1_energy(wp.n, wp.edges(), wp.terms(obs), gams[k, 0], bets[k, 0])
            check_energy(e, ref)
            assert abs(nrm - 1) < 1e-5
    _release(est)


def test_energy_grad_n33_config5b_full_size():
    """n = 33, p = 2: energy + adjoint gradient with two 64 GiB states, against the
    light-cone FP64 adjoint (cones of at most 16 qubits) for both observables."""
    from workloads.configs import config5b

    wp, p, gams, bets = config5b(2)
    pr = A.Problem.from_workload(wp)
    est = A.Estimator(pr, p, OBS_HRED, A.AAQ_PREC_C64, grad=True)
    for k, obs in ((0, OBS_HRED), (1, OBS_HC)):
        e, dg, db, nrm = est.energy_grad(gams[k], bets[k], obs=obs)
        e_lc, dg_lc, db_lc, mb = Rd.light_cone_energy_grad(wp.n, wp.edges(), wp.terms(obs), gams[k], bets[k])
        assert mb <= 16
        check_energy(e, e_lc)
        check_grad(np.concatenate([dg, db]), np.concatenate([dg_lc, db_lc]))
        assert abs(nrm - 1) < 1e-5
    _release(est)


# ------------------------------------------------------------------ tile sizes and autotuning
@pytest.mark.parametrize("g,p", [(G.prufer_tree(14, 2), 2), (G.star(17), 2), (G.prufer_tree(21, 3), 2),
                                 (rand_graph(22, 0.15, 5), 1), (G.random_regular(3, 24, seed=4), 2)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_both_tile_sizes_match_oracle(g, p):
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    rng = np.random.default_rng(g.n + 100 * p)
    gam, bet = rng.uniform(0, math.pi, p), rng.uniform(0, math.pi / 2, p)
    e_ref, dg_ref, db_ref = O.energy_grad(g.n, g.edge_array(), wp.terms(OBS_HRED), gam, bet)
    e_hc = O.energy(g.n, g.edge_array(), wp.terms(OBS_HC), gam, bet)
    est = A.Estimator(pr, p, A.AAQ_OBS_HRED, A.AAQ_PREC_C64, grad=True)
    try:
        for tile in (12, 13):
            A.aaq_set_tile_bits(g.n, A.AAQ_PREC_C64, True, tile)
            A.aaq_set_tile_bits(g.n, A.AAQ_PREC_C64, False, tile)
            assert A.aaq_get_tile_bits(g.n, A.AAQ_PREC_C64, True) == tile
            e, dg, db, nrm = est.energy_grad(gam, bet)
            check_energy(e, e_ref)
            check_grad(np.concatenate([dg, db]), np.concatenate([dg_ref, db_ref]))
            assert abs(nrm - 1) < 1e-5
            check_energy(est.energy(gam, bet, obs=OBS_HC)[0], e_hc)
    finally:
        A.aaq_set_tile_bits(g.n, A.AAQ_PREC_C64, True, 0)
        A.aaq_set_tile_bits(g.n, A.AAQ_PREC_C64, False, 0)


def test_autotune_single_keeps_a_tile_size_and_stays_correct():
    g = G.prufer_tree(22, 9)
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    est = A.Estimator(pr, 2, A.AAQ_OBS_HRED, A.AAQ_PREC_C64, grad=True)
    try:
        best, ms = A.aaq_autotune(pr, 2, True, OBS_HRED, A.AAQ_PREC_C64, est.state, est.lam, est.ws, reps=2)
        assert best in (12, 13) and ms[12] > 0 and ms[13] > 0
        assert A.aaq_get_tile_bits(22, A.AAQ_PREC_C64, True) == best
        gam, bet = np.array([0.3, 1.1]), np.array([0.9, 0.2])
        e_ref, dg_ref, db_ref = O.energy_grad(g.n, g.edge_array(), wp.terms(OBS_HRED), gam, bet)
        e, dg, db, _ = est.energy_grad(gam, bet)
        check_energy(e, e_ref)
        check_grad(np.concatenate([dg, db]), np.concatenate([dg_ref, db_ref]))
    finally:
        A.aaq_set_tile_bits(22, A.AAQ_PREC_C64, True, 0)


# ------------------------------------------------------------------ batched plans
def test_plan_matches_single_calls_and_oracle():
    graphs = [G.star(7), G.complete(9), G.prufer_tree(12, 1), G.binary_tree(13), G.prufer_tree(15, 2),
              G.random_regular(3, 16, seed=3), G.prufer_tree(18, 4)]
    wps = [make_problem(g) for g in graphs]
    prs = [A.Problem.from_workload(w) for w in wps]
    p = 2
    rng = np.random.default_rng(11)
    units = [prs[i % len(prs)] for i in range(2 * len(prs))]
    gam = rng.uniform(0, math.pi, (len(units), p))
    bet = rng.uniform(0, math.pi / 2, (len(units), p))
    for use_graph in (False, True):
        plan = A.Plan(units, p, A.AAQ_OBS_HRED, with_grad=True, use_graph=use_graph)
        plan.params.copy_(torch.from_numpy(np.concatenate([gam, bet], 1)))
        for rep in range(3):  # graph replays with eager work in between
            out = plan.execute().cpu().numpy()
            torch.cuda.synchronize()
            for u, pr in enumerate(units):
                w = wps[u % len(prs)]
                e_ref, dg_ref, db_ref = O.energy_grad(w.n, w.edges(), w.terms(OBS_HRED), gam[u], bet[u])
                check_energy(out[u, 0], e_ref)
                assert abs(out[u, 1] - 1) < 1e-5
                check_grad(out[u, 2:], np.concatenate([dg_ref, db_ref]))
            plan.params.mul_(1.0)
        plan.close()


@pytest.mark.parametrize("prec", [A.AAQ_PREC_C64, A.AAQ_PREC_C128], ids=["c64", "c128"])
@pytest.mark.parametrize("grad", [False, True], ids=["energy", "grad"])
def test_plan_half_state_matches_full_state(prec, grad):
    """Units above the tile size (two and three tile sets, n = 14 ... 23) store and sweep the
    half state in a plan by default: every output equals the full-state plan's (half state
    switched off) within the precision's tolerance, and both match the FP64 oracle."""
    graphs = [G.random_regular(3, 14, seed=2), G.star(16), G.prufer_tree(18, 4), G.prufer_tree(21, 5),
              rand_graph(23, 0.12, 4), G.complete(12)]
    wps = [make_problem(g) for g in graphs]
    units = [A.Problem.from_workload(w) for w in wps]
    p = 2
    rng = np.random.default_rng(41)
    gam = rng.uniform(0, math.pi, (len(units), p))
    bet = rng.uniform(0, math.pi / 2, (len(units), p))
    prm = torch.from_numpy(np.concatenate([gam, bet], 1))
    outs = {}
    for half in (1, 0):
        A.aaq_set_half_state(half)
        try:
            plan = A.Plan(units, p, OBS_HRED, with_grad=grad, use_graph=True, prec=prec)
            plan.params.copy_(prm)
            outs[half] = plan.execute().cpu().numpy()
            plan.close()
        finally:
            A.aaq_set_half_state(1)
    erel, grel = (EREL, GREL) if prec == A.AAQ_PREC_C64 else (1e-10, 1e-10)
    for u, w in enumerate(wps):
        if grad:
            e_ref, dg_ref, db_ref = O.energy_grad(w.n, w.edges(), w.terms(OBS_HRED), gam[u], bet[u])
        else:
            e_ref = O.energy(w.n, w.edges(), w.terms(OBS_HRED), gam[u], bet[u])
        for half in (1, 0):
            check_energy(outs[half][u, 0], e_ref, rel=erel)
            assert abs(outs[half][u, 1] - 1) < (1e-5 if prec == A.AAQ_PREC_C64 else 1e-10)
            if grad:
                check_grad(outs[half][u, 2:], np.concatenate([dg_ref, db_ref]), rel=grel)
        check_energy(outs[1][u, 0], outs[0][u, 0], rel=erel)
        if grad:
            check_grad(outs[1][u, 2:], outs[0][u, 2:], rel=grel)


@pytest.mark.parametrize("p", [8, 40], ids=["p8-checkpoints", "p40-uncompute"])
def test_plan_depth_checkpoints_and_uncompute(p):
    """Plan units above the tile size keep their forward states while there are at most 32
    of them (p = 8, two tile sets: 8 checkpoints) and otherwise uncompute psi in the
    backward steps (p = 40: 40 would be needed), both in the half state: energy, norm and
    gradient against the FP64 oracle."""
    graphs = [G.prufer_tree(16, 7), G.random_regular(3, 14, seed=9), G.prufer_tree(11, 2)]
    wps = [make_problem(g) for g in graphs]
    units = [A.Problem.from_workload(w) for w in wps]
    assert A.aaq_num_sets(16) == 2
    rng = np.random.default_rng(p)
    gam = rng.uniform(0, 0.3, (len(units), p))
    bet = rng.uniform(0, 0.3, (len(units), p))
    plan = A.Plan(units, p, OBS_HRED, with_grad=True, use_graph=True)
    plan.params.copy_(torch.from_numpy(np.concatenate([gam, bet], 1)))
    out = plan.execute().cpu().numpy()
    plan.close()
    for u, w in enumerate(wps):
        e_ref, dg_ref, db_ref = O.energy_grad(w.n, w.edges(), w.terms(OBS_HRED), gam[u], bet[u])
        check_energy(out[u, 0], e_ref)
        assert abs(out[u, 1] - 1) < 1e-5
        check_grad(out[u, 2:], np.concatenate([dg_ref, db_ref]))


@pytest.mark.parametrize("obs", [OBS_HC, OBS_HRED], ids=["H_C", "H_red"])
@pytest.mark.parametrize("grad", [False, True], ids=["energy", "grad"])
def test_plan_groups_of_tile_sets(obs, grad):
    """Units of one, two and three tile sets in one plan (n = 8 ... 23): the large units
    run as batched multi-workgroup sweeps, one group per tile-set count."""
    graphs = [G.prufer_tree(8, 1), G.random_regular(3, 14, seed=2), G.star(16), G.prufer_tree(21, 5),
              G.prufer_tree(22, 6), rand_graph(23, 0.12, 4), G.complete(12)]
    wps = [make_problem(g) for g in graphs]
    units = [A.Problem.from_workload(w) for w in wps]
    assert {A.aaq_num_sets(w.n) for w in wps} == {1, 2, 3}
    p = 2
    rng = np.random.default_rng(23)
    gam = rng.uniform(0, math.pi, (len(units), p))
    bet = rng.uniform(0, math.pi / 2, (len(units), p))
    plan = A.Plan(units, p, obs, with_grad=grad, use_graph=True)
    plan.params.copy_(torch.from_numpy(np.concatenate([gam, bet], 1)))
    for rep in range(2):
        out = plan.execute().cpu().numpy()
        torch.cuda.synchronize()
        for u, w in enumerate(wps):
            if grad:
                e_ref, dg_ref, db_ref = O.energy_grad(w.n, w.edges(), w.terms(obs), gam[u], bet[u])
                check_grad(out[u, 2:], np.concatenate([dg_ref, db_ref]))
            else:
                e_ref = O.energy(w.n, w.edges(), w.terms(obs), gam[u], bet[u])
            check_energy(out[u, 0], e_ref)
            assert abs(out[u, 1] - 1) < 1e-5
    plan.close()


@pytest.mark.parametrize("tl,ts,wg,sl,ss,ms", [(12, 10, 0, 0, 0, 0), (13, 13, 0, 0, 0, 0), (12, 12, 7, 0, 0, 0),
                                               (13, 10, 1, 0, 0, 0), (12, 10, 0, 1, 0, 0), (13, 12, 3, 1, 0, 0),
                                               (12, 10, 0, 0, 1, 0), (13, 10, 0, 1, 1, 0), (12, 10, 0, 0, 0, 12),
                                               (13, 12, 0, 0, 1, 12), (12, 10, 0, 1, 0, 12)])
def test_plan_tile_options_match_oracle(tl, ts, wg, sl, ss, ms):
    """Tile sizes, workgroup counts, the single-launch mode (units with n > 13 swept tile
    by tile inside the persistent kernel), the small-unit launches on streams of their own
    and the 13-qubit unit as batched sweep steps over two 12-bit tiles (max_small_n = 12)
    against the oracle, with graph replays."""
    graphs = [G.prufer_tree(9, 1), G.star(11), G.complete(12), G.binary_tree(13), G.prufer_tree(16, 2),
              G.random_regular(3, 20, seed=5)]
    wps = [make_problem(g) for g in graphs]
    units = [A.Problem.from_workload(w) for w in wps] * 2
    p = 2
    rng = np.random.default_rng(tl * 100 + ts + wg)
    gam = rng.uniform(0, math.pi, (len(units), p))
    bet = rng.uniform(0, math.pi / 2, (len(units), p))
    plan = A.Plan(units, p, OBS_HRED, with_grad=True, tile_bits_large=tl, min_tile_bits_small=ts, workgroups=wg,
                  single_launch=bool(sl), small_streams=bool(ss), max_small_n=ms)
    plan.params.copy_(torch.from_numpy(np.concatenate([gam, bet], 1)))
    for rep in range(2):
        out = plan.execute().cpu().numpy()
        for u in range(len(units)):
            w = wps[u % len(wps)]
            e_ref, dg_ref, db_ref = O.energy_grad(w.n, w.edges(), w.terms(OBS_HRED), gam[u], bet[u])
            check_energy(out[u, 0], e_ref)
            check_grad(out[u, 2:], np.concatenate([dg_ref, db_ref]))
    plan.close()


def test_plan_autotuned():
    graphs = [G.prufer_tree(10, 3), G.star(12), G.prufer_tree(15, 4), G.random_regular(3, 16, seed=1)]
    wps = [make_problem(g) for g in graphs]
    units = [A.Problem.from_workload(w) for w in wps] * 4
    p = 2
    rng = np.random.default_rng(5)
    prm = np.concatenate([rng.uniform(0, math.pi, (len(units), p)), rng.uniform(0, math.pi / 2, (len(units), p))], 1)
    plan = A.Plan.autotuned(units, p, OBS_HRED, True, params=prm, reps=2)
    assert plan.tuned_opts["tile_bits_large"] in (12, 13) and plan.tuned_ms > 0
    plan.params.copy_(torch.from_numpy(prm))
    out = plan.execute().cpu().numpy()
    for u in range(len(units)):
        w = wps[u % len(wps)]
        e_ref, dg_ref, db_ref = O.energy_grad(w.n, w.edges(), w.terms(OBS_HRED), prm[u, :p], prm[u, p:])
        check_energy(out[u, 0], e_ref)
        check_grad(out[u, 2:], np.concatenate([dg_ref, db_ref]))
    plan.close()


def test_plan_energy_only_complex128_grid():
    """Configuration-1 style: the 15-vertex binary tree, p = 1, a parameter grid,
    complex128, both observables equal to the closed form."""
    g = G.binary_tree(15)
    pr = A.Problem.from_workload(make_problem(g))
    a = np.arange(16)
    gg, bb = np.meshgrid(a * math.pi / 15, a * math.pi / 30, indexing="ij")
    gam, bet = gg.reshape(-1), bb.reshape(-1)
    cf = 7 + 0.25 * np.sin(4 * bet) * np.sin(gam) * (8 + 2 * np.cos(gam) + 18 * np.cos(gam) ** 2)
    for obs in (A.AAQ_OBS_HC, A.AAQ_OBS_HRED):
        plan = A.Plan([pr] * 256, 1, obs, with_grad=False, prec=A.AAQ_PREC_C128)
        plan.params.copy_(torch.from_numpy(np.stack([gam, bet], 1)))
        out = plan.execute().cpu().numpy()
        assert np.max(np.abs(out[:, 0] - cf)) < 1e-11
        plan.close()


# ------------------------------------------------------------------ autograd + Adam
def test_autograd_function_and_adam():
    from paper_2410_22247_amd.autograd import adam_maximize, qaoa_energy

    g = G.prufer_tree(16, 2)
    wp = make_problem(g)
    pr = A.Problem.from_workload(wp)
    est = A.Estimator(pr, 2, A.AAQ_OBS_HRED, A.AAQ_PREC_C64, grad=True)
    gam = torch.tensor([0.4, 0.9], dtype=torch.float64, requires_grad=True)
    bet = torch.tensor([0.6, 0.3], dtype=torch.float64, requires_grad=True)
    e = qaoa_energy(gam, bet, est)
    (3.0 * e).backward()
    e_ref, dg_ref, db_ref = O.energy_grad(g.n, g.edge_array(), wp.terms(OBS_HRED), [0.4, 0.9], [0.6, 0.3])
    check_energy(float(e), e_ref)
    check_grad(np.concatenate([gam.grad.numpy(), bet.grad.numpy()]) / 3.0, np.concatenate([dg_ref, db_ref]))
    # Adam maximises <H_red>: the expected cut increases and ends near the oracle value
    gf, bf, hist = adam_maximize(est, [0.4, 0.9], [0.6, 0.3], steps=30, lr=0.05)
    assert hist[-1] > hist[0] + 0.1
    e_end = O.energy(g.n, g.edge_array(), wp.terms(OBS_HRED), gf, bf)
    e_hc = O.energy(g.n, g.edge_array(), wp.terms(OBS_HC), gf, bf)
    assert abs(e_end - e_hc) < 1e-9 and e_end > hist[-1] - 0.05
